"""Parity at full workload size, run the way the benchmark runs it.

The 512^3 workload (134M particles, 150k NFW hosts) goes through rs_fof3d and
the learned 6D form with the shipped proposer on the current stream, exactly
as bench.py times it; the 256^3 workload goes through the plain form; the
1024^3 share (1.07e9 particles, 1.2M hosts, three levels of nested
substructure) goes through the learned form, whose level pipeline then runs
over chunks of groups sized to the device's memory.  Halo properties and
seeds follow on each hierarchy.  At 512^3 and 256^3 the oracle's 3D FoF of
the whole box runs on a host thread meanwhile and every label is compared;
the 6D hierarchy is checked in parts the oracle computes one at a time,
plus properties that hold at any size (tests/fullsize_checks.py):

  * every level-0 node: (a, c, sigma_x^2, sigma_v^2) equal the oracle's
    moments of its member set, for all groups;
  * the whole tree: canonical order, parent levels, sizes as the sum of own
    and child members, deepest[] consistent, level-0 nodes = the 3D groups of
    at least min_group members;
  * 64 3D groups sampled across 10 log-size bins: closed and connected, by
    the oracle FoF of the group's bounding region grown by ll (at 1024^3 for
    the sampled groups up to 2M members);
  * the 6D subtree of every sampled group up to 1.5M members (1M at
    1024^3; the oracle needs minutes per larger group, single-threaded):
    the oracle's hierarchy of that member set, field by field, and the halo
    properties and seeds the oracle computes from it;
  * at 512^3 and 256^3, the halo properties of every node against the
    oracle's from the same hierarchy.
"""
from concurrent.futures import ThreadPoolExecutor
from concurrent.futures import TimeoutError as FuturesTimeout

import numpy as np
import pytest
import torch

import oracle
import paper_2412_18629_amd as rs
from paper_2412_18629_amd import learn, synth

from fullsize_checks import FIELDS, check_all

pytestmark = pytest.mark.gpu


def _run(cfg, form, full3d):
    rs.load_tuning()                   # the launch shapes bench.py times
    dev = torch.device("cuda:0")
    arrs = synth.generate(cfg, 0, device=dev)
    torch.cuda.empty_cache()           # the generator's fp64 temporaries
    oracle3d = None
    if full3d:
        # the oracle's 3D FoF of the whole box, on a host thread while the
        # device works (ctypes releases the interpreter lock)
        pos = [a.cpu().numpy() for a in arrs[:3]]
        pool = ThreadPoolExecutor(1)
        oracle3d = pool.submit(oracle.fof3d, *pos, cfg.box, cfg.link_len)
    labels = torch.empty(cfg.n, dtype=torch.int32, device=dev)
    rs.rs_fof3d(*arrs[:3], cfg.box, cfg.link_len, labels=labels)
    flags = {"learned": rs.RS_LEARNED, "plain": rs.RS_PLAIN}[form]
    tree = rs.rs_phase_fof_batch(*arrs, cfg.box, labels, cfg.min_group, cfg.min_sub, cfg.f,
                                 flags=flags,
                                 model=learn.load_model() if form == "learned" else None)
    props = rs.rs_halo_props(*arrs, cfg.box, tree)
    halo = rs.rs_seed_assign(*arrs, cfg.box, tree, props)
    torch.cuda.synchronize()
    rs.rs_release_workspace()          # the checks below need the device memory
    sl, order = torch.sort(labels.long(), stable=True)
    nc = int(cfg.box // 2.0)
    side = cfg.box / nc
    cell = [torch.clamp((a.double() / side).floor().long(), 0, nc - 1) for a in arrs[:3]]
    key = (cell[0] * nc + cell[1]) * nc + cell[2]
    ks, cperm = torch.sort(key, stable=True)
    cstart = torch.searchsorted(ks, torch.arange(nc ** 3 + 1, device=dev))
    R = dict(host=[a.cpu().numpy() for a in arrs], labels=labels.cpu().numpy(),
             order=order.cpu().numpy(), sorted_labels=sl.cpu().numpy(),
             cperm=cperm.cpu().numpy(), cstart=cstart.cpu().numpy(), nc=nc, side=side,
             tree={k: tree[k].cpu().numpy() for k in FIELDS + ("deepest",)},
             props=props.cpu().numpy(), halo=halo.cpu().numpy())
    del arrs, labels, tree, sl, order, cell, key, ks, cperm, cstart, props, halo
    torch.cuda.empty_cache()
    if oracle3d is not None:
        waited = 0
        while True:
            try:
                R["oracle_labels"] = oracle3d.result(timeout=30)
                break
            except FuturesTimeout:
                waited += 30
                print(f"{cfg.name}: oracle 3D FoF of the whole box still running ({waited} s)",
                      flush=True)
        pool.shutdown()
    return R


@pytest.mark.timeout(1500)
@pytest.mark.parametrize("config,form,full3d,closure_max,subtree_max",
                         [("c512", "learned", True, None, 1_500_000),
                          ("c256", "plain", True, None, None),
                          ("c1024", "learned", False, 2_000_000, 1_000_000)])
def test_fullsize_parity(config, form, full3d, closure_max, subtree_max):
    cfg = synth.CONFIGS[config]
    R = _run(cfg, form, full3d)
    if full3d:
        # every label of the box equals the oracle's
        assert np.array_equal(R["labels"], R["oracle_labels"])
        print(f"{cfg.name}: all {cfg.n} labels equal the oracle's", flush=True)
        # the halo properties of every node, against the oracle's from the
        # same hierarchy (the hierarchy itself is checked below)
        T = R["tree"]
        with ThreadPoolExecutor(1) as pool:
            fut = pool.submit(oracle.halo_props, *R["host"], cfg.box, T["parent"],
                              T["min_index"], T["deepest"])
            waited = 0
            while True:
                try:
                    P = fut.result(timeout=30)
                    break
                except FuturesTimeout:
                    waited += 30
                    print(f"{cfg.name}: oracle halo properties still running ({waited} s)",
                          flush=True)
        assert np.array_equal(R["props"].view(np.int32), P.view(np.int32))
        print(f"{cfg.name}: halo properties of all {P.shape[1]} nodes equal the oracle's",
              flush=True)
    n3, n6 = check_all(R, cfg, subtree_max=subtree_max, closure_max=closure_max,
                       log=lambda s: print(s, flush=True))
    assert n3 >= 50 and n6 >= 45
