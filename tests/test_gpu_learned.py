"""The learned form (RS_LEARNED): a proposal only chooses the bracket, so
every field must equal the exact batched form bit for bit, whatever the
network says -- accepted brackets, brackets that are too high, too low, or an
untrained network -- and the oracle where it is run.  Also: the proposer
features, and what the trained network gains over an untrained one."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2412_18629_amd as rs
from paper_2412_18629_amd import learn, synth

pytestmark = pytest.mark.gpu
FIELDS = ("level", "min_index", "parent", "size", "l2", "a", "c", "sx2", "sv2", "wide", "deepest")


def _workload(n, seed, device="cuda"):
    cfg = synth.scaled(synth.CONFIGS["c32"], n)
    arrs = [a.to(device) for a in synth.generate(cfg, seed)]
    lab, _ = rs.rs_fof3d(*arrs[:3], cfg.box, cfg.link_len)
    return cfg, arrs, lab


def _blob(bias_shift=0.0, seed=0):
    params = learn.init_params(seed)
    params[-1] += bias_shift
    return rs.pack_model(np.zeros(24), np.ones(24), params)


def _trained():
    if not os.path.exists(learn.DEFAULT_MODEL):
        pytest.skip("no trained proposer file")
    return learn.load_model()


def _same(a, b):
    for k in FIELDS:
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("shift", [0.0, 12.0, -40.0])
def test_learned_equals_batched_for_any_proposal(shift):
    cfg, arrs, lab = _workload(400000, 11)
    ref = rs.rs_phase_fof_batch(*arrs, cfg.box, lab)
    got = rs.rs_phase_fof_batch(*arrs, cfg.box, lab, flags=rs.RS_LEARNED, model=_blob(shift))
    _same(ref, got)
    n_large_nodes = got["n_accepted"] + got["n_fallback"]
    assert n_large_nodes == int((ref["size"] > 2048).sum().item())
    if shift != 0.0:
        assert got["n_accepted"] == 0          # bracket far off: every node falls back


def test_learned_trained_accepts_and_matches_oracle():
    blob = _trained()
    cfg = synth.scaled(synth.CONFIGS["c32"], 300000)
    host = [a.numpy() for a in synth.generate(cfg, 12)]
    arrs = [torch.from_numpy(a).cuda() for a in host]
    lab, _ = rs.rs_fof3d(*arrs[:3], cfg.box, cfg.link_len)
    got = rs.rs_phase_fof_batch(*arrs, cfg.box, lab, flags=rs.RS_LEARNED, model=blob)
    ref = oracle.phase_fof(*host, cfg.box, lab.cpu().numpy())
    for k in FIELDS:
        assert np.array_equal(got[k].cpu().numpy(), ref[k]), k
    assert got["n_accepted"] > 0


def test_features():
    cfg, arrs, lab = _workload(200000, 13)
    t = rs.rs_phase_fof_batch(*arrs, cfg.box, lab, flags=rs.RS_BATCHED | rs.RS_FEATURES)
    f = t["features"].cpu().numpy()
    assert f.shape == (t["level"].numel(), 24)
    assert np.allclose(f[:, 0], np.log(t["size"].cpu().numpy()), rtol=1e-6)
    assert np.array_equal(f[:, 23], t["level"].cpu().numpy().astype(np.float32))
    for lo, hi in ((1, 4), (4, 7), (7, 15), (15, 23)):
        assert np.allclose(f[:, lo:hi].sum(1), 1.0, atol=1e-4), (lo, hi)
    # features do not change the result
    _same(t, rs.rs_phase_fof_batch(*arrs, cfg.box, lab))


def test_trained_network_beats_untrained():
    blob = _trained()
    cfg, arrs, lab = _workload(1000000, 200)          # held-out seed
    tr = rs.rs_phase_fof_batch(*arrs, cfg.box, lab, flags=rs.RS_LEARNED, model=blob)
    un = rs.rs_phase_fof_batch(*arrs, cfg.box, lab, flags=rs.RS_LEARNED, model=_blob())
    _same(tr, un)
    acc_tr = tr["n_accepted"] / max(1, tr["n_accepted"] + tr["n_fallback"])
    acc_un = un["n_accepted"] / max(1, un["n_accepted"] + un["n_fallback"])
    assert acc_tr > acc_un and acc_tr >= 0.5, (acc_tr, acc_un)
