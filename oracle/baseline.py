"""CPU baseline driver: the oracle timed on sub-boxes of a workload.

TEST INFRASTRUCTURE ONLY (the benchmark's CPU-baseline leg).  It holds none
of the method's arithmetic: it cuts one process's sub-box (owned particles
plus the ghost shell of width gw, no periodic images needed for a cube away
from the box faces) out of the workload arrays, then times the oracle's
sub-box 3D FoF, its 6D hierarchy of the resulting groups (positions
passed in their original periodic frame), and the halo properties and seed
assignment of that hierarchy.  `run_parts` deals the groups of
one sub-box to worker processes (fresh interpreters, so they never inherit a
GPU context), one per core, and times their 6D hierarchies at once.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(_HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(_HERE))


def cut(arrs, lo, side, gw):
    """(owned-first arrays, n_owned) of the cube [lo, lo + side)^3 with its
    shell of width gw; the cube and shell must stay inside the box."""
    x, y, z = arrs[0], arrs[1], arrs[2]
    # the bounds as the sub-box FoF reads them: fp32 corners, the shell in
    # fp64 from the fp32 corners and the fp32 width
    lo32 = np.asarray(lo, np.float32)
    hi32 = (np.asarray(lo, np.float64) + side).astype(np.float32)
    gw64 = float(np.float32(gw))
    inshell = np.ones(x.shape[0], bool)
    owned = np.ones(x.shape[0], bool)
    for a, c in enumerate((x, y, z)):
        c64 = c.astype(np.float64)
        inshell &= (c64 >= float(lo32[a]) - gw64) & (c64 < float(hi32[a]) + gw64)
        owned &= (c >= lo32[a]) & (c < hi32[a])
    idx = np.concatenate([np.nonzero(owned)[0], np.nonzero(inshell & ~owned)[0]])
    return [np.ascontiguousarray(a[idx]) for a in arrs], int(owned.sum()), lo32, hi32


def run_one(job):
    """Times the oracle on one sub-box: job = (arrays, n_owned, lo, hi, gw,
    box, link_len, min_group, min_sub, f).  Returns (n_owned, n, t3d, t6d,
    labels, rows) with rows = {"halo_props": (seconds, member-levels),
    "seed_assign": (seconds, particles)} over the sub-box's hierarchy."""
    import oracle
    arrs, n_owned, lo, hi, gw, box, ll, min_group, min_sub, f = job
    t0 = time.perf_counter()
    lab, _ = oracle.fof3d_subbox(arrs[0], arrs[1], arrs[2], n_owned, lo, hi, gw, ll)
    t1 = time.perf_counter()
    t = oracle.phase_fof(*arrs, box, lab, min_group, min_sub, f)
    t2 = time.perf_counter()
    P = oracle.halo_props(*arrs, box, t["parent"], t["min_index"], t["deepest"])
    t3 = time.perf_counter()
    oracle.seed_assign(*arrs, box, t["parent"], t["deepest"], t["a"], t["c"], P)
    t4 = time.perf_counter()
    rows = {"halo_props": (t3 - t2, int(np.asarray(t["size"], np.int64).sum())),
            "seed_assign": (t4 - t3, int(arrs[0].size))}
    return n_owned, arrs[0].size, t1 - t0, t2 - t1, lab, rows


def split_groups(arrs, labels, min_group, parts):
    """The 3D groups of at least min_group members dealt to `parts` bins,
    largest first onto the least loaded bin; each bin's member arrays and
    labels renumbered to its own particle indices."""
    ids, cnt = np.unique(labels, return_counts=True)
    keep = cnt >= min_group
    ids, cnt = ids[keep], cnt[keep]
    order = np.argsort(-cnt, kind="stable")
    load = np.zeros(parts, np.int64)
    owner = np.empty(ids.size, np.int64)
    for g in order:
        b = int(np.argmin(load))
        owner[g] = b
        load[b] += cnt[g]
    gbin = dict(zip(ids.tolist(), owner.tolist()))
    pbin = np.array([gbin.get(l, -1) for l in labels.tolist()])
    out = []
    for b in range(parts):
        sel = np.nonzero(pbin == b)[0]
        loc = np.full(labels.size, -1, np.int64)
        loc[sel] = np.arange(sel.size)
        out.append(([np.ascontiguousarray(a[sel]) for a in arrs],
                    loc[labels[sel]].astype(np.int32)))
    return out


def _part_main(path):
    """Worker process: the 6D hierarchy of one bin of groups, timed."""
    import json
    import oracle
    d = np.load(path)
    arrs = [d[k] for k in ("x", "y", "z", "vx", "vy", "vz")]
    t0 = time.perf_counter()
    oracle.phase_fof(*arrs, float(d["box"]), d["labels"], int(d["min_group"]),
                     int(d["min_sub"]), float(d["f"]))
    print(json.dumps([int(arrs[0].size), time.perf_counter() - t0]), flush=True)


def run_parts(parts, box, min_group, min_sub, f, tmpdir, progress=None):
    """Runs the 6D hierarchy of every bin in its own worker process (plain
    interpreters that import only numpy and the oracle), all at once.
    Returns [(members, seconds)] per bin and the wall time."""
    import json
    import subprocess
    import oracle
    oracle.build(force=False)
    root = os.path.dirname(_HERE)
    paths = []
    for k, (arrs, lab) in enumerate(parts):
        path = os.path.join(tmpdir, f"baseline_part_{os.getpid()}_{k}.npz")
        np.savez(path, x=arrs[0], y=arrs[1], z=arrs[2], vx=arrs[3], vy=arrs[4], vz=arrs[5],
                 labels=lab, box=box, min_group=min_group, min_sub=min_sub, f=f)
        paths.append(path)
    code = ("import sys; sys.path.insert(0, %r); from oracle.baseline import _part_main; "
            "_part_main(sys.argv[1])" % root)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = [None] * len(paths)
    t0 = time.perf_counter()
    try:
        procs = [subprocess.Popen([sys.executable, "-c", code, p], stdout=subprocess.PIPE,
                                  env=env) for p in paths]
        for k, pr in enumerate(procs):
            so, _ = pr.communicate()
            if pr.returncode != 0:
                raise RuntimeError(f"oracle baseline worker {k} failed ({pr.returncode})")
            out[k] = tuple(json.loads(so.decode().strip().splitlines()[-1]))
            if progress:
                progress(f"oracle worker {k} done: {out[k][0]} members in {out[k][1]:.1f} s")
    finally:
        for p in paths:
            if os.path.exists(p):
                os.remove(p)
    return out, time.perf_counter() - t0
