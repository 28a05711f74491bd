"""Domain decomposition of a periodic box into non-periodic sub-boxes with
ghost shells, and the union of per-sub-box results (test helpers).

Input generation and bookkeeping only: a sub-box's inputs are its own
particles followed by every periodic image (shift by -L, 0 or +L per axis)
of any particle that falls in the shell [lo - gw, hi + gw) outside
[lo, hi).  With coordinates on a dyadic grid the shifted copies are exact in
fp32, so the unshifted differences inside a sub-box equal the periodic
ones.
"""
from __future__ import annotations

import itertools

import numpy as np

F32 = np.float32


def snap(pos, L, q=2.0 ** -12):
    """Positions on a dyadic grid of spacing q inside [0, L)."""
    p = np.mod(np.round(pos.astype(np.float64) / q) * q, L)
    return p.astype(F32)


def split(L, parts):
    """Sub-box bounds (lo, hi) for `parts` = (px, py, pz) equal slabs per axis."""
    out = []
    for idx in itertools.product(*[range(p) for p in parts]):
        lo = [L * i / p for i, p in zip(idx, parts)]
        hi = [L * (i + 1) / p for i, p in zip(idx, parts)]
        out.append((np.array(lo, F32), np.array(hi, F32)))
    return out


def subbox_inputs(pos, L, lo, hi, gw):
    """(local positions (m, 3) fp32, global ids (m,), n_owned) of one sub-box."""
    inside = np.all((pos >= lo) & (pos < hi), axis=1)
    own = np.nonzero(inside)[0]
    gl = [own]
    gp = [pos[own]]
    glo = lo.astype(np.float64) - gw
    ghi = hi.astype(np.float64) + gw
    for sh in itertools.product((-1, 0, 1), repeat=3):
        q = pos.astype(np.float64) + np.array(sh, np.float64) * float(L)
        inshell = np.all((q >= glo) & (q < ghi), axis=1)
        if sh == (0, 0, 0):
            inshell &= ~inside
        ids = np.nonzero(inshell)[0]
        gl.append(ids)
        gp.append(q[ids].astype(F32))
    return np.concatenate(gp).astype(F32), np.concatenate(gl), own.size


class UnionFind:
    def __init__(self, n):
        self.p = np.arange(n)

    def find(self, a):
        p = self.p
        r = a
        while p[r] != r:
            r = p[r]
        while p[a] != r:
            p[a], a = r, p[a]
        return r

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra != rb:
            self.p[max(ra, rb)] = min(ra, rb)

    def labels(self):
        return np.array([self.find(i) for i in range(self.p.size)])


def union_subboxes(n, results):
    """Global labels (smallest global index per group) from per-sub-box
    (global ids, n_owned, labels, ghost_links) results: owned particles join
    their local group's smallest member, ghosts in a link join theirs."""
    uf = UnionFind(n)
    for gid, n_owned, lab, links in results:
        for k in range(n_owned):
            uf.union(gid[k], gid[lab[k]])
        for g, l in links:
            uf.union(gid[g], gid[l])
    return uf.labels()
