"""Seeded constructions of particle pairs at the edge of the 3D linking test.

Input generation only: nothing here evaluates the pair relation.  Each
construction places pairs whose separation along one axis sits within a few
fp32 steps of the linking length, in lanes far apart on the other two axes
(so the pairs cannot link to each other), at the places a cell grid can get
wrong:

* across the periodic face, one particle a few ulps below L and the other
  swept over the fp32 values around ll - (L - x_i); there the periodic image
  shift rounds the separation to the ulp grid of L, so some pairs whose true
  separation exceeds ll have a computed D <= ll^2;
* across interior cell boundaries of grids of side L/k for the cell counts
  k next to L/ll (the cells one grid scheme or another would use) and of
  their half-cell grids, with the separation swept over the fp32 values
  around ll.

The box side and ll are chosen so that L/ll lies within a few fp32 steps of
an integer, where the choice between two neighbouring cell counts is made.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def steps(v, k):
    """The fp32 values v, and k steps below and above it."""
    v = F32(v)
    out = [v]
    up = dn = v
    for _ in range(k):
        up = np.nextafter(up, F32(np.inf))
        dn = np.nextafter(dn, F32(-np.inf))
        out += [up, dn]
    return np.array(sorted(out), F32)


def near_integer_ratio_lengths(L, counts, k=2):
    """Linking lengths within k fp32 steps of L / c for each count c."""
    out = []
    for c in counts:
        out.extend(steps(F32(float(L) / c), k).tolist())
    return np.array(sorted(set(out)), F32)


def edge_pair_box(L, ll, seed=0, sweep=6):
    """Positions (n, 3) fp32 in [0, L): edge pairs along every axis, each in
    its own lane.  Returns (pos, pairs) with pairs an (m, 2) index array."""
    rng = np.random.default_rng(seed)
    L = F32(L)
    ll = F32(ll)
    Ld = float(L)
    lld = float(ll)
    xs = []
    # across the periodic face: x_i at 1..3 ulps below L, x_j near ll - (L - x_i)
    top = np.nextafter(L, F32(0))
    for u in range(3):
        xi = top
        for _ in range(u):
            xi = np.nextafter(xi, F32(0))
        gap = Ld - float(xi)
        for xj in steps(F32(lld - gap), sweep):
            if 0.0 <= float(xj) < Ld:
                xs.append((xi, xj))
    # interior cell boundaries of the grids next to L / ll, and of their
    # half-cell (octant) grids
    c0 = int(np.floor(Ld / lld))
    for c in (c0 - 1, c0, c0 + 1, 2 * c0 - 2, 2 * c0):
        if c < 3:
            continue
        side = Ld / c
        # the first boundaries (fine fp32 steps near the origin resolve
        # separations within a few steps of ll) and a few random ones
        bs = [1, 2] + rng.choice(np.arange(3, c), size=min(3, c - 3), replace=False).tolist()
        for b in bs:
            edge = F32(b * side)
            k = sweep if b <= 2 else sweep // 2
            for xi in steps(edge, 1):
                for xj in steps(F32(float(xi) + lld), k):
                    if float(xj) < Ld:
                        xs.append((xi, xj))
                for xj in steps(F32(float(xi) - lld), k):
                    if float(xj) >= 0.0:
                        xs.append((xi, xj))
    # lanes: the two other coordinates on a coarse grid of spacing > 3 ll
    m = len(xs)
    lanes_per_axis = max(2, int(Ld // (3.5 * lld)))
    cells = rng.permutation(lanes_per_axis * lanes_per_axis)
    if m > cells.size:
        xs = xs[: cells.size]
        m = cells.size
    pos = np.empty((2 * m, 3), F32)
    pairs = np.empty((m, 2), np.int64)
    spacing = Ld / lanes_per_axis
    for p, (xi, xj) in enumerate(xs):
        ax = p % 3
        o1, o2 = [(a + 1) % 3 for a in (ax, ax + 1)]
        c = cells[p]
        u = F32((c % lanes_per_axis) * spacing + 0.25 * spacing)
        w = F32((c // lanes_per_axis) * spacing + 0.25 * spacing)
        for s, v in ((2 * p, xi), (2 * p + 1, xj)):
            pos[s, ax] = v
            pos[s, o1] = u
            pos[s, o2] = w
        pairs[p] = (2 * p, 2 * p + 1)
    perm = rng.permutation(2 * m)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(2 * m)
    return pos[perm], inv[pairs]


def true_separation(pos, pairs, L):
    """Exact nearest-image separation of each pair along its axis (fp64: the
    differences of fp32 values and the shift by L are exact there; the pair's
    other two coordinates are equal)."""
    a = pos[pairs[:, 0]].astype(np.float64)
    b = pos[pairs[:, 1]].astype(np.float64)
    d = np.abs(a - b)
    d = np.minimum(d, float(L) - d)
    return d.max(axis=1)
