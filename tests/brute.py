"""Independent brute-force checker for tiny inputs (numpy + scipy).

A second implementation of the same definitions as the oracle, written a
different way: whole fp32 distance matrices in numpy (each elementwise
ufunc rounds once, so no contraction), scipy's connected components instead
of union-find, ``np.sort`` for the k-th value and Python integers /
``fractions`` for the dispersions.  O(n^2) memory; meant for n up to a few
thousand.  Shares no code with ``oracle/``.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

F32 = np.float32


def _diff(a, L=None):
    """Pairwise fp32 differences a_i - a_j, with the periodic image shift."""
    d = a[:, None] - a[None, :]
    if L is not None:
        L = F32(L)
        h = F32(0.5) * L
        d = np.where(d > h, d - L, np.where(d < -h, d + L, d)).astype(F32)
    return d


def pos_d2_matrix(x, y, z, L):
    dx, dy, dz = (_diff(np.asarray(c, F32), L) for c in (x, y, z))
    return ((dx * dx) + (dy * dy)) + (dz * dz)


def vel_d2_matrix(vx, vy, vz):
    dx, dy, dz = (_diff(np.asarray(c, F32)) for c in (vx, vy, vz))
    return ((dx * dx) + (dy * dy)) + (dz * dz)


def _components_min_label(adj):
    """Label each vertex with the smallest vertex index of its component."""
    n = adj.shape[0]
    i, j = np.nonzero(adj)
    g = coo_matrix((np.ones(i.size, np.int8), (i, j)), shape=(n, n))
    ncomp, comp = connected_components(g, directed=False)
    first = np.full(ncomp, n, np.int64)
    np.minimum.at(first, comp, np.arange(n))
    return first[comp]


def fof3d(x, y, z, L, ll):
    """3D FoF by all pairs: labels = smallest member index."""
    ll = F32(ll)
    D = pos_d2_matrix(x, y, z, L)
    return _components_min_label(D <= ll * ll).astype(np.int32)


def exact_dispersions(pos, vel, L):
    """(sx2, sv2) as exact Fractions, in units of the quantisation grid.

    Positions are quantised to 2^-20 Mpc/h (round half even in fp64), taken
    relative to the first member and moved to the nearest periodic image in
    integers; velocities are quantised to 2^-10 km/s.  The dispersion is
    the mean squared distance from the mean, summed over the three axes.
    """
    n = pos.shape[0]
    LQ = int(np.rint(np.float64(L) * 2.0 ** 20))
    sx = Fraction(0)
    sv = Fraction(0)
    for ax in range(3):
        q = [int(v) for v in np.rint(pos[:, ax].astype(np.float64) * 2.0 ** 20)]
        d = []
        for v in q:
            t = v - q[0]
            if 2 * t > LQ:
                t -= LQ
            elif 2 * t <= -LQ:
                t += LQ
            d.append(t)
        mean = Fraction(sum(d), n)
        sx += sum((Fraction(t) - mean) ** 2 for t in d) / n
        w = [int(v) for v in np.rint(vel[:, ax].astype(np.float64) * 2.0 ** 10)]
        mw = Fraction(sum(w), n)
        sv += sum((Fraction(t) - mw) ** 2 for t in w) / n
    return sx, sv


def metric_factors(pos, vel, L):
    """a = 1/sigma_x^2, c = 1/sigma_v^2 rounded as the definition fixes:
    N^2 / V in fp64, exact power-of-two scaling, then one rounding to fp32."""
    n = pos.shape[0]
    sx, sv = exact_dispersions(pos, vel, L)
    Vx = sx * n * n          # integer: N^2 * dispersion in quantum units
    Vv = sv * n * n
    assert Vx.denominator == 1 and Vv.denominator == 1
    nn = float(n) * float(n)
    a = F32(1.0) if Vx == 0 else F32((nn / float(Vx.numerator)) * 2.0 ** 40)
    c = F32(1.0) if Vv == 0 else F32((nn / float(Vv.numerator)) * 2.0 ** 20)
    return a, c


def select_rank(n, f):
    ppm = int(round(f * 1e6))
    k = -((-n * ppm) // 10 ** 6)
    return min(max(k, 1), n)


def phase_split(pos, vel, L, f, min_sub):
    """One node: returns (a, c, l2, nn_d2, list of child member-slot arrays)."""
    n = pos.shape[0]
    a, c = metric_factors(pos, vel, L)
    Dx = pos_d2_matrix(pos[:, 0], pos[:, 1], pos[:, 2], L)
    Dv = vel_d2_matrix(vel[:, 0], vel[:, 1], vel[:, 2])
    d2 = (a * Dx) + (c * Dv)
    off = d2.copy()
    np.fill_diagonal(off, np.inf)
    nn = off.min(axis=1)
    k = select_rank(n, f)
    l2 = np.sort(nn)[k - 1]
    adj = d2 <= l2
    lab = _components_min_label(adj)
    kids = []
    for r in np.unique(lab):
        m = np.nonzero(lab == r)[0]
        if min_sub <= m.size < n:
            kids.append(m)
    return a, c, F32(l2), nn, kids


def phase_fof(x, y, z, vx, vy, vz, L, labels, min_group=10, min_sub=10, f=0.7):
    """Whole hierarchy by brute force; node dicts in canonical order."""
    pos = np.stack([np.asarray(q, F32) for q in (x, y, z)], axis=1)
    vel = np.stack([np.asarray(q, F32) for q in (vx, vy, vz)], axis=1)
    labels = np.asarray(labels)
    nodes = []
    ids, cnt = np.unique(labels, return_counts=True)
    todo = []
    for r, c in zip(ids, cnt):
        if c >= min_group:
            todo.append((np.sort(np.nonzero(labels == r)[0]), 0, None))
    while todo:
        mem, level, par = todo.pop()
        a, c, l2, _, kids = phase_split(pos[mem], vel[mem], L, f, min_sub)
        key = (level, int(mem[0]))
        nodes.append(dict(key=key, level=level, min_index=int(mem[0]), size=mem.size,
                          l2=l2, a=a, c=c, parent_key=par, members=mem))
        for k in kids:
            todo.append((mem[k], level + 1, key))
    nodes.sort(key=lambda d: d["key"])
    index = {d["key"]: i for i, d in enumerate(nodes)}
    n = pos.shape[0]
    deepest = np.full(n, -1, np.int64)
    for i, d in enumerate(nodes):
        d["parent"] = -1 if d["parent_key"] is None else index[d["parent_key"]]
        deepest[d["members"]] = i
    return nodes, deepest


def exact_props(pos, vel, L, ref=0):
    """Centre, bulk velocity, second-moment tensor about the centre and mean
    (x - centre) x (v - velocity) of one member set, as exact Fractions.

    Positions are quantised to 2^-20 (round half even in fp64) and moved to
    the nearest periodic image of member `ref` in integers; velocities are
    quantised to 2^-10.  The centre is returned in [0, L) (exact rational, in
    Mpc/h); the tensor rows are xx, yy, zz, xy, xz, yz.
    """
    n = pos.shape[0]
    LQ = int(np.rint(np.float64(L) * 2.0 ** 20))
    d = np.zeros((n, 3), dtype=object)
    w = np.zeros((n, 3), dtype=object)
    qref = [int(v) for v in np.rint(pos[ref].astype(np.float64) * 2.0 ** 20)]
    for ax in range(3):
        q = [int(v) for v in np.rint(pos[:, ax].astype(np.float64) * 2.0 ** 20)]
        for i in range(n):
            t = q[i] - qref[ax]
            if 2 * t > LQ:
                t -= LQ
            elif 2 * t <= -LQ:
                t += LQ
            d[i, ax] = t
            w[i, ax] = int(np.rint(np.float64(vel[i, ax]) * 2.0 ** 10))
    mean_d = [Fraction(sum(d[:, a]), n) for a in range(3)]
    mean_w = [Fraction(sum(w[:, a]), n) for a in range(3)]
    cen = []
    Lf = Fraction(float(L))
    for a in range(3):
        c = (qref[a] + mean_d[a]) / 2 ** 20
        if c < 0:
            c += Lf
        elif c >= Lf:
            c -= Lf
        cen.append(c)
    vbar = [m / 2 ** 10 for m in mean_w]
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    M = [sum((Fraction(d[i, a]) - mean_d[a]) * (Fraction(d[i, b]) - mean_d[b])
             for i in range(n)) / n / 2 ** 40 for a, b in pairs]
    j = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        s = sum((Fraction(d[i, b]) - mean_d[b]) * (Fraction(w[i, c]) - mean_w[c]) -
                (Fraction(d[i, c]) - mean_d[c]) * (Fraction(w[i, b]) - mean_w[b])
                for i in range(n))
        j.append(s / n / 2 ** 30)
    return cen + vbar + M + j


def seed_assign(pos, vel, L, parent, deepest, a, c, props):
    """Seed of each particle by brute force: the leaf, among the leaves below
    the particle's deepest node, with the smallest fp32 phase-space distance
    to the leaf's centre and bulk velocity (ties: smaller node index)."""
    parent = np.asarray(parent)
    m = parent.size
    kids = np.zeros(m, np.int64)
    np.add.at(kids, parent[parent >= 0], 1)
    leaves = np.nonzero(kids == 0)[0]
    below = {k: [] for k in range(m)}
    for s in leaves:
        k = s
        while k >= 0:
            below[k].append(s)
            k = parent[k]
    L32 = F32(L)
    h = F32(0.5) * L32
    out = np.full(pos.shape[0], -1, np.int64)
    for i in range(pos.shape[0]):
        d = int(deepest[i])
        if d < 0:
            continue
        if kids[d] == 0:
            out[i] = d
            continue
        s = np.array(sorted(below[d]))
        dxs = []
        for ax in range(3):
            t = (pos[i, ax] - props[ax, s]).astype(F32)
            t = np.where(t > h, t - L32, np.where(t < -h, t + L32, t)).astype(F32)
            dxs.append(t)
        Dx = ((dxs[0] * dxs[0]) + (dxs[1] * dxs[1])) + (dxs[2] * dxs[2])
        dvs = [(vel[i, ax] - props[3 + ax, s]).astype(F32) for ax in range(3)]
        Dv = ((dvs[0] * dvs[0]) + (dvs[1] * dvs[1])) + (dvs[2] * dvs[2])
        d2 = (np.asarray(a, F32)[s] * Dx) + (np.asarray(c, F32)[s] * Dv)
        out[i] = s[np.lexsort((s, d2))[0]]
    return out.astype(np.int32)
