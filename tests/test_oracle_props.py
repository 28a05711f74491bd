"""Pins for the oracle's per-node halo properties (CPU only).

The paper lists halo properties, among them the inertia tensor, as new
functions of its code (Summary) but prints no values, so the oracle is pinned
by closed forms (two particles, including across the periodic face; a
rotating lattice block), by an exact rational recomputation of random member
sets, by membership through a nested hierarchy, and by invariances.
"""
from fractions import Fraction

import numpy as np
import pytest

import brute
import oracle
from paper_2412_18629_amd import synth

F32 = np.float32


def _one_node(pos, vel, L):
    """props of one level-0 node holding every particle (smallest index 0)."""
    n = pos.shape[0]
    return oracle.halo_props(pos[:, 0], pos[:, 1], pos[:, 2], vel[:, 0], vel[:, 1], vel[:, 2],
                             L, np.array([-1], np.int32), np.array([0], np.int32),
                             np.zeros(n, np.int32))[:, 0]


def _f32_of(fr):
    return F32(float(fr))


def test_two_particles_closed_form():
    L = F32(10.0)
    p = np.array([[1.5, 2.25, 3.0], [1.75, 2.0, 3.5]], F32)
    v = np.array([[10.0, 0.0, -5.0], [20.0, 4.0, 5.0]], F32)
    got = _one_node(p, v, L)
    dx = (p[1] - p[0]).astype(np.float64)
    dv = (v[1] - v[0]).astype(np.float64)
    cen = (p[0] + p[1]).astype(np.float64) / 2
    M = [dx[0] * dx[0] / 4, dx[1] * dx[1] / 4, dx[2] * dx[2] / 4,
         dx[0] * dx[1] / 4, dx[0] * dx[2] / 4, dx[1] * dx[2] / 4]
    j = np.cross(dx, dv) / 4
    want = np.array(list(cen) + list((v[0] + v[1]).astype(np.float64) / 2) + M + list(j), F32)
    assert np.array_equal(got, want)


def test_two_particles_across_the_face():
    # the smallest-index member sits at x = 0.125, the other at L - 0.375: the
    # nearest image puts the centre at -0.125, stored as L - 0.125
    L = F32(10.0)
    p = np.array([[0.125, 4.0, 9.75], [9.625, 4.5, 0.25]], F32)
    v = np.zeros((2, 3), F32)
    got = _one_node(p, v, L)
    assert got[0] == F32(9.875) and got[1] == F32(4.25) and got[2] == F32(0.0)
    # separations -0.5, 0.5, 0.5 (nearest image): M = d d^T / 4
    assert list(got[6:12]) == [0.0625, 0.0625, 0.0625, -0.0625, -0.0625, 0.0625]


def test_rotating_lattice_block():
    # 4 x 3 x 2 lattice of spacing 1/4 rotating rigidly about z (omega = 4)
    # with bulk velocity V: M_aa = s^2 (n_a^2 - 1) / 12, no off-diagonal
    # terms, j = (0, 0, omega (Mxx + Myy)), velocity V
    L = F32(16.0)
    s, om = 0.25, 4.0
    gx, gy, gz = np.meshgrid(np.arange(4), np.arange(3), np.arange(2), indexing="ij")
    p = np.stack([1 + s * gx.ravel(), 2 + s * gy.ravel(), 3 + s * gz.ravel()], 1)
    c = np.array([1 + 1.5 * s, 2 + s, 3 + 0.5 * s])
    V = np.array([100.0, -50.0, 25.5])
    v = np.stack([-om * (p[:, 1] - c[1]), om * (p[:, 0] - c[0]), np.zeros(len(p))], 1) + V
    got = _one_node(p.astype(F32), v.astype(F32), L)
    Mxx = Fraction(1, 16) * 15 / 12
    Myy = Fraction(1, 16) * 8 / 12
    Mzz = Fraction(1, 16) * 3 / 12
    want = [Fraction(c[0]), Fraction(c[1]), Fraction(c[2]), Fraction(V[0]), Fraction(V[1]),
            Fraction(V[2]), Mxx, Myy, Mzz, 0, 0, 0, 0, 0, om * (Mxx + Myy)]
    assert np.array_equal(got, np.array([_f32_of(w) for w in want], F32))


@pytest.mark.parametrize("seed", range(8))
def test_exact_rationals_random_sets(seed):
    # members spread over a few Mpc/h, half of the sets across a periodic face
    rng = np.random.default_rng(seed)
    L = F32(20.0)
    n = int(rng.integers(2, 60))
    cen = rng.uniform(0, 20, 3)
    if seed % 2:
        cen[seed % 3] = 19.9
    p = np.mod(cen + rng.normal(0, 0.8, (n, 3)), 20.0).astype(F32)
    p[p >= L] = 0
    v = rng.normal(0, 300, (n, 3)).astype(F32)
    got = _one_node(p, v, L)
    want = np.array([_f32_of(w) for w in brute.exact_props(p, v, L, ref=0)], F32)
    assert np.array_equal(got, want)


def test_membership_through_the_hierarchy():
    # node 0 holds everything; nodes 1 and 2 (children of 0) hold two subsets,
    # node 3 (child of 1) part of node 1.  Each node equals a standalone node
    # of its members (with the same smallest member).
    rng = np.random.default_rng(3)
    L = F32(20.0)
    n = 200
    p = (rng.uniform(5, 8, (n, 3))).astype(F32)
    v = rng.normal(0, 100, (n, 3)).astype(F32)
    deep = np.zeros(n, np.int32)
    deep[20:80] = 1
    deep[100:150] = 2
    deep[40:60] = 3
    parent = np.array([-1, 0, 0, 1], np.int32)
    mins = np.array([0, 20, 100, 40], np.int32)
    got = oracle.halo_props(*[p[:, k] for k in range(3)], *[v[:, k] for k in range(3)], L,
                            parent, mins, deep)
    for k, sel in ((0, np.arange(n)), (1, np.arange(20, 80)), (2, np.arange(100, 150)),
                   (3, np.arange(40, 60))):
        assert np.array_equal(got[:, k], _one_node(p[sel], v[sel], L))


def _c32_tree(seed=0):
    cfg = synth.CONFIGS["c32"]
    arrs = [a.numpy() for a in synth.generate(cfg, seed)]
    lab = oracle.fof3d(*arrs[:3], cfg.box, cfg.link_len)
    tree = oracle.phase_fof(*arrs, cfg.box, lab)
    return cfg, arrs, tree


def test_invariants_on_the_32cubed_tree():
    cfg, arrs, t = _c32_tree()
    P = oracle.halo_props(*arrs, cfg.box, t["parent"], t["min_index"], t["deepest"])
    # the trace of the tensor is the position dispersion of the node
    tr = P[6].astype(np.float64) + P[7] + P[8]
    assert np.allclose(tr, t["sx2"], rtol=2e-6, atol=0)
    # positive semi-definite (eigenvalues of the symmetric tensor)
    for k in range(P.shape[1]):
        m = np.array([[P[6, k], P[9, k], P[10, k]], [P[9, k], P[7, k], P[11, k]],
                      [P[10, k], P[11, k], P[8, k]]], np.float64)
        assert np.linalg.eigvalsh(m).min() >= -1e-6 * np.trace(m)
    assert np.all((P[:3] >= 0) & (P[:3] < cfg.box))


def test_translation_on_a_dyadic_grid():
    # positions on a 2^-12 grid in a box of 20: a translation by a grid
    # multiple changes no quantised difference, so everything but the centre
    # is bit-identical and the centre moves by the translation (mod L)
    cfg = synth.CONFIGS["c32"]
    arrs = [a.numpy() for a in synth.generate(cfg, 2)]
    q = 2.0 ** -12
    pos = [np.mod(np.round(a.astype(np.float64) / q) * q, 20.0).astype(F32) for a in arrs[:3]]
    lab = oracle.fof3d(*pos, 20.0, cfg.link_len)
    t = oracle.phase_fof(*pos, *arrs[3:], 20.0, lab)
    P = oracle.halo_props(*pos, *arrs[3:], 20.0, t["parent"], t["min_index"], t["deepest"])
    shift = [7.25 + 3 * q, 13.5 + 11 * q, 0.75 + 5 * q]
    moved = [np.mod(a.astype(np.float64) + s, 20.0).astype(F32) for a, s in zip(pos, shift)]
    Pm = oracle.halo_props(*moved, *arrs[3:], 20.0, t["parent"], t["min_index"], t["deepest"])
    assert np.array_equal(P[3:], Pm[3:])
    for a in range(3):
        want = np.mod(P[a].astype(np.float64) + shift[a], 20.0)
        diff = np.abs(Pm[a] - want)
        diff = np.minimum(diff, 20.0 - diff)
        assert diff.max() <= 2.0 ** -19


def test_rejects_inconsistent_hierarchy():
    p = np.zeros((3, 3), F32)
    with pytest.raises(oracle.OracleError):      # a parent cycle
        oracle.halo_props(*[p[:, k] for k in range(3)], *[p[:, k] for k in range(3)], 10.0,
                          np.array([1, 0], np.int32), np.array([0, 1], np.int32),
                          np.array([0, 1, 1], np.int32))
    with pytest.raises(oracle.OracleError):      # deepest out of range
        oracle.halo_props(*[p[:, k] for k in range(3)], *[p[:, k] for k in range(3)], 10.0,
                          np.array([-1], np.int32), np.array([0], np.int32),
                          np.array([0, 1, 0], np.int32))
