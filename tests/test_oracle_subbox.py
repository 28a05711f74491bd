"""Pins for the oracle's 3D FoF over a non-periodic sub-box with a ghost
shell (CPU only).

The paper's decomposition (Parallelization section) runs the 3D FoF per
sub-box and joins halos across sub-boxes through the boundary particles.
The oracle's sub-box FoF is pinned by the numpy brute force without the
periodic shift, by constructed cases, and by the decomposition itself: a
periodic box cut into slabs or octants, each run as a sub-box with its ghost
shell, and the per-sub-box labels and ghost links unioned on the host, must
give exactly the periodic FoF of the whole box.
"""
import numpy as np
import pytest

import brute
import decomp
import oracle
from paper_2412_18629_amd import synth

F32 = np.float32


def _random_subbox(seed, n_own=1500, n_ghost=600, clustered=False):
    rng = np.random.default_rng(seed)
    lo = np.array([2.0, 3.0, 1.0], F32)
    hi = np.array([6.0, 5.5, 4.0], F32)
    gw = F32(0.5)
    if clustered:
        cen = rng.uniform(lo, hi, (15, 3))
        own = cen[rng.integers(0, 15, n_own)] + rng.normal(0, 0.12, (n_own, 3))
        own = np.clip(own, lo, np.nextafter(hi, F32(0)))
    else:
        own = rng.uniform(lo, hi, (n_own, 3))
    own = own.astype(F32)
    own = np.minimum(own, np.nextafter(hi, F32(0)))
    g = rng.uniform(lo - gw, hi + gw, (4 * n_ghost, 3))
    g = g[~np.all((g >= lo) & (g < hi), axis=1)][:n_ghost].astype(F32)
    pos = np.concatenate([own, g])
    return pos, own.shape[0], lo, hi, gw


@pytest.mark.parametrize("seed,clustered", [(0, False), (1, False), (2, True), (3, True)])
def test_matches_brute_without_shift(seed, clustered):
    pos, no, lo, hi, gw = _random_subbox(seed, clustered=clustered)
    ll = F32(0.21)
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    ref = brute.fof3d(x, y, z, None, ll)
    lab, links = oracle.fof3d_subbox(x, y, z, no, lo, hi, gw, ll)
    assert np.array_equal(lab, ref)
    lab_b, _ = oracle.fof3d_subbox(x, y, z, no, lo, hi, gw, ll, brute=True)
    assert np.array_equal(lab_b, ref)
    # links: exactly the ghosts whose group holds an owned particle
    g = np.arange(no, pos.shape[0])
    want = g[ref[g] < no]
    assert np.array_equal(links[:, 0], want) and np.array_equal(links[:, 1], ref[want])
    assert links.shape[0] > 0


def test_no_periodic_shift_and_inclusive_threshold():
    lo = np.array([0.0, 0.0, 0.0], F32)
    hi = np.array([4.0, 4.0, 4.0], F32)
    # a pair at exactly ll links; a pair 4 - 0.1 apart (0.1 through a
    # periodic face of side 4) does not: there is no face here
    pos = np.array([[1.0, 1.0, 1.0], [1.25, 1.0, 1.0], [0.05, 2.0, 2.0], [3.95, 2.0, 2.0]], F32)
    lab, links = oracle.fof3d_subbox(pos[:, 0], pos[:, 1], pos[:, 2], 4, lo, hi, 0.0, 0.25)
    assert list(lab) == [0, 0, 2, 3]
    assert links.shape == (0, 2)


def test_rejects_positions_outside_their_region():
    lo = np.zeros(3, F32)
    hi = np.full(3, 4.0, F32)
    pos = np.array([[1.0, 1.0, 1.0], [4.2, 1.0, 1.0]], F32)
    # particle 1 owned but outside [lo, hi)
    with pytest.raises(oracle.OracleError):
        oracle.fof3d_subbox(pos[:, 0], pos[:, 1], pos[:, 2], 2, lo, hi, 0.5, 0.2)
    # as a ghost it is inside the shell; beyond the shell it is not
    oracle.fof3d_subbox(pos[:, 0], pos[:, 1], pos[:, 2], 1, lo, hi, 0.5, 0.2)
    pos[1, 0] = 4.6
    with pytest.raises(oracle.OracleError):
        oracle.fof3d_subbox(pos[:, 0], pos[:, 1], pos[:, 2], 1, lo, hi, 0.5, 0.2)


def _decomposition(parts, n=12000, seed=0):
    cfg = synth.scaled(synth.CONFIGS["c32"], n)
    arrs = synth.generate(cfg, seed)
    L = F32(20.0)
    pos = decomp.snap(np.stack([a.numpy() for a in arrs[:3]], 1), 20.0)
    ll = F32(cfg.link_len)
    whole = oracle.fof3d(pos[:, 0], pos[:, 1], pos[:, 2], L, ll)
    res = []
    for lo, hi in decomp.split(20.0, parts):
        lp, gid, no = decomp.subbox_inputs(pos, L, lo, hi, 1.5 * float(ll))
        lab, links = oracle.fof3d_subbox(lp[:, 0], lp[:, 1], lp[:, 2], no, lo, hi,
                                         1.5 * float(ll), ll)
        res.append((gid, no, lab, links))
    return whole, decomp.union_subboxes(pos.shape[0], res)


@pytest.mark.parametrize("parts", [(2, 1, 1), (2, 2, 2), (1, 3, 1)])
def test_decomposition_reproduces_the_periodic_box(parts):
    whole, joined = _decomposition(parts)
    assert np.array_equal(joined, whole)


@pytest.mark.parametrize("seed,clustered", [(4, False), (5, True), (6, True)])
def test_small_cell_grid_matches_coarse_and_brute(seed, clustered):
    # the small-cell grid of the sub-box against the coarse grid and all
    # pairs, on sub-boxes with dense clumps (same-cell linking) and faces
    pos, no, lo, hi, gw = _random_subbox(seed, n_own=6000, n_ghost=1500, clustered=clustered)
    ll = F32(0.17)
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    ref = brute.fof3d(x, y, z, None, ll)
    for grid in ("auto", "coarse"):
        lab, _ = oracle.fof3d_subbox(x, y, z, no, lo, hi, gw, ll, grid=grid)
        assert np.array_equal(lab, ref), grid


@pytest.mark.parametrize("ll", [0.2, 0.175, 0.5])
def test_small_cell_linking_stays_inside_ll(ll):
    # pairs along the diagonal of the cells of every grid the sub-box could
    # plausibly use (around E sqrt(3) / ll cells of side E / nc from the
    # shell's corner), separated by between 0.995 ll and the cell's diagonal
    # (or 1.005 ll), all owned: same-cell linking may only join pairs the pair
    # test joins (a cell whose diagonal exceeds ll would link pairs farther
    # apart than ll)
    ll = F32(ll)
    lo = np.array([1.0, 1.0, 1.0], F32)
    hi = np.array([9.0, 9.0, 9.0], F32)
    gw = F32(0.5)
    o = lo.astype(np.float64) - float(gw)
    E = float(hi[0]) + float(gw) - o[0]
    rng = np.random.default_rng(int(float(ll) * 1000))
    pts = []
    n0 = int(round(E * np.sqrt(3.0) / float(ll)))
    for nc in range(n0 - 2, n0 + 3):
        side = E / nc
        k = int(np.ceil((float(gw) + 1.0) / side))   # cells kept clear of the shell
        top = max(side * np.sqrt(3.0) / float(ll), 1.005)
        for f in np.linspace(0.995, top, 24):
            c = rng.integers(k, nc - k, 3)
            p = o + c * side + 2e-6 * side
            pts += [p, p + float(ll) * f / np.sqrt(3.0)]
    pos = np.array(pts).astype(F32)
    assert np.all((pos >= lo) & (pos < hi))
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    ref = brute.fof3d(x, y, z, None, ll)
    lab, _ = oracle.fof3d_subbox(x, y, z, pos.shape[0], lo, hi, gw, ll)
    assert np.array_equal(lab, ref)
    linked = ref[0::2] == ref[1::2]
    assert linked.any() and not linked.all()
