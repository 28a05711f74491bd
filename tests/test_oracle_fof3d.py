"""Pins for the oracle's 3D friends-of-friends (CPU only).

The paper fixes the step (each process runs a 3D FoF over its sub-box,
Parallelization section) but prints no output values, so the oracle is
pinned by brute force on small inputs, by an independent periodic k-d tree
closure on the full 32^3 workload, by constructed cases whose answer is
known, and by invariances of the definition.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import brute
import oracle
from paper_2412_18629_amd import synth

F32 = np.float32


def _np(ts):
    return [t.numpy() for t in ts]


def same_partition(a, b):
    """Two label arrays describe the same partition."""
    a = np.asarray(a); b = np.asarray(b)
    fwd = {}
    for u, v in zip(a.tolist(), b.tolist()):
        if fwd.setdefault(u, v) != v:
            return False
    return len(set(fwd.values())) == len(fwd)


@pytest.mark.parametrize("seed", range(6))
def test_random_uniform_matches_brute(seed):
    rng = np.random.default_rng(seed)
    n = 1500
    L = F32(6.0)
    pos = (rng.random((n, 3)) * 6.0).astype(F32)
    pos[pos >= L] = 0
    ll = F32(rng.uniform(0.25, 0.45))
    got = oracle.fof3d(pos[:, 0], pos[:, 1], pos[:, 2], L, ll)
    ref = brute.fof3d(pos[:, 0], pos[:, 1], pos[:, 2], L, ll)
    assert np.array_equal(got, ref)
    got_b = oracle.fof3d(pos[:, 0], pos[:, 1], pos[:, 2], L, ll, brute=True)
    assert np.array_equal(got_b, ref)


@pytest.mark.parametrize("seed", range(3))
def test_clustered_matches_brute(seed):
    cfg = synth.scaled(synth.CONFIGS["c32"], 2500)
    x, y, z, *_ = _np(synth.generate(cfg, seed))
    got = oracle.fof3d(x, y, z, cfg.box, cfg.link_len)
    ref = brute.fof3d(x, y, z, cfg.box, cfg.link_len)
    assert np.array_equal(got, ref)


def _kdtree_labels(x, y, z, L, ll):
    """Closure of the fp32 pair relation, candidate pairs from a periodic
    k-d tree (scipy) with a generous radius, then the exact fp32 test."""
    pos = np.stack([x, y, z], 1).astype(np.float64)
    tree = cKDTree(pos, boxsize=float(L))
    pairs = tree.query_pairs(float(ll) * 1.001, output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    L32 = F32(L); h = F32(0.5) * L32

    def w(d):
        return np.where(d > h, d - L32, np.where(d < -h, d + L32, d)).astype(F32)
    dx = w(x[i] - x[j]); dy = w(y[i] - y[j]); dz = w(z[i] - z[j])
    D = ((dx * dx) + (dy * dy)) + (dz * dz)
    keep = D <= F32(ll) * F32(ll)
    n = x.size
    g = coo_matrix((np.ones(keep.sum()), (i[keep], j[keep])), shape=(n, n))
    nc, comp = connected_components(g, directed=False)
    first = np.full(nc, n, np.int64)
    np.minimum.at(first, comp, np.arange(n))
    return first[comp]


def test_full_32cubed_matches_kdtree_closure():
    cfg = synth.CONFIGS["c32"]
    x, y, z, *_ = _np(synth.generate(cfg, 0))
    got = oracle.fof3d(x, y, z, cfg.box, cfg.link_len)
    ref = _kdtree_labels(x, y, z, cfg.box, cfg.link_len)
    assert np.array_equal(got, ref)
    # labels are the smallest member index of each group
    assert np.all(got <= np.arange(x.size))
    assert np.all(got[got] == got)


def test_lattice_links_at_exact_spacing():
    # dyadic cubic lattice, spacing 0.5 in a periodic box of 8: neighbours at
    # D = 0.25 exactly; ll = 0.5 links everything, the next float down nothing
    s = 0.5
    g = np.arange(16, dtype=np.float64) * s + 0.125
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = (a.ravel().astype(F32) for a in (X, Y, Z))
    one = oracle.fof3d(x, y, z, 8.0, 0.5)
    assert np.all(one == 0)
    none = oracle.fof3d(x, y, z, 8.0, np.nextafter(F32(0.5), F32(0)))
    assert np.array_equal(none, np.arange(x.size))


def test_pair_at_threshold_inclusive():
    L, ll = F32(4.0), F32(0.25)
    x = np.array([1.0, 1.25], F32); y = np.array([2.0, 2.0], F32); z = np.array([3.0, 3.0], F32)
    assert list(oracle.fof3d(x, y, z, L, ll)) == [0, 0]
    x[1] = np.nextafter(F32(1.25), F32(2))
    assert list(oracle.fof3d(x, y, z, L, ll)) == [0, 1]
    # a diagonal pair whose fp32 D lands exactly on ll^2 = 0.0625:
    # (0.125, 0.125, 0.125*sqrt2 rounded) is decided by the fp32 formula
    x = np.array([0.5, 0.625], F32); y = np.array([0.5, 0.625], F32)
    z = np.array([0.5, 0.5 + 0.17677669], F32)
    ref = brute.fof3d(x, y, z, L, ll)
    assert np.array_equal(oracle.fof3d(x, y, z, L, ll), ref)


def test_pair_across_periodic_face():
    L, ll = F32(10.0), F32(0.2)
    x = np.array([0.05, 9.9, 5.0], F32)
    y = np.array([3.0, 3.0, 3.0], F32)
    z = np.array([9.95, 0.04, 1.0], F32)
    assert list(oracle.fof3d(x, y, z, L, ll)) == [0, 0, 2]


def test_separated_clumps_one_group_each():
    rng = np.random.default_rng(5)
    L = F32(16.0)
    centres = np.array([[2, 2, 2], [6, 2, 9], [12, 12, 3], [8, 8, 8]], np.float64)
    pts, truth = [], []
    for c, cen in enumerate(centres):
        p = cen + rng.uniform(-0.04, 0.04, (50, 3))   # diameter < ll: one group
        pts.append(p); truth += [c] * 50
    pos = np.concatenate(pts).astype(F32)
    perm = rng.permutation(len(pos))
    pos = pos[perm]; truth = np.array(truth)[perm]
    lab = oracle.fof3d(pos[:, 0], pos[:, 1], pos[:, 2], L, F32(0.2))
    assert same_partition(lab, truth)
    for c in range(4):
        assert np.all(lab[truth == c] == np.nonzero(truth == c)[0].min())


def test_permutation_invariance():
    cfg = synth.CONFIGS["c32"]
    x, y, z, *_ = _np(synth.generate(cfg, 1))
    lab = oracle.fof3d(x, y, z, cfg.box, cfg.link_len)
    perm = np.random.default_rng(0).permutation(x.size)
    lab_p = oracle.fof3d(x[perm], y[perm], z[perm], cfg.box, cfg.link_len)
    assert same_partition(lab[perm], lab_p)


def test_periodic_translation_invariance_on_dyadic_grid():
    # positions on a 2^-12 grid in a box of 20: every difference is exact in
    # fp32, so a translation by a grid multiple (mod L) changes no distance
    cfg = synth.CONFIGS["c32"]
    x, y, z, *_ = _np(synth.generate(cfg, 2))
    q = 2.0 ** -12
    snap = [np.mod(np.round(a.astype(np.float64) / q) * q, 20.0).astype(F32) for a in (x, y, z)]
    lab = oracle.fof3d(*snap, 20.0, cfg.link_len)
    shift = [7.25 + 3 * q, 13.5 + 11 * q, 0.75 + 5 * q]
    moved = [np.mod(a.astype(np.float64) + t, 20.0).astype(F32) for a, t in zip(snap, shift)]
    lab_m = oracle.fof3d(*moved, 20.0, cfg.link_len)
    assert np.array_equal(lab, lab_m)


def test_rejects_out_of_range():
    x = np.array([0.0, 1.0], F32)
    with pytest.raises(oracle.OracleError):
        oracle.fof3d(x, x, np.array([0.0, 4.0], F32), 4.0, 0.2)
    with pytest.raises(oracle.OracleError):
        oracle.fof3d(x, x, np.array([0.0, np.nan], F32), 4.0, 0.2)


# Grid margin (cell side >= ll (1 + 2^-20) + L 2^-22): pairs at the edge of
# the linking test, where a cell grid can miss a pair whose computed D <= ll^2.
# L / ll lies within two fp32 steps of an integer, so neighbouring cell counts
# are one rounding apart; pairs straddle the periodic face (where the image
# shift rounds the separation to the ulp grid of L, linking some pairs whose
# true separation exceeds ll and separating some within it) and the interior
# cell boundaries of the grids next to L / ll.  The grid must agree with all
# pairs (the oracle's own brute path and the independent numpy brute force).
EDGE_CASES = [(20.0, [57, 100, 333], [0.2875, 0.25]), (320.0, [1829, 1000, 257], [0.175, 0.3125]),
              (640.0, [3657], [0.175, 0.625]), (100.0, [7, 50], [0.3, 0.78125])]


@pytest.mark.parametrize("L,counts,plain", EDGE_CASES)
def test_grid_margin_edge_pairs(L, counts, plain):
    import edge_pairs as ep
    rounded_in = rounded_out = 0
    lls = np.concatenate([ep.near_integer_ratio_lengths(L, counts, 6), np.array(plain, F32)])
    for ll in lls:
        pos, pairs = ep.edge_pair_box(L, ll, seed=int(float(ll) * 1e6) % 1000)
        x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
        ref = brute.fof3d(x, y, z, L, ll)
        assert np.array_equal(oracle.fof3d(x, y, z, L, ll), ref), (L, ll)
        assert np.array_equal(oracle.fof3d(x, y, z, L, ll, grid="coarse"), ref), (L, ll)
        assert np.array_equal(oracle.fof3d(x, y, z, L, ll, brute=True), ref), (L, ll)
        sep = ep.true_separation(pos, pairs, L)
        linked = ref[pairs[:, 0]] == ref[pairs[:, 1]]
        rounded_in += int((linked & (sep > float(ll))).sum())
        rounded_out += int((~linked & (sep <= float(ll))).sum())
    # the rounding of the image shift decides some pairs either way: the
    # construction reaches the cases the margin is about
    assert rounded_in > 0 or rounded_out > 0


@pytest.mark.parametrize("L,ll", [(20.0, 0.2), (320.0, 0.175), (17.0, 0.5)])
def test_same_cell_linking_stays_inside_ll(L, ll):
    # for every cell count a small-cell grid could plausibly use (around
    # L sqrt(3) / ll), pairs along the diagonal of its cells, from a corner,
    # separated by between 0.995 ll and the cell's diagonal (or 1.005 ll):
    # whichever of these grids the oracle uses, same-cell linking may only
    # join pairs the pair test joins (a cell whose diagonal exceeds ll would
    # link pairs farther apart than ll)
    L, ll = F32(L), F32(ll)
    rng = np.random.default_rng(int(L))
    pts = []
    n0 = int(round(float(L) * np.sqrt(3.0) / float(ll)))
    for nc in range(n0 - 2, n0 + 3):
        side = float(L) / nc
        top = max(side * np.sqrt(3.0) / float(ll), 1.005)
        for f in np.linspace(0.995, top, 24):
            c = rng.integers(2, nc - 3, 3)
            p = c * side + 2e-6 * side
            pts += [p, p + float(ll) * f / np.sqrt(3.0)]
    pos = np.array(pts).astype(F32)
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    ref = brute.fof3d(x, y, z, L, ll)
    assert np.array_equal(oracle.fof3d(x, y, z, L, ll), ref)
    linked = ref[0::2] == ref[1::2]
    assert linked.any() and not linked.all()


@pytest.mark.parametrize("seed", range(3))
def test_dense_clumps_fine_and_coarse_grids(seed):
    # dense cores (many particles per small cell): same-cell linking and the
    # early exit between cells against the coarse grid and all pairs
    rng = np.random.default_rng(40 + seed)
    L = F32(10.0)
    cen = rng.random((6, 3)) * 10
    pos = np.mod(cen[rng.integers(0, 6, 3000)] + rng.normal(0, 0.05 + 0.1 * seed, (3000, 3)),
                 10.0).astype(F32)
    pos[pos >= L] = 0
    ll = F32(0.1)
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    ref = brute.fof3d(x, y, z, L, ll)
    assert np.array_equal(oracle.fof3d(x, y, z, L, ll), ref)
    assert np.array_equal(oracle.fof3d(x, y, z, L, ll, grid="coarse"), ref)
