"""Pins for the oracle's hierarchical 6D phase-space FoF (CPU only).

The paper names the step (subhalo finding per FoF halo in 6D phase space,
Parallelization section) and defers the method to the Rockstar paper it
cites; the readings used (dispersion normalisation, nearest-neighbour
percentile, recursion) are listed with the oracle.  Pins: an independent
numpy/scipy brute force, exact rational dispersions, closed-form node
layouts whose tree is known by construction, and invariances.
"""
import random
from fractions import Fraction

import numpy as np
import pytest

import brute
import oracle
from paper_2412_18629_amd import synth

F32 = np.float32


def _np(ts):
    return [t.numpy() for t in ts]


def test_i128_to_f64_is_correctly_rounded():
    rnd = random.Random(7)
    vals = [0, 1, -1, 2 ** 53 + 1, 2 ** 64 - 1, -(2 ** 100) - 12345, 2 ** 117 + 2 ** 64 + 1,
            (1 << 127) - 1, -(1 << 127)]
    # halfway cases: 2^60 + 2^7 is exactly between two doubles (ulp 2^8)
    vals += [2 ** 60 + 2 ** 7, 2 ** 60 + 3 * 2 ** 7, -(2 ** 90 + 2 ** 37)]
    for _ in range(3000):
        b = rnd.randrange(1, 127)
        vals.append(rnd.randrange(-(1 << b), 1 << b))
    for v in vals:
        assert oracle.i128_to_f64(v) == float(v), v


def test_select_rank_is_ceil_fn():
    for n in list(range(1, 300)) + [10 ** 6 + 7, 2 ** 31 - 1]:
        for f in (0.7, 0.5, 1.0, 0.123456, 1e-6):
            want = max(1, min(n, -((-n * Fraction(round(f * 1e6), 10 ** 6)).__floor__())))
            want = max(1, min(n, int(-(-Fraction(n) * Fraction(round(f * 1e6), 10 ** 6) // 1))))
            assert oracle.select_rank(n, f) == want


def test_two_particle_dispersion_closed_form():
    # sigma^2 of two points is |delta|^2 / 4
    x = np.array([1.0, 1.5], F32); y = np.array([2.0, 2.0], F32); z = np.array([3.0, 3.0], F32)
    vx = np.array([10.0, 12.0], F32); vy = np.zeros(2, F32); vz = np.zeros(2, F32)
    a, c, sx2, sv2 = oracle.node_norm(x, y, z, vx, vy, vz, 8.0, [0, 1])
    assert sx2 == 0.0625 and a == 16.0
    assert sv2 == 1.0 and c == 1.0
    # across the periodic face: 7.875 and 0.125 are 0.25 apart in a box of 8
    x = np.array([7.875, 0.125], F32)
    a, c, sx2, sv2 = oracle.node_norm(x, y, z, vx, vy, vz, 8.0, [0, 1])
    assert sx2 == 2.0 ** -6 and a == 64.0


@pytest.mark.parametrize("seed", range(8))
def test_metric_factors_match_exact_rational(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 400))
    L = F32(rng.choice([20.0, 160.0, 640.0]))
    cen = rng.uniform(0, float(L), 3)
    pos = np.mod(cen + rng.normal(0, rng.uniform(0.01, 3.0), (n, 3)), float(L)).astype(F32)
    pos[pos >= L] = 0
    vel = rng.normal(0, rng.uniform(1, 800), (n, 3)).astype(F32)
    a, c, sx2, sv2 = oracle.node_norm(*pos.T, *vel.T, L, np.arange(n))
    ea, ec = brute.metric_factors(pos, vel, L)
    assert a == ea and c == ec
    # and within one fp32 rounding of the exact 1/sigma^2
    sx, sv = brute.exact_dispersions(pos, vel, L)
    exact_a = float(Fraction(2 ** 40) / sx)
    exact_c = float(Fraction(2 ** 20) / sv)
    assert abs(a - exact_a) <= float(np.spacing(F32(a)))
    assert abs(c - exact_c) <= float(np.spacing(F32(c)))


def _compare(res, nodes, deepest):
    assert len(res["level"]) == len(nodes)
    for i, d in enumerate(nodes):
        assert res["level"][i] == d["level"]
        assert res["min_index"][i] == d["min_index"]
        assert res["size"][i] == d["size"]
        assert res["parent"][i] == d["parent"]
        assert res["a"][i] == d["a"] and res["c"][i] == d["c"]
        assert res["l2"][i] == d["l2"], (i, res["l2"][i], d["l2"])
    assert np.array_equal(res["deepest"], deepest)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("brute_max", [100000, 0])
def test_hierarchy_matches_brute_small(seed, brute_max):
    cfg = synth.scaled(synth.CONFIGS["c32"], 3000)
    x, y, z, vx, vy, vz = _np(synth.generate(cfg, 10 + seed))
    lab = oracle.fof3d(x, y, z, cfg.box, cfg.link_len)
    res = oracle.phase_fof(x, y, z, vx, vy, vz, cfg.box, lab, brute_max=brute_max)
    nodes, deepest = brute.phase_fof(x, y, z, vx, vy, vz, cfg.box, lab)
    assert len(nodes) > 3
    _compare(res, nodes, deepest)


@pytest.mark.slow
def test_full_32cubed_matches_brute():
    cfg = synth.CONFIGS["c32"]
    x, y, z, vx, vy, vz = _np(synth.generate(cfg, 0))
    lab = oracle.fof3d(x, y, z, cfg.box, cfg.link_len)
    res = oracle.phase_fof(x, y, z, vx, vy, vz, cfg.box, lab, brute_max=500)
    nodes, deepest = brute.phase_fof(x, y, z, vx, vy, vz, cfg.box, lab)
    _compare(res, nodes, deepest)


def _single_group(pos, vel, L, **kw):
    pos = np.asarray(pos, F32); vel = np.asarray(vel, F32)
    lab = np.zeros(pos.shape[0], np.int32)
    return oracle.phase_fof(*pos.T, *vel.T, L, lab, **kw)


def test_line_lattice_all_equal_nn_is_leaf():
    # 1D lattice, zero velocities: every NN distance is the spacing, so l^2 is
    # a * fl(s^2) with c = 1 (sigma_v = 0); all pairs at l link into one
    # component equal to the node, which is therefore a leaf
    n, s = 40, 0.125
    pos = np.zeros((n, 3)); pos[:, 0] = 1.0 + s * np.arange(n); pos[:, 1] = 2.0; pos[:, 2] = 3.0
    res = _single_group(pos, np.zeros((n, 3)), 16.0)
    assert len(res["level"]) == 1
    assert res["c"][0] == 1.0 and res["sv2"][0] == 0.0
    assert res["l2"][0] == F32(res["a"][0]) * F32(s * s)
    # sigma_x^2 of a uniform line of n points with spacing s: s^2 (n^2-1)/12
    assert res["sx2"][0] == F32(s * s * (n * n - 1) / 12.0)


def test_clumps_separated_in_velocity_split_at_level_one():
    rng = np.random.default_rng(3)
    m = 120
    pos = np.concatenate([5.0 + rng.normal(0, 0.05, (m, 3)) for _ in range(3)])
    vel = np.concatenate([rng.normal(0, 10.0, (m, 3)) + [4000.0 * k, 0, 0] for k in range(3)])
    res = _single_group(pos, vel, 20.0)
    lev1 = np.nonzero(res["level"] == 1)[0]
    assert res["level"][0] == 0 and res["size"][0] == 3 * m
    clump_of = np.repeat(np.arange(3), m)
    seen = set()
    for i in lev1:
        assert res["parent"][i] == 0
        members = np.nonzero(_members_of(res, i))[0]
        owners = set(clump_of[members].tolist())
        assert len(owners) == 1          # no child mixes clumps
        seen |= owners
    assert seen == {0, 1, 2}


def _members_of(res, node):
    """Boolean membership of ``node`` reconstructed from deepest + parents."""
    n = res["deepest"].size
    out = np.zeros(n, bool)
    for i in range(n):
        d = res["deepest"][i]
        while d >= 0:
            if d == node:
                out[i] = True
                break
            d = res["parent"][d]
    return out


def test_duplicates_give_zero_linking_length():
    # 8 exact duplicate pairs + 4 distinct points: k = ceil(0.7*20) = 14 <= 16
    rng = np.random.default_rng(1)
    base = 3.0 + rng.uniform(0, 0.1, (12, 3))
    vb = rng.normal(0, 50, (12, 3))
    pos = np.concatenate([base[:8], base[:8], base[8:]])
    vel = np.concatenate([vb[:8], vb[:8], vb[8:]])
    res = _single_group(pos, vel, 10.0)
    assert res["l2"][0] == 0.0
    assert len(res["level"]) == 1          # duplicate pairs (size 2) are no subgroups


def test_zero_dispersion():
    pos = np.full((15, 3), 2.5); vel = np.full((15, 3), 7.0)
    res = _single_group(pos, vel, 10.0)
    assert res["a"][0] == 1.0 and res["c"][0] == 1.0
    assert res["sx2"][0] == 0.0 and res["sv2"][0] == 0.0
    assert res["l2"][0] == 0.0 and len(res["level"]) == 1


def _node_sets(res):
    n = res["deepest"].size
    sets = []
    for node in range(len(res["level"])):
        sets.append(frozenset(np.nonzero(_members_of(res, node))[0].tolist()))
    return sets


def test_invariants_32cubed():
    cfg = synth.CONFIGS["c32"]
    x, y, z, vx, vy, vz = _np(synth.generate(cfg, 0))
    lab = oracle.fof3d(x, y, z, cfg.box, cfg.link_len)
    res = oracle.phase_fof(x, y, z, vx, vy, vz, cfg.box, lab)
    keys = list(zip(res["level"].tolist(), res["min_index"].tolist()))
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    sets = _node_sets(res)
    pos = np.stack([x, y, z], 1); vel = np.stack([vx, vy, vz], 1)
    for i in range(len(keys)):
        mem = np.array(sorted(sets[i]))
        assert mem.size == res["size"][i] and mem[0] == res["min_index"][i]
        if res["level"][i] == 0:
            assert res["parent"][i] == -1 and mem.size >= 10
            assert np.all(lab[mem] == lab[mem[0]])
        else:
            p = res["parent"][i]
            assert res["level"][p] == res["level"][i] - 1
            assert sets[i] < sets[p] and mem.size >= 10
        # linked fraction at the chosen length: #(d < l) < k <= #(d <= l)
        if mem.size <= 1500:
            Dx = brute.pos_d2_matrix(*pos[mem].T, cfg.box)
            Dv = brute.vel_d2_matrix(*vel[mem].T)
            d2 = (res["a"][i] * Dx) + (res["c"][i] * Dv)
            np.fill_diagonal(d2, np.inf)
            nn = d2.min(1)
            k = brute.select_rank(mem.size, 0.7)
            assert (nn < res["l2"][i]).sum() < k <= (nn <= res["l2"][i]).sum()
    # depth bound: children hold at most k members without ties
    assert res["level"].max() <= int(np.log(4200 / 10) / np.log(1 / 0.7)) + 1


def test_permutation_invariance_bit_exact():
    cfg = synth.scaled(synth.CONFIGS["c32"], 6000)
    x, y, z, vx, vy, vz = _np(synth.generate(cfg, 4))
    lab = oracle.fof3d(x, y, z, cfg.box, cfg.link_len)
    res = oracle.phase_fof(x, y, z, vx, vy, vz, cfg.box, lab)
    perm = np.random.default_rng(9).permutation(x.size)
    arrs = [a[perm] for a in (x, y, z, vx, vy, vz)]
    lab_p = oracle.fof3d(*arrs[:3], cfg.box, cfg.link_len)
    res_p = oracle.phase_fof(*arrs, cfg.box, lab_p)
    s0 = {frozenset(s): (l2, a, c) for s, l2, a, c in
          zip(_node_sets(res), res["l2"], res["a"], res["c"])}
    s1 = {frozenset(perm[list(s)].tolist()): (l2, a, c) for s, l2, a, c in
          zip(_node_sets(res_p), res_p["l2"], res_p["a"], res_p["c"])}
    assert s0 == s1


def test_translation_invariance_on_dyadic_grid():
    cfg = synth.scaled(synth.CONFIGS["c32"], 5000)
    x, y, z, vx, vy, vz = _np(synth.generate(cfg, 5))
    q = 2.0 ** -12
    L = F32(cfg.box)
    # snap the box and positions to the grid (box side itself a grid multiple)
    Lg = float(np.round(cfg.box / q) * q)
    snap = [np.mod(np.round(a.astype(np.float64) / q) * q, Lg).astype(F32) for a in (x, y, z)]
    lab = oracle.fof3d(*snap, Lg, cfg.link_len)
    res = oracle.phase_fof(*snap, vx, vy, vz, Lg, lab)
    shift = [1.5 + 3 * q, 4.25 + 17 * q, 2.0 + q]
    moved = [np.mod(a.astype(np.float64) + t, Lg).astype(F32) for a, t in zip(snap, shift)]
    lab_m = oracle.fof3d(*moved, Lg, cfg.link_len)
    res_m = oracle.phase_fof(*moved, vx, vy, vz, Lg, lab_m)
    for k in ("level", "min_index", "parent", "size", "l2", "a", "c", "sx2", "sv2"):
        assert np.array_equal(res[k], res_m[k]), k
    assert np.array_equal(res["deepest"], res_m["deepest"])


def _chain(x0, steps, L):
    """Particles 0.125 apart along x from x0 (wrapped into [0, L)) at fixed
    y, z, in index order along the chain; the second half moves at 3000 km/s,
    the first is at rest, so every pair within a half ties at the linking
    length and the 6D pass splits the group into its two halves."""
    xs = np.mod(x0 + 0.125 * np.arange(steps + 1), L)
    pos = np.stack([xs, np.full_like(xs, 2.0), np.full_like(xs, 3.0)], 1).astype(F32)
    vel = np.zeros((steps + 1, 3))
    vel[(steps + 1) // 2:, 0] = 3000.0
    return pos, vel.astype(F32)


@pytest.mark.parametrize("x0,steps,expect", [(1.0, 40, 1), (1.0, 39, 0), (8.0, 32, 0),
                                             (8.0, 48, 1)])
def test_percolation_flag_chain_extent(x0, steps, expect):
    # a chain of extent 0.125 * steps in a box of side 10: 5.0 (half the box)
    # sets the flag, 4.875 does not; a chain across the periodic face is
    # measured in the nearest image (4.0 clear, 6.0 set); every node of the
    # group's hierarchy carries the group's flag
    L = 10.0
    pos, vel = _chain(x0, steps, L)
    lab = oracle.fof3d(*pos.T, L, 0.2)
    assert np.all(lab == lab[0])
    res = oracle.phase_fof(*pos.T, *vel.T, L, lab)
    assert res["level"].max() >= 1
    assert res["wide"][0] == expect
    assert np.all(res["wide"] == expect)


def test_percolation_flag_clear_for_compact_groups():
    # the 32^3 workload's haloes are far smaller than half its box
    cfg = synth.CONFIGS["c32"]
    x, y, z, vx, vy, vz = _np(synth.generate(cfg, 0))
    lab = oracle.fof3d(x, y, z, cfg.box, cfg.link_len)
    res = oracle.phase_fof(x, y, z, vx, vy, vz, cfg.box, lab)
    assert res["level"].size > 0 and not res["wide"].any()
