"""Checks of a whole (3D labels, 6D tree) result at any size, against the
oracle in parts it can compute one at a time.  Shared by the full-size GPU
test and a CPU test that runs them on the oracle's own result.

R is a dict of host arrays:
  host          (x, y, z, vx, vy, vz) float32 [n]
  labels        3D labels [n]
  sorted_labels labels sorted ascending; order: the stable sort permutation
  cperm, cstart coarse periodic cell lists (cell side >= ll; nc per axis)
  nc, side      cells per axis and cell side
  tree          node fields and deepest
  props, halo   (optional) rs_halo_props rows [15, nodes] and rs_seed_assign [n]
"""
from concurrent.futures import ThreadPoolExecutor
from concurrent.futures import TimeoutError as FuturesTimeout

import numpy as np

import oracle

FIELDS = ("level", "min_index", "parent", "size", "l2", "a", "c", "sx2", "sv2", "wide")
WORKERS = 16


def cell_lists_numpy(x, y, z, box):
    """Coarse periodic cell lists on the host (cell side >= 2 length units)."""
    nc = max(1, int(box // 2.0))
    side = box / nc
    c = [np.clip(np.floor(a.astype(np.float64) / side).astype(np.int64), 0, nc - 1)
         for a in (x, y, z)]
    key = (c[0] * nc + c[1]) * nc + c[2]
    cperm = np.argsort(key, kind="stable")
    cstart = np.searchsorted(key[cperm], np.arange(nc ** 3 + 1))
    return cperm, cstart, nc, side


def members(R, g):
    lo = np.searchsorted(R["sorted_labels"], g, side="left")
    hi = np.searchsorted(R["sorted_labels"], g, side="right")
    return np.sort(R["order"][lo:hi])


def region(R, cfg, mem):
    """Indices of every particle inside the members' bounding box (positions
    unwrapped around the first member) grown by the linking length: a
    superset of the group and of every particle within ll of it."""
    L, nc, side = cfg.box, R["nc"], R["side"]
    rng = []
    for d in range(3):
        x = R["host"][d][mem].astype(np.float64)
        u = x - x[0]
        u = np.where(u >= L / 2, u - L, np.where(u < -L / 2, u + L, u)) + x[0]
        lo = int(np.floor((u.min() - cfg.link_len) / side))
        hi = int(np.floor((u.max() + cfg.link_len) / side))
        if hi - lo + 1 >= nc:
            rng.append(np.arange(nc))
        else:
            rng.append(np.arange(lo, hi + 1) % nc)
    cx, cy, cz = np.meshgrid(*rng, indexing="ij")
    cells = ((cx * nc + cy) * nc + cz).ravel()
    st, en = R["cstart"][cells], R["cstart"][cells + 1]
    idx = np.concatenate([R["cperm"][a:b] for a, b in zip(st, en)])
    return np.sort(idx)


def check_3d(R, cfg, g):
    """The group labelled g is closed and connected: in the oracle FoF of its
    grown bounding region, its first member's component is exactly it."""
    mem = members(R, g)
    reg = region(R, cfg, mem)
    h = R["host"]
    lab = oracle.fof3d(h[0][reg], h[1][reg], h[2][reg], cfg.box, cfg.link_len)
    pos = np.searchsorted(reg, mem)
    assert np.array_equal(reg[pos], mem)
    got = reg[lab == lab[pos[0]]]
    return np.array_equal(got, mem), int(g), int(mem.size), int(reg.size)


def check_subtree(R, cfg, g, root_of, canon_root):
    """The subtree of group g equals the oracle hierarchy of its member set;
    with props and halo in R, its nodes' halo properties and its particles'
    seeds equal the oracle's, computed from the oracle's hierarchy."""
    mem = members(R, g)
    h = R["host"]
    ref = oracle.phase_fof(*[a[mem] for a in h], cfg.box, np.zeros(mem.size, np.int32),
                           cfg.min_group, cfg.min_sub, cfg.f)
    T = R["tree"]
    sub = np.flatnonzero(root_of == canon_root[g])
    if sub.size != ref["level"].size:
        return [f"group {g}: {sub.size} nodes, oracle {ref['level'].size}"]
    bad = []
    for k in ("level", "size", "l2", "a", "c", "sx2", "sv2", "wide"):
        if not np.array_equal(T[k][sub], ref[k]):
            bad.append(f"group {g}: field {k}")
    if not np.array_equal(T["min_index"][sub], mem[ref["min_index"]]):
        bad.append(f"group {g}: min_index")
    where = np.full(T["level"].size, -1, np.int64)
    where[sub] = np.arange(sub.size)
    par = np.where(T["parent"][sub] < 0, -1, where[np.maximum(T["parent"][sub], 0)])
    if not np.array_equal(par, ref["parent"]):
        bad.append(f"group {g}: parent")
    if not np.array_equal(where[T["deepest"][mem]], ref["deepest"]):
        bad.append(f"group {g}: deepest")
    if bad or "props" not in R:
        return bad
    # halo properties and seeds of the subtree, from the oracle's own hierarchy
    sub_h = [a[mem] for a in h]
    P = oracle.halo_props(*sub_h, cfg.box, ref["parent"], ref["min_index"], ref["deepest"])
    if not np.array_equal(R["props"][:, sub].view(np.int32), P.view(np.int32)):
        bad.append(f"group {g}: halo properties")
    seeds = oracle.seed_assign(*sub_h, cfg.box, ref["parent"], ref["deepest"], ref["a"],
                               ref["c"], P)
    if not np.array_equal(R["halo"][mem], sub[seeds]):
        bad.append(f"group {g}: seeds")
    return bad


def stratified(sizes, groups, n_pick, min_group, seed=0):
    """n_pick groups spread over 10 equal-width bins of log10(size) between
    min_group and the largest size, round-robin over non-empty bins."""
    rng = np.random.default_rng(seed)
    lg = np.log10(sizes)
    edges = np.linspace(np.log10(min_group), lg.max() + 1e-9, 11)
    b = np.clip(np.digitize(lg, edges) - 1, 0, 9)
    bins = [np.flatnonzero(b == i) for i in range(10)]
    quota = [0] * 10
    left = n_pick
    while left > 0 and any(quota[i] < bins[i].size for i in range(10)):
        for i in range(10):
            if left > 0 and quota[i] < bins[i].size:
                quota[i] += 1
                left -= 1
    pick = [rng.choice(bins[i], quota[i], replace=False) for i in range(10) if quota[i]]
    return groups[np.concatenate(pick)]


def _gather(ex, futs, what, log):
    """Results of the futures in order, with a progress line every 30 s."""
    out = []
    for k, f in enumerate(futs):
        while True:
            try:
                out.append(f.result(timeout=30))
                break
            except FuturesTimeout:
                log(f"{what} checks: {k} of {len(futs)} done")
    return out


def check_all(R, cfg, n_sample=64, subtree_max=150000, closure_max=None, log=print):
    """Structural invariants of the whole tree, level-0 moments of every
    group, 3D closure of sampled groups (up to closure_max members when
    given) and 6D subtrees of sampled groups (up to subtree_max members
    when given).
    Raises AssertionError on the first failure."""
    T, n = R["tree"], cfg.n
    h = R["host"]
    cnt = np.bincount(R["labels"], minlength=n)
    groups = np.flatnonzero(cnt >= cfg.min_group)
    lv = T["level"]
    l0 = np.flatnonzero(lv == 0)
    assert np.array_equal(T["min_index"][l0], groups)
    assert np.array_equal(T["size"][l0], cnt[groups])

    # canonical order and parent structure
    key = lv.astype(np.int64) << 32 | T["min_index"].astype(np.int64)
    assert np.all(np.diff(key) > 0)
    p = T["parent"]
    assert np.all(p[l0] == -1)
    up = np.flatnonzero(lv > 0)
    assert np.all((p[up] >= 0) & (p[up] < up))
    assert np.all(lv[p[up]] == lv[up] - 1)
    assert np.all(T["min_index"][p[up]] <= T["min_index"][up])
    assert np.all(T["size"][up] >= cfg.min_sub)
    assert np.all(T["size"][up] < T["size"][p[up]])
    # sizes: own deepest members plus the children's members
    dp = T["deepest"]
    inn = cnt[R["labels"]] >= cfg.min_group
    assert np.all((dp >= 0) == inn)
    own = np.bincount(dp[dp >= 0], minlength=lv.size)
    child = np.zeros(lv.size, np.int64)
    np.add.at(child, p[up], T["size"][up])
    assert np.array_equal(own + child, T["size"])
    # each particle's deepest node lies in its own group's subtree
    root_of = np.arange(lv.size)
    for level in range(1, int(lv.max()) + 1 if lv.size else 1):   # level by level
        at = np.flatnonzero(lv == level)
        root_of[at] = root_of[p[at]]
    canon_root = np.full(n, -1, np.int64)
    canon_root[groups] = l0
    assert np.array_equal(root_of[dp[inn]], canon_root[R["labels"][inn]])

    # level-0 moments of every group against the oracle
    bounds = np.searchsorted(R["sorted_labels"], groups)
    ends = np.searchsorted(R["sorted_labels"], groups, side="right")

    def norms(chunk):
        return [oracle.node_norm(*h, cfg.box, np.sort(R["order"][bounds[i]:ends[i]]))
                for i in chunk]

    chunks = np.array_split(np.arange(groups.size), max(1, groups.size // 2048))
    with ThreadPoolExecutor(WORKERS) as ex:
        ref4 = np.array([r for part in ex.map(norms, chunks) for r in part],
                        np.float32).reshape(-1, 4)
    for j, k in enumerate(("a", "c", "sx2", "sv2")):
        assert np.array_equal(T[k][l0], ref4[:, j]), k

    # sampled groups: 3D closure and connectivity, 6D subtrees
    pick = stratified(cnt[groups], groups, n_sample, cfg.min_group)
    log(f"{cfg.name}: {groups.size} groups, {lv.size} nodes; sampled sizes "
        f"{sorted(cnt[pick].tolist())}")
    pick3 = [g for g in pick if closure_max is None or cnt[g] <= closure_max]
    with ThreadPoolExecutor(WORKERS) as ex:
        r3 = _gather(ex, [ex.submit(check_3d, R, cfg, g) for g in pick3], "3D closure", log)
    bad3 = [(g, s, r) for ok, g, s, r in r3 if not ok]
    assert not bad3, bad3
    deep = [g for g in pick if subtree_max is None or cnt[g] <= subtree_max]
    deep.sort(key=lambda g: -cnt[g])          # largest first on the pool
    with ThreadPoolExecutor(WORKERS) as ex:
        r6 = _gather(ex, [ex.submit(check_subtree, R, cfg, g, root_of, canon_root)
                          for g in deep], "6D subtree", log)
    bad6 = [b for r in r6 for b in r]
    assert not bad6, bad6[:10]
    log(f"{cfg.name}: 3D checked on {len(pick3)} groups (largest {max(cnt[g] for g in pick3)}), "
        f"6D subtrees on {len(deep)} groups (largest {max(cnt[g] for g in deep)})")
    return len(pick3), len(deep)
