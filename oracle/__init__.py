"""CPU oracle for the 3D FoF and the hierarchical 6D phase-space FoF.

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers; the product package never
imports this module.  The arithmetic lives in ``fof_oracle.c`` (plain C,
single-threaded, fp32 pair arithmetic without contraction, exact integer
moments); this file only compiles it with gcc and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fof_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fexcess-precision=standard", "-lm"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (always, when force is set)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS[:-1], _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("RS_ORACLE_LIB")      # a differently built oracle (sanitizer test)
    if not path:
        path = _LIB
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64, i32, f32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_double
    lib.oracle_fof3d.argtypes = [P, P, P, i64, f32, f32, P]
    lib.oracle_fof3d_brute.argtypes = [P, P, P, i64, f32, f32, P]
    lib.oracle_fof3d_mode.argtypes = [P, P, P, i64, f32, f32, ctypes.c_int, P]
    lib.oracle_phase_fof.argtypes = [P, P, P, P, P, P, i64, f32, P, i32, i32, f64, i64,
                                     i64, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.oracle_i128_to_f64.argtypes = [i64, ctypes.c_uint64]
    lib.oracle_i128_to_f64.restype = f64
    lib.oracle_select_rank.argtypes = [i64, f64]
    lib.oracle_select_rank.restype = i64
    lib.oracle_node_nn.argtypes = [P, P, P, P, P, P, f32, P, i64, f32, f32, P]
    lib.oracle_node_norm.argtypes = [P, P, P, P, P, P, f32, P, i64, P]
    lib.oracle_halo_props.argtypes = [P, P, P, P, P, P, i64, f32, i64, P, P, P, P]
    lib.oracle_seed_assign.argtypes = [P, P, P, P, P, P, i64, f32, i64, P, P, P, P, P, P]
    lib.oracle_fof3d_subbox.argtypes = [P, P, P, i64, i64, P, P, f32, f32, ctypes.c_int, P]
    lib.oracle_fof3d_subbox_mode.argtypes = [P, P, P, i64, i64, P, P, f32, f32, ctypes.c_int, P]
    _lib = lib
    return lib


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def fof3d(x, y, z, box, link_len, brute=False, grid="auto"):
    """3D FoF labels (smallest member index per group), int32[n].  grid:
    "auto" (small cells with same-cell linking where the box allows it),
    "coarse" (cells of side >= ll, every member pair tested); brute=True
    tests all pairs."""
    lib = _load()
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.size
    lab = np.empty(n, dtype=np.int32)
    mode = 1 if brute else {"auto": 0, "coarse": 2}[grid]
    rc = lib.oracle_fof3d_mode(_ptr(x), _ptr(y), _ptr(z), n, float(box), float(link_len), mode,
                               _ptr(lab))
    if rc != 0:
        raise OracleError(f"oracle_fof3d failed: {rc}")
    return lab


def fof3d_subbox(x, y, z, n_owned, lo, hi, ghost_width, link_len, brute=False, grid="auto"):
    """3D FoF over a non-periodic sub-box [lo, hi) whose particles [0, n_owned)
    are owned and the rest are ghosts within ghost_width of it.  Returns
    (labels, ghost_links): labels = smallest member index per group; the
    ghost links are the (ghost index, label) pairs of the ghosts whose group
    holds an owned particle (label < n_owned), by ghost index.  grid: "auto"
    (small cells with same-cell linking where the sub-box allows it) or
    "coarse" (cells of side >= the margin, every member pair tested);
    brute=True tests all pairs."""
    lib = _load()
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.size
    lab = np.empty(n, dtype=np.int32)
    lo3, hi3 = _f32(lo), _f32(hi)
    mode = 1 if brute else {"auto": 0, "coarse": 2}[grid]
    rc = lib.oracle_fof3d_subbox_mode(_ptr(x), _ptr(y), _ptr(z), n, int(n_owned), _ptr(lo3),
                                      _ptr(hi3), float(ghost_width), float(link_len), mode,
                                      _ptr(lab))
    if rc != 0:
        raise OracleError(f"oracle_fof3d_subbox failed: {rc}")
    g = np.arange(int(n_owned), n, dtype=np.int32)
    keep = lab[g] < int(n_owned)
    return lab, np.stack([g[keep], lab[g][keep]], 1).astype(np.int32)


NODE_FIELDS = ("level", "min_index", "parent", "size", "l2", "a", "c", "sx2", "sv2", "wide")


def phase_fof(x, y, z, vx, vy, vz, box, fof_labels, min_group=10, min_sub=10, f=0.7,
              brute_max=32):
    """Hierarchical 6D FoF.  Returns a dict of numpy arrays: the node fields
    in canonical (level, min_index) order, plus ``deepest`` per particle."""
    lib = _load()
    arrs = [_f32(a) for a in (x, y, z, vx, vy, vz)]
    lab = np.ascontiguousarray(np.asarray(fof_labels, dtype=np.int32))
    n = arrs[0].size
    cap = max(64, n // 4)
    while True:
        out = dict(level=np.empty(cap, np.int32), min_index=np.empty(cap, np.int32),
                   parent=np.empty(cap, np.int32), size=np.empty(cap, np.int32),
                   l2=np.empty(cap, np.float32), a=np.empty(cap, np.float32),
                   c=np.empty(cap, np.float32), sx2=np.empty(cap, np.float32),
                   sv2=np.empty(cap, np.float32), wide=np.empty(cap, np.int32))
        deepest = np.empty(n, np.int32)
        nn = ctypes.c_int64(0)
        rc = lib.oracle_phase_fof(*[_ptr(a) for a in arrs], n, float(box), _ptr(lab),
                                  int(min_group), int(min_sub), float(f), int(brute_max),
                                  cap, *[_ptr(out[k]) for k in NODE_FIELDS],
                                  _ptr(deepest), ctypes.byref(nn))
        if rc == -4:
            cap = int(nn.value) + 16
            continue
        if rc != 0:
            raise OracleError(f"oracle_phase_fof failed: {rc}")
        m = int(nn.value)
        res = {k: v[:m].copy() for k, v in out.items()}
        res["deepest"] = deepest
        return res


def i128_to_f64(v: int) -> float:
    lib = _load()
    v &= (1 << 128) - 1
    hi = v >> 64
    if hi >= 1 << 63:
        hi -= 1 << 64
    return lib.oracle_i128_to_f64(hi, v & ((1 << 64) - 1))


def select_rank(n: int, f: float) -> int:
    return int(_load().oracle_select_rank(int(n), float(f)))


def node_nn(x, y, z, vx, vy, vz, box, members, a, c):
    lib = _load()
    arrs = [_f32(q) for q in (x, y, z, vx, vy, vz)]
    mem = np.ascontiguousarray(np.asarray(members, dtype=np.int64))
    d2 = np.empty(mem.size, np.float32)
    lib.oracle_node_nn(*[_ptr(q) for q in arrs], float(box), _ptr(mem), mem.size,
                       float(a), float(c), _ptr(d2))
    return d2


def node_norm(x, y, z, vx, vy, vz, box, members):
    """(a, c, sx2, sv2) of one member set (members ascending)."""
    lib = _load()
    arrs = [_f32(q) for q in (x, y, z, vx, vy, vz)]
    mem = np.ascontiguousarray(np.sort(np.asarray(members, dtype=np.int64)))
    out = np.empty(4, np.float32)
    lib.oracle_node_norm(*[_ptr(q) for q in arrs], float(box), _ptr(mem), mem.size, _ptr(out))
    return tuple(float(v) for v in out)


PROP_NAMES = ("cx", "cy", "cz", "vx", "vy", "vz", "Mxx", "Myy", "Mzz", "Mxy", "Mxz", "Myz",
              "jx", "jy", "jz")


def halo_props(x, y, z, vx, vy, vz, box, parent, min_index, deepest):
    """Per-node properties, float32[15, n_nodes] (rows as in PROP_NAMES):
    centre, bulk velocity, second-moment tensor about the centre and specific
    angular momentum of the members of each node of a hierarchy."""
    lib = _load()
    arrs = [_f32(q) for q in (x, y, z, vx, vy, vz)]
    par = np.ascontiguousarray(np.asarray(parent, dtype=np.int32))
    mi = np.ascontiguousarray(np.asarray(min_index, dtype=np.int32))
    dp = np.ascontiguousarray(np.asarray(deepest, dtype=np.int32))
    m = par.size
    out = np.empty((len(PROP_NAMES), m), np.float32)
    rc = lib.oracle_halo_props(*[_ptr(q) for q in arrs], arrs[0].size, float(box), m, _ptr(par),
                               _ptr(mi), _ptr(dp), _ptr(out))
    if rc != 0:
        raise OracleError(f"oracle_halo_props failed: {rc}")
    return out


def seed_assign(x, y, z, vx, vy, vz, box, parent, deepest, a, c, props):
    """Seed (leaf node) each particle is assigned to, int32[n] (-1 outside
    every node); props as halo_props returns it."""
    lib = _load()
    arrs = [_f32(q) for q in (x, y, z, vx, vy, vz)]
    par = np.ascontiguousarray(np.asarray(parent, dtype=np.int32))
    dp = np.ascontiguousarray(np.asarray(deepest, dtype=np.int32))
    fa, fc = _f32(a), _f32(c)
    pr = np.ascontiguousarray(np.asarray(props, dtype=np.float32))
    m = par.size
    if pr.shape != (len(PROP_NAMES), m):
        raise ValueError("props has the wrong shape")
    out = np.empty(arrs[0].size, np.int32)
    rc = lib.oracle_seed_assign(*[_ptr(q) for q in arrs], arrs[0].size, float(box), m,
                                _ptr(par), _ptr(dp), _ptr(fa), _ptr(fc), _ptr(pr), _ptr(out))
    if rc != 0:
        raise OracleError(f"oracle_seed_assign failed: {rc}")
    return out
