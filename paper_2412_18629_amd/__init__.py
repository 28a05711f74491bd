"""MI355X friends-of-friends halo-finding core: Python binding of librsfof.

Argument marshalling only.  Every step of the computation runs in the HIP
kernels of ``librsfof.so``; PyTorch supplies device memory and streams.  If
the library has not been built, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsfof.so")

RS_OK, RS_EINVAL, RS_ERANGE, RS_ENOMEM, RS_EDEVICE, RS_EINTERNAL, RS_ENOTIMPL = (
    0, -1, -2, -3, -4, -5, -6)
RS_PLAIN, RS_BATCHED, RS_LEARNED = 0, 1, 2
RS_FEATURES = 0x100
RS_NFEAT = 24
RS_MLP_NPARAM = 5825
MODEL_FLOATS = 2 * RS_NFEAT + RS_MLP_NPARAM      # mean[24], std[24], params
MODEL_BYTES = 4 + 4 * MODEL_FLOATS               # "RSM1" tag + floats

EXPORTED = ("rs_fof3d", "rs_phase_fof_batch", "rs_free", "rs_strerror", "rs_version",
            "rs_profile_enable", "rs_profile_get", "rs_mlp_forward", "rs_mlp_grad",
            "rs_mlp_train_step", "rs_mlp_standardize", "rs_mlp_infer",
            "rs_sort_pairs_u64_i32", "rs_release_workspace", "rs_tune_set", "rs_tune_get",
            "rs_tune_name", "rs_halo_props", "rs_fof3d_subbox", "rs_seed_assign")


class RsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status})")


class _Tree(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_particles", ctypes.c_int64),
                ("level", ctypes.c_void_p), ("min_index", ctypes.c_void_p),
                ("parent", ctypes.c_void_p), ("size", ctypes.c_void_p),
                ("l2", ctypes.c_void_p), ("a", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("sx2", ctypes.c_void_p), ("sv2", ctypes.c_void_p),
                ("deepest", ctypes.c_void_p), ("n_accepted", ctypes.c_int64),
                ("n_fallback", ctypes.c_int64), ("n_levels", ctypes.c_int64),
                ("features", ctypes.c_void_p), ("wide", ctypes.c_void_p)]


_lib = None


def load():
    """Load librsfof.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2412_18629_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, i32, f32, f64, u32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_float, ctypes.c_double, ctypes.c_uint32)
    lib.rs_fof3d.argtypes = [P, P, P, i64, f32, f32, P, ctypes.POINTER(i64), P]
    lib.rs_fof3d.restype = ctypes.c_int
    lib.rs_fof3d_noalloc.argtypes = [P, P, P, i64, f32, f32, P, ctypes.POINTER(i64), P]
    lib.rs_fof3d_noalloc.restype = ctypes.c_int
    lib.rs_fof3d_subbox.argtypes = [P, P, P, i64, i64, P, P, f32, f32, P, P,
                                    ctypes.POINTER(i64), P]
    lib.rs_fof3d_subbox.restype = ctypes.c_int
    lib.rs_phase_fof_batch.argtypes = [P, P, P, P, P, P, i64, f32, P, i32, i32, f64, u32, P,
                                       ctypes.POINTER(ctypes.POINTER(_Tree)), P]
    lib.rs_phase_fof_batch.restype = ctypes.c_int
    lib.rs_free.argtypes = [P]
    lib.rs_free.restype = None
    lib.rs_strerror.argtypes = [ctypes.c_int]
    lib.rs_strerror.restype = ctypes.c_char_p
    lib.rs_version.argtypes = []
    lib.rs_version.restype = ctypes.c_char_p
    lib.rs_profile_enable.argtypes = [ctypes.c_int]
    lib.rs_profile_enable.restype = ctypes.c_int
    lib.rs_profile_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(f64), ctypes.POINTER(i64),
                                   ctypes.POINTER(f64)]
    lib.rs_profile_get.restype = ctypes.c_int
    lib.rs_mlp_forward.argtypes = [P, P, i64, P, P]
    lib.rs_mlp_grad.argtypes = [P, P, P, i64, P, P, P]
    lib.rs_mlp_train_step.argtypes = [P, P, P, i64, P, P, i64, f32, P, P]
    lib.rs_mlp_standardize.argtypes = [P, i64, P, P, ctypes.c_int, P]
    lib.rs_mlp_infer.argtypes = [P, i64, P, P, P]
    lib.rs_sort_pairs_u64_i32.argtypes = [P, P, P, P, i64, ctypes.c_int, P]
    lib.rs_halo_props.argtypes = [P, P, P, P, P, P, i64, f32, i64, i64, P, P, P, P, P, P, P]
    lib.rs_seed_assign.argtypes = [P, P, P, P, P, P, i64, f32, i64, i64, P, P, P, P, P, P, P, P,
                                   P, P]
    lib.rs_release_workspace.argtypes = []
    lib.rs_tune_set.argtypes = [ctypes.c_char_p, ctypes.c_int]
    lib.rs_tune_set.restype = ctypes.c_int
    lib.rs_tune_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int32), ctypes.c_int]
    lib.rs_tune_get.restype = ctypes.c_int
    lib.rs_tune_name.argtypes = [ctypes.c_int]
    lib.rs_tune_name.restype = ctypes.c_char_p
    for fn in ("rs_mlp_forward", "rs_mlp_grad", "rs_mlp_train_step", "rs_mlp_standardize",
               "rs_mlp_infer", "rs_sort_pairs_u64_i32", "rs_release_workspace", "rs_halo_props",
               "rs_seed_assign"):
        getattr(lib, fn).restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().rs_strerror(int(status)).decode()


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def rs_fof3d(x, y, z, box, link_len, labels=None, stream=None):
    """3D FoF labels (int32 device tensor, smallest member index per group)
    and the number of groups."""
    lib = load()
    n = x.numel()
    for t, nm in ((y, "y"), (z, "z")):
        if t.numel() != n:
            raise ValueError(f"{nm} size differs from x")
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=x.device)
    ptrs = [_dev(t, torch.float32, nm) for t, nm in ((x, "x"), (y, "y"), (z, "z"))]
    ng = ctypes.c_int64(-1)
    rc = lib.rs_fof3d(*ptrs, n, float(box), float(link_len), _dev(labels, torch.int32, "labels"),
                      ctypes.byref(ng), _stream(stream))
    if rc != RS_OK:
        raise RsError(rc, "rs_fof3d")
    return labels, int(ng.value)


def rs_fof3d_subbox(x, y, z, n_owned, lo, hi, ghost_width, link_len, labels=None,
                    links=True, stream=None):
    """3D FoF over a non-periodic sub-box [lo, hi) with owned particles
    [0, n_owned) and ghosts after them.  Returns (labels, ghost_links): int32
    device tensors, ghost_links of shape (n_links, 2) holding (ghost index,
    label) for the ghosts whose group holds an owned particle (None when
    links is False)."""
    lib = load()
    n = x.numel()
    for t, nm in ((y, "y"), (z, "z")):
        if t.numel() != n:
            raise ValueError(f"{nm} size differs from x")
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=x.device)
    lo3 = (ctypes.c_float * 3)(*[float(v) for v in lo])
    hi3 = (ctypes.c_float * 3)(*[float(v) for v in hi])
    ng = max(n - int(n_owned), 0)
    buf = torch.empty(max(2 * ng, 2), dtype=torch.int32, device=x.device) if links else None
    cnt = ctypes.c_int64(-1)
    ptrs = [_dev(t, torch.float32, nm) for t, nm in ((x, "x"), (y, "y"), (z, "z"))]
    rc = lib.rs_fof3d_subbox(*ptrs, n, int(n_owned), lo3, hi3, float(ghost_width),
                             float(link_len), _dev(labels, torch.int32, "labels"),
                             _dev(buf, torch.int32, "ghost_links") if links else None,
                             ctypes.byref(cnt) if links else None, _stream(stream))
    if rc != RS_OK:
        raise RsError(rc, "rs_fof3d_subbox")
    if not links:
        return labels, None
    return labels, buf[: 2 * int(cnt.value)].view(-1, 2)


def rs_sort_pairs(keys, vals, bits=64, stream=None):
    """Stable sort of (keys uint64 as int64 storage, vals int32) by the low
    `bits` bits of the key; returns new (keys, vals) device tensors."""
    n = keys.numel()
    if vals.numel() != n:
        raise ValueError("vals size differs from keys")
    ko = torch.empty_like(keys)
    vo = torch.empty_like(vals)
    _ck(load().rs_sort_pairs_u64_i32(_dev(keys, torch.int64, "keys"), _dev(ko, torch.int64, "keys"),
                                     _dev(vals, torch.int32, "vals"), _dev(vo, torch.int32, "vals"),
                                     n, int(bits), _stream(stream)), "rs_sort_pairs_u64_i32")
    return ko, vo


def tune_knobs():
    """{knob: (current value, allowed values)} of the launch-shape table."""
    lib = load()
    out = {}
    i = 0
    while True:
        name = lib.rs_tune_name(i)
        if name is None:
            return out
        cur = ctypes.c_int(0)
        ch = (ctypes.c_int32 * 8)()
        k = lib.rs_tune_get(name, ctypes.byref(cur), ch, 8)
        if k < 0:
            raise RsError(k, "rs_tune_get")
        out[name.decode()] = (int(cur.value), [int(ch[j]) for j in range(min(k, 8))])
        i += 1


def tune_set(knob, value):
    _ck(load().rs_tune_set(knob.encode(), int(value)), f"rs_tune_set({knob})")


def load_tuning(path=None):
    """Apply a tuning table written by paper_2412_18629_amd.autotune (the
    default table next to this package when present); returns it or None."""
    import json
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    for knob, value in table["choice"].items():
        tune_set(knob, value)
    return table


def rs_release_workspace():
    """Give the library's device workspaces back (the next call reallocates)."""
    _ck(load().rs_release_workspace(), "rs_release_workspace")


class _DevArray:
    """Zero-copy view descriptor of a device array owned by the library."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr,
                                         "data": (int(ptr or 0), False), "version": 3,
                                         "strides": None}


def _copy_out(ptr, n, dtype, device):
    if n == 0:
        return torch.empty(0, dtype=dtype, device=device)
    typestr = {torch.int32: "<i4", torch.float32: "<f4"}[dtype]
    view = torch.as_tensor(_DevArray(ptr, n, typestr), device=device)
    return view.clone()


TREE_FIELDS = (("level", torch.int32), ("min_index", torch.int32), ("parent", torch.int32),
               ("size", torch.int32), ("l2", torch.float32), ("a", torch.float32),
               ("c", torch.float32), ("sx2", torch.float32), ("sv2", torch.float32),
               ("wide", torch.int32))


def rs_phase_fof_batch(x, y, z, vx, vy, vz, box, fof_labels, min_group=10, min_sub=10, f=0.7,
                       flags=RS_BATCHED, model=None, stream=None):
    """Hierarchical 6D FoF.  Returns a dict of device tensors: the node fields
    in canonical (level, min_index) order, ``deepest`` per particle, and the
    statistics n_accepted, n_fallback, n_levels."""
    lib = load()
    if model is not None and not isinstance(model, (bytes, bytearray)):
        raise TypeError("model must be a bytes blob")
    if model is not None and (len(model) != MODEL_BYTES or bytes(model[:4]) != b"RSM1"):
        raise ValueError(f"model must be the {MODEL_BYTES}-byte RSM1 proposer blob")
    n = x.numel()
    arrs = (x, y, z, vx, vy, vz)
    names = ("x", "y", "z", "vx", "vy", "vz")
    for t, nm in zip(arrs, names):
        if t.numel() != n:
            raise ValueError(f"{nm} size differs from x")
    ptrs = [_dev(t, torch.float32, nm) for t, nm in zip(arrs, names)]
    lab = _dev(fof_labels, torch.int32, "fof_labels")
    mbuf = ctypes.create_string_buffer(bytes(model), len(model)) if model is not None else None
    out = ctypes.POINTER(_Tree)()
    st = _stream(stream)
    rc = lib.rs_phase_fof_batch(*ptrs, n, float(box), lab, int(min_group), int(min_sub),
                                float(f), int(flags),
                                ctypes.cast(mbuf, ctypes.c_void_p) if mbuf is not None else None,
                                ctypes.byref(out), st)
    if rc != RS_OK:
        raise RsError(rc, "rs_phase_fof_batch")
    try:
        t = out.contents
        m = int(t.n_nodes)
        res = {k: _copy_out(getattr(t, k), m, dt, x.device) for k, dt in TREE_FIELDS}
        res["deepest"] = _copy_out(t.deepest, n, torch.int32, x.device)
        res["n_accepted"] = int(t.n_accepted)
        res["n_fallback"] = int(t.n_fallback)
        res["n_levels"] = int(t.n_levels)
        if t.features:
            res["features"] = _copy_out(t.features, m * RS_NFEAT, torch.float32,
                                        x.device).view(m, RS_NFEAT)
        torch.cuda.current_stream().synchronize()
    finally:
        lib.rs_free(out)
    return res


PROP_NAMES = ("cx", "cy", "cz", "vx", "vy", "vz", "Mxx", "Myy", "Mzz", "Mxy", "Mxz", "Myz",
              "jx", "jy", "jz")
RS_NPROP = len(PROP_NAMES)


def rs_halo_props(x, y, z, vx, vy, vz, box, tree, out=None, stream=None):
    """Per-node halo properties of a hierarchy (the dict rs_phase_fof_batch
    returns): float32 device tensor [RS_NPROP, n_nodes], rows as in
    PROP_NAMES (centre, bulk velocity, second-moment tensor, specific angular
    momentum)."""
    lib = load()
    n = x.numel()
    arrs = (x, y, z, vx, vy, vz)
    names = ("x", "y", "z", "vx", "vy", "vz")
    for t, nm in zip(arrs, names):
        if t.numel() != n:
            raise ValueError(f"{nm} size differs from x")
    m = tree["level"].numel()
    for k in ("parent", "min_index", "size"):
        if tree[k].numel() != m:
            raise ValueError(f"tree field {k} has the wrong size")
    if tree["deepest"].numel() != n:
        raise ValueError("tree field deepest has the wrong size")
    if out is None:
        out = torch.empty((RS_NPROP, m), dtype=torch.float32, device=x.device)
    if out.shape != (RS_NPROP, m):
        raise ValueError("out has the wrong shape")
    ptrs = [_dev(t, torch.float32, nm) for t, nm in zip(arrs, names)]
    tp = [_dev(tree[k], torch.int32, k) for k in ("level", "parent", "min_index", "size",
                                                  "deepest")]
    _ck(lib.rs_halo_props(*ptrs, n, float(box), m, int(tree["n_levels"]), *tp,
                          _dev(out, torch.float32, "out"), _stream(stream)), "rs_halo_props")
    return out


def rs_seed_assign(x, y, z, vx, vy, vz, box, tree, props, out=None, stream=None):
    """Seed halo (leaf node index, -1 outside every node) of each particle,
    int32 device tensor [n]; tree as rs_phase_fof_batch returns it, props as
    rs_halo_props returns it."""
    lib = load()
    n = x.numel()
    arrs = (x, y, z, vx, vy, vz)
    names = ("x", "y", "z", "vx", "vy", "vz")
    for t, nm in zip(arrs, names):
        if t.numel() != n:
            raise ValueError(f"{nm} size differs from x")
    m = tree["level"].numel()
    for k in ("parent", "min_index", "size", "a", "c"):
        if tree[k].numel() != m:
            raise ValueError(f"tree field {k} has the wrong size")
    if tree["deepest"].numel() != n:
        raise ValueError("tree field deepest has the wrong size")
    if props.shape != (RS_NPROP, m):
        raise ValueError("props has the wrong shape")
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=x.device)
    if out.numel() != n:
        raise ValueError("out has the wrong size")
    ptrs = [_dev(t, torch.float32, nm) for t, nm in zip(arrs, names)]
    tp = [_dev(tree[k], torch.int32, k) for k in ("level", "parent", "min_index", "size",
                                                  "deepest")]
    _ck(lib.rs_seed_assign(*ptrs, n, float(box), m, int(tree["n_levels"]), *tp,
                           _dev(tree["a"], torch.float32, "a"), _dev(tree["c"], torch.float32, "c"),
                           _dev(props, torch.float32, "props"), _dev(out, torch.int32, "out"),
                           _stream(stream)), "rs_seed_assign")
    return out


def rs_profile_enable(on=True) -> None:
    """Record HIP events around the library's main kernels (instrumentation);
    on=2 also counts the searches' pair tests ("pairs_fof3d", "pairs_nn",
    "pairs_link"), with slower counting kernels."""
    load().rs_profile_enable(2 if on == 2 else (1 if on else 0))


def rs_profile_get(name: str):
    """(total_ms, launches, units) recorded for one instrumented kernel."""
    ms, n, u = ctypes.c_double(0), ctypes.c_int64(0), ctypes.c_double(0)
    rc = load().rs_profile_get(name.encode(), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(u))
    if rc != RS_OK:
        raise RsError(rc, "rs_profile_get")
    return ms.value, int(n.value), u.value


# ---------------------------------------------------------------------------
# linking-length proposer (MLP) entry points
# ---------------------------------------------------------------------------

def _ck(rc, where):
    if rc != RS_OK:
        raise RsError(rc, where)


def rs_mlp_forward(params, X, stream=None):
    if params.numel() != RS_MLP_NPARAM or X.dim() != 2 or X.shape[1] != RS_NFEAT:
        raise ValueError("params must hold RS_MLP_NPARAM floats and X be (n, RS_NFEAT)")
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _ck(load().rs_mlp_forward(_dev(params, torch.float32, "params"), _dev(X, torch.float32, "X"),
                              X.shape[0], _dev(y, torch.float32, "y"), _stream(stream)),
        "rs_mlp_forward")
    return y


def rs_mlp_grad(params, X, t, stream=None):
    if params.numel() != RS_MLP_NPARAM or X.dim() != 2 or X.shape[1] != RS_NFEAT or \
            t.numel() != X.shape[0]:
        raise ValueError("params, X (n, RS_NFEAT) and t (n) have inconsistent sizes")
    g = torch.empty(RS_MLP_NPARAM, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _ck(load().rs_mlp_grad(_dev(params, torch.float32, "params"), _dev(X, torch.float32, "X"),
                           _dev(t, torch.float32, "t"), X.shape[0], _dev(g, torch.float32, "g"),
                           _dev(loss, torch.float32, "loss"), _stream(stream)), "rs_mlp_grad")
    return g, loss


def rs_mlp_train_step(params, m, v, step, X, t, lr, loss, stream=None):
    if any(a.numel() != RS_MLP_NPARAM for a in (params, m, v)) or X.dim() != 2 or \
            X.shape[1] != RS_NFEAT or t.numel() != X.shape[0] or loss.numel() < 1:
        raise ValueError("params, m, v, X (n, RS_NFEAT), t (n) have inconsistent sizes")
    _ck(load().rs_mlp_train_step(_dev(params, torch.float32, "params"),
                                 _dev(m, torch.float32, "m"), _dev(v, torch.float32, "v"),
                                 int(step), _dev(X, torch.float32, "X"),
                                 _dev(t, torch.float32, "t"), X.shape[0], float(lr),
                                 _dev(loss, torch.float32, "loss"), _stream(stream)),
        "rs_mlp_train_step")


def rs_mlp_standardize(X, mean, std, compute=True, stream=None):
    _ck(load().rs_mlp_standardize(_dev(X, torch.float32, "X"), X.shape[0],
                                  _dev(mean, torch.float32, "mean"),
                                  _dev(std, torch.float32, "std"), 1 if compute else 0,
                                  _stream(stream)), "rs_mlp_standardize")


def rs_mlp_infer(model, feats, stream=None):
    if model.numel() != MODEL_FLOATS:
        raise ValueError(f"model must hold {MODEL_FLOATS} floats")
    if feats.dim() != 2 or feats.shape[1] != RS_NFEAT:
        raise ValueError(f"features must be (n, {RS_NFEAT})")
    out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
    _ck(load().rs_mlp_infer(_dev(model, torch.float32, "model"),
                            feats.shape[0], _dev(feats, torch.float32, "features"),
                            _dev(out, torch.float32, "out"), _stream(stream)), "rs_mlp_infer")
    return out


def pack_model(mean, std, params) -> bytes:
    """The proposer blob rs_phase_fof_batch takes: b"RSM1" + float32
    mean[24], std[24], params[5825]."""
    import numpy as np
    body = np.concatenate([np.asarray(mean, np.float32).ravel(), np.asarray(std, np.float32).ravel(),
                           np.asarray(params, np.float32).ravel()])
    if body.size != 2 * RS_NFEAT + RS_MLP_NPARAM:
        raise ValueError("model has the wrong size")
    return b"RSM1" + body.astype("<f4").tobytes()


def unpack_model(blob: bytes):
    import numpy as np
    if blob[:4] != b"RSM1":
        raise ValueError("not a proposer blob")
    body = np.frombuffer(blob[4:], dtype="<f4")
    return body[:RS_NFEAT], body[RS_NFEAT:2 * RS_NFEAT], body[2 * RS_NFEAT:]
