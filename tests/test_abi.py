"""The C ABI: library loads, exports every declared symbol, rejects bad
arguments before touching a device (CPU only; no compute call)."""
import ctypes
import os
import re

import pytest
import torch

import paper_2412_18629_amd as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsfof.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z0-9_]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = rs.load()
    names = declared_functions()
    assert {"rs_fof3d", "rs_phase_fof_batch", "rs_free", "rs_strerror"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    assert set(rs.EXPORTED) <= set(names)


def test_strerror_and_version():
    lib = rs.load()
    for code in range(-6, 1):
        assert lib.rs_strerror(code)
    assert b"unknown" in lib.rs_strerror(-99)
    assert lib.rs_version().startswith(b"rsfof")


def test_free_null_is_noop():
    rs.load().rs_free(None)


def _fof3d_raw(n, box, ll, ptr=1):
    lib = rs.load()
    p = ctypes.c_void_p(ptr)
    ng = ctypes.c_int64(7)
    rc = lib.rs_fof3d(p, p, p, n, box, ll, p, ctypes.byref(ng), None)
    return rc, ng.value


@pytest.mark.parametrize("n,box,ll", [(-1, 10.0, 0.2), (1 << 31, 10.0, 0.2), (10, 0.0, 0.2),
                                      (10, -1.0, 0.2), (10, 10.0, 0.0), (10, 10.0, 5.0),
                                      (10, float("nan"), 0.2), (10, float("inf"), 0.2),
                                      (10, 10.0, float("nan"))])
def test_fof3d_rejects_bad_arguments_before_device_work(n, box, ll):
    rc, ng = _fof3d_raw(n, box, ll)
    assert rc == rs.RS_EINVAL
    assert ng == 7                      # outputs untouched


def test_fof3d_null_pointers():
    rc, _ = _fof3d_raw(5, 10.0, 0.2, ptr=0)
    assert rc == rs.RS_EINVAL


def _phase_raw(n=10, box=10.0, min_group=10, min_sub=10, f=0.7, flags=1, ptr=1, model=None,
               out=True):
    lib = rs.load()
    p = ctypes.c_void_p(ptr)
    tree = ctypes.POINTER(rs._Tree)()
    return lib.rs_phase_fof_batch(p, p, p, p, p, p, n, box, p, min_group, min_sub, f, flags,
                                  model, ctypes.byref(tree) if out else None, None)


@pytest.mark.parametrize("kw", [dict(n=-1), dict(box=0.0), dict(min_group=1), dict(min_sub=1),
                                dict(f=0.0), dict(f=1.5), dict(f=float("nan")), dict(flags=7),
                                dict(flags=2, model=None), dict(ptr=0), dict(out=False)])
def test_phase_rejects_bad_arguments_before_device_work(kw):
    assert _phase_raw(**kw) == rs.RS_EINVAL


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device path")
def test_no_device_reports_edevice():
    rc, ng = _fof3d_raw(10, 10.0, 0.2)
    assert rc == rs.RS_EDEVICE and ng == 7


@pytest.mark.parametrize("n,bits,alias", [(-1, 8, False), (1 << 31, 8, False), (4, 0, False),
                                          (4, 65, False), (4, 8, True)])
def test_sort_rejects_bad_arguments(n, bits, alias):
    lib = rs.load()
    a = ctypes.c_void_p(0x1000)
    b = a if alias else ctypes.c_void_p(0x2000)
    rc = lib.rs_sort_pairs_u64_i32(a, b, ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), n,
                                   bits, None)
    assert rc == rs.RS_EINVAL


def test_tuning_table_rejects_unknown_knobs_and_values():
    knobs = rs.tune_knobs()
    assert set(knobs) == {"small_threads_256", "small_threads_1024", "small_threads_2048",
                          "xcd_chunk"}
    for name, (cur, allowed) in knobs.items():
        assert cur in allowed
    lib = rs.load()
    assert lib.rs_tune_set(b"no_such_knob", 1) == rs.RS_EINVAL
    assert lib.rs_tune_set(b"xcd_chunk", 3) == rs.RS_EINVAL


@pytest.mark.parametrize("n,box,m,nlev", [(10, 2048.0, 1, 1), (10, 0.0, 1, 1), (-1, 10.0, 1, 1),
                                          (10, 10.0, 1, 2), (10, 10.0, 1, 0), (10, 10.0, -1, 0),
                                          (0, 10.0, 1, 1)])
def test_halo_props_rejects_bad_arguments_before_device_work(n, box, m, nlev):
    lib = rs.load()
    p = ctypes.c_void_p(1)
    rc = lib.rs_halo_props(p, p, p, p, p, p, n, box, m, nlev, p, p, p, p, p, p, None)
    if rc == rs.RS_EDEVICE:
        pytest.skip("argument check passed; no device here")
    assert rc == rs.RS_EINVAL


def test_fof3d_subbox_rejects_bad_arguments_before_device_work():
    lib = rs.load()
    p = ctypes.c_void_p(1)
    F3 = ctypes.c_float * 3
    good_lo, good_hi = F3(0, 0, 0), F3(1, 1, 1)
    cnt = ctypes.c_int64(5)
    cases = [(10, 11, good_lo, good_hi, 0.1, 0.2, p, ctypes.byref(cnt)),     # n_owned > n
             (10, 5, good_lo, F3(1, 0, 1), 0.1, 0.2, p, ctypes.byref(cnt)),  # hi <= lo
             (10, 5, good_lo, good_hi, -0.1, 0.2, p, ctypes.byref(cnt)),     # ghost width
             (10, 5, good_lo, good_hi, 0.1, 0.0, p, ctypes.byref(cnt)),      # link length
             (10, 5, good_lo, good_hi, 0.1, float("nan"), p, ctypes.byref(cnt)),
             (10, 5, None, good_hi, 0.1, 0.2, p, ctypes.byref(cnt)),
             (10, 5, good_lo, good_hi, 0.1, 0.2, p, None)]                   # links, no count
    for n, no, lo, hi, gw, ll, links, nl in cases:
        rc = lib.rs_fof3d_subbox(p, p, p, n, no, lo, hi, gw, ll, p, links, nl, None)
        assert rc == rs.RS_EINVAL
    assert cnt.value == 5


def test_binding_checks_the_proposer_blob():
    # a truncated or foreign blob never reaches the library (it copies a
    # fixed number of floats from it)
    from paper_2412_18629_amd import learn
    blob = learn.load_model()
    assert len(blob) == rs.MODEL_BYTES
    t = torch.zeros(4)
    for bad in (blob[:-4], b"XXXX" + blob[4:], blob + b"\0\0\0\0"):
        with pytest.raises(ValueError):
            rs.rs_phase_fof_batch(t, t, t, t, t, t, 1.0, torch.zeros(4, dtype=torch.int32),
                                  flags=rs.RS_LEARNED, model=bad)
