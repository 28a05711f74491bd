"""The allocation-free 3D entry point (rs_fof3d_noalloc), called through the
C ABI, against rs_fof3d on the same inputs: labels and group counts
identical on two calls in a row, the second on a smaller input (the shared
fixed work space keeps the first call's contents), and a call that needs
more than the fixed work space rejected before any device work.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2412_18629_amd as rs
from paper_2412_18629_amd import synth

pytestmark = pytest.mark.gpu


def _noalloc(x, y, z, box, ll):
    lib = rs.load()
    n = x.numel()
    lab = torch.full((n,), -3, dtype=torch.int32, device=x.device)
    ng = ctypes.c_int64(-1)
    rc = lib.rs_fof3d_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                              ctypes.c_void_p(z.data_ptr()), n, float(box), float(ll),
                              ctypes.c_void_p(lab.data_ptr()), ctypes.byref(ng),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, lab, ng.value


def _inputs(n, seed):
    cfg = synth.scaled(synth.CONFIGS["c32"], n)
    x, y, z, *_ = synth.generate(cfg, seed)
    return [a.cuda() for a in (x, y, z)], cfg


def test_two_calls_match_rs_fof3d_second_smaller():
    for n, seed in ((900000, 3), (120001, 4)):
        (x, y, z), cfg = _inputs(n, seed)
        rc, lab, ng = _noalloc(x, y, z, cfg.box, cfg.link_len)
        assert rc == rs.RS_OK
        ref, ref_ng = rs.rs_fof3d(x, y, z, cfg.box, cfg.link_len)
        torch.cuda.synchronize()
        assert torch.equal(lab, ref)
        assert ng == ref_ng


def test_rejects_a_pass_larger_than_the_work_space():
    (x, y, z), cfg = _inputs(2_000_000, 5)
    rc, lab, ng = _noalloc(x, y, z, cfg.box, cfg.link_len)
    assert rc == rs.RS_EINVAL
    assert ng == -1 and bool((lab == -3).all())
