"""The library's stable key/value radix sort (rs_sort_pairs_u64_i32) against
numpy's stable argsort of the masked keys: keys and values equal element by
element, over sizes around the tile length, bit widths that leave high bits
to carry, and degenerate key sets."""
import numpy as np
import pytest
import torch

import paper_2412_18629_amd as rs

pytestmark = pytest.mark.gpu

TILE = 4096


def _check(keys_u64, bits, seed=0):
    n = keys_u64.size
    vals = np.random.default_rng(seed).permutation(n).astype(np.int32)
    k = torch.from_numpy(keys_u64.view(np.int64).copy()).cuda()
    v = torch.from_numpy(vals).cuda()
    ko, vo = rs.rs_sort_pairs(k, v, bits)
    torch.cuda.synchronize()
    mask = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    order = np.argsort(keys_u64 & mask, kind="stable")
    assert np.array_equal(ko.cpu().numpy().view(np.uint64), keys_u64[order])
    assert np.array_equal(vo.cpu().numpy(), vals[order])
    # inputs untouched
    assert np.array_equal(k.cpu().numpy().view(np.uint64), keys_u64)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, TILE - 1, TILE, TILE + 1, 3 * TILE + 17,
                               1_000_003])
@pytest.mark.parametrize("bits", [1, 8, 13, 36, 64])
def test_random_keys(n, bits):
    rng = np.random.default_rng(n * 131 + bits)
    keys = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, n).astype(np.uint64)
    _check(keys, bits, seed=n)


@pytest.mark.parametrize("kind", ["equal", "two", "sorted", "reversed", "skewed"])
def test_degenerate_keys(kind):
    n = 5 * TILE + 123
    rng = np.random.default_rng(7)
    if kind == "equal":
        keys = np.full(n, 12345, np.uint64)
    elif kind == "two":
        keys = rng.integers(0, 2, n).astype(np.uint64) << np.uint64(40)
    elif kind == "sorted":
        keys = np.arange(n, dtype=np.uint64)
    elif kind == "reversed":
        keys = np.arange(n, dtype=np.uint64)[::-1].copy()
    else:
        keys = (rng.geometric(0.3, n) - 1).astype(np.uint64)
    _check(keys, 48)


def test_empty():
    k = torch.empty(0, dtype=torch.int64, device="cuda")
    v = torch.empty(0, dtype=torch.int32, device="cuda")
    ko, vo = rs.rs_sort_pairs(k, v, 64)
    assert ko.numel() == 0 and vo.numel() == 0
