"""The allocation-free sort (gs_sort_pairs_noalloc) against gs_sort_pairs,
through the C ABI: two calls in a row on one GPU, the second on fewer pairs
(the library's scratch keeps the first call's contents), both bit-exact
with the allocating entry point and with numpy's stable sort; sizes above
the scratch limit are rejected before any GPU work."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2410_00486_amd import _lib as L
from synth import scenes

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
NMAX = 1 << 20


def _device_pairs(n, bits, seed):
    keys, vals = scenes.random_keys(1000 + seed, n, max(1, bits - 32))
    kt = torch.from_numpy(keys.view(np.int64).copy()).to(DEV)
    vt = torch.from_numpy(vals.view(np.int32).copy()).to(DEV)
    return keys, vals, kt, vt


def _sort_allocating(kt, vt, bits):
    n = kt.numel()
    tmp = torch.empty(max(int(L.lib().gs_sort_tmp_bytes(n)), 256), dtype=torch.uint8, device=DEV)
    st = L.lib().gs_sort_pairs(ctypes.c_void_p(kt.data_ptr()), ctypes.c_void_p(vt.data_ptr()), n,
                               bits, ctypes.c_void_p(tmp.data_ptr()), None)
    assert st == L.GS_OK, L.lib().gs_last_error()


def _sort_noalloc(kt, vt, bits, stream=None):
    st = L.lib().gs_sort_pairs_noalloc(ctypes.c_void_p(kt.data_ptr()),
                                       ctypes.c_void_p(vt.data_ptr()), kt.numel(), bits, stream)
    assert st == L.GS_OK, L.lib().gs_last_error()


def test_noalloc_sort_matches_allocating_sort_twice():
    # first call at the scratch limit (odd pass count: the result comes back
    # through the scratch), then a smaller one (even pass count)
    for n, bits, seed in ((NMAX, 40, 1), (300_007, 48, 2)):
        print(f"noalloc sort n={n} bits={bits}", flush=True)
        keys, vals, kt, vt = _device_pairs(n, bits, seed)
        ka, va = kt.clone(), vt.clone()
        _sort_noalloc(kt, vt, bits)
        _sort_allocating(ka, va, bits)
        torch.cuda.synchronize()
        assert torch.equal(kt, ka) and torch.equal(vt, va)
        order = np.argsort(keys, kind="stable")
        np.testing.assert_array_equal(kt.cpu().numpy().view(np.uint64), keys[order])
        np.testing.assert_array_equal(vt.cpu().numpy().view(np.uint32), vals[order])


def test_noalloc_sort_on_a_side_stream_and_tiny_sizes():
    s = torch.cuda.Stream()
    for n, bits in ((1, 40), (17, 38), (4097, 44)):
        keys, vals, kt, vt = _device_pairs(n, bits, 3)
        ka, va = kt.clone(), vt.clone()
        torch.cuda.synchronize()
        _sort_noalloc(kt, vt, bits, ctypes.c_void_p(s.cuda_stream))
        s.synchronize()
        _sort_allocating(ka, va, bits)
        torch.cuda.synchronize()
        assert torch.equal(kt, ka) and torch.equal(vt, va)


def test_noalloc_sort_rejects_sizes_above_the_limit():
    kt = torch.zeros(4, dtype=torch.int64, device=DEV)
    vt = torch.zeros(4, dtype=torch.int32, device=DEV)
    # the size check comes first: the pointers are never dereferenced
    st = L.lib().gs_sort_pairs_noalloc(ctypes.c_void_p(kt.data_ptr()),
                                       ctypes.c_void_p(vt.data_ptr()), NMAX + 1, 40, None)
    assert st == L.GS_ERR_INVALID_ARG
    assert b"0.." in L.lib().gs_last_error()
    st = L.lib().gs_sort_pairs_noalloc(ctypes.c_void_p(kt.data_ptr()),
                                       ctypes.c_void_p(vt.data_ptr()), 4, 65, None)
    assert st == L.GS_ERR_INVALID_ARG
    assert int(L.lib().gs_sort_pairs_noalloc(None, None, 0, 40, None)) == L.GS_OK
