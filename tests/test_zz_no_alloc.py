"""The allocation-free top-k (dt_topk_noalloc) against dt_topk through the C
ABI: two calls in a row on one GPU, the second with a smaller input, then
an input beyond the fixed scratch (rejected before any launch)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _scores(n, seed):
    """S/N-like values with exact ties, NaNs and values below the threshold."""
    rng = np.random.default_rng(seed)
    x = rng.normal(0.0, 2.0, n).astype(np.float32)
    x[rng.choice(n, n // 50, replace=False)] = np.float32(6.5)       # a block of ties
    x[rng.choice(n, n // 1000 + 1, replace=False)] = np.nan
    return x


def _call(fn, ctx, snr, k, thr):
    import torch
    dev = snr.device
    idx = torch.full((k,), -7, dtype=torch.int64, device=dev)
    val = torch.full((k,), -7.0, dtype=torch.float32, device=dev)
    cnt = torch.full((1,), -7, dtype=torch.int32, device=dev)
    st = fn(ctx.handle, C.c_void_p(snr.data_ptr()), C.c_int64(snr.numel()), C.c_int32(k), C.c_float(thr),
            C.c_void_p(idx.data_ptr()), C.c_void_p(val.data_ptr()), C.c_void_p(cnt.data_ptr()))
    torch.cuda.synchronize()
    return st, idx.cpu().numpy(), val.cpu().numpy(), int(cnt.cpu()[0])


def test_topk_noalloc_matches_topk():
    import torch
    import paper_2503_08854_amd as dt
    L = dt.lib()
    ctx = dt.Context(0)
    dev = torch.device("cuda:0")
    # (n, k, threshold): a multi-round tournament, then a smaller input that
    # reuses the same scratch, then the single-workgroup path
    for n, k, thr, seed in [(3_000_000, 100, 5.0, 1), (200_000, 37, float("-inf"), 2), (5000, 10, 1.0, 3)]:
        snr = torch.from_numpy(_scores(n, seed)).to(dev)
        ref = _call(L.dt_topk, ctx, snr, k, thr)
        got = _call(L.dt_topk_noalloc, ctx, snr, k, thr)
        assert ref[0] == 0 and got[0] == 0, L.dt_last_error().decode()
        assert got[3] == ref[3] and ref[3] > 0
        np.testing.assert_array_equal(got[1], ref[1])
        np.testing.assert_array_equal(got[2].view(np.uint32), ref[2].view(np.uint32))
        # the oracle-free property check: the reported orbits are the k largest
        # (S/N desc, index asc) of those >= threshold
        h = snr.cpu().numpy().astype(np.float64)
        ok = np.nonzero(~np.isnan(h) & (h >= thr))[0]
        order = ok[np.lexsort((ok, -h[ok]))][:k]
        np.testing.assert_array_equal(got[1][:got[3]], order)
    # beyond the fixed scratch: refused with DT_E_ARG, outputs untouched
    big = torch.zeros(200_000_000, dtype=torch.float32, device=dev)
    st, idx, val, cnt = _call(L.dt_topk_noalloc, ctx, big, 4096, 0.0)
    assert st == dt.binding.DT_E_ARG and b"allocation-free" in L.dt_last_error()
    assert cnt == -7 and (idx == -7).all()
    del big
    ctx.close()
