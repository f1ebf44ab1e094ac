"""ks_scan_batch_noalloc (the entry point for callers that cannot allocate) against ks_scan_batch.

Both run on the GPU through the C ABI on the same seeded inputs; every field of
every result and every U_c must be bit-identical (the two share the scan
kernels; the no-allocation call keeps the ordered plan's scratch in a fixed
device array). Two calls in a row, the second on a smaller batch, show that
no state of the first call leaks into the second; a third call repeats the
first batch after the smaller one. A few series are also checked against the
oracle, and the host rejects sizes beyond the scratch without launching.
"""

import numpy as np
import pytest

import oracle as O
import paper_2511_05958_amd as P
from paper_2511_05958_amd import synth as S

pytestmark = pytest.mark.gpu


def _batch(recipe, num, first=0):
    b = S.make_batch(recipe, num_series=num, first_series=first)
    x = S.fill_host(b)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    return x, d


def _both(ctx, x, d, max_K):
    import torch

    n = len(d)
    prm = P.ks_params_init(0.05)
    prm.max_K = max_K
    s_d, d_d = P.to_device(x), P.to_device(d)
    rows = int(d["K"].astype(np.int64).sum())
    out_a, out_b = P.empty_results(n), P.empty_results(n)
    out_b.fill_(0xA5)  # stale bytes: every result must be written
    ua = torch.full((rows,), -1, dtype=torch.int32, device="cuda")
    ub = torch.full((rows,), -1, dtype=torch.int32, device="cuda")  # slots of flagged series stay as they are
    P.ks_scan_batch(ctx.handle, s_d, d_d, n, prm, out_a, ua)
    P.ks_scan_batch_noalloc(ctx.handle, s_d, d_d, n, prm, out_b, ub)
    torch.cuda.synchronize()
    a, b = P.results_to_numpy(out_a), P.results_to_numpy(out_b)
    return a, b, ua.cpu().numpy().view(np.uint32), ub.cpu().numpy().view(np.uint32)


def _assert_same(a, b, ua, ub):
    assert a.tobytes() == b.tobytes()
    assert np.array_equal(ua, ub)


def test_noalloc_matches_scan_batch_twice():
    import torch

    assert torch.cuda.is_available()
    with P.Context(0) as ctx:
        # first call: uneven recipe-3 series (K up to 512, N up to 4096)
        x1, d1 = _batch(3, 300)
        a, b, ua, ub = _both(ctx, x1, d1, 512)
        _assert_same(a, b, ua, ub)
        for t in (0, 7, 150, 299):
            o0, K, N = int(d1[t]["offset"]), int(d1[t]["K"]), int(d1[t]["N"])
            o = O.scan_series(x1[o0:o0 + K * N].reshape(K, N))
            assert (b[t]["cp"], b[t]["U"], b[t]["n"], b[t]["m"]) == (o["cp"], o["U"], o["n"], o["m"]), t
        # second call, smaller: 24 recipe-2 series
        x2, d2 = _batch(2, 24, first=500)
        a, b, ua, ub = _both(ctx, x2, d2, 256)
        _assert_same(a, b, ua, ub)
        # the larger batch again after the smaller one
        a, b, ua, ub = _both(ctx, x1, d1, 512)
        _assert_same(a, b, ua, ub)


def test_noalloc_flags_and_limits():
    import ctypes

    import torch

    with P.Context(0) as ctx:
        # malformed descriptors are flagged exactly as ks_scan_batch flags them
        x, d = _batch(2, 6, first=40)
        d[1]["K"] = 1
        d[3]["offset"] = len(x)
        a, b, ua, ub = _both(ctx, x, d, 256)
        _assert_same(a, b, ua, ub)
        assert b[1]["flags"] & P.KS_BAD_SHAPE and b[3]["flags"] & P.KS_OUT_OF_RANGE
        # sizes beyond the scratch are rejected on the host, before any launch
        prm = P.ks_params_init(0.05)
        dummy = torch.zeros(16, dtype=torch.int32, device="cuda")
        rc = P.lib().ks_scan_batch_noalloc(ctx.handle, dummy.data_ptr(), 16, dummy.data_ptr(),
                                           P.KS_NOALLOC_MAX_SERIES + 1, ctypes.byref(prm), dummy.data_ptr(),
                                           None, 0, None)
        assert rc == P.KS_E_RANGE
        assert P.lib().ks_scan_batch_noalloc(ctx.handle, None, 0, None, 0, ctypes.byref(prm), dummy.data_ptr(),
                                             None, 0, None) == P.KS_OK
        assert P.lib().ks_scan_batch_noalloc(None, None, 0, None, 1, ctypes.byref(prm), None, None, 0,
                                             None) == P.KS_E_INVALID
