"""The allocation-free min-max entry point against the allocating one.

fno_field_minmax_noalloc keeps its per-block partials in a fixed device
array instead of a hipMalloc'd buffer; called twice in a row (the second
time on a smaller input, so stale partials of the first call would show),
it must give the same per-channel minima and maxima as fno_field_minmax,
bit for bit (min and max are exact in any order).  Sizes beyond the array
are rejected with LBM_EINVAL before any device work."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call(L, name, x, S, C, P, stream):
    lo = (ctypes.c_float * C)()
    hi = (ctypes.c_float * C)()
    rc = getattr(L, name)(ctypes.c_void_p(x.data_ptr()), S, C, P, stream, lo, hi)
    assert rc == 0, (name, rc, L.fno_last_error(None))
    return np.array(lo[:]), np.array(hi[:])


def test_no_alloc_minmax_matches_the_allocating_entry_point():
    import torch
    from paper_2606_16765_amd._lib import load
    L = load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = torch.Generator(device="cuda").manual_seed(3)
    # (S, C, P): the surrogate's dataset layout first (4 fields of 128x64x64,
    # the 448-sample training set: 229376 partial pairs, 44% of the
    # array), then a smaller ragged input whose partials cover only a
    # prefix of what the first call wrote
    for S, C, P in ((448, 4, 128 * 64 * 64), (3, 5, 4096 * 2 + 77)):
        x = torch.randn((S, C, P), device="cuda", generator=g) * 3.0 + 0.5
        x[S - 1, C - 1, P - 1] = 42.0      # extremes in the last ragged chunk
        x[0, 0, 0] = -37.0
        a = _call(L, "fno_field_minmax", x, S, C, P, stream)
        b = _call(L, "fno_field_minmax_noalloc", x, S, C, P, stream)
        xs = x.transpose(0, 1).reshape(C, -1)
        ref = (xs.min(1).values.cpu().numpy(), xs.max(1).values.cpu().numpy())
        for k in range(2):
            assert np.array_equal(a[k], b[k]), (S, C, P, k, a[k], b[k])
            assert np.array_equal(b[k], ref[k]), (S, C, P, k)


def test_no_alloc_minmax_rejects_sizes_beyond_its_array():
    import torch
    from paper_2606_16765_amd._lib import load
    L = load()
    x = torch.zeros(16, device="cuda")
    lo = (ctypes.c_float * 16)()
    hi = (ctypes.c_float * 16)()
    # 512 samples x 16 channels x 1024 chunks of 4096 points: far beyond
    rc = L.fno_field_minmax_noalloc(ctypes.c_void_p(x.data_ptr()), 512, 16, 4096 * 1024, None, lo, hi)
    assert rc == 1
    assert b"fixed scratch" in L.fno_last_error(None)
