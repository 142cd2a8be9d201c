"""dpmm_suffstats_static (no allocation; scratch in a static device array)
against dpmm_suffstats on the same inputs, through the C ABI: the same
kernels in the same order, so the statistics must agree bit for bit.  Two
calls in a row on one context, the second smaller, for every kernel path
(d <= 4 per-lane accumulators, its sorted large-K fallback, the d <= 32 wave
kernel, the d = 128 matrix-core kernel, the generic sorted kernel, the
multinomial family), and a call too large for the array."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _make(family, d, k_max):
    from paper_2204_08988_amd.sampler import Sampler
    if family == "gaussian":
        return Sampler("gaussian", d, k_max, 2.0, 5, m=np.zeros(d), psi=np.eye(d))
    return Sampler("multinomial", d, k_max, 2.0, 5, beta=np.ones(d))


def _inputs(family, d, K, n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    z = g.integers(0, K, n)
    z[: n // 4] = K - 1
    zs = g.integers(0, 2, n)
    if family == "gaussian":
        x = (g.standard_normal((n, d)) * 1.5 + z[:, None] * 0.25).astype(np.float32)
    else:
        x = g.integers(0, 9, size=(n, d)).astype(np.int32)
    return x, z.astype(np.int32), zs.astype(np.uint8)


def _stats_both(S, x, z, zs, K):
    torch = _torch()
    from paper_2204_08988_amd.sampler import _tptr
    xt, zt, zst = (torch.from_numpy(a).cuda() for a in (x, z, zs))
    S.set_state(K, [0] * K)
    S.suffstats(xt, zt, zst)
    ref = S.get_stats()
    S.set_state(K, [0] * K)
    st = S._L.dpmm_suffstats_static(S._ctx, _tptr(xt), x.shape[0], _tptr(zt), _tptr(zst))
    assert st == 0, S._L.dpmm_last_error(S._ctx)
    got = S.get_stats()
    return ref, got


@pytest.mark.parametrize("family,d,cases", [
    ("gaussian", 2, [(6, 300001), (5, 70000)]),
    ("gaussian", 4, [(14, 200003), (12, 9999)]),
    ("gaussian", 32, [(20, 250000), (7, 30001)]),
    ("gaussian", 128, [(5, 60001), (3, 4000)]),
    ("gaussian", 20, [(9, 120001), (4, 5000)]),
    ("multinomial", 40, [(9, 80000), (3, 1000)]),
])
def test_static_matches_allocating_entry_point(family, d, cases):
    S = _make(family, d, max(K for K, _ in cases) + 1)
    for j, (K, n) in enumerate(cases):
        x, z, zs = _inputs(family, d, K, n, 700 + d + j)
        ref, got = _stats_both(S, x, z, zs, K)
        assert np.array_equal(ref, got)
        assert int(got[..., 0].sum()) == n
    S.close()


def test_static_rejects_calls_beyond_the_array():
    from paper_2204_08988_amd import _lib
    S = _make("gaussian", 128, 8)
    S.set_state(4, [0] * 4)
    one = ctypes.c_void_p(1)  # never dereferenced: the size check comes first
    L = _lib.lib()
    assert L.dpmm_suffstats_static(S._ctx, one, 30_000_000, one, one) == -3  # DPMM_E_CAPACITY
    assert b"scratch" in L.dpmm_last_error(S._ctx)
    S.close()
