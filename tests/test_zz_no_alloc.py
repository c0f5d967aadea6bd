"""The allocation-free k-means entry point (sc_kmeans_assign_static, for
callers that cannot allocate device memory) against sc_kmeans_assign with a
caller workspace: identical labels, centroids, inertia, chosen restart and
Lloyd count on two calls in a row, the second on a smaller input (the fixed
scratch keeps the first call's contents), and a clear error for a problem
that does not fit the fixed scratch."""
import ctypes as C

import numpy as np
import pytest

from synth import kmeans_draws
from tests.gpu_common import gpu_ctx, host, to_dev

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20


def _opts(K, R, fp32):
    from paper_1708_07481_amd import _lib
    return _lib.sc_kmeans_opts(K, R, 100, 1, int(fp32), 0)


def _run(ctx, X, K, draws, static, ws=None):
    import torch
    from paper_1708_07481_amd import _lib
    lib = _lib.lib()
    n, dim = X.shape
    opts = _opts(K, draws.shape[0], X.dtype == torch.float32)
    labels = torch.full((n,), -7, dtype=torch.int32, device=X.device)
    cent = torch.full((K, dim), np.nan, dtype=torch.float64, device=X.device)
    inertia, iq, br, its = C.c_double(), C.c_uint64(), C.c_int(), C.c_int()
    p = lambda t: C.c_void_p(t.data_ptr())
    args = [ctx.handle, n, dim, p(X), X.stride(0), C.byref(opts), p(draws), None, p(labels),
            p(cent), C.byref(inertia), C.byref(iq), C.byref(br), C.byref(its)]
    if static:
        st = lib.sc_kmeans_assign_static(*args)
    else:
        st = lib.sc_kmeans_assign(*args, p(ws), ws.numel())
    ctx.check(st, "sc_kmeans_assign_static" if static else "sc_kmeans_assign")
    torch.cuda.synchronize()
    return host(labels), host(cent), inertia.value, iq.value, br.value, its.value


def _workspace(ctx, n, dim, K, R, fp32):
    from paper_1708_07481_amd import _lib
    nb = C.c_size_t()
    opts = _opts(K, R, fp32)
    ctx.check(_lib.lib().sc_kmeans_workspace(ctx.handle, n, dim, C.byref(opts), C.byref(nb)),
              "sc_kmeans_workspace")
    return nb.value


def _points(n, dim, K, seed, fp32):
    rng = np.random.default_rng(seed)
    centers = rng.standard_normal((K, dim))
    X = centers[rng.integers(0, K, n)] + 0.5 * rng.standard_normal((n, dim))
    return X.astype(np.float32) if fp32 else X


def test_static_scratch_equals_workspace_entry_point():
    import torch
    ctx = gpu_ctx()
    cases = [(20011, 44, 44, 3, True, 1), (3001, 19, 19, 4, False, 2)]   # second one smaller
    for n, dim, K, R, fp32, seed in cases:
        nb = _workspace(ctx, n, dim, K, R, fp32)
        assert nb <= STATIC_BYTES, nb
        X = _points(n, dim, K, seed, fp32)
        big = np.zeros((n, dim + 3), X.dtype)
        big[:, :dim] = X
        Xd = to_dev(big)[:, :dim]
        draws = to_dev(kmeans_draws(R, K, seed).view(np.int64))
        a = _run(ctx, Xd, K, draws, static=True)
        ws = torch.full((nb,), 0xFF, dtype=torch.uint8, device="cuda")
        b = _run(ctx, Xd, K, draws, static=False, ws=ws)
        print(f"n={n} dim={dim} K={K} R={R}: workspace {nb} bytes, Lloyd {a[5]}, "
              f"best restart {a[4]}")
        assert np.array_equal(a[0], b[0])
        assert np.array_equal(a[1], b[1])
        assert a[2] == b[2] and a[3] == b[3] and a[4] == b[4] and a[5] == b[5]
        assert (a[0] >= 0).all() and np.isfinite(a[1]).all()
    ctx.close()


def test_static_scratch_rejects_large_problems():
    """Checked on the host before any launch: the outputs stay untouched."""
    import torch
    from paper_1708_07481_amd._lib import SC_E_UNSUPPORTED, lib
    ctx = gpu_ctx()
    n, dim, K, R = 200_000, 160, 160, 10
    assert _workspace(ctx, n, dim, K, R, True) > STATIC_BYTES
    X = torch.zeros((n, dim), dtype=torch.float32, device="cuda")
    draws = torch.zeros((R, K), dtype=torch.int64, device="cuda")
    labels = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    cent = torch.zeros((K, dim), dtype=torch.float64, device="cuda")
    opts = _opts(K, R, True)
    p = lambda t: C.c_void_p(t.data_ptr())
    st = lib().sc_kmeans_assign_static(ctx.handle, n, dim, p(X), dim, C.byref(opts), p(draws),
                                       None, p(labels), p(cent), None, None, None, None)
    assert st == SC_E_UNSUPPORTED
    assert b"fixed scratch" in lib().sc_last_error(ctx.handle)
    opts = _opts(4, 65, True)
    st = lib().sc_kmeans_assign_static(ctx.handle, 1000, 8, p(X), 8, C.byref(opts), p(draws),
                                       None, p(labels), p(cent), None, None, None, None)
    assert st == SC_E_UNSUPPORTED
    torch.cuda.synchronize()
    assert (labels == -7).all()
    ctx.close()
