"""GPU parity: graph symmetrisation, Laplacian values and SpMM through the
C ABI against the oracle, element by element (bit-exact: integer CSR and
degrees by definition; Laplacian values and FP64 SpMM because both sides
evaluate the same IEEE operations in the same order)."""
import numpy as np
import pytest

from synth import dcsbm
from tests import graphs
from tests.gpu_common import gpu_ctx, host, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _both(orc, ctx, n, src, dst, w=None, algebraic=False):
    from paper_1708_07481_amd import api
    go = orc.graph_build(n, src, dst, w, algebraic)
    gd = api.graph_build(ctx, n, to_dev(src), to_dev(dst), None if w is None else to_dev(w),
                         algebraic)
    return go, gd


def _assert_same_csr(go, gd):
    assert gd.nnz == go.nnz
    assert np.array_equal(host(gd.row_ptr), go.row_ptr)
    assert np.array_equal(host(gd.col)[: go.nnz], go.col)
    assert np.array_equal(host(gd.degree), go.degree)
    assert gd.self_loops == go.self_loops


CASES = [
    ("tiny-multigraph", lambda: graphs.random_multigraph(17, 60, 1)),
    ("isolated+loops", lambda: (50, np.array([0, 1, 1, 7, 7, 3], np.int32),
                                np.array([1, 0, 1, 3, 49, 3], np.int32))),
    ("cliques", lambda: graphs.cliques([5, 9, 13])),
    ("ragged-2k", lambda: graphs.random_multigraph(2003, 30011, 4)),
    ("sbm1k", lambda: (lambda g: (g.n, g.src, g.dst))(dcsbm(1000, 8, 20.0, 0.8, seed=1))),
    ("sbm20k", lambda: (lambda g: (g.n, g.src, g.dst))(
        dcsbm(20000, 32, 40.0, 0.75, "dirichlet", 5.0, seed=2))),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_graph_build_bit_exact(orc, ctx, name, make):
    n, src, dst = make()
    go, gd = _both(orc, ctx, n, src, dst)
    _assert_same_csr(go, gd)


def test_graph_build_algebraic_bit_exact(orc, ctx):
    n, src, dst = graphs.random_multigraph(300, 5000, 9)
    w = np.random.default_rng(9).random(src.shape[0])  # non-dyadic: order of the sums matters
    go, gd = _both(orc, ctx, n, src, dst, w, True)
    _assert_same_csr(go, gd)
    assert np.array_equal(host(gd.w_sym)[: go.nnz], go.w)


def test_graph_build_empty_and_errors(orc, ctx):
    from paper_1708_07481_amd import api
    from paper_1708_07481_amd._lib import SpectralError, SC_E_INVAL
    go, gd = _both(orc, ctx, 5, np.zeros(0, np.int32), np.zeros(0, np.int32))
    _assert_same_csr(go, gd)
    with pytest.raises(SpectralError) as e:
        api.graph_build(ctx, 4, to_dev(np.array([0, 4], np.int32)), to_dev(np.array([1, 2], np.int32)))
    assert e.value.status == SC_E_INVAL


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_laplacian_bit_exact(orc, ctx, name, make):
    from paper_1708_07481_amd import api
    n, src, dst = make()
    go, gd = _both(orc, ctx, n, src, dst)
    vo, dio = orc.laplacian(go)
    v64, v32, di = api.laplacian_csr(ctx, gd, True, True)
    assert np.array_equal(host(v64)[: go.nnz], vo)
    assert np.array_equal(host(v32)[: go.nnz], vo.astype(np.float32))
    assert np.array_equal(host(di), dio)


@pytest.mark.parametrize("k", [1, 5, 8, 19, 32, 44, 64, 96, 98, 130, 160])
def test_spmm_fp64_bit_exact(orc, ctx, k):
    from paper_1708_07481_amd import api
    import torch
    g0 = dcsbm(3001, 7, 24.0, 0.7, "dirichlet", 2.0, seed=k)
    go, gd = _both(orc, ctx, g0.n, g0.src, g0.dst)
    vo, _ = orc.laplacian(go)
    v64, _, _ = api.laplacian_csr(ctx, gd)
    X = np.random.default_rng(k).standard_normal((g0.n, k))
    Yo = orc.spmm(go, vo, X)
    Yd = host(api.spmm(ctx, gd, v64, to_dev(X)))
    assert np.array_equal(Yd, Yo)
    # strided operands (a block inside a wider row-major array)
    big = torch.zeros((g0.n, 3 * k + 5), dtype=torch.float64, device="cuda")
    big[:, k:2 * k] = to_dev(X)
    out = torch.zeros((g0.n, 3 * k + 5), dtype=torch.float64, device="cuda")
    api.spmm(ctx, gd, v64, big[:, k:2 * k], out[:, 2 * k:3 * k])
    assert np.array_equal(host(out[:, 2 * k:3 * k]), Yo)
    assert float(out[:, :2 * k].abs().max()) == 0.0
    # a block inside rows of 3k (the solver's layout: 16-byte aligned when k is even)
    big = torch.zeros((g0.n, 3 * k), dtype=torch.float64, device="cuda")
    big[:, k:2 * k] = to_dev(X)
    out = torch.zeros((g0.n, 3 * k), dtype=torch.float64, device="cuda")
    api.spmm(ctx, gd, v64, big[:, k:2 * k], out[:, 2 * k:3 * k])
    assert np.array_equal(host(out[:, 2 * k:3 * k]), Yo)
    assert float(out[:, :2 * k].abs().max()) == 0.0


@pytest.mark.parametrize("k", [8, 44, 160])
def test_spmm_fp32(orc, ctx, k):
    from paper_1708_07481_amd import api
    g0 = dcsbm(4000, 9, 30.0, 0.7, seed=k + 1)
    go, gd = _both(orc, ctx, g0.n, g0.src, g0.dst)
    vo, _ = orc.laplacian(go)
    _, v32, _ = api.laplacian_csr(ctx, gd, False, True)
    X = np.random.default_rng(k).standard_normal((g0.n, k)).astype(np.float32)
    Yo = orc.spmm(go, vo, X.astype(np.float64))
    Yd = host(api.spmm(ctx, gd, v32, to_dev(X))).astype(np.float64)
    # FP32 arithmetic: |err| <= (deg + 1) * 2^-24 * (|x| + sum |v x|), well below 1e-5 here
    assert np.max(np.abs(Yd - Yo)) < 1e-5 * max(1.0, np.abs(Yo).max())


@pytest.mark.parametrize("k", [4, 32, 64, 96, 128, 160, 192, 200])
def test_spmm_fp32_access_widths_bit_identical(ctx, k):
    """4-byte lane reads of the neighbour rows and 16-byte ones (where k allows
    them) run the same fma chains: identical FP32 results, with and without the
    diagonal and the longest-first row order, also inside rows of 3k."""
    from paper_1708_07481_amd import api
    import torch
    g0 = dcsbm(3001, 7, 24.0, 0.7, "dirichlet", 2.0, seed=k + 3)
    gd = api.graph_build(ctx, g0.n, torch.from_numpy(g0.src).cuda(), torch.from_numpy(g0.dst).cuda())
    _, v32, _ = api.laplacian_csr(ctx, gd, False, True)
    X = to_dev(np.random.default_rng(k).standard_normal((g0.n, k)).astype(np.float32))
    d32 = gd.degree.to(torch.float32)
    order = api.row_order(ctx, gd)
    for diag in (None, d32):
        for o in (None, order):
            Y = api.spmm_ex(ctx, gd, v32, X, order=o, diag=diag)
            Y16 = api.spmm_ex(ctx, gd, v32, X, order=o, diag=diag, lane16=True)
            assert torch.equal(Y, Y16), (k, diag is None, o is None)
    big = torch.zeros((g0.n, 3 * k), dtype=torch.float32, device="cuda")
    big[:, k:2 * k] = X
    out = torch.zeros((g0.n, 3 * k), dtype=torch.float32, device="cuda")
    api.spmm_ex(ctx, gd, v32, big[:, k:2 * k], out[:, 2 * k:3 * k], order=order, lane16=True)
    Y4 = api.spmm_ex(ctx, gd, v32, X, order=order)
    assert torch.equal(out[:, 2 * k:3 * k], Y4)
    assert float(out[:, :2 * k].abs().max()) == 0.0


@pytest.mark.parametrize("k", [32, 160, 200])
def test_spmm_fp32_16bit_gather_copy(ctx, k):
    """FP32 product with the neighbour rows from a 16-bit copy (16-byte lane
    reads where k is a multiple of 32, 2-byte ones otherwise): within the FP32
    rounding of the exact product with the widened copy."""
    from paper_1708_07481_amd import api
    import scipy.sparse as sp
    import torch
    g0 = dcsbm(3001, 7, 24.0, 0.7, "dirichlet", 2.0, seed=k + 5)
    gd = api.graph_build(ctx, g0.n, torch.from_numpy(g0.src).cuda(), torch.from_numpy(g0.dst).cuda())
    _, v32, _ = api.laplacian_csr(ctx, gd, False, True)
    nnz = gd.nnz
    A = sp.csr_matrix((host(v32)[:nnz].astype(np.float64), host(gd.col)[:nnz], host(gd.row_ptr)),
                      shape=(g0.n, g0.n))
    X = np.random.default_rng(k).standard_normal((g0.n, k)).astype(np.float32)
    Xd = to_dev(X)
    order = api.row_order(ctx, gd)
    lens = np.diff(host(gd.row_ptr)).astype(np.float64)[:, None]
    for dt in (torch.float16, torch.bfloat16):
        Xg = Xd.to(dt)
        Xw = Xg.float().cpu().numpy().astype(np.float64)
        ref = X.astype(np.float64) + A @ Xw
        mag = np.abs(X.astype(np.float64)) + abs(A) @ np.abs(Xw)
        for o in (None, order):
            Y = host(api.spmm_ex(ctx, gd, v32, Xd, Xg=Xg, order=o)).astype(np.float64)
            assert np.all(np.abs(Y - ref) <= 2 * (lens + 1) * 2.0 ** -24 * mag + 1e-30), (k, dt)


def test_spmm_ex_argument_errors(ctx):
    """sc_spmm_ex rejects an unknown gather type and a 16-bit gather without
    its copy, before any launch."""
    from paper_1708_07481_amd import _lib, api
    from paper_1708_07481_amd._lib import SC_E_INVAL, SpectralError
    from paper_1708_07481_amd.api import _ptr
    import torch
    g0 = dcsbm(500, 4, 10.0, 0.8, seed=3)
    gd = api.graph_build(ctx, g0.n, torch.from_numpy(g0.src).cuda(), torch.from_numpy(g0.dst).cuda())
    _, v32, _ = api.laplacian_csr(ctx, gd, False, True)
    X = torch.zeros((g0.n, 32), dtype=torch.float32, device="cuda")
    Y = torch.empty_like(X)
    for gather in (_lib.SC_GATHER_FP16, _lib.SC_GATHER_BF16, 7):
        with pytest.raises(SpectralError) as e:
            ctx.check(_lib.lib().sc_spmm_ex(ctx.handle, g0.n, gd.nnz, _ptr(gd.row_ptr),
                                            _ptr(gd.col), _ptr(v32), None, 32, _ptr(X), 32,
                                            None, 0, gather, None, _ptr(Y), 32), "sc_spmm_ex")
        assert e.value.status == SC_E_INVAL
