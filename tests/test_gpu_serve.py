"""Continuous batching on the GPU: solves of different streams overlap on
their own HIP streams, and every result is the same as when the request is
served alone (bitwise: each solve's kernels are deterministic and share no
state with the others).  Also: a cold stage served through the asynchronous
iteration API equals the blocking solve, and warm starts save iterations."""
import numpy as np
import pytest
import torch

from paper_1708_07481_amd import api
from paper_1708_07481_amd.serve import LibraryBackend, Server, make_streams

pytestmark = pytest.mark.gpu

SPECS = [("e5k", "sbm5k", "emerging"), ("s5k", "sbm5k", "snowball"),
         ("e1k", "sbm1k", "emerging"), ("s1k", "sbm1k", "snowball")]
STAGES = 3


@pytest.fixture(scope="module")
def requests():
    return make_streams(SPECS, rate=50.0, seed=3, stages=STAGES)


def _serve(reqs, slots, warm=True):
    for r in reqs:
        r.warm = warm
    be = LibraryBackend(slots, precision="fp64", maxit=30, tol=1e-2, restarts=4)
    srv = Server(be, slots=slots, hbm_budget=8 << 30)
    out = srv.run(reqs)
    torch.cuda.synchronize()
    return {(r.request.stream, r.request.stage): r for r in out}, srv


def test_alone_equals_mix(requests):
    mix, srv = _serve(list(requests), slots=4)
    assert len(mix) == len(SPECS) * STAGES
    print("mix stats", srv.stats(), flush=True)
    assert srv.peak_active > 1                       # solves really overlapped
    for name, _, _ in SPECS:
        alone, _ = _serve([r for r in requests if r.stream == name], slots=1)
        for (s, st), a in alone.items():
            b = mix[(s, st)]
            assert a.iterations == b.iterations, (s, st)
            assert a.converged == b.converged
            assert np.array_equal(a.theta, b.theta), (s, st, a.theta, b.theta)
            assert np.array_equal(a.labels, b.labels), (s, st)
            assert a.warm_started == b.warm_started == (st > 0)


def test_async_step_equals_blocking_solve(requests):
    r0 = next(r for r in requests if r.stream == "e5k" and r.stage == 0)
    res, _ = _serve([r0], slots=1)
    got = res[("e5k", 0)]
    be = LibraryBackend(1, precision="fp64", maxit=30, tol=1e-2)
    dev = torch.device("cuda:0")
    ctx = be.ctxs[0]
    with torch.cuda.stream(be.streams[0]):
        g = api.graph_build(ctx, r0.n, torch.from_numpy(r0.src).to(dev), torch.from_numpy(r0.dst).to(dev))
        v64, _, _ = api.laplacian_csr(ctx, g)
        x0, warm = be.x0(r0, None)
        assert not warm
        ref = api.lobpcg_solve(ctx, g, v64, x0, 30, 1e-2, "fp64")
        th = ref.theta.cpu().numpy()
    assert ref.iterations == got.iterations
    assert np.array_equal(th, got.theta)


def test_warm_start_saves_iterations(requests):
    warm, _ = _serve(list(requests), slots=4, warm=True)
    cold, _ = _serve(list(requests), slots=4, warm=False)
    for r in requests:
        r.warm = True
    wi = sum(v.iterations for (s, st), v in warm.items() if st > 0)
    ci = sum(v.iterations for (s, st), v in cold.items() if st > 0)
    print(f"later-stage iterations: warm {wi}, cold {ci}", flush=True)
    assert all(not v.warm_started for v in cold.values())
    assert wi < ci


@pytest.mark.parametrize("fp32", [False, True])
def test_warm_fill_bit_exact(orc, fp32):
    """Start rows of the vertices a snowball stage adds: the mean of their old
    neighbours' rows, bit for bit the oracle's (FP32 blocks: the oracle's FP64
    mean rounded once)."""
    import torch
    from paper_1708_07481_amd import api
    from synth import dcsbm, snowball_stages
    from tests.gpu_common import gpu_ctx, host, to_dev
    ctx = gpu_ctx()
    g0 = dcsbm(4000, 10, 20.0, 0.8, seed=7)
    stages, _ = snowball_stages(g0, 10, seed=2)
    (n1, _, _), (n2, s2, d2) = stages[4], stages[5]
    rng = np.random.default_rng(1)
    X = np.zeros((n2, 10))
    X[:n1] = rng.standard_normal((n1, 10))
    if fp32:
        X = X.astype(np.float32).astype(np.float64)
    go = orc.graph_build(n2, s2, d2)
    want = orc.warm_fill(go, n1, X)
    gd = api.graph_build(ctx, n2, to_dev(s2), to_dev(d2))
    Xd = to_dev(X.astype(np.float32) if fp32 else X)
    api.warm_fill(ctx, gd, Xd, n1)
    got = host(Xd)
    assert np.array_equal(got, want.astype(np.float32) if fp32 else want)
    assert np.any(got[n1:] != 0)


def test_warm_fill_edge_cases(orc):
    """n_old == n changes nothing; n_old == 0 has no old neighbours: zero rows."""
    from paper_1708_07481_amd import api
    from synth import dcsbm
    from tests.gpu_common import gpu_ctx, host, to_dev
    ctx = gpu_ctx()
    g0 = dcsbm(500, 4, 10.0, 0.8, seed=3)
    gd = api.graph_build(ctx, g0.n, to_dev(g0.src), to_dev(g0.dst))
    X = np.random.default_rng(2).standard_normal((g0.n, 4))
    Xd = to_dev(X)
    api.warm_fill(ctx, gd, Xd, g0.n)
    assert np.array_equal(host(Xd), X)
    api.warm_fill(ctx, gd, Xd, 0)
    assert np.all(host(Xd) == 0.0)
