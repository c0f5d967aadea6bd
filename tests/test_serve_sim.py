"""Host logic of the continuous-batching server on a virtual clock:
admission by slots and device footprint, stage ordering within a stream,
warm-start bookkeeping and eviction, latency accounting."""
import numpy as np
import pytest

from paper_1708_07481_amd.serve import (Request, Server, SimulatedBackend, footprint_bytes,
                                        percentile)


def req(stream, stage, n=1000, m=5000, k=8, arrival=0.0, warm=True):
    e = np.zeros(m, dtype=np.int32)
    return Request(stream=stream, stage=stage, n=n, src=e, dst=e, k=k, arrival=arrival, warm=warm)


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50
    assert percentile(v, 99) == 99
    assert percentile(v, 100) == 100
    assert percentile([7.0], 99) == 7.0
    assert percentile([3, 1, 2], 50) == 2
    assert percentile([1, 2, 3, 4], 0) == 1
    assert np.isnan(percentile([], 50))


def test_every_request_once_and_latency_positive():
    be = SimulatedBackend()
    srv = Server(be, slots=3, hbm_budget=1 << 40)
    rs = [req(f"s{i}", st, arrival=0.01 * i) for i in range(5) for st in range(4)]
    out = srv.run(rs)
    assert sorted((r.request.stream, r.request.stage) for r in out) == \
        sorted((r.stream, r.stage) for r in rs)
    assert all(r.latency > 0 and r.queued >= 0 and r.finished > r.admitted for r in out)
    assert srv.peak_active <= 3
    st = srv.stats()
    assert st["solves"] == 20 and st["p99_latency_s"] >= st["p50_latency_s"]


def test_stage_order_and_warm_start():
    be = SimulatedBackend(cold_iters=12, warm_iters=5)
    srv = Server(be, slots=4, hbm_budget=1 << 40)
    # all stages arrive at once: later stages must still wait for their predecessor
    rs = [req("a", st) for st in range(5)]
    out = srv.run(rs)
    out_a = sorted(out, key=lambda r: r.request.stage)
    for prev, nxt in zip(out_a, out_a[1:]):
        assert nxt.admitted >= prev.finished
    assert [r.warm_started for r in out_a] == [False, True, True, True, True]
    assert [r.iterations for r in out_a] == [12, 5, 5, 5, 5]
    assert srv.peak_active == 1            # one stream: stages are sequential
    # the block of the last stage is not kept; the four earlier blocks were released
    assert srv.warm == {} and be.released == 5


def test_cold_when_disabled():
    be = SimulatedBackend(cold_iters=9, warm_iters=3)
    srv = Server(be, slots=2, hbm_budget=1 << 40)
    out = srv.run([req("a", st, warm=False) for st in range(3)])
    assert all(not r.warm_started and r.iterations == 9 for r in out)


def test_admission_by_footprint():
    be = SimulatedBackend()
    fp = be.footprint(req("x", 0))
    # room for exactly two solves (plus warm blocks of a few KB)
    srv = Server(be, slots=8, hbm_budget=2 * fp + 1_000_000)
    rs = [req(f"s{i}", 0) for i in range(6)]
    out = srv.run(rs)
    assert len(out) == 6
    assert srv.peak_active == 2
    assert srv.peak_bytes <= 2 * fp + 1_000_000


def test_fifo_head_of_line():
    # a large request at the head blocks smaller later ones until memory frees up
    be = SimulatedBackend()
    small, big = req("s", 0, n=1000), req("b", 0, n=100_000, m=500_000, arrival=0.001)
    later = req("t", 0, n=1000, arrival=0.002)
    fs, fb = be.footprint(small), be.footprint(big)
    srv = Server(be, slots=4, hbm_budget=fb + fs // 2)
    out = {r.request.stream: r for r in srv.run([small, big, later])}
    assert out["b"].admitted >= out["s"].finished
    assert out["t"].admitted >= out["b"].admitted


def test_too_large_raises():
    be = SimulatedBackend()
    r = req("x", 0, n=10**6, m=10**7)
    srv = Server(be, slots=1, hbm_budget=be.footprint(r) - 1)
    with pytest.raises(RuntimeError, match="budget"):
        srv.run([r])


def test_missing_stage_raises():
    srv = Server(SimulatedBackend(), slots=2, hbm_budget=1 << 40)
    with pytest.raises(RuntimeError, match="missing earlier stages"):
        srv.run([req("a", 0), req("a", 2)])


def test_eviction_makes_room():
    be = SimulatedBackend()
    a0, a1 = req("a", 0, n=200_000, k=64), req("a", 1, n=200_000, k=64, arrival=10.0)
    b0 = req("b", 0, n=200_000, k=64, arrival=1.0)
    fa = be.footprint(a0)
    warm_bytes = 200_000 * 64 * 4
    # one solve fits, but not one solve plus a resident warm block
    srv = Server(be, slots=2, hbm_budget=fa + warm_bytes // 2)
    out = {(r.request.stream, r.request.stage): r for r in srv.run([a0, a1, b0])}
    assert srv.evictions == 1
    assert not out[("a", 1)].warm_started       # its block was evicted for b's stage 0


def test_processor_sharing_latency():
    # two equal solves started together on a shared device finish together,
    # each taking twice as long as alone
    cost = lambda n, k: 1.0
    alone = Server(SimulatedBackend(cold_iters=4, iter_cost=cost), slots=1, hbm_budget=1 << 40)
    ra = alone.run([req("a", 0)])
    both = Server(SimulatedBackend(cold_iters=4, iter_cost=cost), slots=2, hbm_budget=1 << 40)
    rb = both.run([req("a", 0), req("b", 0)])
    assert ra[0].latency == pytest.approx(4.0)
    assert [r.latency for r in rb] == pytest.approx([8.0, 8.0])


def test_footprint_monotone():
    a = footprint_bytes(1000, 10_000, 8, 4)
    assert footprint_bytes(2000, 10_000, 8, 4) > a
    assert footprint_bytes(1000, 20_000, 8, 4) > a
    assert footprint_bytes(1000, 10_000, 16, 4) > a
    assert footprint_bytes(1000, 10_000, 8, 8) > a
