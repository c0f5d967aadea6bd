"""Continuous-batching solve server for streaming graph partitioning.

The paper treats a streaming graph as a sequence of stages, each partitioned
by a LOBPCG solve warm-started from the previous stage's approximate
eigenvectors (Section III): with emerging edges the previous block is reused
as is; in the snowball case the previously seen vertices keep their ids and
come first, so the previous block fills the top rows and the new vertices
start from zero.

This module serves many such streams at once on one GPU:
  - requests (one stage of one stream) arrive over time and wait in a queue;
    a stage becomes eligible once its predecessor has finished, because its
    warm start is that predecessor's result;
  - an eligible request is admitted when a slot is free and its device
    footprint (CSR, Laplacian values, solver and k-means workspaces, blocks)
    fits in the HBM budget next to everything already admitted and every
    resident warm-start block;
  - each tick enqueues one LOBPCG iteration for every admitted solve that has
    none in flight (each slot owns a library context and HIP stream, so the
    iterations of different solves overlap on the device) and polls the
    in-flight ones; finished solves run k-means, record their latency, keep
    their eigenvector block resident as the stream's next warm start and
    release their memory.
The scheduling logic is backend-independent: `LibraryBackend` drives the HIP
library, `SimulatedBackend` replays a cost model on a virtual clock (used by
the CPU tests of admission, queueing and latency accounting).
"""
from __future__ import annotations

import heapq
import math
import time
from dataclasses import dataclass, field
from typing import Any, Callable

import numpy as np


@dataclass
class Request:
    stream: str                 # stream (graph) identifier
    stage: int                  # 0-based stage index within the stream
    n: int                      # vertices of this stage
    src: np.ndarray             # directed COO edges of this stage (int32)
    dst: np.ndarray
    k: int                      # eigenvectors = clusters
    arrival: float              # seconds on the server clock
    kind: str = "emerging"      # "emerging" or "snowball"
    warm: bool = True           # warm start from the previous stage if available
    seed: int = 0               # seed of the Gaussian start block when cold
    precision: str | None = None  # "fp64" | "fp32" | "fp32_bf16gram"; None: backend default
    truth: np.ndarray | None = None


@dataclass
class Result:
    request: Request
    arrived: float              # server clock at arrival
    admitted: float
    finished: float
    iterations: int
    converged: bool
    theta: np.ndarray
    labels: np.ndarray
    warm_started: bool

    @property
    def latency(self) -> float:
        return self.finished - self.arrived

    @property
    def queued(self) -> float:
        return self.admitted - self.arrived


@dataclass
class Job:
    request: Request
    slot: int
    footprint: int
    arrived: float
    admitted: float
    handle: Any = None          # backend state
    in_flight: bool = False
    done: bool = False
    warm_started: bool = False


def _name(req: Request) -> str:
    return f"{req.stream} stage {req.stage} (n={req.n}, edges={len(req.src)}, k={req.k})"


def percentile(values, q) -> float:
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence."""
    v = sorted(values)
    if not v:
        return float("nan")
    rank = max(1, math.ceil(q / 100.0 * len(v)))
    return float(v[rank - 1])


class Server:
    def __init__(self, backend, slots: int = 4, hbm_budget: int = 64 << 30,
                 clock: Callable[[], float] | None = None):
        if slots < 1:
            raise ValueError("need at least one slot")
        self.backend = backend
        self.slots = slots
        self.hbm_budget = int(hbm_budget)
        self.clock = clock or backend.now
        self.waiting: list[tuple[float, int, Request]] = []   # heap by arrival
        self.ready: list[tuple[float, Request]] = []   # arrived, in arrival order
        self.active: dict[int, Job] = {}
        self.results: list[Result] = []
        self.warm: dict[str, tuple[Any, int, int]] = {}        # stream -> (block, n, bytes)
        self.last_stage: dict[str, int] = {}                   # stream -> finished stage
        self.remaining: dict[str, int] = {}                    # stream -> stages still to come
        self.peak_bytes = 0
        self.peak_active = 0
        self.evictions = 0
        self.t0 = None              # server clock when run() started; arrivals are offsets
        self._seq = 0

    # -- bookkeeping -------------------------------------------------------
    def used_bytes(self) -> int:
        return sum(j.footprint for j in self.active.values()) + \
            sum(b for _, _, b in self.warm.values())

    def submit(self, req: Request):
        if self.t0 is None:
            self.t0 = self.clock()
        heapq.heappush(self.waiting, (self.t0 + req.arrival, self._seq, req))
        self._seq += 1
        self.remaining[req.stream] = self.remaining.get(req.stream, 0) + 1

    def _eligible(self, req: Request) -> bool:
        return req.stage == 0 or self.last_stage.get(req.stream, -1) == req.stage - 1

    # -- one scheduling round ---------------------------------------------
    def tick(self) -> bool:
        """One round; returns True if anything changed."""
        now = self.clock()
        progressed = False
        while self.waiting and self.waiting[0][0] <= now:
            t_arr, _, req = heapq.heappop(self.waiting)
            self.ready.append((t_arr, req))
            progressed = True
        # admission: FIFO over eligible requests, by slot and footprint
        free = [s for s in range(self.slots) if s not in self.active]
        for item in list(self.ready):
            t_arr, req = item
            if not free:
                break
            if not self._eligible(req):
                continue
            fp = self.backend.footprint(req)
            if self.used_bytes() + fp > self.hbm_budget and not self.active:
                self._evict(fp, keep=req.stream)
            if self.used_bytes() + fp > self.hbm_budget:
                if not self.active:
                    raise RuntimeError(f"request {req.stream}/{req.stage} needs {fp} bytes, "
                                       f"more than the {self.hbm_budget}-byte budget")
                break                       # FIFO: wait for memory to free up
            warm = self.warm.get(req.stream) if req.warm else None
            slot = free.pop(0)
            self.ready = [it for it in self.ready if it is not item]
            job = Job(req, slot, fp, t_arr, now)
            try:
                job.handle, job.warm_started = self.backend.start(slot, req, warm)
            except Exception as e:
                raise RuntimeError(f"starting {_name(req)} (warm start: {warm is not None}) "
                                   f"failed: {e}") from e
            self.active[slot] = job
            self.peak_bytes = max(self.peak_bytes, self.used_bytes())
            self.peak_active = max(self.peak_active, len(self.active))
            progressed = True
        # one iteration in flight for every admitted solve
        for job in self.active.values():
            if not job.in_flight and not job.done:
                self.backend.step_async(job.handle)
                job.in_flight = True
                progressed = True
        for slot, job in list(self.active.items()):
            if not job.in_flight:
                continue
            try:
                ready, done = self.backend.poll(job.handle)
                if not ready:
                    continue
                job.in_flight = False
                progressed = True
                if done:
                    self._finish(slot, job)
            except Exception as e:
                if isinstance(e, RuntimeError) and str(e).startswith("solve of "):
                    raise
                raise RuntimeError(f"solve of {_name(job.request)} (warm start: "
                                   f"{job.warm_started}) failed: {e}") from e
        return progressed

    def _evict(self, need: int, keep: str):
        """Drop resident warm-start blocks, oldest first, until `need` more
        bytes fit; the streams they belonged to restart cold."""
        for stream in list(self.warm):
            if self.used_bytes() + need <= self.hbm_budget:
                break
            if stream == keep:
                continue
            block, _, _ = self.warm.pop(stream)
            self.backend.release(block)
            self.evictions += 1

    def _finish(self, slot: int, job: Job):
        req = job.request
        out = self.backend.finish(job.handle)
        now = self.clock()
        del self.active[slot]
        old = self.warm.pop(req.stream, None)
        if old is not None:
            self.backend.release(old[0])
        self.remaining[req.stream] -= 1
        if self.remaining[req.stream] > 0:
            self.warm[req.stream] = (out["block"], req.n, out["block_bytes"])
        else:
            self.backend.release(out["block"])
        self.last_stage[req.stream] = req.stage
        self.results.append(Result(req, job.arrived, job.admitted, now, out["iterations"],
                                   out["converged"], out["theta"], out["labels"], job.warm_started))

    def run(self, requests=(), idle_wait: float = 2e-4):
        self.t0 = self.clock()
        for r in requests:
            self.submit(r)
        while self.waiting or self.ready or self.active:
            if not self.tick():
                if not self.active and not self.waiting and not any(
                        self._eligible(r) for _, r in self.ready):
                    missing = sorted({(r.stream, r.stage) for _, r in self.ready})
                    raise RuntimeError(f"requests can never start (missing earlier stages): {missing}")
                nxt = self.waiting[0][0] if self.waiting else None
                self.backend.idle(nxt, idle_wait)
        return self.results

    def stats(self) -> dict:
        lat = [r.latency for r in self.results]
        if not self.results:
            return {}
        t0 = min(r.arrived for r in self.results)
        t1 = max(r.finished for r in self.results)
        return {"solves": len(self.results), "makespan_s": t1 - t0,
                "solves_per_s": len(self.results) / max(t1 - t0, 1e-12),
                "p50_latency_s": percentile(lat, 50), "p99_latency_s": percentile(lat, 99),
                "mean_latency_s": float(np.mean(lat)),
                "mean_queue_s": float(np.mean([r.queued for r in self.results])),
                "iterations": int(sum(r.iterations for r in self.results)),
                "peak_bytes": self.peak_bytes, "peak_active": self.peak_active,
                "evictions": self.evictions,
                "warm_started": sum(r.warm_started for r in self.results)}


# ---------------------------------------------------------------------------
# Backends
# ---------------------------------------------------------------------------
class SimulatedBackend:
    """Virtual-clock backend: a solve of n vertices and k vectors costs
    `iter_cost(n, k)` seconds per iteration on its own, slots share the device
    by processor sharing, warm starts take `warm_iters` iterations and cold
    starts `cold_iters`.  Footprints follow the same formula as the GPU path."""

    def __init__(self, cold_iters=12, warm_iters=5, iter_cost=None, finish_cost=0.0):
        self.t = 0.0
        self.cold_iters = cold_iters
        self.warm_iters = warm_iters
        self.iter_cost = iter_cost or (lambda n, k: 1e-9 * n * k + 1e-4)
        self.finish_cost = finish_cost
        self.running: dict[int, dict] = {}
        self.released = 0

    def now(self):
        return self.t

    def footprint(self, req: Request) -> int:
        return footprint_bytes(req.n, 2 * len(req.src), req.k, 4, restarts=10)

    def start(self, slot, req, warm):
        warm_ok = warm is not None
        h = {"slot": slot, "req": req, "left": self.warm_iters if warm_ok else self.cold_iters,
             "iters": 0, "busy_until": None, "work": 0.0}
        return h, warm_ok

    def step_async(self, h):
        h["work"] = self.iter_cost(h["req"].n, h["req"].k)
        self.running[id(h)] = h

    def _advance(self, dt):
        # processor sharing among the running iterations
        while dt > 0 and self.running:
            share = len(self.running)
            first = min(self.running.values(), key=lambda h: h["work"])
            need = first["work"] * share
            step = min(dt, need)
            for h in self.running.values():
                h["work"] -= step / share
            self.t += step
            dt -= step
            for key in [k for k, h in self.running.items() if h["work"] <= 1e-15]:
                h = self.running.pop(key)
                h["iters"] += 1
                h["left"] -= 1
                h["completed"] = True
        if dt > 0:
            self.t += dt

    def poll(self, h):
        if h.get("completed"):
            h["completed"] = False
            return True, h["left"] <= 0
        return False, False

    def finish(self, h):
        self.t += self.finish_cost
        req = h["req"]
        return {"iterations": h["iters"], "converged": True, "theta": np.zeros(req.k),
                "labels": np.zeros(req.n, dtype=np.int32), "block": ("block", req.stream, req.stage),
                "block_bytes": req.n * req.k * 4}

    def release(self, block):
        self.released += 1

    def idle(self, next_arrival, wait):
        # jump to the next event: an iteration completing or a request arriving
        cands = []
        if self.running:
            share = len(self.running)
            cands.append(min(h["work"] for h in self.running.values()) * share)
        if next_arrival is not None:
            cands.append(max(next_arrival - self.t, 0.0))
        self._advance(min(cands) if cands else wait)


def footprint_bytes(n: int, nnz: int, k: int, elem: int, restarts: int = 10,
                    lobpcg_ws: int | None = None, kmeans_ws: int | None = None,
                    graph_ws: int | None = None) -> int:
    """Device bytes of one admitted solve: edges, CSR, Laplacian values, start
    and result blocks, and the graph-build, solver and k-means workspaces
    (the library's exact *_workspace sizes; closed-form estimates only where
    they are not given, as in the CPU scheduling tests)."""
    m = nnz // 2
    kp = (k + 3) // 4 * 4
    # edges (int32 src, dst), row_ptr, col, degree, values (FP64 and/or FP32), dinv_sqrt
    graph = 8 * m + 8 * (n + 1) + 4 * nnz + 8 * n + elem * nnz + 8 * n
    if lobpcg_ws is None:
        lobpcg_ws = 2 * n * 3 * kp * elem + 8 * (3 * kp) ** 2 * 12 + 64 * n
    if kmeans_ws is None:
        kmeans_ws = 8 * n * k * 2 + restarts * n * (8 * 6 + 4 * 6)
    if graph_ws is None:
        graph_ws = 2 * m * (8 * 3 + 4 * 2) + 64 * m
    # the graph-build workspace is released before the solve's and k-means's
    return graph + 2 * n * k * elem + lobpcg_ws + max(kmeans_ws, graph_ws)


class LibraryBackend:
    """Drives the HIP library: one context (own HIP stream) per slot."""

    def __init__(self, slots: int, precision: str = "fp32", maxit: int = 30, tol: float = 1e-2,
                 restarts: int = 10, kmeans_iters: int = 100, device: int = 0,
                 warm_fill: str = "neighbors"):
        import torch
        from . import api
        self.torch = torch
        self.api = api
        self.dev = torch.device(f"cuda:{device}")
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]
        self.ctxs = [api.Context(device, stream=s) for s in self.streams]
        self.precision = precision
        self.maxit, self.tol, self.restarts, self.kmeans_iters = maxit, tol, restarts, kmeans_iters
        if warm_fill not in ("neighbors", "zero"):
            raise ValueError(f"warm_fill must be 'neighbors' or 'zero', not {warm_fill!r}")
        self.warm_fill = warm_fill   # rows of vertices a snowball stage adds

    def _prec(self, req: Request):
        prec = req.precision or self.precision
        fp64 = prec == "fp64"
        return prec, (8 if fp64 else 4), (self.torch.float64 if fp64 else self.torch.float32)

    def now(self):
        return time.perf_counter()

    def footprint(self, req: Request) -> int:
        import ctypes as C
        from ._lib import lib, sc_kmeans_opts
        nnz_cap = 2 * len(req.src)
        prec, elem, _ = self._prec(req)
        ctx = self.ctxs[0]
        opts = self.api.lobpcg_opts(req.k, self.maxit, self.tol, prec, req.k)
        lw = self.api.lobpcg_workspace(ctx, req.n, nnz_cap, opts)
        kw = C.c_size_t()
        ko = sc_kmeans_opts(req.k, self.restarts, self.kmeans_iters, 1, int(elem == 4), 0)
        ctx.check(lib().sc_kmeans_workspace(ctx.handle, req.n, req.k, C.byref(ko), C.byref(kw)),
                  "sc_kmeans_workspace")
        gw = C.c_size_t()
        ctx.check(lib().sc_graph_build_workspace(ctx.handle, req.n, len(req.src), C.byref(gw)),
                  "sc_graph_build_workspace")
        return footprint_bytes(req.n, nnz_cap, req.k, elem, self.restarts, lw, kw.value, gw.value)

    def x0(self, req: Request, warm, stream=None, ctx=None, g=None):
        """Start block: the previous stage's eigenvectors or a seeded Gaussian
        block.  The rows of vertices a snowball stage adds are the mean of
        their old neighbours' rows (warm_fill "neighbors", with the stage's
        graph g on ctx) or zero."""
        torch = self.torch
        _, _, dtype = self._prec(req)
        if warm is not None:
            block, n_prev, _ = warm
            if stream is not None:
                block.record_stream(stream)
            if n_prev == req.n and block.dtype == dtype:
                return block, True
            x0 = torch.zeros((req.n, req.k), dtype=dtype, device=self.dev)
            x0[:n_prev].copy_(block)        # snowball: old vertices first
            if self.warm_fill == "neighbors" and g is not None:
                self.api.warm_fill(ctx, g, x0, n_prev)
            return x0, True
        # cold start: a Gaussian block from the device Philox stream keyed by
        # the request's seed (Section III), on the slot's context
        X = torch.empty((req.n, req.k), dtype=dtype, device=self.dev)
        self.api.randn(ctx if ctx is not None else self.ctxs[0], req.n, req.k, req.seed, 2,
                       "normal", dtype, out=X)
        return X, False

    def start(self, slot: int, req: Request, warm):
        import ctypes as C
        from ._lib import lib
        torch, api = self.torch, self.api
        ctx = self.ctxs[slot]
        prec, elem, _ = self._prec(req)
        with torch.cuda.stream(self.streams[slot]):
            src = torch.from_numpy(np.ascontiguousarray(req.src)).to(self.dev, non_blocking=False)
            dst = torch.from_numpy(np.ascontiguousarray(req.dst)).to(self.dev, non_blocking=False)
            g = api.graph_build(ctx, req.n, src, dst)
            v64, v32, _ = api.laplacian_csr(ctx, g, elem == 8, elem == 4)
            val = v64 if elem == 8 else v32
            x0, warm_ok = self.x0(req, warm, self.streams[slot], ctx, g)
            opts = api.lobpcg_opts(req.k, self.maxit, self.tol, prec, req.k)
            nb = api.lobpcg_workspace(ctx, req.n, g.nnz, opts)
            ws = ctx.workspace(nb)
            state = C.c_void_p()
            done = C.c_int()
            p = lambda t: C.c_void_p(t.data_ptr())
            ctx.check(lib().sc_lobpcg_begin(ctx.handle, req.n, g.nnz, p(g.row_ptr), p(g.col), p(val),
                                            C.byref(opts), p(x0), p(ws), nb, C.byref(state),
                                            C.byref(done)), "sc_lobpcg_begin")
        h = {"slot": slot, "req": req, "g": g, "val": val, "x0": x0, "ws": ws, "state": state,
             "opts": opts, "done": bool(done.value)}
        return h, warm_ok

    def step_async(self, h):
        from ._lib import lib
        if h["done"]:
            return
        ctx = self.ctxs[h["slot"]]
        ctx.check(lib().sc_lobpcg_step_async(ctx.handle, h["state"]), "sc_lobpcg_step_async")

    def poll(self, h):
        import ctypes as C
        from ._lib import lib
        if h["done"]:
            return True, True
        ctx = self.ctxs[h["slot"]]
        ready, done = C.c_int(), C.c_int()
        ctx.check(lib().sc_lobpcg_step_poll(ctx.handle, h["state"], C.byref(ready), C.byref(done)),
                  "sc_lobpcg_step_poll")
        h["done"] = bool(done.value)
        return bool(ready.value), bool(done.value)

    def finish(self, h):
        import ctypes as C
        from ._lib import lib, sc_lobpcg_info
        torch, api = self.torch, self.api
        req = h["req"]
        ctx = self.ctxs[h["slot"]]
        _, _, dtype = self._prec(req)
        with torch.cuda.stream(self.streams[h["slot"]]):
            X = torch.empty((req.n, req.k), dtype=dtype, device=self.dev)
            theta = torch.empty(req.k, dtype=torch.float64, device=self.dev)
            info = sc_lobpcg_info()
            p = lambda t: C.c_void_p(t.data_ptr())
            ctx.check(lib().sc_lobpcg_end(ctx.handle, h["state"], p(X), p(theta), None,
                                          C.byref(info)), "sc_lobpcg_end")
            from synth import kmeans_draws
            draws = torch.from_numpy(kmeans_draws(self.restarts, req.k, req.seed + 7919 * req.stage)
                                     .view(np.int64)).to(self.dev)
            km = api.kmeans_assign(ctx, X, req.k, draws, max_iter=self.kmeans_iters)
            labels = km.labels.cpu().numpy()
            th = theta.cpu().numpy()
        return {"iterations": info.iterations, "converged": bool(info.converged), "theta": th,
                "labels": labels, "block": X, "block_bytes": X.numel() * X.element_size()}

    def release(self, block):
        pass                                  # torch frees the tensor when unreferenced

    def close(self):
        """Synchronise the slots' streams and destroy their library contexts."""
        for s in self.streams:
            s.synchronize()
        for c in self.ctxs:
            c.close()

    def idle(self, next_arrival, wait):
        if next_arrival is not None:
            dt = next_arrival - self.now()
            if dt > 0:
                time.sleep(min(dt, wait))
                return
        time.sleep(0)


# ---------------------------------------------------------------------------
# Workload: Poisson-arriving streams of staged graphs
# ---------------------------------------------------------------------------
def make_streams(specs, rate: float, seed: int = 0, stages: int = 10, warm: bool = True,
                 stage_rate: float | None = None):
    """specs: list of (name, config-name, kind).  Stream starts follow a
    Poisson process of the given rate (per second); within a stream, stage
    arrivals follow a Poisson process of rate `stage_rate` (all at the stream
    start if None), and a stage is held in any case until its predecessor has
    finished.  Returns the list of requests."""
    from synth import emerging_stages, snowball_stages
    from synth.configs import CONFIGS, graph_for
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for si, (name, cfg_name, kind) in enumerate(specs):
        t += rng.exponential(1.0 / rate)
        cfg = CONFIGS[cfg_name]
        g = graph_for(cfg_name, seed=1000 + si)
        if kind == "snowball":
            st, truth = snowball_stages(g, stages, seed=si)
        else:
            st, truth = emerging_stages(g, stages, seed=si)
        ta = t
        for s, (n, src, dst) in enumerate(st):
            if s > 0 and stage_rate:
                ta += rng.exponential(1.0 / stage_rate)
            reqs.append(Request(stream=name, stage=s, n=n, src=src, dst=dst, k=cfg["k"],
                                arrival=ta, kind=kind, warm=warm, seed=si,
                                precision=cfg["precision"], truth=truth[:n]))
    return reqs
