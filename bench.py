#!/usr/bin/env python3
"""Time-to-partition of the spectral-clustering hot path on one MI355X.

One step = the whole path on one synthetic graph already resident in HBM:
symmetrised CSR build, normalised Laplacian, LOBPCG (no preconditioning) to
relative residual 1e-2 from a Gaussian start block, and k-means on the
row-normalised eigenvectors.  The default workload is the 2M-vertex /
40M-edge / 160-block degree-corrected SBM (Table I's largest static graph
shape) in FP32 with FP64 Rayleigh-Ritz.

    python bench.py [--steps K] [--warmup W] [--config sbm2m]
    python bench.py --config serve [--streams S] [--rate R]

The serve workload is the continuous-batching mix: Poisson-arriving streams
of 5K / 50K / 500K-vertex graphs (60/30/10 % by count, half emerging-edge,
half snowball), each in 10 stages, every stage warm-started from the previous
stage's eigenvectors; a second pass serves the same requests cold.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from types import SimpleNamespace

HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
X0_SEED, X0_STREAM = 1, 2       # key of the start block's Philox stream


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def spmm_algorithmic_bytes(n, nnz, k, s, diag=False):
    """Compulsory bytes of one Y = L X: row pointers, column indices and
    values once (and the diagonal, for D - W), X read once and Y written once."""
    return 8 * (n + 1) + nnz * (4 + s) + 2 * n * k * s + (n * s if diag else 0)


def gram_counters(cfg_name):
    """Counter record of the Gram kernel (MFMA busy fraction, HBM traffic) if it
    was taken on the current dense.hip; else None."""
    path = os.path.join(HERE, "profiles", f"gram_{cfg_name}_counters.json")
    src = os.path.join(HERE, "paper_1708_07481_amd", "csrc", "dense.hip")
    try:
        with open(path) as fh:
            t = json.load(fh)
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if t.get("dense_source_sha256") != sha:
            return None
        return {"mfma_busy_frac": t["mfma_busy_frac"], "mfma_flop_per_launch": t["mfma_flop_per_launch"],
                "traffic": t["traffic_bytes_per_launch"]}
    except (OSError, ValueError, KeyError):
        return None


def spmm_traffic(cfg_name, launches_bytes):
    """HBM bytes per SpMM launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(HERE, "profiles", f"spmm_{cfg_name}_traffic.json")
    src = os.path.join(HERE, "paper_1708_07481_amd", "csrc", "spmm.hip")
    try:
        with open(path) as fh:
            t = json.load(fh)
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if t.get("spmm_source_sha256") != sha:
            return None
        return t.get("bytes_per_launch")
    except (OSError, ValueError):
        return None


def copy_rate_gbs(torch, dev):
    """Achievable HBM rate of a plain device copy: 512 MiB read and 512 MiB
    written per launch (torch.mul by 1.0), 2 untimed then 10 timed launches
    between HIP events on torch's stream; bytes read plus written per second."""
    x = torch.ones(128 << 20, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    for _ in range(2):
        torch.mul(x, 1.0, out=y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        torch.mul(x, 1.0, out=y)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 10
    return 2 * x.numel() * 4 / (ms * 1e-3) / 1e9


def host_info():
    """Host CPU of this run: logical CPUs, model name and sockets (lscpu)."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            key, _, val = line.partition(":")
            if key.strip() in ("Model name", "Socket(s)", "Thread(s) per core", "Core(s) per socket"):
                info[key.strip()] = val.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_record_path(name):
    return os.path.join(HERE, "profiles", f"cpu_baseline_{name}.json")


def record_cpu_baseline(args, cfg, g0):
    """One-time full-size measurement of the oracle on this host, written to
    profiles/cpu_baseline_<workload>.json: graph build + Laplacian, one SpMM
    with the k-column block, LOBPCG start-up and one iteration, and k-means
    (row normalisation, one restart's seeding with its first assignment, one
    Lloyd update), all on the full graph and its k = B eigenvector block."""
    import oracle
    from synth import gaussian_block, kmeans_draws
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n, k = g0.n, cfg["k"]
    os.environ.setdefault("ORC_TRACE", "1")
    log(f"oracle on the full graph: n={n}, k={k}, {threads} threads")
    t0 = time.perf_counter()
    g = oracle.graph_build(g0.n, g0.src, g0.dst)
    val, _ = oracle.laplacian(g)
    t_graph = time.perf_counter() - t0
    log(f"graph build + Laplacian {t_graph:.1f} s")
    X0 = gaussian_block(n, k, 1)
    t0 = time.perf_counter()
    Y = oracle.spmm(g, val, X0)
    t_spmm = time.perf_counter() - t0
    del Y
    log(f"SpMM {t_spmm:.1f} s")
    r = oracle.lobpcg(g, val, X0, 1, 0.0)
    del X0
    log(f"LOBPCG start-up {r.seconds_setup:.1f} s, one iteration {r.seconds_iters:.1f} s")
    km = oracle.kmeans(r.X, k, kmeans_draws(1, k, 1), max_iter=1)
    t_norm, t_seed, t_lloyd, n_lloyd = km.timing
    log(f"k-means: normalisation {t_norm:.1f} s, seeding {t_seed:.1f} s, "
        f"{n_lloyd} Lloyd update {t_lloyd:.1f} s")
    rec = {
        "workload": args.config, "n": n, "nnz": int(g.nnz), "k": k, "kind": "oracle",
        "threads": threads, "host": host_info(),
        "seconds": {"graph_build_laplacian": round(t_graph, 3), "spmm": round(t_spmm, 3),
                    "lobpcg_setup": round(r.seconds_setup, 3),
                    "lobpcg_iteration": round(r.seconds_iters, 3),
                    "kmeans_normalise": round(t_norm, 3),
                    "kmeans_seeding_per_restart": round(t_seed, 3),
                    "kmeans_lloyd_update": round(t_lloyd / max(n_lloyd, 1), 3)},
        "command": f"OMP_NUM_THREADS={threads} python bench.py --config {args.config} "
                   "--record-cpu-baseline",
    }
    with open(cpu_record_path(args.config), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return rec


def cpu_baseline(g0, cfg, name, gpu_iters, restarts, lloyd_iters, combinatorial=False):
    """The oracle on this host's cores for one partition of the workload.
    Timed live on the full graph (a bounded sample, about 15 s of CPU work):
    graph build + Laplacian, one SpMM with the k-column block, and k-means
    normalisation plus one restart's seeding.  The phases too long to repeat
    in every run come from the full-size record
    profiles/cpu_baseline_<workload>.json (measured once on a GPU machine's host
    by record_cpu_baseline): LOBPCG start-up and per-iteration time, k-means
    per-Lloyd-update time.  One partition = graph + start-up + the GPU
    solve's iterations x iteration + normalisation + restarts x seeding +
    restarts x the GPU's Lloyd updates (of its slowest restart, so an upper
    estimate) x update."""
    import oracle
    from synth import gaussian_block, kmeans_draws
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    g = oracle.graph_build(g0.n, g0.src, g0.dst)
    val, diag = oracle.laplacian_combinatorial(g) if combinatorial else (oracle.laplacian(g)[0], None)
    t_graph = time.perf_counter() - t0
    X0 = gaussian_block(g0.n, cfg["k"], 1)
    t0 = time.perf_counter()
    oracle.spmm(g, val, X0, diag)
    t_spmm = time.perf_counter() - t0
    del g, val
    # one k-means++ seeding (with its first assignment) on the n x k block
    km = oracle.kmeans(X0, cfg["k"], kmeans_draws(1, cfg["k"], 1), max_iter=0)
    t_norm, t_seed = km.timing[0], km.timing[1]
    del X0
    try:
        with open(cpu_record_path(name)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        rec = None
    if rec is None or rec.get("n") != g0.n or rec.get("k") != cfg["k"] or combinatorial:
        return {"value": None, "unit": "s", "cores": threads, "kind": "oracle",
                "sample": (f"live on the full graph: graph build + Laplacian {t_graph:.1f} s, "
                           f"one SpMM with k={cfg['k']} columns {t_spmm:.1f} s; no full-size "
                           f"record of the other phases for this workload")}
    sec = rec["seconds"]
    value = (t_graph + sec["lobpcg_setup"] + gpu_iters * sec["lobpcg_iteration"]
             + t_norm + restarts * t_seed
             + restarts * lloyd_iters * sec["kmeans_lloyd_update"])
    return {"value": round(value, 1), "unit": "s", "cores": threads, "kind": "oracle",
            "host": host_info(),
            "sample": (f"oracle on the full graph (n={g0.n}, k={cfg['k']}). Live in this run "
                       f"(about {t_graph + t_spmm + t_norm + t_seed:.0f} s of CPU): graph build "
                       f"+ Laplacian {t_graph:.1f} s, one SpMM {t_spmm:.1f} s (the record's: "
                       f"{sec['spmm']:.1f} s), k-means normalisation {t_norm:.1f} s and one "
                       f"restart's seeding with its first assignment {t_seed:.1f} s (the "
                       f"record's: {sec['kmeans_seeding_per_restart']:.1f} s). From the "
                       f"full-size record profiles/cpu_baseline_{name}.json "
                       f"({rec['threads']} threads on {rec['host'].get('Model name', '?')}): "
                       f"LOBPCG start-up {sec['lobpcg_setup']:.1f} s and {gpu_iters} iterations "
                       f"x {sec['lobpcg_iteration']:.1f} s, {restarts} restarts x {lloyd_iters} "
                       f"Lloyd updates x {sec['kmeans_lloyd_update']:.1f} s (the GPU's Lloyd "
                       f"count of its slowest restart: an upper estimate). One partition = "
                       f"graph + start-up + iterations + normalisation + {restarts} seedings + "
                       f"Lloyd updates")}


def serve_specs(S, seed=11):
    """The serving mix: 60/30/10 % of S streams are 5K / 50K / 500K graphs,
    alternately emerging-edge and snowball."""
    import numpy as np
    n5 = round(0.6 * S)
    n50 = round(0.3 * S)
    sizes = ["sbm5k"] * n5 + ["sbm50k"] * n50 + ["sbm500k"] * (S - n5 - n50)
    order = np.random.default_rng(seed).permutation(S)
    return [(f"{sizes[i]}-{j}", sizes[i], "emerging" if j % 2 == 0 else "snowball")
            for j, i in enumerate(order)], (n5, n50, S - n5 - n50)


def serve_pass(be, reqs, slots, budget, warm=True, discard_before=0.0, stages=10):
    """Serve the requests (warm or cold starts) on the library backend; stats
    over the requests that arrive at or after `discard_before` seconds."""
    import numpy as np
    import torch
    from paper_1708_07481_amd.metrics import partition_scores
    from paper_1708_07481_amd.serve import Server, percentile
    batch = [_clone(r, warm=warm) for r in reqs]
    srv = Server(be, slots=slots, hbm_budget=budget)
    t0 = time.perf_counter()
    out = srv.run(batch)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kept = [r for r in out if r.request.arrival >= discard_before]
    lat = [r.latency for r in kept]
    t_first = min(r.arrived for r in kept)
    t_last = max(r.finished for r in kept)
    st = {"requests": len(out), "measured": len(kept), "wall_s": wall,
          "solves_per_s": len(kept) / max(t_last - t_first, 1e-12),
          "p50_latency_s": percentile(lat, 50), "p99_latency_s": percentile(lat, 99),
          "mean_latency_s": float(np.mean(lat)),
          "mean_queue_s": float(np.mean([r.queued for r in kept])),
          "later_stage_iterations": int(sum(r.iterations for r in kept if r.request.stage > 0)),
          "converged": int(sum(r.converged for r in kept)),
          "peak_active": srv.peak_active, "evictions": srv.evictions}
    pm = {}
    for r in out:
        if r.request.stage == stages - 1 and r.request.truth is not None:
            pm.setdefault(r.request.stream.split("-")[0], []).append(
                partition_scores(r.request.truth, r.labels)["PM"])
    st["final_stage_PM"] = {z: round(float(np.mean(v)), 4) for z, v in pm.items()}
    return {kk: (round(v, 5) if isinstance(v, float) else v) for kk, v in st.items()}


def serve_warm_cold(S, stages, rate, stage_rate, slots, budget_gb, warm_fill):
    """The serving mix served warm, then cold: solves/s, p50/p99 latency and
    later-stage LOBPCG iterations of each pass."""
    import torch
    from paper_1708_07481_amd.serve import LibraryBackend, Server, make_streams
    specs, counts = serve_specs(S)
    log(f"serving: generating {S} streams x {stages} stages {counts}")
    t = time.perf_counter()
    reqs = make_streams(specs, rate=rate, seed=5, stages=stages, stage_rate=stage_rate)
    log(f"serving: {len(reqs)} requests ready in {time.perf_counter() - t:.1f} s")
    budget = int(budget_gb * (1 << 30))
    be = LibraryBackend(slots, precision="fp64", maxit=30, tol=1e-2, restarts=10,
                        warm_fill=warm_fill)
    small = min(reqs, key=lambda r: r.n)      # warm-up: one small solve loads the kernels
    Server(be, slots=1, hbm_budget=budget).run([_clone(small, arrival=0.0, stage=0, warm=False)])
    torch.cuda.synchronize()
    passes = {}
    for mode in ("warm", "cold"):
        passes[mode] = serve_pass(be, reqs, slots, budget, warm=(mode == "warm"), stages=stages)
        log(f"serving {mode}: {passes[mode]}")
    be.close()
    return passes, counts, len(reqs)


def serve_protocol(args):
    """Load sweep of the serving mix: the capacity (solves/s with every stream
    started at once, each stage held until its predecessor finishes), then
    Poisson arrivals at 0.5, 0.8 and 0.95 of it with at least 1,000 requests
    per load; the requests arriving in the first 10 % of each pass's arrival
    span are discarded as warm-up.  Written to profiles/serve_mix_loads.json."""
    import torch
    from paper_1708_07481_amd.serve import LibraryBackend, Server, make_streams
    budget = int(args.budget_gb * (1 << 30))
    stages = args.stages
    be = LibraryBackend(args.slots, precision="fp64", maxit=30, tol=1e-2, restarts=10,
                        warm_fill=args.warm_fill)
    specs, counts = serve_specs(20, seed=21)
    reqs = make_streams(specs, rate=1e6, seed=7, stages=stages, stage_rate=None)
    small = min(reqs, key=lambda r: r.n)
    Server(be, slots=1, hbm_budget=budget).run([_clone(small, arrival=0.0, stage=0, warm=False)])
    sat = serve_pass(be, reqs, args.slots, budget, stages=stages)
    cap = sat["solves_per_s"]
    log(f"capacity (20 streams started at once): {cap:.2f} solves/s; {sat}")
    S = max(100, -(-args.protocol_requests // stages))
    loads = {}
    for rho in (0.5, 0.8, 0.95):
        rate = rho * cap / stages                   # stream starts per second
        specs, counts = serve_specs(S, seed=int(100 * rho))
        t = time.perf_counter()
        reqs = make_streams(specs, rate=rate, seed=int(1000 * rho), stages=stages,
                            stage_rate=args.stage_rate)
        span = max(r.arrival for r in reqs)
        log(f"load {rho}: {len(reqs)} requests over {span:.0f} s of arrivals "
            f"(generated in {time.perf_counter() - t:.0f} s)")
        loads[str(rho)] = serve_pass(be, reqs, args.slots, budget, discard_before=0.1 * span,
                                     stages=stages)
        loads[str(rho)]["offered_solves_per_s"] = round(rho * cap, 3)
        log(f"load {rho}: {loads[str(rho)]}")
    be.close()
    rec = {"workload": (f"serving mix (60/30/10 % of streams 5K/19, 50K/44, 500K/98 DC-SBM; half "
                        f"emerging-edge, half snowball; {stages} stages), warm starts, "
                        f"{args.slots} slots, {args.budget_gb} GB admission budget, maxit 30, "
                        f"tol 1e-2, FP64 (5K, 50K) / FP32 + BF16 Gram (500K)"),
           "capacity_solves_per_s": round(cap, 3), "capacity_run": sat,
           "streams_per_load": S, "requests_per_load": S * stages,
           "warmup_discarded": "requests arriving in the first 10 % of the arrival span",
           "loads": loads,
           "command": f"python bench.py --config serve --protocol --slots {args.slots}"}
    with open(os.path.join(HERE, "profiles", "serve_mix_loads.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec), flush=True)


def run_serve(args):
    """Continuous-batching mix, served warm then cold; one JSON line."""
    if args.protocol:
        return serve_protocol(args)
    S = args.streams
    passes, (n5, n50, n500), nreq = serve_warm_cold(S, args.stages, args.rate, args.stage_rate,
                                                     args.slots, args.budget_gb, args.warm_fill)
    w, c = passes["warm"], passes["cold"]
    out = {
        "metric": "LOBPCG time-to-partition at rel-residual 1e-2; SpMM HBM GB/s; p99 solve latency",
        "value": w["p99_latency_s"], "unit": "s", "n_gpus": 1, "steps": nreq, "warmup": 1,
        "ms_per_step": round(1000.0 / max(w["solves_per_s"], 1e-12), 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (5K, 50K) / f32+bf16gram (500K)", "data": "synthetic",
        "config": {"workload": (f"serving mix: {S} streams ({n5} x 5K/19, {n50} x 50K/44, "
                                f"{n500} x 500K/98 degree-corrected SBM), half emerging-edge, "
                                f"half snowball, {args.stages} stages each; stream starts Poisson "
                                f"{args.rate}/s, stage arrivals Poisson {args.stage_rate}/s held "
                                f"until the previous stage finishes; {args.slots} slots, "
                                f"{args.budget_gb} GB admission budget; maxit 30, tol 1e-2"),
                   "name": "serve"},
        "serving": {"warm": w, "cold": c, "warm_fill": args.warm_fill,
                    "iterations_saved": c["later_stage_iterations"] - w["later_stage_iterations"]},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def spmm_variants(args, cfg, g0):
    """Time the FP32 product Y = L X (k = the workload's block width) in the
    layouts that change its memory traffic: natural row order; rows longest
    first (bit-identical); both with 16-byte instead of 4-byte lane reads of
    the neighbour rows (bit-identical); 16-bit gather copies of X (FP16, BF16: accuracy
    against the FP32 product reported); the vertices renumbered by reverse
    Cuthill-McKee (SciPy on the host, its time included) and, as the best any
    community-finding order could do, by the generator's blocks.  Each variant:
    2 untimed then 10 timed launches on the library's stream (HIP events).
    Dispatch order: natural, longest first, their 16-byte-lane twins, FP16,
    BF16, RCM, blocks."""
    import numpy as np
    import torch
    from paper_1708_07481_amd import api
    n, k = g0.n, cfg["k"]
    dev = torch.device("cuda:0")
    ctx = api.Context(0)
    out = {"workload": f"n={n} nnz~{2 * g0.m} k={k} FP32", "launches_timed": 10}

    def timed(fn, reps=10):
        for _ in range(2):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def build(src, dst):
        g = api.graph_build(ctx, n, torch.from_numpy(src).to(dev), torch.from_numpy(dst).to(dev))
        _, v32, _ = api.laplacian_csr(ctx, g, False, True)
        return g, v32

    g, v32 = build(g0.src, g0.dst)
    X = api.randn(ctx, n, k, 1, 2, "normal", torch.float32)
    Y0 = torch.empty_like(X)
    Y = torch.empty_like(X)
    nb = spmm_algorithmic_bytes(n, g.nnz, k, 4)
    rate = lambda ms: round(nb / (ms * 1e-3) / 1e9, 1)
    ms = timed(lambda: api.spmm(ctx, g, v32, X, Y0))
    out["natural"] = {"ms": round(ms, 4), "algorithmic_GBs": rate(ms)}
    log(f"natural order: {ms:.3f} ms")
    t0 = time.perf_counter()
    order = api.row_order(ctx, g)
    torch.cuda.synchronize()
    t_order = time.perf_counter() - t0
    ms = timed(lambda: api.spmm_ex(ctx, g, v32, X, Y, order=order))
    out["longest_rows_first"] = {"ms": round(ms, 4), "algorithmic_GBs": rate(ms),
                                 "order_ms": round(1e3 * t_order, 2),
                                 "bit_identical": bool(torch.equal(Y, Y0))}
    log(f"longest rows first: {ms:.3f} ms (order {1e3 * t_order:.1f} ms)")
    for name, o in (("natural_lane16", None), ("longest_rows_first_lane16", order)):
        ms = timed(lambda: api.spmm_ex(ctx, g, v32, X, Y, order=o, lane16=True))
        out[name] = {"ms": round(ms, 4), "algorithmic_GBs": rate(ms),
                     "bit_identical": bool(torch.equal(Y, Y0))}
        log(f"{name}: {ms:.3f} ms")
    ref = Y0.double()
    scale = float(ref.abs().max())
    for name, dt in (("fp16_gather", torch.float16), ("bf16_gather", torch.bfloat16)):
        Xg = X.to(dt)
        ms = timed(lambda: api.spmm_ex(ctx, g, v32, X, Y, Xg=Xg))
        err = float((Y.double() - ref).abs().max()) / scale
        out[name] = {"ms": round(ms, 4), "algorithmic_GBs": rate(ms),
                     "max_abs_err_rel_to_max": err}
        log(f"{name}: {ms:.3f} ms, max error / max |y| {err:.2e}")
        del Xg
    # renumberings: new id of vertex v is inv[v]
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    t0 = time.perf_counter()
    A = sp.csr_matrix((np.ones(g0.m, np.int8), (g0.src, g0.dst)), shape=(n, n))
    A = (A + A.T).tocsr()
    perm_rcm = reverse_cuthill_mckee(A, symmetric_mode=True)
    t_rcm = time.perf_counter() - t0
    del A
    perms = {"rcm": (perm_rcm, t_rcm), "generator_blocks": (np.argsort(g0.truth, kind="stable"), 0.0)}
    for name, (perm, t_host) in perms.items():
        inv = np.empty(n, np.int32)
        inv[perm] = np.arange(n, dtype=np.int32)
        gp, vp = build(inv[g0.src], inv[g0.dst])
        Xp = X[torch.from_numpy(perm.astype(np.int64)).to(dev)].contiguous()
        Yp = torch.empty_like(Xp)
        ms = timed(lambda: api.spmm(ctx, gp, vp, Xp, Yp))
        out[name] = {"ms": round(ms, 4), "algorithmic_GBs": rate(ms),
                     "host_order_s": round(t_host, 2)}
        log(f"{name}: {ms:.3f} ms (host order {t_host:.1f} s)")
        del gp, vp, Xp, Yp
    # reference kernel for the byte counters: a plain 512 MiB device copy, 3 times
    x = torch.ones(128 << 20, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    out["copy_calibration_bytes"] = {"read": x.numel() * 4, "write": y.numel() * 4}
    ctx.close()
    return out


def compare_fp64(args, api, ctx, cfg, n, k, src, dst, draws, res, km, t_mixed, truth):
    """The same graph and start block (the same Philox stream, in FP64) in
    FP64: timing and the differences."""
    import numpy as np
    import torch
    from paper_1708_07481_amd.metrics import partition_scores
    X0 = torch.empty((n, k), dtype=torch.float64, device=src.device)

    def step():
        gd = api.graph_build(ctx, n, src, dst)
        v64, _, _ = api.laplacian_csr(ctx, gd, True, False)
        api.randn(ctx, n, k, X0_SEED, X0_STREAM, "normal", torch.float64, out=X0)
        r = api.lobpcg_solve(ctx, gd, v64, X0, cfg["maxit"], cfg["tol"], "fp64")
        kk = api.kmeans_assign(ctx, r.X, k, draws, max_iter=100)
        return r, kk

    log("fp64 comparison run ...")
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r64, k64 = step()
    torch.cuda.synchronize()
    t64 = (time.perf_counter() - t0) / args.steps
    th64 = r64.theta.cpu().numpy()
    th = res.theta.cpu().numpy()
    Xr = res.X.double()
    Xo = r64.X
    A = Xr - Xo @ (Xo.T @ Xr)
    sine = float(torch.linalg.eigvalsh(A.T @ A).max().clamp(min=0).sqrt())
    s64 = partition_scores(truth, k64.labels.cpu().numpy())
    sm = partition_scores(truth, km.labels.cpu().numpy())
    return {"fp64_s": round(t64, 4), "mixed_s": round(t_mixed, 4),
            "speedup": round(t64 / t_mixed, 3),
            "fp64_iterations": r64.iterations, "mixed_iterations": res.iterations,
            "theta_max_abs_err": float(np.max(np.abs(th - th64))),
            "theta_max_rel_err": float(np.max(np.abs(th - th64) / np.maximum(np.abs(th64), 1e-12))),
            "subspace_sine": sine,
            "PM_fp64": round(s64["PM"], 5), "PM_mixed": round(sm["PM"], 5),
            "labels_agree_fraction": float(partition_scores(k64.labels.cpu().numpy(),
                                                            km.labels.cpu().numpy())["PM"])}


def _clone(r, **kw):
    import dataclasses
    return dataclasses.replace(r, **kw)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="sbm2m")
    ap.add_argument("--restarts", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--streams", type=int, default=10, help="serve: number of streams")
    ap.add_argument("--rate", type=float, default=2.0, help="serve: stream starts per second")
    ap.add_argument("--stage-rate", type=float, default=10.0, help="serve: stage arrivals per second")
    ap.add_argument("--stages", type=int, default=10)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--warm-fill", default="neighbors", choices=["neighbors", "zero"],
                    help="serve: start rows of the vertices a snowball stage adds")
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the short serving pass after the timed steps")
    ap.add_argument("--protocol", action="store_true",
                    help="serve: load sweep (capacity, then 0.5 / 0.8 / 0.95 of it, >= 1,000 "
                         "requests per load) written to profiles/serve_mix_loads.json")
    ap.add_argument("--protocol-requests", type=int, default=1000)
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32", "fp32_bf16gram"],
                    help="override the workload's precision")
    ap.add_argument("--cluster", default="kmeans", choices=["kmeans", "cpqr"],
                    help="labelling: k-means++ with restarts (default) or QR with column pivoting")
    ap.add_argument("--eigengap", action="store_true",
                    help="cluster count from the gap in the Ritz values (use with --extra-cols), "
                         "labels on that many leading columns")
    ap.add_argument("--extra-cols", type=int, default=0,
                    help="LOBPCG block of k + E columns, stopping test and labels on the first k")
    ap.add_argument("--lock-tol", type=float, default=0.0,
                    help="soft locking: W columns with relres at or below this leave the basis")
    ap.add_argument("--tol", type=float, default=None, help="override the workload's tolerance")
    ap.add_argument("--maxit", type=int, default=None, help="override the workload's iteration cap")
    ap.add_argument("--laplacian", default="normalized", choices=["normalized", "combinatorial"],
                    help="operator: I - D^-1/2 W D^-1/2 (default) or D - W (relres scaled by "
                         "2 max degree)")
    ap.add_argument("--compare", action="store_true",
                    help="also solve the same graph from the same start block in FP64 and report "
                         "speedup, eigenvalue error, subspace sine and accuracy of both")
    ap.add_argument("--spmm-variants", action="store_true",
                    help="time the SpMM in the layouts that change its traffic (row order, "
                         "16-bit gathers, RCM and block renumbering) on the workload's graph")
    ap.add_argument("--record-cpu-baseline", action="store_true",
                    help="time the oracle once on the full graph (several minutes, host only) "
                         "and write profiles/cpu_baseline_<config>.json")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, run a plain 512 MiB device copy three times "
                         "(reference kernel for the HBM byte counters)")
    args = ap.parse_args()
    if args.compare and (args.laplacian == "combinatorial" or args.extra_cols or args.lock_tol):
        ap.error("--compare runs the default operator, block width and locking only")
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build runs a single solve per GPU and has "
              "no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.config == "serve":
        return run_serve(args)

    import numpy as np
    import torch
    from paper_1708_07481_amd import api
    from paper_1708_07481_amd.metrics import partition_scores
    from synth import kmeans_draws
    from synth.configs import config, graph_for

    cfg = config(args.config)
    if args.tol is not None:
        cfg["tol"] = args.tol
    if args.maxit is not None:
        cfg["maxit"] = args.maxit
    restarts = args.restarts if args.restarts is not None else cfg["restarts"]
    prec = args.precision or cfg["precision"]
    fp64 = prec == "fp64"
    n, k = cfg["n"], cfg["k"]
    log(f"generating {args.config}: n={n} blocks={cfg['blocks']} k={k} precision={prec}")
    t = time.perf_counter()
    g0 = graph_for(args.config, seed=1)
    log(f"graph: m={g0.m} in {time.perf_counter() - t:.1f} s")
    if args.spmm_variants:
        rec = spmm_variants(args, cfg, g0)
        print(json.dumps(rec), flush=True)
        return
    if args.record_cpu_baseline:
        rec = record_cpu_baseline(args, cfg, g0)
        print(json.dumps(rec), flush=True)
        return
    kb = k + args.extra_cols
    draws_h = kmeans_draws(restarts, k, 1)

    dev = torch.device("cuda:0")
    src = torch.from_numpy(g0.src).to(dev)
    dst = torch.from_numpy(g0.dst).to(dev)
    X0 = torch.empty((n, kb), dtype=torch.float64 if fp64 else torch.float32, device=dev)
    draws = torch.from_numpy(draws_h.view(np.int64)).to(dev)
    ctx = api.Context(0)

    comb = args.laplacian == "combinatorial"

    def step():
        gd = api.graph_build(ctx, n, src, dst)
        diag = None
        if comb:
            v64, v32, d32 = api.laplacian_combinatorial(ctx, gd, fp64, not fp64)
            diag = gd.degree if fp64 else d32
        else:
            v64, v32, _ = api.laplacian_csr(ctx, gd, fp64, not fp64)
        val = v64 if fp64 else v32
        # Gaussian start block from the device Philox stream (Section III)
        api.randn(ctx, n, kb, X0_SEED, X0_STREAM, "normal", X0.dtype, out=X0)
        res = api.lobpcg_solve(ctx, gd, val, X0, cfg["maxit"], cfg["tol"], prec, diag=diag,
                               lock_tol=args.lock_tol, k_conv=k if kb > k else 0)
        kc = k
        if args.eigengap:
            kc, _ = api.eigengap(ctx, res.theta)
        Xk = res.X[:, :kc]
        if args.cluster == "cpqr":
            cq = api.cpqr_labels(ctx, Xk)
            km = SimpleNamespace(labels=cq.labels, lloyd_iterations=None, clusters=kc)
        else:
            km = api.kmeans_assign(ctx, Xk, kc, draws[:, :kc].contiguous(), max_iter=100)
            km.clusters = kc
        return gd, res, km

    for w in range(args.warmup):
        gd, res, km = step()
        log(f"warmup {w}: iterations={res.iterations} converged={res.converged} "
            f"relres={res.max_relres:.3e}")
    torch.cuda.synchronize()
    ctx.set_profiling(["spmm", "gram", "rayleigh_ritz", "block_update", "cholqr", "residual",
                       "graph_build", "kmeans", "gram_fp64acc"])
    ctx.profile_reset()
    times = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        gd, res, km = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        log(f"step {s}: {times[-1]:.3f} s iterations={res.iterations} "
            f"relres={res.max_relres:.3e}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    prof = ctx.profile()
    ctx.set_profiling([])

    labels = km.labels.cpu().numpy()
    scores = partition_scores(g0.truth, labels)
    ms_per_step = 1000.0 * total / args.steps
    es = 8 if fp64 else 4
    spmm = prof.get("spmm", {"avg_ms": float("nan"), "launches": 0})
    alg_bytes = spmm_algorithmic_bytes(n, gd.nnz, k, es, comb)
    achieved = alg_bytes / (spmm["avg_ms"] * 1e-3) / 1e9
    lob_ms = sum(prof.get(x, {}).get("total_ms", 0.0) for x in
                 ("spmm", "gram", "rayleigh_ritz", "block_update", "cholqr", "residual",
                  "gram_fp64acc"))
    iters_total = res.iterations * args.steps
    out = {
        "metric": "LOBPCG time-to-partition at rel-residual 1e-2; SpMM HBM GB/s; p99 solve latency",
        "value": round(total / args.steps, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else ("f32+bf16gram" if prec == "fp32_bf16gram" else "f32"),
        "data": "synthetic",
        "config": {"workload": (f"degree-corrected SBM n={n} m={g0.m} blocks={cfg['blocks']} "
                                f"mean_degree={cfg['mean_degree']} intra={cfg['intra']} "
                                f"sizes={cfg['sizes']}({cfg['alpha']}); LOBPCG k={k} "
                                f"maxit={cfg['maxit']} tol={cfg['tol']} {prec}"
                                f"{f' block {kb}' if kb > k else ''}"
                                f"{f' lock_tol={args.lock_tol}' if args.lock_tol > 0 else ''}"
                                f"{'; Laplacian D - W' if comb else ''}; "
                                + ("labels by QR with column pivoting" if args.cluster == "cpqr"
                                   else f"k-means restarts={restarts}")),
                   "name": args.config, "n": n, "nnz": gd.nnz, "k": k},
        "lobpcg_iterations": res.iterations,
        "converged_cols_per_iteration": ([] if res.relres_hist is None else
                                         [int((row[:k] <= cfg["tol"]).sum())
                                          for row in res.relres_hist]),
        "clusters": getattr(km, "clusters", k),
        "kmeans_lloyd_iterations": km.lloyd_iterations,
        "converged": res.converged,
        "max_relres": res.max_relres,
        "solver_events": {"p_drops": res.p_drops, "w_drops": res.w_drops,
                          "gram_fallbacks": res.gram_fallbacks, "restarts": res.restarts,
                          "locked_cols": res.locked_cols},
        "iterations_per_s": round(iters_total / (lob_ms * 1e-3), 3) if lob_ms > 0 else None,
        "spmm_hbm_gbs_algorithmic": round(achieved, 1),
        "phase_ms_per_step": {kk: round(v["total_ms"] / args.steps, 3) for kk, v in prof.items()},
        "kernel_avg_ms": {kk: round(v["avg_ms"], 4) for kk, v in prof.items()},
        "accuracy_vs_truth": {kk: round(v, 5) for kk, v in scores.items()},
    }
    spmm_line = {"kernel": "spmm (L W, the product of the metric)", "bound": "hbm",
                 "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(achieved / HBM_PEAK_GBS, 4), "avg_ms": round(spmm["avg_ms"], 4),
                 "algorithmic_bytes_per_launch": alg_bytes,
                 "traffic": spmm_traffic(args.config, alg_bytes)}
    # the achievable HBM rate on this machine beside the published peak (after the
    # timed steps)
    copy_gbs = copy_rate_gbs(torch, dev)
    spmm_line["copy_GBs"] = round(copy_gbs, 1)
    spmm_line["frac_of_copy"] = round(achieved / copy_gbs, 4)
    # The dominant kernel: the Gram products of the Rayleigh-Ritz step, S'LS and
    # S'S in one launch (split over row chunks, then an ordered reduction), one
    # launch per Rayleigh-Ritz step; its algorithmic work is the two
    # symmetric K3 x K3 outputs over n rows.
    gram = prof.get("gram")
    if gram:
        K3 = 3 * ((kb + 3) // 4 * 4)
        gflop = 2.0 * n * K3 * (K3 + 1) / 1e9
        peak = 78.6 if fp64 else (2500.0 if prec == "fp32_bf16gram" else 157.3)
        tflops = gflop / gram["avg_ms"]
        counters = gram_counters(args.config) if (prec == "fp32" and kb == 160) else None
        out["roofline"] = {"bound": "mfma", "kernel": "gram (S'LS and S'S)",
                           "achieved": round(tflops, 2), "peak": peak, "unit": "TFLOP/s",
                           "frac": round(tflops / peak, 4), "avg_ms": round(gram["avg_ms"], 4),
                           "launches": gram["launches"],
                           "algorithmic_gflop_per_launch": round(gflop, 1),
                           "traffic": counters["traffic"] if counters else None,
                           "counters": counters}
        out["rooflines_other"] = [spmm_line]
    else:
        out["roofline"] = dict(spmm_line, kernel="spmm")
    if args.compare and not fp64:
        out["precision_comparison"] = compare_fp64(args, api, ctx, cfg, n, k, src, dst, draws,
                                                   res, km, total / args.steps, g0.truth)
    if args.calibrate_copy:
        x = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": x.numel() * 4, "write": y.numel() * 4}
    out["hip_runtime"] = api.runtime_info()
    ctx.close()
    if not args.no_serve:
        # the serving mix after the timed steps (not part of `value`)
        passes, counts, nreq = serve_warm_cold(args.streams, args.stages, args.rate,
                                               args.stage_rate, args.slots, args.budget_gb,
                                               args.warm_fill)
        w, c = passes["warm"], passes["cold"]
        out["serving"] = {
            "workload": (f"{args.streams} streams ({counts[0]} x 5K/19, {counts[1]} x 50K/44, "
                         f"{counts[2]} x 500K/98 DC-SBM), half emerging-edge, half snowball, "
                         f"{args.stages} stages, Poisson stream starts {args.rate}/s and stage "
                         f"arrivals {args.stage_rate}/s, {args.slots} slots"),
            "requests": nreq, "p50_s": w["p50_latency_s"], "p99_s": w["p99_latency_s"],
            "solves_per_s": w["solves_per_s"],
            "iterations_saved": c["later_stage_iterations"] - w["later_stage_iterations"],
            "cold": {"p50_s": c["p50_latency_s"], "p99_s": c["p99_latency_s"],
                     "solves_per_s": c["solves_per_s"]},
            "warm_later_stage_iterations": w["later_stage_iterations"],
            "cold_later_stage_iterations": c["later_stage_iterations"],
            "final_stage_PM": w["final_stage_PM"]}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        try:
            out["cpu_baseline"] = cpu_baseline(g0, cfg, args.config, res.iterations, restarts,
                                               km.lloyd_iterations or 0, combinatorial=comb)
        except Exception as e:  # the GPU result stands on its own
            out["cpu_baseline"] = {"value": None, "error": str(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
