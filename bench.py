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
    Timed live on the full graph (a bounded sample, about 10 s of CPU work):
    graph build + Laplacian, and one SpMM with the k-column block.  The
    phases too long to repeat in every run come from the full-size record
    profiles/cpu_baseline_<workload>.json (measured once on a GPU machine's host
    by record_cpu_baseline): LOBPCG start-up and per-iteration time, k-means
    normalisation, per-restart seeding and per-Lloyd-update time.  One
    partition = graph + start-up + the GPU solve's iterations x iteration +
    normalisation + restarts x seeding + restarts x the GPU's Lloyd updates
    (of its slowest restart, so an upper estimate) x update."""
    import oracle
    from synth import gaussian_block
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    g = oracle.graph_build(g0.n, g0.src, g0.dst)
    val, diag = oracle.laplacian_combinatorial(g) if combinatorial else (oracle.laplacian(g)[0], None)
    t_graph = time.perf_counter() - t0
    X0 = gaussian_block(g0.n, cfg["k"], 1)
    t0 = time.perf_counter()
    oracle.spmm(g, val, X0, diag)
    t_spmm = time.perf_counter() - t0
    del g, val, X0
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
             + sec["kmeans_normalise"] + restarts * sec["kmeans_seeding_per_restart"]
             + restarts * lloyd_iters * sec["kmeans_lloyd_update"])
    return {"value": round(value, 1), "unit": "s", "cores": threads, "kind": "oracle",
            "host": host_info(),
            "sample": (f"oracle on the full graph (n={g0.n}, k={cfg['k']}). Live in this run: "
                       f"graph build + Laplacian {t_graph:.1f} s, one SpMM {t_spmm:.1f} s (the "
                       f"record's: {sec['spmm']:.1f} s). From the full-size record "
                       f"profiles/cpu_baseline_{name}.json ({rec['threads']} threads on "
                       f"{rec['host'].get('Model name', '?')}): LOBPCG start-up "
                       f"{sec['lobpcg_setup']:.1f} s + {gpu_iters} iterations x "
                       f"{sec['lobpcg_iteration']:.1f} s; k-means normalisation "
                       f"{sec['kmeans_normalise']:.1f} s + {restarts} restarts x seeding "
                       f"{sec['kmeans_seeding_per_restart']:.1f} s + {restarts} x {lloyd_iters} "
                       f"Lloyd updates x {sec['kmeans_lloyd_update']:.1f} s (the GPU's count for "
                       f"its slowest restart: an upper estimate)")}


def run_serve(args):
    """Continuous-batching mix, served warm then cold; one JSON line."""
    import numpy as np
    import torch
    from paper_1708_07481_amd.metrics import partition_scores
    from paper_1708_07481_amd.serve import LibraryBackend, Server, make_streams

    S = args.streams
    n5 = round(0.6 * S)
    n50 = round(0.3 * S)
    sizes = ["sbm5k"] * n5 + ["sbm50k"] * n50 + ["sbm500k"] * (S - n5 - n50)
    order = np.random.default_rng(11).permutation(S)
    specs = [(f"{sizes[i]}-{j}", sizes[i], "emerging" if j % 2 == 0 else "snowball")
             for j, i in enumerate(order)]
    log(f"generating {S} streams x {args.stages} stages: {dict((z, sizes.count(z)) for z in set(sizes))}")
    t = time.perf_counter()
    reqs = make_streams(specs, rate=args.rate, seed=5, stages=args.stages,
                        stage_rate=args.stage_rate)
    log(f"streams ready in {time.perf_counter() - t:.1f} s; {len(reqs)} requests")
    budget = int(args.budget_gb * (1 << 30))

    # warm-up: one small solve loads every kernel
    be = LibraryBackend(args.slots, precision="fp64", maxit=30, tol=1e-2, restarts=10,
                        warm_fill=args.warm_fill)
    small = min(reqs, key=lambda r: r.n)
    Server(be, slots=1, hbm_budget=budget).run([_clone(small, arrival=0.0, stage=0, warm=False)])
    torch.cuda.synchronize()

    passes = {}
    for mode in ("warm", "cold"):
        batch = [_clone(r, warm=(mode == "warm")) for r in reqs]
        srv = Server(be, slots=args.slots, hbm_budget=budget)
        t0 = time.perf_counter()
        out = srv.run(batch)
        torch.cuda.synchronize()
        st = srv.stats()
        st["wall_s"] = time.perf_counter() - t0
        later = [r for r in out if r.request.stage > 0]
        st["later_stage_iterations"] = int(sum(r.iterations for r in later))
        st["converged"] = int(sum(r.converged for r in out))
        pm = {}
        for r in out:
            if r.request.stage == args.stages - 1:
                cfg_name = r.request.stream.split("-")[0]
                pm.setdefault(cfg_name, []).append(
                    partition_scores(r.request.truth, r.labels)["PM"])
        st["final_stage_PM"] = {z: round(float(np.mean(v)), 4) for z, v in pm.items()}
        passes[mode] = {kk: (round(v, 5) if isinstance(v, float) else v) for kk, v in st.items()}
        log(f"{mode}: {passes[mode]}")
    be.close()
    w, c = passes["warm"], passes["cold"]
    out = {
        "metric": "LOBPCG time-to-partition at rel-residual 1e-2; SpMM HBM GB/s; p99 solve latency",
        "value": w["p99_latency_s"], "unit": "s", "n_gpus": 1, "steps": len(reqs), "warmup": 1,
        "ms_per_step": round(1000.0 * w["makespan_s"] / max(len(reqs), 1), 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (5K, 50K) / f32+bf16gram (500K)", "data": "synthetic",
        "config": {"workload": (f"serving mix: {S} streams ({n5} x 5K/19, {n50} x 50K/44, "
                                f"{S - n5 - n50} x 500K/98 degree-corrected SBM), half emerging-edge, "
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
                       "graph_build", "kmeans"])
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
                 ("spmm", "gram", "rayleigh_ritz", "block_update", "cholqr", "residual"))
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
        "clusters": getattr(km, "clusters", k),
        "kmeans_lloyd_iterations": km.lloyd_iterations,
        "converged": res.converged,
        "max_relres": res.max_relres,
        "solver_events": {"p_drops": res.p_drops, "w_drops": res.w_drops,
                          "gram_fallbacks": res.gram_fallbacks, "restarts": res.restarts},
        "iterations_per_s": round(iters_total / (lob_ms * 1e-3), 3) if lob_ms > 0 else None,
        "spmm_hbm_gbs_algorithmic": round(achieved, 1),
        "phase_ms_per_step": {kk: round(v["total_ms"] / args.steps, 3) for kk, v in prof.items()},
        "kernel_avg_ms": {kk: round(v["avg_ms"], 4) for kk, v in prof.items()},
        "accuracy_vs_truth": {kk: round(v, 5) for kk, v in scores.items()},
        "roofline": {"bound": "hbm", "kernel": "spmm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "traffic": spmm_traffic(args.config, alg_bytes)},
    }
    # Gram products of the Rayleigh-Ritz step (S'LS and S'S, one pair per RR)
    gram = prof.get("gram")
    if gram:
        n_rr = (res.iterations + 1 + res.restarts) * args.steps
        gram_ms = gram["total_ms"] / n_rr
        K3 = 3 * ((k + 3) // 4 * 4)
        gflop = 2.0 * n * K3 * (K3 + 1) / 1e9      # two symmetric K3 x K3 outputs
        peak = 78.6 if fp64 else (2500.0 if prec == "fp32_bf16gram" else 157.3)
        out["rooflines_other"] = [{
            "kernel": "gram (S'LS and S'S)", "bound": "mfma", "unit": "TFLOP/s",
            "achieved": round(gflop / gram_ms, 2), "peak": peak,
            "frac": round(gflop / gram_ms / peak, 4), "ms_per_rr": round(gram_ms, 3),
            "algorithmic_gflop": round(gflop, 1),
            "counters": gram_counters(args.config) if (prec == "fp32" and k == 160) else None}]
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
