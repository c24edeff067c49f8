"""Benchmark of the SCSF hot path on one MI355X.

One step = the whole path over one synthetic dataset: truncated-FFT sort of the coefficient
fields (Algorithm 2) and the warm-started Chebyshev filtered subspace iteration over every
operator in sorted order (Algorithm 3), split into `--chains` contiguous chunks that run
concurrently (the chunk parallelism of App. D.6).  Inputs are resident in HBM before timing;
the step ends with all eigenpairs resident in HBM.

Workload (default): 200 generalized-Poisson operators -div(K grad u) on a 100 x 100 grid
(n = 10^4), K = exp(GRF with 16 x 16 cosine modes), L = 100 smallest eigenpairs, block width
k = 120, Chebyshev degree 30 (the configuration's range is 16-30), p0 = 20, relative residual
1e-8, FP64.  `--config` selects the other workloads (1 small, 3 uneven batch, 4 mixed
precision, 5 learned window, 6 thin-plate vibration).

Prints one JSON line (rank 0).  `roofline` describes the dominant kernel (the filter's
Chebyshev step), timed live with HIP events around each filter launch (or filter graph) inside
the timed region; `cpu_baseline` times the CPU oracle (NumPy/SciPy) on a bounded prefix of the
same sorted sequence.  After the timed steps, for the working-size workload: `comparison`
(the same operators solved cold and unsorted) and `spmm_isolated` (the filter step alone).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(cfg_index: int, count: int | None):
    import scsf_inputs as si
    cfg = si.CONFIGS[cfg_index]
    t = time.time()
    ops = si.operators(cfg, count)
    log(f"[bench] generated {len(ops)} operators of {cfg.name} in {time.time() - t:.1f}s")
    return cfg, ops


def measured_traffic(cfg_name: str, launch: dict):
    """HBM bytes per filter launch from the committed counter record of this workload, while
    the filter step's source and the launch configuration (chains, lanes, schedule, graphs)
    are those the counters were taken with (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"spmm_traffic_{cfg_name}.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            key, _, val = line.partition(" ")
            rec[key] = val.strip()
    src = os.path.join(ROOT, rec.get("source", ""))
    if not os.path.isfile(src):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if digest != rec.get("source_sha256_16"):
        return None
    if any(str(v) != rec.get(key) for key, v in launch.items()):
        return None
    return float(rec["bytes_per_launch"])


def isolated_spmm(scsf, torch, h, dops, k, degree, blocks):
    """The filter step alone: `blocks` operators of the workload, k columns each, `degree`
    Chebyshev steps through scsf_filter_batched (one launch per step over all blocks, the
    solver's kernel and tile), each launch timed with HIP events on the stream it runs on.
    Window: lambda = 0 below the spectrum, [0.1 ub, ub] damped, ub the Gershgorin bound."""
    ops = [dops[i % len(dops)] for i in range(blocks)]
    ld = max(d.n for d in ops)
    gen = torch.Generator(device="cuda").manual_seed(11)
    X = torch.randn((blocks, k, ld), device="cuda", dtype=torch.float64, generator=gen)
    wins = []
    for d in ops:
        ub = scsf.scsf_bounds(h, d)["gershgorin"]
        wins.append((0.0, 0.55 * ub, 0.45 * ub))
    Y = scsf.scsf_filter_batched(h, ops, X, degree, wins)          # untimed first pass
    torch.cuda.synchronize()
    scsf.scsf_profile_read(h, reset=True)
    scsf.scsf_profile_enable(h, True)
    scsf.scsf_filter_batched(h, ops, X, degree, wins, Y)
    torch.cuda.synchronize()
    prof = scsf.scsf_profile_read(h, reset=True)
    scsf.scsf_profile_enable(h, False)
    del X, Y
    ms = prof["filter_ms"] / max(prof["filter_launches"], 1)
    bytes_ = prof["filter_bytes"] / max(prof["filter_launches"], 1)
    gbs = bytes_ / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    kern = "spmm_plate_kernel" if ops[0].struct.kind == scsf.SCSF_PLATE else "spmm_lds_kernel"
    return {"kernel": f"{kern}, alone (scsf_filter_batched)", "blocks": blocks,
            "columns": k, "launches": prof["filter_launches"], "avg_launch_ms": ms,
            "algorithmic_bytes_per_launch": bytes_, "achieved": gbs, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}


FP64_MFMA_PEAK_TFS = 78.6


def isolated_gram(scsf, torch, h, n, k, blocks):
    """The Gram product of CholeskyQR2 alone: `blocks` random n x k blocks through
    scsf_gram_batched (the solvers' f64 MFMA kernel and reduction), timed with HIP events;
    algorithmic flops n k (k + 1) per block (the unique entries of a symmetric product)."""
    gen = torch.Generator(device="cuda").manual_seed(12)
    X = torch.randn((blocks, k, n), device="cuda", dtype=torch.float64, generator=gen)
    scsf.scsf_gram_batched(h, X)                                   # untimed first pass
    _, ms = scsf.scsf_gram_batched(h, X, timed=True)
    del X
    flops = blocks * n * k * (k + 1)
    tfs = flops / (ms * 1e-3) / 1e12
    return {"kernel": "gemm_tn_kernel + gemm_tn_reduce_kernel (Gram, f64 MFMA 16x16x4)",
            "blocks": blocks, "n": n, "k": k, "ms": ms, "flops": flops, "achieved": tfs,
            "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s", "frac": tfs / FP64_MFMA_PEAK_TFS}


def family_order_host(ops, p0):
    """Algorithm 2 within each operator family, concatenated (oracle; CPU baseline only)."""
    from oracle import sort as S
    order = []
    for fam in ("divk", "potential", "aniso"):
        idx = [i for i, o in enumerate(ops) if o.family == fam]
        if idx:
            sub = S.scsf_sort([ops[i].field for i in idx], p0)
            order += [idx[j] for j in sub]
    return order


def cpu_baseline(cfg, ops, budget_s: float, Ls=None, ks=None, degree=None, adaptive=False):
    """The oracle (plain NumPy/SciPy SCSF) on a bounded prefix of the sorted sequence, with the
    filter degree (and per-vector degrees) of the timed run."""
    import math
    import numpy as np
    from oracle import operator as O, sort as S, chfsi as C, transfer as T
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    degree = degree or cfg.degree
    t0 = time.time()
    if Ls is None:
        order = S.scsf_sort([o.field for o in ops], cfg.p0)
        Ls, ks = [cfg.L] * len(ops), [cfg.k] * len(ops)
    else:
        order = family_order_host(ops, cfg.p0)
    prev, prev_key, done, pairs = None, None, 0, 0
    for i in order:
        A = O.assemble(ops[i])
        key = (ops[i].family, Ls[i], ks[i])
        if prev is None or key != prev_key:
            r = C.chfsi(A, Ls[i], ks[i], degree, cfg.tol, seed=1, adaptive=adaptive)
        else:
            X0 = prev.X_next
            if X0.shape[0] != A.shape[0]:
                X0 = T.interpolate_block(X0, math.isqrt(X0.shape[0]), ops[i].N)
            r = C.chfsi(A, Ls[i], ks[i], degree, cfg.tol, X0=X0, theta0=prev.theta_next,
                        adaptive=adaptive)
        prev, prev_key = r, key
        done += 1
        pairs += Ls[i]
        log(f"[bench] cpu oracle: operator {done} ({r.iterations} iterations) "
            f"{time.time() - t0:.1f}s")
        if time.time() - t0 > budget_s:
            break
    dt = time.time() - t0
    return {"value": pairs / dt, "unit": "eigenpairs/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"sort of all {len(ops)} fields + the first {done} operators of the sorted "
                      f"sequence (one warm-started chain, cold first solve), {dt:.1f}s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--count", type=int, default=None, help="operators (default: all)")
    ap.add_argument("--chains", type=int, default=128)
    ap.add_argument("--lanes", type=int, default=6)
    ap.add_argument("--degree", type=int, default=None)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="default: the configuration's (fp64; mixed for config 4)")
    ap.add_argument("--schedule", choices=["static", "dynamic"], default="dynamic",
                    help="static: contiguous chunks of the sorted order (App. D.6); dynamic: "
                         "each chain takes the next unsolved operator of the sorted order")
    ap.add_argument("--graphs", choices=["on", "off"], default="on",
                    help="replay each outer iteration as HIP graphs (on) or launch its kernels "
                         "one by one (off)")
    ap.add_argument("--eig", choices=["jacobi", "tridiag"], default="jacobi",
                    help="Rayleigh-Ritz eigensolver")
    ap.add_argument("--autotune", choices=["on", "off"], default="on",
                    help="tune filter tiles (and, for the uneven workload, block widths) on the "
                         "dataset once before the warmup; the timed steps use the result")
    ap.add_argument("--form", choices=["learned", "plain"], default=None,
                    help="learned-window workload only: learned (train on the first solves, "
                         "predict windows and degrees for the rest; default) or plain")
    ap.add_argument("--train", type=int, default=500,
                    help="learned form: operators solved plainly to train the network")
    ap.add_argument("--epochs", type=int, default=600)
    ap.add_argument("--tile", type=int, choices=[1, 2, 4], default=None,
                    help="pin the filter-step tile instead of the autotuned one")
    ap.add_argument("--adaptive", choices=["on", "off"], default="off",
                    help="per-vector filter degrees in [degree, min(2 degree, 64)] (FP64 "
                         "solves without degree hints)")
    ap.add_argument("--compare", choices=["on", "off"], default="on",
                    help="working-size workload: also time the same operators solved cold and "
                         "unsorted (outside the timed steps)")
    ap.add_argument("--spmm-isolated", choices=["on", "off"], default="on",
                    help="working-size workload: also time the filter step alone on 32 blocks "
                         "(after the timed steps)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="before timing, run a plain 1 GiB device-to-device copy kernel three "
                         "times (reference for the HBM byte counters)")
    args = ap.parse_args()
    # HIP maps every stream to one of GPU_MAX_HW_QUEUES hardware queues (4 by default); the
    # concurrent lanes of the chained solver plus the default stream need one queue each, or
    # two lanes share a queue and run one after the other.  Set before HIP initialises.
    os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(8, args.lanes + 2)))

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; multi-GPU chunking is not "
                                   "implemented (--gpus must be 1)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2510_23215_amd import scsf

    torch.cuda.set_device(0)
    cfg, ops = workload(args.config, args.count)
    degree = args.degree or cfg.degree
    n_op = len(ops)
    uneven = cfg.family == "mixed"
    windowed = cfg.family == "aniso"             # the learned-window workload
    form = (args.form or "learned") if windowed else "plain"
    import scsf_inputs as si
    Ls = [si.mixed_L(cfg, i) for i in range(n_op)] if uneven else [cfg.L] * n_op
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, args.lanes)
    scsf.scsf_set_graphs(h, args.graphs == "on")
    scsf.scsf_set_eigensolver(h, scsf.SCSF_EIG_TRIDIAG if args.eig == "tridiag"
                              else scsf.SCSF_EIG_JACOBI)
    dops = [scsf.DeviceOperator(o) for o in ops]
    if uneven:
        # fields grouped by family and side: features per side, one greedy order per family
        groups = {}
        for i, o in enumerate(ops):
            groups.setdefault((o.family, o.N), []).append(i)
        gfields = {key: torch.tensor(np.stack([ops[i].field for i in idx]), device="cuda")
                   for key, idx in groups.items()}
        fams = sorted({key[0] for key in groups})
    else:
        fields = torch.tensor(np.stack([o.field for o in ops]), device="cuda")
    precision = args.precision or ("mixed" if cfg.precision == "mixed" or form == "learned"
                                   else "fp64")
    adaptive = args.adaptive == "on"
    if adaptive and (precision != "fp64" or form == "learned"):
        print(json.dumps({"error": "--adaptive needs FP64 solves without degree hints "
                                   "(--precision fp64, and --form plain on the learned-window "
                                   "workload)"}))
        sys.exit(2)
    prm = scsf.make_params(cfg.L, cfg.k, degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_DYNAMIC if args.schedule == "dynamic"
                           else scsf.SCSF_SCHED_STATIC,
                           precision=scsf.SCSF_MIXED if precision == "mixed" else scsf.SCSF_FP64,
                           adaptive=int(adaptive))
    if not uneven:
        evals = torch.empty((n_op, cfg.L), device="cuda", dtype=torch.float64)
        evecs = torch.empty((n_op, cfg.L, dops[0].n), device="cuda", dtype=torch.float64)
    torch.cuda.synchronize()
    if args.calibrate_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy calibration: 3 x 1 GiB device copy done")

    prm64 = scsf.make_params(cfg.L, cfg.k, degree, cfg.tol, seed=1,
                             schedule=scsf.SCSF_SCHED_DYNAMIC if args.schedule == "dynamic"
                             else scsf.SCSF_SCHED_STATIC, precision=scsf.SCSF_FP64)

    def make_order():
        if uneven:
            order = []
            for fam in fams:
                keys = [key for key in groups if key[0] == fam]
                idx = [i for key in keys for i in groups[key]]
                feats = torch.cat([scsf.scsf_features(h, gfields[key], cfg.p0) for key in keys])
                order += [idx[j] for j in scsf.scsf_order_features(h, feats)]
            return order
        return scsf.scsf_sort(h, fields, cfg.p0)

    n_train = min(args.train, n_op // 2) if windowed else 0
    train_info = {}

    def step_learned():
        """Sort; plain solves of the first n_train operators of the order (their Ritz values
        and bounds give the labels); FP32 training; BF16 inference for the rest, whose solves
        take the predicted window and degree."""
        order = scsf.scsf_sort(h, fields, cfg.p0)
        head, tail = [int(i) for i in order[:n_train]], [int(i) for i in order[n_train:]]
        ritz = torch.empty((n_train, cfg.k), device="cuda", dtype=torch.float64)
        _, _, st1 = scsf.scsf_solve_sequence(h, [dops[i] for i in head], np.arange(n_train),
                                             args.chains, prm, ritz=ritz)
        beta = torch.tensor([s["beta"] for s in st1], device="cuda", dtype=torch.float64)
        target = scsf.scsf_window_labels(h, ritz, cfg.L, beta)
        x = scsf.scsf_window_input(h, scsf.scsf_features(h, fields, 16))
        params = scsf.scsf_window_init(h, 5)
        hist = scsf.scsf_window_train(h, params, x[torch.tensor(head, device="cuda")], target,
                                      args.epochs, 1e-3)
        out = scsf.scsf_window_forward(h, params, x[torch.tensor(tail, device="cuda")], bf16=True)
        hints = scsf.scsf_window_hints(h, out).cpu().numpy()
        _, _, st2 = scsf.scsf_solve_sequence(h, [dops[i] for i in tail], np.arange(len(tail)),
                                             args.chains, prm, hints=hints)
        train_info.update(loss_first=float(hist[0]), loss_last=float(hist[-1]),
                          hints_used=int(sum(s["hint"] == 2 for s in st2)),
                          mean_degree=float(np.mean([s["degree"] for s in st2])))
        return st1 + st2

    def step():
        if form == "learned":
            return step_learned()
        order = make_order()
        if uneven:
            _, _, stats = scsf.scsf_solve_batched(h, dops, Ls, order, args.chains, prm)
            return stats
        _, _, stats = scsf.scsf_solve_sequence(h, dops, order, args.chains, prm, evals, evecs)
        return stats

    tune_s = 0.0
    if args.autotune == "on":
        t = time.time()
        scsf.scsf_autotune(h, dops, Ls, make_order(), prm64, probe=4)
        tune_s = time.time() - t
        log(f"[bench] autotune {tune_s:.2f}s")
    if args.tile:
        scsf.scsf_set_tile(h, args.tile)
    ks = [scsf.scsf_tuned_width(h, L) for L in Ls] if uneven else [cfg.k] * n_op
    tile_used = scsf.scsf_tuned_tile(h, max(d.n for d in dops), max(ks))

    for w in range(args.warmup):
        t = time.time()
        stats = step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w}: {time.time() - t:.2f}s, iterations "
            f"mean {np.mean([s['iterations'] for s in stats]):.1f}")

    scsf.scsf_profile_read(h, reset=True)
    scsf.scsf_profile_enable(h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for s in range(args.steps):
        stats = step()
        iters += [st["iterations"] for st in stats]
        log(f"[bench] step {s} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = scsf.scsf_profile_read(h, reset=True)
    scsf.scsf_profile_enable(h, False)

    comparison = None
    if cfg.index == 2 and args.compare == "on":
        # the same operators in their generated order, every solve from a random block
        prm_cold = scsf.make_params(cfg.L, cfg.k, degree, cfg.tol, seed=1,
                                    schedule=scsf.SCSF_SCHED_DYNAMIC if args.schedule == "dynamic"
                                    else scsf.SCSF_SCHED_STATIC, cold_start=1)
        t = time.perf_counter()
        _, _, stc = scsf.scsf_solve_sequence(h, dops, np.arange(n_op), args.chains, prm_cold,
                                             evals, evecs)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t
        comparison = {"cold_unsorted_value": n_op * cfg.L / tc, "cold_unsorted_ms": tc * 1e3,
                      "cold_unsorted_mean_iterations":
                          float(np.mean([s["iterations"] for s in stc]))}
        log(f"[bench] cold unsorted comparison: {n_op * cfg.L / tc:.0f} eigenpairs/s")
    if windowed and form == "learned":
        # the plain FP64 method (window from Ritz values, degree 20) on the same operators
        t = time.perf_counter()
        order = scsf.scsf_sort(h, fields, cfg.p0)
        _, _, stp = scsf.scsf_solve_sequence(h, dops, order, args.chains, prm64)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        comparison = {"plain_fp64_value": n_op * cfg.L / tp, "plain_fp64_ms": tp * 1e3,
                      "plain_fp64_mean_iterations": float(np.mean([s["iterations"] for s in stp]))}
        log(f"[bench] plain fp64 comparison: {n_op * cfg.L / tp:.0f} eigenpairs/s")

    pairs = args.steps * sum(Ls)
    value = pairs / dt
    avg_ms = prof["filter_ms"] / max(prof["filter_launches"], 1)
    avg_bytes = prof["filter_bytes"] / max(prof["filter_launches"], 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0

    out = {
        "metric": "eigenpairs/sec at residual %g (SCSF GPU, %s%s)" % (
            cfg.tol, "learned window, " if form == "learned" else "",
            "FP64" if precision == "fp64" else "FP32 filter / FP64 rest"),
        "value": value,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32 filter + f64",
        "data": "synthetic (seeded GRF coefficient fields)",
        "config": {
            "workload": (f"{cfg.name}: {n_op} operators ({cfg.family}), {ops[0].N}x{ops[0].N} "
                         f"grid (n={dops[0].n}), L={cfg.L}, k={cfg.k}, degree={degree}"
                         f"{' (range 16-30)' if cfg.index == 2 else ''}, "
                         f"p0={cfg.p0}, tol={cfg.tol:g}") if not uneven else
                        (f"{cfg.name}: {n_op} operators (half -div(K grad u), half -Laplace u + "
                         f"V u), sides {min(o.N for o in ops)}..{max(o.N for o in ops)}, "
                         f"L in {{32, 64, 128}} (sum {sum(Ls)}), k autotuned per L, "
                         f"degree={degree}, p0={cfg.p0}, tol={cfg.tol:g}"),
            "chains": args.chains,
            "lanes": args.lanes,
            "schedule": args.schedule,
            "graphs": args.graphs,
            "eigensolver": args.eig,
            "autotune_s": tune_s,
            "form": form,
            "block_widths": ({str(L): scsf.scsf_tuned_width(h, L) for L in sorted(set(Ls))}
                             if uneven else {str(cfg.L): cfg.k}),
            "spmm_columns_per_thread": tile_used,
            "precision": precision,
            "adaptive_degree": args.adaptive,
            "mean_outer_iterations": float(np.mean(iters)),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("spmm_plate_kernel (Chebyshev three-term step, 13-point thin-plate "
                       "standard form, FP64)" if cfg.family == "plate" else
                       "spmm_lds_kernel (Chebyshev three-term step, %s stencil, %s)" % (
                           "9-point Q1" if windowed else "5-point",
                           "FP64" if precision == "fp64" else "FP32 residual form")),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (measured_traffic(cfg.name, {"chains": args.chains, "lanes": args.lanes,
                                                    "schedule": args.schedule,
                                                    "graphs": args.graphs,
                                                    "tile": tile_used})
                        if (cfg.index == 2 and form == "plain" and precision == "fp64"
                            and not adaptive)
                        else None),
            "avg_launch_ms": avg_ms,
            "launches": prof["filter_launches"],
            "algorithmic_bytes_per_launch": avg_bytes,
        },
    }
    if comparison and "plain_fp64_value" in comparison:
        comparison["ratio"] = value / comparison["plain_fp64_value"]
        out["config"]["learned"] = dict(train_info, trained_on=n_train, epochs=args.epochs)
        out["comparison"] = comparison
    elif comparison:
        comparison["ratio"] = value / comparison["cold_unsorted_value"]
        out["comparison"] = comparison
    if cfg.index in (2, 6) and precision == "fp64" and args.spmm_isolated == "on":
        out["spmm_isolated"] = isolated_spmm(scsf, torch, h, dops, cfg.k, degree,
                                             32 if cfg.index == 2 else 16)
        out["dense_isolated"] = isolated_gram(scsf, torch, h, dops[0].n, cfg.k, 32)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, ops, args.cpu_budget,
                                           Ls if uneven else None, ks if uneven else None,
                                           degree=degree, adaptive=adaptive)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
