"""Benchmark of the SCSF hot path on one MI355X.

One step = the whole path over one synthetic dataset: truncated-FFT sort of the coefficient
fields (Algorithm 2) and the warm-started Chebyshev filtered subspace iteration over every
operator in sorted order (Algorithm 3), split into `--chains` chains that run concurrently
(the chunk parallelism of App. D.6).  Inputs are resident in HBM before timing; the step ends
with all eigenpairs resident in HBM.

Workload (default, the largest): 2000 anisotropic operators -div(K grad u) with an SPD tensor
field K (9-point Q1 stencil) on a 128 x 128 grid (n = 16384), L = 64 smallest eigenpairs,
block width k = 80, relative residual 1e-8, FP64, in the learned-window form: the plain
solves (degree 96, `--head-degree`) of the first 500 operators of the sorted order give the
labels of the window network, which is trained (FP32, 150 epochs) and predicts, in BF16, the
window and the filter degree of the other 1500 solves.  Every operator is solved once per
step, training included.  `--config` selects the other workloads (1 small, 2 working size, 3 uneven batch,
4 mixed precision, 6 thin-plate vibration, 7 Helmholtz).

Prints one JSON line (rank 0).  `roofline` describes the dominant kernel (the filter's
Chebyshev step): its algorithmic bytes per step over the wall time per step.  `cpu_baseline`
times the CPU oracle (NumPy/SciPy) on a bounded sample of the same workload, on one core and
on all cores the process may use (chunk model of App. D.6).  After the timed steps:
`comparison` (learned window: the plain FP64 method at the configured degree and at the best
fixed degree, and the learned form with the FP32 filter; working size: cold unsorted solves
and the static schedule), `spmm_isolated` (the filter step alone) and `dense_isolated` (the
Gram product alone).
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
    """HBM bytes per Chebyshev step (FETCH_SIZE + WRITE_SIZE of the filter kernels, each scaled
    by what the counter reads for a device copy of known size) from the committed counter
    record of this workload, while the filter step's source and the launch configuration
    (chains, lanes, schedule, graphs, tile, form, precision, fused steps, degrees, training
    epochs) are those the counters were taken with (else None)."""
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
    val = rec.get("bytes_per_chebyshev_step")
    return float(val) if val is not None else None


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
    for fam in ("divk", "potential", "aniso", "plate"):
        idx = [i for i, o in enumerate(ops) if o.family == fam]
        if idx:
            sub = S.scsf_sort([ops[i].field for i in idx], p0)
            order += [idx[j] for j in sub]
    return order


def _cpu_chain(task):
    """One chunk of the sorted order solved by the oracle as one warm-started chain (first
    solve cold), on one core, until `budget` seconds have passed.  Runs in a child process."""
    cfg_index, chunk, degree, budget, uneven = task
    from threadpoolctl import threadpool_limits
    import math
    import scsf_inputs as si
    from oracle import operator as O, chfsi as C, transfer as T
    cfg = si.CONFIGS[cfg_index]
    t0 = time.perf_counter()
    prev, prev_key, done, pairs = None, None, 0, 0
    with threadpool_limits(1):
        for i in chunk:
            op = si.operator(cfg, i)
            A = O.assemble(op)
            L = si.mixed_L(cfg, i) if uneven else cfg.L
            k = -(-(L + -(-L // 5)) // 8) * 8 if uneven else cfg.k   # L + 20%, multiple of 8
            key = (op.family, L, k)
            if prev is None or key != prev_key:
                r = C.chfsi(A, L, k, degree, cfg.tol, seed=1)
            else:
                X0 = prev.X_next
                if X0.shape[0] != A.shape[0]:
                    X0 = T.interpolate_block(X0, math.isqrt(X0.shape[0]), op.N)
                r = C.chfsi(A, L, k, degree, cfg.tol, X0=X0, theta0=prev.theta_next)
            prev, prev_key = r, key
            done += 1
            pairs += L
            if time.perf_counter() - t0 > budget:
                break
    return done, pairs, time.perf_counter() - t0


def cpu_baseline(cfg, ops, budget_s: float, degree=None):
    """The oracle (plain NumPy/SciPy SCSF, one BLAS thread per process) on a bounded sample of
    the same workload, in the chunk model of App. D.6: the sorted order is cut into W
    contiguous chunks and W processes each run their chunk as one warm-started chain for
    `budget_s` seconds.  W = 1 (one core) and W = the cores this process may use (at most 16).
    The oracle's sort of all fields is timed once and charged to both rates in proportion to
    the operators solved."""
    import multiprocessing as mp
    from oracle import sort as S
    degree = degree or cfg.degree
    uneven = cfg.family == "mixed"
    t = time.perf_counter()
    order = (family_order_host(ops, cfg.p0) if uneven
             else [int(i) for i in S.scsf_sort([o.field for o in ops], cfg.p0)])
    t_sort = time.perf_counter() - t
    log(f"[bench] cpu oracle: sort of {len(ops)} fields {t_sort:.1f}s")
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        avail = nproc
    workers = max(1, min(avail, 16))
    ctx = mp.get_context("spawn")
    out = {}
    for W in (1, workers):
        chunks = [order[(len(order) * c) // W:(len(order) * (c + 1)) // W] for c in range(W)]
        t = time.perf_counter()
        with ctx.Pool(W) as pool:
            res = pool.map(_cpu_chain, [(cfg.index, ch, degree, budget_s, uneven)
                                        for ch in chunks])
        wall = time.perf_counter() - t
        done = sum(r[0] for r in res)
        pairs = sum(r[1] for r in res)
        busy = max(r[2] for r in res)
        charged = busy + t_sort * done / len(ops)
        out[W] = {"value": pairs / charged, "cores": W, "operators": done,
                  "seconds": charged, "wall_s": wall}
        log(f"[bench] cpu oracle on {W} core(s): {done} operators, {pairs / charged:.1f} "
            f"eigenpairs/s")
    one, many = out[1], out[workers]
    sample = ("{ops} operators of the sorted sequence in {W} contiguous chunk(s), each a "
              "warm-started chain with a cold first solve, degree {d}, one BLAS thread per "
              "process, {sec:.1f}s, plus the oracle sort of all {n} fields ({ts:.1f}s) charged "
              "in proportion")
    return {"value": many["value"], "unit": "eigenpairs/s", "cores": workers, "nproc": nproc,
            "kind": "oracle",
            "sample": sample.format(ops=many["operators"], W=workers, d=degree,
                                    sec=many["seconds"], n=len(ops), ts=t_sort),
            "one_core": {"value": one["value"], "unit": "eigenpairs/s", "cores": 1,
                         "sample": sample.format(ops=one["operators"], W=1, d=degree,
                                                 sec=one["seconds"], n=len(ops), ts=t_sort)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=5,
                    help="workload: 1 small, 2 working size, 3 uneven batch, 4 mixed "
                         "precision, 5 learned window (default: the largest), 6 thin plates, "
                         "7 Helmholtz")
    ap.add_argument("--count", type=int, default=None, help="operators (default: all)")
    ap.add_argument("--chains", type=int, default=128)
    ap.add_argument("--lanes", type=int, default=6)
    ap.add_argument("--degree", type=int, default=None)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="default: the configuration's (fp64; mixed for config 4)")
    ap.add_argument("--schedule", choices=["static", "dynamic"], default=None,
                    help="static: contiguous chunks of the sorted order (App. D.6); dynamic: "
                         "each chain takes the next unsolved operator of the sorted order; "
                         "default: static for the learned-window workload (measured faster: "
                         "every chain warm-starts from its true neighbour), dynamic otherwise")
    ap.add_argument("--graphs", choices=["on", "off"], default="on",
                    help="replay each outer iteration as HIP graphs (on) or launch its kernels "
                         "one by one (off)")
    ap.add_argument("--eig", choices=["jacobi", "tridiag"], default="jacobi",
                    help="Rayleigh-Ritz eigensolver")
    ap.add_argument("--batch-form", choices=["grouped", "one-sweep"], default="grouped",
                    help="uneven workload: one lockstep batch per (L, k) group, or one batch over "
                         "every width (each sweep covers all groups); the comparison times the "
                         "other")
    ap.add_argument("--autotune", choices=["on", "off"], default="on",
                    help="tune filter tiles (and, for the uneven workload, block widths) on the "
                         "dataset once before the warmup; the timed steps use the result")
    ap.add_argument("--form", choices=["learned", "plain"], default=None,
                    help="learned-window workload only: learned (plain solves of the first "
                         "operators train the network, whose predictions steer the rest; "
                         "default) or plain")
    ap.add_argument("--train", type=int, default=500,
                    help="learned form: operators solved plainly to train the network")
    ap.add_argument("--head-degree", type=int, default=96,
                    help="learned form: filter degree of the plain solves that give the "
                         "labels (the best fixed degree measured on this family)")
    ap.add_argument("--epochs", type=int, default=150,
                    help="learned form: training epochs (c5: 150 / 300 / 600 epochs ran at "
                         "16.4k / 16.0k / 15.2k eigenpairs/s with 5.83 / 5.77 / 5.76 tail "
                         "iterations)")
    ap.add_argument("--tile", type=int, choices=[1, 2, 4, 8], default=None,
                    help="pin the filter-step tile instead of the autotuned one")
    ap.add_argument("--fused-steps", type=int, choices=[0, 2, 3, 4], default=None,
                    help="Chebyshev steps per fused filter launch (0: one step per launch); "
                         "default: 3 for the equal-size 5-point workloads (measured faster: "
                         "working size +6%%, Helmholtz +2.5%%), 0 for the uneven batch "
                         "(measured 9%% slower), the 9-point and the thin-plate ones")
    ap.add_argument("--adaptive", choices=["on", "off"], default="off",
                    help="per-vector filter degrees in [degree, min(2 degree, 64)] (FP64 "
                         "solves without degree hints)")
    ap.add_argument("--compare", choices=["on", "off"], default="on",
                    help="after the timed steps, time the baselines of the workload once: "
                         "working size: cold unsorted and the static schedule; learned "
                         "window: plain FP64 at the configured and at the best fixed degree, "
                         "and the learned form with the FP32 filter")
    ap.add_argument("--best-degree", type=int, default=96,
                    help="learned window: the fixed degree of the plain baseline that the "
                         "network's degree competes with (plain c5, static schedule: degree "
                         "64 / 80 / 96 / 128 ran at 17.1k / 17.5k / 17.6k / 17.3k eigenpairs/s)")
    ap.add_argument("--spmm-isolated", choices=["on", "off"], default="on",
                    help="also time the filter step and the Gram product alone (after the "
                         "timed steps)")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle work per CPU baseline run (one core, all cores)")
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
    if args.fused_steps is None:
        args.fused_steps = 3 if cfg.family in ("divk", "helmholtz") else 0
    scsf.scsf_set_fused_steps(h, args.fused_steps)
    scsf.scsf_set_eigensolver(h, scsf.SCSF_EIG_TRIDIAG if args.eig == "tridiag"
                              else scsf.SCSF_EIG_JACOBI)
    form_ids = {"grouped": scsf.SCSF_BATCH_GROUPED, "one-sweep": scsf.SCSF_BATCH_ONE_SWEEP}
    scsf.scsf_set_batch_form(h, form_ids[args.batch_form])
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
    precision = args.precision or ("mixed" if cfg.precision == "mixed" else "fp64")
    adaptive = args.adaptive == "on"
    if adaptive and (precision != "fp64" or form == "learned"):
        print(json.dumps({"error": "--adaptive needs FP64 solves without degree hints "
                                   "(--precision fp64, and --form plain on the learned-window "
                                   "workload)"}))
        sys.exit(2)
    if args.schedule is None:
        args.schedule = "static" if windowed and form == "learned" else "dynamic"
    sched = scsf.SCSF_SCHED_DYNAMIC if args.schedule == "dynamic" else scsf.SCSF_SCHED_STATIC
    other_sched = "dynamic" if args.schedule == "static" else "static"
    other_sched_id = (scsf.SCSF_SCHED_DYNAMIC if other_sched == "dynamic"
                      else scsf.SCSF_SCHED_STATIC)

    target = scsf.SCSF_TARGET_SMALLEST

    def params(prec=precision, deg=degree, **kw):
        return scsf.make_params(cfg.L, cfg.k, deg, cfg.tol, seed=1, schedule=kw.pop(
            "schedule", sched), precision=scsf.SCSF_MIXED if prec == "mixed" else scsf.SCSF_FP64,
            target=target, **kw)

    prm = params(adaptive=int(adaptive))
    prm64 = params(prec="fp64")
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

    def step_learned(p, p_head):
        """Sort; plain solves of the first n_train operators of the order (their Ritz values
        and bounds are the labels); FP32 training; BF16 inference for the rest, whose solves
        take the predicted window and degree.  Every operator is solved once."""
        t = time.perf_counter()
        order = scsf.scsf_sort(h, fields, cfg.p0)
        t_sort = time.perf_counter() - t
        head, tail = [int(i) for i in order[:n_train]], [int(i) for i in order[n_train:]]
        ritz = torch.empty((n_train, cfg.k), device="cuda", dtype=torch.float64)
        _, _, st1 = scsf.scsf_solve_sequence(h, [dops[i] for i in head], np.arange(n_train),
                                             args.chains, p_head, evals[:n_train],
                                             evecs[:n_train], ritz=ritz)
        t_head = time.perf_counter() - t
        beta = torch.tensor([s["beta"] for s in st1], device="cuda", dtype=torch.float64)
        target = scsf.scsf_window_labels(h, ritz, cfg.L, beta)
        x = scsf.scsf_window_input(h, scsf.scsf_features(h, fields, 16))
        params_ = scsf.scsf_window_init(h, 5)
        hist = scsf.scsf_window_train(h, params_, x[torch.tensor(head, device="cuda")], target,
                                      args.epochs, 1e-3)
        out = scsf.scsf_window_forward(h, params_, x[torch.tensor(tail, device="cuda")],
                                       bf16=True)
        hints = scsf.scsf_window_hints(h, out).cpu().numpy()
        t_train = time.perf_counter() - t - t_head
        _, _, st2 = scsf.scsf_solve_sequence(h, [dops[i] for i in tail], np.arange(len(tail)),
                                             args.chains, p, evals[n_train:], evecs[n_train:],
                                             hints=hints)
        train_info.update(loss_first=float(hist[0]), loss_last=float(hist[-1]),
                          hints_used=int(sum(s["hint"] == 2 for s in st2)),
                          mean_degree=float(np.mean([s["degree"] for s in st2])),
                          sort_s=t_sort, head_s=t_head - t_sort, train_and_infer_s=t_train,
                          tail_s=time.perf_counter() - t - t_head - t_train,
                          head_mean_iterations=float(np.mean([s["iterations"] for s in st1])),
                          tail_mean_iterations=float(np.mean([s["iterations"] for s in st2])))
        return st1 + st2

    def step_plain(p):
        order = make_order()
        if uneven:
            _, _, stats = scsf.scsf_solve_batched(h, dops, Ls, order, args.chains, p)
            return stats
        _, _, stats = scsf.scsf_solve_sequence(h, dops, order, args.chains, p, evals, evecs)
        return stats

    head_deg_used = args.head_degree if precision == "fp64" else min(args.head_degree, 64)

    def step():
        head_deg = head_deg_used
        return (step_learned(prm, params(deg=head_deg)) if form == "learned"
                else step_plain(prm))

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
        ts = time.perf_counter()
        stats = step()
        iters += [st["iterations"] for st in stats]
        log(f"[bench] step {s} done, {time.perf_counter() - ts:.2f}s"
            + (f" {train_info}" if form == "learned" else ""))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = scsf.scsf_profile_read(h, reset=True)
    scsf.scsf_profile_enable(h, False)
    pairs = args.steps * sum(Ls)
    value = pairs / dt
    log(f"[bench] {value:.0f} eigenpairs/s, {dt / args.steps * 1e3:.1f} ms per step")
    timed_info = dict(train_info)      # the comparison runs below update train_info again

    def timed(fn, label):
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = fn()
        torch.cuda.synchronize()
        tt = time.perf_counter() - t
        log(f"[bench] {label}: {sum(Ls) / tt:.0f} eigenpairs/s")
        return {"value": sum(Ls) / tt, "ms": tt * 1e3,
                "mean_iterations": float(np.mean([s["iterations"] for s in st]))}

    comparison = None
    if args.compare == "on" and cfg.index == 2:
        comparison = {
            # the same operators in their generated order, every solve from a random block
            "cold_unsorted": timed(lambda: scsf.scsf_solve_sequence(
                h, dops, np.arange(n_op), args.chains, params(cold_start=1), evals, evecs)[2],
                "cold unsorted"),
            # the other schedule (static: App. D.6 chunks, every chain warm-starts from its
            # true neighbour in the order; dynamic: chains take the next unsolved operator)
            f"{other_sched}_schedule": timed(lambda: step_plain(params(
                schedule=other_sched_id)), f"{other_sched} schedule")}
        comparison["ratio_to_cold_unsorted"] = value / comparison["cold_unsorted"]["value"]
    if args.compare == "on" and uneven and not adaptive:
        other_form = "one-sweep" if args.batch_form == "grouped" else "grouped"
        scsf.scsf_set_batch_form(h, form_ids[other_form])
        comparison = {f"batch_form_{other_form.replace('-', '_')}": timed(
            lambda: step_plain(prm), f"batch form {other_form}")}
        scsf.scsf_set_batch_form(h, form_ids[args.batch_form])
    if args.compare == "on" and windowed and form == "learned":
        comparison = {
            "plain_fp64": timed(lambda: step_plain(prm64), f"plain fp64 degree {degree}"),
            f"plain_fp64_degree{args.best_degree}": timed(
                lambda: step_plain(params(prec="fp64", deg=args.best_degree)),
                f"plain fp64 degree {args.best_degree}"),
            # the same with the other schedule
            f"plain_fp64_degree{args.best_degree}_{other_sched}_schedule": timed(
                lambda: step_plain(params(prec="fp64", deg=args.best_degree,
                                          schedule=other_sched_id)),
                f"plain fp64 degree {args.best_degree}, {other_sched} schedule"),
            # the FP32 filter takes degrees up to 64 (the library clamps its hints there)
            "learned_fp32_filter": timed(lambda: step_learned(
                params(prec="mixed"), params(prec="mixed", deg=min(args.head_degree, 64))),
                "learned window, FP32 filter")}
        comparison["learned_fp32_filter"]["mean_degree"] = train_info["mean_degree"]
        comparison["plain_fp64"]["degree"] = degree
        comparison[f"plain_fp64_degree{args.best_degree}"]["degree"] = args.best_degree
        comparison["ratio_to_plain_fp64"] = value / comparison["plain_fp64"]["value"]
        comparison["ratio_to_best_fixed_degree"] = (
            value / comparison[f"plain_fp64_degree{args.best_degree}"]["value"])

    # The dominant kernel's rate inside the timed run: the filter's algorithmic bytes per step
    # (every Chebyshev step reads its input and previous blocks' active columns, writes its
    # output, and reads each operator's coefficients once) over the wall time of a step.  The
    # HIP events around the filter launches (or filter graphs) on the lanes' streams give the
    # filter's own live time beside it; the lanes overlap, so their sum can exceed a step.
    bytes_step = prof["filter_bytes"] / args.steps
    achieved = bytes_step / (dt / args.steps) / 1e9
    # the library counts Chebyshev steps: a fused launch of S steps counts S
    live_ms = prof["filter_ms"] / max(prof["filter_launches"], 1)
    # HBM bytes of the filter per step: the committed counter record's bytes per Chebyshev
    # step (while it matches this source and launch configuration) times the live Chebyshev
    # steps per step.  The degrees and the training length set the mix of launch widths, so
    # they are part of the key.
    learned_key = ({"head_degree": head_deg_used, "epochs": args.epochs} if form == "learned"
                   else {})
    per_cheb_step = (measured_traffic(cfg.name, {"chains": args.chains, "lanes": args.lanes,
                                              "schedule": args.schedule, "graphs": args.graphs,
                                              "tile": tile_used, "form": form,
                                              "precision": precision,
                                              "fused_steps": args.fused_steps,
                                              "degree": degree, **learned_key,
                                              **({"batch_form": args.batch_form} if uneven
                                                 else {})})
                  if not adaptive else None)
    traffic_step = (per_cheb_step * prof["filter_launches"] / args.steps
                    if per_cheb_step is not None else None)
    stencil = "9-point Q1" if windowed else "5-point"
    if cfg.family == "plate":
        kname = ("spmm_plate_kernel (Chebyshev three-term step, 13-point thin-plate standard "
                 "form, FP64)")
    elif args.fused_steps and precision == "fp64":
        kname = ("spmm_fused_kernel (%d Chebyshev three-term steps per launch, %s stencil, "
                 "FP64)" % (args.fused_steps, stencil))
    else:
        kname = "spmm_lds_kernel (Chebyshev three-term step, %s stencil, %s)" % (
            stencil, "FP64" if precision == "fp64" else "FP32 residual form")
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
            "batch_form": args.batch_form if uneven else None,
            "autotune_s": tune_s,
            "form": form,
            "block_widths": ({str(L): scsf.scsf_tuned_width(h, L) for L in sorted(set(Ls))}
                             if uneven else {str(cfg.L): cfg.k}),
            "spmm_columns_per_thread": tile_used,
            "fused_steps": args.fused_steps,
            "precision": precision,
            "adaptive_degree": args.adaptive,
            "mean_outer_iterations": float(np.mean(iters)),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_step,
            "basis": "filter algorithmic bytes per step / wall time per step",
            "algorithmic_bytes_per_step": bytes_step,
            "chebyshev_steps_per_step": prof["filter_launches"] / args.steps,
            "live_filter_ms_per_step": prof["filter_ms"] / args.steps,
            "live_ms_per_chebyshev_step": live_ms,
        },
    }
    # device time of each step of Algorithm 3 summed over the lanes (they overlap), per step,
    # and each step's share: the cost split the paper reports for its CPU runs (App. E.3)
    ph = {k: v / args.steps for k, v in prof["phase_ms"].items()}
    tot = sum(ph.values()) or 1.0
    out["phases"] = {"ms_per_step_summed_over_lanes": ph,
                     "share": {k: v / tot for k, v in ph.items()}}
    if form == "learned":
        out["config"]["learned"] = dict(timed_info, trained_on=n_train, epochs=args.epochs,
                                        head_degree=head_deg_used)
    if comparison:
        out["comparison"] = comparison
    if cfg.index in (2, 5, 6) and precision == "fp64" and args.spmm_isolated == "on":
        # the one-step kernel alone (its HBM rate; the fused form moves fewer bytes than its
        # algorithmic count)
        scsf.scsf_set_fused_steps(h, 0)
        out["spmm_isolated"] = isolated_spmm(scsf, torch, h, dops, cfg.k, degree,
                                             {2: 32, 5: 48, 6: 16}[cfg.index])
        scsf.scsf_set_fused_steps(h, args.fused_steps)
        out["dense_isolated"] = isolated_gram(scsf, torch, h, dops[0].n, cfg.k, 32)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, ops, args.cpu_budget, degree=degree)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
