"""Sort diagnostics on the GPU: the study of the truncation threshold p0 (the appendix on the
truncation threshold, App. F) for a set of operators.

For the generated order, Algorithm 2 at each p0, and the full greedy order (untruncated fields,
Section 3.1), it reports:
- sort_s: time of the ordering (DFT + distances + greedy walk);
- one_sided: mean one-sided distance between the q-dimensional lowest eigenvector subspaces of
  consecutive operators in the order (scsf_subspace_distance; smaller = more similar);
- solve_s, iterations: the chained, warm-started solve of the whole set in that order;
- highfreq: mean ratio of the fields' DFT norm at or above frequency p0 (scsf_highfreq_ratio).

    python -m paper_2510_23215_amd.diagnostics --config 2 --chains 8 --lanes 8
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import scsf


def sort_sweep(h, fields: torch.Tensor, dops: list, prm, chains: int, p0s=(10, 20, 30, 40),
               q: int = 10, full_greedy: bool = True) -> list:
    """fields: (n_op, C, p, p) float64 device tensor; dops: DeviceOperator list; prm: Params."""
    n_op = fields.shape[0]
    L = prm.L
    evals = torch.empty((n_op, L), device="cuda", dtype=torch.float64)
    evecs = torch.empty((n_op, L, dops[0].n), device="cuda", dtype=torch.float64)
    orders = [("generated", None, lambda: np.arange(n_op, dtype=np.int32))]
    for p0 in p0s:
        orders.append((f"p0={p0}", p0, lambda p0=p0: scsf.scsf_sort(h, fields, p0)))
    if full_greedy:
        flat = fields.reshape(n_op, -1).to(torch.complex128)
        orders.append(("greedy", None, lambda: scsf.scsf_order_features(h, flat)))
    out = []
    for name, p0, make in orders:
        torch.cuda.synchronize()
        t = time.perf_counter()
        order = np.asarray(make(), dtype=np.int32)
        torch.cuda.synchronize()
        sort_s = time.perf_counter() - t
        t = time.perf_counter()
        _, _, stats = scsf.scsf_solve_sequence(h, dops, order, chains, prm, evals, evecs)
        torch.cuda.synchronize()
        solve_s = time.perf_counter() - t
        pairs = np.stack([order[:-1], order[1:]], 1)
        dist = scsf.scsf_subspace_distance(h, evecs, min(q, L), pairs)
        row = {"order": name, "sort_s": sort_s, "one_sided": float(dist.mean()),
               "solve_s": solve_s,
               "iterations": float(np.mean([s["iterations"] for s in stats]))}
        if p0 is not None:
            row["highfreq"] = float(scsf.scsf_highfreq_ratio(h, fields, p0).mean().item())
        out.append(row)
    return out


def main():
    import scsf_inputs as si
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--count", type=int, default=None)
    ap.add_argument("--chains", type=int, default=8)
    ap.add_argument("--lanes", type=int, default=8)
    ap.add_argument("--p0", type=int, nargs="*", default=[5, 10, 20, 30, 40])
    args = ap.parse_args()
    cfg = si.CONFIGS[args.config]
    ops = si.operators(cfg, args.count)
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, args.lanes)
    dops = [scsf.DeviceOperator(o) for o in ops]
    fields = torch.tensor(np.stack([o.field for o in ops]), device="cuda")
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_STATIC)
    scsf.scsf_solve_sequence(h, dops[:args.chains], np.arange(args.chains), args.chains, prm)
    rows = sort_sweep(h, fields, dops, prm, args.chains, args.p0)
    for r in rows:
        print(json.dumps(dict(r, workload=cfg.name, operators=len(ops), chains=args.chains,
                              degree=cfg.degree)), flush=True)


if __name__ == "__main__":
    main()
