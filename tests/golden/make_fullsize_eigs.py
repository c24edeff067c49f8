"""Write the oracle's eigenvalues of every operator of the full-size workloads.

For each operator of the working-size (200 x n = 10^4, L = 100), uneven (1000 operators,
sides 48..128, L in {32, 64, 128}), mixed-precision (200 x n = 25600, L = 200),
anisotropic (2000 x n = 16384, L = 64), thin-plate (100 x n = 10^4, L = 200) and Helmholtz
(100 x n = 6400, L = 200, indefinite) workloads this stores the L + 1 algebraically smallest
eigenvalues of the assembled matrix, computed by the oracle's plain definition
(`oracle.eig.smallest_eigenpairs`: ARPACK shift-invert to machine tolerance, about 0 for the
positive definite families and about the Gershgorin lower end for the indefinite one; eq.
eq_basic of Section 2.1).  The (L + 1)-th value records the gap after the
L-th.  Entries are keyed by (configuration, operator index) and carry the operator seed, so
a changed generator is detected by the tests that read them.

Only `oracle/` does the arithmetic; `scsf_inputs` only generates the operators.

    python tests/golden/make_fullsize_eigs.py [--jobs 8] [--configs 2 3 4 5 6 7]

Output: tests/golden/fullsize_eigs_c<config>.npz with arrays
    index (n_op,) int64, seed (n_op,) int64, L (n_op,) int64,
    evals (n_op, max L + 1) float64, NaN past L_i + 1.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))


def _one(task):
    cfg_index, i = task
    import numpy as np
    import scsf_inputs as si
    from oracle import operator as O, eig as E
    cfg = si.CONFIGS[cfg_index]
    L = si.mixed_L(cfg, i) if cfg.family == "mixed" else cfg.L
    A = O.assemble(si.operator(cfg, i))
    w, _ = E.smallest_eigenpairs(A, L + 1, method="shift_invert")
    return cfg_index, i, si.op_seed(cfg.index, i), L, np.asarray(w, dtype=np.float64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--configs", type=int, nargs="+", default=[4, 6, 7, 5, 3, 2])
    args = ap.parse_args()
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import multiprocessing as mp
    import numpy as np
    import scsf_inputs as si

    tasks = [(c, i) for c in args.configs for i in range(si.CONFIGS[c].n_op)]
    results = {c: {} for c in args.configs}
    t0 = time.time()
    with mp.get_context("fork").Pool(args.jobs) as pool:
        for done, (c, i, seed, L, w) in enumerate(pool.imap_unordered(_one, tasks, chunksize=1)):
            results[c][i] = (seed, L, w)
            if (done + 1) % 50 == 0 or done + 1 == len(tasks):
                print(f"{done + 1}/{len(tasks)} operators, {time.time() - t0:.0f}s", flush=True)
    for c in args.configs:
        n_op = si.CONFIGS[c].n_op
        Lmax = max(results[c][i][1] for i in range(n_op))
        ev = np.full((n_op, Lmax + 1), np.nan)
        seeds = np.zeros(n_op, np.int64)
        Ls = np.zeros(n_op, np.int64)
        for i in range(n_op):
            seed, L, w = results[c][i]
            seeds[i], Ls[i] = seed, L
            ev[i, :L + 1] = w
        path = os.path.join(HERE, f"fullsize_eigs_c{c}.npz")
        np.savez_compressed(path, index=np.arange(n_op, dtype=np.int64), seed=seeds, L=Ls,
                            evals=ev)
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
