"""CPU oracle for the SCSF hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, fp64 NumPy/SciPy implementation of what the hot path computes, written from the
paper (arXiv 2510.23215, "Accelerating Eigenvalue Dataset Generation via Chebyshev Subspace
Filter").  Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py` may
import it.  It shares no code with the HIP library and never imports it; both read their inputs
from the seeded generator module `scsf_inputs`.

Modules
  operator   sparse matrix of a stencil operator, assembled face by face / cell by cell
  eig        the L algebraically smallest eigenpairs (the plain definition), cyclic Jacobi
  chebyshev  Chebyshev polynomials and the scaled filter of Algorithm 1
  chfsi      Chebyshev filtered subspace iteration with locking (Algorithm 3) and the
             warm-started sequence of Section 3.2
  sort       truncated-FFT features and the greedy nearest-neighbour order (Algorithm 2)
  lanczos    upper spectral bound (Gershgorin, and the k-step Lanczos bound of Zhou & Li)
"""
from . import operator, eig, chebyshev, chfsi, sort, lanczos  # noqa: F401
