"""Sort diagnostics (oracle): the quantities the paper uses to judge an ordering and the
truncation threshold p0 (App. F and the appendix on the truncation threshold).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU baseline use this
package.

- one_sided_distance: similarity of two operators measured between the invariant subspaces
  spanned by their q lowest eigenvectors.  Reading: the paper names the measure "one-sided
  distance", says it is built from the cosines of the principal angles and that smaller means
  more similar; the quantity with those properties is the one-sided (gap) distance
  ||(I - U U^T) V||_2 = sin of the largest principal angle, 0 for equal subspaces and 1 when
  some direction of V is orthogonal to U.
- highfreq_ratio: the share of a coefficient field's DFT that lies at or above frequency p0,
  as a ratio of Frobenius norms.  Reading: "frequency" is the signed frequency of the DFT index
  (a in (-p/2, p/2]); a coefficient is low when both |a| < p0 and |b| < p0.
- order_neighbour_distances: the one-sided distance of every consecutive pair of an order.
"""
from __future__ import annotations

import numpy as np


def one_sided_distance(U: np.ndarray, V: np.ndarray) -> float:
    """||(I - U U^T) V||_2 for U, V (n x q) with orthonormal columns."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    R = V - U @ (U.T @ V)
    return float(np.linalg.norm(R, 2))


def order_neighbour_distances(evecs, order, q: int) -> np.ndarray:
    """evecs[i]: n x L (orthonormal columns, ascending eigenvalues) of operator i; the
    distance between the q-dimensional lowest subspaces of order[j] and order[j + 1]."""
    return np.array([one_sided_distance(evecs[a][:, :q], evecs[b][:, :q])
                     for a, b in zip(order[:-1], order[1:])])


def signed_frequencies(p: int) -> np.ndarray:
    """Signed frequency of each DFT index 0..p-1: a for a <= p/2, a - p above."""
    a = np.arange(p)
    return np.where(a <= p // 2, a, a - p)


def highfreq_ratio(field: np.ndarray, p0: int) -> float:
    """field: (C, p, p) or (p, p) real.  ||F_high||_F / ||F||_F over all channels, F the 2-D
    DFT, high = the coefficients with |a| >= p0 or |b| >= p0 (signed frequencies)."""
    field = np.asarray(field, dtype=np.float64)
    if field.ndim == 2:
        field = field[None]
    p = field.shape[-1]
    F = np.fft.fft2(field, axes=(-2, -1))
    f = np.abs(signed_frequencies(p))
    low = (f[:, None] < p0) & (f[None, :] < p0)
    e = np.abs(F) ** 2
    total = e.sum()
    if total == 0.0:
        return 0.0
    return float(np.sqrt(e[:, ~low].sum() / total))
