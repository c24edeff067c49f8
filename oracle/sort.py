"""Truncated-FFT sorting of the operator sequence (oracle, Algorithm 2).

Each operator i has a parameter matrix P^(i) (the nodal coefficient field, p x p per channel).
Algorithm 2 keeps the low-frequency block P_low = Trunc_p0(FFT(P)) and orders the problems
greedily: start from the first problem, then repeatedly append the not-yet-used problem whose
P_low is nearest (Frobenius norm) to that of the last appended one.

Readings: the kept block is the p0 x p0 corner k1, k2 in [0, p0) of the unshifted 2-D DFT,
scaled by 1/p^2 so that the DC term is the field mean (App. F calls the FFT normalised; with
equal p every uniform scaling gives the same order); multi-channel fields add their squared
distances; the running minimum starts at +infinity instead of the printed 1000, the scan is
in increasing problem index with a strict '<', so exact ties go to the lowest index; squared
distances are compared (same order as the distances).
"""
from __future__ import annotations

import numpy as np


def truncated_features(field: np.ndarray, p0: int) -> np.ndarray:
    """field: (C, p, p) real -> (C, p0, p0) complex, DFT / p^2 truncated to [0, p0)^2."""
    field = np.asarray(field, dtype=np.float64)
    if field.ndim == 2:
        field = field[None]
    p = field.shape[-1]
    if p0 > p:
        raise ValueError("p0 > p")
    F = np.fft.fft2(field, axes=(-2, -1)) / float(p * p)
    return F[:, :p0, :p0]


def sq_distances(feats: np.ndarray, cur: int, cand: np.ndarray) -> np.ndarray:
    """||P_low^(cur) - P_low^(j)||_F^2 for j in cand (summed over channels)."""
    d = feats[cand] - feats[cur][None]
    return np.sum(d.real ** 2 + d.imag ** 2, axis=tuple(range(1, d.ndim)))


def greedy_step(feats: np.ndarray, cur: int, remaining: np.ndarray):
    """One pick of the greedy loop: (chosen index, its squared distance, all squared distances)."""
    remaining = np.sort(np.asarray(remaining))
    d = sq_distances(feats, cur, remaining)
    j = int(np.argmin(d))            # first occurrence of the minimum = lowest index on ties
    return int(remaining[j]), float(d[j]), d


def greedy_order(feats: np.ndarray, start: int = 0) -> np.ndarray:
    n = feats.shape[0]
    order = [start]
    remaining = np.array([i for i in range(n) if i != start], dtype=np.int64)
    cur = start
    while remaining.size:
        j, _, _ = greedy_step(feats, cur, remaining)
        order.append(j)
        remaining = remaining[remaining != j]
        cur = j
    return np.array(order, dtype=np.int32)


def scsf_sort(fields, p0: int, start: int = 0) -> np.ndarray:
    """Algorithm 2 end to end: fields is a list/array of (C, p, p) parameter matrices."""
    feats = np.stack([truncated_features(f, p0) for f in fields])
    return greedy_order(feats, start)
