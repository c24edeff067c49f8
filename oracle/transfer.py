"""Transfer of eigenvector fields between grids of different sides (oracle; test infrastructure).

Only tests, the smoke check and the CPU baseline of the benchmark use this module.

The warm start of Algorithm 3 (Section 3.2) hands the previous problem's Ritz vectors to the
next one.  When two consecutive operators of a chain live on interior grids of different
sides N0 and N1 (the uneven batched workload), a vector of length N0^2 is read as a nodal
field on the unit square with zero Dirichlet boundary and evaluated at the nodes of the other
grid by bilinear interpolation.  The paper does not treat this case; the reading is ours.

Grid convention (shared with the operator assembly): interior node (iy, ix) of an N x N grid
sits at (x, y) = ((ix + 1) h, (iy + 1) h), h = 1 / (N + 1), and is vector entry iy * N + ix.
The boundary nodes (index -1 and N along either axis) carry the value 0.
"""
from __future__ import annotations

import numpy as np


def source_position(i1: int, N0: int, N1: int) -> float:
    """Fractional node index on the N0 grid of node i1 of the N1 grid (same coordinate)."""
    return (i1 + 1) * (N0 + 1) / (N1 + 1) - 1.0


def interpolate_field(F: np.ndarray, N1: int) -> np.ndarray:
    """Bilinear interpolation of the nodal field F (N0 x N0, zero boundary) at the N1 x N1 nodes.

    Each output node takes the four source nodes around its position, weighted by the
    products of the 1-D distances; a source index outside [0, N0) is a boundary node (value
    0).  Plain loops: this is the definition written out.
    """
    N0 = F.shape[0]
    assert F.shape == (N0, N0)

    def at(iy: int, ix: int) -> float:
        if 0 <= iy < N0 and 0 <= ix < N0:
            return float(F[iy, ix])
        return 0.0

    out = np.zeros((N1, N1))
    for oy in range(N1):
        sy = source_position(oy, N0, N1)
        jy = int(np.floor(sy))
        fy = sy - jy
        for ox in range(N1):
            sx = source_position(ox, N0, N1)
            jx = int(np.floor(sx))
            fx = sx - jx
            out[oy, ox] = ((1 - fy) * ((1 - fx) * at(jy, jx) + fx * at(jy, jx + 1))
                           + fy * ((1 - fx) * at(jy + 1, jx) + fx * at(jy + 1, jx + 1)))
    return out


def interpolate_block(X: np.ndarray, N0: int, N1: int) -> np.ndarray:
    """Columns of X (N0^2 x k) interpolated to the N1 grid: an N1^2 x k block."""
    X = np.asarray(X, dtype=np.float64)
    assert X.shape[0] == N0 * N0
    cols = [interpolate_field(X[:, j].reshape(N0, N0), N1).reshape(-1) for j in range(X.shape[1])]
    return np.stack(cols, axis=1) if cols else np.zeros((N1 * N1, 0))
