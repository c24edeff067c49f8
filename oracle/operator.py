"""Assembly of the discretised operators as explicit sparse matrices (oracle).

Section 2.1 turns an operator eigenvalue problem into a matrix one by finite differences; the
datasets of App. D.2 use -div(K grad u) with Dirichlet boundary conditions and a central
difference scheme.  Here the matrix is built as a sum of rank-one face terms
    A = sum_f w_f (e_a - e_b)(e_a - e_b)^T   (interior face between nodes a and b)
      + sum_f w_f e_a e_a^T                   (boundary face next to node a)
      + diag(v)
which is the conservative central-difference matrix written out face by face.  It is
symmetric positive definite whenever all w_f > 0 and v >= 0.

The 9-point family is assembled cell by cell from the bilinear (Q1) element stiffness of a
cell-centred tensor K, divided by the lumped nodal mass h^2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def node_index(N: int, iy, ix):
    return iy * N + ix


def assemble5(op) -> sp.csr_matrix:
    """Sparse matrix of a `scsf_inputs.Stencil5` operator, face by face."""
    N = op.N
    n = N * N
    rows, cols, vals = [], [], []

    def couple(a, b, w):
        # w (e_a - e_b)(e_a - e_b)^T ; a or b may be -1 meaning "boundary node" (u = 0 there)
        ia = a >= 0
        ib = b >= 0
        rows.extend([a[ia], b[ib]])
        cols.extend([a[ia], b[ib]])
        vals.extend([w[ia], w[ib]])
        both = ia & ib
        rows.extend([a[both], b[both]])
        cols.extend([b[both], a[both]])
        vals.extend([-w[both], -w[both]])

    iy, f = np.meshgrid(np.arange(N), np.arange(N + 1), indexing="ij")      # x-faces (N, N+1)
    left = np.where(f >= 1, node_index(N, iy, f - 1), -1)
    right = np.where(f < N, node_index(N, iy, np.minimum(f, N - 1)), -1)
    couple(left.ravel(), right.ravel(), np.asarray(op.wx, dtype=np.float64).ravel())

    f, ix = np.meshgrid(np.arange(N + 1), np.arange(N), indexing="ij")      # y-faces (N+1, N)
    below = np.where(f >= 1, node_index(N, f - 1, ix), -1)
    above = np.where(f < N, node_index(N, np.minimum(f, N - 1), ix), -1)
    couple(below.ravel(), above.ravel(), np.asarray(op.wy, dtype=np.float64).ravel())

    if op.v is not None:
        rows.append(np.arange(n))
        cols.append(np.arange(n))
        vals.append(np.asarray(op.v, dtype=np.float64).ravel())

    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A.tocsr()


def q1_element_stiffness(k11: float, k12: float, k22: float) -> np.ndarray:
    """4x4 stiffness int grad(phi_a)^T K grad(phi_b) of a square bilinear element.

    Local node order: 0 = (0,0), 1 = (1,0), 2 = (0,1), 3 = (1,1) in (x, y) cell coordinates.
    The integral is independent of the cell size in two dimensions.
    """
    sxx = np.array([[2, -2, 1, -1], [-2, 2, -1, 1], [1, -1, 2, -2], [-1, 1, -2, 2]]) / 6.0
    syy = np.array([[2, 1, -2, -1], [1, 2, -1, -2], [-2, -1, 2, 1], [-1, -2, 1, 2]]) / 6.0
    gx = np.array([-1.0, 1.0, -1.0, 1.0])      # sign of d(phi)/dx, each factor integrates to 1/2
    gy = np.array([-1.0, -1.0, 1.0, 1.0])
    sxy = np.outer(gx, gy) / 4.0               # int d(phi_a)/dx d(phi_b)/dy
    return k11 * sxx + k22 * syy + k12 * (sxy + sxy.T)


def assemble9(op) -> sp.csr_matrix:
    """Sparse matrix of a `scsf_inputs.Stencil9` operator, element by element."""
    N = op.N
    n = N * N
    h = 1.0 / (N + 1)
    rows, cols, vals = [], [], []
    for cy in range(N + 1):
        for cx in range(N + 1):
            k11, k12, k22 = op.cell[cy, cx]
            ke = q1_element_stiffness(k11, k12, k22) / (h * h)
            corner = [(cy - 1, cx - 1), (cy - 1, cx), (cy, cx - 1), (cy, cx)]
            idx = [node_index(N, y, x) if (0 <= y < N and 0 <= x < N) else -1 for (y, x) in corner]
            for a in range(4):
                if idx[a] < 0:
                    continue
                for b in range(4):
                    if idx[b] < 0:
                        continue
                    rows.append(idx[a])
                    cols.append(idx[b])
                    vals.append(ke[a, b])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n))
    return A.tocsr()


def dirichlet_laplacian(N: int) -> sp.csr_matrix:
    """The 5-point Dirichlet Laplacian / h^2 (positive definite sign) as the Kronecker sum of
    the 1-D second-difference matrix tridiag(-1, 2, -1) / h^2 (App. C)."""
    h = 1.0 / (N + 1)
    T = sp.diags([-np.ones(N - 1), 2.0 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1]) / (h * h)
    I = sp.identity(N)
    return (sp.kron(I, T) + sp.kron(T, I)).tocsr()


def assemble_plate_pair(op):
    """(K, M) of the thin-plate vibration problem K u = lambda M u (App. D.2, item 4):
    K = L diag(D) L discretises del^2 (D del^2 u) with simply supported edges (u = 0 and
    del^2 u = 0 on the boundary: the same Dirichlet Laplacian L on both sides), M = diag(rho)
    the lumped mass."""
    L = dirichlet_laplacian(op.N)
    K = (L @ sp.diags(np.asarray(op.D, np.float64).ravel()) @ L).tocsr()
    M = sp.diags(np.asarray(op.rho, np.float64).ravel()).tocsr()
    return K, M


def assemble_plate(op) -> sp.csr_matrix:
    """The standard symmetric form A = M^{-1/2} K M^{-1/2}: A y = lambda y with y = M^{1/2} u."""
    K, M = assemble_plate_pair(op)
    s = sp.diags(1.0 / np.sqrt(np.asarray(op.rho, np.float64).ravel()))
    return (s @ K @ s).tocsr()


def assemble(op) -> sp.csr_matrix:
    if hasattr(op, "rho"):
        return assemble_plate(op)
    if hasattr(op, "wx"):
        return assemble5(op)
    return assemble9(op)

