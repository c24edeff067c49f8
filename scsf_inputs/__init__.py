"""Seeded synthetic workloads for the SCSF hot path.

This module is shared by the CPU oracle and the HIP path, so it holds no arithmetic of the
method itself (no filtering, orthonormalisation, Rayleigh-Ritz, eigen-solving or sorting).
It only draws random coefficient fields and writes down the face coefficients of the
finite-difference operators they define:

* generalized Poisson  -div(K grad u) = lambda u, K = exp(g), Dirichlet boundary
  (paper App. D.2 "Dataset", item 1; Section 2.1 for the discretisation idea);
* Schroedinger-type    -Laplace(u) + V u = lambda u, V = exp(g) rescaled to [0, 100];
* anisotropic elliptic -div(K grad u) with a 2x2 SPD tensor field K (9-point Q1 stencil);
* thin-plate vibration  del^2 (D del^2 u) = lambda rho u, D = exp(g1), rho = exp(g2) on the
  nodes (App. D.2 "Dataset", item 4); only the two nodal fields are drawn here;
* Helmholtz            -div(p grad u) - k^2 u = lambda u, p = exp(g1), k^2 = k2 exp(g2) on the
  nodes (App. D.2 "Dataset", item 3): the 5-point family with a negative diagonal term.

g is a cosine series  g(x,y) = sum_{k1,k2<M} xi_{k1k2} (1+k1^2+k2^2)^-1 cos(pi k1 x) cos(pi k2 y),
xi ~ N(0,1), so the coefficient variance is (1+k1^2+k2^2)^-2 -- a Gaussian random field
(the paper generates its coefficient fields by GRF sampling, App. D.2).

Grid convention (row-major node order, as in the worked 2x2 example of Section 2.1):
N x N interior nodes, h = 1/(N+1), node (iy, ix) sits at (x, y) = ((ix+1) h, (iy+1) h)
and has linear index p = iy*N + ix.  Face coefficients already carry the 1/h^2 factor:

* wx[iy, f], shape (N, N+1): x-face f between nodes ix=f-1 and ix=f of row iy
  (f = 0 and f = N touch the boundary), value K(x=(f+1/2) h, y=(iy+1) h) / h^2;
* wy[f, ix], shape (N+1, N): y-face f between rows iy=f-1 and iy=f, value K((ix+1) h, (f+1/2) h) / h^2;
* v[iy, ix], shape (N, N) or None: the zeroth-order (potential) term on the diagonal.

The operator these describe is (A u)_p = sum over the 4 faces of p of w_f (u_p - u_nbr) + v_p u_p
with u = 0 beyond the boundary.  For the 9-point family the coefficient set is the Q1
element stiffness of each cell (cell-centred K); see `aniso_operator`.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_STRIDE = 1_000_003


def op_seed(config: int, index: int) -> int:
    """Seed of operator `index` in configuration `config` (NumPy PCG64)."""
    return SEED_STRIDE * config + index


def grf_xi(rng: np.random.Generator, modes: int) -> np.ndarray:
    """Cosine-series weights xi_{k1k2} (1+k1^2+k2^2)^-1, shape (modes, modes)."""
    k = np.arange(modes, dtype=np.float64)
    decay = 1.0 / (1.0 + k[:, None] ** 2 + k[None, :] ** 2)
    return rng.standard_normal((modes, modes)) * decay


def grf_eval(w: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """g(x, y) = sum_{k1,k2} w[k1,k2] cos(pi k1 x) cos(pi k2 y) on broadcastable x, y."""
    modes = w.shape[0]
    k = np.arange(modes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.ndim == 2 and y.ndim == 2 and x.shape[0] == 1 and y.shape[1] == 1:
        # tensor grid (x along columns, y along rows): the series is separable,
        # g[iy, ix] = sum_{k2} cos(pi k2 y_iy) sum_{k1} w[k1, k2] cos(pi k1 x_ix)
        cx = np.cos(np.pi * np.outer(x[0], k))     # (Nx, M) over k1
        cy = np.cos(np.pi * np.outer(y[:, 0], k))  # (Ny, M) over k2
        return (cy @ w.T) @ cx.T
    shape = np.broadcast(x, y).shape
    xf = np.broadcast_to(x, shape).reshape(-1)
    yf = np.broadcast_to(y, shape).reshape(-1)
    cx = np.cos(np.pi * np.outer(xf, k))          # (P, M) over k1
    cy = np.cos(np.pi * np.outer(yf, k))          # (P, M) over k2
    g = np.einsum("pa,ab,pb->p", cx, w, cy)
    return g.reshape(shape)


@dataclasses.dataclass
class Stencil5:
    """5-point conservative operator on an N x N interior grid (see module docstring)."""
    N: int
    wx: np.ndarray            # (N, N+1)
    wy: np.ndarray            # (N+1, N)
    v: np.ndarray | None      # (N, N) or None
    field: np.ndarray         # (C, N, N) nodal parameter field(s) used by the sort
    family: str = "divk"

    @property
    def n(self) -> int:
        return self.N * self.N


@dataclasses.dataclass
class Stencil9:
    """9-point symmetric operator on an N x N interior grid.

    `cell` has shape (N+1, N+1, 3): for cell (cy, cx) -- the square between node rows cy-1, cy
    and node columns cx-1, cx (index -1 / N meaning the boundary) -- the cell-centred tensor
    entries (K11, K12, K22).  The operator is the Q1 bilinear stiffness assembled from those
    cells divided by the lumped mass h^2 (so its units match the 5-point family).
    """
    N: int
    cell: np.ndarray          # (N+1, N+1, 3)
    field: np.ndarray         # (3, N, N) nodal K11, K12, K22 used by the sort
    family: str = "aniso"

    @property
    def n(self) -> int:
        return self.N * self.N


@dataclasses.dataclass
class Plate:
    """Thin-plate vibration operator on an N x N interior grid: nodal flexural rigidity D and
    nodal density rho (the lumped mass), both (N, N)."""
    N: int
    D: np.ndarray             # (N, N)
    rho: np.ndarray           # (N, N)
    field: np.ndarray         # (2, N, N): D and rho, used by the sort
    family: str = "plate"

    @property
    def n(self) -> int:
        return self.N * self.N


def _face_grids(N: int):
    h = 1.0 / (N + 1)
    node = (np.arange(N) + 1.0) * h            # node coordinates
    face = (np.arange(N + 1) + 0.5) * h         # face-midpoint coordinates
    return h, node, face


def divk_operator(N: int, modes: int, seed: int) -> Stencil5:
    """-div(K grad u), K = exp(g) evaluated analytically at face midpoints and nodes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return divk_from_weights(N, grf_xi(rng, modes))


def perturbed_divk_chain(N: int, modes: int, seed: int, count: int, step: float = 0.01):
    """`count` operators -div(K grad u) whose GRF weights move along a straight line,
    w_j = w + j * step * (|w| / |d|) d with w, d two weight draws: consecutive weight vectors
    differ by `step` times the norm of the first (a slowly varying family of operators)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w, d = grf_xi(rng, modes), grf_xi(rng, modes)
    d = d * (np.linalg.norm(w) / np.linalg.norm(d))
    return [divk_from_weights(N, w + j * step * d) for j in range(count)]


def divk_from_weights(N: int, w: np.ndarray) -> Stencil5:
    """-div(K grad u) with K = exp(g) for the cosine-series weights w (grf_xi's layout)."""
    h, node, face = _face_grids(N)
    inv_h2 = 1.0 / (h * h)
    wx = np.exp(grf_eval(w, face[None, :], node[:, None])) * inv_h2     # (N, N+1): x=face, y=node
    wy = np.exp(grf_eval(w, node[None, :], face[:, None])) * inv_h2     # (N+1, N): x=node, y=face
    field = np.exp(grf_eval(w, node[None, :], node[:, None]))[None]     # (1, N, N)
    return Stencil5(N=N, wx=wx, wy=wy, v=None, field=field, family="divk")


def potential_operator(N: int, modes: int, seed: int, vmax: float = 100.0) -> Stencil5:
    """-Laplace(u) + V u with V = exp(g) on the nodes, affinely rescaled to [0, vmax]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = grf_xi(rng, modes)
    h, node, _ = _face_grids(N)
    inv_h2 = 1.0 / (h * h)
    e = np.exp(grf_eval(w, node[None, :], node[:, None]))
    v = vmax * (e - e.min()) / (e.max() - e.min())
    wx = np.full((N, N + 1), inv_h2)
    wy = np.full((N + 1, N), inv_h2)
    return Stencil5(N=N, wx=wx, wy=wy, v=v, field=v[None].copy(), family="potential")


def laplace_operator(N: int) -> Stencil5:
    """K == 1: the Dirichlet Laplacian, whose spectrum has a closed form."""
    h = 1.0 / (N + 1)
    inv_h2 = 1.0 / (h * h)
    return Stencil5(N=N, wx=np.full((N, N + 1), inv_h2), wy=np.full((N + 1, N), inv_h2),
                    v=None, field=np.ones((1, N, N)), family="divk")


def aniso_tensor(w1, w2, wt, x, y, lo=0.1, hi=10.0):
    """K = R(theta) diag(e1, e2) R(theta)^T with e_i = exp(clip(g_i, ln lo, ln hi)), theta = pi g_t."""
    e1 = np.exp(np.clip(grf_eval(w1, x, y), np.log(lo), np.log(hi)))
    e2 = np.exp(np.clip(grf_eval(w2, x, y), np.log(lo), np.log(hi)))
    th = np.pi * grf_eval(wt, x, y)
    c, s = np.cos(th), np.sin(th)
    k11 = c * c * e1 + s * s * e2
    k12 = c * s * (e1 - e2)
    k22 = s * s * e1 + c * c * e2
    return k11, k12, k22


def aniso_operator(N: int, modes: int, seed: int) -> Stencil9:
    """Anisotropic -div(K grad u) with an SPD tensor field, Q1 stiffness on cells."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w1, w2, wt = grf_xi(rng, modes), grf_xi(rng, modes), grf_xi(rng, modes)
    h = 1.0 / (N + 1)
    centre = (np.arange(N + 1) + 0.5) * h       # cell centres, cells indexed 0..N
    node = (np.arange(N) + 1.0) * h
    k11, k12, k22 = aniso_tensor(w1, w2, wt, centre[None, :], centre[:, None])
    cell = np.stack([k11, k12, k22], axis=-1)   # (N+1, N+1, 3) indexed [cy, cx]
    n11, n12, n22 = aniso_tensor(w1, w2, wt, node[None, :], node[:, None])
    field = np.stack([n11, n12, n22], axis=0)
    return Stencil9(N=N, cell=cell, field=field)


def helmholtz_operator(N: int, modes: int, seed: int, k2: float = 200.0) -> Stencil5:
    """-div(p grad u) - k^2 u: p = exp(g1) at faces and nodes, k^2 = k2 exp(g2 / 2) at nodes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w1, w2 = grf_xi(rng, modes), grf_xi(rng, modes)
    h, node, face = _face_grids(N)
    inv_h2 = 1.0 / (h * h)
    wx = np.exp(grf_eval(w1, face[None, :], node[:, None])) * inv_h2
    wy = np.exp(grf_eval(w1, node[None, :], face[:, None])) * inv_h2
    p = np.exp(grf_eval(w1, node[None, :], node[:, None]))
    ksq = k2 * np.exp(0.5 * grf_eval(w2, node[None, :], node[:, None]))
    return Stencil5(N=N, wx=wx, wy=wy, v=-ksq, field=np.stack([p, ksq]), family="helmholtz")


def plate_operator(N: int, modes: int, seed: int) -> Plate:
    """Rigidity D = exp(g1) and density rho = exp(g2 / 2) at the nodes (two independent GRFs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w1, w2 = grf_xi(rng, modes), grf_xi(rng, modes)
    _, node, _ = _face_grids(N)
    D = np.exp(grf_eval(w1, node[None, :], node[:, None]))
    rho = np.exp(0.5 * grf_eval(w2, node[None, :], node[:, None]))
    return Plate(N=N, D=D, rho=rho, field=np.stack([D, rho]))


def gaussian_block(n: int, k: int, seed: int) -> np.ndarray:
    """A seeded i.i.d. N(0,1) block (n x k, column-major order of the returned Fortran array)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asfortranarray(rng.standard_normal((n, k)))


# ---------------------------------------------------------------------------------------------
# The benchmark configurations (sizes of the paper's workloads: n from 10^3 to 2.6*10^4,
# L up to a few hundred, degree 20, p0 = 20; App. D.4).
# ---------------------------------------------------------------------------------------------

@dataclasses.dataclass
class Config:
    name: str
    index: int
    n_op: int
    L: int
    k: int
    degree: int
    p0: int
    tol: float
    modes: int
    sides: tuple            # grid side per operator family draw, see `operators`
    family: str             # "divk", "mixed", "aniso", "plate"
    precision: str = "fp64"


CONFIGS = {
    1: Config("c1_poisson32", 1, 20, 16, 24, 20, 4, 1e-8, 8, (32,), "divk"),
    # degree: the working-size configuration allows 16..30; the top of that range
    2: Config("c2_poisson100", 2, 200, 100, 120, 30, 20, 1e-8, 16, (100,), "divk"),
    3: Config("c3_batched_uneven", 3, 1000, 0, 0, 20, 20, 1e-8, 16, tuple(range(48, 129)), "mixed"),
    4: Config("c4_mixed160", 4, 200, 200, 240, 20, 20, 1e-8, 16, (160,), "divk", "mixed"),
    5: Config("c5_aniso128", 5, 2000, 64, 80, 20, 16, 1e-8, 16, (128,), "aniso"),
    # thin-plate vibration at the paper's vibration size (n = 10^4, L = 200); tol 1e-6: the
    # FP64 floor of the relative residual of the lowest modes, eps ||A|| / lambda_1, is about
    # 2e-8 for these plates
    6: Config("c6_plate100", 6, 100, 200, 240, 30, 20, 1e-6, 16, (100,), "plate"),
    # Helmholtz at the paper's size (n = 6400, L = 200, tol 1e-8): the 200 lowest eigenvalues
    # of the indefinite -div(p grad u) - k^2 u
    7: Config("c7_helmholtz80", 7, 100, 200, 240, 20, 20, 1e-8, 16, (80,), "helmholtz"),
}


def operator(cfg: Config, i: int):
    """Operator i of configuration cfg (deterministic in (cfg.index, i))."""
    seed = op_seed(cfg.index, i)
    if cfg.family == "divk":
        return divk_operator(cfg.sides[0], cfg.modes, seed)
    if cfg.family == "aniso":
        return aniso_operator(cfg.sides[0], cfg.modes, seed)
    if cfg.family == "plate":
        return plate_operator(cfg.sides[0], cfg.modes, seed)
    if cfg.family == "helmholtz":
        return helmholtz_operator(cfg.sides[0], cfg.modes, seed)
    if cfg.family == "mixed":
        rng = np.random.Generator(np.random.PCG64(seed + 7))
        side = int(rng.integers(cfg.sides[0], cfg.sides[-1] + 1))
        if i % 2 == 0:
            return divk_operator(side, cfg.modes, seed)
        return potential_operator(side, cfg.modes, seed)
    raise ValueError(cfg.family)


def mixed_L(cfg: Config, i: int) -> int:
    """L of operator i in the uneven configuration: drawn from {32, 64, 128}."""
    rng = np.random.Generator(np.random.PCG64(op_seed(cfg.index, i) + 11))
    return int(rng.choice([32, 64, 128]))


def operators(cfg: Config, count: int | None = None):
    count = cfg.n_op if count is None else count
    return [operator(cfg, i) for i in range(count)]
