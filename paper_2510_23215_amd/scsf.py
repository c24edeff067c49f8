"""Thin Python binding of libscsf (the C ABI in include/scsf.h).

Argument marshalling only: every step runs in the HIP library.  PyTorch provides device
memory and the stream.  Blocks of vectors are n x k torch tensors in column-major layout
(stride (1, ld)); `colmajor(n, k)` allocates one.  The library must have been built
(`paper_2510_23215_amd.build.build()`); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_uint64, c_void_p

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libscsf.so")

SCSF_OK, SCSF_EINVAL, SCSF_ENOMEM, SCSF_ENOTCONV = 0, -1, -2, -3
SCSF_EBREAKDOWN, SCSF_EHIP, SCSF_ENUMERIC = -4, -5, -6
SCSF_STENCIL5, SCSF_STENCIL9, SCSF_CSR, SCSF_PLATE = 1, 2, 3, 4
SCSF_FP64, SCSF_MIXED = 0, 1
SCSF_SCHED_STATIC, SCSF_SCHED_DYNAMIC = 0, 1
SCSF_TARGET_SMALLEST, SCSF_TARGET_MAGNITUDE = 0, 1
SCSF_EIG_JACOBI, SCSF_EIG_TRIDIAG = 0, 1
SCSF_BATCH_GROUPED, SCSF_BATCH_ONE_SWEEP = 0, 1


class ScsfError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


class Operator(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("nx", c_int32), ("n", c_int64), ("wx", c_void_p),
                ("wy", c_void_p), ("v", c_void_p), ("cell", c_void_p), ("row_ptr", c_void_p),
                ("col_idx", c_void_p), ("val", c_void_p), ("nnz", c_int64)]


class Params(ctypes.Structure):
    _fields_ = [("L", c_int32), ("k", c_int32), ("degree", c_int32), ("max_iter", c_int32),
                ("lanczos_steps", c_int32), ("precision", c_int32), ("schedule", c_int32),
                ("adaptive", c_int32), ("cold_start", c_int32), ("target", c_int32),
                ("tol", c_double), ("seed", c_uint64)]


PHASES = ("filter", "orth", "rr", "resid", "bound")


class Profile(ctypes.Structure):
    _fields_ = [("filter_launches", c_int64), ("filter_ms", c_double), ("filter_bytes", c_double),
                ("phase_ms", c_double * 5)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("nconv", c_int32), ("status", c_int32),
                ("chol_shifts", c_int32), ("degree", c_int32), ("hint", c_int32),
                ("filter_cols", c_int64), ("beta", c_double), ("max_rel_resid", c_double),
                ("ms_filter", ctypes.c_float), ("ms_orth", ctypes.c_float),
                ("ms_rr", ctypes.c_float), ("ms_resid", ctypes.c_float),
                ("ms_bound", ctypes.c_float), ("ms_wall", ctypes.c_float),
                ("magnitude_route", c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2510_23215_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl, u64 = c_void_p, c_int32, c_int64, c_double, c_uint64
        sig = {
            "scsf_create": [POINTER(c_void_p), vp],
            "scsf_destroy": [vp],
            "scsf_set_stream": [vp, vp],
            "scsf_spmm": [vp, POINTER(Operator), vp, i64, i32, vp, i64],
            "scsf_filter": [vp, POINTER(Operator), vp, i64, i32, i32, dbl, dbl, dbl, vp, i64],
            "scsf_filter_batched": [vp, POINTER(Operator), i32, vp, i64, i64, i32, i32,
                                    POINTER(c_double), vp, i64, i64],
            "scsf_highfreq_ratio": [vp, vp, i32, i32, i32, i32, vp],
            "scsf_gram_batched": [vp, i32, i64, i32, vp, i64, i64, vp, i32, POINTER(c_double)],
            "scsf_subspace_distance": [vp, i64, i32, vp, i64, i64, i32, POINTER(c_int32),
                                       POINTER(c_int32), i32, POINTER(c_double)],
            "scsf_orthonormalize": [vp, i64, vp, i64, i32, vp, i64, i32],
            "scsf_rayleigh_ritz": [vp, POINTER(Operator), vp, i64, i32, vp, vp],
            "scsf_bounds": [vp, POINTER(Operator), i32, u64, POINTER(c_double)],
            "scsf_bounds_noalloc": [vp, POINTER(Operator), i32, u64, POINTER(c_double)],
            "scsf_features": [vp, vp, i32, i32, i32, i32, vp],
            "scsf_sort": [vp, vp, i32, i32, i32, i32, i32, POINTER(c_int32)],
            "scsf_solve": [vp, POINTER(Operator), POINTER(Params), vp, vp, vp, vp, vp, vp,
                           POINTER(Stats)],
            "scsf_solve_sequence": [vp, POINTER(Operator), i32, POINTER(c_int32), i32,
                                    POINTER(Params), vp, vp, POINTER(Stats)],
        }
        sig["scsf_solve_sequence_hinted"] = [vp, POINTER(Operator), i32, POINTER(c_int32), i32,
                                             POINTER(Params), POINTER(c_double), vp, vp, vp,
                                             POINTER(Stats)]
        sig["scsf_window_init"] = [vp, vp, u64]
        sig["scsf_window_input"] = [vp, vp, i32, i32, i32, vp]
        sig["scsf_window_forward"] = [vp, vp, vp, i32, i32, vp]
        sig["scsf_window_loss_grad"] = [vp, vp, vp, vp, i32, vp, POINTER(c_double)]
        sig["scsf_window_train"] = [vp, vp, vp, vp, i32, i32, ctypes.c_float, POINTER(c_double)]
        sig["scsf_window_labels"] = [vp, vp, i32, i32, i32, vp, vp]
        sig["scsf_window_hints"] = [vp, vp, i32, vp]
        sz = ctypes.c_size_t
        sig["scsf_workspace_bytes"] = [POINTER(Params), i64, POINTER(sz)]
        sig["scsf_workspace_bytes_sequence"] = [vp, POINTER(Params), i64, i32, i32, i32,
                                                POINTER(sz)]
        sig["scsf_set_workspace"] = [vp, vp, sz]
        sig["scsf_workspace_peak"] = [vp, POINTER(sz)]
        sig["scsf_profile_enable"] = [vp, i32]
        sig["scsf_set_lanes"] = [vp, i32]
        sig["scsf_set_fused_steps"] = [vp, i32]
        sig["scsf_set_batch_form"] = [vp, i32]
        sig["scsf_set_graphs"] = [vp, i32]
        sig["scsf_set_eigensolver"] = [vp, i32]
        sig["scsf_profile_read"] = [vp, POINTER(Profile), i32]
        sig["scsf_order_features"] = [vp, vp, i32, i32, i32, POINTER(c_int32)]
        sig["scsf_interpolate"] = [vp, i32, i32, i32, vp, i64, vp, i64]
        sig["scsf_block_width"] = [i32]
        sig["scsf_autotune"] = [vp, POINTER(Operator), i32, POINTER(c_int32), POINTER(c_int32),
                                POINTER(Params), i32]
        sig["scsf_tuned_width"] = [vp, i32]
        sig["scsf_tuned_tile"] = [vp, i64, i32]
        sig["scsf_set_tile"] = [vp, i32]
        sig["scsf_solve_batched"] = [vp, POINTER(Operator), i32, POINTER(c_int32),
                                     POINTER(c_int32), POINTER(c_int32), i32, POINTER(Params),
                                     vp, vp, POINTER(Stats)]
        sig["scsf_solve_batched_hinted"] = [vp, POINTER(Operator), i32, POINTER(c_int32),
                                            POINTER(c_int32), POINTER(c_int32), i32,
                                            POINTER(Params), POINTER(c_double), vp, vp,
                                            POINTER(Stats)]
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c_int32
        L.scsf_status_string.argtypes = [c_int32]
        L.scsf_status_string.restype = ctypes.c_char_p
        L.scsf_window_param_count.argtypes = []
        L.scsf_window_param_count.restype = c_int32
        L.scsf_version.argtypes = []
        L.scsf_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().scsf_status_string(int(s)).decode()


def _check(status: int, what: str, allow=(SCSF_OK,)):
    if status not in allow:
        raise ScsfError(status, what)
    return status


def colmajor(n: int, k: int, device="cuda", dtype=torch.float64) -> torch.Tensor:
    """An n x k tensor with column-major strides (1, n)."""
    return torch.empty((k, n), device=device, dtype=dtype).t()


def as_colmajor(x: torch.Tensor) -> torch.Tensor:
    if x.dim() == 1:
        x = x[:, None]
    if x.stride(0) == 1 and x.stride(1) >= x.shape[0]:
        return x
    return x.t().contiguous().t()


def _ld(x: torch.Tensor) -> int:
    return max(int(x.stride(1)), int(x.shape[0])) if x.dim() == 2 else int(x.shape[0])


def _ptr(x):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


class Handle:
    """scsf_handle bound to a torch CUDA (HIP) stream (default: the current stream)."""

    def __init__(self, stream: torch.cuda.Stream | None = None):
        self._h = c_void_p()
        stream = stream or torch.cuda.current_stream()
        self.stream = stream
        _check(lib().scsf_create(ctypes.byref(self._h), c_void_p(stream.cuda_stream)),
               "scsf_create")

    @property
    def ptr(self):
        return self._h

    def close(self):
        if self._h:
            lib().scsf_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceOperator:
    """Device copy of an operator from `scsf_inputs` (Stencil5 / Stencil9 / Plate) or a CSR
    matrix."""

    def __init__(self, op=None, *, csr=None, device="cuda"):
        self._keep = []
        s = Operator()
        if csr is not None:
            indptr, indices, data = csr
            n = len(indptr) - 1
            rp = torch.as_tensor(np.asarray(indptr, np.int32), device=device)
            ci = torch.as_tensor(np.asarray(indices, np.int32), device=device)
            va = torch.as_tensor(np.asarray(data, np.float64), device=device)
            self._keep += [rp, ci, va]
            s.kind, s.nx, s.n = SCSF_CSR, 0, n
            s.row_ptr, s.col_idx, s.val, s.nnz = rp.data_ptr(), ci.data_ptr(), va.data_ptr(), len(data)
        elif hasattr(op, "rho"):
            D = torch.as_tensor(np.ascontiguousarray(op.D, np.float64).ravel(), device=device)
            rho = torch.as_tensor(np.ascontiguousarray(op.rho, np.float64).ravel(), device=device)
            self._keep += [D, rho]
            s.kind, s.nx, s.n = SCSF_PLATE, op.N, op.N * op.N
            s.wx, s.wy = D.data_ptr(), rho.data_ptr()
        elif hasattr(op, "wx"):
            wx = torch.as_tensor(np.ascontiguousarray(op.wx, np.float64), device=device)
            wy = torch.as_tensor(np.ascontiguousarray(op.wy, np.float64), device=device)
            self._keep += [wx, wy]
            s.kind, s.nx, s.n = SCSF_STENCIL5, op.N, op.N * op.N
            s.wx, s.wy = wx.data_ptr(), wy.data_ptr()
            if op.v is not None:
                v = torch.as_tensor(np.ascontiguousarray(op.v, np.float64), device=device)
                self._keep.append(v)
                s.v = v.data_ptr()
        else:
            cell = torch.as_tensor(np.ascontiguousarray(op.cell, np.float64), device=device)
            self._keep.append(cell)
            s.kind, s.nx, s.n = SCSF_STENCIL9, op.N, op.N * op.N
            s.cell = cell.data_ptr()
        self.struct = s
        self.n = int(s.n)

    def ref(self):
        return ctypes.byref(self.struct)


# --------------------------------------------------------------------------- entry points
def scsf_spmm(h: Handle, A: DeviceOperator, X: torch.Tensor, Y: torch.Tensor | None = None):
    X = as_colmajor(X)
    if Y is None:
        Y = colmajor(X.shape[0], X.shape[1], device=X.device)
    _check(lib().scsf_spmm(h.ptr, A.ref(), _ptr(X), _ld(X), X.shape[1], _ptr(Y), _ld(Y)),
           "scsf_spmm")
    return Y


def scsf_filter(h: Handle, A: DeviceOperator, X: torch.Tensor, degree: int, lam: float, c: float,
                e: float, Y: torch.Tensor | None = None):
    X = as_colmajor(X)
    if Y is None:
        Y = colmajor(X.shape[0], X.shape[1], device=X.device)
    _check(lib().scsf_filter(h.ptr, A.ref(), _ptr(X), _ld(X), X.shape[1], int(degree), float(lam),
                             float(c), float(e), _ptr(Y), _ld(Y)), "scsf_filter")
    return Y


def scsf_filter_batched(h: Handle, ops: list, X: torch.Tensor, degree: int, windows,
                        Y: torch.Tensor | None = None):
    """X: B x ncols x ldx tensor (block b column-major, rows beyond operator b's n ignored);
    windows: B x 3 (lambda, c, e).  Returns Y of the same shape."""
    B, ncols, ld = X.shape
    assert X.is_contiguous() and len(ops) == B
    if Y is None:
        Y = torch.empty_like(X)
    arr = (Operator * B)(*[o.struct for o in ops])
    wv = np.ascontiguousarray(np.asarray(windows, dtype=np.float64).reshape(B, 3))
    _check(lib().scsf_filter_batched(h.ptr, arr, B, _ptr(X), ld, ncols * ld, ncols, int(degree),
                                     wv.ctypes.data_as(POINTER(c_double)), _ptr(Y), ld, ncols * ld),
           "scsf_filter_batched")
    return Y


def scsf_gram_batched(h: Handle, X: torch.Tensor, timed: bool = False):
    """X: (B, k, n) tensor (block b = n x k column-major) -> (G (B, k, k) with G[b] = X_b^T X_b,
    kernel milliseconds or None)."""
    assert X.is_contiguous()
    B, k, n = X.shape
    G = torch.empty((B, k, k), device=X.device, dtype=torch.float64)
    ms = c_double(0.0)
    _check(lib().scsf_gram_batched(h.ptr, B, n, k, _ptr(X), n, k * n, _ptr(G), k,
                                   ctypes.byref(ms) if timed else None), "scsf_gram_batched")
    return G, (ms.value if timed else None)


def scsf_orthonormalize(h: Handle, X: torch.Tensor, V: torch.Tensor | None = None):
    """In place: X <- orthonormal basis of (I - V V^T) X.  X must be column-major."""
    assert X.stride(0) == 1
    nl = 0 if V is None else V.shape[1]
    if V is not None:
        V = as_colmajor(V)
    _check(lib().scsf_orthonormalize(h.ptr, X.shape[0], _ptr(X), _ld(X), X.shape[1], _ptr(V),
                                     _ld(V) if V is not None else 0, nl), "scsf_orthonormalize")
    return X


def scsf_rayleigh_ritz(h: Handle, A: DeviceOperator, X: torch.Tensor):
    """In place: X <- Ritz vectors; returns (theta, relative residuals) as device tensors."""
    assert X.stride(0) == 1
    k = X.shape[1]
    theta = torch.empty(k, device=X.device, dtype=torch.float64)
    res = torch.empty(k, device=X.device, dtype=torch.float64)
    _check(lib().scsf_rayleigh_ritz(h.ptr, A.ref(), _ptr(X), _ld(X), k, _ptr(theta), _ptr(res)),
           "scsf_rayleigh_ritz")
    return theta, res


def scsf_bounds(h: Handle, A: DeviceOperator, steps: int = 20, seed: int = 0):
    out = (c_double * 4)()
    _check(lib().scsf_bounds(h.ptr, A.ref(), int(steps), c_uint64(seed), out), "scsf_bounds")
    return {"gershgorin": out[0], "lanczos": out[1], "theta_min": out[2], "beta": out[3]}


def scsf_bounds_noalloc(h: Handle, A: DeviceOperator, steps: int = 20, seed: int = 0):
    """scsf_bounds with its scratch in the library's fixed device array (no allocation)."""
    out = (c_double * 4)()
    _check(lib().scsf_bounds_noalloc(h.ptr, A.ref(), int(steps), c_uint64(seed), out),
           "scsf_bounds_noalloc")
    return {"gershgorin": out[0], "lanczos": out[1], "theta_min": out[2], "beta": out[3]}


def scsf_highfreq_ratio(h: Handle, fields: torch.Tensor, p0: int) -> torch.Tensor:
    """fields: (n_op, C, p, p) float64 device tensor -> (n_op,) high-frequency norm ratio."""
    fields = fields.contiguous()
    n_op, C, p, _ = fields.shape
    out = torch.empty(n_op, device=fields.device, dtype=torch.float64)
    _check(lib().scsf_highfreq_ratio(h.ptr, _ptr(fields), n_op, C, p, int(p0), _ptr(out)),
           "scsf_highfreq_ratio")
    return out


def scsf_subspace_distance(h: Handle, evecs: torch.Tensor, q: int, pairs) -> np.ndarray:
    """evecs: (n_blocks, L, n) tensor as returned by the solvers (block i = n x L column-major);
    pairs: sequence of (a, b) block indices -> one-sided distances of the first q columns."""
    assert evecs.is_contiguous()
    nb, L, n = evecs.shape
    pairs = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    P = pairs.shape[0]
    a = np.ascontiguousarray(pairs[:, 0])
    b = np.ascontiguousarray(pairs[:, 1])
    out = np.zeros(max(P, 1), dtype=np.float64)
    _check(lib().scsf_subspace_distance(h.ptr, n, int(q), _ptr(evecs), n, L * n, nb,
                                        a.ctypes.data_as(POINTER(c_int32)),
                                        b.ctypes.data_as(POINTER(c_int32)), P,
                                        out.ctypes.data_as(POINTER(c_double))),
           "scsf_subspace_distance")
    return out[:P]


def scsf_features(h: Handle, fields: torch.Tensor, p0: int):
    """fields: (n_op, C, p, p) float64 device tensor -> (n_op, C, p0, p0) complex128."""
    fields = fields.contiguous()
    n_op, C, p, _ = fields.shape
    out = torch.empty((n_op, C, p0, p0, 2), device=fields.device, dtype=torch.float64)
    _check(lib().scsf_features(h.ptr, _ptr(fields), n_op, C, p, p0, _ptr(out)), "scsf_features")
    return torch.view_as_complex(out)


def scsf_sort(h: Handle, fields: torch.Tensor, p0: int, start: int = 0) -> np.ndarray:
    fields = fields.contiguous()
    n_op, C, p, _ = fields.shape
    order = (c_int32 * n_op)()
    _check(lib().scsf_sort(h.ptr, _ptr(fields), n_op, C, p, p0, int(start), order), "scsf_sort")
    return np.frombuffer(order, dtype=np.int32).copy()


def scsf_order_features(h: Handle, feats: torch.Tensor, start: int = 0) -> np.ndarray:
    """Greedy order of Algorithm 2 on precomputed features: feats (n_op, ...) complex128."""
    feats = torch.view_as_real(feats.contiguous()).contiguous()
    n_op = feats.shape[0]
    flen = feats[0].numel() // 2
    order = (c_int32 * n_op)()
    _check(lib().scsf_order_features(h.ptr, _ptr(feats), n_op, flen, int(start), order),
           "scsf_order_features")
    return np.frombuffer(order, dtype=np.int32).copy()


def scsf_interpolate(h: Handle, X: torch.Tensor, N0: int, N1: int) -> torch.Tensor:
    """X: (ncols, N0*N0) float64 device tensor (one field per row) -> (ncols, N1*N1)."""
    X = X.contiguous()
    ncols = X.shape[0]
    Y = torch.empty((ncols, N1 * N1), device=X.device, dtype=torch.float64)
    _check(lib().scsf_interpolate(h.ptr, int(N0), int(N1), ncols, _ptr(X), N0 * N0, _ptr(Y),
                                  N1 * N1), "scsf_interpolate")
    return Y


def scsf_block_width(L: int) -> int:
    k = int(lib().scsf_block_width(int(L)))
    if k < 0:
        raise ScsfError(k, "scsf_block_width")
    return k


def scsf_autotune(h: Handle, ops: list, Ls, order, prm: Params, probe: int = 4):
    """Tune filter tiles and block widths on this dataset; the handle keeps the results."""
    n_op = len(ops)
    arr = (Operator * n_op)(*[o.struct for o in ops])
    Lc = (c_int32 * n_op)(*[int(x) for x in Ls])
    ordc = (c_int32 * n_op)(*np.asarray(order, dtype=np.int32).tolist())
    _check(lib().scsf_autotune(h.ptr, arr, n_op, Lc, ordc, ctypes.byref(prm), int(probe)),
           "scsf_autotune")


def scsf_tuned_width(h: Handle, L: int) -> int:
    k = int(lib().scsf_tuned_width(h.ptr, int(L)))
    if k < 0:
        raise ScsfError(k, "scsf_tuned_width")
    return k


def scsf_tuned_tile(h: Handle, n: int, k: int) -> int:
    c = int(lib().scsf_tuned_tile(h.ptr, int(n), int(k)))
    if c < 0:
        raise ScsfError(c, "scsf_tuned_tile")
    return c


def scsf_set_tile(h: Handle, tile: int):
    _check(lib().scsf_set_tile(h.ptr, int(tile)), "scsf_set_tile")


def scsf_solve_batched(h: Handle, ops: list, Ls, order, chains: int, prm: Params, ks=None,
                       allow_notconv=False, hints=None):
    """Operators of different sizes and L in one call.  Returns (evals, evecs, stats): evals[i]
    a length-L_i view, evecs[i] an (L_i, n_i) view (row j = eigenvector j), both into the
    packed device arrays, and the per-operator stats dicts.  hints: (n_op, 3) host array of
    (lambda_1, lambda_{L+1}, degree) per operator (scsf_solve_batched_hinted)."""
    n_op = len(ops)
    arr = (Operator * n_op)(*[o.struct for o in ops])
    Ls = [int(x) for x in Ls]
    Lc = (c_int32 * n_op)(*Ls)
    kc = None if ks is None else (c_int32 * n_op)(*[int(x) for x in ks])
    ordc = (c_int32 * n_op)(*np.asarray(order, dtype=np.int32).tolist())
    ne = sum(Ls)
    nv = sum(o.n * L for o, L in zip(ops, Ls))
    ev = torch.empty(ne, device="cuda", dtype=torch.float64)
    vec = torch.empty(nv, device="cuda", dtype=torch.float64)
    stats = (Stats * n_op)()
    allow = (SCSF_OK, SCSF_ENOTCONV) if allow_notconv else (SCSF_OK,)
    if hints is None:
        _check(lib().scsf_solve_batched(h.ptr, arr, n_op, Lc, kc, ordc, int(chains),
                                        ctypes.byref(prm), _ptr(ev), _ptr(vec), stats),
               "scsf_solve_batched", allow)
    else:
        hh = np.ascontiguousarray(hints, dtype=np.float64).reshape(-1)
        assert hh.size == 3 * n_op
        hc = (c_double * hh.size)(*hh.tolist())
        _check(lib().scsf_solve_batched_hinted(h.ptr, arr, n_op, Lc, kc, ordc, int(chains),
                                               ctypes.byref(prm), hc, _ptr(ev), _ptr(vec),
                                               stats), "scsf_solve_batched_hinted", allow)
    evals, evecs = [], []
    e = v = 0
    for o, L in zip(ops, Ls):
        evals.append(ev[e:e + L])
        evecs.append(vec[v:v + o.n * L].view(L, o.n))
        e += L
        v += o.n * L
    return evals, evecs, [st.as_dict() for st in stats]


def make_params(L, k, degree=20, tol=1e-8, max_iter=0, lanczos_steps=20, seed=0,
                precision=SCSF_FP64, schedule=SCSF_SCHED_STATIC, adaptive=0,
                cold_start=0, target=0) -> Params:
    return Params(L=L, k=k, degree=degree, max_iter=max_iter, lanczos_steps=lanczos_steps,
                  precision=precision, schedule=schedule, adaptive=adaptive,
                  cold_start=cold_start, target=target, tol=tol, seed=seed)


def scsf_solve(h: Handle, A: DeviceOperator, prm: Params, X_prev=None, theta_prev=None,
               allow_notconv=False, out=None):
    """Returns (evals[L], evecs n x L, X_next n x k, theta_next[k], stats dict); `out` may
    supply the four output tensors (as returned by an earlier call)."""
    n, L, k = A.n, prm.L, prm.k
    dev = torch.device("cuda")
    if out is not None:
        evals, evecs, X_next, theta_next = out[:4]
        assert evals.numel() == L and evecs.shape == (n, L) and _ld(evecs) == n
        assert X_next.shape == (n, k) and _ld(X_next) == n and theta_next.numel() == k
    else:
        evals = torch.empty(L, device=dev, dtype=torch.float64)
        evecs = colmajor(n, L)
        X_next = colmajor(n, k)
        theta_next = torch.empty(k, device=dev, dtype=torch.float64)
    if X_prev is not None:
        X_prev = as_colmajor(X_prev)
        assert _ld(X_prev) == n
    st = Stats()
    allow = (SCSF_OK, SCSF_ENOTCONV) if allow_notconv else (SCSF_OK,)
    _check(lib().scsf_solve(h.ptr, A.ref(), ctypes.byref(prm), _ptr(X_prev), _ptr(theta_prev),
                            _ptr(evals), _ptr(evecs), _ptr(X_next), _ptr(theta_next),
                            ctypes.byref(st)), "scsf_solve", allow)
    return evals, evecs, X_next, theta_next, st.as_dict()


def scsf_solve_sequence(h: Handle, ops: list, order, chains: int, prm: Params,
                        evals: torch.Tensor | None = None, evecs: torch.Tensor | None = None,
                        allow_notconv=False, hints=None, ritz: torch.Tensor | None = None):
    """Solve every operator in `ops` (DeviceOperator list) in `order`, `chains` chunks.
    Returns (evals n_op x L, evecs n_op x (n x L column-major) tensor, list of stats dicts)."""
    n_op = len(ops)
    n, L = ops[0].n, prm.L
    arr = (Operator * n_op)(*[o.struct for o in ops])
    order = np.asarray(order, dtype=np.int32)
    ordc = (c_int32 * n_op)(*order.tolist())
    if evals is None:
        evals = torch.empty((n_op, L), device="cuda", dtype=torch.float64)
    if evecs is None:
        evecs = torch.empty((n_op, L, n), device="cuda", dtype=torch.float64)
    stats = (Stats * n_op)()
    allow = (SCSF_OK, SCSF_ENOTCONV) if allow_notconv else (SCSF_OK,)
    if hints is None and ritz is None:
        _check(lib().scsf_solve_sequence(h.ptr, arr, n_op, ordc, int(chains), ctypes.byref(prm),
                                         _ptr(evals), _ptr(evecs), stats), "scsf_solve_sequence",
               allow)
    else:
        hp = None
        if hints is not None:
            hv = np.ascontiguousarray(np.asarray(hints, dtype=np.float64).reshape(n_op, 3))
            hp = hv.ctypes.data_as(POINTER(c_double))
        _check(lib().scsf_solve_sequence_hinted(h.ptr, arr, n_op, ordc, int(chains),
                                                ctypes.byref(prm), hp, _ptr(evals), _ptr(evecs),
                                                _ptr(ritz), stats),
               "scsf_solve_sequence_hinted", allow)
    return evals, evecs, [s.as_dict() for s in stats]


def scsf_set_lanes(h: Handle, lanes: int):
    _check(lib().scsf_set_lanes(h.ptr, int(lanes)), "scsf_set_lanes")


def scsf_set_graphs(h: Handle, on: bool = True):
    _check(lib().scsf_set_graphs(h.ptr, 1 if on else 0), "scsf_set_graphs")


def scsf_set_eigensolver(h: Handle, which: int):
    _check(lib().scsf_set_eigensolver(h.ptr, int(which)), "scsf_set_eigensolver")


def scsf_workspace_bytes(prm: Params, n: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().scsf_workspace_bytes(ctypes.byref(prm), int(n), ctypes.byref(out)),
           "scsf_workspace_bytes")
    return int(out.value)


def scsf_workspace_bytes_sequence(h: Handle, prm: Params, n: int, n_op: int, chains: int,
                                  hinted: bool = False) -> int:
    out = ctypes.c_size_t()
    _check(lib().scsf_workspace_bytes_sequence(h.ptr, ctypes.byref(prm), int(n), int(n_op),
                                               int(chains), 1 if hinted else 0,
                                               ctypes.byref(out)),
           "scsf_workspace_bytes_sequence")
    return int(out.value)


def scsf_set_workspace(h: Handle, buf: torch.Tensor | None):
    """Give the handle a caller-owned device workspace (a uint8 tensor kept alive by the
    caller), or return to library-allocated buffers with None."""
    if buf is None:
        _check(lib().scsf_set_workspace(h.ptr, None, 0), "scsf_set_workspace")
    else:
        _check(lib().scsf_set_workspace(h.ptr, ctypes.c_void_p(buf.data_ptr()),
                                        buf.numel() * buf.element_size()), "scsf_set_workspace")


def scsf_workspace_peak(h: Handle) -> int:
    out = ctypes.c_size_t()
    _check(lib().scsf_workspace_peak(h.ptr, ctypes.byref(out)), "scsf_workspace_peak")
    return int(out.value)


def scsf_set_batch_form(h: Handle, form: int):
    """SCSF_BATCH_GROUPED (per-(L, k) batches) or SCSF_BATCH_ONE_SWEEP (one batch per kind)."""
    _check(lib().scsf_set_batch_form(h.ptr, int(form)), "scsf_set_batch_form")


def scsf_set_fused_steps(h: Handle, steps: int):
    """Chebyshev steps per fused filter launch (2, 3, 4; 0 = one step per launch)."""
    _check(lib().scsf_set_fused_steps(h.ptr, int(steps)), "scsf_set_fused_steps")


def scsf_profile_enable(h: Handle, on: bool = True):
    _check(lib().scsf_profile_enable(h.ptr, 1 if on else 0), "scsf_profile_enable")


def scsf_profile_read(h: Handle, reset: bool = False) -> dict:
    p = Profile()
    _check(lib().scsf_profile_read(h.ptr, ctypes.byref(p), 1 if reset else 0), "scsf_profile_read")
    return {"filter_launches": p.filter_launches, "filter_ms": p.filter_ms,
            "filter_bytes": p.filter_bytes,
            "phase_ms": dict(zip(PHASES, list(p.phase_ms)))}


# ----------------------------------------------------------------- spectral-window network
def window_param_count() -> int:
    return int(lib().scsf_window_param_count())


def scsf_window_init(h: Handle, seed: int = 0) -> torch.Tensor:
    p = torch.empty(window_param_count(), device="cuda", dtype=torch.float32)
    _check(lib().scsf_window_init(h.ptr, _ptr(p), c_uint64(seed)), "scsf_window_init")
    return p


def scsf_window_input(h: Handle, feats: torch.Tensor) -> torch.Tensor:
    """feats: (n, 3, 16, 16) complex128 device tensor -> (n, 6, 16, 16) float32."""
    n, C, p0, _ = feats.shape
    fr = torch.view_as_real(feats.contiguous())
    x = torch.empty((n, 2 * C, p0, p0), device=feats.device, dtype=torch.float32)
    _check(lib().scsf_window_input(h.ptr, _ptr(fr), n, C, p0, _ptr(x)), "scsf_window_input")
    return x


def scsf_window_forward(h: Handle, params: torch.Tensor, x: torch.Tensor, bf16=False):
    n = x.shape[0]
    out = torch.empty((n, 3), device=x.device, dtype=torch.float32)
    _check(lib().scsf_window_forward(h.ptr, _ptr(params), _ptr(x.contiguous()), n,
                                     1 if bf16 else 0, _ptr(out)), "scsf_window_forward")
    return out


def scsf_window_loss_grad(h: Handle, params, x, target):
    grad = torch.empty_like(params)
    loss = c_double()
    _check(lib().scsf_window_loss_grad(h.ptr, _ptr(params), _ptr(x.contiguous()),
                                       _ptr(target.contiguous()), x.shape[0], _ptr(grad),
                                       ctypes.byref(loss)), "scsf_window_loss_grad")
    return loss.value, grad


def scsf_window_train(h: Handle, params, x, target, epochs: int, lr: float):
    hist = (c_double * epochs)()
    _check(lib().scsf_window_train(h.ptr, _ptr(params), _ptr(x.contiguous()),
                                   _ptr(target.contiguous()), x.shape[0], int(epochs),
                                   ctypes.c_float(lr), hist), "scsf_window_train")
    return np.frombuffer(hist, dtype=np.float64).copy()


def scsf_window_labels(h: Handle, ritz: torch.Tensor, L: int, beta: torch.Tensor):
    n, k = ritz.shape
    t = torch.empty((n, 3), device=ritz.device, dtype=torch.float32)
    _check(lib().scsf_window_labels(h.ptr, _ptr(ritz.contiguous()), n, k, L,
                                    _ptr(beta.contiguous()), _ptr(t)), "scsf_window_labels")
    return t


def scsf_window_hints(h: Handle, out: torch.Tensor) -> torch.Tensor:
    n = out.shape[0]
    hints = torch.empty((n, 3), device=out.device, dtype=torch.float64)
    _check(lib().scsf_window_hints(h.ptr, _ptr(out.contiguous()), n, _ptr(hints)),
           "scsf_window_hints")
    return hints


def version() -> str:
    return lib().scsf_version().decode()
