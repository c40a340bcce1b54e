"""ctypes wrapper of the FP64 sequential GenCD oracle (oracle/gencd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, by the package smoke check and by
the CPU-baseline leg of the benchmark, never by the product path.  It shares
no code with the HIP library.

All floating-point arguments are promoted to float64 here; matrices are the
CSC triple (col_ptr int64, row_idx int32, val) of the synthetic generators.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

SQUARED, LOGISTIC = 0, 1
CYCLIC, STOCHASTIC, SHOTGUN, THREAD_GREEDY, GREEDY, COLORING, TOP_GREEDY, BLOCK_SHOTGUN = range(8)
OK, NOT_CONVERGED = 0, 1


class _Csc(C.Structure):
    _fields_ = [("n", C.c_int64), ("k", C.c_int64), ("nnz", C.c_int64),
                ("col_ptr", C.c_void_p), ("row_idx", C.c_void_p), ("val", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("loss", C.c_int32), ("rule", C.c_int32), ("lam", C.c_double),
                ("select_size", C.c_int64), ("block", C.c_int64), ("seed", C.c_uint64),
                ("tol", C.c_double), ("max_epochs", C.c_int64), ("check_every", C.c_int64),
                ("color", C.c_void_p), ("num_colors", C.c_int32), ("improve", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("iters", C.c_int64), ("epochs", C.c_int64), ("coord_updates", C.c_int64),
                ("nnz_updates", C.c_int64), ("objective", C.c_double), ("kkt_max", C.c_double),
                ("nnz_w", C.c_int64), ("converged", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("GENCD_ORACLE_LIB") or _build.LIB
        if path == _build.LIB and (not os.path.exists(path)
                                   or os.path.getmtime(path) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = C.CDLL(path)
        P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int, C.c_double
        L.orc_loss.restype = D
        L.orc_loss.argtypes = [I32, D, D]
        L.orc_dloss.restype = D
        L.orc_dloss.argtypes = [I32, D, D]
        L.orc_mix64.restype = C.c_uint64
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_perm.restype = I64
        L.orc_perm.argtypes = [I64, C.c_uint64, I64, I64]
        L.orc_curvature.restype = None
        L.orc_curvature.argtypes = [P, I32, P]
        L.orc_lambda_max.restype = D
        L.orc_lambda_max.argtypes = [P, P, I32]
        L.orc_propose.restype = None
        L.orc_propose.argtypes = [D, D, D, D, P, P]
        L.orc_step.restype = I32
        L.orc_step.argtypes = [P, P, I32, D, P, P, I64, I64, I64, I32, P, P, P, P, P, P, P, P]
        L.orc_check.restype = None
        L.orc_check.argtypes = [P, P, I32, D, P, P, P, P, P, P]
        L.orc_duality_gap.restype = D
        L.orc_duality_gap.argtypes = [P, P, I32, D, P, P]
        L.orc_color.restype = I32
        L.orc_rho.restype = D
        L.orc_rho.argtypes = [P, I32, P, P]
        L.orc_pstar.restype = I64
        L.orc_pstar.argtypes = [I64, D, I64]
        L.orc_block_base.restype = I64
        L.orc_block_base.argtypes = [P, C.c_uint64, P]
        L.orc_block_pstar.argtypes = [P, C.c_uint64, I64, I32, P, P]
        L.orc_balance_colors.restype = I32
        L.orc_balance_colors.argtypes = [I64, P, P, I32, I64, P]
        L.orc_color.argtypes = [I64, I64, P, P, I32, P, P, P]
        L.orc_solve.restype = I32
        L.orc_solve.argtypes = [P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class Matrix:
    """Holds float64 copies of a CSC matrix for the oracle."""

    def __init__(self, n, k, col_ptr, row_idx, val):
        self.n, self.k = int(n), int(k)
        self.col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int64)
        self.row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self._s = _Csc(self.n, self.k, int(self.col_ptr[-1]), _p(self.col_ptr).value,
                       _p(self.row_idx).value, _p(self.val).value)

    @classmethod
    def of(cls, prob):
        return cls(prob.n, prob.k, prob.col_ptr, prob.row_idx, prob.val)

    @property
    def ref(self):
        return C.byref(self._s)

    def dense(self):
        A = np.zeros((self.n, self.k))
        for j in range(self.k):
            a, b = self.col_ptr[j], self.col_ptr[j + 1]
            A[self.row_idx[a:b], j] = self.val[a:b]
        return A


def loss(kind, y, t):
    return lib().orc_loss(kind, float(y), float(t))


def dloss(kind, y, t):
    return lib().orc_dloss(kind, float(y), float(t))


def mix64(x):
    return int(lib().orc_mix64(C.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def perm(m, seed, epoch):
    L = lib()
    return np.array([L.orc_perm(m, C.c_uint64(seed), epoch, p) for p in range(m)], dtype=np.int64)


def curvature(X: Matrix, kind):
    c = np.zeros(X.k)
    lib().orc_curvature(X.ref, kind, _p(c))
    return c


def lambda_max(X: Matrix, y, kind):
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().orc_lambda_max(X.ref, _p(y), kind)


def propose(g, c, w, lam):
    d, p = C.c_double(), C.c_double()
    lib().orc_propose(float(g), float(c), float(w), float(lam), C.byref(d), C.byref(p))
    return d.value, p.value


@dataclass
class StepResult:
    g: np.ndarray
    delta: np.ndarray
    phi: np.ndarray
    accepted: np.ndarray
    nnz_updates: int


def step(X: Matrix, y, kind, lam, J, w, z, block=0, forced=None, c=None, top=0, improve=0):
    """One Jacobi iteration on J; w and z (float64) are updated in place.
    top > 0 accepts the `top` best proposals of the window (forced: the
    accepted positions instead); block > 0 the best of each block."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    J = np.ascontiguousarray(J, dtype=np.int32)
    if c is None:
        c = curvature(X, kind)
    m = J.size
    g, d, ph = np.zeros(m), np.zeros(m), np.zeros(m)
    acc = np.zeros(m, dtype=np.int32)
    f = None if forced is None else np.ascontiguousarray(forced, dtype=np.int32)
    nu = C.c_int64()
    assert w.dtype == np.float64 and z.dtype == np.float64
    st = lib().orc_step(X.ref, _p(y), kind, float(lam), _p(c), _p(J), m, int(block), int(top),
                        int(improve), _p(f),
                        _p(w), _p(z), _p(g), _p(d), _p(ph), _p(acc), C.byref(nu))
    if st != 0:
        raise ValueError(f"orc_step failed: {st}")
    return StepResult(g, d, ph, acc, nu.value)


@dataclass
class Check:
    z: np.ndarray
    g: np.ndarray
    kkt: float
    objective: float
    nnz_w: int


def check(X: Matrix, y, kind, lam, w):
    y = np.ascontiguousarray(y, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    z, g = np.zeros(X.n), np.zeros(X.k)
    kkt, obj, nz = C.c_double(), C.c_double(), C.c_int64()
    lib().orc_check(X.ref, _p(y), kind, float(lam), _p(w), _p(z), _p(g), C.byref(kkt),
                    C.byref(obj), C.byref(nz))
    return Check(z, g, kkt.value, obj.value, nz.value)


def duality_gap(X: Matrix, y, kind, lam, w):
    """(gap, primal) at w: P(w) - D(u) for the scaled-residual dual point."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    prim = C.c_double()
    gap = lib().orc_duality_gap(X.ref, _p(y), kind, float(lam), _p(w), C.byref(prim))
    return gap, prim.value


def rho(X: Matrix, iters=20):
    """(rho, history, k_live): power-iteration estimate of the spectral radius
    of the column-normalised Gram matrix (section 4.1)."""
    hist = np.zeros(max(int(iters), 1), dtype=np.float64)
    kl = C.c_int64()
    r = lib().orc_rho(X.ref, int(iters), _p(hist), C.byref(kl))
    return r, hist[:int(iters)], kl.value


def pstar(k_live, rho_est, cap=None):
    """Selection size floor(k_live / (2 rho)) clamped to [1, cap] (cap: k_live)."""
    cap = int(k_live) if cap is None else int(cap)
    return int(lib().orc_pstar(int(k_live), float(rho_est), max(cap, 1)))


def block_base(X: Matrix, seed):
    """Preset order of the non-empty columns; block b is the range
    [b k_live / nb, (b+1) k_live / nb) of it."""
    out = np.zeros(max(X.k, 1), dtype=np.int32)
    kl = lib().orc_block_base(X.ref, C.c_uint64(seed).value, _p(out))
    return out[:kl]


def block_pstar(X: Matrix, seed, nb, iters=20):
    """(rho_b, P_b*) of every preset block."""
    rho = np.zeros(nb)
    ps = np.zeros(nb, dtype=np.int64)
    st = lib().orc_block_pstar(X.ref, C.c_uint64(seed).value, int(nb), int(iters), _p(rho), _p(ps))
    if st != 0:
        raise ValueError(f"orc_block_pstar failed: {st}")
    return rho, ps


def balance_colors(k, col_ptr, color, num_colors, cap=0):
    """Split every class above `cap` live columns into near-equal parts
    (members in column order); returns (new colours, number of colours)."""
    col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int64)
    color = np.ascontiguousarray(color, dtype=np.int32)
    out = np.zeros(k, dtype=np.int32)
    nc = lib().orc_balance_colors(int(k), _p(col_ptr), _p(color), int(num_colors), int(cap), _p(out))
    return out, int(nc)


def color(n, k, col_ptr, row_idx, order_mode=0):
    col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int64)
    row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
    out = np.zeros(k, dtype=np.int32)
    order = np.zeros(k, dtype=np.int32)
    nc = C.c_int32()
    st = lib().orc_color(int(n), int(k), _p(col_ptr), _p(row_idx), int(order_mode), _p(out),
                         C.byref(nc), _p(order))
    if st != 0:
        raise ValueError(f"orc_color failed: {st}")
    return out, nc.value, order


@dataclass
class SolveResult:
    status: int
    w: np.ndarray
    z: np.ndarray
    iters: int
    epochs: int
    coord_updates: int
    nnz_updates: int
    objective: float
    kkt: float
    nnz_w: int
    converged: bool


def solve(X: Matrix, y, kind, lam, rule, select_size=1, block=1, seed=0, tol=1e-6,
          max_epochs=1000, check_every=1, colors=None, w0=None, improve=0):
    y = np.ascontiguousarray(y, dtype=np.float64)
    w = np.zeros(X.k) if w0 is None else np.array(w0, dtype=np.float64)
    z = np.zeros(X.n)
    col = None
    nc = 0
    if colors is not None:
        col = np.ascontiguousarray(colors, dtype=np.int32)
        nc = int(col.max()) + 1 if col.size else 0
    prm = _Params(kind, rule, float(lam), int(select_size), int(block), C.c_uint64(seed).value,
                  float(tol), int(max_epochs), int(check_every),
                  _p(col).value if col is not None else None, nc, int(improve))
    st = _Stats()
    rc = lib().orc_solve(X.ref, _p(y), C.byref(prm), _p(w), _p(z), C.byref(st))
    if rc < 0:
        raise ValueError(f"orc_solve failed: {rc}")
    return SolveResult(rc, w, z, st.iters, st.epochs, st.coord_updates, st.nnz_updates,
                       st.objective, st.kkt_max, st.nnz_w, bool(st.converged))
