"""Python binding of libgencd (include/gencd.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Tensors are torch tensors on the current HIP device; the work is enqueued on
torch's current stream.  If the library has not been built this module raises
on first use; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgencd.so")

OK, NOT_CONVERGED = 0, 1
ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_TOO_LARGE = -1, -5, -9
SQUARED, LOGISTIC = 0, 1
CYCLIC, STOCHASTIC, SHOTGUN, THREAD_GREEDY, GREEDY, COLORING, TOP_GREEDY, BLOCK_SHOTGUN = range(8)
WARM_START, VALIDATE_DEVICE, USE_GRAPH, PROFILE, EXACT_ACCUM, FUSED = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
FUSED_EPOCH = 0x40
RULES = {"cyclic": CYCLIC, "stochastic": STOCHASTIC, "shotgun": SHOTGUN,
         "thread_greedy": THREAD_GREEDY, "greedy": GREEDY, "coloring": COLORING,
         "top_greedy": TOP_GREEDY, "block_shotgun": BLOCK_SHOTGUN}


class GencdError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


class Csc(C.Structure):
    _fields_ = [("n", C.c_int64), ("k", C.c_int64), ("nnz", C.c_int64),
                ("col_ptr", C.c_void_p), ("row_idx", C.c_void_p), ("val", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("loss", C.c_int32), ("rule", C.c_int32), ("lam", C.c_double),
                ("select_size", C.c_int64), ("block", C.c_int64), ("seed", C.c_uint64),
                ("kkt_tol", C.c_double), ("gap_tol", C.c_double), ("max_epochs", C.c_int64),
                ("check_every", C.c_int64),
                ("flags", C.c_uint32), ("color", C.c_void_p), ("num_colors", C.c_int32),
                ("piece", C.c_int32), ("group", C.c_int32), ("improve_steps", C.c_int32),
                ("residual", C.c_int32), ("stagger", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int64), ("epochs", C.c_int64), ("coord_updates", C.c_int64),
                ("nnz_visits", C.c_int64), ("nnz_updates", C.c_int64), ("objective", C.c_double),
                ("kkt_max", C.c_double), ("gap", C.c_double), ("lambda_max", C.c_double),
                ("seconds", C.c_double),
                ("nnz_w", C.c_int64), ("converged", C.c_int32), ("num_colors", C.c_int32),
                ("prof_launches", C.c_int64), ("prof_kernel_ms", C.c_double),
                ("prof_bytes", C.c_double), ("rho", C.c_double), ("select_size", C.c_int64),
                ("prof_update_launches", C.c_int64), ("prof_update_ms", C.c_double),
                ("prof_update_bytes", C.c_double), ("nnz_scattered", C.c_int64),
                ("z_drift", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

_SIGS = {
    "gencd_status_string": (C.c_char_p, [C.c_int]),
    "gencd_workspace_bytes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gencd_lambda_max": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_size_t, C.c_void_p]),
    "gencd_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "gencd_solve_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p]),
    "gencd_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "gencd_check": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                              C.c_void_p]),
    "gencd_select_perm": (C.c_int, [C.c_int64, C.c_uint64, C.c_int64, C.c_void_p, C.c_void_p]),
    "gencd_rho_workspace_bytes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gencd_autotune_path": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                      C.c_char_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                      C.c_void_p]),
    "gencd_balance_workspace_bytes": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "gencd_balance_colors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "gencd_block_rho_workspace_bytes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "gencd_estimate_block_rho": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "gencd_estimate_rho": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "gencd_color_workspace_bytes": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gencd_path_workspace_bytes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "gencd_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_char_p,
                                 C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "gencd_server_create": (C.c_int, [C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p, C.c_void_p]),
    "gencd_gen_workspace_bytes": (C.c_int, [C.c_int64, C.c_int64, C.c_void_p]),
    "gencd_gen_count": (C.c_int, [C.c_int64, C.c_int64, C.c_double, C.c_uint64, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "gencd_gen_fill": (C.c_int, [C.c_int64, C.c_int64, C.c_double, C.c_uint64, C.c_int32, C.c_int32,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_size_t, C.c_void_p]),
    "gencd_server_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gencd_server_request_bytes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gencd_server_overhead_bytes": (C.c_size_t, [C.c_int32]),
    "gencd_server_poll": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "gencd_server_info": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gencd_server_destroy": (C.c_int, [C.c_void_p]),
    "gencd_server_plan": (C.c_int, [C.c_size_t, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "gencd_solve_path": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                   C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                   C.c_void_p, C.c_void_p]),
    "gencd_color": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                              C.c_void_p]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1206_6409_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def status_string(status):
    return lib().gencd_status_string(int(status)).decode()


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(status, where, allow=(OK,)):
    if status not in allow:
        raise GencdError(status, where)
    return status


@dataclass
class Matrix:
    """A CSC matrix on the device (int64 col_ptr, int32 row_idx, float32 val)."""
    n: int
    k: int
    col_ptr: torch.Tensor
    row_idx: torch.Tensor
    val: torch.Tensor
    _s: Csc = field(default=None, repr=False)

    def __post_init__(self):
        assert self.col_ptr.dtype == torch.int64 and self.row_idx.dtype == torch.int32
        assert self.val.dtype == torch.float32
        self._s = Csc(int(self.n), int(self.k), int(self.row_idx.numel()),
                      self.col_ptr.data_ptr(), self.row_idx.data_ptr() if self.row_idx.numel() else None,
                      self.val.data_ptr() if self.val.numel() else None)

    @property
    def nnz(self):
        return int(self.row_idx.numel())

    @property
    def ref(self):
        return C.byref(self._s)

    @classmethod
    def from_numpy(cls, n, k, col_ptr, row_idx, val, device="cuda"):
        return cls(int(n), int(k), torch.as_tensor(col_ptr, dtype=torch.int64).to(device),
                   torch.as_tensor(row_idx, dtype=torch.int32).to(device),
                   torch.as_tensor(val, dtype=torch.float32).to(device))

    @classmethod
    def of(cls, prob, device="cuda"):
        return cls.from_numpy(prob.n, prob.k, prob.col_ptr, prob.row_idx, prob.val, device)


def make_params(loss, lam, rule=SHOTGUN, select_size=1, block=1, seed=0, tol=1e-6,
                gap_tol=0.0, max_epochs=1000, check_every=1, flags=0, colors=None,
                num_colors=0, piece=0, group=0, improve=0, residual=0, stagger=0):
    if isinstance(rule, str):
        rule = RULES[rule]
    return Params(int(loss), int(rule), float(lam), int(select_size), int(block),
                  C.c_uint64(seed).value, float(tol), float(gap_tol), int(max_epochs),
                  int(check_every),
                  int(flags), colors.data_ptr() if colors is not None else None, int(num_colors),
                  int(piece), int(group), int(improve), int(residual), int(stagger))


def workspace_bytes(X: Matrix, params: Params = None):
    out = C.c_size_t()
    _check(lib().gencd_workspace_bytes(X.ref, C.byref(params) if params is not None else None,
                                       C.byref(out)), "gencd_workspace_bytes")
    return out.value


def workspace(X: Matrix, params: Params = None, device=None):
    nbytes = workspace_bytes(X, params)
    dev = device if device is not None else X.col_ptr.device
    return torch.empty(nbytes, dtype=torch.uint8, device=dev)


def lambda_max(X: Matrix, y: torch.Tensor, loss, ws=None):
    ws = workspace(X) if ws is None else ws
    out = C.c_double()
    _check(lib().gencd_lambda_max(X.ref, _ptr(y), int(loss), C.byref(out), _ptr(ws), ws.numel(),
                                  _stream()), "gencd_lambda_max")
    return out.value


@dataclass
class RhoResult:
    rho: float            # estimate after the last iteration
    history: list         # estimate after each iteration
    k_live: int
    select_size: int      # floor(k_live / (2 rho)) clamped to [1, k_live]


def estimate_rho(X: Matrix, iters=20, params=None):
    """Power-iteration estimate of the largest eigenvalue of the
    column-normalised Gram matrix (section 4.1's P* = k / (2 rho))."""
    pp = C.byref(params) if params is not None else None
    nb = C.c_size_t()
    _check(lib().gencd_rho_workspace_bytes(X.ref, pp, C.byref(nb)), "gencd_rho_workspace_bytes")
    ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=X.col_ptr.device)
    hist = (C.c_double * int(iters))()
    kl, sel = C.c_int64(), C.c_int64()
    _check(lib().gencd_estimate_rho(X.ref, pp, int(iters), hist, C.byref(kl), C.byref(sel),
                                    _ptr(ws), ws.numel(), _stream()), "gencd_estimate_rho")
    h = list(hist)
    return RhoResult(h[-1], h, kl.value, sel.value)


def balance_colors(X: Matrix, colors: torch.Tensor, num_colors, cap=0):
    """Split every colour class above `cap` live columns into near-equal
    parts (column order); returns (colours, number of colours)."""
    nb = C.c_size_t()
    _check(lib().gencd_balance_workspace_bytes(X.ref, int(num_colors), C.byref(nb)),
           "gencd_balance_workspace_bytes")
    ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=X.col_ptr.device)
    out = torch.empty(X.k, dtype=torch.int32, device=X.col_ptr.device)
    nc = C.c_int32()
    _check(lib().gencd_balance_colors(X.ref, _ptr(colors), int(num_colors), int(cap), _ptr(out),
                                      C.byref(nc), _ptr(ws), ws.numel(), _stream()),
           "gencd_balance_colors")
    return out, nc.value


def estimate_block_rho(X: Matrix, num_blocks, iters=20, params=None):
    """(rho_b, P_b*) of the preset blocks of Block Shotgun (section 7)."""
    pp = C.byref(params) if params is not None else None
    nb = C.c_size_t()
    _check(lib().gencd_block_rho_workspace_bytes(X.ref, pp, int(num_blocks), C.byref(nb)),
           "gencd_block_rho_workspace_bytes")
    ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=X.col_ptr.device)
    rho = (C.c_double * int(num_blocks))()
    ps = (C.c_int64 * int(num_blocks))()
    _check(lib().gencd_estimate_block_rho(X.ref, pp, int(num_blocks), int(iters), rho, ps, _ptr(ws),
                                          ws.numel(), _stream()), "gencd_estimate_block_rho")
    return list(rho), list(ps)


@dataclass
class SolveResult:
    status: int
    w: torch.Tensor
    z: torch.Tensor
    stats: dict


def solve(X: Matrix, y: torch.Tensor, params: Params, w0=None, ws=None, want_z=True):
    ws = workspace(X, params) if ws is None else ws
    if w0 is not None:
        w = w0.clone().to(torch.float32)
        params.flags |= WARM_START
    else:
        w = torch.empty(X.k, dtype=torch.float32, device=X.col_ptr.device)
    z = torch.empty(X.n, dtype=torch.float32, device=X.col_ptr.device) if want_z else None
    st = Stats()
    rc = lib().gencd_solve(X.ref, _ptr(y), C.byref(params), _ptr(w), _ptr(z), _ptr(ws),
                           ws.numel(), _stream(), C.byref(st))
    _check(rc, "gencd_solve", allow=(OK, NOT_CONVERGED))
    return SolveResult(rc, w, z, st.as_dict())


def solve_noalloc(X: Matrix, y: torch.Tensor, params: Params, w0=None, want_z=True):
    """gencd_solve with the library's static device scratch as workspace (no
    device allocation inside the call; w and z are the caller's outputs)."""
    if w0 is not None:
        w = w0.clone().to(torch.float32)
        params.flags |= WARM_START
    else:
        w = torch.empty(X.k, dtype=torch.float32, device=X.col_ptr.device)
    z = torch.empty(X.n, dtype=torch.float32, device=X.col_ptr.device) if want_z else None
    st = Stats()
    rc = lib().gencd_solve_noalloc(X.ref, _ptr(y), C.byref(params), _ptr(w), _ptr(z), _stream(),
                                   C.byref(st))
    _check(rc, "gencd_solve_noalloc", allow=(OK, NOT_CONVERGED))
    return SolveResult(rc, w, z, st.as_dict())


@dataclass
class StepResult:
    g: torch.Tensor
    delta: torch.Tensor
    phi: torch.Tensor
    accepted: torch.Tensor


def step(X: Matrix, y, params: Params, J: torch.Tensor, w, z_hi, z_lo, ws=None):
    """One iteration on J; w, z_hi, z_lo (float32 device tensors) are updated in place."""
    ws = workspace(X, params) if ws is None else ws
    m = J.numel()
    dev = X.col_ptr.device
    g = torch.empty(m, dtype=torch.float32, device=dev)
    d = torch.empty(m, dtype=torch.float32, device=dev)
    ph = torch.empty(m, dtype=torch.float32, device=dev)
    acc = torch.empty(m, dtype=torch.int32, device=dev)
    rc = lib().gencd_step(X.ref, _ptr(y), C.byref(params), _ptr(J), m, _ptr(w), _ptr(z_hi),
                          _ptr(z_lo), _ptr(g), _ptr(d), _ptr(ph), _ptr(acc), _ptr(ws), ws.numel(),
                          _stream())
    _check(rc, "gencd_step")
    return StepResult(g, d, ph, acc)


@dataclass
class CheckResult:
    objective: float
    kkt: float
    nnz_w: int
    z64: torch.Tensor
    g64: torch.Tensor
    gap: float = 0.0


def check(X: Matrix, y, loss, lam, w, ws=None):
    ws = workspace(X) if ws is None else ws
    dev = X.col_ptr.device
    z64 = torch.empty(X.n, dtype=torch.float64, device=dev)
    g64 = torch.empty(X.k, dtype=torch.float64, device=dev)
    st = Stats()
    rc = lib().gencd_check(X.ref, _ptr(y), int(loss), float(lam), _ptr(w), _ptr(z64), _ptr(g64),
                           C.byref(st), _ptr(ws), ws.numel(), _stream())
    _check(rc, "gencd_check")
    return CheckResult(st.objective, st.kkt_max, st.nnz_w, z64, g64, st.gap)


def select_perm(m, seed, epoch, device="cuda"):
    out = torch.empty(max(m, 1), dtype=torch.int32, device=device)
    _check(lib().gencd_select_perm(int(m), C.c_uint64(seed).value, int(epoch), _ptr(out),
                                   _stream()), "gencd_select_perm")
    return out[:m]


def color(X: Matrix, ws=None):
    """Greedy partial distance-2 colouring of the columns: (int32[k] colours, count)."""
    if ws is None:
        nb = C.c_size_t()
        _check(lib().gencd_color_workspace_bytes(X.ref, C.byref(nb)), "gencd_color_workspace_bytes")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=X.col_ptr.device)
    out = torch.empty(X.k, dtype=torch.int32, device=X.col_ptr.device)
    nc = C.c_int32()
    _check(lib().gencd_color(X.ref, _ptr(out), C.byref(nc), _ptr(ws), ws.numel(), _stream()),
           "gencd_color")
    return out, nc.value


@dataclass
class PathResult:
    status: int
    W: torch.Tensor      # [L, k]
    stats: list
    Z: torch.Tensor = None  # [L, n] fitted values X W[t] (want_z)


def solve_path(X: Matrix, y, params: Params, lambdas, B=32, ws=None, want_z=False):
    """Batched regularisation path (B lambda slots per launch sequence)."""
    import numpy as _np
    lam = _np.ascontiguousarray(_np.asarray(lambdas, dtype=_np.float64))
    L = int(lam.size)
    if ws is None:
        nb = C.c_size_t()
        _check(lib().gencd_path_workspace_bytes(X.ref, C.byref(params), int(B), C.byref(nb)),
               "gencd_path_workspace_bytes")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=X.col_ptr.device)
    W = torch.empty((L, X.k), dtype=torch.float32, device=X.col_ptr.device)
    Z = torch.empty((L, X.n), dtype=torch.float32, device=X.col_ptr.device) if want_z else None
    st = (Stats * L)()
    rc = lib().gencd_solve_path(X.ref, _ptr(y), C.byref(params),
                                lam.ctypes.data_as(C.c_void_p), L, int(B), _ptr(W), _ptr(Z),
                                _ptr(ws), ws.numel(), _stream(), st)
    _check(rc, "gencd_solve_path", allow=(OK, NOT_CONVERGED))
    return PathResult(rc, W, [s.as_dict() for s in st], Z)


class Request(C.Structure):
    _fields_ = [("X", Csc), ("y", C.c_void_p), ("params", Params), ("w", C.c_void_p),
                ("z", C.c_void_p), ("user_tag", C.c_int64)]


class Result(C.Structure):
    _fields_ = [("ticket", C.c_int64), ("user_tag", C.c_int64), ("status", C.c_int32),
                ("stats", Stats), ("submit_s", C.c_double), ("start_s", C.c_double),
                ("finish_s", C.c_double)]

    def as_dict(self):
        return {"ticket": self.ticket, "user_tag": self.user_tag, "status": self.status,
                "stats": self.stats.as_dict(), "submit_s": self.submit_s,
                "start_s": self.start_s, "finish_s": self.finish_s}


class ServerStatus(C.Structure):
    _fields_ = [("running", C.c_int32), ("waiting", C.c_int32), ("finished_unpolled", C.c_int32),
                ("arena_used", C.c_size_t), ("arena_bytes", C.c_size_t),
                ("rounds", C.c_int64), ("slot_rounds", C.c_int64), ("shared_rounds", C.c_int64)]


class Server:
    """Continuous-batching solve server over a torch-owned device arena; its
    rounds run on `stream` (a new torch stream of default priority when
    None)."""

    def __init__(self, arena_bytes, max_slots=8, device=None, stream=None):
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self._h = C.c_void_p()
        self._keep = {}
        torch.cuda.current_stream(dev).synchronize()  # the arena and inputs exist before rounds
        _check(lib().gencd_server_create(_ptr(self.arena), self.arena.numel(), int(max_slots),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(self._h)),
               "gencd_server_create")

    @staticmethod
    def request_bytes(X: Matrix, params: Params):
        """Arena bytes the request holds while admitted."""
        out = C.c_size_t()
        _check(lib().gencd_server_request_bytes(X.ref, C.byref(params), C.byref(out)),
               "gencd_server_request_bytes")
        return out.value

    @staticmethod
    def overhead_bytes(max_slots):
        """Fixed arena bytes of the server's work tables."""
        return int(lib().gencd_server_overhead_bytes(int(max_slots)))

    def submit(self, X: Matrix, y, params: Params, w, z=None, tag=0):
        """Non-blocking; X, y, w (and z) must stay alive until the result is
        polled.  Work on torch's current stream that produced them must be
        complete (the server's streams do not wait for it)."""
        req = Request(X._s, y.data_ptr(), params, w.data_ptr(),
                      z.data_ptr() if z is not None else None, int(tag))
        t = C.c_int64()
        _check(lib().gencd_server_submit(self._h, C.byref(req), C.byref(t)), "gencd_server_submit")
        self._keep[t.value] = (X, y, w, z)
        return t.value

    def poll(self, max_results=1024, wait_for=0):
        buf = (Result * max(1, max_results))()
        n = C.c_int32()
        _check(lib().gencd_server_poll(self._h, buf, int(max_results), int(wait_for), C.byref(n)),
               "gencd_server_poll")
        out = [buf[i].as_dict() for i in range(n.value)]
        for r in out:
            self._keep.pop(r["ticket"], None)
        return out

    def info(self):
        """running, waiting, finished_unpolled, arena_used, arena_bytes, rounds
        (Propose/Update launch pairs), slot_rounds (sum of the requests each
        round advanced) and shared_rounds (rounds advancing two or more)."""
        s = ServerStatus()
        _check(lib().gencd_server_info(self._h, C.byref(s)), "gencd_server_info")
        return {f: getattr(s, f) for f, _ in s._fields_}

    def close(self):
        if self._h:
            lib().gencd_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def generate_request(n, k, density, loss, seed, support=50, device=None):
    """A synthetic serving request generated on the device (Bernoulli(density)
    pattern, N(0, 1) values, labels from a `support`-sparse ground truth):
    (Matrix, y).  Runs on torch's current stream."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    nb = C.c_size_t()
    _check(lib().gencd_gen_workspace_bytes(int(n), int(k), C.byref(nb)), "gencd_gen_workspace_bytes")
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    col_ptr = torch.empty(int(k) + 1, dtype=torch.int64, device=dev)
    nnz = C.c_int64()
    _check(lib().gencd_gen_count(int(n), int(k), float(density), C.c_uint64(seed).value,
                                 _ptr(col_ptr), C.byref(nnz), _ptr(ws), ws.numel(), _stream()),
           "gencd_gen_count")
    row_idx = torch.empty(max(int(nnz.value), 1), dtype=torch.int32, device=dev)[:int(nnz.value)]
    val = torch.empty(max(int(nnz.value), 1), dtype=torch.float32, device=dev)[:int(nnz.value)]
    y = torch.empty(int(n), dtype=torch.float32, device=dev)
    _check(lib().gencd_gen_fill(int(n), int(k), float(density), C.c_uint64(seed).value, int(loss),
                                int(support), _ptr(col_ptr), _ptr(row_idx) if nnz.value else None,
                                _ptr(val) if nnz.value else None, _ptr(y), _ptr(ws), ws.numel(),
                                _stream()), "gencd_gen_fill")
    return Matrix(int(n), int(k), col_ptr, row_idx, val), y


def server_plan(arena_bytes, max_slots, bytes_, arrival, service):
    """Start times under the server's admission policy (host-only replay)."""
    import numpy as _np
    b = _np.ascontiguousarray(bytes_, dtype=_np.uint64)
    a = _np.ascontiguousarray(arrival, dtype=_np.float64)
    sv = _np.ascontiguousarray(service, dtype=_np.float64)
    out = _np.zeros(b.size, dtype=_np.float64)
    _check(lib().gencd_server_plan(int(arena_bytes), int(max_slots), int(b.size),
                                   b.ctypes.data_as(C.c_void_p), a.ctypes.data_as(C.c_void_p),
                                   sv.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p)),
           "gencd_server_plan")
    return out


class Schedule(C.Structure):
    _fields_ = [("group", C.c_int32), ("piece", C.c_int32), ("flags", C.c_uint32),
                ("seconds_per_epoch", C.c_double), ("from_cache", C.c_int32),
                ("residual", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def autotune(X: Matrix, y, params: Params, epochs=2, cache_path=None):
    """Fastest (group, piece, graph, residual) schedule for this problem; apply with
    apply_schedule."""
    # the candidate needing the most workspace: smallest pieces and groups
    pmax = Params.from_buffer_copy(params)
    pmax.piece, pmax.group = 128, 4
    ws = workspace(X, pmax)
    w = torch.empty(X.k, dtype=torch.float32, device=X.col_ptr.device)
    out = Schedule()
    _check(lib().gencd_autotune(X.ref, _ptr(y), C.byref(params), int(epochs),
                                cache_path.encode() if cache_path else None, _ptr(w), _ptr(ws),
                                ws.numel(), _stream(), C.byref(out)), "gencd_autotune")
    return out.as_dict()


class PathSchedule(C.Structure):
    _fields_ = [("B", C.c_int32), ("flags", C.c_uint32), ("seconds", C.c_double),
                ("from_cache", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def autotune_path(X: Matrix, y, params: Params, lambdas, cache_path=None):
    """Fastest (B, fused or not) for gencd_solve_path on these lambdas."""
    import numpy as _np
    lam = _np.ascontiguousarray(_np.asarray(lambdas, dtype=_np.float64))
    nb = C.c_size_t()
    _check(lib().gencd_path_workspace_bytes(X.ref, C.byref(params), 64, C.byref(nb)),
           "gencd_path_workspace_bytes")
    ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=X.col_ptr.device)
    W = torch.empty((lam.size, X.k), dtype=torch.float32, device=X.col_ptr.device)
    out = PathSchedule()
    _check(lib().gencd_autotune_path(X.ref, _ptr(y), C.byref(params),
                                     lam.ctypes.data_as(C.c_void_p), int(lam.size),
                                     cache_path.encode() if cache_path else None, _ptr(W), _ptr(ws),
                                     ws.numel(), _stream(), C.byref(out)), "gencd_autotune_path")
    return out.as_dict()


def apply_schedule(params: Params, sched: dict):
    params.group = int(sched["group"])
    params.piece = int(sched["piece"])
    params.flags = (params.flags & ~USE_GRAPH) | int(sched["flags"])
    params.residual = int(sched.get("residual", 0))
    return params
