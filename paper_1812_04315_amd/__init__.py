"""Compressed NeNMF on MI355X (gfx950): thin Python binding of libcnmf.

The work happens in ``libcnmf.so`` (HIP kernels behind the C ABI declared in
``include/cnmf.h``).  This module only marshals torch tensors (device memory
and the current HIP stream) into those calls.  There is no fallback: if the
library is missing or no GPU is present, every entry point raises.

Method: Yahaya, Puigt, Delmaire, Roussel, "Faster-than-fast NMF using random
projections and Nesterov iterations": randomized subspace iteration
(Sec. 3, Algorithm 2) feeding compressed NeNMF (Sec. 3, Algorithm 1) whose
factor updates are NeNMF's Nesterov inner loops (Sec. 2).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcnmf.so")

OK, EINVAL, ENOMEM, EHIP, EDEVICE, ENODERIV, ETOOBIG = 0, -1, -2, -3, -4, -5, -6
NOALLOC_SCRATCH_BYTES = 32 << 20
ST_NONFINITE, ST_NEGATIVE, ST_BREAKDOWN, ST_ZERO_LIPS, ST_TIMEOUT = 1, 2, 4, 8, 16
STOP_GLOBAL, STOP_SUBPROBLEM = 0, 1
PREC_FP32, PREC_BF16 = 0, 1
FLAG_VALIDATE_INPUT = 1
METHOD_PLAIN, METHOD_COMPRESSED = 0, 1
SOLVER_NESTEROV, SOLVER_HALS, SOLVER_MU = 0, 1, 2
RESTART_NONE, RESTART_GRADIENT = 0, 1
COMPRESS_RSI, COMPRESS_GAUSSIAN, COMPRESS_POWER = 0, 1, 2

EXPORTED = [
    "cnmf_params_default", "cnmf_strerror", "cnmf_create", "cnmf_destroy",
    "cnmf_set_stream", "cnmf_clock_hz", "cnmf_status", "cnmf_rsi", "cnmf_rsi_bf16",
    "cnmf_compress",
    "cnmf_to_bf16", "cnmf_solve", "cnmf_solve_noalloc", "cnmf_rre", "cnmf_sweep_right", "cnmf_sweep_left",
    "cnmf_sweep_dual", "cnmf_sweep_right_bf16", "cnmf_sweep_left_bf16", "cnmf_sweep_dual_bf16",
    "cnmf_orth", "cnmf_lipschitz", "cnmf_nnls",
    "cnmf_batch_create", "cnmf_batch_destroy", "cnmf_batch_rsi", "cnmf_batch_tune",
    "cnmf_batch_solve", "cnmf_adj_forward", "cnmf_adj_backward", "cnmf_tape_bytes",
    "cnmf_tape_destroy",
]


class CnmfError(RuntimeError):
    def __init__(self, code: int, what: str, status: int = 0):
        super().__init__(f"{what}: {strerror(code)} (code {code}, status 0x{status:x})")
        self.code = code
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int32), ("nu", ctypes.c_int32), ("q", ctypes.c_int32),
        ("outer_iters", ctypes.c_int32), ("inner_max", ctypes.c_int32),
        ("inner_min", ctypes.c_int32), ("inner_ratio", ctypes.c_double),
        ("tau2", ctypes.c_double), ("stop_rule", ctypes.c_int32),
        ("sweep_prec", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("solver", ctypes.c_int32), ("restart", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("time_budget", ctypes.c_double),
    ]


class Instance(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64), ("p", ctypes.c_int32),
        ("nu", ctypes.c_int32), ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64),
        ("omega_L", ctypes.c_void_p), ("omega_R", ctypes.c_void_p),
        ("Q_L", ctypes.c_void_p), ("Q_R", ctypes.c_void_p), ("X_L", ctypes.c_void_p),
        ("X_R", ctypes.c_void_p), ("G", ctypes.c_void_p), ("F", ctypes.c_void_p),
        ("steps", ctypes.c_void_p), ("replay", ctypes.c_void_p),
    ]


class Trace(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_void_p), ("lips", ctypes.c_void_p),
                ("tols", ctypes.c_void_p), ("ticks", ctypes.c_void_p),
                ("G_hist", ctypes.c_void_p), ("F_hist", ctypes.c_void_p),
                ("W_hist", ctypes.c_void_p), ("outer_done", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcnmf.so (built by ``python -m paper_1812_04315_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1812_04315_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        sig = {
            "cnmf_params_default": (None, [ctypes.POINTER(Params)]),
            "cnmf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "cnmf_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, P]),
            "cnmf_destroy": (ctypes.c_int, [P]),
            "cnmf_set_stream": (ctypes.c_int, [P, P]),
            "cnmf_clock_hz": (ctypes.c_int, [P, ctypes.POINTER(D)]),
            "cnmf_status": (ctypes.c_int, [P, ctypes.POINTER(I32)]),
            "cnmf_rsi": (ctypes.c_int, [P, I64, I64, P, I64, ctypes.POINTER(Params), P, P, P, P, P, P]),
            "cnmf_rsi_bf16": (ctypes.c_int, [P, I64, I64, P, I64, ctypes.POINTER(Params), P, P, P, P, P, P]),
            "cnmf_to_bf16": (ctypes.c_int, [P, I64, I64, P, I64, P, I64]),
            "cnmf_compress": (ctypes.c_int, [P, I32, I64, I64, P, I64, ctypes.POINTER(Params), P, P,
                                             P, P, P, P]),
            "cnmf_solve": (ctypes.c_int, [P, ctypes.c_int, I64, I64, P, I64, P, P, P, P,
                                          ctypes.POINTER(Params), P, P, ctypes.POINTER(Trace), P]),
            "cnmf_solve_noalloc": (ctypes.c_int, [P, ctypes.c_int, I64, I64, P, I64, P, P, P, P,
                                                  ctypes.POINTER(Params), P, P,
                                                  ctypes.POINTER(Trace), P]),
            "cnmf_rre": (ctypes.c_int, [P, I64, I64, P, I64, I32, P, I64, P, I64, I32, P]),
            "cnmf_sweep_right": (ctypes.c_int, [P, I64, I64, P, I64, I32, P, I64, I32, P, I64]),
            "cnmf_sweep_left": (ctypes.c_int, [P, I64, I64, P, I64, I32, P, I64, P, I64, I32]),
            "cnmf_sweep_dual": (ctypes.c_int, [P, I64, I64, P, I64, I32, P, I64, P, I64, P, I64,
                                               P, I64, I32]),
            "cnmf_sweep_right_bf16": (ctypes.c_int, [P, I64, I64, P, I64, I32, P, I64, I32, P, I64]),
            "cnmf_sweep_left_bf16": (ctypes.c_int, [P, I64, I64, P, I64, I32, P, I64, P, I64, I32]),
            "cnmf_sweep_dual_bf16": (ctypes.c_int, [P, I64, I64, P, I64, I32, P, I64, P, I64, P, I64,
                                                    P, I64, I32]),
            "cnmf_orth": (ctypes.c_int, [P, I64, I32, P, P, I32, D, P, P]),
            "cnmf_lipschitz": (ctypes.c_int, [P, I32, P, P]),
            "cnmf_nnls": (ctypes.c_int, [P, I64, I32, P, I64, I64, P, P, D, I32, I32, I32, P, P, P]),
            "cnmf_batch_create": (ctypes.c_int, [P, ctypes.POINTER(Instance), I32,
                                                 ctypes.POINTER(Params), I32, I32, ctypes.POINTER(P)]),
            "cnmf_batch_destroy": (ctypes.c_int, [P]),
            "cnmf_batch_rsi": (ctypes.c_int, [P]),
            "cnmf_batch_tune": (ctypes.c_int, [P, I32, ctypes.POINTER(I32)]),
            "cnmf_batch_solve": (ctypes.c_int, [P, I32]),
            "cnmf_adj_forward": (ctypes.c_int, [P, I64, I64, P, I64, ctypes.POINTER(Params), I32,
                                                P, P, P, P, P, P, ctypes.POINTER(P)]),
            "cnmf_adj_backward": (ctypes.c_int, [P, P, P, P, I64, P, P]),
            "cnmf_tape_bytes": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_uint64)]),
            "cnmf_tape_destroy": (ctypes.c_int, [P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().cnmf_strerror(code).decode()
    except Exception:  # noqa: BLE001
        return "unknown"


def params(p: int, nu: int = 10, q: int = 4, outer_iters: int = 200, inner_max: int = 500,
           inner_min: int = 1, inner_ratio: float = 1e-3, tau2: float = 1e-9,
           stop_rule: int = STOP_GLOBAL, sweep_prec: int = PREC_FP32, flags: int = 0,
           solver: int = SOLVER_NESTEROV, restart: int = RESTART_NONE,
           time_budget: float = 0.0) -> Params:
    return Params(p, nu, q, outer_iters, inner_max, inner_min, inner_ratio, tau2, stop_rule,
                  sweep_prec, flags, solver, restart, 0, time_budget)


# ---------------------------------------------------------------------------
# Context (one per device and stream)
# ---------------------------------------------------------------------------
_contexts: dict = {}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libcnmf needs a ROCm GPU; none is visible")
    return torch


class Context:
    def __init__(self, device: int, stream_handle: int):
        h = ctypes.c_void_p()
        rc = lib().cnmf_create(ctypes.byref(h), device, ctypes.c_void_p(stream_handle))
        if rc != OK:
            raise CnmfError(rc, "cnmf_create")
        self.h = h
        self.device = device
        hz = ctypes.c_double()
        lib().cnmf_clock_hz(h, ctypes.byref(hz))
        self.clock_hz = hz.value

    def status(self, clear_ok: bool = True) -> int:
        st = ctypes.c_int32()
        rc = lib().cnmf_status(self.h, ctypes.byref(st))
        if rc not in (OK, EDEVICE):
            raise CnmfError(rc, "cnmf_status")
        return st.value


def context(device=None):
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else int(device)
    stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev, stream)
    ctx = _contexts.get(key)
    if ctx is None:
        ctx = Context(dev, stream)
        _contexts[key] = ctx
    return ctx


def check(ctx: Context | None = None) -> int:
    """Synchronise, read and clear the device status word; raise on errors
    (the zero-Lipschitz warning alone does not raise)."""
    ctx = ctx or context()
    st = ctx.status()
    if st & ~ST_ZERO_LIPS:
        raise CnmfError(EDEVICE, "device status", st)
    return st


def _call(name: str, *args):
    rc = getattr(lib(), name)(*args)
    if rc != OK:
        raise CnmfError(rc, name)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t, dtype, name, shape=None, ld_ok=False):
    torch = _torch()
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.dim() == 2:
        if t.stride(1) != 1 or (not ld_ok and not t.is_contiguous()):
            raise ValueError(f"{name} must be row-major" + (" with unit column stride" if ld_ok else " and contiguous"))
    elif not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    del torch


def _ld(t) -> int:
    return t.stride(0) if t.dim() == 2 else t.shape[-1]


# ---------------------------------------------------------------------------
# Hot path
# ---------------------------------------------------------------------------

def rsi(X, omega_L, omega_R, p: int, nu: int, q: int = 4, tau2: float = 1e-9,
        validate: bool = False, out=None):
    """Randomized subspace iteration (Algorithm 2).  X (n x m, float32, any
    row pitch), omega_L (m x l), omega_R (l x n).  Returns (Q_L, Q_R, X_L, X_R)."""
    torch = _torch()
    n, m = X.shape
    ell = p + nu
    _need(X, torch.float32, "X", ld_ok=True)
    _need(omega_L, torch.float32, "omega_L", (m, ell))
    _need(omega_R, torch.float32, "omega_R", (ell, n))
    if out is None:
        dev = X.device
        out = (torch.empty(n, ell, device=dev), torch.empty(m, ell, device=dev),
               torch.empty(ell, m, device=dev), torch.empty(n, ell, device=dev))
    QL, QR, XL, XR = out
    prm = params(p, nu, q, tau2=tau2, flags=FLAG_VALIDATE_INPUT if validate else 0)
    _call("cnmf_rsi", context().h, n, m, _ptr(X), _ld(X), ctypes.byref(prm), _ptr(omega_L),
          _ptr(omega_R), _ptr(QL), _ptr(QR), _ptr(XL), _ptr(XR))
    return QL, QR, XL, XR


def compress(X, omega_L, omega_R, p: int, nu: int, q: int = 4, kind: int = COMPRESS_RSI,
             tau2: float = 1e-9, out=None):
    """Compression matrices and compressed data of Sec. 3 (``kind``: RSI,
    the scaled Gaussian projection, or power iteration without
    re-orthonormalisation).  Returns (Q_L, Q_R, X_L, X_R) as ``rsi``."""
    torch = _torch()
    n, m = X.shape
    ell = p + nu
    _need(X, torch.float32, "X", ld_ok=True)
    _need(omega_L, torch.float32, "omega_L", (m, ell))
    _need(omega_R, torch.float32, "omega_R", (ell, n))
    if out is None:
        dev = X.device
        out = (torch.empty(n, ell, device=dev), torch.empty(m, ell, device=dev),
               torch.empty(ell, m, device=dev), torch.empty(n, ell, device=dev))
    QL, QR, XL, XR = out
    prm = params(p, nu, q, tau2=tau2)
    _call("cnmf_compress", context().h, kind, n, m, _ptr(X), _ld(X), ctypes.byref(prm),
          _ptr(omega_L), _ptr(omega_R), _ptr(QL), _ptr(QR), _ptr(XL), _ptr(XR))
    return QL, QR, XL, XR


def rsi_bf16(Xb, omega_L, omega_R, p: int, nu: int, q: int = 4, tau2: float = 1e-9, out=None):
    """Algorithm 2 with the X-sized sweeps in BF16.  Xb is an int16 tensor
    holding bfloat16 bit patterns (see ``to_bf16``)."""
    torch = _torch()
    n, m = Xb.shape
    ell = p + nu
    _need(Xb, torch.int16, "Xb", ld_ok=True)
    _need(omega_L, torch.float32, "omega_L", (m, ell))
    _need(omega_R, torch.float32, "omega_R", (ell, n))
    if out is None:
        dev = Xb.device
        out = (torch.empty(n, ell, device=dev), torch.empty(m, ell, device=dev),
               torch.empty(ell, m, device=dev), torch.empty(n, ell, device=dev))
    QL, QR, XL, XR = out
    prm = params(p, nu, q, tau2=tau2, sweep_prec=PREC_BF16)
    _call("cnmf_rsi_bf16", context().h, n, m, _ptr(Xb), _ld(Xb), ctypes.byref(prm),
          _ptr(omega_L), _ptr(omega_R), _ptr(QL), _ptr(QR), _ptr(XL), _ptr(XR))
    return QL, QR, XL, XR


def to_bf16(X, ld: int | None = None):
    """bfloat16 (round to nearest even) copy of X as an int16 tensor whose
    row pitch is a multiple of 8 elements."""
    torch = _torch()
    _need(X, torch.float32, "X", ld_ok=True)
    n, m = X.shape
    ldb = ld or ((m + 7) // 8) * 8
    buf = torch.empty(n, ldb, dtype=torch.int16, device=X.device)
    _call("cnmf_to_bf16", context().h, n, m, _ptr(X), _ld(X), _ptr(buf), ldb)
    return buf[:, :m]


@dataclass
class SolveTrace:
    steps: object
    lips: object
    tols: object
    ticks: object
    G_hist: object
    F_hist: object
    W_hist: object = None
    outer_done: object = None


def make_trace(n: int, m: int, p: int, T: int, device, history: bool = True,
               grams: bool = False) -> SolveTrace:
    torch = _torch()
    return SolveTrace(
        steps=torch.zeros(T, 2, dtype=torch.int32, device=device),
        lips=torch.zeros(T, 2, dtype=torch.float64, device=device),
        tols=torch.zeros(T, 2, dtype=torch.float64, device=device),
        ticks=torch.zeros(T + 1, dtype=torch.int64, device=device),
        G_hist=torch.empty(T, n, p, device=device) if history else None,
        F_hist=torch.empty(T, p, m, device=device) if history else None,
        W_hist=torch.empty(T, 2, p, p, device=device) if grams else None,
        outer_done=torch.zeros(1, dtype=torch.int32, device=device))


def solve(G, F, *, X=None, compressed=None, p: int | None = None, nu: int = 10,
          outer_iters: int = 200, inner_max: int = 500, inner_min: int = 1,
          inner_ratio: float = 1e-3, stop_rule: int = STOP_GLOBAL, trace: SolveTrace | None = None,
          replay=None, solver: int = SOLVER_NESTEROV, restart: int = RESTART_NONE,
          time_budget: float = 0.0, noalloc: bool = False):
    """NeNMF outer loop in place on G (n x p) and F (p x m).  Plain when
    ``compressed`` is None (needs X), else ``compressed = (Q_L, Q_R, X_L, X_R)``
    from ``rsi`` (or any other compression of the same shapes).  ``noalloc``
    calls the entry point that allocates no device memory (its scratch is the
    library's static array on each GPU)."""
    torch = _torch()
    n, pp = G.shape
    p = pp if p is None else p
    m = F.shape[1]
    _need(G, torch.float32, "G", (n, p))
    _need(F, torch.float32, "F", (p, m))
    method = METHOD_PLAIN if compressed is None else METHOD_COMPRESSED
    ell = p
    QL = QR = XL = XR = None
    if compressed is not None:
        QL, QR, XL, XR = compressed
        ell = QL.shape[1]
        nu = ell - p
        _need(QL, torch.float32, "Q_L", (n, ell))
        _need(QR, torch.float32, "Q_R", (m, ell))
        _need(XL, torch.float32, "X_L", (ell, m))
        _need(XR, torch.float32, "X_R", (n, ell))
    if X is not None:
        _need(X, torch.float32, "X", (n, m), ld_ok=True)
    elif method == METHOD_PLAIN:
        raise ValueError("plain NeNMF needs X")
    if replay is not None:
        _need(replay, torch.int32, "replay", (outer_iters, 2))
    prm = params(p, nu, 1, outer_iters, inner_max, inner_min, inner_ratio, stop_rule=stop_rule,
                 solver=solver, restart=restart, time_budget=time_budget)
    tr = None
    if trace is not None:
        tr = Trace(*[ctypes.c_void_p(0 if t is None else t.data_ptr()) for t in
                     (trace.steps, trace.lips, trace.tols, trace.ticks, trace.G_hist, trace.F_hist,
                      trace.W_hist, trace.outer_done)])
    _call("cnmf_solve_noalloc" if noalloc else "cnmf_solve", context().h, method, n, m,
          _ptr(X), _ld(X) if X is not None else m,
          _ptr(QL), _ptr(QR), _ptr(XL), _ptr(XR), ctypes.byref(prm), _ptr(G), _ptr(F),
          ctypes.byref(tr) if tr is not None else None, _ptr(replay))
    return G, F


def rre(X, G, F, out=None):
    """Relative reconstruction error (Eq. (4)); G (n x p) or (count, n, p),
    F (p x m) or (count, p, m).  Returns a float64 device tensor."""
    torch = _torch()
    n, m = X.shape
    _need(X, torch.float32, "X", ld_ok=True)
    single = G.dim() == 2
    G3 = G.unsqueeze(0) if single else G
    F3 = F.unsqueeze(0) if single else F
    count, _, p = G3.shape
    if not (G3.is_contiguous() and F3.is_contiguous()) or F3.shape != (count, p, m):
        raise ValueError("G, F must be contiguous (count, n, p), (count, p, m)")
    if out is None:
        out = torch.empty(count, dtype=torch.float64, device=X.device)
    _call("cnmf_rre", context().h, n, m, _ptr(X), _ld(X), p, _ptr(G3), n * p, _ptr(F3), p * m,
          count, _ptr(out))
    return out[0] if single else out


# ---------------------------------------------------------------------------
# Kernel-level entry points
# ---------------------------------------------------------------------------

def sweep_right(X, A, a_trans: bool = False, out=None):
    """Y = X A with A (C x k), or A given as its transpose (k x C)."""
    torch = _torch()
    _need(X, torch.float32, "X", ld_ok=True)
    _need(A, torch.float32, "A", ld_ok=True)
    R, C = X.shape
    k = A.shape[0] if a_trans else A.shape[1]
    if (A.shape[1] if a_trans else A.shape[0]) != C:
        raise ValueError("inner dimensions differ")
    Y = torch.empty(R, k, device=X.device) if out is None else out
    _call("cnmf_sweep_right", context().h, R, C, _ptr(X), _ld(X), k, _ptr(A), _ld(A),
          1 if a_trans else 0, _ptr(Y), _ld(Y))
    return Y


def sweep_left(X, B, z_trans: bool = False, out=None):
    """Z = X^T B (C x k), or its transpose (k x C)."""
    torch = _torch()
    _need(X, torch.float32, "X", ld_ok=True)
    _need(B, torch.float32, "B", ld_ok=True)
    R, C = X.shape
    k = B.shape[1]
    if B.shape[0] != R:
        raise ValueError("inner dimensions differ")
    Z = (torch.empty(k, C, device=X.device) if z_trans else torch.empty(C, k, device=X.device)) \
        if out is None else out
    _call("cnmf_sweep_left", context().h, R, C, _ptr(X), _ld(X), k, _ptr(B), _ld(B), _ptr(Z),
          _ld(Z), 1 if z_trans else 0)
    return Z


def sweep_dual(X, AT, B, z_trans: bool = False):
    """(Y, Z) = (X A, X^T B) from one read of X, A given as its transpose AT
    (k x C), B (R x k); Z is C x k, or k x C if z_trans."""
    torch = _torch()
    _need(X, torch.float32, "X", ld_ok=True)
    _need(AT, torch.float32, "AT", ld_ok=True)
    _need(B, torch.float32, "B", ld_ok=True)
    R, C = X.shape
    k = AT.shape[0]
    if AT.shape[1] != C or B.shape[0] != R or B.shape[1] != k:
        raise ValueError("inner dimensions differ")
    Y = torch.empty(R, k, device=X.device)
    Z = torch.empty(k, C, device=X.device) if z_trans else torch.empty(C, k, device=X.device)
    _call("cnmf_sweep_dual", context().h, R, C, _ptr(X), _ld(X), k, _ptr(AT), _ld(AT), _ptr(B),
          _ld(B), _ptr(Y), _ld(Y), _ptr(Z), _ld(Z), 1 if z_trans else 0)
    return Y, Z


def sweep_right_bf16(Xb, A, a_trans: bool = False, out=None):
    """Y = X A on the matrix cores in BF16: Xb holds bfloat16 bit patterns
    (int16), A (C x k, or k x C if a_trans) is rounded to bfloat16."""
    torch = _torch()
    _need(Xb, torch.int16, "Xb", ld_ok=True)
    _need(A, torch.float32, "A", ld_ok=True)
    R, C = Xb.shape
    k = A.shape[0] if a_trans else A.shape[1]
    if (A.shape[1] if a_trans else A.shape[0]) != C:
        raise ValueError("inner dimensions differ")
    Y = torch.empty(R, k, device=Xb.device) if out is None else out
    _call("cnmf_sweep_right_bf16", context().h, R, C, _ptr(Xb), _ld(Xb), k, _ptr(A), _ld(A),
          1 if a_trans else 0, _ptr(Y), _ld(Y))
    return Y


def sweep_left_bf16(Xb, B, z_trans: bool = False, out=None):
    """Z = X^T B on the matrix cores in BF16 (B rounded to bfloat16)."""
    torch = _torch()
    _need(Xb, torch.int16, "Xb", ld_ok=True)
    _need(B, torch.float32, "B", ld_ok=True)
    R, C = Xb.shape
    k = B.shape[1]
    if B.shape[0] != R:
        raise ValueError("inner dimensions differ")
    Z = (torch.empty(k, C, device=Xb.device) if z_trans else torch.empty(C, k, device=Xb.device)) \
        if out is None else out
    _call("cnmf_sweep_left_bf16", context().h, R, C, _ptr(Xb), _ld(Xb), k, _ptr(B), _ld(B),
          _ptr(Z), _ld(Z), 1 if z_trans else 0)
    return Z


def sweep_dual_bf16(Xb, AT, B, z_trans: bool = False):
    """(Y, Z) = (X bf16(A), X^T bf16(B)) from one read of X in bfloat16 (Xb:
    int16 bit patterns), A given as its transpose AT (k x C), B (R x k)."""
    torch = _torch()
    _need(Xb, torch.int16, "Xb", ld_ok=True)
    _need(AT, torch.float32, "AT", ld_ok=True)
    _need(B, torch.float32, "B", ld_ok=True)
    R, C = Xb.shape
    k = AT.shape[0]
    if AT.shape[1] != C or B.shape[0] != R or B.shape[1] != k:
        raise ValueError("inner dimensions differ")
    Y = torch.empty(R, k, device=Xb.device)
    Z = torch.empty(k, C, device=Xb.device) if z_trans else torch.empty(C, k, device=Xb.device)
    _call("cnmf_sweep_dual_bf16", context().h, R, C, _ptr(Xb), _ld(Xb), k, _ptr(AT), _ld(AT),
          _ptr(B), _ld(B), _ptr(Y), _ld(Y), _ptr(Z), _ld(Z), 1 if z_trans else 0)
    return Y, Z


def orth(Y, pool, pool_trans: bool = False, tau2: float = 1e-9):
    """CholeskyQR basis of Y (N x l) with the rank rule (second pass for an
    ill-conditioned panel); returns (Q, replaced)."""
    torch = _torch()
    N, ell = Y.shape
    _need(Y, torch.float32, "Y", (N, ell))
    _need(pool, torch.float32, "pool", (ell, N) if pool_trans else (N, ell))
    Q = torch.empty_like(Y)
    rep = torch.zeros(ell, dtype=torch.int32, device=Y.device)
    _call("cnmf_orth", context().h, N, ell, _ptr(Y), _ptr(pool), 1 if pool_trans else 0,
          tau2, _ptr(Q), _ptr(rep))
    return Q, rep


def lipschitz(W):
    torch = _torch()
    p = W.shape[0]
    _need(W, torch.float32, "W", (p, p))
    out = torch.empty(1, dtype=torch.float64, device=W.device)
    _call("cnmf_lipschitz", context().h, p, _ptr(W), _ptr(out))
    return out


def nnls(Z, W, B, tol: float, inner_max: int, inner_min: int = 1, forced: int = -1,
         by_columns: bool = False):
    """One Nesterov inner loop in place on Z: rows of Z (G side) or, with
    by_columns, columns of Z (F side, Z is p x m).  Returns (steps, L, pg0^2)
    as device tensors."""
    torch = _torch()
    p = W.shape[0]
    _need(W, torch.float32, "W", (p, p))
    if by_columns:
        _need(Z, torch.float32, "Z", (p, Z.shape[1]))
        rows, rs, cs = Z.shape[1], 1, Z.shape[1]
    else:
        _need(Z, torch.float32, "Z", (Z.shape[0], p))
        rows, rs, cs = Z.shape[0], p, 1
    _need(B, torch.float32, "B", (rows, p))
    steps = torch.zeros(1, dtype=torch.int32, device=Z.device)
    L = torch.zeros(1, dtype=torch.float64, device=Z.device)
    pg2 = torch.zeros(1, dtype=torch.float64, device=Z.device)
    _call("cnmf_nnls", context().h, rows, p, _ptr(Z), rs, cs, _ptr(W), _ptr(B), tol,
          inner_max, inner_min, forced, _ptr(steps), _ptr(L), _ptr(pg2))
    return steps, L, pg2


# ---------------------------------------------------------------------------
# Batched form
# ---------------------------------------------------------------------------
class Batch:
    """Many independent compressed-NeNMF instances planned together.

    ``instances``: list of dicts with device tensors X (n x m, may be None if
    the compressed data is supplied), omega_L, omega_R, Q_L, Q_R, X_L, X_R,
    G, F and optional int32 ``steps`` / ``replay`` (T x 2), plus ``p`` and
    ``nu``.  The tensors must stay alive while the batch is used."""

    def __init__(self, instances, *, q: int = 2, outer_iters: int = 100, inner_max: int = 500,
                 inner_min: int = 1, inner_ratio: float = 1e-3, stop_rule: int = STOP_GLOBAL,
                 tau2: float = 1e-9, tiles_g: int = 0, tiles_f: int = 0, tune_cache=None):
        """``tune_cache``: path of a JSON table of tuned tile shapes, keyed by
        the device and the batch's shapes and loop settings; a known key
        supplies tiles_g / tiles_f, and ``tune`` records its result there."""
        self._keep = list(instances)
        self._cache = tune_cache
        self._key = None
        if tune_cache is not None:
            import hashlib
            import json
            torch = _torch()
            sig = [torch.cuda.get_device_name(), q, outer_iters, inner_max, inner_min, inner_ratio,
                   stop_rule, [(int(d["G"].shape[0]), int(d["F"].shape[1]), int(d["p"]), int(d["nu"]))
                               for d in instances]]
            self._key = hashlib.sha256(json.dumps(sig).encode()).hexdigest()[:32]
            if tiles_g == 0 and tiles_f == 0 and os.path.exists(tune_cache):
                with open(tune_cache) as fh:
                    hit = json.load(fh).get(self._key)
                if hit:
                    tiles_g, tiles_f = int(hit[0]), int(hit[1])
        self.tiles = (tiles_g, tiles_f)
        arr = (Instance * len(instances))()
        for k, d in enumerate(instances):
            G, F = d["G"], d["F"]
            n, p = G.shape
            m = F.shape[1]
            X = d.get("X")
            arr[k] = Instance(n, m, d["p"], d["nu"], _ptr(X) if X is not None else None,
                              _ld(X) if X is not None else m,
                              _ptr(d["omega_L"]) if d.get("omega_L") is not None else None,
                              _ptr(d["omega_R"]) if d.get("omega_R") is not None else None,
                              _ptr(d["Q_L"]), _ptr(d["Q_R"]), _ptr(d["X_L"]), _ptr(d["X_R"]),
                              _ptr(G), _ptr(F),
                              _ptr(d["steps"]) if d.get("steps") is not None else None,
                              _ptr(d["replay"]) if d.get("replay") is not None else None)
        prm = params(1, 0, q, outer_iters, inner_max, inner_min, inner_ratio, tau2, stop_rule)
        self._ctx = context()
        h = ctypes.c_void_p()
        _call("cnmf_batch_create", self._ctx.h, arr, len(instances), ctypes.byref(prm),
              tiles_g, tiles_f, ctypes.byref(h))
        self.h = h

    def rsi(self):
        _call("cnmf_batch_rsi", self.h)

    def tune(self, iters: int = 3):
        """Time every tile shape on scratch copies, keep the fastest (and
        record it in the tune cache, if one was given)."""
        out = (ctypes.c_int32 * 2)()
        _call("cnmf_batch_tune", self.h, iters, out)
        self.tiles = (int(out[0]), int(out[1]))
        if self._cache is not None:
            import json
            table = {}
            if os.path.exists(self._cache):
                with open(self._cache) as fh:
                    table = json.load(fh)
            table[self._key] = list(self.tiles)
            tmp = f"{self._cache}.tmp{os.getpid()}"
            with open(tmp, "w") as fh:
                json.dump(table, fh, indent=1)
            os.replace(tmp, self._cache)
        return self.tiles

    def solve(self, use_graph: bool = True):
        _call("cnmf_batch_solve", self.h, 1 if use_graph else 0)

    def close(self):
        if self.h:
            lib().cnmf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


# ---------------------------------------------------------------------------
# Differentiation form
# ---------------------------------------------------------------------------
class Tape:
    """Forward state of an unrolled compressed-NeNMF run (library-owned)."""

    def __init__(self, h, keep, shapes):
        self.h = h
        self._keep = keep          # X, omega_L, omega_R must outlive the tape
        self.n, self.m, self.p = shapes

    @property
    def bytes(self) -> int:
        v = ctypes.c_uint64()
        _call("cnmf_tape_bytes", self.h, ctypes.byref(v))
        return int(v.value)

    def backward(self, dG, dF, want_factors: bool = True):
        """dL/dX (n x m) and, optionally, dL/dG0, dL/dF0 from dL/dG_T, dL/dF_T."""
        torch = _torch()
        dG = dG.detach().float().contiguous()
        dF = dF.detach().float().contiguous()
        dX = torch.empty(self.n, self.m, device=dG.device)
        dG0 = torch.empty_like(dG) if want_factors else None
        dF0 = torch.empty_like(dF) if want_factors else None
        _call("cnmf_adj_backward", self.h, _ptr(dG), _ptr(dF), _ptr(dX), self.m,
              _ptr(dG0) if dG0 is not None else None, _ptr(dF0) if dF0 is not None else None)
        return dX, dG0, dF0

    def close(self):
        if self.h:
            lib().cnmf_tape_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def adj_forward(X, omega_L, omega_R, G0, F0, *, p: int, nu: int = 10, q: int = 2,
                outer_iters: int = 50, inner_steps: int = 5, ckpt: int = 10):
    """Compressed NeNMF with exactly ``inner_steps`` inner steps, keeping the
    tape for the reverse pass.  Returns (G_T, F_T, Tape)."""
    torch = _torch()
    _need(X, torch.float32, "X", ld_ok=True)
    n, m = X.shape
    ell = p + nu
    _need(omega_L, torch.float32, "omega_L", (m, ell))
    _need(omega_R, torch.float32, "omega_R", (ell, n))
    _need(G0, torch.float32, "G0", (n, p))
    _need(F0, torch.float32, "F0", (p, m))
    G = torch.empty_like(G0)
    F = torch.empty_like(F0)
    prm = params(p, nu, q, outer_iters, inner_steps, stop_rule=STOP_SUBPROBLEM)
    h = ctypes.c_void_p()
    _call("cnmf_adj_forward", context().h, n, m, _ptr(X), _ld(X), ctypes.byref(prm), ckpt,
          _ptr(omega_L), _ptr(omega_R), _ptr(G0), _ptr(F0), _ptr(G), _ptr(F), ctypes.byref(h))
    return G, F, Tape(h, (X, omega_L, omega_R), (n, m, p))


def _autograd_function():
    torch = _torch()

    class CompressedNeNMF(torch.autograd.Function):
        """(X, G0, F0) -> (G_T, F_T) of unrolled compressed NeNMF; backward by
        the library's hand-written adjoint."""

        @staticmethod
        def forward(ctx, X, G0, F0, omega_L, omega_R, p, nu, q, outer_iters, inner_steps, ckpt):
            Xc = X.detach().contiguous()
            G, F, tape = adj_forward(Xc, omega_L.detach().contiguous(),
                                     omega_R.detach().contiguous(), G0.detach().contiguous(),
                                     F0.detach().contiguous(), p=p, nu=nu, q=q,
                                     outer_iters=outer_iters, inner_steps=inner_steps, ckpt=ckpt)
            ctx.tape = tape
            return G, F

        @staticmethod
        def backward(ctx, gG, gF):
            torch_ = _torch()
            gG = torch_.zeros_like(ctx.tape._keep[0][:, :ctx.tape.p]) if gG is None else gG
            gF = torch_.zeros(ctx.tape.p, ctx.tape.m, device=gG.device) if gF is None else gF
            dX, dG0, dF0 = ctx.tape.backward(gG, gF)
            return dX, dG0, dF0, None, None, None, None, None, None, None, None

    return CompressedNeNMF


def compressed_nenmf(X, G0, F0, omega_L, omega_R, *, p: int, nu: int = 10, q: int = 2,
                     outer_iters: int = 50, inner_steps: int = 5, ckpt: int = 10):
    """Differentiable compressed NeNMF: returns (G_T, F_T); gradients with
    respect to X, G0 and F0 come from the hand-written adjoint."""
    return _autograd_function().apply(X, G0, F0, omega_L, omega_R, p, nu, q, outer_iters,
                                      inner_steps, ckpt)
