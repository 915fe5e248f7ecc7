"""FP64 CPU oracle for plain and compressed NeNMF.

TEST INFRASTRUCTURE ONLY.  This module is the independent reference that the
HIP library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
never does.  It shares no code with the HIP path: it consumes the same seeded
FP32 inputs (``synth``), promotes them to FP64 and follows the paper's steps.

Paper: F. Yahaya, M. Puigt, G. Delmaire, G. Roussel, "Faster-than-fast NMF
using random projections and Nesterov iterations" (arXiv 1812.04315).

  * NMF model X ~ G F, G (n x p) >= 0, F (p x m) >= 0: Sec. 1, Eq. (1).
  * Alternating subproblems: Sec. 1, Eqs. (2) and (3).
  * NeNMF inner loop (Nesterov optimal gradient, alpha series, KKT-based
    stopping with Max_iter and a gradient bound): Sec. 2.
  * Compressed NMF strategy: Sec. 3, Algorithm 1.
  * Randomized subspace iteration: Sec. 3, Algorithm 2.
  * Relative reconstruction error: Sec. 4, Eq. (4).

Readings taken where the paper is silent (each one is restated where it is
used): two independent RSI chains; thin QR with positive diagonal and a
numerical-rank rule that swaps a deficient column for the matching column of
the other Gaussian draw; step 1/L with L = lambda_max(W); alpha restarts at 1
for every inner loop; the inner loop returns its last projected iterate; the
gradient bound is ratio * (initial projected-gradient norm), divided by 10
for a factor whose inner loop stops within its minimum step count.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, library routines or brute force, except the full
noisy end-to-end iterate sequence, whose noise-bulk basis columns are fixed
only up to roundoff (parity for it is checked on range-invariant outputs).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F64 = np.float64

STOP_GLOBAL = "global"
STOP_SUBPROBLEM = "subproblem"


class OrthBreakdown(RuntimeError):
    """A deficient column's replacement from the Gaussian pool is deficient too."""


# ---------------------------------------------------------------------------
# Nesterov weights (Sec. 2): alpha_0 = 1, alpha_{k+1} = (1 + sqrt(4 alpha_k^2 + 1)) / 2
# ---------------------------------------------------------------------------

def alpha_series(K: int) -> np.ndarray:
    """alpha_0 .. alpha_K of Sec. 2."""
    a = np.empty(K + 1, dtype=F64)
    a[0] = 1.0
    for k in range(K):
        a[k + 1] = (1.0 + math.sqrt(4.0 * a[k] * a[k] + 1.0)) / 2.0
    return a


def momentum_weights(K: int) -> np.ndarray:
    """beta_k = (alpha_{k-1} - 1) / alpha_k for k = 1..K (index 0 unused).

    After inner step k, the next point slides from F_k along F_k - F_{k-1}
    with this weight (Sec. 2).  beta_1 = 0 because alpha_0 = 1.
    """
    a = alpha_series(K)
    b = np.zeros(K + 1, dtype=F64)
    for k in range(1, K + 1):
        b[k] = (a[k - 1] - 1.0) / a[k]
    return b


# ---------------------------------------------------------------------------
# Orthonormal bases for Algorithm 2 ("QR decomposition", "orthonormal bases")
# ---------------------------------------------------------------------------

def orth(Y, pool, tau2: float = 1e-9):
    """Thin Q factor of Y (N x l) with positive-diagonal R, by classical
    Gram-Schmidt with one re-orthogonalisation pass per column (CGS2).

    Numerical-rank reading (Algorithm 2 leaves rank deficiency open): column j
    is deficient when its squared residual after projection onto the columns
    before it is <= tau2 * max_i ||y_i||^2.  A deficient column is replaced by
    column j of ``pool`` (the other Gaussian draw of Algorithm 2, in the same
    space) and projected again; if the replacement's squared residual is
    <= tau2 * ||pool_j||^2 the basis cannot be completed (OrthBreakdown).

    Returns (Q, replaced) where replaced[j] is True for swapped columns.
    """
    Y = np.asarray(Y, dtype=F64)
    P = np.asarray(pool, dtype=F64)
    N, ell = Y.shape
    if P.shape != (N, ell):
        raise ValueError("pool must have the shape of Y")
    scale = max(float(np.max(np.sum(Y * Y, axis=0))), 0.0) if ell else 0.0
    Q = np.zeros((N, ell), dtype=F64)
    replaced = np.zeros(ell, dtype=bool)

    def residual(v, j):
        for _ in range(2):
            if j:
                v = v - Q[:, :j] @ (Q[:, :j].T @ v)
        return v

    for j in range(ell):
        v = residual(Y[:, j].copy(), j)
        if float(v @ v) <= tau2 * scale:
            replaced[j] = True
            w = P[:, j].copy()
            ref = float(w @ w)
            v = residual(w, j)
            if not float(v @ v) > tau2 * ref:
                raise OrthBreakdown(f"column {j}: replacement is deficient")
        Q[:, j] = v / math.sqrt(float(v @ v))
    return Q, replaced


# ---------------------------------------------------------------------------
# bfloat16 rounding for the precision form (round to nearest, ties to even)
# ---------------------------------------------------------------------------

def bf16_bits(x) -> np.ndarray:
    """bfloat16 bit patterns of FP32 values: keep the upper 16 bits after
    rounding the lower 16 to nearest, ties to even; NaN stays a quiet NaN."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    is_nan = ((u & 0x7F800000) == 0x7F800000) & ((u & 0x007FFFFF) != 0)
    half = 0x7FFF + ((u >> 16) & 1)
    r = ((u + half) >> 16) & 0xFFFF
    r = np.where(is_nan, (u >> 16) | 0x40, r)
    return r.astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    """FP64 values of bfloat16 bit patterns (exact)."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    with np.errstate(invalid="ignore"):
        return b.view(np.float32).astype(F64)


def bf16_round(x) -> np.ndarray:
    """Round FP32 (or FP64, first rounded to FP32) values to bfloat16,
    returned as FP64."""
    return bf16_value(bf16_bits(np.asarray(x, dtype=np.float32)))


@dataclass
class RSIResult:
    Q_L: np.ndarray   # n x l, orthonormal columns (left basis: X_L = Q_L^T X)
    Q_R: np.ndarray   # m x l, orthonormal columns (right basis: X_R = X Q_R)
    X_L: np.ndarray   # l x m
    X_R: np.ndarray   # n x l
    replaced: list = field(default_factory=list)  # (stage, bool array) per orth


def rsi(X, omega_L, omega_R, q: int, tau2: float = 1e-9, bf16: bool = False) -> RSIResult:
    """Randomized subspace iteration, Sec. 3, Algorithm 2, in FP64.

    Readings: the two sketches X Omega_L and Omega_R X start two independent
    chains; every half-step re-orthonormalises.  Algorithm 2's final L and R
    (the k = q bases of the transposed half-step) have shapes m x l and l x n;
    by their shapes the l x n one multiplies X on the left and the m x l one on
    the right, which gives Algorithm 1's compressed data.  Its last products
    X Q~_L^(q) and Q~_R^(q) X are then exactly X_R and X_L, so the final QR of
    the loop is not needed.  Panels of the Omega_R chain are kept transposed
    (n x l and m x l) so every basis here has orthonormal columns.

    Replacement pools: n-space panels take columns of Omega_R^T, m-space
    panels take columns of Omega_L.

    bf16=True emulates the precision form: X and, before every product with
    X, the skinny operand are rounded to bfloat16; the products and all the
    rest stay FP64.
    """
    if q < 1:
        raise ValueError("q >= 1 required")
    X = bf16_round(X) if bf16 else np.asarray(X, dtype=F64)
    oL = np.asarray(omega_L, dtype=F64)       # m x l
    oRt = np.asarray(omega_R, dtype=F64).T    # n x l
    reps = []
    rnd = bf16_round if bf16 else (lambda a: a)

    def right(P):                             # X P
        return X @ rnd(P)

    def left(P):                              # X^T P
        return X.T @ rnd(P)

    def orth_n(Y, tag):
        Q, r = orth(Y, oRt, tau2)
        reps.append((tag, r))
        return Q

    def orth_m(Y, tag):
        Q, r = orth(Y, oL, tau2)
        reps.append((tag, r))
        return Q

    # Sketches of step 0 and their bases.
    QL = orth_n(right(oL), "L0")       # basis of X Omega_L           (n x l)
    QRt = orth_m(left(oRt), "R0")      # basis of (Omega_R X)^T       (m x l)
    A = B = Qt_L = Qt_Rt = None
    for k in range(1, q + 1):
        Qt_L = orth_m(left(QL), f"Lt{k}")      # X^T Q_L^(k-1)          (m x l)
        Qt_Rt = orth_n(right(QRt), f"Rt{k}")   # (Q_R^(k-1) X^T)^T      (n x l)
        A = right(Qt_L)                        # X Q~_L^(k)             (n x l)
        B = left(Qt_Rt)                        # (Q~_R^(k) X)^T         (m x l)
        if k < q:
            QL = orth_n(A, f"L{k}")
            QRt = orth_m(B, f"R{k}")
    return RSIResult(Q_L=Qt_Rt, Q_R=Qt_L, X_L=B.T.copy(), X_R=A, replaced=reps)


# ---------------------------------------------------------------------------
# NeNMF inner loop (Sec. 2)
# ---------------------------------------------------------------------------

def lipschitz(W) -> float:
    """Lipschitz constant of Z -> Z W - B: the largest eigenvalue of the
    symmetric PSD p x p matrix W (step 1/L of the single gradient step)."""
    W = np.asarray(W, dtype=F64)
    if W.size == 0:
        return 0.0
    return float(np.linalg.eigvalsh(0.5 * (W + W.T))[-1])


def gradient(Z, W, B, side: str):
    """Gradient of 0.5||X - G F||^2 in the free factor: Z W - B for G
    (Eq. (2), Z = G, W = F F^T, B = X F^T) and W Z - B for F (Eq. (3),
    Z = F, W = G^T G, B = G^T X)."""
    return Z @ W - B if side == "G" else W @ Z - B


def projected_gradient(Z, grad):
    """KKT projected gradient: grad where Z > 0, min(0, grad) where Z = 0."""
    return np.where(Z > 0, grad, np.minimum(grad, 0.0))


def pg_norm(Z, W, B, side: str) -> float:
    return float(np.linalg.norm(projected_gradient(Z, gradient(Z, W, B, side))))


def nesterov_nnls(Z0, W, B, side: str, tol: float, inner_max: int,
                  inner_min: int = 1, forced_steps: int | None = None):
    """One NeNMF inner loop (Sec. 2) for min_{Z >= 0} 0.5||X - G F||^2 in one factor.

    Y_0 = Z_0 (the outer iterate), alpha_0 = 1.  Step k: Z_k is one projected
    gradient step from Y_k with step 1/L; Y_{k+1} slides Z_k along
    Z_k - Z_{k-1} with weight (alpha_{k-1} - 1)/alpha_k.  Stop after
    ``inner_max`` steps or at the first k >= inner_min whose projected
    gradient at Z_k has norm <= tol; return Z_k (the last feasible iterate).
    With ``forced_steps`` the loop runs exactly that many steps and ignores
    the tolerance.  L = 0 (W = 0) leaves Z_0 unchanged and reports 0 steps.

    Returns (Z, steps, L).
    """
    Z0 = np.asarray(Z0, dtype=F64)
    W = np.asarray(W, dtype=F64)
    B = np.asarray(B, dtype=F64)
    L = lipschitz(W)
    if not L > 0.0:
        return Z0.copy(), 0, L
    kmax = inner_max if forced_steps is None else forced_steps
    Y = Z0.copy()
    Zprev = Z0.copy()
    Z = Z0.copy()
    alpha = 1.0
    k = 0
    for k in range(1, kmax + 1):
        Z = np.maximum(Y - gradient(Y, W, B, side) / L, 0.0)
        alpha_next = (1.0 + math.sqrt(4.0 * alpha * alpha + 1.0)) / 2.0
        Y = Z + ((alpha - 1.0) / alpha_next) * (Z - Zprev)
        Zprev = Z
        alpha = alpha_next
        if forced_steps is None and k >= inner_min and pg_norm(Z, W, B, side) <= tol:
            break
    return Z, k, L


# ---------------------------------------------------------------------------
# Subproblem data, plain (Eqs. (2), (3)) and compressed (Algorithm 1)
# ---------------------------------------------------------------------------

def g_data_plain(X, F):
    """W = F F^T, B = X F^T for Eq. (2)."""
    return F @ F.T, X @ F.T


def f_data_plain(X, G):
    """W = G^T G, B = G^T X for Eq. (3)."""
    return G.T @ G, G.T @ X


def g_data_compressed(X_R, Q_R, F):
    """Algorithm 1: F_R = F R, then Eq. (2) with X -> X_R and F -> F_R."""
    F_R = F @ Q_R
    return F_R @ F_R.T, X_R @ F_R.T


def f_data_compressed(X_L, Q_L, G):
    """Algorithm 1: G_L = L G, then Eq. (3) with X -> X_L and G -> G_L."""
    G_L = Q_L.T @ G
    return G_L.T @ G_L, G_L.T @ X_L


@dataclass
class NeNMFResult:
    G: np.ndarray
    F: np.ndarray
    steps: np.ndarray        # T x 2 inner step counts (G, F)
    lips: np.ndarray         # T x 2 Lipschitz constants
    tols: np.ndarray         # T x 2 tolerances in force at each solve
    tol0: float
    history: list            # [(G_t, F_t)] after each outer iteration (if kept)


def nenmf(X, G0, F0, outer_iters: int, inner_max: int, inner_min: int = 1,
          ratio: float = 1e-3, stop_rule: str = STOP_GLOBAL,
          compressed: RSIResult | None = None, replay=None,
          keep_history: bool = False) -> NeNMFResult:
    """Plain NeNMF (Sec. 2) or, given RSI output, compressed NeNMF (Algorithm 1).

    Each outer iteration updates G (Eq. (2)) and then F (Eq. (3)) with one
    Nesterov inner loop each.  Compressed data is used as is: X_L, X_R, G_L
    and F_R may be negative (semi-NMF remark of Sec. 3); only G and F are
    projected.

    Gradient bound (reading of Sec. 2's KKT criterion):
      * ``global``: tol_G = tol_F = ratio * ||(P grad_G, P grad_F)||_F at
        (G0, F0) on the method's own subproblems; a factor's tolerance is
        divided by 10 whenever its inner loop stops within ``inner_min``
        steps.
      * ``subproblem``: each inner loop uses ratio * ||P grad(Z_0)||_F.
    ``replay`` (T x 2 ints) forces the inner step counts.
    """
    X = None if X is None else np.asarray(X, dtype=F64)
    G = np.asarray(G0, dtype=F64).copy()
    F = np.asarray(F0, dtype=F64).copy()
    if compressed is not None:
        QL = np.asarray(compressed.Q_L, dtype=F64)
        QR = np.asarray(compressed.Q_R, dtype=F64)
        XL = np.asarray(compressed.X_L, dtype=F64)
        XR = np.asarray(compressed.X_R, dtype=F64)

        def gdata(F_):
            return g_data_compressed(XR, QR, F_)

        def fdata(G_):
            return f_data_compressed(XL, QL, G_)
    else:
        def gdata(F_):
            return g_data_plain(X, F_)

        def fdata(G_):
            return f_data_plain(X, G_)

    tol0 = 0.0
    if stop_rule == STOP_GLOBAL:
        Wg, Bg = gdata(F)
        Wf, Bf = fdata(G)
        pg_g = projected_gradient(G, gradient(G, Wg, Bg, "G"))
        pg_f = projected_gradient(F, gradient(F, Wf, Bf, "F"))
        tol0 = ratio * math.sqrt(float(np.sum(pg_g * pg_g)) + float(np.sum(pg_f * pg_f)))
    elif stop_rule != STOP_SUBPROBLEM:
        raise ValueError(stop_rule)
    tol_g = tol_f = tol0
    steps = np.zeros((outer_iters, 2), dtype=np.int64)
    lips = np.zeros((outer_iters, 2), dtype=F64)
    tols = np.zeros((outer_iters, 2), dtype=F64)
    hist = []
    for t in range(outer_iters):
        forced = None if replay is None else replay[t]
        W, B = gdata(F)
        tg = tol_g if stop_rule == STOP_GLOBAL else ratio * pg_norm(G, W, B, "G")
        tols[t, 0] = tg
        G, kg, lg = nesterov_nnls(G, W, B, "G", tg, inner_max, inner_min,
                                  None if forced is None else int(forced[0]))
        if stop_rule == STOP_GLOBAL and 1 <= kg <= inner_min:
            tol_g /= 10.0
        W, B = fdata(G)
        tf = tol_f if stop_rule == STOP_GLOBAL else ratio * pg_norm(F, W, B, "F")
        tols[t, 1] = tf
        F, kf, lf = nesterov_nnls(F, W, B, "F", tf, inner_max, inner_min,
                                  None if forced is None else int(forced[1]))
        if stop_rule == STOP_GLOBAL and 1 <= kf <= inner_min:
            tol_f /= 10.0
        steps[t] = (kg, kf)
        lips[t] = (lg, lf)
        if keep_history:
            hist.append((G.copy(), F.copy()))
    return NeNMFResult(G=G, F=F, steps=steps, lips=lips, tols=tols, tol0=tol0,
                       history=hist)


# ---------------------------------------------------------------------------
# Measurement (Sec. 4)
# ---------------------------------------------------------------------------

def rre(X, G, F) -> float:
    """Relative reconstruction error ||X - G F||_F / ||X||_F, Sec. 4, Eq. (4)."""
    X = np.asarray(X, dtype=F64)
    R = X - np.asarray(G, dtype=F64) @ np.asarray(F, dtype=F64)
    return float(np.linalg.norm(R) / np.linalg.norm(X))


def svd_floor(X, p: int) -> float:
    """Smallest RRE any rank-p factorisation can reach (truncated SVD), for
    small matrices by a full SVD."""
    X = np.asarray(X, dtype=F64)
    s = np.linalg.svd(X, compute_uv=False)
    return float(math.sqrt(float(np.sum(s[p:] ** 2))) / math.sqrt(float(np.sum(s ** 2))))
