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


def compress_gaussian(X, omega_L, omega_R) -> RSIResult:
    """The plain random projection of Sec. 3 (Algorithm 1 with scaled
    Gaussian compression matrices): L = Omega / sqrt(nu) for a nu x n
    Gaussian Omega, and likewise R.  Here nu = l, L = Omega_R / sqrt(l)
    (l x n, so Q_L = L^T is n x l), R = Omega_L / sqrt(l) (m x l), and the
    compressed data are X_L = L X and X_R = X R.  Q_L, Q_R are not
    orthonormal."""
    X = np.asarray(X, dtype=F64)
    oL = np.asarray(omega_L, dtype=F64)
    oR = np.asarray(omega_R, dtype=F64)
    ell = oL.shape[1]
    R = oL / math.sqrt(ell)
    Lt = oR.T / math.sqrt(ell)
    return RSIResult(Q_L=Lt, Q_R=R, X_L=Lt.T @ X, X_R=X @ R)


def compress_power(X, omega_L, omega_R, q: int, tau2: float = 1e-9) -> RSIResult:
    """Randomized power iteration without re-orthonormalisation (the
    structured random projection Sec. 3 cites, of which Algorithm 2 is the
    stable variant): the same two chains as ``rsi`` with the same number of
    products, but only the final panels are orthonormalised:
        Q_R = orth((X^T X)^q Omega_L),   Q_L = orth((X X^T)^q Omega_R^T),
    then X_R = X Q_R and X_L = Q_L^T X.  Every intermediate panel is divided
    by its Frobenius norm, which leaves its range unchanged (in exact
    arithmetic the bases span the same subspaces as those of ``rsi``).
    The final orthonormalisation uses the rank rule of ``orth`` with the same
    pools as ``rsi``."""
    if q < 1:
        raise ValueError("q >= 1 required")
    X = np.asarray(X, dtype=F64)
    oL = np.asarray(omega_L, dtype=F64)
    oRt = np.asarray(omega_R, dtype=F64).T

    def unit(Y):
        return Y / np.linalg.norm(Y)

    Ym = oL                      # m-space chain: (X^T X)^q Omega_L
    Yn = oRt                     # n-space chain: (X X^T)^q Omega_R^T
    for _ in range(q):
        Ym = unit(X.T @ unit(X @ Ym))
        Yn = unit(X @ unit(X.T @ Yn))
    QR, rR = orth(Ym, oL, tau2)
    QL, rL = orth(Yn, oRt, tau2)
    return RSIResult(Q_L=QL, Q_R=QR, X_L=QL.T @ X, X_R=X @ QR,
                     replaced=[("R", rR), ("L", rL)])


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
                  inner_min: int = 1, forced_steps: int | None = None,
                  pg_trace: list | None = None, restart: bool = False):
    """One NeNMF inner loop (Sec. 2) for min_{Z >= 0} 0.5||X - G F||^2 in one factor.

    Y_0 = Z_0 (the outer iterate), alpha_0 = 1.  Step k: Z_k is one projected
    gradient step from Y_k with step 1/L; Y_{k+1} slides Z_k along
    Z_k - Z_{k-1} with weight (alpha_{k-1} - 1)/alpha_k.  Stop after
    ``inner_max`` steps or at the first k >= inner_min whose projected
    gradient at Z_k has norm <= tol; return Z_k (the last feasible iterate).
    With ``forced_steps`` the loop runs exactly that many steps and ignores
    the tolerance.  L = 0 (W = 0) leaves Z_0 unchanged and reports 0 steps.
    ``pg_trace`` (a list) receives the projected-gradient norm at every Z_k,
    also in forced runs (a record of how close each stop decision was).

    ``restart``: adaptive restart (O'Donoghue and Candes, suggested in the
    footnote of Sec. 4 for the non-monotone compressed error).  The
    subproblem separates into independent rows of G (columns of F), each
    with its own alpha series; a row restarts (alpha back to 1, so its next
    point is Z_k itself) when its gradient-mapping step Y_k - Z_k and its
    last move Z_k - Z_{k-1} have a positive inner product.

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
    # restart: one alpha per independent row (G) or column (F)
    axis = 1 if side == "G" else 0
    alphas = np.ones(Z0.shape[1 - axis], dtype=F64) if restart else None
    k = 0
    for k in range(1, kmax + 1):
        Z = np.maximum(Y - gradient(Y, W, B, side) / L, 0.0)
        if restart:
            again = np.sum((Y - Z) * (Z - Zprev), axis=axis) > 0.0
            alphas = np.where(again, 1.0, alphas)
            nxt = (1.0 + np.sqrt(4.0 * alphas * alphas + 1.0)) / 2.0
            w = (alphas - 1.0) / nxt
            Y = Z + (w[:, None] if side == "G" else w[None, :]) * (Z - Zprev)
            alphas = nxt
        else:
            alpha_next = (1.0 + math.sqrt(4.0 * alpha * alpha + 1.0)) / 2.0
            Y = Z + ((alpha - 1.0) / alpha_next) * (Z - Zprev)
            alpha = alpha_next
        Zprev = Z
        if forced_steps is None or pg_trace is not None:
            pg = pg_norm(Z, W, B, side)
            if pg_trace is not None:
                pg_trace.append(pg)
            if forced_steps is None and k >= inner_min and pg <= tol:
                break
    return Z, k, L


def hals_update(Z0, W, B, side: str, sweeps: int):
    """HALS (Sec. 1 lists it among the classical NMF solvers; the compressed
    form is the randomized HALS that Sec. 1 cites): ``sweeps`` passes over
    the p coordinates in order, each coordinate set to the exact minimiser
    of the subproblem in it with the others fixed, then clipped at 0:
        z_j <- max(0, z_j - grad_j(z) / W_jj)
    for every row of G (every column of F), with the gradient of the current
    point.  A coordinate with W_jj = 0 is left unchanged."""
    Z = np.asarray(Z0, dtype=F64).copy()
    W = np.asarray(W, dtype=F64)
    B = np.asarray(B, dtype=F64)
    p = W.shape[0]
    for _ in range(sweeps):
        for j in range(p):
            if not W[j, j] > 0.0:
                continue
            if side == "G":
                g = Z @ W[:, j] - B[:, j]
                Z[:, j] = np.maximum(Z[:, j] - g / W[j, j], 0.0)
            else:
                g = W[j, :] @ Z - B[j, :]
                Z[j, :] = np.maximum(Z[j, :] - g / W[j, j], 0.0)
    return Z


def mu_update(Z0, W, B, side: str, iters: int):
    """Multiplicative updates for the subproblem when W and B may have
    negative entries (the compressed data of Algorithm 1 are instances of
    semi-NMF, Sec. 3, after Ding et al.): with A+ = max(A, 0) and
    A- = max(-A, 0) entrywise,
        Z <- Z * sqrt((B+ + Z W-) / (B- + Z W+))      (G side; F: W- Z, W+ Z),
    ``iters`` times.  A zero denominator leaves that entry unchanged."""
    Z = np.asarray(Z0, dtype=F64).copy()
    W = np.asarray(W, dtype=F64)
    B = np.asarray(B, dtype=F64)
    Wp, Wn = np.maximum(W, 0.0), np.maximum(-W, 0.0)
    Bp, Bn = np.maximum(B, 0.0), np.maximum(-B, 0.0)
    for _ in range(iters):
        if side == "G":
            num, den = Bp + Z @ Wn, Bn + Z @ Wp
        else:
            num, den = Bp + Wn @ Z, Bn + Wp @ Z
        ratio = np.divide(num, den, out=np.ones_like(num), where=den > 0.0)
        Z = Z * np.sqrt(ratio)
    return Z


def subproblem_objective(Z, W, B, side: str) -> float:
    """0.5 tr(Z^T Z W) - tr(B^T Z) (G) or 0.5 tr(Z^T W Z) - tr(B^T Z) (F):
    ||X - G F||^2 / 2 in the free factor, up to a constant."""
    Z = np.asarray(Z, dtype=F64)
    W = np.asarray(W, dtype=F64)
    B = np.asarray(B, dtype=F64)
    if side == "G":
        return float(0.5 * np.sum((Z @ W) * Z) - np.sum(B * Z))
    return float(0.5 * np.sum((W @ Z) * Z) - np.sum(B * Z))


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
    pg: list = field(default_factory=list)   # [t][side] norms at every inner step (if kept)


def nenmf(X, G0, F0, outer_iters: int, inner_max: int, inner_min: int = 1,
          ratio: float = 1e-3, stop_rule: str = STOP_GLOBAL,
          compressed: RSIResult | None = None, replay=None,
          keep_history: bool = False, keep_pg: bool = False,
          solver: str = "nesterov", restart: bool = False, on_outer=None) -> NeNMFResult:
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
    ``replay`` (T x 2 ints) forces the inner step counts; a negative entry
    leaves that inner loop to the gradient bound.  ``keep_pg`` records the
    projected-gradient norm at every inner step of every subproblem.
    ``solver``: "nesterov" (Sec. 2), or "hals" / "mu", which take exactly
    inner_max updates per subproblem (or the replayed count) and no bound.
    ``restart``: adaptive restart of the Nesterov loops (see nesterov_nnls).
    ``on_outer(t, G, F)`` is called after every outer iteration (timing).
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
    pgs = []

    def forced_at(t, side):
        if replay is None or int(replay[t][side]) < 0:
            return None
        return int(replay[t][side])

    if solver not in ("nesterov", "hals", "mu"):
        raise ValueError(solver)

    def update(Z, W, B, side, tol_, forced, trace):
        if solver == "nesterov":
            return nesterov_nnls(Z, W, B, side, tol_, inner_max, inner_min, forced, trace,
                                 restart=restart)
        k = inner_max if forced is None else forced
        fn = hals_update if solver == "hals" else mu_update
        return fn(Z, W, B, side, k), k, 0.0

    for t in range(outer_iters):
        tr_g = [] if keep_pg else None
        tr_f = [] if keep_pg else None
        W, B = gdata(F)
        tg = tol_g if stop_rule == STOP_GLOBAL else ratio * pg_norm(G, W, B, "G")
        tols[t, 0] = tg
        G, kg, lg = update(G, W, B, "G", tg, forced_at(t, 0), tr_g)
        if stop_rule == STOP_GLOBAL and solver == "nesterov" and 1 <= kg <= inner_min:
            tol_g /= 10.0
        W, B = fdata(G)
        tf = tol_f if stop_rule == STOP_GLOBAL else ratio * pg_norm(F, W, B, "F")
        tols[t, 1] = tf
        F, kf, lf = update(F, W, B, "F", tf, forced_at(t, 1), tr_f)
        if stop_rule == STOP_GLOBAL and solver == "nesterov" and 1 <= kf <= inner_min:
            tol_f /= 10.0
        steps[t] = (kg, kf)
        lips[t] = (lg, lf)
        if keep_history:
            hist.append((G.copy(), F.copy()))
        if keep_pg:
            pgs.append((tr_g, tr_f))
        if on_outer is not None:
            on_outer(t, G, F)
    return NeNMFResult(G=G, F=F, steps=steps, lips=lips, tols=tols, tol0=tol0,
                       history=hist, pg=pgs)


# ---------------------------------------------------------------------------
# Measurement (Sec. 4)
# ---------------------------------------------------------------------------

def rre(X, G, F) -> float:
    """Relative reconstruction error ||X - G F||_F / ||X||_F, Sec. 4, Eq. (4)."""
    X = np.asarray(X, dtype=F64)
    R = X - np.asarray(G, dtype=F64) @ np.asarray(F, dtype=F64)
    return float(np.linalg.norm(R) / np.linalg.norm(X))


def rre_expanded(X, G, F, x_norm2: float | None = None) -> float:
    """The same error from ||X||^2 - 2 <G^T X, F> + <G^T G, F F^T>, all in
    FP64: one product G^T X instead of the n x m residual, for large X (the
    expansion loses about eps64 ||X||^2 / ||X - G F||^2 relative, far below
    FP32 resolution at any error level met here)."""
    X = np.asarray(X)
    G = np.asarray(G, dtype=F64)
    F = np.asarray(F, dtype=F64)
    if x_norm2 is None:
        x_norm2 = float(np.einsum("ij,ij->", X, X, dtype=F64))
    GtX = (X.T @ G).T if X.dtype == F64 else (np.asarray(X, dtype=F64).T @ G).T
    cross = float(np.sum(GtX * F))
    quad = float(np.sum((G.T @ G) * (F @ F.T)))
    r2 = max(x_norm2 - 2.0 * cross + quad, 0.0)
    return math.sqrt(r2 / x_norm2)


def rre_history(X, history, chunk: int = 48) -> np.ndarray:
    """rre_expanded for every (G_t, F_t) of a history, with the products
    G_t^T X of up to ``chunk`` snapshots formed in one pass over X."""
    X = np.asarray(X)
    Xd = X if X.dtype == F64 else X.astype(F64)
    x_norm2 = float(np.einsum("ij,ij->", Xd, Xd))
    out = np.empty(len(history), dtype=F64)
    for c0 in range(0, len(history), chunk):
        part = history[c0:c0 + chunk]
        Gs = np.concatenate([np.asarray(g, dtype=F64) for g, _ in part], axis=1)
        XtG = Xd.T @ Gs                                  # m x (count p)
        col = 0
        for i, (g, f) in enumerate(part):
            g = np.asarray(g, dtype=F64)
            f = np.asarray(f, dtype=F64)
            p = g.shape[1]
            cross = float(np.sum(XtG[:, col:col + p].T * f))
            col += p
            quad = float(np.sum((g.T @ g) * (f @ f.T)))
            out[c0 + i] = math.sqrt(max(x_norm2 - 2.0 * cross + quad, 0.0) / x_norm2)
    return out


def svd_floor(X, p: int) -> float:
    """Smallest RRE any rank-p factorisation can reach (truncated SVD), for
    small matrices by a full SVD."""
    X = np.asarray(X, dtype=F64)
    s = np.linalg.svd(X, compute_uv=False)
    return float(math.sqrt(float(np.sum(s[p:] ** 2))) / math.sqrt(float(np.sum(s ** 2))))
