"""Pins for the oracle's variants: the plain Gaussian random projection and
randomized power iteration without re-orthonormalisation (Sec. 3), HALS and
multiplicative updates on the (semi-NMF) subproblems (Sec. 1, Sec. 3), and
adaptive restart of the Nesterov loop (Sec. 4 footnote)."""
import numpy as np
import pytest
from scipy.optimize import nnls

import oracle


def _orthonormal(rng, n, k):
    q, r = np.linalg.qr(rng.standard_normal((n, k)))
    return q * np.sign(np.diag(r))


def _proj(Q):
    return Q @ np.linalg.pinv(Q)


# ---------------------------------------------------------------- Gaussian RP

def test_gaussian_projection_is_unbiased():
    """With L = Omega / sqrt(nu): E[R R^T] = I and E[L^T L] = I, hence
    E[X_R X_R^T] = X X^T and E[X_L^T X_L] = X^T X (averages over 600 draws
    against CLT bounds; the scale 1/nu or no scale would miss by 10x)."""
    rng = np.random.default_rng(0)
    n, m, ell = 14, 12, 8
    X = rng.random((n, m))
    draws = 600
    acc_r = np.zeros((m, m))
    acc_l = np.zeros((n, n))
    acc_xr = np.zeros((n, n))
    acc_xl = np.zeros((m, m))
    for _ in range(draws):
        c = oracle.compress_gaussian(X, rng.standard_normal((m, ell)),
                                     rng.standard_normal((ell, n)))
        assert c.Q_R.shape == (m, ell) and c.Q_L.shape == (n, ell)
        assert c.X_R.shape == (n, ell) and c.X_L.shape == (ell, m)
        acc_r += c.Q_R @ c.Q_R.T
        acc_l += c.Q_L @ c.Q_L.T
        acc_xr += c.X_R @ c.X_R.T
        acc_xl += c.X_L.T @ c.X_L
    # entries of R R^T have variance <= 2 / l; six standard errors
    bound = 6 * np.sqrt(2.0 / ell / draws)
    assert np.max(np.abs(acc_r / draws - np.eye(m))) <= bound
    assert np.max(np.abs(acc_l / draws - np.eye(n))) <= bound
    XXt, XtX = X @ X.T, X.T @ X
    assert np.linalg.norm(acc_xr / draws - XXt) <= 6 * np.linalg.norm(XXt) * np.sqrt(2.0 / ell / draws)
    assert np.linalg.norm(acc_xl / draws - XtX) <= 6 * np.linalg.norm(XtX) * np.sqrt(2.0 / ell / draws)


# ------------------------------------------------------- randomized power iteration

@pytest.mark.parametrize("q", [1, 2])
def test_power_iteration_closed_form_range(q):
    """X = U diag(s) V^T built from its SVD: (X^T X)^q Omega_L = V diag(s^2q)
    V^T Omega_L and (X X^T)^q Omega_R^T = U diag(s^2q) U^T Omega_R^T, so the
    bases must span these closed-form panels."""
    rng = np.random.default_rng(q)
    n, m, r, ell = 60, 45, 12, 8
    U, V = _orthonormal(rng, n, r), _orthonormal(rng, m, r)
    s = np.linspace(3.0, 1.0, r)
    X = U @ np.diag(s) @ V.T
    oL = rng.standard_normal((m, ell))
    oR = rng.standard_normal((ell, n))
    c = oracle.compress_power(X, oL, oR, q)
    right = V @ np.diag(s ** (2 * q)) @ V.T @ oL
    left = U @ np.diag(s ** (2 * q)) @ U.T @ oR.T
    assert np.linalg.norm(_proj(c.Q_R) - _proj(right)) <= 1e-10
    assert np.linalg.norm(_proj(c.Q_L) - _proj(left)) <= 1e-10
    assert np.linalg.norm(c.Q_R.T @ c.Q_R - np.eye(ell)) <= 1e-12


def test_power_iteration_spans_the_subspace_iteration_range():
    """Power iteration and subspace iteration (Algorithm 2) reach the same
    subspaces in exact arithmetic; on a well-conditioned X (singular values
    between 1 and 2, so no direction drowns in roundoff) the FP64 results
    agree."""
    rng = np.random.default_rng(4)
    n, m, ell, q, r = 80, 70, 10, 3, 20
    X = _orthonormal(rng, n, r) @ np.diag(np.linspace(2.0, 1.0, r)) @ _orthonormal(rng, m, r).T
    oL = rng.standard_normal((m, ell))
    oR = rng.standard_normal((ell, n))
    a = oracle.compress_power(X, oL, oR, q)
    b = oracle.rsi(X, oL, oR, q)
    assert np.linalg.norm(_proj(a.Q_R) - _proj(b.Q_R)) <= 1e-8
    assert np.linalg.norm(_proj(a.Q_L) - _proj(b.Q_L)) <= 1e-8


def test_power_iteration_exact_for_low_rank():
    """rank(X) <= l with singular values within a factor 2: the range finder
    captures X exactly (the columns beyond the rank are replaced from the
    Gaussian pool).  Widely spread singular values would let the weakest
    directions fall under the rank threshold after the powers, the known
    weakness of the method without re-orthonormalisation."""
    rng = np.random.default_rng(5)
    n, m, r, ell = 50, 40, 4, 9
    X = _orthonormal(rng, n, r) @ np.diag([2.0, 1.7, 1.3, 1.0]) @ _orthonormal(rng, m, r).T
    c = oracle.compress_power(X, rng.standard_normal((m, ell)), rng.standard_normal((ell, n)), 2)
    assert np.linalg.norm(X - c.Q_L @ c.X_L) <= 1e-10 * np.linalg.norm(X)
    assert np.linalg.norm(X - c.X_R @ c.Q_R.T) <= 1e-10 * np.linalg.norm(X)
    assert sum(int(f.sum()) for _, f in c.replaced) == 2 * (ell - r)


# ---------------------------------------------------------------- HALS and MU

def _problem(rng, rows, p, interior=False, signed=False):
    A = rng.random((3 * p, p))
    if signed:
        A = A - 0.35
    W = A.T @ A
    if interior:
        Zs = 0.5 + rng.random((rows, p))
        B = Zs @ W
    else:
        B = rng.random((rows, 3 * p)) @ A
    return W, B, rng.random((rows, p))


def test_hals_one_coordinate_is_exact():
    rng = np.random.default_rng(0)
    W = np.array([[2.5]])
    B = rng.standard_normal((6, 1))
    Z = oracle.hals_update(rng.random((6, 1)), W, B, "G", 1)
    np.testing.assert_allclose(Z, np.maximum(B / 2.5, 0.0), rtol=0, atol=1e-15)


@pytest.mark.parametrize("side", ["G", "F"])
def test_hals_converges_to_nnls(side):
    rng = np.random.default_rng(1)
    W, B, Z0 = _problem(rng, 7, 5)
    if side == "F":
        B, Z0 = B.T.copy(), Z0.T.copy()
    Z = oracle.hals_update(Z0, W, B, side, 3000)
    A = np.linalg.cholesky(W).T            # W = A^T A
    for r in range(7):
        b = B[r] if side == "G" else B[:, r]
        x, _ = nnls(A, np.linalg.solve(A.T, b))
        got = Z[r] if side == "G" else Z[:, r]
        np.testing.assert_allclose(got, x, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("fn", ["hals", "mu"])
def test_updates_never_increase_the_objective(fn):
    """HALS minimises exactly along each coordinate; the semi-NMF
    multiplicative rule is non-increasing (Ding et al.), also with signed
    W and B as in the compressed subproblems."""
    rng = np.random.default_rng(2)
    W, B, Z = _problem(rng, 20, 6, signed=True)
    f = oracle.hals_update if fn == "hals" else oracle.mu_update
    prev = oracle.subproblem_objective(Z, W, B, "G")
    for _ in range(60):
        Z = f(Z, W, B, "G", 1)
        cur = oracle.subproblem_objective(Z, W, B, "G")
        assert cur <= prev + 1e-12 * abs(prev)
        assert np.all(Z >= 0)
        prev = cur


def test_mu_fixed_point_is_the_interior_solution():
    """An interior solution Z* = B W^-1 > 0 is a fixed point of the
    multiplicative rule, and the iteration converges to it (signed W)."""
    rng = np.random.default_rng(3)
    W, B, Z0 = _problem(rng, 5, 3, interior=True, signed=True)
    Zs = np.linalg.solve(W, B.T).T
    assert np.all(Zs > 0)
    np.testing.assert_allclose(oracle.mu_update(Zs, W, B, "G", 1), Zs, rtol=1e-12)
    Z = oracle.mu_update(Z0, W, B, "G", 20000)
    np.testing.assert_allclose(Z, Zs, rtol=1e-6)


def test_mu_keeps_zeros():
    rng = np.random.default_rng(4)
    W, B, Z0 = _problem(rng, 6, 4, signed=True)
    Z0[2, 1] = 0.0
    assert oracle.mu_update(Z0, W, B, "G", 25)[2, 1] == 0.0


# ------------------------------------------------------------- adaptive restart

def test_restart_rows_are_independent():
    """The restart state is per row (G) or per column (F): solving rows
    together equals solving each row alone, for a fixed step count."""
    rng = np.random.default_rng(6)
    A = rng.random((12, 5)) @ np.diag([1, 1, 1, 1, 30])
    W = A.T @ A
    B = rng.random((4, 12)) @ A
    Z0 = rng.random((4, 5))
    Z, _, _ = oracle.nesterov_nnls(Z0, W, B, "G", 0.0, 40, forced_steps=40, restart=True)
    for r in range(4):
        Zr, _, _ = oracle.nesterov_nnls(Z0[r:r + 1], W, B[r:r + 1], "G", 0.0, 40,
                                        forced_steps=40, restart=True)
        np.testing.assert_allclose(Z[r], Zr[0], rtol=1e-13, atol=1e-15)
    Zf, _, _ = oracle.nesterov_nnls(Z0.T, W, B.T, "F", 0.0, 40, forced_steps=40, restart=True)
    np.testing.assert_allclose(Zf, Z.T, rtol=1e-13, atol=1e-15)


def test_restart_speeds_up_ill_conditioned_problems():
    """On ill-conditioned subproblems momentum overshoots; restarting it
    (O'Donoghue and Candes) reaches a tight bound in fewer steps and at the
    same objective value."""
    rng = np.random.default_rng(7)
    A = rng.random((40, 8)) @ np.diag(np.geomspace(1, 50, 8))
    W = A.T @ A
    B = rng.random((30, 40)) @ A
    Z0 = rng.random((30, 8))
    tol = 1e-9 * oracle.pg_norm(Z0, W, B, "G")
    Za, ka, _ = oracle.nesterov_nnls(Z0, W, B, "G", tol, 100000)
    Zb, kb, _ = oracle.nesterov_nnls(Z0, W, B, "G", tol, 100000, restart=True)
    assert kb < 0.7 * ka, (ka, kb)
    fa = oracle.subproblem_objective(Za, W, B, "G")
    fb = oracle.subproblem_objective(Zb, W, B, "G")
    assert abs(fa - fb) <= 1e-9 * abs(fa)
