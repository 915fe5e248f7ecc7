"""Pins for the oracle's orthonormalisation and randomized subspace
iteration (Sec. 3, Algorithm 2): LAPACK QR, exact low-rank range finding,
closed-form ranges for q = 1, convergence to the dominant singular subspace,
and the numerical-rank replacement rule on constructed rank-deficient panels.
"""
import numpy as np
import pytest

import oracle


def _sign_fixed_qr(Y):
    Q, R = np.linalg.qr(Y)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s, (R.T * s).T


def _proj(Q):
    return Q @ Q.T


def test_orth_matches_lapack_full_rank():
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((50, 9)) @ np.diag(np.geomspace(1, 1e-3, 9))
    P = rng.standard_normal((50, 9))
    Q, rep = oracle.orth(Y, P)
    Ql, Rl = _sign_fixed_qr(Y)
    assert not rep.any()
    np.testing.assert_allclose(Q, Ql, atol=1e-12)
    assert np.linalg.norm(Q.T @ Q - np.eye(9)) <= 1e-12
    R = Q.T @ Y
    assert np.all(np.diag(R) > 0)
    np.testing.assert_allclose(np.tril(R, -1), 0, atol=1e-12)
    np.testing.assert_allclose(Q @ np.triu(R), Y, atol=1e-12)


def test_orth_replaces_dependent_columns_by_pool():
    rng = np.random.default_rng(1)
    N = 40
    Y = rng.standard_normal((N, 6))
    Y[:, 3] = 2.0 * Y[:, 0] - Y[:, 1]          # exactly dependent
    Y[:, 5] = 0.0                               # zero column
    P = rng.standard_normal((N, 6))
    Q, rep = oracle.orth(Y, P)
    assert rep.tolist() == [False, False, False, True, False, True]
    M = Y.copy()
    M[:, 3] = P[:, 3]
    M[:, 5] = P[:, 5]
    np.testing.assert_allclose(Q, _sign_fixed_qr(M)[0], atol=1e-11)


def test_orth_threshold_is_relative_to_largest_column():
    """A column that is pure roundoff (tiny compared with the panel) counts
    as deficient even though it is independent of the columns before it."""
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((30, 3))
    Y[:, 2] = 1e-8 * rng.standard_normal(30)
    P = rng.standard_normal((30, 3))
    _, rep = oracle.orth(Y, P, tau2=1e-9)
    assert rep.tolist() == [False, False, True]
    Y[:, 2] *= 1e5                               # now 1e-3 of the panel: kept
    _, rep = oracle.orth(Y, P, tau2=1e-9)
    assert rep.tolist() == [False, False, False]


def test_orth_breakdown():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((20, 3))
    Y[:, 2] = Y[:, 0]
    P = rng.standard_normal((20, 3))
    P[:, 2] = Y[:, 1] + Y[:, 0]
    with pytest.raises(oracle.OrthBreakdown):
        oracle.orth(Y, P)


def _low_rank(rng, n, m, r):
    return rng.random((n, r)) @ rng.random((r, m))   # FP64, exact rank r


@pytest.mark.parametrize("q", [1, 2, 4])
def test_rsi_exact_for_low_rank(q):
    rng = np.random.default_rng(4)
    n, m, r, ell = 60, 45, 4, 9
    X = _low_rank(rng, n, m, r)
    oL = rng.standard_normal((m, ell))
    oR = rng.standard_normal((ell, n))
    res = oracle.rsi(X, oL, oR, q)
    nx = np.linalg.norm(X)
    assert np.linalg.norm(X - res.Q_L @ (res.Q_L.T @ X)) <= 1e-12 * nx
    assert np.linalg.norm(X - (X @ res.Q_R) @ res.Q_R.T) <= 1e-12 * nx
    for Q in (res.Q_L, res.Q_R):
        assert np.linalg.norm(Q.T @ Q - np.eye(ell)) <= 1e-12
    np.testing.assert_allclose(res.X_L, res.Q_L.T @ X, atol=1e-12 * nx)
    np.testing.assert_allclose(res.X_R, X @ res.Q_R, atol=1e-12 * nx)
    # columns r..l-1 of every panel are numerically absent and get replaced
    for tag, rep in res.replaced:
        assert rep.tolist() == [False] * r + [True] * (ell - r), tag


def test_rsi_q1_closed_form_ranges():
    """q = 1: range(Q_R) = range(X^T X Omega_L), range(Q_L) = range(X X^T Omega_R^T)."""
    rng = np.random.default_rng(5)
    n, m, ell = 30, 25, 5
    X = rng.standard_normal((n, m))
    oL = rng.standard_normal((m, ell))
    oR = rng.standard_normal((ell, n))
    res = oracle.rsi(X, oL, oR, 1)
    QR_ref = np.linalg.qr(X.T @ (X @ oL))[0]
    QL_ref = np.linalg.qr(X @ (X.T @ oR.T))[0]
    np.testing.assert_allclose(_proj(res.Q_R), _proj(QR_ref), atol=1e-10)
    np.testing.assert_allclose(_proj(res.Q_L), _proj(QL_ref), atol=1e-10)


def test_rsi_converges_to_dominant_subspace():
    """With a spectral gap at p, the top-p singular subspaces fall inside the
    RSI ranges, faster for larger q."""
    rng = np.random.default_rng(6)
    n, m, p, ell = 80, 70, 4, 8
    U = np.linalg.qr(rng.standard_normal((n, n)))[0]
    V = np.linalg.qr(rng.standard_normal((m, m)))[0]
    s = np.concatenate([[100, 80, 60, 50], np.linspace(5, 1, m - 4)])
    X = U[:, :m] @ np.diag(s) @ V.T
    oL = rng.standard_normal((m, ell))
    oR = rng.standard_normal((ell, n))
    errs = []
    for q in (1, 2, 4):
        res = oracle.rsi(X, oL, oR, q)
        eR = np.linalg.norm(V[:, :p] - res.Q_R @ (res.Q_R.T @ V[:, :p]), 2)
        eL = np.linalg.norm(U[:, :p] - res.Q_L @ (res.Q_L.T @ U[:, :p]), 2)
        errs.append(max(eR, eL))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


def test_rsi_rejects_q0():
    with pytest.raises(ValueError):
        oracle.rsi(np.ones((4, 4)), np.ones((4, 2)), np.ones((2, 4)), 0)
