"""Pins for the oracle's Nesterov inner loop (Sec. 2) and its weights.

Every check here compares the oracle with something other than itself:
hand-derived closed forms, the alpha recursion's algebraic invariant, the
O(1/k^2) convergence theorem of accelerated projected gradient, scipy's NNLS
solver, brute-force active-set enumeration, and finite differences.
"""
import itertools
import math
import types

import numpy as np
import pytest
from scipy.optimize import nnls

import oracle
import importlib
onm = importlib.import_module("oracle.nenmf")
from conftest import read_golden


def test_alpha_closed_forms():
    g = read_golden("alpha_closed_form.txt")
    a = oracle.alpha_series(3)
    b = oracle.momentum_weights(3)
    assert a[0] == 1.0
    for k in (1, 2, 3):
        assert abs(a[k] - g[f"alpha_{k}"]) <= 1e-15 * g[f"alpha_{k}"]
        assert abs(b[k] - g[f"beta_{k}"]) <= 1e-15
    assert b[1] == 0.0


def test_alpha_invariant_and_bounds():
    K = 2000
    a = oracle.alpha_series(K)
    k = np.arange(K + 1)
    # alpha_{k+1} is the positive root of x^2 - x - alpha_k^2 = 0.
    np.testing.assert_allclose(a[1:] ** 2 - a[1:], a[:-1] ** 2, rtol=1e-13)
    assert np.all(a >= (k + 2) / 2 - 1e-12)
    assert np.all(a <= k + 1 + 1e-12)
    b = oracle.momentum_weights(K)
    assert np.all((b[1:] >= 0) & (b[1:] < 1))
    assert np.all(np.diff(b[1:]) > 0)


def _random_nnls(rng, rows, p, cond=1.0):
    A = rng.standard_normal((3 * p, p))
    U, _, Vt = np.linalg.svd(A, full_matrices=False)
    s = np.geomspace(1.0, 1.0 / cond, p)
    A = U @ np.diag(s) @ Vt                       # design with chosen spectrum
    Xrows = rng.standard_normal((rows, 3 * p))
    W = A.T @ A
    B = Xrows @ A
    return A, Xrows, W, B


def _nnls_rows(A, Xrows):
    return np.stack([nnls(A, x)[0] for x in Xrows])


def test_fixed_point_is_scipy_nnls_g_side():
    rng = np.random.default_rng(1)
    A, Xr, W, B = _random_nnls(rng, 12, 6, cond=5.0)
    Zs = _nnls_rows(A, Xr)
    Z, k, L = oracle.nesterov_nnls(np.ones((12, 6)), W, B, "G", tol=1e-13,
                                   inner_max=20000)
    np.testing.assert_allclose(Z, Zs, atol=1e-9)
    assert k < 20000


def test_fixed_point_is_scipy_nnls_f_side():
    rng = np.random.default_rng(2)
    A, Xr, W, B = _random_nnls(rng, 9, 5, cond=3.0)
    Zs = _nnls_rows(A, Xr).T                      # F side: columns are problems
    Z, k, L = oracle.nesterov_nnls(np.full((5, 9), 0.5), W, B.T, "F", tol=1e-13,
                                   inner_max=20000)
    np.testing.assert_allclose(Z, Zs, atol=1e-9)


def _brute_force_row(W, b):
    """min 0.5 z^T W z - b^T z over z >= 0 by enumerating active sets."""
    p = len(b)
    best, bestz = np.inf, None
    for r in range(p + 1):
        for S in itertools.combinations(range(p), r):
            z = np.zeros(p)
            if S:
                S = list(S)
                z[S] = np.linalg.solve(W[np.ix_(S, S)], b[S])
                if np.any(z[S] < 0):
                    continue
            g = W @ z - b
            if np.any(g[z == 0] < -1e-12):
                continue
            f = 0.5 * z @ W @ z - b @ z
            if f < best:
                best, bestz = f, z
    return bestz


def test_brute_force_active_sets():
    rng = np.random.default_rng(3)
    for p in (1, 2, 3, 4, 5):
        A, Xr, W, B = _random_nnls(rng, 6, p, cond=4.0)
        Zb = np.stack([_brute_force_row(W, b) for b in B])
        Z, _, _ = oracle.nesterov_nnls(np.zeros((6, p)) + 0.1, W, B, "G",
                                       tol=1e-13, inner_max=50000)
        np.testing.assert_allclose(Z, Zb, atol=1e-9)


def test_interior_solution_is_linear_solve():
    rng = np.random.default_rng(4)
    p = 4
    M = rng.standard_normal((p, p))
    W = M @ M.T + p * np.eye(p)
    Zstar = rng.random((7, p)) + 0.5                 # strictly positive
    B = Zstar @ W
    Z, _, _ = oracle.nesterov_nnls(np.ones((7, p)), W, B, "G", 1e-14, 20000)
    np.testing.assert_allclose(Z, np.linalg.solve(W, B.T).T, atol=1e-10)


def test_kkt_at_convergence():
    rng = np.random.default_rng(5)
    A, Xr, W, B = _random_nnls(rng, 20, 8, cond=10.0)
    Z, _, _ = oracle.nesterov_nnls(np.ones((20, 8)), W, B, "G", 1e-12, 100000)
    grad = Z @ W - B
    assert np.all(Z >= 0)
    assert np.abs(np.minimum(Z, grad)).max() <= 1e-10


def _fista_bound_holds(rng, nnls_fn, K=300):
    """Accelerated projected gradient with these weights satisfies
    f(Z_k) - f* <= 2 L ||Z_0 - Z*||^2 / (k + 1)^2 for every k."""
    A, Xr, W, B = _random_nnls(rng, 4, 6, cond=300.0)
    Zs = _nnls_rows(A, Xr)
    Z0 = np.ones_like(Zs) * 2.0

    def f(Z):
        return 0.5 * np.sum((Z @ W) * Z) - np.sum(B * Z)
    fstar = f(Zs)
    L = oracle.lipschitz(W)
    R2 = np.sum((Z0 - Zs) ** 2)
    ok = True
    for k in range(1, K + 1):
        Zk, steps, _ = nnls_fn(Z0, W, B, "G", 0.0, k, forced_steps=k)
        assert steps == k
        if f(Zk) - fstar > 2.0 * L * R2 / (k + 1) ** 2 + 1e-12:
            ok = False
            break
    return ok


def test_accelerated_rate_bound():
    assert _fista_bound_holds(np.random.default_rng(6), oracle.nesterov_nnls)


def test_rate_bound_catches_missing_momentum(monkeypatch):
    """Plant a mistake in the oracle (alpha stuck at 1 => no momentum): the
    plain projected gradient method then breaks the O(1/k^2) bound on an
    ill-conditioned problem, so the bound test has teeth."""
    fake = types.SimpleNamespace(sqrt=lambda x: 1.0)
    monkeypatch.setattr(onm, "math", fake)
    assert not _fista_bound_holds(np.random.default_rng(6), onm.nesterov_nnls)


def test_stop_is_first_step_below_tolerance():
    rng = np.random.default_rng(7)
    A, Xr, W, B = _random_nnls(rng, 10, 5, cond=20.0)
    Z0 = np.ones((10, 5))
    Zstop, k, _ = oracle.nesterov_nnls(Z0, W, B, "G", tol=1e-4, inner_max=10000)
    assert 1 < k < 10000
    assert oracle.pg_norm(Zstop, W, B, "G") <= 1e-4
    for j in range(1, k):
        Zj, _, _ = oracle.nesterov_nnls(Z0, W, B, "G", 0.0, 10000, forced_steps=j)
        assert oracle.pg_norm(Zj, W, B, "G") > 1e-4
    Zk, _, _ = oracle.nesterov_nnls(Z0, W, B, "G", 0.0, 10000, forced_steps=k)
    np.testing.assert_array_equal(Zk, Zstop)


def test_zero_lipschitz_leaves_factor():
    Z0 = np.arange(6.0).reshape(2, 3)
    Z, k, L = oracle.nesterov_nnls(Z0, np.zeros((3, 3)), np.ones((2, 3)), "G", 1e-3, 10)
    assert k == 0 and L == 0.0
    np.testing.assert_array_equal(Z, Z0)


def test_lipschitz_is_spectral_norm():
    rng = np.random.default_rng(8)
    M = rng.standard_normal((15, 40))
    W = M @ M.T
    assert abs(oracle.lipschitz(W) - np.linalg.norm(M, 2) ** 2) <= 1e-10 * oracle.lipschitz(W)


@pytest.mark.parametrize("side", ["G", "F"])
def test_gradient_matches_finite_differences(side):
    """grad of 0.5||X - G F||^2 in G (resp. F) by central differences."""
    rng = np.random.default_rng(9)
    n, m, p = 7, 6, 3
    X = rng.random((n, m))
    G = rng.random((n, p))
    F = rng.random((p, m))

    def obj(G_, F_):
        return 0.5 * np.sum((X - G_ @ F_) ** 2)
    if side == "G":
        W, B = oracle.g_data_plain(X, F)
        g = oracle.gradient(G, W, B, "G")
        Z = G
    else:
        W, B = oracle.f_data_plain(X, G)
        g = oracle.gradient(F, W, B, "F")
        Z = F
    h = 1e-6
    num = np.zeros_like(Z)
    for idx in np.ndindex(Z.shape):
        Zp = Z.copy(); Zp[idx] += h
        Zm = Z.copy(); Zm[idx] -= h
        if side == "G":
            num[idx] = (obj(Zp, F) - obj(Zm, F)) / (2 * h)
        else:
            num[idx] = (obj(G, Zp) - obj(G, Zm)) / (2 * h)
    np.testing.assert_allclose(g, num, atol=1e-7)


@pytest.mark.parametrize("side", ["G", "F"])
def test_compressed_gradient_matches_finite_differences(side):
    """Algorithm 1's compressed subproblems: 0.5||X_R - G F_R||^2 in G with
    F_R = F Q_R, and 0.5||X_L - G_L F||^2 in F with G_L = Q_L^T G."""
    rng = np.random.default_rng(10)
    n, m, p, ell = 8, 7, 2, 4
    X = rng.random((n, m))
    QL = np.linalg.qr(rng.standard_normal((n, ell)))[0]
    QR = np.linalg.qr(rng.standard_normal((m, ell)))[0]
    XL, XR = QL.T @ X, X @ QR
    G = rng.random((n, p))
    F = rng.random((p, m))
    h = 1e-6
    if side == "G":
        W, B = oracle.g_data_compressed(XR, QR, F)
        g = oracle.gradient(G, W, B, "G")

        def obj(Z):
            return 0.5 * np.sum((XR - Z @ (F @ QR)) ** 2)
        Z = G
    else:
        W, B = oracle.f_data_compressed(XL, QL, G)
        g = oracle.gradient(F, W, B, "F")

        def obj(Z):
            return 0.5 * np.sum((XL - (QL.T @ G) @ Z) ** 2)
        Z = F
    num = np.zeros_like(Z)
    for idx in np.ndindex(Z.shape):
        Zp = Z.copy(); Zp[idx] += h
        Zm = Z.copy(); Zm[idx] -= h
        num[idx] = (obj(Zp) - obj(Zm)) / (2 * h)
    np.testing.assert_allclose(g, num, atol=1e-7)


def test_projected_gradient_definition():
    Z = np.array([[0.0, 0.0, 1.0, 2.0]])
    g = np.array([[-1.0, 3.0, -2.0, 4.0]])
    np.testing.assert_array_equal(oracle.projected_gradient(Z, g), [[-1.0, 0.0, -2.0, 4.0]])
