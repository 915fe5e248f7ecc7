"""Pins for the oracle's outer loops: plain NeNMF (Sec. 2) and compressed
NeNMF (Algorithm 1), by identities that the mathematics fixes.
"""
import numpy as np
import pytest

import oracle
import synth


def test_compressed_equals_plain_with_square_orthogonal_bases():
    """l = n = m makes Q_L, Q_R square orthogonal, so Algorithm 1's
    subproblems coincide with Eqs. (2)-(3) and so do all iterates."""
    inst = synth.instance(12, 12, 3, 9, seed=0, snr_db=20.0)   # l = 12
    r = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 2)
    assert np.linalg.norm(r.Q_L @ r.Q_L.T - np.eye(12)) < 1e-12
    kw = dict(outer_iters=15, inner_max=30)
    a = oracle.nenmf(inst.X, inst.G0, inst.F0, compressed=r, **kw)
    b = oracle.nenmf(inst.X, inst.G0, inst.F0, **kw)
    assert np.array_equal(a.steps, b.steps)
    np.testing.assert_allclose(a.G, b.G, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(a.F, b.F, rtol=1e-9, atol=1e-11)


def test_planted_recovery_noiseless():
    """Noiseless X = G* F*: the reconstruction error goes to the FP32
    rounding level of X (~2e-8 here); the factors themselves are not unique."""
    ok = 0
    for seed in range(10):
        inst = synth.instance(40, 30, 3, 5, seed=seed)
        res = oracle.nenmf(inst.X, inst.G0, inst.F0, 2000, 500, ratio=1e-9)
        if oracle.rre(inst.X, res.G, res.F) <= 1e-6:
            ok += 1
    assert ok >= 8


def test_rre_bounded_below_by_svd_floor():
    """No rank-p factorisation beats the truncated SVD (Eckart-Young)."""
    inst = synth.instance(60, 50, 4, 6, seed=1, snr_db=20.0)
    floor = oracle.svd_floor(inst.X, 4)
    res = oracle.nenmf(inst.X, inst.G0, inst.F0, 200, 100, keep_history=True)
    errs = [oracle.rre(inst.X, g, f) for g, f in res.history]
    assert min(errs) >= floor - 1e-12
    assert errs[-1] <= floor * 1.02


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plain_rre_monotone_small_instance(seed):
    inst = synth.instance(200, 150, 5, 10, seed=seed)
    res = oracle.nenmf(inst.X, inst.G0, inst.F0, 20, 10, keep_history=True)
    errs = [oracle.rre(inst.X, g, f) for g, f in res.history]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:]))


def test_rre_definition():
    rng = np.random.default_rng(3)
    X = rng.random((5, 4))
    G = rng.random((5, 2))
    F = rng.random((2, 4))
    R = X - G @ F
    assert abs(oracle.rre(X, G, F) - np.sqrt((R ** 2).sum() / (X ** 2).sum())) < 1e-15


def test_global_tolerance_division():
    """Global rule: a factor's tolerance drops tenfold after an inner loop
    that stops within inner_min steps, and only then."""
    inst = synth.instance(30, 20, 3, 3, seed=4, snr_db=30.0)
    res = oracle.nenmf(inst.X, inst.G0, inst.F0, 40, 50, ratio=1e-1)
    for t in range(1, 40):
        for s in range(2):
            expect = res.tols[t - 1, s] / 10 if res.steps[t - 1, s] <= 1 else res.tols[t - 1, s]
            assert res.tols[t, s] == expect
    assert (res.steps[:, 0] == 1).any() or (res.steps[:, 1] == 1).any()


def test_replay_reproduces_counts():
    inst = synth.instance(30, 25, 3, 4, seed=5, snr_db=30.0)
    a = oracle.nenmf(inst.X, inst.G0, inst.F0, 10, 40)
    b = oracle.nenmf(inst.X, inst.G0, inst.F0, 10, 40, replay=a.steps)
    assert np.array_equal(a.steps, b.steps)
    np.testing.assert_array_equal(a.G, b.G)


def test_compressed_small_instance_reaches_low_error():
    inst = synth.instance(200, 150, 5, 10, seed=0)
    r = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 4)
    res = oracle.nenmf(inst.X, inst.G0, inst.F0, 300, 100, compressed=r, ratio=1e-6)
    assert oracle.rre(inst.X, res.G, res.F) < 1e-3


_BOUND_X = np.array([[1, 0, 1], [0, 3, 1]], dtype=np.float32)
_BOUND_G0 = np.array([[1, 0], [2, 1]], dtype=np.float32)
_BOUND_F0 = np.array([[1, 1, 0], [0, 2, 1]], dtype=np.float32)


def test_gradient_bounds_hand_derived():
    """The gradient bounds of both stop rules on a 2 x 3, p = 2 problem
    derived by hand (tests/golden/gradient_bounds.txt): the global bound uses
    the projected gradients of both factors at (G0, F0) (leaving out the F
    part, or not projecting, gives another value); the per-subproblem bound
    uses the factor's own projected gradient at the start of its loop."""
    from conftest import read_golden
    g = read_golden("gradient_bounds.txt")
    res = oracle.nenmf(_BOUND_X, _BOUND_G0, _BOUND_F0, 1, 5)
    assert abs(res.tol0 - g["tol0_global"]) <= 1e-15
    assert abs(res.tols[0, 0] - g["tol0_global"]) <= 1e-15
    assert abs(res.tols[0, 1] - g["tol0_global"]) <= 1e-15
    sub = oracle.nenmf(_BOUND_X, _BOUND_G0, _BOUND_F0, 1, 5, stop_rule="subproblem",
                       replay=[[0, 0]])
    assert abs(sub.tols[0, 0] - g["tol_subproblem_G"]) <= 1e-15
    assert abs(sub.tols[0, 1] - g["tol_subproblem_F"]) <= 1e-15


def test_partial_replay_and_norm_trace():
    """A negative replay entry leaves that loop to the bound; the recorded
    norms are those of the iterates (the last one of a free loop is the
    first at or below its bound)."""
    inst = synth.instance(30, 25, 3, 4, seed=6, snr_db=30.0)
    a = oracle.nenmf(inst.X, inst.G0, inst.F0, 6, 40, keep_pg=True)
    rep = -np.ones((6, 2), dtype=int)
    rep[2, 1] = a.steps[2, 1] + 1
    b = oracle.nenmf(inst.X, inst.G0, inst.F0, 6, 40, replay=rep, keep_pg=True)
    assert np.array_equal(a.steps[:2], b.steps[:2]) and a.steps[2, 0] == b.steps[2, 0]
    assert b.steps[2, 1] == a.steps[2, 1] + 1
    for t in range(6):
        for s in range(2):
            trace = a.pg[t][s]
            assert len(trace) == a.steps[t, s]
            assert trace[-1] <= a.tols[t, s] or a.steps[t, s] == 40
            assert all(v > a.tols[t, s] for v in trace[:-1])


def test_rre_expanded_equals_direct():
    """The expanded residual norm equals the direct one (Sec. 4, Eq. (4))."""
    rng = np.random.default_rng(8)
    for n, m, p in ((7, 5, 2), (60, 40, 6), (300, 200, 15)):
        X = rng.random((n, m)).astype(np.float32)
        G = rng.random((n, p))
        F = rng.random((p, m)) / p
        assert abs(oracle.rre_expanded(X, G, F) - oracle.rre(X, G, F)) <= 1e-12


def test_rre_history_equals_direct():
    rng = np.random.default_rng(9)
    X = rng.random((80, 60)).astype(np.float32)
    hist = [(rng.random((80, 4)), rng.random((4, 60)) / 4) for _ in range(7)]
    got = oracle.rre_history(X, hist, chunk=3)
    for e, (g, f) in zip(got, hist):
        assert abs(e - oracle.rre(X, g, f)) <= 1e-12
