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
