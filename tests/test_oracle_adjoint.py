"""Pins of the FP64 reference gradient (differentiation form): its forward
equals the numpy oracle, and its gradient equals central differences."""
import numpy as np
import pytest

import oracle
import synth


def _setup(n=60, m=45, p=3, nu=5, seed=3):
    inst = synth.instance(n, m, p, nu, seed=seed, snr_db=30.0)
    rng = np.random.default_rng(seed + 7)
    Gt = rng.random(inst.G0.shape)
    Ft = rng.random(inst.F0.shape)
    return inst, Gt, Ft


def test_forward_equals_numpy_oracle():
    import torch
    inst, _, _ = _setup()
    q, T, K = 2, 4, 5
    G, F = oracle.adjoint.unrolled(torch.as_tensor(inst.X.astype(np.float64)), inst.omega_L,
                                   inst.omega_R, torch.as_tensor(inst.G0.astype(np.float64)),
                                   torch.as_tensor(inst.F0.astype(np.float64)), q, T, K)
    comp = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, q)
    ref = oracle.nenmf(inst.X, inst.G0, inst.F0, T, K, compressed=comp,
                       replay=np.full((T, 2), K))
    assert np.allclose(G.numpy(), ref.G, rtol=0, atol=1e-9 * np.abs(ref.G).max())
    assert np.allclose(F.numpy(), ref.F, rtol=0, atol=1e-9 * np.abs(ref.F).max())


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    inst, Gt, Ft = _setup(seed=seed)
    q, T, K = 2, 3, 5
    Lv, gX, gG, gF = oracle.adjoint.loss_grad(inst.X, inst.omega_L, inst.omega_R, inst.G0,
                                              inst.F0, Gt, Ft, q, T, K)
    rng = np.random.default_rng(seed)
    h = 1e-6
    X = inst.X.astype(np.float64)
    for _ in range(3):
        D = rng.standard_normal(X.shape)
        D *= np.linalg.norm(X) / np.linalg.norm(D)
        lp = oracle.adjoint.loss(X + h * D, inst.omega_L, inst.omega_R, inst.G0, inst.F0, Gt,
                                 Ft, q, T, K)
        lm = oracle.adjoint.loss(X - h * D, inst.omega_L, inst.omega_R, inst.G0, inst.F0, Gt,
                                 Ft, q, T, K)
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(gX * D))
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3 * Lv)
    # and in G0
    D = rng.standard_normal(inst.G0.shape)
    lp = oracle.adjoint.loss(X, inst.omega_L, inst.omega_R, inst.G0 + h * D, inst.F0, Gt, Ft, q, T, K)
    lm = oracle.adjoint.loss(X, inst.omega_L, inst.omega_R, inst.G0 - h * D, inst.F0, Gt, Ft, q, T, K)
    assert abs((lp - lm) / (2 * h) - float(np.sum(gG * D))) <= 1e-6 * abs(Lv)


def test_deficient_basis_has_no_derivative():
    import torch
    inst = synth.instance(40, 30, 2, 6, seed=1)     # exactly rank 2 < l = 8
    with pytest.raises(ValueError):
        oracle.adjoint.rsi(torch.as_tensor(inst.X.astype(np.float64)), inst.omega_L,
                           inst.omega_R, 2)
