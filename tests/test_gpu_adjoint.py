"""Differentiation form: the hand-written adjoint of unrolled compressed
NeNMF (through RSI, projections, momentum and L = lambda_max) against the
FP64 CPU reference gradient (torch autograd through an independent FP64
implementation) and against central differences of the GPU forward."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

cnmf = pytest.importorskip("paper_1812_04315_amd")


def _case(n, m, p, nu, seed):
    inst = synth.instance(n, m, p, nu, seed=seed, snr_db=30.0)
    rng = np.random.default_rng(seed + 99)
    Gt = rng.random(inst.G0.shape).astype(np.float32)
    Ft = rng.random(inst.F0.shape).astype(np.float32)
    return inst, Gt, Ft


def _loss64(G, F, Gt, Ft):
    """||G - Gt||^2 + ||F - Ft||^2 summed in FP64 on the host."""
    return float(np.sum((host(G) - Gt) ** 2) + np.sum((host(F) - Ft) ** 2))


def _gpu_loss_grad(inst, Gt, Ft, q, T, K, ckpt):
    import torch
    X = dev(inst.X, (inst.X.shape[1] + 3) // 4 * 4)
    G, F, tape = cnmf.adj_forward(X, dev(inst.omega_L), dev(inst.omega_R), dev(inst.G0),
                                  dev(inst.F0), p=inst.p, nu=inst.ell - inst.p, q=q,
                                  outer_iters=T, inner_steps=K, ckpt=ckpt)
    dG = 2 * (G - dev(Gt))
    dF = 2 * (F - dev(Ft))
    dX, dG0, dF0 = tape.backward(dG, dF)
    cnmf.check()
    Lv = float(torch.sum((G - dev(Gt)) ** 2) + torch.sum((F - dev(Ft)) ** 2))
    tape.close()
    return Lv, host(dX), host(dG0), host(dF0), host(G), host(F)


@pytest.mark.parametrize("n,m,p,nu,q,T,K,ckpt", [(60, 45, 3, 5, 2, 3, 5, 2),
                                                 (200, 150, 5, 10, 2, 6, 5, 4),
                                                 (300, 260, 10, 10, 2, 10, 5, 10),
                                                 (130, 110, 16, 4, 1, 3, 8, 2),
                                                 (170, 140, 21, 5, 1, 4, 6, 3)])
def test_adjoint_matches_fp64_reference(n, m, p, nu, q, T, K, ckpt):
    """Ranks up to 16 keep the reverse's iterates in LDS, wider ranks in an
    HBM tape; K = 8 is the longest inner loop the reverse supports; 130 and
    170 rows leave ragged last workgroups."""
    say("adjoint_ref", n, m, p, nu, q, T, K, ckpt)
    inst, Gt, Ft = _case(n, m, p, nu, seed=n)
    Lg, gX, gG, gF, G, F = _gpu_loss_grad(inst, Gt, Ft, q, T, K, ckpt)
    Lr, rX, rG, rF = oracle.adjoint.loss_grad(inst.X, inst.omega_L, inst.omega_R, inst.G0,
                                              inst.F0, Gt, Ft, q, T, K)
    assert abs(Lg - Lr) <= 1e-3 * Lr
    for g, r in ((gX, rX), (gG, rG), (gF, rF)):
        cos = float(np.sum(g * r) / (np.linalg.norm(g) * np.linalg.norm(r)))
        rel = float(np.linalg.norm(g - r) / np.linalg.norm(r))
        assert cos >= 0.999 and rel <= 1e-2, (cos, rel)


def test_adjoint_matches_gpu_central_differences():
    """32 random directions D (||D|| = ||X||), h = 1e-3: the directional
    derivative <dL/dX, D> against (L(X + hD) - L(X - hD)) / 2h of the GPU
    forward itself."""
    say("adjoint_fd")
    import torch
    n, m, p, nu, q, T, K = 200, 150, 5, 10, 2, 6, 5
    inst, Gt, Ft = _case(n, m, p, nu, seed=11)
    Lv, gX, _, _, _, _ = _gpu_loss_grad(inst, Gt, Ft, q, T, K, 3)
    rng = np.random.default_rng(5)
    X = inst.X.astype(np.float64)
    h = 1e-3
    fd, an = [], []
    for _ in range(32):
        D = rng.standard_normal(X.shape)
        D *= np.linalg.norm(X) / np.linalg.norm(D)
        vals = []
        for s in (1.0, -1.0):
            Xs = (X + s * h * D).astype(np.float32)
            G, F, tape = cnmf.adj_forward(dev(Xs, 152), dev(inst.omega_L), dev(inst.omega_R),
                                          dev(inst.G0), dev(inst.F0), p=p, nu=nu, q=q,
                                          outer_iters=T, inner_steps=K, ckpt=3)
            vals.append(_loss64(G, F, Gt, Ft))
            tape.close()
        fd.append((vals[0] - vals[1]) / (2 * h))
        an.append(float(np.sum(gX * D)))
    fd, an = np.array(fd), np.array(an)
    cos = float(fd @ an / (np.linalg.norm(fd) * np.linalg.norm(an)))
    rel = float(np.linalg.norm(fd - an) / np.linalg.norm(fd))
    assert cos >= 0.999 and rel <= 1e-2, (cos, rel)


def test_autograd_function():
    say("adjoint_autograd")
    import torch
    n, m, p, nu, q, T, K = 120, 100, 4, 6, 2, 4, 5
    inst, Gt, Ft = _case(n, m, p, nu, seed=21)
    X = dev(inst.X, 100).clone().requires_grad_(True)
    G0 = dev(inst.G0).requires_grad_(True)
    F0 = dev(inst.F0).requires_grad_(True)
    G, F = cnmf.compressed_nenmf(X, G0, F0, dev(inst.omega_L), dev(inst.omega_R), p=p, nu=nu,
                                 q=q, outer_iters=T, inner_steps=K, ckpt=2)
    loss = torch.sum((G - dev(Gt)) ** 2) + torch.sum((F - dev(Ft)) ** 2)
    loss.backward()
    cnmf.check()
    _, rX, rG, rF = oracle.adjoint.loss_grad(inst.X, inst.omega_L, inst.omega_R, inst.G0,
                                             inst.F0, Gt, Ft, q, T, K)
    for g, r in ((host(X.grad), rX), (host(G0.grad), rG), (host(F0.grad), rF)):
        assert np.linalg.norm(g - r) <= 1e-2 * np.linalg.norm(r)


def test_checkpoint_interval_does_not_change_the_gradient():
    say("adjoint_ckpt")
    inst, Gt, Ft = _case(150, 120, 4, 8, seed=31)
    a = _gpu_loss_grad(inst, Gt, Ft, 2, 8, 5, 1)
    b = _gpu_loss_grad(inst, Gt, Ft, 2, 8, 5, 8)
    c = _gpu_loss_grad(inst, Gt, Ft, 2, 8, 5, 3)
    for x, y in ((a, b), (a, c)):
        assert np.array_equal(x[1], y[1])


def test_adjoint_refuses_replaced_basis_columns():
    """Noiseless rank-5 data with l = 15: the rank rule replaces ten columns
    of every panel, where the bases of Algorithm 2 have no derivative.  The
    backward pass refuses (CNMF_ENODERIV), as the FP64 reference does."""
    say("adjoint_refuses")
    inst = synth.instance(200, 150, 5, 10, seed=0)
    G, F, tape = cnmf.adj_forward(dev(inst.X, 152), dev(inst.omega_L), dev(inst.omega_R),
                                  dev(inst.G0), dev(inst.F0), p=5, nu=10, q=2, outer_iters=3,
                                  inner_steps=5, ckpt=1)
    with pytest.raises(cnmf.CnmfError) as ei:
        tape.backward(G * 0 + 1, F * 0 + 1)
    assert ei.value.code == cnmf.ENODERIV
    tape.close()
    cnmf.check()
    rng = np.random.default_rng(1)
    with pytest.raises(ValueError):
        oracle.adjoint.loss_grad(inst.X, inst.omega_L, inst.omega_R, inst.G0, inst.F0,
                                 rng.random(inst.G0.shape), rng.random(inst.F0.shape), 2, 3, 5)


def test_adjoint_central_differences_at_full_size():
    """The differentiation form's own check: n = m = 2000, p = 10, l = 20,
    q = 2, 30 dB, 50 outer iterations x 5 inner steps, checkpoints every 10;
    32 directions D (||D|| = ||X||), h = 1e-3, on the GPU forward.  The
    entries of the final factors whose zero pattern differs between X + hD
    and X - hD (kinks of max(0, .) crossed inside the difference) are
    counted and reported per direction."""
    say("adjoint_fd_full")
    n = m = 2000
    p, nu, q, T, K, ck = 10, 10, 2, 50, 5, 10
    inst, Gt, Ft = _case(n, m, p, nu, seed=0)
    Lv, gX, _, _, _, _ = _gpu_loss_grad(inst, Gt, Ft, q, T, K, ck)
    rng = np.random.default_rng(5)
    X = inst.X.astype(np.float64)
    nX = np.linalg.norm(X)
    h = 1e-3
    fd, an, flips = [], [], []
    for j in range(32):
        D = rng.standard_normal(X.shape)
        D *= nX / np.linalg.norm(D)
        vals, zeros = [], []
        for sgn in (1.0, -1.0):
            Xs = (X + sgn * h * D).astype(np.float32)
            G, F, tape = cnmf.adj_forward(dev(Xs, 2048), dev(inst.omega_L), dev(inst.omega_R),
                                          dev(inst.G0), dev(inst.F0), p=p, nu=nu, q=q,
                                          outer_iters=T, inner_steps=K, ckpt=ck)
            vals.append(_loss64(G, F, Gt, Ft))
            zeros.append((host(G) == 0, host(F) == 0))
            tape.close()
        flips.append(int(np.sum(zeros[0][0] != zeros[1][0]) + np.sum(zeros[0][1] != zeros[1][1])))
        fd.append((vals[0] - vals[1]) / (2 * h))
        an.append(float(np.sum(gX * D)))
    cnmf.check()
    fd, an = np.array(fd), np.array(an)
    cos = float(fd @ an / (np.linalg.norm(fd) * np.linalg.norm(an)))
    rel = float(np.linalg.norm(fd - an) / np.linalg.norm(fd))
    per = np.abs(fd - an) / np.abs(fd)
    say("central differences: cosine", cos, "rel", rel, "per direction rel", np.round(per, 4).tolist(),
        "flipped entries per direction", flips)
    assert cos >= 0.999 and rel <= 1e-2, (cos, rel)
