"""Parity at the full sizes of the measured workloads, in the launch
configurations bench.py times: sampled outputs recomputed one by one in
FP64, properties that hold at any size, and short oracle runs on the GPU's
own compressed data (step counts replayed)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import PARITY_RTOL, dev, host, rel_fro, say

pytestmark = pytest.mark.gpu

cnmf = pytest.importorskip("paper_1812_04315_amd")


@pytest.fixture(scope="module")
def big():
    """The 10000 x 10000, p = 15 instance (30 dB), X with the bench's pitch."""
    import torch
    inst = synth.instance(10000, 10000, 15, 10, seed=0, snr_db=30.0)
    X = dev(inst.X, 10048)
    comp = cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R), 15, 10, 4)
    cnmf.check()
    torch.cuda.synchronize()
    return inst, X, comp


def test_fullsize_sweeps_sampled(big):
    say("fullsize_sweeps")
    inst, X, _ = big
    rng = np.random.default_rng(0)
    F = inst.F0.astype(np.float32)
    Y = host(cnmf.sweep_right(X, dev(F), a_trans=True))          # X F^T, the roofline call
    rows = rng.choice(10000, 64, replace=False)
    Xr = inst.X[rows].astype(np.float64)
    ref = Xr @ F.T.astype(np.float64)
    assert np.all(np.abs(Y[rows] - ref) <= 1e-5 * (np.abs(Xr) @ np.abs(F.T)) + 1e-30)
    G = inst.G0.astype(np.float32)
    Z = host(cnmf.sweep_left(X, dev(G)))                          # X^T G
    cols = rng.choice(10000, 64, replace=False)
    Xc = inst.X[:, cols].astype(np.float64)
    ref = Xc.T @ G.astype(np.float64)
    assert np.all(np.abs(Z[cols] - ref) <= 1e-5 * (np.abs(Xc.T) @ np.abs(G)) + 1e-30)


def test_fullsize_rsi_properties_and_signal_subspace(big):
    say("fullsize_rsi")
    inst, X, comp = big
    QL, QR, XL, XR = (host(a) for a in comp)
    for Q in (QL, QR):
        assert np.linalg.norm(Q.T @ Q - np.eye(25)) <= 1e-5
    rng = np.random.default_rng(1)
    rows = rng.choice(10000, 32, replace=False)
    ref = inst.X[rows].astype(np.float64) @ QR
    assert rel_fro(XR[rows], ref) <= 1e-5
    cols = rng.choice(10000, 32, replace=False)
    ref = QL.T @ inst.X[:, cols].astype(np.float64)
    assert rel_fro(XL[:, cols], ref) <= 1e-5
    # range-invariant agreement with the FP64 oracle
    r = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 4)
    Xh = inst.X.astype(np.float64)
    e_gpu = np.linalg.norm(Xh - QL @ XL) / np.linalg.norm(Xh)
    e_ref = np.linalg.norm(Xh - r.Q_L @ r.X_L) / np.linalg.norm(Xh)
    assert abs(e_gpu - e_ref) <= 1e-4 * e_ref
    # projector onto the planted signal directions (top 15 of the oracle basis)
    U, _, _ = np.linalg.svd(r.Q_L.T @ Xh @ r.Q_R, full_matrices=False)
    S = r.Q_L @ U[:, :15]
    assert rel_fro(QL @ (QL.T @ S), S) <= 1e-4


@pytest.mark.parametrize("method", ["compressed", "plain"])
def test_fullsize_solve_against_oracle(big, method):
    """A few outer iterations of the bench's solve; the oracle runs on the
    GPU's compressed data (FP32 values) with the GPU's step counts."""
    say("fullsize_solve", method)
    import torch
    inst, X, comp = big
    T = 4 if method == "compressed" else 2
    G, F = dev(inst.G0), dev(inst.F0)
    tr = cnmf.make_trace(10000, 10000, 15, T, G.device, history=False)
    cnmf.solve(G, F, X=None if method == "compressed" else X,
               compressed=comp if method == "compressed" else None, p=15, nu=10,
               outer_iters=T, trace=tr)
    cnmf.check()
    steps = host(tr.steps).astype(int)
    shared = oracle.RSIResult(*(host(a) for a in comp)) if method == "compressed" else None
    ref = oracle.nenmf(inst.X, inst.G0, inst.F0, T, 500, compressed=shared, replay=steps)
    assert rel_fro(host(G), ref.G) <= PARITY_RTOL
    assert rel_fro(host(F), ref.F) <= PARITY_RTOL


def test_fullsize_bf16_sweeps_sampled():
    say("fullsize_bf16")
    import torch
    n, m, k = 20000, 8000, 30
    rng = np.random.default_rng(2)
    Xf = rng.random((n, m), dtype=np.float32)
    Xd = dev(Xf, 8064)
    Xb = cnmf.to_bf16(Xd, 8064)
    bits = Xb.cpu().numpy().view(np.uint16)
    assert np.array_equal(bits[:7], oracle.bf16_bits(Xf[:7]))
    A = rng.standard_normal((m, k)).astype(np.float32)
    B = rng.standard_normal((n, k)).astype(np.float32)
    Y = host(cnmf.sweep_right_bf16(Xb, dev(A.T.copy()), a_trans=True))
    Z = host(cnmf.sweep_left_bf16(Xb, dev(B)))
    rows = rng.choice(n, 32, replace=False)
    Xv = oracle.bf16_value(bits[rows])
    Ar = oracle.bf16_round(A)
    assert np.all(np.abs(Y[rows] - Xv @ Ar) <= 1e-5 * (np.abs(Xv) @ np.abs(Ar)) + 1e-30)
    cols = rng.choice(m, 32, replace=False)
    Xc = oracle.bf16_value(bits[:, cols])
    Br = oracle.bf16_round(B)
    assert np.all(np.abs(Z[cols] - Xc.T @ Br) <= 1e-5 * (np.abs(Xc.T) @ np.abs(Br)) + 1e-30)


def test_fullsize_batched_sampled_instances():
    """All 256 instances of the batched workload (3 outer iterations); four
    sampled instances against the oracle on the batch's own compressed data
    with the batch's step counts."""
    say("fullsize_batched")
    import torch
    shapes = synth.batched_shapes(256, seed=0)
    descs, insts = [], []
    T = 3
    for k, (n, m, p) in enumerate(shapes):
        inst = synth.instance(n, m, p, 10, seed=k, snr_db=20.0)
        ell = p + 10
        d = dict(p=p, nu=10, X=dev(inst.X, (m + 63) // 64 * 64), omega_L=dev(inst.omega_L),
                 omega_R=dev(inst.omega_R), Q_L=torch.empty(n, ell, device="cuda"),
                 Q_R=torch.empty(m, ell, device="cuda"), X_L=torch.empty(ell, m, device="cuda"),
                 X_R=torch.empty(n, ell, device="cuda"), G=dev(inst.G0), F=dev(inst.F0),
                 steps=torch.zeros(T, 2, dtype=torch.int32, device="cuda"))
        descs.append(d)
        insts.append(inst)
    b = cnmf.Batch(descs, q=2, outer_iters=T, inner_max=500)
    b.rsi()
    b.solve(True)
    cnmf.check()
    for k in (0, 77, 150, 255):
        d, inst = descs[k], insts[k]
        comp = oracle.RSIResult(*(host(d[key]) for key in ("Q_L", "Q_R", "X_L", "X_R")))
        ref = oracle.nenmf(inst.X, inst.G0, inst.F0, T, 500, compressed=comp,
                           replay=host(d["steps"]).astype(int))
        assert rel_fro(host(d["G"]), ref.G) <= PARITY_RTOL
        assert rel_fro(host(d["F"]), ref.F) <= PARITY_RTOL
    b.close()


def test_fullsize_adjoint_against_fp64_reference():
    say("fullsize_adjoint")
    import torch
    n = m = 2000
    p, nu, q, T, K = 10, 10, 2, 50, 5
    inst = synth.instance(n, m, p, nu, seed=0, snr_db=30.0)
    rng = np.random.default_rng(99)
    Gt = rng.random(inst.G0.shape).astype(np.float32)
    Ft = rng.random(inst.F0.shape).astype(np.float32)
    G, F, tape = cnmf.adj_forward(dev(inst.X), dev(inst.omega_L), dev(inst.omega_R),
                                  dev(inst.G0), dev(inst.F0), p=p, nu=nu, q=q, outer_iters=T,
                                  inner_steps=K, ckpt=10)
    dX, _, _ = tape.backward(2 * (G - dev(Gt)), 2 * (F - dev(Ft)))
    cnmf.check()
    g = host(dX)
    tape.close()
    _, r, _, _ = oracle.adjoint.loss_grad(inst.X, inst.omega_L, inst.omega_R, inst.G0, inst.F0,
                                          Gt, Ft, q, T, K)
    cos = float(np.sum(g * r) / (np.linalg.norm(g) * np.linalg.norm(r)))
    assert cos >= 0.999 and np.linalg.norm(g - r) <= 1e-2 * np.linalg.norm(r)
