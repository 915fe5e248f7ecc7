"""Precision form: bfloat16 conversion, BF16 sweeps on the matrix cores and
randomized subspace iteration with BF16 sweeps, against the oracle's
bfloat16 emulation (rounded operands, exact FP64 products)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import PARITY_RTOL, dev, host, rel_fro, say

pytestmark = pytest.mark.gpu

cnmf = pytest.importorskip("paper_1812_04315_amd")

# The BF16 solve against the oracle's BF16 emulation.  Both round X and the
# skinny operand of every X product to bfloat16, but the operand is the
# current basis, which the GPU holds in FP32 and the oracle in FP64: where
# the two round to neighbouring bfloat16 values the products differ by up to
# the bfloat16 unit roundoff u = 2^-9 in that entry's contribution, and the
# noise-bulk columns of the bases (fixed only up to rounding) follow.  The
# compressed data of the two runs therefore agree to O(u), not to FP32
# resolution: the relative errors and G F are compared at u, and the stop
# decisions (whose margin is far below u) are not compared -- the oracle
# replays the GPU's step counts.
BF16_SOLVE_RTOL = 2.0 ** -9


def dev_bits(bits, ld=None):
    """uint16 bfloat16 patterns -> int16 device tensor (optional row pitch)."""
    import torch
    b = np.ascontiguousarray(bits, dtype=np.uint16).view(np.int16)
    if ld is None or ld == b.shape[1]:
        return torch.from_numpy(b).cuda()
    buf = torch.zeros(b.shape[0], ld, dtype=torch.int16)
    buf[:, :b.shape[1]] = torch.from_numpy(b)
    return buf.cuda()[:, :b.shape[1]]


def _bound(X, A):
    return np.abs(X) @ np.abs(A)


@pytest.mark.parametrize("R,C,ld", [(1, 1, None), (37, 1001, None), (300, 257, 264), (1000, 4096, None)])
def test_to_bf16_bit_exact(R, C, ld):
    say("to_bf16", R, C, ld)
    rng = np.random.default_rng(R + C)
    X = (rng.standard_normal((R, C)) * 10.0 ** rng.integers(-30, 30, (R, C))).astype(np.float32)
    bits = X.view(np.uint32)
    k = X.size // 4
    flat = bits.reshape(-1)
    flat[:k] = (flat[:k] & 0xFFFF0000) | 0x8000          # exact ties
    if X.size > 8:
        flat[-4:] = np.array([0x7F800000, 0xFF800000, 0x7FC00001, 0x00000001], np.uint32)
    got = cnmf.to_bf16(dev(X, ld)).cpu().numpy().view(np.uint16)
    want = oracle.bf16_bits(X)
    nan = np.isnan(X)
    assert np.array_equal(got[~nan], want[~nan])
    assert np.all(np.isnan(oracle.bf16_value(got[nan])))


@pytest.mark.parametrize("R,C,k,ld", [
    (1, 1, 1, None), (31, 33, 5, None), (200, 150, 15, None), (257, 1000, 25, 1003),
    (1000, 97, 32, 100), (64, 4096, 16, None), (3, 2000, 7, None), (513, 777, 30, 784)])
@pytest.mark.parametrize("a_trans", [False, True])
def test_sweep_right_bf16(R, C, k, ld, a_trans):
    say("sweep_right_bf16", R, C, k, ld, a_trans)
    rng = np.random.default_rng(R * 11 + C + k)
    bits = oracle.bf16_bits(rng.random((R, C)).astype(np.float32))
    A = rng.standard_normal((C, k)).astype(np.float32)
    Xv = oracle.bf16_value(bits)
    Ar = oracle.bf16_round(A)
    Ad = dev(A.T.copy()) if a_trans else dev(A)
    Y = host(cnmf.sweep_right_bf16(dev_bits(bits, ld), Ad, a_trans=a_trans))
    ref = Xv @ Ar
    assert np.all(np.abs(Y - ref) <= 1e-5 * _bound(Xv, Ar) + 1e-30)


@pytest.mark.parametrize("R,C,k,ld", [
    (1, 1, 1, None), (33, 31, 5, None), (200, 150, 15, None), (1000, 257, 25, 260),
    (97, 1000, 32, 1001), (4096, 64, 16, None), (2000, 3, 7, None), (777, 513, 30, 520)])
@pytest.mark.parametrize("z_trans", [False, True])
def test_sweep_left_bf16(R, C, k, ld, z_trans):
    say("sweep_left_bf16", R, C, k, ld, z_trans)
    rng = np.random.default_rng(R * 13 + C + k)
    bits = oracle.bf16_bits(rng.random((R, C)).astype(np.float32))
    B = rng.standard_normal((R, k)).astype(np.float32)
    Xv = oracle.bf16_value(bits)
    Br = oracle.bf16_round(B)
    Z = host(cnmf.sweep_left_bf16(dev_bits(bits, ld), dev(B), z_trans=z_trans))
    if z_trans:
        Z = Z.T
    ref = Xv.T @ Br
    assert np.all(np.abs(Z - ref) <= 1e-5 * _bound(Xv.T, Br) + 1e-30)


@pytest.mark.parametrize("R,C,k,ld,ldat,z_trans", [
    (1, 1, 1, None, None, False), (31, 33, 5, None, None, True), (200, 150, 15, None, 151, False),
    (257, 1000, 25, 1003, None, True), (1000, 97, 32, 104, 100, False), (64, 4096, 16, None, None, False),
    (3, 2000, 7, None, 2001, True), (513, 777, 30, 784, 777, False), (2000, 3, 17, None, None, True),
    (4100, 2304, 25, None, None, False)])
def test_sweep_dual_bf16(R, C, k, ld, ldat, z_trans):
    """Both BF16 products of one read of X (every half-step of Algorithm 2
    in the precision form) against the oracle's emulation: ragged rows and
    columns, unaligned pitches (ld = 1003: rows not 16-byte aligned), column
    tiles of 512 and row slices."""
    say("sweep_dual_bf16", R, C, k, ld, ldat, z_trans)
    rng = np.random.default_rng(R * 17 + C + k)
    bits = oracle.bf16_bits(rng.random((R, C)).astype(np.float32))
    A = rng.standard_normal((C, k)).astype(np.float32)
    B = rng.standard_normal((R, k)).astype(np.float32)
    Y, Z = cnmf.sweep_dual_bf16(dev_bits(bits, ld), dev(A.T.copy(), ldat), dev(B), z_trans=z_trans)
    Y, Z = host(Y), host(Z)
    if z_trans:
        Z = Z.T
    Xv = oracle.bf16_value(bits)
    Ar, Br = oracle.bf16_round(A), oracle.bf16_round(B)
    assert np.all(np.abs(Y - Xv @ Ar) <= 1e-5 * _bound(Xv, Ar) + 1e-30)
    assert np.all(np.abs(Z - Xv.T @ Br) <= 1e-5 * _bound(Xv.T, Br) + 1e-30)


def test_sweep_dual_bf16_wide_pitch():
    """Row pitch of 2^25 + 8 elements (64-bit lane offsets within a group of
    32 rows), ragged rows and a ragged second column tile; X lives only on
    the device."""
    import torch
    say("sweep_dual_bf16_wide_pitch")
    rng = np.random.default_rng(13)
    R, C, k, ld = 40, 700, 25, (1 << 25) + 8
    bits = oracle.bf16_bits(rng.random((R, C)).astype(np.float32))
    A = rng.standard_normal((C, k)).astype(np.float32)
    B = rng.standard_normal((R, k)).astype(np.float32)
    buf = torch.zeros(R, ld, dtype=torch.int16, device="cuda")
    buf[:, :C] = torch.from_numpy(bits.view(np.int16)).cuda()
    Y, Z = cnmf.sweep_dual_bf16(buf[:, :C], dev(A.T.copy()), dev(B))
    del buf
    Xv = oracle.bf16_value(bits)
    Ar, Br = oracle.bf16_round(A), oracle.bf16_round(B)
    assert np.all(np.abs(host(Y) - Xv @ Ar) <= 1e-5 * _bound(Xv, Ar) + 1e-30)
    assert np.all(np.abs(host(Z) - Xv.T @ Br) <= 1e-5 * _bound(Xv.T, Br) + 1e-30)


def test_sweep_dual_bf16_bitwise_repeatable():
    rng = np.random.default_rng(2)
    bits = dev_bits(oracle.bf16_bits(rng.random((3000, 2000)).astype(np.float32)))
    AT = dev(rng.standard_normal((25, 2000)))
    B = dev(rng.standard_normal((3000, 25)))
    a = [host(t) for t in cnmf.sweep_dual_bf16(bits, AT, B)]
    b = [host(t) for t in cnmf.sweep_dual_bf16(bits, AT, B)]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _rsi_bf16(inst, q):
    import torch
    X = dev(inst.X)
    Xb = cnmf.to_bf16(X)
    out = cnmf.rsi_bf16(Xb, dev(inst.omega_L), dev(inst.omega_R), inst.p, inst.ell - inst.p, q)
    cnmf.check()
    return out


@pytest.mark.parametrize("n,m,p,nu,snr,seed", [(400, 300, 6, 10, 30.0, 3), (1000, 777, 12, 18, 30.0, 4),
                                               (200, 150, 5, 10, None, 0)])
def test_rsi_bf16_range_invariants(n, m, p, nu, snr, seed):
    """Orthonormal bases, and the same signal subspace and compressed
    reconstruction error as the emulation (the noise-bulk columns are fixed
    only up to roundoff, as in FP32)."""
    say("rsi_bf16", n, m, p, nu, snr, seed)
    inst = synth.instance(n, m, p, nu, seed=seed, snr_db=snr)
    QL, QR, XL, XR = (host(a) for a in _rsi_bf16(inst, 3))
    ref = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 3, bf16=True)
    ell = p + nu
    for Q in (QL, QR):
        assert np.linalg.norm(Q.T @ Q - np.eye(ell)) <= 1e-5
    Xv = oracle.bf16_round(inst.X)
    U, s, Vt = np.linalg.svd(Xv, full_matrices=False)
    for Q, Qo, S in ((QL, ref.Q_L, U[:, :p]), (QR, ref.Q_R, Vt[:p].T)):
        assert rel_fro(Q @ (Q.T @ S), Qo @ (Qo.T @ S)) <= PARITY_RTOL
    # compressed reconstruction errors lie between the best rank-l and the
    # best rank-p errors of bf16(X)
    nx = np.linalg.norm(Xv)
    e_l = np.sqrt(np.sum(s[ell:] ** 2)) / nx
    e_p = np.sqrt(np.sum(s[p:] ** 2)) / nx
    pairs = ((np.linalg.norm(Xv - QL @ XL) / nx, np.linalg.norm(Xv - ref.Q_L @ ref.X_L) / nx),
             (np.linalg.norm(Xv - XR @ QR.T) / nx, np.linalg.norm(Xv - ref.X_R @ ref.Q_R.T) / nx))
    for e_gpu, e_ref in pairs:
        assert e_l * (1 - 1e-6) <= e_gpu <= e_p * (1 + 1e-3)
        if snr is not None:
            # noisy data: the error is dominated by the noise beyond l and is
            # fixed to within the rounding flips of the bf16 operands
            assert abs(e_gpu - e_ref) <= 1e-3 * e_ref
        # noiseless data: beyond rank p only the bf16 quantisation noise of X
        # is left, and which part of it the l - p extra columns capture
        # depends on roundoff (parity unpinned for that part)


@pytest.mark.parametrize("n,m,p,nu,snr,T,K", [(200, 150, 5, 10, None, 20, 10),
                                              (1500, 1100, 10, 10, 30.0, 60, 100)])
def test_bf16_compressed_solve_against_oracle_emulation(n, m, p, nu, snr, T, K):
    """The precision form end to end: the GPU's BF16 randomized subspace
    iteration and its own free-running compressed solve against the oracle's
    BF16 emulation (X and every skinny operand rounded to bfloat16, FP64
    products) followed by its own solve, on the small noiseless instance and
    a noisy one.  Compared: RRE(t) on the FP32 X after every outer
    iteration, the final G F, and both against the FP32 oracle's result."""
    say("bf16_solve_vs_oracle", n, m, p, snr)
    from gpu_util import gf_rel_err
    inst = synth.instance(n, m, p, nu, seed=7, snr_db=snr)
    X = dev(inst.X)
    comp = cnmf.rsi_bf16(cnmf.to_bf16(X), dev(inst.omega_L), dev(inst.omega_R), p, nu, 4)
    G, F = dev(inst.G0), dev(inst.F0)
    tr = cnmf.make_trace(n, m, p, T, G.device)
    cnmf.solve(G, F, compressed=comp, p=p, outer_iters=T, inner_max=K, trace=tr)
    cnmf.check()
    ref_comp = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 4, bf16=True)
    steps = host(tr.steps).astype(int)
    ref = oracle.nenmf(None, inst.G0, inst.F0, T, K, compressed=ref_comp, keep_history=True,
                       replay=steps)
    free = oracle.nenmf(None, inst.G0, inst.F0, T, K, compressed=ref_comp)
    followed = int(np.sum(free.steps != steps))
    errs = host(cnmf.rre(X, tr.G_hist, tr.F_hist))
    errs_ref = oracle.rre_history(inst.X, ref.history)
    d_rre = float(np.max(np.abs(errs - errs_ref) / errs_ref))
    d_gf = gf_rel_err(host(G), host(F), ref.G, ref.F)
    ref32 = oracle.nenmf(None, inst.G0, inst.F0, T, K,
                         compressed=oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 4))
    d_gf32 = gf_rel_err(host(G), host(F), ref32.G, ref32.F)
    say("bf16 vs emulation: max rel dRRE", d_rre, "GF", d_gf, "step counts differing", followed,
        "| GF vs FP32 oracle", d_gf32, "final RRE", errs[-1], errs_ref[-1])
    assert d_rre <= BF16_SOLVE_RTOL
    assert d_gf <= BF16_SOLVE_RTOL
