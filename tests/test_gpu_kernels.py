"""Per-kernel parity of the HIP path (through the C ABI) with the FP64
oracle and library primitives, on identical seeded FP32 inputs."""
import numpy as np
import pytest

import oracle
from gpu_util import STOP_MARGIN, dev, host, rel_fro, say

pytestmark = pytest.mark.gpu

cnmf = pytest.importorskip("paper_1812_04315_amd")


def _bound(X, A):
    """Elementwise FP32 dot-product error scale |X| |A|."""
    return np.abs(X) @ np.abs(A)


@pytest.mark.parametrize("R,C,k,ld", [
    (1, 1, 1, None), (31, 33, 5, None), (200, 150, 15, None), (257, 1000, 25, 1003),
    (1000, 97, 32, 100), (64, 4096, 16, 4096), (3, 2000, 7, None), (513, 777, 30, 780)])
@pytest.mark.parametrize("a_trans", [False, True])
def test_sweep_right(R, C, k, ld, a_trans):
    say("sweep_right", R, C, k, ld, a_trans)
    rng = np.random.default_rng(R * 7 + C + k)
    X = rng.random((R, C)).astype(np.float32)
    A = rng.standard_normal((C, k)).astype(np.float32)
    Xd = dev(X, ld)
    Ad = dev(A.T.copy()) if a_trans else dev(A)
    Y = host(cnmf.sweep_right(Xd, Ad, a_trans=a_trans))
    ref = X.astype(np.float64) @ A.astype(np.float64)
    assert np.all(np.abs(Y - ref) <= 1e-5 * _bound(X, A) + 1e-30)


@pytest.mark.parametrize("R,C,k,ld", [
    (1, 1, 1, None), (33, 31, 5, None), (200, 150, 15, None), (1000, 257, 25, 260),
    (97, 1000, 32, 1001), (4096, 64, 16, None), (2000, 3, 7, None), (777, 513, 30, 516)])
@pytest.mark.parametrize("z_trans", [False, True])
def test_sweep_left(R, C, k, ld, z_trans):
    say("sweep_left", R, C, k, ld, z_trans)
    rng = np.random.default_rng(R * 5 + C + k)
    X = rng.random((R, C)).astype(np.float32)
    B = rng.standard_normal((R, k)).astype(np.float32)
    Z = host(cnmf.sweep_left(dev(X, ld), dev(B), z_trans=z_trans))
    if z_trans:
        Z = Z.T
    ref = X.T.astype(np.float64) @ B.astype(np.float64)
    assert np.all(np.abs(Z - ref) <= 1e-5 * _bound(X.T, B) + 1e-30)


@pytest.mark.parametrize("R,C,k,ld,ldat", [
    (1, 1, 1, None, None), (31, 33, 5, None, None), (200, 150, 15, None, 151),
    (257, 1000, 25, 1003, None), (1000, 97, 32, 100, 100), (64, 4096, 16, 4096, None),
    (3, 2000, 7, None, 2001), (513, 777, 30, 780, 777), (2000, 3, 17, None, None),
    (4100, 2304, 25, None, None)])
@pytest.mark.parametrize("z_trans", [False, True])
def test_sweep_dual(R, C, k, ld, ldat, z_trans):
    """Both products of one read of X (every half-step of Algorithm 2):
    ragged rows and columns, unaligned pitches of X and of the A panel,
    column tiles and row slices (4100 x 2304: nine full tiles, several
    slices)."""
    say("sweep_dual", R, C, k, ld, ldat, z_trans)
    rng = np.random.default_rng(R * 3 + C + k)
    X = rng.random((R, C)).astype(np.float32)
    A = rng.standard_normal((C, k)).astype(np.float32)
    B = rng.standard_normal((R, k)).astype(np.float32)
    Y, Z = cnmf.sweep_dual(dev(X, ld), dev(A.T.copy(), ldat), dev(B), z_trans=z_trans)
    Y, Z = host(Y), host(Z)
    if z_trans:
        Z = Z.T
    X64 = X.astype(np.float64)
    assert np.all(np.abs(Y - X64 @ A.astype(np.float64)) <= 1e-5 * _bound(X, A) + 1e-30)
    assert np.all(np.abs(Z - X64.T @ B.astype(np.float64)) <= 1e-5 * _bound(X.T, B) + 1e-30)


def test_sweep_dual_fp32_accuracy():
    """The dual pass forms its products from three-way BF16 splits of every
    FP32 operand (six cross terms on the BF16 matrix cores): its error
    against the FP64 product stays within a few times that of a plain FP32
    product of the same operands (torch FP32 matmul on the GPU)."""
    import torch
    say("sweep_dual_fp32_accuracy")
    rng = np.random.default_rng(11)
    R, C, k = 2000, 3000, 25
    X = rng.random((R, C)).astype(np.float32)
    A = rng.standard_normal((C, k)).astype(np.float32)
    B = rng.standard_normal((R, k)).astype(np.float32)
    Y, Z = cnmf.sweep_dual(dev(X), dev(A.T.copy()), dev(B))
    Yt = host(dev(X) @ dev(A))
    Zt = host(dev(X).T.contiguous() @ dev(B))
    Y64 = X.astype(np.float64) @ A.astype(np.float64)
    Z64 = X.T.astype(np.float64) @ B.astype(np.float64)
    for got, fp32, ref, bound in ((host(Y), Yt, Y64, _bound(X, A)), (host(Z), Zt, Z64, _bound(X.T, B))):
        e_split = np.max(np.abs(got - ref) / bound)
        e_fp32 = np.max(np.abs(fp32 - ref) / bound)
        say("max error / (|X| |A|): split", e_split, "fp32", e_fp32)
        assert e_split <= 4 * e_fp32 + 1e-9, (e_split, e_fp32)


def test_sweep_dual_wide_pitch():
    """Row pitch of 2^25 + 4 floats (64-bit lane offsets within a group of
    32 rows), ragged rows and a ragged second column tile; X lives only on
    the device."""
    import torch
    say("sweep_dual_wide_pitch")
    rng = np.random.default_rng(12)
    R, C, k, ld = 40, 300, 25, (1 << 25) + 4
    X = rng.random((R, C)).astype(np.float32)
    A = rng.standard_normal((C, k)).astype(np.float32)
    B = rng.standard_normal((R, k)).astype(np.float32)
    buf = torch.zeros(R, ld, dtype=torch.float32, device="cuda")
    buf[:, :C] = torch.from_numpy(X).cuda()
    Y, Z = cnmf.sweep_dual(buf[:, :C], dev(A.T.copy()), dev(B))
    del buf
    X64 = X.astype(np.float64)
    assert np.all(np.abs(host(Y) - X64 @ A.astype(np.float64)) <= 1e-5 * _bound(X, A) + 1e-30)
    assert np.all(np.abs(host(Z) - X64.T @ B.astype(np.float64)) <= 1e-5 * _bound(X.T, B) + 1e-30)


def test_sweep_dual_bitwise_repeatable():
    rng = np.random.default_rng(1)
    X = dev(rng.random((3000, 2000)))
    AT = dev(rng.standard_normal((25, 2000)))
    B = dev(rng.standard_normal((3000, 25)))
    a = [host(t) for t in cnmf.sweep_dual(X, AT, B)]
    b = [host(t) for t in cnmf.sweep_dual(X, AT, B)]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_sweep_bitwise_repeatable():
    rng = np.random.default_rng(0)
    X = dev(rng.random((3000, 2000)))
    A = dev(rng.standard_normal((2000, 25)))
    a = host(cnmf.sweep_right(X, A))
    b = host(cnmf.sweep_right(X, A))
    assert np.array_equal(a, b)
    c = host(cnmf.sweep_left(X, dev(rng.standard_normal((3000, 25)))))
    d = host(cnmf.sweep_left(X, dev(rng.standard_normal((3000, 25)))))
    assert not np.array_equal(c, d)   # different inputs, sanity
    B = dev(rng.standard_normal((3000, 25)))
    assert np.array_equal(host(cnmf.sweep_left(X, B)), host(cnmf.sweep_left(X, B)))


# 40000 and 70001 rows give every workgroup several 32-row tiles (the last
# ragged); 16 and 17 columns sit either side of the 16-column blocks of the
# matrix-core products (R^-1's corner block, Q's second column block)
@pytest.mark.parametrize("N,ell", [(40, 1), (200, 15), (1000, 25), (3001, 32), (32, 32),
                                   (40000, 25), (70001, 32), (3000, 16), (3000, 17)])
def test_orth_full_rank(N, ell):
    say("orth_full_rank", N, ell)
    rng = np.random.default_rng(N + ell)
    Y = (rng.standard_normal((N, ell)) @ np.diag(np.geomspace(1, 1e-3, ell))).astype(np.float32)
    P = rng.standard_normal((N, ell)).astype(np.float32)
    Q, rep = cnmf.orth(dev(Y), dev(P))
    Qh = host(Q)
    Qo, repo = oracle.orth(Y, P)
    assert host(rep).astype(bool).tolist() == repo.tolist()
    assert rel_fro(Qh, Qo) <= 1e-4
    assert np.linalg.norm(Qh.T @ Qh - np.eye(ell)) <= 1e-5


@pytest.mark.parametrize("delta,tau2", [(3e-4, 1e-9), (1e-6, 1e-14), (1e-2, 1e-9)])
def test_orth_nearly_collinear_columns(delta, tau2):
    """Columns y_j = y_0 + delta n_j: the pivots fall to about delta^2 of the
    diagonal.  At delta = 1e-2 one FP64 CholeskyQR pass is kept; at 3e-4 and
    1e-6 (with a rank threshold that keeps every column) the second pass runs,
    and at 1e-6 it is needed: one pass would leave an orthogonality loss near
    eps64 / delta^4 = 1e-4.  Orthonormal to FP32 rounding and spanning Y."""
    say("orth_collinear", delta, tau2)
    rng = np.random.default_rng(8)
    N, ell = 3000, 10
    y0 = rng.standard_normal((N, 1))
    Y = (y0 + delta * rng.standard_normal((N, ell))).astype(np.float32)
    P = rng.standard_normal((N, ell)).astype(np.float32)
    Q, rep = cnmf.orth(dev(Y), dev(P), tau2=tau2)
    Qh = host(Q)
    assert not host(rep).any()
    assert np.linalg.norm(Qh.T @ Qh - np.eye(ell)) <= 1e-5
    Y64 = Y.astype(np.float64)
    assert np.linalg.norm(Y64 - Qh @ (Qh.T @ Y64)) <= 1e-5 * np.linalg.norm(Y64)


# The augmented Gram [Y P] has 2 ell columns: 24 (two 16-column blocks), 40
# (three) and 64 (four: ten upper blocks, three on some waves); 3000 rows give
# one 32-row tile per workgroup, 25600 and 40000 several
@pytest.mark.parametrize("N,ell,r", [(300, 12, 5), (3000, 20, 8), (25600, 20, 8),
                                     (3000, 32, 10), (40000, 32, 10)])
@pytest.mark.parametrize("pool_trans", [False, True])
def test_orth_rank_deficient(pool_trans, N, ell, r):
    say("orth_rank_deficient", pool_trans, N, ell, r)
    rng = np.random.default_rng(3)
    Y = (rng.random((N, r)) @ rng.random((r, ell))).astype(np.float32)
    Y[:, 7] = 0.0
    P = rng.standard_normal((N, ell)).astype(np.float32)
    Q, rep = cnmf.orth(dev(Y), dev(P.T.copy()) if pool_trans else dev(P), pool_trans=pool_trans)
    Qo, repo = oracle.orth(Y, P)
    assert host(rep).astype(bool).tolist() == repo.tolist()
    assert repo.sum() == ell - r
    assert rel_fro(host(Q), Qo) <= 1e-4


def test_orth_breakdown_flag():
    say("orth_breakdown")
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((100, 4)).astype(np.float32)
    Y[:, 3] = Y[:, 0]
    P = rng.standard_normal((100, 4)).astype(np.float32)
    P[:, 3] = Y[:, 1]
    cnmf.orth(dev(Y), dev(P))
    with pytest.raises(cnmf.CnmfError) as ei:
        cnmf.check()
    assert ei.value.status & cnmf.ST_BREAKDOWN


@pytest.mark.parametrize("p", [1, 2, 3, 5, 15, 20, 31, 32])
def test_lipschitz(p):
    say("lipschitz", p)
    rng = np.random.default_rng(p)
    M = rng.random((p, 3 * p + 5)).astype(np.float32)
    W = (M.astype(np.float64) @ M.T).astype(np.float32)
    L = float(host(cnmf.lipschitz(dev(W)))[0])
    Lo = oracle.lipschitz(W)
    assert abs(L - Lo) <= 1e-12 * Lo
    Wz = np.zeros((p, p), np.float32)
    assert float(host(cnmf.lipschitz(dev(Wz)))[0]) == 0.0


@pytest.mark.parametrize("rows,p", [(1, 1), (200, 5), (1000, 15), (5000, 20), (257, 32)])
@pytest.mark.parametrize("forced", [1, 2, 7, 60])
def test_nnls_forced_rows(rows, p, forced):
    say("nnls_forced_rows", rows, p, forced)
    rng = np.random.default_rng(rows + p + forced)
    A = rng.random((3 * p + 2, p))
    W = (A.T @ A).astype(np.float32)
    B = (rng.random((rows, 3 * p + 2)) @ A).astype(np.float32)
    Z0 = rng.random((rows, p)).astype(np.float32)
    Z = dev(Z0)
    steps, L, _ = cnmf.nnls(Z, dev(W), dev(B), 0.0, 1000, forced=forced)
    Zo, ko, Lo = oracle.nesterov_nnls(Z0, W, B, "G", 0.0, 1000, forced_steps=forced)
    assert int(host(steps)[0]) == forced == ko
    assert abs(float(host(L)[0]) - Lo) <= 1e-12 * Lo
    assert rel_fro(host(Z), Zo) <= 1e-5


@pytest.mark.parametrize("m,p", [(150, 5), (3000, 15), (777, 25)])
def test_nnls_forced_columns(m, p):
    say("nnls_forced_columns", m, p)
    rng = np.random.default_rng(m + p)
    A = rng.random((2 * p + 1, p))
    W = (A.T @ A).astype(np.float32)
    Bt = (rng.random((m, 2 * p + 1)) @ A).astype(np.float32)   # m x p = B^T
    F0 = rng.random((p, m)).astype(np.float32)
    F = dev(F0)
    cnmf.nnls(F, dev(W), dev(Bt), 0.0, 100, forced=9, by_columns=True)
    Fo, _, _ = oracle.nesterov_nnls(F0, W, Bt.T, "F", 0.0, 100, forced_steps=9)
    assert rel_fro(host(F), Fo) <= 1e-5


@pytest.mark.parametrize("rows,p,tol", [(500, 5, 1e-2), (3000, 15, 1e-3), (9000, 20, 1e-1)])
def test_nnls_stopping_rule(rows, p, tol):
    """Tolerance-driven stop: same count as the oracle unless the oracle's
    margin at the decisive step is below FP32 resolution."""
    say("nnls_stop", rows, p, tol)
    rng = np.random.default_rng(rows)
    A = rng.random((3 * p, p))
    W = (A.T @ A).astype(np.float32)
    B = (rng.random((rows, 3 * p)) @ A).astype(np.float32)
    Z0 = rng.random((rows, p)).astype(np.float32)
    pg0 = oracle.pg_norm(Z0.astype(float), W.astype(float), B.astype(float), "G")
    t = tol * pg0
    Z = dev(Z0)
    steps, _, pg2 = cnmf.nnls(Z, dev(W), dev(B), t, 5000)
    Zo, ko, _ = oracle.nesterov_nnls(Z0, W, B, "G", t, 5000)
    assert abs(np.sqrt(float(host(pg2)[0])) - pg0) <= 1e-5 * pg0
    k = int(host(steps)[0])
    _check_decision(Z0, W, B, "G", t, k, ko, host(Z), Zo)


def _oracle_pg_at(Z0, W, B, side, steps):
    """Projected-gradient norm of the oracle's iterate after exactly `steps` steps."""
    Zk, _, _ = oracle.nesterov_nnls(Z0, W, B, side, 0.0, steps, forced_steps=steps)
    return oracle.pg_norm(Zk, W.astype(float), B.astype(float), side)


def _check_decision(Z0, W, B, side, t, k, ko, Zg, Zo):
    """Equal step counts, or counts one apart with the oracle's norm at the
    smaller count within the stop margin of the bound; the iterate is then
    compared with the oracle's after the GPU's count."""
    if k != ko:
        d = min(k, ko)
        assert abs(k - ko) == 1 and d >= 1, (k, ko)
        pg = _oracle_pg_at(Z0, W, B, side, d)
        assert abs(pg - t) <= STOP_MARGIN * t, (k, ko, pg, t)
        Zo, _, _ = oracle.nesterov_nnls(Z0, W, B, side, 0.0, k, forced_steps=k)
    assert rel_fro(Zg, Zo) <= 1e-4


@pytest.mark.parametrize("rows,p,frac,inner_max,inner_min", [
    (300, 5, 0.9, 5000, 1),      # stops after the first step
    (300, 5, 0.06, 5000, 1),     # stops inside the first group of four steps
    (300, 5, 0.025, 5000, 1),    # at a group boundary
    (300, 5, 0.01, 5000, 1),
    (1, 1, 0.5, 50, 1),          # one variable: exact after one step
    (2000, 15, 0.03, 5000, 1),
    (2000, 15, 0.5, 5000, 6),    # the lower bound on the step count binds
    (2000, 15, 1e-7, 5, 1),      # the step cap binds, not a multiple of four
    (2000, 15, 1e-7, 3, 1),
    (700, 12, 1e-7, 10, 1),
    (700, 12, 0.0085, 5000, 1),
    (700, 12, 0.2, 9, 9),        # lower bound equal to the cap
    (4000, 20, 0.004, 5000, 3),
    (257, 32, 0.0021, 5000, 2),
])
def test_nnls_stop_edges(rows, p, frac, inner_max, inner_min):
    """Stopping rule near its edges (early stops, a binding lower bound or cap):
    the step count equals the oracle's unless the oracle's norm at the
    decisive step lies within 1e-3 of the tolerance, where one step either
    way is allowed."""
    say("nnls_stop_edges", rows, p, frac, inner_max, inner_min)
    rng = np.random.default_rng(rows * 7 + p)
    A = rng.random((3 * p, p))
    W = (A.T @ A).astype(np.float32)
    B = (rng.random((rows, 3 * p)) @ A).astype(np.float32)
    Z0 = rng.random((rows, p)).astype(np.float32)
    t = frac * oracle.pg_norm(Z0.astype(float), W.astype(float), B.astype(float), "G")
    Z = dev(Z0)
    steps, _, _ = cnmf.nnls(Z, dev(W), dev(B), t, inner_max, inner_min=inner_min)
    Zo, ko, _ = oracle.nesterov_nnls(Z0, W, B, "G", t, inner_max, inner_min=inner_min)
    k = int(host(steps)[0])
    assert inner_min <= k <= inner_max or (k == ko == 0)
    _check_decision(Z0, W, B, "G", t, k, ko, host(Z), Zo)


@pytest.mark.parametrize("m,p,frac,inner_min", [(150, 5, 0.5, 1), (3000, 15, 0.05, 4)])
def test_nnls_stop_columns(m, p, frac, inner_min):
    """Tolerance-driven stop on the F side (columns of a p x m factor)."""
    say("nnls_stop_columns", m, p, frac, inner_min)
    rng = np.random.default_rng(m + 3 * p)
    A = rng.random((2 * p + 1, p))
    W = (A.T @ A).astype(np.float32)
    Bt = (rng.random((m, 2 * p + 1)) @ A).astype(np.float32)
    F0 = rng.random((p, m)).astype(np.float32)
    t = frac * oracle.pg_norm(F0.astype(float), W.astype(float), Bt.T.astype(float), "F")
    F = dev(F0)
    steps, _, _ = cnmf.nnls(F, dev(W), dev(Bt), t, 5000, inner_min=inner_min, by_columns=True)
    Fo, ko, _ = oracle.nesterov_nnls(F0, W, Bt.T, "F", t, 5000, inner_min=inner_min)
    k = int(host(steps)[0])
    _check_decision(F0, W, Bt.T, "F", t, k, ko, host(F), Fo)


def test_rre_matches_oracle():
    say("rre")
    rng = np.random.default_rng(9)
    n, m, p = 333, 517, 7
    X = rng.random((n, m)).astype(np.float32)
    Gs = rng.random((3, n, p)).astype(np.float32)
    Fs = rng.random((3, p, m)).astype(np.float32)
    out = host(cnmf.rre(dev(X, 520), dev(Gs.reshape(3 * n, p)).view(3, n, p),
                        dev(Fs.reshape(3 * p, m)).view(3, p, m)))
    for i in range(3):
        assert abs(out[i] - oracle.rre(X, Gs[i], Fs[i])) <= 1e-10 * out[i]
