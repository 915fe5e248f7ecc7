"""The compressions Sec. 3 sets Algorithm 2 against, through cnmf_compress:
the scaled Gaussian projection and randomized power iteration without
re-orthonormalisation, against the FP64 oracle on identical seeded inputs,
and the compressed solve on each."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import PARITY_RTOL, dev, follow_decisions, gf_rel_err, host, rel_fro, say

pytestmark = pytest.mark.gpu

cnmf = pytest.importorskip("paper_1812_04315_amd")


def _proj_top(Q, S):
    """Projection of the columns S onto range(Q) (orthonormal Q)."""
    return Q @ (Q.T @ S)


def test_rsi_kind_equals_cnmf_rsi():
    say("compress_rsi")
    inst = synth.instance(500, 400, 8, 10, seed=3, snr_db=30.0)
    X = dev(inst.X)
    a = cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R), 8, 10, 3)
    b = cnmf.compress(X, dev(inst.omega_L), dev(inst.omega_R), 8, 10, 3, kind=cnmf.COMPRESS_RSI)
    cnmf.check()
    for x, y in zip(a, b):
        assert np.array_equal(host(x), host(y))


@pytest.mark.parametrize("n,m,p,nu,ld", [(300, 250, 5, 10, None), (1000, 777, 12, 18, 780),
                                         (97, 131, 3, 6, None)])
def test_gaussian_projection(n, m, p, nu, ld):
    """Q_L = Omega_R^T / sqrt(l), Q_R = Omega_L / sqrt(l) and the compressed
    data X_L = Q_L^T X, X_R = X Q_R against the oracle (elementwise at the
    FP32 dot-product bound of the sweeps)."""
    say("compress_gaussian", n, m, p, nu, ld)
    inst = synth.instance(n, m, p, nu, seed=n, snr_db=30.0)
    QL, QR, XL, XR = (host(a) for a in cnmf.compress(
        dev(inst.X, ld), dev(inst.omega_L), dev(inst.omega_R), p, nu, kind=cnmf.COMPRESS_GAUSSIAN))
    cnmf.check()
    ref = oracle.compress_gaussian(inst.X, inst.omega_L, inst.omega_R)
    assert np.max(np.abs(QL - ref.Q_L)) <= 1e-6 * np.max(np.abs(ref.Q_L))
    assert np.max(np.abs(QR - ref.Q_R)) <= 1e-6 * np.max(np.abs(ref.Q_R))
    X = inst.X.astype(np.float64)
    bound_r = np.abs(X) @ np.abs(ref.Q_R)
    bound_l = np.abs(ref.Q_L).T @ np.abs(X)
    assert np.all(np.abs(XR - ref.X_R) <= 1e-5 * bound_r + 1e-30)
    assert np.all(np.abs(XL - ref.X_L) <= 1e-5 * bound_l + 1e-30)


def test_power_iteration_low_rank_exact():
    """rank(X) = 4 with singular values within a factor 2, l = 9: the bases
    capture X to FP32 resolution; the five missing columns come from the
    Gaussian pools."""
    say("compress_power_low_rank")
    rng = np.random.default_rng(5)
    n, m, r, p, nu = 300, 240, 4, 4, 5

    def orthonormal(k, c):
        q, rr = np.linalg.qr(rng.standard_normal((k, c)))
        return q * np.sign(np.diag(rr))

    # the range finder does not need X >= 0 (that is the solver's requirement)
    Xl = (orthonormal(n, r) @ np.diag([2.0, 1.7, 1.3, 1.0]) @ orthonormal(m, r).T).astype(np.float32)
    inst = synth.instance(n, m, p, nu, seed=1)   # for the projection draws only
    QL, QR, XL, XR = (host(a) for a in cnmf.compress(
        dev(Xl), dev(inst.omega_L), dev(inst.omega_R), p, nu, 2, kind=cnmf.COMPRESS_POWER))
    cnmf.check()
    X64 = Xl.astype(np.float64)
    nx = np.linalg.norm(X64)
    assert np.linalg.norm(X64 - QL @ XL) <= 1e-5 * nx
    assert np.linalg.norm(X64 - XR @ QR.T) <= 1e-5 * nx
    for Q in (QL, QR):
        assert np.linalg.norm(Q.T @ Q - np.eye(p + nu)) <= 1e-5


@pytest.mark.parametrize("n,m,p,nu,q", [(400, 300, 6, 10, 1), (1500, 1100, 10, 15, 1)])
def test_power_iteration_signal_subspace(n, m, p, nu, q):
    """Noisy data, one power: the leading p directions of X are captured as by
    the oracle; the remaining columns follow noise directions that rounding
    decides (parity unpinned for them, as for Algorithm 2).  After more
    powers the weaker signal directions themselves fall below FP32 (and the
    rank threshold) without re-orthonormalisation -- the instability that
    Algorithm 2 removes -- see test_power_iteration_loses_weak_directions."""
    say("compress_power_signal", n, m, p, nu, q)
    inst = synth.instance(n, m, p, nu, seed=m, snr_db=30.0)
    QL, QR, XL, XR = (host(a) for a in cnmf.compress(
        dev(inst.X), dev(inst.omega_L), dev(inst.omega_R), p, nu, q, kind=cnmf.COMPRESS_POWER))
    cnmf.check()
    ref = oracle.compress_power(inst.X, inst.omega_L, inst.omega_R, q)
    X = inst.X.astype(np.float64)
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    for Q, Qo, S in ((QL, ref.Q_L, U[:, :p]), (QR, ref.Q_R, Vt[:p].T)):
        assert np.linalg.norm(Q.T @ Q - np.eye(p + nu)) <= 1e-5
        assert rel_fro(_proj_top(Q, S), _proj_top(Qo, S)) <= PARITY_RTOL
    # the data compressed on the right fits X no worse than its best rank-p
    # approximation (the signal is captured)
    floor = np.sqrt(np.sum(s[p:] ** 2)) / np.linalg.norm(X)
    assert np.linalg.norm(X - XR @ QR.T) / np.linalg.norm(X) <= floor * (1 + 1e-3)


@pytest.mark.parametrize("kind", ["gaussian", "power"])
def test_compressed_solve_on_variant_data(kind):
    """The compressed solve (Algorithm 1) on each variant's compressed data,
    shared with the oracle (the GPU's compression, rounded to FP32), free
    running: G, F after 20 outer iterations at the parity bound."""
    say("variant_solve", kind)
    n, m, p, nu = 800, 600, 8, 12
    inst = synth.instance(n, m, p, nu, seed=11, snr_db=30.0)
    X = dev(inst.X)
    k = cnmf.COMPRESS_GAUSSIAN if kind == "gaussian" else cnmf.COMPRESS_POWER
    comp = cnmf.compress(X, dev(inst.omega_L), dev(inst.omega_R), p, nu, 1, kind=k)
    shared = oracle.RSIResult(*(host(a) for a in comp))
    G, F = dev(inst.G0), dev(inst.F0)
    T, K = 20, 100
    tr = cnmf.make_trace(n, m, p, T, G.device)
    cnmf.solve(G, F, compressed=comp, p=p, outer_iters=T, inner_max=K, trace=tr)
    cnmf.check()
    ref, followed = follow_decisions(host(tr.steps).astype(int), lambda rep: oracle.nenmf(
        None, inst.G0, inst.F0, T, K, compressed=shared, keep_pg=True, keep_history=True,
        replay=rep))
    errs = host(cnmf.rre(X, tr.G_hist, tr.F_hist))
    errs_ref = oracle.rre_history(inst.X, ref.history)
    say(kind, "followed", followed, "final RRE", errs[-1], errs_ref[-1])
    assert rel_fro(host(G), ref.G) <= PARITY_RTOL
    assert rel_fro(host(F), ref.F) <= PARITY_RTOL
    assert np.max(np.abs(errs - errs_ref) / errs_ref) <= PARITY_RTOL
    assert gf_rel_err(host(G), host(F), ref.G, ref.F) <= PARITY_RTOL


def test_power_iteration_loses_weak_directions():
    """q = 4 on planted U[0, 1) factors: the dominant direction of X is
    still captured exactly and the bases stay orthonormal, but the weaker
    signal directions, (sigma_i / sigma_1)^8 below the rank threshold after
    the powers, are replaced from the Gaussian pools, so the compressed fit
    misses the signal that Algorithm 2 keeps at the same q."""
    say("compress_power_instability")
    n, m, p, nu, q = 1500, 1100, 10, 15, 4
    inst = synth.instance(n, m, p, nu, seed=m, snr_db=30.0)
    X = dev(inst.X)
    QLp, QRp, XLp, XRp = (host(a) for a in cnmf.compress(
        X, dev(inst.omega_L), dev(inst.omega_R), p, nu, q, kind=cnmf.COMPRESS_POWER))
    QLr, QRr, XLr, XRr = (host(a) for a in cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R),
                                                   p, nu, q))
    cnmf.check()
    Xh = inst.X.astype(np.float64)
    U, s, Vt = np.linalg.svd(Xh, full_matrices=False)
    nx = np.linalg.norm(Xh)
    for Q in (QLp, QRp):
        assert np.linalg.norm(Q.T @ Q - np.eye(p + nu)) <= 1e-5
    assert np.linalg.norm(U[:, 0] - QLp @ (QLp.T @ U[:, 0])) <= 1e-4
    assert np.linalg.norm(Vt[0] - QRp @ (QRp.T @ Vt[0])) <= 1e-4
    floor = np.sqrt(np.sum(s[p:] ** 2)) / nx
    e_power = np.linalg.norm(Xh - XRp @ QRp.T) / nx
    e_rsi = np.linalg.norm(Xh - XRr @ QRr.T) / nx
    say("fit: power", e_power, "subspace iteration", e_rsi, "rank-p floor", floor)
    assert e_rsi <= floor * (1 + 1e-3)
    assert e_power > 1.2 * e_rsi
