"""End-to-end parity of the HIP path (randomized subspace iteration and the
plain / compressed NeNMF outer loops, through the C ABI) with the FP64
oracle on identical seeded inputs."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import PARITY_RTOL, dev, follow_decisions, host, rel_fro, say

pytestmark = pytest.mark.gpu

cnmf = pytest.importorskip("paper_1812_04315_amd")


def _gpu_rsi(inst, q, ld=None):
    X = dev(inst.X, ld)
    out = cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R), inst.p, inst.ell - inst.p, q)
    cnmf.check()
    return X, out


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("ld", [None, 152])
def test_rsi_small_instance(seed, ld):
    """200 x 150, rank 5, l = 15, q = 4: columns 6..15 of every panel are
    numerically absent and come from the other Gaussian draw on both sides."""
    say("rsi_small_instance", seed, ld)
    inst = synth.instance(200, 150, 5, 10, seed=seed)
    _, (QL, QR, XL, XR) = _gpu_rsi(inst, 4, ld)
    ref = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 4)
    for name, a, b in (("Q_L", QL, ref.Q_L), ("Q_R", QR, ref.Q_R), ("X_L", XL, ref.X_L),
                       ("X_R", XR, ref.X_R)):
        assert rel_fro(host(a), b) <= PARITY_RTOL, name


def test_rsi_noisy_signal_subspace():
    """Noisy data: the noise-bulk basis columns are fixed only up to
    roundoff, so compare what is range-invariant: the projector onto the
    leading p directions of X_R and the compressed reconstruction error."""
    say("rsi_noisy")
    inst = synth.instance(400, 300, 6, 10, seed=3, snr_db=30.0)
    X, (QL, QR, XL, XR) = _gpu_rsi(inst, 4)
    ref = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 4)
    Xh = inst.X.astype(np.float64)
    for Q, Qo in ((host(QL), ref.Q_L), (host(QR), ref.Q_R)):
        assert np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) <= 1e-5
    # projector onto the range of the whole sketch basis, restricted to the
    # top-p singular directions of X
    U, s, Vt = np.linalg.svd(Xh, full_matrices=False)
    Up, Vp = U[:, :6], Vt[:6].T
    for Q, Qo, S in ((host(QL), ref.Q_L, Up), (host(QR), ref.Q_R, Vp)):
        a = Q @ (Q.T @ S)
        b = Qo @ (Qo.T @ S)
        assert rel_fro(a, b) <= PARITY_RTOL
    e_gpu = np.linalg.norm(Xh - host(QL) @ host(XL)) / np.linalg.norm(Xh)
    e_ref = np.linalg.norm(Xh - ref.Q_L @ ref.X_L) / np.linalg.norm(Xh)
    assert abs(e_gpu - e_ref) <= PARITY_RTOL * e_ref


def _solve_gpu(inst, X, comp, T, inner_max, stop_rule=cnmf.STOP_GLOBAL, replay=None):
    import torch
    G = dev(inst.G0)
    F = dev(inst.F0)
    n, m = inst.X.shape
    tr = cnmf.make_trace(n, m, inst.p, T, G.device)
    cnmf.solve(G, F, X=X, compressed=comp, p=inst.p, outer_iters=T, inner_max=inner_max,
               stop_rule=stop_rule, trace=tr,
               replay=None if replay is None else torch.from_numpy(
                   np.ascontiguousarray(replay, dtype=np.int32)).cuda())
    cnmf.check()
    return G, F, tr


@pytest.mark.parametrize("method", ["plain", "compressed"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_solve_small_instance(method, seed):
    """The small instance: 20 outer iterations x <= 10 inner steps, global bound."""
    say("solve_small_instance", method, seed)
    inst = synth.instance(200, 150, 5, 10, seed=seed)
    X = dev(inst.X)
    comp = ref_comp = None
    if method == "compressed":
        comp = cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R), 5, 10, 4)
        ref_comp = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 4)
    G, F, tr = _solve_gpu(inst, X, comp, 20, 10)
    steps = host(tr.steps).astype(int)
    # the oracle's own run; where a stop decision differs it must lie within
    # the margin of the bound, and the oracle then follows the GPU's count
    ref, followed = follow_decisions(steps, lambda rep: oracle.nenmf(
        inst.X, inst.G0, inst.F0, 20, 10, compressed=ref_comp, keep_history=True,
        keep_pg=True, replay=rep))
    if followed:
        say("followed", followed)
    assert rel_fro(host(G), ref.G) <= PARITY_RTOL
    assert rel_fro(host(F), ref.F) <= PARITY_RTOL
    np.testing.assert_allclose(host(tr.lips), ref.lips, rtol=1e-4)
    GFg = host(G) @ host(F)
    assert rel_fro(GFg, ref.G @ ref.F) <= PARITY_RTOL
    # history and RRE trace on the device
    errs = host(cnmf.rre(X, tr.G_hist, tr.F_hist))
    errs_ref = [oracle.rre(inst.X, g, f) for g, f in ref.history]
    np.testing.assert_allclose(errs, errs_ref, rtol=PARITY_RTOL)
    ticks = host(tr.ticks)
    assert np.all(np.diff(ticks) >= 0) and ticks[-1] > ticks[0]


@pytest.mark.parametrize("method", ["plain", "compressed"])
def test_solve_subproblem_rule(method):
    say("solve_subproblem_rule", method)
    inst = synth.instance(200, 150, 5, 10, seed=4)
    X = dev(inst.X)
    comp = ref_comp = None
    if method == "compressed":
        comp = cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R), 5, 10, 4)
        ref_comp = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 4)
    G, F, tr = _solve_gpu(inst, X, comp, 10, 50, stop_rule=cnmf.STOP_SUBPROBLEM)
    steps = host(tr.steps).astype(int)
    ref, followed = follow_decisions(steps, lambda rep: oracle.nenmf(
        inst.X, inst.G0, inst.F0, 10, 50, stop_rule="subproblem", compressed=ref_comp,
        keep_pg=True, replay=rep))
    if followed:
        say("followed", followed)
    np.testing.assert_allclose(host(tr.tols), ref.tols, rtol=PARITY_RTOL)
    assert rel_fro(host(G), ref.G) <= PARITY_RTOL
    assert rel_fro(host(F), ref.F) <= PARITY_RTOL


@pytest.mark.parametrize("n,m,p,nu", [(97, 131, 1, 2), (300, 41, 7, 9), (1000, 777, 12, 20),
                                      (64, 32, 3, 29)])
def test_ragged_shapes_compressed(n, m, p, nu):
    """Ragged sizes (no multiple of any tile), p = 1, and l = min(n, m)."""
    say("ragged", n, m, p, nu)
    inst = synth.instance(n, m, p, nu, seed=n + m, snr_db=40.0)
    X = dev(inst.X)
    comp = cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R), p, nu, 2)
    cnmf.check()
    ref_comp = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 2)
    # feed both solvers the same compressed data (the oracle's, rounded to
    # FP32) so the outer loop is compared on identical inputs
    shared = tuple(dev(a) for a in (ref_comp.Q_L, ref_comp.Q_R, ref_comp.X_L, ref_comp.X_R))
    shared32 = oracle.RSIResult(*(host(a) for a in shared))
    ref = oracle.nenmf(inst.X, inst.G0, inst.F0, 8, 30, compressed=shared32)
    G, F, tr = _solve_gpu(inst, None, shared, 8, 30, replay=ref.steps)
    assert rel_fro(host(G), ref.G) <= PARITY_RTOL
    assert rel_fro(host(F), ref.F) <= PARITY_RTOL
    QL = host(comp[0])
    assert np.linalg.norm(QL.T @ QL - np.eye(p + nu)) <= 1e-5


@pytest.mark.parametrize("p,nu", [(16, 8), (16, 16), (17, 6), (24, 8), (30, 2)])
def test_wide_ranks_compressed(p, nu):
    """Ranks at and past 16 (the 16-lane and the 32-lane forms of the warm
    lambda_max certificate): iterates and every subproblem's L against the
    oracle on shared compressed data and replayed step counts."""
    say("wide_ranks", p, nu)
    inst = synth.instance(300, 260, p, nu, seed=p + nu, snr_db=40.0)
    ref_comp = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 2)
    shared = tuple(dev(a) for a in (ref_comp.Q_L, ref_comp.Q_R, ref_comp.X_L, ref_comp.X_R))
    shared32 = oracle.RSIResult(*(host(a) for a in shared))
    ref = oracle.nenmf(inst.X, inst.G0, inst.F0, 8, 30, compressed=shared32)
    G, F, tr = _solve_gpu(inst, None, shared, 8, 30, replay=ref.steps)
    assert rel_fro(host(G), ref.G) <= PARITY_RTOL
    assert rel_fro(host(F), ref.F) <= PARITY_RTOL
    np.testing.assert_allclose(host(tr.lips), ref.lips, rtol=1e-4)


def test_zero_outer_iterations_and_zero_factor():
    say("degenerate")
    inst = synth.instance(50, 40, 3, 2, seed=1)
    X = dev(inst.X)
    G, F, _ = _solve_gpu(inst, X, None, 0, 10)
    assert np.array_equal(host(G), inst.G0.astype(np.float64))
    # F = 0 makes W = F F^T = 0: L = 0, G is left unchanged, warning only
    G = dev(inst.G0)
    F = dev(np.zeros_like(inst.F0))
    cnmf.solve(G, F, X=X, p=3, outer_iters=1, inner_max=5)
    st = cnmf.check()
    assert st & cnmf.ST_ZERO_LIPS
    assert np.array_equal(host(G), inst.G0.astype(np.float64))


def test_validate_input_flags_negative_and_nan():
    say("validate")
    inst = synth.instance(64, 48, 3, 4, seed=2)
    Xbad = inst.X.copy()
    Xbad[3, 5] = -1.0
    cnmf.rsi(dev(Xbad), dev(inst.omega_L), dev(inst.omega_R), 3, 4, 1, validate=True)
    with pytest.raises(cnmf.CnmfError) as ei:
        cnmf.check()
    assert ei.value.status & cnmf.ST_NEGATIVE
    Xbad[3, 5] = np.nan
    cnmf.rsi(dev(Xbad), dev(inst.omega_L), dev(inst.omega_R), 3, 4, 1, validate=True)
    with pytest.raises(cnmf.CnmfError) as ei:
        cnmf.check()
    assert ei.value.status & cnmf.ST_NONFINITE


def test_invalid_arguments_rejected():
    say("einval")
    inst = synth.instance(20, 10, 3, 2, seed=0)
    X = dev(inst.X)
    with pytest.raises(cnmf.CnmfError) as ei:      # l = 3 + 8 > m = 10
        cnmf.rsi(X, dev(np.zeros((10, 11))), dev(np.zeros((11, 20))), 3, 8, 1)
    assert ei.value.code == cnmf.EINVAL
    with pytest.raises(cnmf.CnmfError):             # q = 0
        cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R), 3, 2, 0)


@pytest.mark.parametrize("method", ["plain", "compressed"])
def test_solve_bitwise_repeatable(method):
    """Every reduction runs in a fixed order: two free-running solves on the
    same inputs give the same bits (factors, step counts, bounds)."""
    say("repeatable", method)
    inst = synth.instance(2000, 1500, 12, 10, seed=8, snr_db=30.0)
    X = dev(inst.X)
    comp = None
    if method == "compressed":
        comp = cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R), 12, 10, 4)
    runs = []
    for _ in range(2):
        G, F, tr = _solve_gpu(inst, X, comp, 25, 500)
        runs.append((host(G), host(F), host(tr.steps), host(tr.tols), host(tr.lips)))
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def test_rows_beyond_the_limit_rejected():
    """n or m above CNMF_MAX_ROWS: CNMF_EINVAL before anything is enqueued
    (the buffers are never read)."""
    say("max_rows")
    import torch
    n, m, p, nu = 70000, 40, 3, 2
    G = torch.zeros(n, p, device="cuda")
    F = torch.zeros(p, m, device="cuda")
    comp = (torch.zeros(n, p + nu, device="cuda"), torch.zeros(m, p + nu, device="cuda"),
            torch.zeros(p + nu, m, device="cuda"), torch.zeros(n, p + nu, device="cuda"))
    with pytest.raises(cnmf.CnmfError) as ei:
        cnmf.solve(G, F, compressed=comp, p=p, outer_iters=1, inner_max=5)
    assert ei.value.code == cnmf.EINVAL
    assert cnmf.check() == 0
