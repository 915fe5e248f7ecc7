"""Further subproblem solvers on the same machinery, against the FP64 oracle
on identical seeded inputs: HALS and multiplicative updates (Sec. 1, Sec. 3)
on compressed and plain data, adaptive restart of the Nesterov loop (Sec. 4
footnote), and the device-time budget of the outer loop (Sec. 3)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import PARITY_RTOL, dev, follow_decisions, gf_rel_err, host, rel_fro, say

pytestmark = pytest.mark.gpu

cnmf = pytest.importorskip("paper_1812_04315_amd")


def _shared(inst, q=2):
    r = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, q)
    d = tuple(dev(a) for a in (r.Q_L, r.Q_R, r.X_L, r.X_R))
    return d, oracle.RSIResult(*(host(a) for a in d))


@pytest.mark.parametrize("solver", ["hals", "mu"])
@pytest.mark.parametrize("method", ["compressed", "plain"])
@pytest.mark.parametrize("n,m,p,nu,K", [(300, 250, 6, 10, 3), (1000, 700, 20, 8, 2),
                                        (20000, 300, 9, 6, 1)])
def test_hals_and_mu_against_oracle(solver, method, n, m, p, nu, K):
    """K updates per subproblem, 8 outer iterations (ranks on both sides of
    16; 20000 rows take two row tiles per wave)."""
    say("solver", solver, method, n, m, p, K)
    inst = synth.instance(n, m, p, nu, seed=n + p, snr_db=30.0)
    X = dev(inst.X)
    comp = comp32 = None
    if method == "compressed":
        comp, comp32 = _shared(inst)
    code = cnmf.SOLVER_HALS if solver == "hals" else cnmf.SOLVER_MU
    G, F = dev(inst.G0), dev(inst.F0)
    T = 8
    tr = cnmf.make_trace(n, m, p, T, G.device, history=False)
    cnmf.solve(G, F, X=None if comp else X, compressed=comp, p=p, nu=nu, outer_iters=T,
               inner_max=K, trace=tr, solver=code)
    cnmf.check()
    assert np.all(host(tr.steps) == K)
    ref = oracle.nenmf(None if comp else inst.X, inst.G0, inst.F0, T, K, compressed=comp32,
                       solver=solver)
    assert rel_fro(host(G), ref.G) <= PARITY_RTOL
    assert rel_fro(host(F), ref.F) <= PARITY_RTOL
    assert np.all(host(G) >= 0) and np.all(host(F) >= 0)


@pytest.mark.parametrize("n,m,p,nu", [(400, 300, 6, 10), (900, 700, 20, 8), (20000, 300, 9, 6)])
def test_restart_forced_steps(n, m, p, nu):
    """Adaptive restart with every loop held at a fixed step count (the
    restart decisions alone differ from the plain loop): iterates against the
    oracle's per-row restart."""
    say("restart_forced", n, m, p)
    inst = synth.instance(n, m, p, nu, seed=n + 1, snr_db=30.0)
    comp, comp32 = _shared(inst)
    T = 6
    rng = np.random.default_rng(p)
    replay = rng.integers(5, 40, size=(T, 2))
    G, F = dev(inst.G0), dev(inst.F0)
    import torch
    cnmf.solve(G, F, compressed=comp, p=p, nu=nu, outer_iters=T, inner_max=100,
               restart=cnmf.RESTART_GRADIENT,
               replay=torch.from_numpy(replay.astype(np.int32)).cuda())
    cnmf.check()
    ref = oracle.nenmf(None, inst.G0, inst.F0, T, 100, compressed=comp32, restart=True,
                       replay=replay)
    plain = oracle.nenmf(None, inst.G0, inst.F0, T, 100, compressed=comp32, replay=replay)
    assert rel_fro(ref.G, plain.G) > 10 * PARITY_RTOL   # restarts happened and matter
    assert rel_fro(host(G), ref.G) <= PARITY_RTOL
    assert rel_fro(host(F), ref.F) <= PARITY_RTOL


@pytest.mark.parametrize("method", ["compressed", "plain"])
def test_restart_free_running(method):
    """Restart with the global gradient bound, free running: the GPU's own
    stop decisions, followed by the oracle within the margin, and RRE(t)
    and G F against the oracle.  Every row takes a restart decision at every
    step (here about 10^6 of them); late in a loop a row's last move and its
    gradient-mapping step are both small, and those whose inner product lies
    within the FP32-against-FP64 difference of the iterates of zero go either
    way, each changing that row's path by about one momentum step.  The
    factors agree to the size of those steps (measured: 1e-3 relative, G F
    6e-5, RRE(t) 4e-4 at 1200 x 900), not to FP32 resolution, and are held
    to 1e-2, 1e-3 and 1e-3; test_restart_forced_steps checks the restart
    arithmetic itself at the parity bound."""
    say("restart_free", method)
    inst = synth.instance(1200, 900, 12, 10, seed=3, snr_db=30.0)
    X = dev(inst.X)
    comp = comp32 = None
    if method == "compressed":
        comp, comp32 = _shared(inst)
    T, K = 15, 100
    G, F = dev(inst.G0), dev(inst.F0)
    tr = cnmf.make_trace(1200, 900, 12, T, G.device)
    cnmf.solve(G, F, X=None if comp else X, compressed=comp, p=12, outer_iters=T, inner_max=K,
               trace=tr, restart=cnmf.RESTART_GRADIENT)
    cnmf.check()
    ref, followed = follow_decisions(host(tr.steps).astype(int), lambda rep: oracle.nenmf(
        None if comp else inst.X, inst.G0, inst.F0, T, K, compressed=comp32, restart=True,
        keep_pg=True, keep_history=True, replay=rep))
    errs = host(cnmf.rre(X, tr.G_hist, tr.F_hist))
    errs_ref = oracle.rre_history(inst.X, ref.history)
    d_rre = float(np.max(np.abs(errs - errs_ref) / errs_ref))
    d_gf = gf_rel_err(host(G), host(F), ref.G, ref.F)
    d_g = rel_fro(host(G), ref.G)
    say("followed", followed, "dRRE", d_rre, "GF", d_gf, "G", d_g, "F", rel_fro(host(F), ref.F))
    assert d_rre <= 1e-3
    assert d_gf <= 1e-3
    assert d_g <= 1e-2


@pytest.mark.parametrize("method", ["plain", "compressed"])
def test_time_budget_stops_the_outer_loop(method):
    """A device-time budget ends the outer loop early: the completed count
    is reported, and the factors are those of an unbudgeted run of that many
    iterations with the same inner step counts (bitwise).  The compressed
    solve runs its whole loop in one launch, where every workgroup leaves
    after the outer iteration at whose end workgroup 0 found the deadline
    passed."""
    say("time_budget", method)
    import torch
    inst = synth.instance(2000, 2000, 15, 10, seed=1, snr_db=30.0)
    X = dev(inst.X)
    comp = None
    if method == "compressed":
        comp = cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R), 15, 10, 2)
    T = 400 if comp is None else 2000
    budget = 2e-3
    G, F = dev(inst.G0), dev(inst.F0)
    tr = cnmf.make_trace(2000, 2000, 15, T, G.device, history=False)
    cnmf.solve(G, F, X=None if comp else X, compressed=comp, p=15, outer_iters=T, inner_max=100,
               trace=tr, time_budget=budget)
    cnmf.check()
    done = int(host(tr.outer_done)[0])
    say("outer iterations within 2 ms:", done)
    assert 1 <= done < T
    steps = host(tr.steps).astype(np.int32)[:done]
    G2, F2 = dev(inst.G0), dev(inst.F0)
    cnmf.solve(G2, F2, X=None if comp else X, compressed=comp, p=15, outer_iters=done,
               inner_max=100, replay=torch.from_numpy(np.ascontiguousarray(steps)).cuda())
    cnmf.check()
    assert np.array_equal(host(G), host(G2)) and np.array_equal(host(F), host(F2))
    # a budget that is not reached changes nothing
    tr2 = cnmf.make_trace(2000, 2000, 15, 5, G.device, history=False)
    G3, F3 = dev(inst.G0), dev(inst.F0)
    cnmf.solve(G3, F3, X=None if comp else X, compressed=comp, p=15, outer_iters=5, inner_max=100,
               trace=tr2, time_budget=100.0)
    cnmf.check()
    assert int(host(tr2.outer_done)[0]) == 5
