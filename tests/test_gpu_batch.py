"""Batched form: many instances of uneven n, m, p in persistent launches
(schedule of rounds), outer loop captured in a HIP graph.  Checked against
the FP64 oracle per instance on shared compressed data, and bitwise against
the single-instance path on the same workgroup decomposition."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import PARITY_RTOL, dev, follow_decisions, host, rel_fro, say

pytestmark = pytest.mark.gpu

cnmf = pytest.importorskip("paper_1812_04315_amd")

SHAPES = [(97, 131, 3, 6), (300, 41, 7, 9), (500, 420, 12, 10), (64, 200, 5, 10),
          (256, 256, 20, 10), (1000, 300, 16, 10)]


def _shared(inst, q=2):
    """The oracle's compressed data rounded to FP32, on the device and back."""
    r = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, q)
    d = tuple(dev(a) for a in (r.Q_L, r.Q_R, r.X_L, r.X_R))
    return d, oracle.RSIResult(*(host(a) for a in d))


def _desc(inst, comp, T, replay=None):
    import torch
    return dict(p=inst.p, nu=inst.ell - inst.p, Q_L=comp[0], Q_R=comp[1], X_L=comp[2],
                X_R=comp[3], G=dev(inst.G0), F=dev(inst.F0),
                steps=torch.zeros(T, 2, dtype=torch.int32, device="cuda"),
                replay=None if replay is None else torch.from_numpy(
                    np.ascontiguousarray(replay, dtype=np.int32)).cuda())


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_matches_oracle_on_shared_data(use_graph):
    say("batch_oracle", use_graph)
    T, K = 8, 30
    insts = [synth.instance(n, m, p, nu, seed=10 + k, snr_db=40.0)
             for k, (n, m, p, nu) in enumerate(SHAPES)]
    descs, refs = [], []
    for inst in insts:
        comp, comp32 = _shared(inst)
        ref = oracle.nenmf(inst.X, inst.G0, inst.F0, T, K, compressed=comp32)
        refs.append(ref)
        descs.append(_desc(inst, comp, T, replay=ref.steps))
    b = cnmf.Batch(descs, outer_iters=T, inner_max=K)
    b.solve(use_graph)
    cnmf.check()
    first = [(host(d["G"]), host(d["F"])) for d in descs]
    for d, ref, (G, F) in zip(descs, refs, first):
        assert np.array_equal(host(d["steps"]).astype(int), ref.steps)
        assert rel_fro(G, ref.G) <= PARITY_RTOL
        assert rel_fro(F, ref.F) <= PARITY_RTOL
    if use_graph:
        # replays of the captured loop, with eager work in between, give the
        # same result every time
        for rep in range(2):
            for d, inst in zip(descs, insts):
                d["G"].copy_(dev(inst.G0))
                d["F"].copy_(dev(inst.F0))
            b.solve(True)
            cnmf.check()
            for d, (G, F) in zip(descs, first):
                assert np.array_equal(host(d["G"]), G)
                assert np.array_equal(host(d["F"]), F)
    b.close()


def test_batch_stopping_rule_without_replay():
    say("batch_stop")
    T, K = 10, 60
    insts = [synth.instance(n, m, p, nu, seed=30 + k, snr_db=40.0)
             for k, (n, m, p, nu) in enumerate(SHAPES[:4])]
    descs, comps = [], []
    for inst in insts:
        comp, comp32 = _shared(inst)
        comps.append(comp32)
        descs.append(_desc(inst, comp, T))
    b = cnmf.Batch(descs, outer_iters=T, inner_max=K)
    b.solve(True)
    cnmf.check()
    for d, inst, comp32 in zip(descs, insts, comps):
        steps = host(d["steps"]).astype(int)
        # the oracle's own decisions, following the GPU's only within the
        # margin of the bound
        ref, followed = follow_decisions(steps, lambda rep: oracle.nenmf(
            inst.X, inst.G0, inst.F0, T, K, compressed=comp32, keep_pg=True, replay=rep))
        if followed:
            say("followed", followed)
        assert rel_fro(host(d["G"]), ref.G) <= PARITY_RTOL
        assert rel_fro(host(d["F"]), ref.F) <= PARITY_RTOL
    b.close()


def test_batch_many_rounds_bitwise_equals_single_instance():
    """More workgroups than resident slots: several rounds per launch.  With
    one tile per workgroup on both sides the batched and the single-instance
    launches decompose every instance identically, so results are bitwise
    equal."""
    say("batch_rounds")
    rng = np.random.default_rng(5)
    T, K = 4, 20
    descs, singles = [], []
    for k in range(48):
        n, m = int(rng.integers(300, 900)), int(rng.integers(200, 700))
        p = int(rng.integers(5, 21))
        inst = synth.instance(n, m, p, 10, seed=100 + k, snr_db=20.0)
        comp, _ = _shared(inst)
        replay = rng.integers(1, K + 1, size=(T, 2))
        descs.append(_desc(inst, comp, T, replay=replay))
        import torch
        G, F = dev(inst.G0), dev(inst.F0)
        cnmf.solve(G, F, compressed=comp, p=p, nu=10, outer_iters=T, inner_max=K,
                   replay=torch.from_numpy(replay.astype(np.int32)).cuda())
        singles.append((host(G), host(F)))
    cnmf.check()
    b = cnmf.Batch(descs, outer_iters=T, inner_max=K, tiles_g=1, tiles_f=1)
    b.solve(True)
    cnmf.check()
    for d, (G, F) in zip(descs, singles):
        assert np.array_equal(host(d["G"]), G)
        assert np.array_equal(host(d["F"]), F)
    b.close()


def test_batch_rsi_and_tune():
    say("batch_rsi_tune")
    T, K = 6, 30
    insts = [synth.instance(n, m, p, nu, seed=50 + k, snr_db=20.0)
             for k, (n, m, p, nu) in enumerate(SHAPES)]
    import torch
    descs = []
    for inst in insts:
        n, m = inst.X.shape
        ell = inst.ell
        comp = (torch.empty(n, ell, device="cuda"), torch.empty(m, ell, device="cuda"),
                torch.empty(ell, m, device="cuda"), torch.empty(n, ell, device="cuda"))
        d = _desc(inst, comp, T)
        d.update(X=dev(inst.X, (m + 3) // 4 * 4), omega_L=dev(inst.omega_L),
                 omega_R=dev(inst.omega_R))
        descs.append(d)
    b = cnmf.Batch(descs, q=2, outer_iters=T, inner_max=K)
    b.rsi()
    cnmf.check()
    for d, inst in zip(descs, insts):
        # noisy data: compare what is range-invariant (signal projector,
        # compressed reconstruction error) with the oracle
        ref = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 2)
        QL, QR, XL = host(d["Q_L"]), host(d["Q_R"]), host(d["X_L"])
        ell = inst.ell
        for Q in (QL, QR):
            assert np.linalg.norm(Q.T @ Q - np.eye(ell)) <= 1e-5
        Xh = inst.X.astype(np.float64)
        U, s, Vt = np.linalg.svd(Xh, full_matrices=False)
        for Q, Qo, S in ((QL, ref.Q_L, U[:, :inst.p]), (QR, ref.Q_R, Vt[:inst.p].T)):
            assert rel_fro(Q @ (Q.T @ S), Qo @ (Qo.T @ S)) <= PARITY_RTOL
        e_gpu = np.linalg.norm(Xh - QL @ XL) / np.linalg.norm(Xh)
        e_ref = np.linalg.norm(Xh - ref.Q_L @ ref.X_L) / np.linalg.norm(Xh)
        assert abs(e_gpu - e_ref) <= 1e-3 * e_ref
    tg, tf = b.tune(2)
    assert tg in (1, 2, 4) and tf in (1, 2, 4)
    # the tuned schedule solves the same problems: replay the oracle's counts
    refs = []
    for d, inst in zip(descs, insts):
        comp32 = oracle.RSIResult(*(host(d[k]) for k in ("Q_L", "Q_R", "X_L", "X_R")))
        ref = oracle.nenmf(inst.X, inst.G0, inst.F0, T, K, compressed=comp32)
        refs.append(ref)
    b.close()
    descs2 = []
    for d, ref, inst in zip(descs, refs, insts):
        d2 = _desc(inst, (d["Q_L"], d["Q_R"], d["X_L"], d["X_R"]), T, replay=ref.steps)
        descs2.append(d2)
    b2 = cnmf.Batch(descs2, outer_iters=T, inner_max=K, tiles_g=tg, tiles_f=tf)
    b2.solve(True)
    cnmf.check()
    for d, ref in zip(descs2, refs):
        assert rel_fro(host(d["G"]), ref.G) <= PARITY_RTOL
        assert rel_fro(host(d["F"]), ref.F) <= PARITY_RTOL
    b2.close()


def test_batch_rejects_bad_descriptors():
    say("batch_einval")
    inst = synth.instance(50, 40, 3, 2, seed=1)
    comp, _ = _shared(inst, 1)
    d = _desc(inst, comp, 2)
    d["nu"] = 60                      # l > min(n, m)
    with pytest.raises(cnmf.CnmfError) as ei:
        cnmf.Batch([d], outer_iters=2)
    assert ei.value.code == cnmf.EINVAL
    d["nu"] = 2
    with pytest.raises(cnmf.CnmfError):
        cnmf.Batch([d], outer_iters=2, tiles_g=3)


def test_batch_rsi_noiseless_bases_match_oracle():
    """Exactly low-rank instances of uneven shapes: every basis column is
    fixed (deficient columns come from the other Gaussian draw), so the
    batched bases and compressed data match the oracle entry by entry."""
    say("batch_rsi_exact")
    import torch
    shapes = [(200, 150, 5, 10), (97, 131, 3, 6), (300, 41, 7, 9), (500, 420, 12, 10)]
    insts = [synth.instance(n, m, p, nu, seed=70 + k) for k, (n, m, p, nu) in enumerate(shapes)]
    descs = []
    for inst in insts:
        n, m = inst.X.shape
        ell = inst.ell
        ld = (m + 3) // 4 * 4
        comp = (torch.empty(n, ell, device="cuda"), torch.empty(m, ell, device="cuda"),
                torch.empty(ell, m, device="cuda"), torch.empty(n, ell, device="cuda"))
        d = _desc(inst, comp, 2)
        d.update(X=dev(inst.X, ld), omega_L=dev(inst.omega_L), omega_R=dev(inst.omega_R))
        descs.append(d)
    b = cnmf.Batch(descs, q=4, outer_iters=2, inner_max=10)
    b.rsi()
    cnmf.check()
    for d, inst in zip(descs, insts):
        ref = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 4)
        for key, r in (("Q_L", ref.Q_L), ("Q_R", ref.Q_R), ("X_L", ref.X_L), ("X_R", ref.X_R)):
            assert rel_fro(host(d[key]), r) <= PARITY_RTOL, key
    b.close()


def test_tuned_tiles_persist(tmp_path):
    """cnmf_batch_tune's choice is recorded in a JSON table keyed by device,
    shapes and loop settings, and a later batch of the same shapes starts
    from it without tuning again."""
    say("batch_tune_cache")
    T, K = 4, 30
    insts = [synth.instance(n, m, p, nu, seed=60 + k, snr_db=30.0)
             for k, (n, m, p, nu) in enumerate(SHAPES[:3])]
    cache = str(tmp_path / "tiles.json")
    descs = [_desc(inst, _shared(inst)[0], T) for inst in insts]
    b = cnmf.Batch(descs, outer_iters=T, inner_max=K, tune_cache=cache)
    tiles = b.tune(2)
    b.close()
    import json
    table = json.load(open(cache))
    assert list(table.values()) == [list(tiles)]
    b2 = cnmf.Batch([_desc(inst, _shared(inst)[0], T) for inst in insts], outer_iters=T,
                    inner_max=K, tune_cache=cache)
    assert b2.tiles == tiles
    b2.solve(True)
    cnmf.check()
    b2.close()
