"""Helpers shared by the GPU tests (device transfer, tolerances)."""
import sys

import numpy as np

# Relative Frobenius tolerance for FP32 GPU results against the FP64 oracle
# on identical seeded inputs.
PARITY_RTOL = 1e-4


def dev(a, ld=None):
    """Copy a host array to the GPU as float32, optionally with a row pitch."""
    import torch
    a = np.ascontiguousarray(a, dtype=np.float32)
    if ld is None or a.ndim != 2 or ld == a.shape[1]:
        return torch.from_numpy(a).cuda()
    buf = torch.zeros(a.shape[0], ld, dtype=torch.float32)
    buf[:, :a.shape[1]] = torch.from_numpy(a)
    return buf.cuda()[:, :a.shape[1]]


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_fro(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def say(*msg):
    print("[case]", *msg, flush=True)
    sys.stdout.flush()


# Relative distance of the oracle's projected-gradient norm from the bound
# within which a stop decision may go either way: FP32 iterates carry norms
# about 1e-6 from the FP64 ones, so 1e-3 leaves a wide safety factor while a
# step off by one elsewhere (a norm 10 % or more from the bound) fails.
STOP_MARGIN = 1e-3


def follow_decisions(gpu_steps, run_oracle, margin=STOP_MARGIN, max_follow=64):
    """The oracle's own run of an outer loop, following a GPU stop decision
    only where it differs from the oracle's and the oracle's projected-
    gradient norm at the decisive step lies within ``margin`` of the bound.

    ``run_oracle(replay)`` runs ``oracle.nenmf(..., replay=replay,
    keep_pg=True)``; a replay entry < 0 leaves that inner loop to the
    bound.  At the first differing (t, side) the counts must differ by one
    and the oracle's norm at the smaller count must be within the margin;
    the oracle is then rerun taking the GPU's count there and its own
    decisions elsewhere.  Returns (result, followed [(t, side, k_gpu, k_ref)])."""
    import numpy as np
    gpu_steps = np.asarray(gpu_steps, dtype=int)
    T = gpu_steps.shape[0]
    replay = -np.ones((T, 2), dtype=int)
    followed = []
    while True:
        ref = run_oracle(replay)
        diff = np.argwhere(ref.steps != gpu_steps)
        if len(diff) == 0:
            return ref, followed
        t, s = (int(v) for v in diff[0])
        kg, ko = int(gpu_steps[t, s]), int(ref.steps[t, s])
        d = min(kg, ko)
        tol = float(ref.tols[t, s])
        pg = float(ref.pg[t][s][d - 1]) if d >= 1 else float("nan")
        assert abs(kg - ko) == 1, f"(t={t}, side={s}): GPU {kg} steps, oracle {ko}"
        assert abs(pg - tol) <= margin * tol, (
            f"(t={t}, side={s}): GPU {kg} steps, oracle {ko}; oracle norm {pg:.9e} at step {d} "
            f"is not within {margin} of the bound {tol:.9e}")
        followed.append((t, s, kg, ko))
        assert len(followed) <= max_follow, "too many decisions at the margin"
        replay[t, s] = kg


def gf_rel_err(G1, F1, G2, F2):
    """||G1 F1 - G2 F2||_F / ||G2 F2||_F without forming the n x m products."""
    import numpy as np
    G1, F1, G2, F2 = (np.asarray(a, dtype=np.float64) for a in (G1, F1, G2, F2))
    a = float(np.sum((G1.T @ G1) * (F1 @ F1.T)))
    b = float(np.sum((G2.T @ G2) * (F2 @ F2.T)))
    c = float(np.sum((G1.T @ G2) * (F1 @ F2.T)))
    return float(np.sqrt(max(a + b - 2.0 * c, 0.0) / b))
