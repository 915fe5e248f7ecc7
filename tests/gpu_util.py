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
