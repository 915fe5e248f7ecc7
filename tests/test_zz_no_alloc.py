"""cnmf_solve_noalloc, the solve that allocates no device memory (its
scratch is the library's static array on each GPU), against cnmf_solve on
two calls in a row, the second on a smaller problem, for both methods; and
its size limit."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

cnmf = pytest.importorskip("paper_1812_04315_amd")


def _pair(n, m, p, nu, seed, method):
    inst = synth.instance(n, m, p, nu, seed=seed, snr_db=30.0)
    X = dev(inst.X)
    comp = None
    if method == "compressed":
        comp = cnmf.rsi(X, dev(inst.omega_L), dev(inst.omega_R), p, nu, 2)
    out = []
    for noalloc in (False, True):
        G, F = dev(inst.G0), dev(inst.F0)
        tr = cnmf.make_trace(n, m, p, 12, G.device, history=False)
        cnmf.solve(G, F, X=X if comp is None else None, compressed=comp, p=p, nu=nu,
                   outer_iters=12, inner_max=50, trace=tr, noalloc=noalloc)
        cnmf.check()
        out.append((host(G), host(F), host(tr.steps), host(tr.lips)))
    (Ga, Fa, sa, la), (Gb, Fb, sb, lb) = out
    assert np.array_equal(sa, sb)
    assert np.array_equal(la, lb)
    # the same kernels on the same decomposition: bitwise equal
    assert np.array_equal(Ga, Gb) and np.array_equal(Fa, Fb)


@pytest.mark.parametrize("method", ["compressed", "plain"])
def test_noalloc_matches_solve_on_two_calls(method):
    say("noalloc", method)
    _pair(3000, 2500, 12, 10, 1, method)    # first call
    _pair(700, 450, 6, 8, 2, method)        # second call, smaller


def test_noalloc_rejects_problems_beyond_its_scratch():
    """Plain NeNMF at 60000 x 60000, p = 32 needs more scratch than the
    static array (32 MiB) holds: CNMF_ETOOBIG, and nothing is enqueued (X is never
    read, so a small buffer stands in for it)."""
    say("noalloc_limit")
    import torch
    ctx = cnmf.context()
    small = torch.zeros(64, device="cuda")
    prm = cnmf.params(32, 0, 1, 1, 5)
    rc = cnmf.lib().cnmf_solve_noalloc(ctx.h, cnmf.METHOD_PLAIN, 60000, 60000,
                                       ctypes.c_void_p(small.data_ptr()), 60000, None, None,
                                       None, None, ctypes.byref(prm),
                                       ctypes.c_void_p(small.data_ptr()),
                                       ctypes.c_void_p(small.data_ptr()), None, None)
    assert rc == cnmf.ETOOBIG
    assert cnmf.check() == 0
