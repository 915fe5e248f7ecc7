"""Seeded synthetic inputs for compressed NeNMF.

This module only draws inputs. It holds none of the method's arithmetic and
is the one piece shared by the FP64 oracle (``oracle/``) and the HIP path
(``paper_1812_04315_amd``): both consume exactly the FP32 arrays returned here.

Data model (Sec. 4, experimental validation): nonnegative random factors
G* (n x p) and F* (p x m), X = G* F* plus Gaussian noise at a stated
signal-to-noise ratio.  The paper says only "random nonnegative" and "around
30 dB"; the reading used here is G*, F* ~ Uniform[0, 1), E ~ N(0, 1) scaled so
that 10 log10(||G*F*||^2 / ||E||^2) equals the SNR exactly, then
X = max(0, G*F* + E) because NMF requires X >= 0 (Sec. 1, Eq. (1)).

The random matrices the method itself draws (Algorithm 2: Omega_L, Omega_R)
and the initial factors G0, F0 (Algorithm 1 takes them as inputs) are drawn
here too and passed to both implementations, so no RNG lives in either.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = ["Instance", "planted", "solver_inputs", "instance", "batched_shapes"]


@dataclass
class Instance:
    X: np.ndarray        # n x m, float32, >= 0
    G_true: np.ndarray   # n x p, float32 (planted factor, for reference only)
    F_true: np.ndarray   # p x m, float32
    omega_L: np.ndarray  # m x l, float32, N(0,1)   (Algorithm 2, Omega_L)
    omega_R: np.ndarray  # l x n, float32, N(0,1)   (Algorithm 2, Omega_R)
    G0: np.ndarray       # n x p, float32, U[0,1)
    F0: np.ndarray       # p x m, float32, U[0,1)
    p: int
    ell: int
    snr_db: float | None
    seed: int


def planted(n: int, m: int, p: int, seed: int, snr_db: float | None = None,
            chunk_rows: int = 2048):
    """X = max(0, G* F* + E) with the exact SNR; returns (X, G*, F*) in FP32.

    Draw order from ``numpy.random.default_rng(seed)``: G* (n x p), F* (p x m),
    then E (n x m) row-chunk by row-chunk.  E is drawn twice from the same
    stream state (once for its norm, once to add) so that peak memory stays at
    one FP64 chunk for large instances.
    """
    rng = np.random.default_rng(seed)
    G = rng.random((n, p))
    F = rng.random((p, m))
    X = np.empty((n, m), dtype=np.float32)
    if snr_db is None:
        for r0 in range(0, n, chunk_rows):
            r1 = min(n, r0 + chunk_rows)
            X[r0:r1] = (G[r0:r1] @ F).astype(np.float32)
        return X, G.astype(np.float32), F.astype(np.float32)
    state = rng.bit_generator.state
    sig2 = 0.0
    noise2 = 0.0
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        S = G[r0:r1] @ F
        sig2 += float(np.dot(S.ravel(), S.ravel()))
        E = rng.standard_normal((r1 - r0, m))
        noise2 += float(np.dot(E.ravel(), E.ravel()))
    scale = math.sqrt(sig2 / (noise2 * 10.0 ** (snr_db / 10.0)))
    rng.bit_generator.state = state
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        S = G[r0:r1] @ F
        E = rng.standard_normal((r1 - r0, m))
        S += scale * E
        np.maximum(S, 0.0, out=S)
        X[r0:r1] = S.astype(np.float32)
    return X, G.astype(np.float32), F.astype(np.float32)


def solver_inputs(n: int, m: int, p: int, ell: int, seed: int):
    """Omega_L (m x l), Omega_R (l x n), G0 (n x p), F0 (p x m), all FP32.

    Drawn from ``default_rng(seed + 1)`` in that order, so that the same data
    seed gives the same projections for every caller.
    """
    rng = np.random.default_rng(seed + 1)
    omega_L = rng.standard_normal((m, ell)).astype(np.float32)
    omega_R = rng.standard_normal((ell, n)).astype(np.float32)
    G0 = rng.random((n, p)).astype(np.float32)
    F0 = rng.random((p, m)).astype(np.float32)
    return omega_L, omega_R, G0, F0


def instance(n: int, m: int, p: int, nu: int, seed: int = 0,
             snr_db: float | None = None) -> Instance:
    """One planted instance with its projection and initial matrices; l = p + nu."""
    ell = p + nu
    X, Gt, Ft = planted(n, m, p, seed, snr_db)
    oL, oR, G0, F0 = solver_inputs(n, m, p, ell, seed)
    return Instance(X, Gt, Ft, oL, oR, G0, F0, p, ell, snr_db, seed)


def batched_shapes(count: int, seed: int = 0, n_range=(500, 4000),
                   m_range=(300, 3000), p_range=(5, 20)):
    """Uneven instance shapes: n, m log-uniform in the ranges, p uniform."""
    rng = np.random.default_rng(seed)
    ln = rng.uniform(math.log(n_range[0]), math.log(n_range[1]), count)
    lm = rng.uniform(math.log(m_range[0]), math.log(m_range[1]), count)
    n = np.floor(np.exp(ln)).astype(int)
    m = np.floor(np.exp(lm)).astype(int)
    p = rng.integers(p_range[0], p_range[1] + 1, count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(n, m, p)]
