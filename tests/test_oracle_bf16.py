"""Pins of the oracle's bfloat16 emulation (precision form): the rounding
itself (round to nearest, ties to even) and the range property of the
emulated randomized subspace iteration."""
import numpy as np
import pytest
import torch

import oracle
import synth


def _f32(bits):
    return np.array(bits, dtype=np.uint32).view(np.float32)


def test_hand_rounded_values():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even
    # pattern 0x3F80; 1 + 3 * 2^-8 is halfway between 0x3F81 and 0x3F82 -> 0x3F82.
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 0.0, -0.0,
                  np.inf, -np.inf], dtype=np.float32)
    want = [0x3F80, 0x3F80, 0x3F82, 0x3F81, 0xC020, 0x0000, 0x8000, 0x7F80, 0xFF80]
    assert oracle.bf16_bits(x).tolist() == want
    # just above a tie rounds up, just below rounds down
    assert oracle.bf16_bits(_f32([0x3F808001, 0x3F807FFF])).tolist() == [0x3F81, 0x3F80]
    # the largest finite values round to infinity past the last tie
    assert oracle.bf16_bits(_f32([0x7F7FFFFF]))[0] == 0x7F80
    assert np.isnan(oracle.bf16_value(oracle.bf16_bits(np.float32(np.nan)))).all()


def test_matches_library_conversion():
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 2 ** 32, size=200000, dtype=np.uint64).astype(np.uint32)
    # force many exact ties and near-ties
    bits[:50000] = (bits[:50000] & 0xFFFF0000) | 0x8000
    bits[50000:60000] = (bits[50000:60000] & 0xFFFF0000) | 0x7FFF
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(oracle.bf16_bits(x), ref)


def test_round_trip_is_identity_on_representable_values():
    rng = np.random.default_rng(1)
    b = rng.integers(0, 2 ** 16, size=50000, dtype=np.uint32).astype(np.uint16)
    v = oracle.bf16_value(b)
    keep = np.isfinite(v)
    assert np.array_equal(oracle.bf16_bits(v[keep].astype(np.float32)), b[keep])


@pytest.mark.parametrize("q", [1, 3])
def test_emulated_rsi_keeps_exact_range(q):
    """Rounding the operands never leaves range(X): for rank(X) <= l the
    emulated bases still capture X exactly (to FP64 roundoff)."""
    inst = synth.instance(120, 90, 4, 6, seed=5)
    Xb = oracle.bf16_round(inst.X)
    r = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, q, bf16=True)
    for Q in (r.Q_L, r.Q_R):
        assert np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) <= 1e-12
    # rounding X makes it full rank; the captured part is the dominant one
    s = np.linalg.svd(Xb, compute_uv=False)
    tail = np.sqrt(np.sum(s[10:] ** 2)) / np.linalg.norm(Xb)
    assert np.linalg.norm(Xb - r.Q_L @ (r.Q_L.T @ Xb)) <= 10 * tail * np.linalg.norm(Xb) + 1e-12
    assert np.linalg.norm(Xb - (Xb @ r.Q_R) @ r.Q_R.T) <= 10 * tail * np.linalg.norm(Xb) + 1e-12


def test_emulated_products_use_rounded_operands():
    """X_R of the emulation is bf16(X) times bf16(Q_R): with the rounding of
    Q_R dropped the difference is of the order of bf16 resolution."""
    inst = synth.instance(150, 110, 5, 5, seed=6, snr_db=30.0)
    r = oracle.rsi(inst.X, inst.omega_L, inst.omega_R, 2, bf16=True)
    Xb = oracle.bf16_round(inst.X)
    exact = Xb @ oracle.bf16_round(r.Q_R)
    assert np.allclose(r.X_R, exact, rtol=0, atol=1e-12 * np.abs(exact).max())
    unrounded = Xb @ r.Q_R
    d = np.abs(unrounded - r.X_R).max() / np.abs(unrounded).max()
    assert 1e-5 < d < 2 ** -7
