"""Pins of the oracle's storage rounding (round to nearest even, FP32 and BF16)
and of the 12-real reconstruction, independent of the oracle itself:
hand-worked values from the definition of the formats, brute-force nearest
neighbours, torch's own float32 -> bfloat16 conversion on values that are
exact in float32, the unitarity identity for row 2, and planted mistakes
(truncation, round half up, double rounding through FP32) that must fail."""
import numpy as np
import pytest

import lgt_inputs as li
from oracle import rounding as R

torch = pytest.importorskip("torch")

# BF16 at 1.0: 7 stored mantissa bits, so neighbours 1, 1 + 2^-7, 1 + 2^-6, ...
BF16_CASES = [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                                  # tie, 1 has an even last bit
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),                  # tie, 1 + 2^-7 is odd: up
    (1.0 + 2.0 ** -8 + 2.0 ** -40, 1.0 + 2.0 ** -7),         # above the tie by less than an FP32 ulp
    (1.0 + 3 * 2.0 ** -8 - 2.0 ** -40, 1.0 + 2.0 ** -7),     # below the tie by less than an FP32 ulp
    (-(1.0 + 3 * 2.0 ** -8), -(1.0 + 2.0 ** -6)),            # symmetric for negative values
    (2.0 - 2.0 ** -9, 2.0),                                  # carries into the exponent
    (0.75 + 2.0 ** -10, 0.75),                               # ulp at 0.75 is 2^-8: tie, 0.75 even
    (0.0, 0.0),
    (3.0 * 2.0 ** -100 + 2.0 ** -108, 3.0 * 2.0 ** -100),    # tie far from 1: to even
]
F32_CASES = [
    (1.0 + 2.0 ** -24, 1.0),                                 # tie, to even
    (1.0 + 3 * 2.0 ** -24, 1.0 + 2.0 ** -22),                # tie, up to even
    (1.0 + 2.0 ** -24 + 2.0 ** -50, 1.0 + 2.0 ** -23),       # just above the tie
    (-(1.0 + 2.0 ** -24), -1.0),
]


def _check_cases(fn, cases):
    x = np.array([c[0] for c in cases])
    want = np.array([c[1] for c in cases])
    got = fn(x)
    return np.array_equal(got, want) and np.array_equal(np.signbit(got), np.signbit(want))


def _bf16_nearest_ok(fn, x):
    """Brute force from the definition: the result is a BF16 value, no BF16
    neighbour is closer, and a tie picks the even last bit."""
    r = fn(x)
    bits = r.view(np.uint64)
    if np.any(bits & ((np.uint64(1) << np.uint64(45)) - np.uint64(1))):
        return False
    kept = bits >> np.uint64(45)
    lo = (kept - np.uint64(1)) << np.uint64(45)
    hi = (kept + np.uint64(1)) << np.uint64(45)
    d = np.abs(x - r)
    dlo = np.abs(x - lo.view(np.float64))
    dhi = np.abs(x - hi.view(np.float64))
    if np.any(d > dlo) or np.any(d > dhi):
        return False
    tie = (d == dlo) | (d == dhi)
    return not np.any(tie & ((kept & np.uint64(1)) == np.uint64(1)))


def _random_values(seed, n=200000):
    g = np.random.default_rng(seed)
    x = g.standard_normal(n) * np.exp2(g.integers(-60, 60, n))
    # planted ties and near-ties of BF16 at random BF16 values
    t = g.standard_normal(n // 4).astype(np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    tie = (t | np.uint32(0x8000)).view(np.float32).astype(np.float64)
    eps = np.abs(tie) * 2.0 ** -40
    return np.concatenate([x, tie, tie + eps, tie - eps])


def test_round_bf16_hand_values():
    assert _check_cases(R.round_bf16, BF16_CASES)


def test_round_f32_hand_values():
    assert _check_cases(R.round_f32, F32_CASES)


def test_round_bf16_nearest_even_brute_force():
    assert _bf16_nearest_ok(R.round_bf16, _random_values(7))


def test_round_bf16_matches_torch_on_float32_values():
    """For values exact in float32 there is one rounding step either way, so
    torch's float32 -> bfloat16 conversion (round to nearest even) must agree."""
    x = _random_values(8).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = R.round_bf16(x.astype(np.float64))
    np.testing.assert_array_equal(got, want)


def test_round_bf16_rejects_out_of_range():
    for bad in (2.0 ** -130, 2.0 ** 128, np.inf, np.nan):
        with pytest.raises(ValueError):
            R.round_bf16(np.array([bad]))


def _truncate(x):
    b = np.ascontiguousarray(x, np.float64).view(np.uint64)
    return ((b >> np.uint64(45)) << np.uint64(45)).view(np.float64)


def _half_up(x):
    b = np.ascontiguousarray(x, np.float64).view(np.uint64)
    return (((b + (np.uint64(1) << np.uint64(44))) >> np.uint64(45)) << np.uint64(45)).view(np.float64)


def _via_f32(x):
    f = np.asarray(x, np.float64).astype(np.float32)
    return torch.from_numpy(f).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("mutant", [_truncate, _half_up, _via_f32])
def test_rounding_pins_catch_mutants(mutant):
    """Each planted mistake fails the hand values or the brute-force check."""
    fails = (not _check_cases(mutant, BF16_CASES)) or (not _bf16_nearest_ok(mutant, _random_values(9)))
    assert fails


def test_reconstruct_row2_unitary_identity():
    """Row 2 of a special unitary matrix is conj(row0 x row1); a matrix of
    determinant -1 gets the negated row, and a swap of the cross product's
    operands is caught."""
    L = (2, 2, 2, 4)
    U = li.links(L, "haar", 11)
    u = U[..., 0] + 1j * U[..., 1]
    got = R.reconstruct_row2(u)
    assert np.abs(got - u).max() < 1e-14
    v = u.copy()
    v[..., 2, :] *= -1.0                       # det = -1: still unitary
    assert np.abs(R.reconstruct_row2(v)[..., 2, :] + v[..., 2, :]).max() < 1e-14
    a, b = u[..., 0, :], u[..., 1, :]
    wrong = np.conj(np.cross(b, a))            # operands swapped
    assert np.abs(wrong - u[..., 2, :]).max() > 0.5


def test_stored_links():
    L = (2, 2, 2, 4)
    U = li.links(L, "haar", 12)
    np.testing.assert_array_equal(R.stored_links(U, R.PREC_F64, 18), U)
    assert np.abs(R.stored_links(U, R.PREC_F64, 12) - U).max() < 1e-14
    S = R.stored_links(U, R.PREC_BF16, 12)
    np.testing.assert_array_equal(S[..., :2, :, :], R.round_bf16(U[..., :2, :, :]))
    assert np.abs(S - U).max() < 2.0 ** -7
    F = R.stored_links(U, R.PREC_F32, 18)
    np.testing.assert_array_equal(F, U.astype(np.float32).astype(np.float64))
