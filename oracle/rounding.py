"""Rounding of float64 link elements to the stored FP32 / BF16 formats, and the
12-real reconstruction, as plain definitions.

TEST INFRASTRUCTURE ONLY: used by the test suite to state what a packed link
field must hold element by element; the library never imports it.

The paper's complex numbers have FP32 or FP64 real and imaginary parts (Sec. 4);
the links are SU(3) matrices (Sec. 1). A stored reduced-precision link holds
each real part rounded to the nearest representable value, ties to the value
with an even last mantissa bit (round to nearest even). BF16 keeps the FP32
exponent range with 7 stored mantissa bits; FP32 has 23.

* ``round_f32``: numpy's float64 -> float32 conversion (IEEE round to nearest
  even), widened back; exact in float64.
* ``round_bf16``: round to nearest even at 7 mantissa bits, done on the
  integer bits of the float64 value: the 45 dropped mantissa bits are compared
  with half a unit of the last kept place. One rounding step from the float64
  value, so no double rounding (a float64 just above a BF16 tie that first
  rounded to FP32 could land exactly on the tie and then round the wrong way).
  Defined for 0 and for magnitudes in [2^-126, 2^127] (BF16 normal numbers),
  the range a link element of an SU(3) matrix lives in.
* ``reconstruct_row2``: for a special unitary matrix the third row is the
  complex conjugate of the cross product of the first two; a 12-real field
  stores rows 0 and 1 and rebuilds row 2 this way.
"""
from __future__ import annotations

import numpy as np

_DROP = 52 - 7                  # float64 mantissa bits that BF16 drops
_HALF = np.uint64(1) << np.uint64(_DROP - 1)
_LOW = (np.uint64(1) << np.uint64(_DROP)) - np.uint64(1)


def round_f32(x):
    """float64 -> nearest float32 (ties to even), as float64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    """float64 -> nearest BF16 value (ties to even), as float64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    a = np.abs(x)
    ok = (a == 0) | ((a >= 2.0 ** -126) & (a <= 2.0 ** 127))
    if not np.all(ok):
        raise ValueError("round_bf16 is defined for 0 and magnitudes in [2^-126, 2^127]")
    bits = x.view(np.uint64)
    low = bits & _LOW
    kept = bits >> np.uint64(_DROP)
    up = (low > _HALF) | ((low == _HALF) & ((kept & np.uint64(1)) == np.uint64(1)))
    kept = kept + up.astype(np.uint64)
    return (kept << np.uint64(_DROP)).view(np.float64)


def reconstruct_row2(u):
    """u: complex [..., 3, 3]; returns a copy whose row 2 is conj(row0 x row1)."""
    u = np.array(u, dtype=np.complex128)
    a, b = u[..., 0, :], u[..., 1, :]
    c = np.empty_like(a)
    for j in range(3):
        k, l = (j + 1) % 3, (j + 2) % 3
        c[..., j] = a[..., k] * b[..., l] - a[..., l] * b[..., k]
    u[..., 2, :] = np.conj(c)
    return u


def _as_complex(U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    return U[..., 0] + 1j * U[..., 1]


def _as_real(u):
    return np.ascontiguousarray(np.stack([u.real, u.imag], axis=-1))


PREC_F64, PREC_F32, PREC_BF16 = 0, 1, 2


def round_elements(U, prec):
    """Every real of a canonical float64 array rounded to the storage precision."""
    if prec == PREC_F64:
        return np.array(U, dtype=np.float64)
    if prec == PREC_F32:
        return round_f32(U)
    if prec == PREC_BF16:
        return round_bf16(U)
    raise ValueError(f"bad precision {prec}")


def stored_links(U, prec, recon):
    """The link field a Dslash on a packed field of (prec, recon) applies, as
    canonical float64 [4][V][3][3][2]: every stored real rounded; for 12 reals,
    rows 0 and 1 rounded and row 2 rebuilt from them (in float64)."""
    R = round_elements(U, prec)
    if recon == 18:
        return R
    if recon != 12:
        raise ValueError(f"bad recon {recon}")
    return _as_real(reconstruct_row2(_as_complex(R)))
