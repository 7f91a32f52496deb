"""Element-by-element checks of reduced-precision Dslash outputs.

The reference is the FP64 oracle applied to exactly the numbers the GPU
computes with: the links as stored (every real rounded to nearest even; for 12
reals, row 2 rebuilt from the rounded rows) and the input vector rounded to
FP32. What remains is the FP32 arithmetic of the kernel, bounded per output
real by

    |got - ref| <= u32 * (64 * S + 8 * C)

with S the sum over the 8 hops of |U_ij| |chi_j| for that output row (which
bounds the sum of the magnitudes of the 48 real products an output real
accumulates: error <= 48 u32 S for chained FMAs) and C the sum of |chi_j| over
the hops, which covers the FP32 rebuild of row 2 (absolute error a few u32
for rows of norm <= 1). A truncated or otherwise mis-rounded BF16 link
changes the output by ~2^-9 relative and fails this by orders of magnitude.
"""
import numpy as np

import oracle
from oracle import rounding as R

U32 = 2.0 ** -24


def stored_links(U, prec, recon):
    return R.stored_links(U, prec, recon)


def stored_vec(chi, prec):
    return np.array(chi, dtype=np.float64) if prec == R.PREC_F64 else R.round_f32(chi)


def _cabs(a):
    return np.abs(a[..., 0] + 1j * a[..., 1])


def hop_sums(L, U, chi, out_par, nbr=None):
    """(S, C), each [V/2][3]: S = sum over hops and j of |U_ij| |chi_j| along the
    row of the output, C = sum over hops and j of |chi_j|."""
    if nbr is None:
        _, nbr = oracle.index_maps(L)
    Vh = chi.shape[0]
    p = int(out_par)
    ua = _cabs(U)                 # [4][V][3][3]
    ca = _cabs(chi)               # [Vh][3]
    S = np.zeros((Vh, 3))
    C = np.zeros((Vh, 3))
    own = p * Vh + np.arange(Vh)
    for mu in range(4):
        f, b = nbr[p][mu], nbr[p][4 + mu]
        S += np.einsum("sij,sj->si", ua[mu][own], ca[f])
        S += np.einsum("sji,sj->si", ua[mu][(1 - p) * Vh + b], ca[b])
        C += ca[f].sum(axis=1, keepdims=True) + ca[b].sum(axis=1, keepdims=True)
    return S, C


def check_dslash(got, L, U, chi, out_par, prec, recon, bc=None, nbr=None, what=""):
    """Assert the GPU's reduced-precision Dslash output `got` ([V/2][3][2]) meets
    the per-element bound against the oracle on the stored links and input.
    Returns the largest |got - ref| / bound (<= 1)."""
    Us = stored_links(U, prec, recon)
    cs = stored_vec(chi, prec)
    ref = oracle.dslash(L, Us, cs, out_par, bc)
    S, C = hop_sums(L, Us, cs, out_par, nbr)
    bound = U32 * (64.0 * S + 8.0 * C)[..., None]
    d = np.abs(got - ref)
    worst = float((d / bound).max())
    assert worst <= 1.0, (what, "largest |got - ref| / bound", worst, float(d.max()))
    return worst


def _walk(nbr, p, h, idx, steps):
    """cb index after `steps` hops h from cb idx of parity p (parities alternate)."""
    for k in range(steps):
        idx = nbr[(p + k) & 1][h][idx]
    return idx


def hop_sums_improved(L, F, N, chi, out_par, nbr=None):
    """(S, C) of hop_sums over the 16 hops of the improved operator: the fat
    one-link hops from F and the three-link hops from N, whose backward link
    N_mu(x - 3 mu) sits at x - 3 mu (other parity)."""
    if nbr is None:
        _, nbr = oracle.index_maps(L)
    Vh = chi.shape[0]
    p = int(out_par)
    fa, na, ca = _cabs(F), _cabs(N), _cabs(chi)
    S = np.zeros((Vh, 3))
    C = np.zeros((Vh, 3))
    own = np.arange(Vh)
    for mu in range(4):
        for links, steps in ((fa, 1), (na, 3)):
            f = _walk(nbr, p, mu, own, steps)
            b = _walk(nbr, p, 4 + mu, own, steps)
            S += np.einsum("sij,sj->si", links[mu][p * Vh + own], ca[f])
            S += np.einsum("sji,sj->si", links[mu][(1 - p) * Vh + b], ca[b])
            C += ca[f].sum(axis=1, keepdims=True) + ca[b].sum(axis=1, keepdims=True)
    return S, C


def check_dslash_improved(got, L, F, N, chi, out_par, bc=None, nbr=None, what=""):
    """The improved operator with FP32 x 18 fields: every output real within
    u32 (128 S + 8 C) (96 real products per output real) of the oracle's
    improved Dslash on the rounded fields and input."""
    Fs, Ns = R.round_f32(F), R.round_f32(N)
    cs = R.round_f32(chi)
    ref = oracle.dslash_imp(L, Fs, Ns, cs, out_par, bc)
    S, C = hop_sums_improved(L, Fs, Ns, cs, out_par, nbr)
    bound = U32 * (128.0 * S + 8.0 * C)[..., None]
    d = np.abs(got - ref)
    worst = float((d / bound).max())
    assert worst <= 1.0, (what, "largest |got - ref| / bound", worst, float(d.max()))
    return worst
