"""Packed link formats element by element, and the reduced-precision Dslash
against the oracle on the stored numbers.

* lgt_unpack_links after lgt_pack_links returns every stored real bit for bit
  as the oracle's round-to-nearest-even gives it (FP32: numpy's conversion;
  BF16: one rounding step on the float64 bits), on fields planted with BF16
  and FP32 ties, values just above and below a tie (where rounding through
  FP32 first would go the wrong way), signed zeros and magnitudes from 2^-40
  to 2^40; row 2 of the 12-real formats against the rebuilt row.
* FP32 / BF16 Dslash, every kernel variant, on lattices up to 16^4 (128
  workgroups, so the XCD block remap is not the identity): each output real
  within the FP32-arithmetic bound of tests/lowprec.py of the oracle's Dslash
  on the rounded links and input.
* FP64 Dslash in the variants the benchmark tunes to, over every 32^4 site.
"""
import numpy as np
import pytest

import lgt_inputs as li
import lowprec
import oracle
from oracle import rounding as R

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1309_0551_amd")

pytestmark = pytest.mark.gpu

FMTS = {
    "f64r18": (P.LGT_F64, P.LGT_R18),
    "f64r12": (P.LGT_F64, P.LGT_R12),
    "f32r18": (P.LGT_F32, P.LGT_R18),
    "f32r12": (P.LGT_F32, P.LGT_R12),
    "bf16r12": (P.LGT_BF16, P.LGT_R12),
}
LOW = ["f32r18", "f32r12", "bf16r12"]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _special_values(g, n):
    """Values that separate rounding rules: BF16 ties at random BF16 values,
    the same +- 2^-40 relative (below an FP32 ulp), FP32 ties and near-ties,
    signed zeros, and magnitudes 2^-40 .. 2^40."""
    b = g.standard_normal(n).astype(np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    tie16 = (b | np.uint32(0x8000)).view(np.float32).astype(np.float64)
    f = g.standard_normal(n).astype(np.float32)
    tie32 = (f.astype(np.float64) + np.nextafter(f, np.float32(np.inf)).astype(np.float64)) / 2.0
    wide = g.standard_normal(n) * np.exp2(g.integers(-40, 40, n))
    near = 1.0 + 2.0 ** -40
    pool = np.concatenate([tie16, tie16 * near, tie16 / near, tie32, tie32 * near, tie32 / near, wide,
                           np.zeros(8), -np.zeros(8)])
    return g.choice(pool, size=n)


def special_links(L, seed):
    U = li.links(L, "haar", seed)
    g = np.random.default_rng(seed + 7)
    flat = U.reshape(-1)
    pos = g.choice(flat.size, size=flat.size // 4, replace=False)
    flat[pos] = _special_values(g, pos.size)
    return U


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("L", [(2, 2, 2, 2), (6, 4, 6, 8), (16, 16, 16, 16)])
def test_pack_unpack_links_bit_exact(dev, fmt, L):
    prec, recon = FMTS[fmt]
    print("pack/unpack", fmt, L, flush=True)
    U = special_links(L, 301)
    with P.Lattice(L) as lat:
        got = lat.unpack_links(lat.pack_links(_t(U, dev), prec, recon)).cpu().numpy()
    want = R.round_elements(U, prec)
    rows = 3 if recon == 18 else 2
    np.testing.assert_array_equal(_bits(got[..., :rows, :, :]), _bits(want[..., :rows, :, :]))
    if recon == 12:
        # row 2 = conj(row0 x row1) in the field's arithmetic precision
        rebuilt = R.stored_links(U, prec, recon)[..., 2, :, :]
        w = want[..., 0] + 1j * want[..., 1]
        a, b = np.abs(w[..., 0, :]), np.abs(w[..., 1, :])
        scale = np.stack([a[..., (j + 1) % 3] * b[..., (j + 2) % 3] + a[..., (j + 2) % 3] * b[..., (j + 1) % 3]
                          for j in range(3)], axis=-1)
        u = 2.0 ** -53 if prec == P.LGT_F64 else 2.0 ** -24
        assert np.all(np.abs(got[..., 2, :, :] - rebuilt) <= 8 * u * scale[..., None])


def test_pack_bf16_ties_and_near_ties(dev):
    """Hand-made BF16 cases on one link element each: ties go to the even
    neighbour, values within 2^-40 of a tie go to the nearer neighbour."""
    L = (2, 2, 2, 2)
    cases = [(1.0 + 2.0 ** -8, 1.0), (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),
             (1.0 + 2.0 ** -8 + 2.0 ** -40, 1.0 + 2.0 ** -7), (1.0 + 3 * 2.0 ** -8 - 2.0 ** -40, 1.0 + 2.0 ** -7),
             (-(1.0 + 3 * 2.0 ** -8), -(1.0 + 2.0 ** -6)), (2.0 - 2.0 ** -9, 2.0)]
    U = li.links(L, "haar", 311)
    flat = U.reshape(4, 16, 18)
    for i, (x, _) in enumerate(cases):
        flat[0, i, 0] = x                                  # row 0, column 0, real part
    with P.Lattice(L) as lat:
        got = lat.unpack_links(lat.pack_links(_t(U, dev), P.LGT_BF16, P.LGT_R12)).cpu().numpy()
    got = got.reshape(4, 16, 18)
    for i, (_, want) in enumerate(cases):
        assert got[0, i, 0] == want, (i, got[0, i, 0], want)


def test_unpack_links_arguments(dev):
    with P.Lattice((4, 4, 4, 4)) as lat:
        Up = lat.pack_links(_t(li.links((4, 4, 4, 4), "haar", 1), dev), P.LGT_F32, P.LGT_R12)
        bad = P.PackedLinks(Up.data, P.LGT_BF16, P.LGT_R18)
        with pytest.raises(P.LgtError):
            lat.unpack_links(bad)


# ---------------------------------------------------- reduced-precision Dslash ---

@pytest.mark.parametrize("fmt", LOW)
@pytest.mark.parametrize("L,bc,kind", [
    ((2, 2, 2, 2), (1, 1, 1, 1), "haar"),
    ((6, 4, 6, 8), (1, 1, 1, -1), "haar"),
    ((8, 8, 8, 12), (-1, 1, 1, -1), "expih"),
    ((16, 16, 16, 16), (1, 1, 1, 1), "expih"),
])
def test_dslash_lowprec_per_element(dev, fmt, L, bc, kind):
    prec, recon = FMTS[fmt]
    U = li.links(L, kind, 321, c=0.3)
    _, nbr = oracle.index_maps(L)
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), prec, recon)
        for par in (0, 1):
            chi = li.vector(L, 322 + par)
            got = lat.unpack_vec(lat.dslash(Up, lat.pack_vec(_t(chi, dev), P.LGT_F32), par), P.LGT_F32)
            w = lowprec.check_dslash(got.cpu().numpy(), L, U, chi, par, prec, recon, bc, nbr, (fmt, L, par))
            print(f"  {fmt} {L} parity {par}: largest error / bound {w:.3f}", flush=True)


VARIANTS = [(8, 1), (2, 1), (1, 1), (4, 1), (8, 0), (2, 0), (1, 0), (4, 0)]


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("hops,streaming", VARIANTS)
def test_every_variant_many_workgroups(dev, fmt, hops, streaming):
    """12x16x16x18, antiperiodic t: 27648 sites per parity, 108 workgroups
    (112 launched), so the XCD remap of workgroups is not the identity and the
    last workgroup is ragged. FP64: per component <= 1e-12 max|ref|; FP32 and
    BF16: the per-element bound on the stored numbers."""
    prec, recon = FMTS[fmt]
    L, bc = (12, 16, 16, 18), (1, 1, 1, -1)
    U = li.links(L, "haar", 331)
    vp = P.LGT_F64 if prec == P.LGT_F64 else P.LGT_F32
    _, nbr = oracle.index_maps(L)
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), prec, recon)
        lat.set_dslash_variant(prec, recon, hops, streaming)
        for par in (0, 1):
            chi = li.vector(L, 332 + par)
            got = lat.unpack_vec(lat.dslash(Up, lat.pack_vec(_t(chi, dev), vp), par), vp).cpu().numpy()
            if prec == P.LGT_F64:
                ref = oracle.dslash(L, U, chi, par, bc)
                assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
            else:
                lowprec.check_dslash(got, L, U, chi, par, prec, recon, bc, nbr, (fmt, hops, streaming, par))


@pytest.mark.parametrize("hops,streaming", [(8, 1), (4, 1), (2, 1), (8, 0)])
def test_dslash_32_tuned_variants(dev, hops, streaming):
    """The 32^4 Haar field of the benchmark, FP64, in the variants its tuner
    chooses between: every output site of both parities per component."""
    L = (32, 32, 32, 32)
    print("dslash 32^4 variant", hops, streaming, flush=True)
    U = li.links(L, "haar", 3001)
    with P.Lattice(L) as lat:
        Up = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        lat.set_dslash_variant(P.LGT_F64, P.LGT_R18, hops, streaming)
        for par in (0, 1):
            chi = li.vector(L, 3002 + par)
            out = lat.unpack_vec(lat.dslash(Up, lat.pack_vec(_t(chi, dev)), par)).cpu().numpy()
            ref = oracle.dslash(L, U, chi, par)
            assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)
            assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("fmt", LOW)
def test_dslash_32_lowprec_per_element(dev, fmt):
    """32^4 Haar, FP32 / BF16 in the default (size-dependent) variant: every
    output real within the per-element bound on the stored numbers."""
    prec, recon = FMTS[fmt]
    L = (32, 32, 32, 32)
    print("dslash 32^4", fmt, flush=True)
    U = li.links(L, "haar", 3001)
    chi = li.vector(L, 3002)
    with P.Lattice(L) as lat:
        Up = lat.pack_links(_t(U, dev), prec, recon)
        got = lat.unpack_vec(lat.dslash(Up, lat.pack_vec(_t(chi, dev), P.LGT_F32), 1), P.LGT_F32).cpu().numpy()
    w = lowprec.check_dslash(got, L, U, chi, 1, prec, recon, None, None, fmt)
    print(f"  largest error / bound {w:.3f}", flush=True)
