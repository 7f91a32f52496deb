"""The Dslash with 64- and 128-site workgroups (a tuned choice for small
lattices) against the oracle: every load grouping at a lattice with several
hundred workgroups and a ragged tail, the LDS-staged variant bit for bit
against the 2-hop one it repeats (the staged range now spans fewer x rows),
the normal operator and its dot product (four times as many partial sums),
CG solves in every scheme, and the force."""
import numpy as np
import pytest

import lgt_inputs as li
import lowprec
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1309_0551_amd")

pytestmark = pytest.mark.gpu

FMTS = {"f64r18": (P.LGT_F64, P.LGT_R18), "f64r12": (P.LGT_F64, P.LGT_R12), "f32r18": (P.LGT_F32, P.LGT_R18),
        "f32r12": (P.LGT_F32, P.LGT_R12), "bf16r12": (P.LGT_BF16, P.LGT_R12)}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("bs", [64, 128])
@pytest.mark.parametrize("hops,streaming", [(8, 1), (2, 1), (1, 0), (4, 1), (8, 0)])
def test_dslash_small_workgroups(dev, fmt, bs, hops, streaming):
    """12x16x16x18 (27648 sites per parity: 432 / 216 workgroups of 64 / 128,
    none ragged for 64; 10x8x12x6, 2880 sites: ragged last workgroups)."""
    prec, recon = FMTS[fmt]
    vp = P.LGT_F64 if prec == P.LGT_F64 else P.LGT_F32
    for L, bc in (((12, 16, 16, 18), (1, 1, 1, -1)), ((10, 8, 12, 6), (-1, 1, 1, 1))):
        U = li.links(L, "haar", 351)
        _, nbr = oracle.index_maps(L)
        with P.Lattice(L, bc) as lat:
            Up = lat.pack_links(_t(U, dev), prec, recon)
            lat.set_dslash_variant(prec, recon, hops, streaming)
            lat.set_dslash_workgroup(prec, recon, bs)
            assert lat.dslash_workgroup(prec, recon) == bs
            for par in (0, 1):
                chi = li.vector(L, 352 + par)
                got = lat.unpack_vec(lat.dslash(Up, lat.pack_vec(_t(chi, dev), vp), par), vp).cpu().numpy()
                if prec == P.LGT_F64:
                    ref = oracle.dslash(L, U, chi, par, bc)
                    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (fmt, bs, L, par)
                else:
                    lowprec.check_dslash(got, L, U, chi, par, prec, recon, bc, nbr, (fmt, bs, L, par))


@pytest.mark.parametrize("bs", [64, 128])
@pytest.mark.parametrize("L", [(2, 2, 2, 2), (32, 4, 4, 6), (6, 4, 6, 8), (768, 2, 2, 2)])
def test_lds_variant_bitwise_small_workgroups(dev, bs, L):
    U = li.links(L, "haar", 361)
    with P.Lattice(L, (1, 1, 1, -1)) as lat:
        Up = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        lat.set_dslash_workgroup(P.LGT_F64, P.LGT_R18, bs)
        for par in (0, 1):
            x = lat.pack_vec(_t(li.vector(L, 362 + par), dev))
            out = {}
            for hops in (4, 2):
                lat.set_dslash_variant(P.LGT_F64, P.LGT_R18, hops, 1)
                out[hops] = lat.dslash(Up, x, par).clone()
            assert torch.equal(out[4], out[2]), (bs, L, par)


@pytest.mark.parametrize("bs", [64, 128])
def test_apply_normal_small_workgroups(dev, bs):
    L, bc, mass = (8, 8, 8, 12), (1, 1, 1, -1), 0.2
    U = li.links(L, "expih", 371, c=0.3)
    chi = li.vector(L, 372)
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        lat.set_dslash_workgroup(P.LGT_F64, P.LGT_R18, bs)
        out, pap = lat.apply_normal(Up, lat.pack_vec(_t(chi, dev)), mass)
        got = lat.unpack_vec(out).cpu().numpy()
    ref = oracle.apply_A(L, U, mass, chi, bc)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    assert pap == pytest.approx(float(np.sum(chi * ref)), rel=1e-12)


@pytest.mark.parametrize("scheme,lo", [(P.LGT_CG_FP64, None), (P.LGT_CG_RELIABLE, (P.LGT_F32, P.LGT_R12)),
                                       (P.LGT_CG_REFINE, (P.LGT_BF16, P.LGT_R12))],
                         ids=["fp64", "rel_f32r12", "ir_bf16r12"])
@pytest.mark.parametrize("bs_hi,bs_lo", [(64, 64), (128, 64), (64, 256)])
def test_cg_small_workgroups(dev, scheme, lo, bs_hi, bs_lo):
    """FP64 and inner formats with different workgroup sizes (different
    partial-sum counts for the update's alpha and for the FP64 residual)."""
    L, mass, tol = (8, 8, 8, 8), 0.1, 1e-10
    U = li.links(L, "haar", 381)
    b = li.vector(L, 382)
    with P.Lattice(L) as lat:
        Uh = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        Ul = lat.pack_links(_t(U, dev), *lo) if lo else None
        lat.set_dslash_workgroup(P.LGT_F64, P.LGT_R18, bs_hi)
        if lo:
            lat.set_dslash_workgroup(*lo, bs_lo)
        x, res = lat.cg_solve(Uh, _t(b, dev), mass, tol=tol, scheme=scheme, U_lo=Ul, ru_interval=50,
                              inner_tol=0.1 if scheme == P.LGT_CG_REFINE else 0.0)
    xg = x.cpu().numpy()
    r = b - oracle.apply_A(L, U, mass, xg)
    rr = float(np.linalg.norm(r) / np.linalg.norm(b))
    assert res.status == 0 and rr <= 1.05 * tol, (res, rr)
    assert abs(res.true_rel_resid - rr) <= 1e-3 * tol + 0.05 * rr


@pytest.mark.parametrize("bs", [64, 128])
def test_force_small_workgroups(dev, bs):
    L, bc = (6, 4, 6, 8), (1, 1, 1, -1)
    U = li.links(L, "expih", 391, c=0.5)
    X = li.vector(L, 392)
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        lat.set_dslash_workgroup(P.LGT_F64, P.LGT_R18, bs)
        G = lat.force(Up, _t(X, dev)).cpu().numpy()
    ref = oracle.force(L, U, X, bc)
    assert np.linalg.norm(G - ref) <= 1e-12 * np.linalg.norm(ref)


def test_workgroup_arguments(dev):
    with P.Lattice((4, 4, 4, 4)) as lat:
        for bad in (0, 32, 96, 512):
            with pytest.raises(P.LgtError):
                lat.set_dslash_workgroup(P.LGT_F64, P.LGT_R18, bad)
        with pytest.raises(P.LgtError):
            lat.set_dslash_workgroup(P.LGT_BF16, P.LGT_R18, 64)
        assert lat.dslash_workgroup(P.LGT_F64, P.LGT_R18) == 256
