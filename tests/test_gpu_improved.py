"""Improved (fat one-link + Naik three-link) staggered operator on the GPU
against the FP64 oracle: Dslash element by element, the CG in every scheme,
and the argument checks of its entry points."""
import numpy as np
import pytest

import lgt_inputs as li
import lowprec
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1309_0551_amd")

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
FMTS = {"f64r18": (P.LGT_F64, 1e-12), "f32r18": (P.LGT_F32, 32 * U32)}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("L,bc", [((2, 4, 2, 6), (1, 1, 1, -1)),    # extents 2, 4, 6: hops coincide
                                  ((4, 2, 6, 4), (-1, 1, -1, 1)),
                                  ((8, 4, 6, 8), (1, 1, 1, -1)),
                                  ((10, 8, 12, 6), (1, -1, 1, -1)),  # several workgroups, ragged tail
                                  ((16, 16, 16, 32), (1, 1, 1, 1))])
def test_improved_dslash_parity(dev, fmt, L, bc):
    prec, tol = FMTS[fmt]
    F, N = li.improved_links(L, 401)
    vp = prec
    with P.Lattice(L, bc) as lat:
        Fp = lat.pack_links(_t(F, dev), prec, P.LGT_R18)
        Np = lat.pack_links(_t(N, dev), prec, P.LGT_R18)
        for par in (0, 1):
            chi = li.vector(L, 402 + par)
            x = lat.pack_vec(_t(chi, dev), vp)
            got = lat.unpack_vec(lat.dslash_improved(Fp, Np, x, par), vp).cpu().numpy()
            ref = oracle.dslash_imp(L, F, N, chi, par, bc)
            assert _rel(got, ref) <= tol, (fmt, L, par)
            if prec == P.LGT_F64:
                assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
            else:
                lowprec.check_dslash_improved(got, L, F, N, chi, par, bc, None, (fmt, L, par))


def test_improved_dslash_full_size_32(dev):
    """32^4, the benchmark's lattice and launch configuration: every output site."""
    L = li.CONFIGS["imp_32x32x32x32"]["L"]
    F, N = li.improved_links(L, li.CONFIGS["imp_32x32x32x32"]["link_seed"])
    chi = li.vector(L, 411)
    with P.Lattice(L) as lat:
        Fp = lat.pack_links(_t(F, dev), P.LGT_F64, P.LGT_R18)
        Np = lat.pack_links(_t(N, dev), P.LGT_F64, P.LGT_R18)
        x = lat.pack_vec(_t(chi, dev))
        got = lat.unpack_vec(lat.dslash_improved(Fp, Np, x, 1)).cpu().numpy()
    ref = oracle.dslash_imp(L, F, N, chi, 1)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


CG_CASES = [("fp64", P.LGT_CG_FP64), ("reliable_f32r18", P.LGT_CG_RELIABLE), ("refine_f32r18", P.LGT_CG_REFINE)]


@pytest.mark.parametrize("name,scheme", CG_CASES, ids=[c[0] for c in CG_CASES])
def test_improved_cg_parity(dev, name, scheme):
    L, mass, tol = (8, 8, 8, 8), 0.1, 1e-10
    F, N = li.improved_links(L, 421)
    b = li.vector(L, 422)
    st, xo, it_o, rr_o = oracle.cg_imp(L, F, N, mass, b, tol=tol)
    assert st == 0
    with P.Lattice(L) as lat:
        Ft, Nt = _t(F, dev), _t(N, dev)
        Fh, Nh = lat.pack_links(Ft, P.LGT_F64, P.LGT_R18), lat.pack_links(Nt, P.LGT_F64, P.LGT_R18)
        lo = {}
        if scheme != P.LGT_CG_FP64:
            lo = dict(F_lo=lat.pack_links(Ft, P.LGT_F32, P.LGT_R18), N_lo=lat.pack_links(Nt, P.LGT_F32, P.LGT_R18))
        x, res = lat.cg_solve_improved(Fh, Nh, _t(b, dev), mass, tol=tol, scheme=scheme,
                                       inner_tol=0.1 if scheme == P.LGT_CG_REFINE else 0.0, **lo)
    xg = x.cpu().numpy()
    rr = float(np.linalg.norm(b - oracle.apply_A_imp(L, F, N, mass, xg)) / np.linalg.norm(b))
    print(f"\nimproved {name}: iters {res.iters} (oracle {it_o}) updates {res.updates} resid {rr:.3e}", flush=True)
    assert res.status == 0
    assert rr <= 1.05 * tol
    assert abs(res.true_rel_resid - rr) <= 1e-3 * tol + 0.05 * rr
    assert np.linalg.norm(xg - xo) <= (1.05 * tol + rr_o) * np.linalg.norm(b) / (4 * mass * mass)
    if scheme == P.LGT_CG_FP64:
        assert abs(res.iters - it_o) <= 3


def test_improved_argument_checks(dev):
    L = (4, 4, 4, 4)
    F, N = li.improved_links(L, 431)
    with P.Lattice(L) as lat:
        Ft, Nt = _t(F, dev), _t(N, dev)
        F64, N64 = lat.pack_links(Ft, P.LGT_F64, P.LGT_R18), lat.pack_links(Nt, P.LGT_F64, P.LGT_R18)
        N32 = lat.pack_links(Nt, P.LGT_F32, P.LGT_R18)
        F12 = lat.pack_links(Ft, P.LGT_F32, P.LGT_R12)
        x = lat.pack_vec(_t(li.vector(L, 432), dev))
        with pytest.raises(P.LgtError):          # fat and Naik in different formats
            lat.dslash_improved(F64, N32, x, 0)
        with pytest.raises(P.LgtError):          # 12-real fields cannot hold general matrices
            lat.dslash_improved(F12, lat.pack_links(Nt, P.LGT_F32, P.LGT_R12),
                                lat.pack_vec(_t(li.vector(L, 433), dev), P.LGT_F32), 0)
        with pytest.raises(P.LgtError):          # mixed scheme without F32 x 18 inner fields
            lat.cg_solve_improved(F64, N64, _t(li.vector(L, 434), dev), 0.1, scheme=P.LGT_CG_RELIABLE)


@pytest.mark.parametrize("fmt", sorted(FMTS))
def test_improved_dslash_antihermitian(dev, fmt):
    """<phi_e, D_eo psi_o> = -<D_oe phi_e, psi_o> for the GPU improved operator
    (antiperiodic t, Naik hops crossing the boundary)."""
    prec, tol = FMTS[fmt]
    L, bc = (8, 4, 6, 8), (1, 1, 1, -1)
    F, N = li.improved_links(L, 441)
    phi, psi = li.vector(L, 442), li.vector(L, 443)
    with P.Lattice(L, bc) as lat:
        Fp = lat.pack_links(_t(F, dev), prec, P.LGT_R18)
        Np = lat.pack_links(_t(N, dev), prec, P.LGT_R18)
        Dpsi = li.to_complex(lat.unpack_vec(lat.dslash_improved(Fp, Np, lat.pack_vec(_t(psi, dev), prec), 0),
                                            prec).cpu().numpy())
        Dphi = li.to_complex(lat.unpack_vec(lat.dslash_improved(Fp, Np, lat.pack_vec(_t(phi, dev), prec), 1),
                                            prec).cpu().numpy())
    lhs = np.vdot(li.to_complex(phi), Dpsi)
    rhs = -np.vdot(Dphi, li.to_complex(psi))
    assert abs(lhs - rhs) <= 4 * tol * np.linalg.norm(Dpsi) * np.linalg.norm(phi)


@pytest.mark.parametrize("L,bc", [((8, 4, 6, 8), (1, 1, 1, -1)), ((10, 8, 12, 6), (-1, 1, 1, 1))])
def test_improved_force_vs_oracle(dev, L, bc):
    """dS/dF and dS/dN on the GPU against the oracle given the same X."""
    F, N = li.improved_links(L, 451)
    X = li.vector(L, 452)
    GFo, GNo = oracle.force_imp(L, F, N, X, bc)
    with P.Lattice(L, bc) as lat:
        Fp = lat.pack_links(_t(F, dev), P.LGT_F64, P.LGT_R18)
        Np = lat.pack_links(_t(N, dev), P.LGT_F64, P.LGT_R18)
        GF, GN = lat.force_improved(Fp, Np, _t(X, dev), scale=0.5)
        GF, GN = GF.cpu().numpy(), GN.cpu().numpy()
        with pytest.raises(P.LgtError):  # 32-bit fields are not accepted for the force
            lat.force_improved(lat.pack_links(_t(F, dev), P.LGT_F32, P.LGT_R18),
                               lat.pack_links(_t(N, dev), P.LGT_F32, P.LGT_R18), _t(X, dev))
    assert np.abs(GF - 0.5 * GFo).max() <= 1e-12 * np.abs(GFo).max()
    assert np.abs(GN - 0.5 * GNo).max() <= 1e-12 * np.abs(GNo).max()


def test_improved_force_central_differences_gpu(dev):
    """The GPU improved force from the GPU improved CG's X against central
    differences of the GPU action S = Re <phi, A^-1 phi> (variational
    estimator), along random directions in F and in N."""
    L, mass, h = (8, 4, 4, 8), 0.1, 1e-5
    F, N = li.improved_links(L, 461)
    phi = li.vector(L, 462)
    rng = np.random.default_rng(463)
    with P.Lattice(L) as lat:
        ph = _t(phi, dev)

        def solve(Fx, Nx):
            Fp = lat.pack_links(_t(Fx, dev), P.LGT_F64, P.LGT_R18)
            Np = lat.pack_links(_t(Nx, dev), P.LGT_F64, P.LGT_R18)
            x, _ = lat.cg_solve_improved(Fp, Np, ph, mass, tol=1e-13)
            return Fp, Np, x

        def S(Fx, Nx):
            Fp, Np, x = solve(Fx, Nx)
            xa = x.cpu().numpy()
            Ax = oracle.apply_A_imp(L, Fx, Nx, mass, xa)
            return 2.0 * float(np.sum(phi * xa)) - float(np.sum(xa * Ax))

        Fp, Np, X = solve(F, N)
        GF, GN = (g.cpu().numpy() for g in lat.force_improved(Fp, Np, X))
        for which in ("F", "N"):
            E = rng.standard_normal(F.shape)
            if which == "F":
                fd = (S(F + h * E, N) - S(F - h * E, N)) / (2 * h)
                an = float(np.sum(GF * E))
            else:
                fd = (S(F, N + h * E) - S(F, N - h * E)) / (2 * h)
                an = float(np.sum(GN * E))
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, fd, an)


def test_improved_autograd_action(dev):
    """ImprovedPseudofermionAction: S and dS/dF, dS/dN, dS/dphi against the
    oracle's solve and force."""
    L, mass = (8, 4, 6, 4), 0.1
    F, N = li.improved_links(L, 491)
    phi = li.vector(L, 492)
    st, Xo, _, _ = oracle.cg_imp(L, F, N, mass, phi, tol=1e-13)
    GFo, GNo = oracle.force_imp(L, F, N, Xo)
    with P.Lattice(L) as lat:
        Ft, Nt, pt = (_t(a, dev).requires_grad_(True) for a in (F, N, phi))
        S = P.ImprovedPseudofermionAction.apply(Ft, Nt, pt, lat, mass, 1e-13)
        (1.5 * S).backward()
    assert abs(S.item() - float(np.sum(phi * Xo))) <= 1e-10 * abs(S.item())
    assert _rel(Ft.grad.cpu().numpy(), 1.5 * GFo) <= 1e-8
    assert _rel(Nt.grad.cpu().numpy(), 1.5 * GNo) <= 1e-8
    assert _rel(pt.grad.cpu().numpy(), 1.5 * 2 * Xo) <= 1e-8


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("streaming,bs", [(1, 256), (0, 256), (1, 128), (0, 128), (1, 64), (0, 64)])
def test_improved_variants(dev, fmt, streaming, bs):
    """Every improved-operator variant (link loads x workgroup size) against the
    oracle at 12x16x16x18 (several hundred workgroups) and 10x8x12x6 (ragged),
    and the one-link choice for the same format left as it was."""
    prec, _ = FMTS[fmt]
    for L, bc in (((12, 16, 16, 18), (1, 1, 1, -1)), ((10, 8, 12, 6), (-1, 1, 1, 1))):
        F, N = li.improved_links(L, 431)
        with P.Lattice(L, bc) as lat:
            one_link = (lat.dslash_variant(prec, P.LGT_R18), lat.dslash_workgroup(prec, P.LGT_R18))
            lat.set_dslash_improved_variant(prec, streaming, bs)
            assert lat.dslash_improved_variant(prec) == (streaming, bs)
            assert (lat.dslash_variant(prec, P.LGT_R18), lat.dslash_workgroup(prec, P.LGT_R18)) == one_link
            Fp = lat.pack_links(_t(F, dev), prec, P.LGT_R18)
            Np = lat.pack_links(_t(N, dev), prec, P.LGT_R18)
            for par in (0, 1):
                chi = li.vector(L, 432 + par)
                got = lat.unpack_vec(lat.dslash_improved(Fp, Np, lat.pack_vec(_t(chi, dev), prec), par),
                                     prec).cpu().numpy()
                ref = oracle.dslash_imp(L, F, N, chi, par, bc)
                if prec == P.LGT_F64:
                    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (fmt, L, par)
                else:
                    lowprec.check_dslash_improved(got, L, F, N, chi, par, bc, None, (fmt, L, par))


def test_improved_tuner_and_small_workgroup_solve(dev):
    """lgt_tune_dslash_improved keeps one of the variants it timed; a mixed CG
    and the force with 64-site workgroups match the oracle."""
    L, mass, tol = (8, 8, 8, 8), 0.1, 1e-10
    F, N = li.improved_links(L, 441)
    b = li.vector(L, 442)
    with P.Lattice(L) as lat:
        Ft, Nt = _t(F, dev), _t(N, dev)
        Fh, Nh = lat.pack_links(Ft, P.LGT_F64, P.LGT_R18), lat.pack_links(Nt, P.LGT_F64, P.LGT_R18)
        Fl, Nl = lat.pack_links(Ft, P.LGT_F32, P.LGT_R18), lat.pack_links(Nt, P.LGT_F32, P.LGT_R18)
        t = lat.tune_dslash_improved(Fh, Nh)
        assert (1, 256) in t and (0, 64) in t  # 8^4: 8 workgroups of 256, so all six are timed
        assert lat.dslash_improved_variant(P.LGT_F64) in t
        for prec in (P.LGT_F64, P.LGT_F32):
            lat.set_dslash_improved_variant(prec, 0, 64)
        x, res = lat.cg_solve_improved(Fh, Nh, _t(b, dev), mass, tol=tol, scheme=P.LGT_CG_RELIABLE, F_lo=Fl, N_lo=Nl)
        xg = x.cpu().numpy()
        GF, GN = lat.force_improved(Fh, Nh, x)
        GFo, GNo = oracle.force_imp(L, F, N, xg)
    rr = float(np.linalg.norm(b - oracle.apply_A_imp(L, F, N, mass, xg)) / np.linalg.norm(b))
    assert res.status == 0 and rr <= 1.05 * tol
    for g, o in ((GF.cpu().numpy(), GFo), (GN.cpu().numpy(), GNo)):
        assert np.abs(g - o).max() <= 1e-12 * np.abs(o).max()
