"""GPU parity against the FP64 oracle, through the C ABI (Python binding).

Tolerances (norm-wise relative error of the output):
* index maps: bit-exact.
* FP64 Dslash (18 and 12 reals): <= 1e-12 and per component <= 1e-12 max|out|.
* FP32 links + FP32 vectors: 32 u32 = 1.9e-6, u32 = 2^-24 the storage rounding of
  links and input; the kernel sums 8 hops of 3x3 products in FP32.
* BF16 links + FP32 vectors: 8 u16 = 1.6e-2, u16 = 2^-9; rows 0-1 are rounded
  and row 2 is rebuilt from the rounded rows.
* FP32 / BF16 also element by element: every component within tol max|ref|,
  and every output real within the FP32-arithmetic bound of tests/lowprec.py
  against the oracle on the stored (rounded) links and input, which a
  mis-rounded BF16 link fails by orders of magnitude.
* CG: the oracle recomputes the true residual of the GPU's x in FP64, which must
  meet the tolerance; and |x - x_oracle| <= (tol_gpu + tol_oracle) |b| / (4 m^2),
  since lambda_min(A) >= 4 m^2.
"""
import math

import numpy as np
import pytest

import brute
import lgt_inputs as li
import lowprec
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1309_0551_amd")

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U16 = 2.0 ** -9
FMTS = {
    "f64r18": (P.LGT_F64, P.LGT_R18, 1e-12),
    "f64r12": (P.LGT_F64, P.LGT_R12, 1e-12),
    "f32r18": (P.LGT_F32, P.LGT_R18, 32 * U32),
    "f32r12": (P.LGT_F32, P.LGT_R12, 32 * U32),
    "bf16r12": (P.LGT_BF16, P.LGT_R12, 8 * U16),
}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ------------------------------------------------------------- geometry ---

@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 6, 8), (8, 6, 4, 2), (16, 16, 16, 32),
                               (24, 24, 24, 48), (32, 32, 32, 32)])
def test_index_maps_bit_exact(dev, L):
    print("index maps", L, flush=True)
    with P.Lattice(L) as lat:
        lex, nbr = lat.index_maps()
        torch.cuda.synchronize()
        e_lex, e_nbr = oracle.index_maps(L)
        np.testing.assert_array_equal(lex.cpu().numpy(), e_lex)
        np.testing.assert_array_equal(nbr.cpu().numpy(), e_nbr)


# --------------------------------------------------------------- Dslash ---

@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("L,bc,kind", [
    ((2, 2, 2, 2), (1, 1, 1, 1), "haar"),       # coincident +mu / -mu neighbours
    ((4, 4, 4, 4), (1, 1, 1, 1), "haar"),       # 128 sites: one partial workgroup
    ((6, 4, 6, 8), (1, 1, 1, -1), "haar"),      # 576 sites: 3 workgroups, ragged tail
    ((8, 8, 8, 12), (-1, 1, 1, -1), "expih"),
    ((16, 16, 16, 16), (1, 1, 1, 1), "expih"),  # 32768 sites: 128 workgroups
])
def test_dslash_parity(dev, fmt, L, bc, kind):
    prec, recon, tol = FMTS[fmt]
    print("dslash", fmt, L, bc, flush=True)
    U = li.links(L, kind, 101, c=0.3)
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), prec, recon)
        for out_par in (0, 1):
            chi = li.vector(L, 102 + out_par)
            vp = P.LGT_F64 if prec == P.LGT_F64 else P.LGT_F32
            out = lat.unpack_vec(lat.dslash(Up, lat.pack_vec(_t(chi, dev), vp), out_par), vp)
            got = out.cpu().numpy()
            ref = oracle.dslash(L, U, chi, out_par, bc)
            assert _rel(got, ref) <= tol, (fmt, out_par, _rel(got, ref))
            assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
            if prec != P.LGT_F64:
                lowprec.check_dslash(got, L, U, chi, out_par, prec, recon, bc, None, (fmt, L, out_par))


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("hops,streaming", [(1, 1), (2, 1), (8, 1), (4, 1), (1, 0), (2, 0), (8, 0), (4, 0)])
def test_dslash_every_variant(dev, fmt, hops, streaming):
    """Each kernel variant (loads of 1, 2 or 8 hops issued together, or 2 with
    the input staged in LDS; streaming or cached link loads) gives the same
    operator."""
    prec, recon, tol = FMTS[fmt]
    L, bc = (6, 4, 6, 8), (1, 1, 1, -1)
    U = li.links(L, "haar", 121)
    chi = li.vector(L, 122)
    vp = P.LGT_F64 if prec == P.LGT_F64 else P.LGT_F32
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), prec, recon)
        lat.set_dslash_variant(prec, recon, hops, streaming)
        assert lat.dslash_variant(prec, recon) == (hops, streaming)
        x = lat.pack_vec(_t(chi, dev), vp)
        got = lat.unpack_vec(lat.dslash(Up, x, 0), vp).cpu().numpy()
        lat.set_dslash_variant(prec, recon, 8, 1)
        ref8 = lat.unpack_vec(lat.dslash(Up, x, 0), vp).cpu().numpy()
    ref = oracle.dslash(L, U, chi, 0, bc)
    assert _rel(got, ref) <= tol
    if prec == P.LGT_F64:
        assert _rel(got, ref8) <= 1e-15


@pytest.mark.parametrize("fmt", ["f64r18", "f32r12"])
@pytest.mark.parametrize("L,bc", [((2, 2, 2, 2), (1, 1, 1, 1)),        # every neighbour inside the staged range
                                  ((4, 6, 2, 4), (1, -1, 1, -1)),
                                  ((32, 4, 4, 6), (1, 1, 1, -1)),      # 8 rows per workgroup, ragged tail
                                  ((768, 2, 2, 2), (-1, 1, 1, 1)),     # staged range at its 1024-site limit
                                  ((776, 2, 2, 2), (1, 1, 1, -1))])    # beyond it: runs the 2-hop kernel
def test_dslash_lds_variant_bitwise(dev, fmt, L, bc):
    """The LDS-staged variant does the 2-hop variant's arithmetic in the same
    order: bit-identical output, and the oracle's within the format's bound."""
    prec, recon, tol = FMTS[fmt]
    U = li.links(L, "haar", 141)
    vp = P.LGT_F64 if prec == P.LGT_F64 else P.LGT_F32
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), prec, recon)
        for par in (0, 1):
            chi = li.vector(L, 142 + par)
            x = lat.pack_vec(_t(chi, dev), vp)
            out = {}
            for hops in (4, 2):
                lat.set_dslash_variant(prec, recon, hops, 1)
                out[hops] = lat.unpack_vec(lat.dslash(Up, x, par), vp).cpu().numpy()
            np.testing.assert_array_equal(out[4], out[2])
            assert _rel(out[4], oracle.dslash(L, U, chi, par, bc)) <= tol


def _gpu_dslash(lat, Up, vp, chi, par, dev):
    return lat.unpack_vec(lat.dslash(Up, lat.pack_vec(_t(chi, dev), vp), par), vp).cpu().numpy()


@pytest.mark.parametrize("fmt", ["f64r18", "f64r12", "f32r12"])
@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (-1, 1, 1, -1)])
def test_gpu_dslash_antihermitian(dev, fmt, bc):
    """<phi_e, D_eo psi_o> = -<D_oe phi_e, psi_o> on the GPU operator itself."""
    prec, recon, tol = FMTS[fmt]
    L = (6, 4, 8, 4)
    U = li.links(L, "haar", 161)
    phi, psi = li.vector(L, 162), li.vector(L, 163)
    vp = P.LGT_F64 if prec == P.LGT_F64 else P.LGT_F32
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), prec, recon)
        Dpsi = li.to_complex(_gpu_dslash(lat, Up, vp, psi, 0, dev))
        Dphi = li.to_complex(_gpu_dslash(lat, Up, vp, phi, 1, dev))
    lhs = np.vdot(li.to_complex(phi), Dpsi)
    rhs = -np.vdot(Dphi, li.to_complex(psi))
    assert abs(lhs - rhs) <= 4 * tol * np.linalg.norm(Dpsi) * np.linalg.norm(phi)


@pytest.mark.parametrize("fmt", ["f64r18", "f64r12", "f32r12"])
def test_gpu_dslash_gauge_covariance(dev, fmt):
    """D[U^g] (g chi) = g (D[U] chi) for a random SU(3) gauge transform g, on
    the GPU operator (12-real fields hold the transformed links exactly too)."""
    prec, recon, tol = FMTS[fmt]
    L, bc = (4, 6, 4, 6), (1, 1, 1, -1)
    V = int(np.prod(L))
    Vh = V // 2
    U = li.links(L, "haar", 171)
    G = li.haar_su3(V, li.rng(173))
    Uc = li.to_complex(U)
    UG = np.empty_like(Uc)
    for lex, c in brute.sites(L):
        e = brute.eo_index(L, c)
        for mu in range(4):
            f = brute.eo_index(L, brute.shift(L, c, mu, +1))
            UG[mu, e] = G[e] @ Uc[mu, e] @ G[f].conj().T
    vp = P.LGT_F64 if prec == P.LGT_F64 else P.LGT_F32
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), prec, recon)
        UGp = lat.pack_links(_t(li.to_real(UG), dev), prec, recon)
        for par in (0, 1):
            chi = li.vector(L, 172 + par)
            Gin, Gout = G[(1 - par) * Vh:(2 - par) * Vh], G[par * Vh:(par + 1) * Vh]
            lhs = li.to_complex(_gpu_dslash(lat, UGp, vp, li.to_real(np.einsum("nij,nj->ni", Gin,
                                                                               li.to_complex(chi))), par, dev))
            rhs = np.einsum("nij,nj->ni", Gout, li.to_complex(_gpu_dslash(lat, Up, vp, chi, par, dev)))
            assert np.linalg.norm(lhs - rhs) <= 4 * tol * np.linalg.norm(rhs), (fmt, par)


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("L,bc", [((4, 4, 4, 4), (1, 1, 1, 1)), ((6, 4, 6, 8), (1, 1, 1, -1)),
                                  ((10, 8, 12, 6), (-1, 1, 1, -1))])
def test_apply_normal_parity(dev, fmt, L, bc):
    """A = 4m^2 - D_eo D_oe applied once, and Re <x, A x>, against the oracle
    (two Dslash applications: twice the single-Dslash bound)."""
    prec, recon, tol = FMTS[fmt]
    mass = 0.07
    U = li.links(L, "haar", 151)
    chi = li.vector(L, 152)
    vp = P.LGT_F64 if prec == P.LGT_F64 else P.LGT_F32
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), prec, recon)
        x = lat.pack_vec(_t(chi, dev), vp)
        out, pap = lat.apply_normal(Up, x, mass)
        got = lat.unpack_vec(out, vp).cpu().numpy()
        with pytest.raises(P.LgtError):
            lat.apply_normal(Up, x, mass, out=x)       # in and out alias
        with pytest.raises(P.LgtError):
            lat.apply_normal(Up, x, -1.0)
    ref = oracle.apply_A(L, U, mass, chi, bc)
    assert _rel(got, ref) <= 2 * tol
    ref_pap = float(np.sum(chi * ref))  # Re <chi, A chi> over the real layout
    assert ref_pap > 4 * mass * mass * float(np.sum(chi * chi))
    assert pap == pytest.approx(ref_pap, rel=2 * tol)


def test_tune_dslash_picks_a_variant(dev, tmp_path, monkeypatch):
    L = (8, 8, 8, 8)
    U = li.links(L, "haar", 131)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LGT_TUNE_CACHE", str(cache))
    with P.Lattice(L) as lat:
        Up = lat.pack_links(_t(U, dev), P.LGT_F32, P.LGT_R12)
        t = lat.tune_dslash(Up)
        # 8^4: 8 workgroups of 256 sites, so the 128- and 64-site ones are timed too
        assert set(t) == set(P.Lattice.TUNE_VARIANTS) and all(v > 0 for v in t.values())
        # the first variant in list order within 1 % of the fastest
        fastest = min(t.values())
        best = next(v for v in P.Lattice.TUNE_VARIANTS if t[v] <= 1.01 * fastest)
        assert lat.dslash_variant(P.LGT_F32, P.LGT_R12) + (lat.dslash_workgroup(P.LGT_F32, P.LGT_R12),) == best
    assert "f32r12" in cache.read_text()
    with P.Lattice(L) as lat2:
        other = (8, 1) if best[:2] != (8, 1) else (1, 0)
        lat2.set_dslash_variant(P.LGT_F32, P.LGT_R12, *other)
        lat2.set_dslash_workgroup(P.LGT_F32, P.LGT_R12, 128 if best[2] != 128 else 64)
        lat2.tune_dslash(Up, report=False)  # cached: no timing
        assert lat2.dslash_variant(P.LGT_F32, P.LGT_R12) + (lat2.dslash_workgroup(P.LGT_F32, P.LGT_R12),) == best


def test_tune_dslash_large_lattice_keeps_256(dev):
    """At 32^4 (2048 workgroups of 256 sites) only 256-site workgroups are timed."""
    L = (32, 32, 32, 32)
    with P.Lattice(L) as lat:
        U = torch.zeros((4, lat.V, 3, 3, 2), dtype=torch.float64, device=dev)
        U[..., 0, 0, 0] = U[..., 1, 1, 0] = U[..., 2, 2, 0] = 1.0
        Up = lat.pack_links(U, P.LGT_BF16, P.LGT_R12)
        del U
        t = lat.tune_dslash(Up)
        assert set(t) == {v for v in P.Lattice.TUNE_VARIANTS if v[2] == 256}
        assert lat.dslash_workgroup(P.LGT_BF16, P.LGT_R12) == 256


@pytest.mark.parametrize("L,f32r18,f32r12,bf16r12,f64", [((32, 32, 32, 32), 0, 0, 0, (2, 1)),
                                                           ((40, 40, 40, 40), 1, 1, 0, (2, 1)),
                                                           ((48, 48, 48, 48), 1, 1, 1, (2, 1)),
                                                           ((24, 24, 24, 48), 0, 0, 0, (2, 1)),
                                                           ((16, 16, 16, 16), 0, 0, 0, (8, 0)),
                                                           ((16, 16, 16, 32), 0, 0, 0, (8, 0))])
def test_default_link_loads_follow_field_size(dev, L, f32r18, f32r12, bf16r12, f64):
    """FP32/BF16 link loads default to cached while the field (mostly) fits
    in the 256 MB Infinity Cache -- up to 384 MB -- and to streaming beyond;
    FP64 x 18 fields up to 128 MB take 8 hops with cached loads, larger ones
    2 hops streaming; every format starts with 256-site workgroups."""
    with P.Lattice(L) as lat:
        assert lat.dslash_variant(P.LGT_F32, P.LGT_R18)[1] == f32r18
        assert lat.dslash_variant(P.LGT_F32, P.LGT_R12)[1] == f32r12
        assert lat.dslash_variant(P.LGT_BF16, P.LGT_R12)[1] == bf16r12
        assert lat.dslash_variant(P.LGT_F64, P.LGT_R18) == f64
        assert lat.dslash_workgroup(P.LGT_F64, P.LGT_R18) == 256


def test_dslash_full_size_32(dev):
    """32^4 Haar, FP64, the benchmark's launch configuration: every output site."""
    L = (32, 32, 32, 32)
    print("dslash 32^4", flush=True)
    U = li.links(L, "haar", 3001)
    chi = li.vector(L, 3002)
    with P.Lattice(L) as lat:
        Up = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        out = lat.unpack_vec(lat.dslash(Up, lat.pack_vec(_t(chi, dev)), 1)).cpu().numpy()
    ref = oracle.dslash(L, U, chi, 1)
    assert _rel(out, ref) <= 1e-12
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_dslash_run_twice_bit_identical(dev):
    L = (8, 8, 8, 8)
    U = li.links(L, "haar", 111)
    chi = li.vector(L, 112)
    with P.Lattice(L) as lat:
        Up = lat.pack_links(_t(U, dev))
        x = lat.pack_vec(_t(chi, dev))
        a = lat.dslash(Up, x, 0).clone()
        b = lat.dslash(Up, x, 0).clone()
        assert torch.equal(a, b)


def test_dslash_on_a_side_stream(dev):
    """A context on a non-default stream (default priority) orders its work on
    that stream: results read there without a device-wide sync are the
    default-stream results bit for bit."""
    L = (8, 8, 8, 12)
    U = li.links(L, "haar", 121)
    chi = li.vector(L, 122)
    with P.Lattice(L) as lat:
        ref = lat.dslash(lat.pack_links(_t(U, dev)), lat.pack_vec(_t(chi, dev)), 1).clone()
        b = li.vector(L, 123)
        xr, _ = lat.cg_solve(lat.pack_links(_t(U, dev)), _t(b, dev), 0.1)
    torch.cuda.synchronize()
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        with P.Lattice(L, stream=side) as lat:
            Up = lat.pack_links(_t(U, dev))
            out = lat.dslash(Up, lat.pack_vec(_t(chi, dev)), 1)
            got = out.clone()  # ordered after the Dslash on the same stream
            x, _ = lat.cg_solve(Up, _t(b, dev), 0.1)
            xs = x.clone()
    side.synchronize()
    assert torch.equal(got, ref)
    assert torch.equal(xs, xr)


def test_dslash_graph_capture_replay(dev):
    """lgt_dslash is only a kernel launch, so it can be captured in a HIP graph:
    every replay (with new input written eagerly between replays) equals the
    eager call bit for bit."""
    L = (8, 8, 8, 8)
    U = li.links(L, "haar", 131)
    side = torch.cuda.Stream(dev)
    with P.Lattice(L, stream=side) as lat:
        with torch.cuda.stream(side):
            Up = lat.pack_links(_t(U, dev))
            x = lat.pack_vec(_t(li.vector(L, 132), dev))
            out = torch.empty_like(x)
            lat.dslash(Up, x, 0, out)  # warm-up outside the capture
        side.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            lat.dslash(Up, x, 0, out)
        for k in range(4):
            with torch.cuda.stream(side):
                x.copy_(lat.pack_vec(_t(li.vector(L, 140 + k), dev)))
            side.synchronize()
            g.replay()
            side.synchronize()
            with torch.cuda.stream(side):
                got = out.clone()
                ref = lat.dslash(Up, x, 0)
                got64 = lat.unpack_vec(got)
            side.synchronize()
            assert torch.equal(got, ref), k
            want = oracle.dslash(L, U, li.vector(L, 140 + k), 0)
            assert _rel(got64.cpu().numpy(), want) <= 1e-12


def test_force_and_mrhs_graph_capture_replay(dev):
    """lgt_force (pack X, Y = D_oe X, outer products; its workspace exists after
    a first call) and lgt_dslash_mrhs are kernel launches only: captured in one
    HIP graph and replayed three times with new inputs written eagerly in
    between, every replay equals the eager calls bit for bit."""
    L = (8, 8, 8, 8)
    U = li.links(L, "haar", 151)
    side = torch.cuda.Stream(dev)
    with P.Lattice(L, stream=side) as lat:
        with torch.cuda.stream(side):
            Ut = _t(U, dev)
            Up = lat.pack_links(Ut)
            U32 = lat.pack_links(Ut, P.LGT_F32, P.LGT_R12)
            X = _t(li.vector(L, 152), dev)
            vm = lat.pack_vec_mrhs(_t(li.vectors(L, 153, 4), dev), P.LGT_F32)
            om = torch.empty_like(vm)
            G = lat.force(Up, X)  # first call: allocates the force workspace
            lat.dslash_mrhs(U32, vm, 1, om)
        side.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            Gc = lat.force(Up, X)
            lat.dslash_mrhs(U32, vm, 1, om)
        for k in range(3):
            with torch.cuda.stream(side):
                X.copy_(_t(li.vector(L, 160 + k), dev))
                vm.copy_(lat.pack_vec_mrhs(_t(li.vectors(L, 170 + k, 4), dev), P.LGT_F32))
            side.synchronize()
            g.replay()
            side.synchronize()
            with torch.cuda.stream(side):
                got_G, got_m = Gc.clone(), om.clone()
                ref_G = lat.force(Up, X)
                ref_m = lat.dslash_mrhs(U32, vm, 1)
            side.synchronize()
            assert torch.equal(got_G, ref_G), k
            assert torch.equal(got_m, ref_m), k
        Gr = oracle.force(L, U, li.vector(L, 162))
        assert _rel(got_G.cpu().numpy(), Gr) <= 1e-12


def test_pack_unpack_roundtrip(dev):
    L = (4, 6, 4, 8)
    v = li.vector(L, 5)
    with P.Lattice(L) as lat:
        back = lat.unpack_vec(lat.pack_vec(_t(v, dev), P.LGT_F64), P.LGT_F64).cpu().numpy()
        np.testing.assert_array_equal(back, v)
        back32 = lat.unpack_vec(lat.pack_vec(_t(v, dev), P.LGT_F32), P.LGT_F32).cpu().numpy()
        np.testing.assert_array_equal(back32, v.astype(np.float32).astype(np.float64))


# ------------------------------------------------------------------- CG ---

def _true_resid(L, U, mass, b, x, bc=None):
    r = b - oracle.apply_A(L, U, mass, x, bc)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


CG_CASES = [
    # name, L, kind, c, mass, scheme, lo-format
    ("c1_fp64", (4, 4, 4, 4), "haar", None, 0.1, P.LGT_CG_FP64, None),
    ("fp64_8", (8, 8, 8, 8), "expih", 0.3, 0.05, P.LGT_CG_FP64, None),
    ("rel_f32r12", (8, 8, 8, 8), "haar", None, 0.1, P.LGT_CG_RELIABLE, (P.LGT_F32, P.LGT_R12)),
    ("rel_f32r18", (6, 4, 6, 8), "haar", None, 0.1, P.LGT_CG_RELIABLE, (P.LGT_F32, P.LGT_R18)),
    ("rel_bf16r12", (4, 4, 4, 4), "haar", None, 0.1, P.LGT_CG_RELIABLE, (P.LGT_BF16, P.LGT_R12)),
    ("ir_bf16r12", (8, 8, 8, 8), "haar", None, 0.1, P.LGT_CG_REFINE, (P.LGT_BF16, P.LGT_R12)),
    ("ir_f32r12", (8, 8, 8, 8), "expih", 0.3, 0.05, P.LGT_CG_REFINE, (P.LGT_F32, P.LGT_R12)),
]


@pytest.mark.parametrize("case", CG_CASES, ids=[c[0] for c in CG_CASES])
def test_cg_parity(dev, case):
    name, L, kind, c, mass, scheme, lo = case
    print("cg", name, flush=True)
    tol = 1e-10
    U = li.links(L, kind, 201, c=c if c else 0.3)
    b = li.vector(L, 202)
    st, xo, it_o, rr_o = oracle.cg(L, U, mass, b, tol=tol)
    assert st == 0
    with P.Lattice(L) as lat:
        Uh = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        Ul = lat.pack_links(_t(U, dev), *lo) if lo else None
        x, res = lat.cg_solve(Uh, _t(b, dev), mass, tol=tol, scheme=scheme, U_lo=Ul, ru_interval=50,
                              inner_tol=0.1 if scheme == P.LGT_CG_REFINE else 0.0)
    xg = x.cpu().numpy()
    rr = _true_resid(L, U, mass, b, xg)
    print(f"  {name}: gpu iters {res.iters} updates {res.updates} gpu resid {res.true_rel_resid:.3e} "
          f"oracle-resid {rr:.3e}; oracle iters {it_o}", flush=True)
    assert res.status == 0
    assert rr <= tol * 1.05
    assert abs(res.true_rel_resid - rr) <= 1e-3 * tol + 0.05 * rr
    bound = (tol * 1.05 + rr_o) * np.linalg.norm(b) / (4 * mass * mass)
    assert np.linalg.norm(xg - xo) <= bound
    if scheme == P.LGT_CG_FP64:
        assert abs(res.iters - it_o) <= 3


@pytest.mark.parametrize("scheme", [P.LGT_CG_FP64, P.LGT_CG_RELIABLE], ids=["fp64", "rel_f32r12"])
def test_cg_fp64_12real_links(dev, scheme):
    """FP64 links stored as 12 reals (third row rebuilt in FP64) in the FP64
    solve and in the FP64 residuals of reliable updates: same bound as with 18
    reals, and the same iteration count to within a few."""
    L, mass, tol = (8, 8, 8, 8), 0.1, 1e-10
    U = li.links(L, "haar", 211)
    b = li.vector(L, 212)
    st, xo, it_o, rr_o = oracle.cg(L, U, mass, b, tol=tol)
    with P.Lattice(L) as lat:
        Uh = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R12)
        Ul = lat.pack_links(_t(U, dev), P.LGT_F32, P.LGT_R12) if scheme == P.LGT_CG_RELIABLE else None
        x, res = lat.cg_solve(Uh, _t(b, dev), mass, tol=tol, scheme=scheme, U_lo=Ul)
    xg = x.cpu().numpy()
    rr = _true_resid(L, U, mass, b, xg)
    assert res.status == 0 and rr <= 1.05 * tol
    assert np.linalg.norm(xg - xo) <= (1.05 * tol + rr_o) * np.linalg.norm(b) / (4 * mass * mass)
    if scheme == P.LGT_CG_FP64:
        assert abs(res.iters - it_o) <= 3


def test_cg_free_field_plane_wave(dev):
    """Unit links: b is an eigenvector of A with eigenvalue 4 (m^2 + sum sin^2 p)."""
    L = (8, 4, 6, 4)
    m = 0.2
    n = (1, 1, 2, 0)
    U = li.links(L, "unit")
    import brute
    z = np.zeros((int(np.prod(L)) // 2, 3), complex)
    for lex, co in brute.sites(L):
        e = brute.eo_index(L, co)
        if e < len(z):
            z[e] = np.exp(1j * sum(2 * math.pi * n[mu] * co[mu] / L[mu] for mu in range(4))) * \
                np.array([1.0, -0.5j, 0.25])
    b = li.to_real(z)
    lam = 4 * (m * m + sum(math.sin(2 * math.pi * n[mu] / L[mu]) ** 2 for mu in range(4)))
    with P.Lattice(L) as lat:
        x, res = lat.cg_solve(lat.pack_links(_t(U, dev)), _t(b, dev), m, tol=1e-12)
    np.testing.assert_allclose(x.cpu().numpy(), b / lam, atol=1e-12)
    assert res.iters <= 2


def test_cg_status_paths(dev):
    L = (4, 4, 4, 4)
    U = li.links(L, "haar", 301)
    b = li.vector(L, 302)
    with P.Lattice(L) as lat:
        Up = lat.pack_links(_t(U, dev))
        # zero source: x = 0 at once
        x, res = lat.cg_solve(Up, torch.zeros((128, 3, 2), dtype=torch.float64, device=dev), 0.1)
        assert res.status == 0 and res.iters == 0 and not x.any()
        # iteration cap: NOT_CONVERGED with the best x written
        x, res = lat.cg_solve(Up, _t(b, dev), 0.1, max_iter=5, raise_on_fail=False)
        assert res.status == -5 and res.iters == 5
        assert _true_resid(L, U, 0.1, b, x.cpu().numpy()) == pytest.approx(res.true_rel_resid, rel=1e-6)
        with pytest.raises(P.LgtError) as e:
            lat.cg_solve(Up, _t(b, dev), 0.1, max_iter=5)
        assert e.value.status == -5
        # non-finite source
        bn = b.copy()
        bn[3, 1, 0] = np.nan
        x, res = lat.cg_solve(Up, _t(bn, dev), 0.1, raise_on_fail=False)
        assert res.status == -6
        # warm restart from a returned x
        x5, _ = lat.cg_solve(Up, _t(b, dev), 0.1, max_iter=5, raise_on_fail=False)
        x, res = lat.cg_solve(Up, _t(b, dev), 0.1, x0=x5)
        assert res.status == 0
        assert _true_resid(L, U, 0.1, b, x.cpu().numpy()) <= 1.05e-10


def test_cg_deterministic(dev):
    L = (8, 8, 8, 8)
    U = li.links(L, "haar", 401)
    b = li.vector(L, 402)
    with P.Lattice(L) as lat:
        Uh = lat.pack_links(_t(U, dev))
        Ul = lat.pack_links(_t(U, dev), P.LGT_F32, P.LGT_R12)
        for scheme, lo in ((P.LGT_CG_FP64, None), (P.LGT_CG_RELIABLE, Ul)):
            x1, r1 = lat.cg_solve(Uh, _t(b, dev), 0.1, scheme=scheme, U_lo=lo)
            x2, r2 = lat.cg_solve(Uh, _t(b, dev), 0.1, scheme=scheme, U_lo=lo)
            assert torch.equal(x1, x2) and r1.iters == r2.iters


def test_cg_dslash_profile_by_kind(dev):
    """With timing on every iteration, lgt_cg_dslash_profile counts one
    iteration D_oe and one D_eo per iteration, and the FP64-update pairs of a
    mixed solve; every mean time is positive, and timing leaves the solve
    bit-identical."""
    L = (8, 8, 8, 8)
    U = li.links(L, "haar", 431)
    b = li.vector(L, 432)
    with P.Lattice(L) as lat:
        Uh = lat.pack_links(_t(U, dev))
        Ul = lat.pack_links(_t(U, dev), P.LGT_F32, P.LGT_R12)
        for scheme, lo in ((P.LGT_CG_FP64, None), (P.LGT_CG_RELIABLE, Ul)):
            x0, r0 = lat.cg_solve(Uh, _t(b, dev), 0.1, scheme=scheme, U_lo=lo)
            lat.set_timing(1)
            x1, r1 = lat.cg_solve(Uh, _t(b, dev), 0.1, scheme=scheme, U_lo=lo)
            lat.set_timing(0)
            prof = lat.cg_dslash_profile()
            assert torch.equal(x0, x1) and r0.iters == r1.iters
            assert prof["iter_doe"]["n"] == prof["iter_deo_update"]["n"] == r1.iters
            assert prof["iter_doe"]["ms"] > 0 and prof["iter_deo_update"]["ms"] > 0
            if scheme == P.LGT_CG_RELIABLE:
                assert prof["ru_doe"]["n"] == prof["ru_deo_residual"]["n"] >= 1
                assert prof["ru_doe"]["ms"] > 0 and prof["ru_deo_residual"]["ms"] > 0


@pytest.mark.parametrize("L", [(8, 8, 8, 8), (16, 16, 16, 32)])
def test_cg_alpha_step_fused_or_separate(dev, L, monkeypatch):
    """alpha = rho / <p, Ap> summed from D_oe's partials by every workgroup of
    the D_eo that applies the update (small lattices) or by one finalize
    workgroup first (large lattices; forced here with LGT_FUSE_ALPHA_MAX=0):
    the same solve bit for bit, in every scheme, and a non-finite source still
    ends in LGT_ERR_NONFINITE."""
    U = li.links(L, "haar", 421)
    b = li.vector(L, 422)
    with P.Lattice(L) as lat:
        Uh = lat.pack_links(_t(U, dev))
        Ul = lat.pack_links(_t(U, dev), P.LGT_F32, P.LGT_R12)
        Ub = lat.pack_links(_t(U, dev), P.LGT_BF16, P.LGT_R12)
        for scheme, lo, itol in ((P.LGT_CG_FP64, None, 0.0), (P.LGT_CG_RELIABLE, Ul, 0.0),
                                 (P.LGT_CG_REFINE, Ub, 0.1)):
            out = []
            for limit in ("1073741824", "0"):
                monkeypatch.setenv("LGT_FUSE_ALPHA_MAX", limit)
                out.append(lat.cg_solve(Uh, _t(b, dev), 0.1, scheme=scheme, U_lo=lo, inner_tol=itol))
            assert torch.equal(out[0][0], out[1][0])
            assert out[0][1].iters == out[1][1].iters and out[0][1].updates == out[1][1].updates
            assert out[0][1].true_rel_resid == out[1][1].true_rel_resid
            assert out[1][1].true_rel_resid <= 1e-10
        # a NaN source: both paths stop with LGT_ERR_NONFINITE
        bn = b.copy()
        bn[3, 1, 0] = np.nan
        for limit in ("1073741824", "0"):
            monkeypatch.setenv("LGT_FUSE_ALPHA_MAX", limit)
            _, r = lat.cg_solve(Uh, _t(bn, dev), 0.1, raise_on_fail=False)
            assert r.status == -6
    assert _true_resid(L, U, 0.1, b, out[1][0].cpu().numpy()) <= 1.05e-10


@pytest.mark.parametrize("L", [(8, 8, 8, 8), (32, 4, 4, 6)])
def test_cg_lds_variant_bit_identical(dev, L):
    """The CG's Dslash launches (plain, 4m^2 p - D with <p,Ap>, and the FP64
    residual epilogues of the reliable updates) give bit-identical solves with
    the LDS-staged variant and the 2-hop variant it repeats."""
    U = li.links(L, "haar", 411)
    b = li.vector(L, 412)
    with P.Lattice(L) as lat:
        Uh = lat.pack_links(_t(U, dev))
        Ul = lat.pack_links(_t(U, dev), P.LGT_F32, P.LGT_R12)
        for scheme, lo in ((P.LGT_CG_FP64, None), (P.LGT_CG_RELIABLE, Ul)):
            out = []
            for hops in (4, 2):
                lat.set_dslash_variant(P.LGT_F64, P.LGT_R18, hops, 1)
                lat.set_dslash_variant(P.LGT_F32, P.LGT_R12, hops, 0)
                out.append(lat.cg_solve(Uh, _t(b, dev), 0.1, scheme=scheme, U_lo=lo))
            assert torch.equal(out[0][0], out[1][0]) and out[0][1].iters == out[1][1].iters
            assert out[0][1].updates == out[1][1].updates
    assert _true_resid(L, U, 0.1, b, out[0][0].cpu().numpy()) <= 1.05e-10


# ---------------------------------------------------------------- force ---

@pytest.mark.parametrize("L,bc", [((4, 4, 4, 4), (1, 1, 1, 1)), ((6, 4, 6, 8), (1, 1, 1, -1)),
                                  ((16, 16, 16, 32), (1, 1, 1, 1))])
def test_force_parity(dev, L, bc):
    print("force", L, flush=True)
    U = li.links(L, "expih", 501, c=0.5)
    X = li.vector(L, 502)
    with P.Lattice(L, bc) as lat:
        G = lat.force(lat.pack_links(_t(U, dev)), _t(X, dev), scale=1.0).cpu().numpy()
    Gr = oracle.force(L, U, X, bc)
    assert _rel(G, Gr) <= 1e-12
    assert np.abs(G - Gr).max() <= 1e-12 * np.abs(Gr).max()


def test_action_phi_grad(dev):
    """lgt_action_phi_grad: scale * dS/dphi = 2 scale X, against the oracle's derivative."""
    L = (6, 4, 6, 8)
    X = li.vector(L, 591)
    with P.Lattice(L) as lat:
        for scale in (1.0, -0.75, 3.1):
            got = lat.action_phi_grad(_t(X, dev), scale).cpu().numpy()
            want = scale * oracle.action_phi_grad(X)
            assert np.abs(got - want).max() <= 2.0 ** -52 * np.abs(want).max()


def test_autograd_action_vs_oracle(dev):
    L, mass = (4, 4, 4, 8), 0.05
    U = li.links(L, "expih", 601, c=0.5)
    phi = li.vector(L, 602)
    st, Xo, _, _ = oracle.cg(L, U, mass, phi, tol=1e-13)
    Go = oracle.force(L, U, Xo)
    S_o = oracle.cdot(phi, Xo).real
    with P.Lattice(L) as lat:
        Ut = _t(U, dev).requires_grad_(True)
        pt = _t(phi, dev).requires_grad_(True)
        S = P.PseudofermionAction.apply(Ut, pt, lat, mass, 1e-13)
        (2.5 * S).backward()
    assert abs(S.item() - S_o) <= 1e-11 * abs(S_o)
    kappa = (4 * (mass ** 2) + 64) / (4 * mass ** 2)
    assert _rel(Ut.grad.cpu().numpy(), 2.5 * Go) <= kappa * 1e-13 * 10
    np.testing.assert_allclose(pt.grad.cpu().numpy(), 2.5 * 2 * Xo, atol=1e-8 * np.abs(Xo).max())


def test_autograd_action_mixed_precision(dev):
    """The action's forward solve with FP32 x 12 links and FP64 reliable
    updates: S and dS/dU against the oracle to the same O(kappa tol) bound."""
    L, mass, tol = (4, 4, 4, 8), 0.05, 1e-12
    U = li.links(L, "expih", 611, c=0.5)
    phi = li.vector(L, 612)
    st, Xo, _, _ = oracle.cg(L, U, mass, phi, tol=1e-13)
    Go = oracle.force(L, U, Xo)
    S_o = oracle.cdot(phi, Xo).real
    with P.Lattice(L) as lat:
        Ut = _t(U, dev).requires_grad_(True)
        S = P.PseudofermionAction.apply(Ut, _t(phi, dev), lat, mass, tol, 100000, True)
        S.backward()
    kappa = (4 * (mass ** 2) + 64) / (4 * mass ** 2)
    assert abs(S.item() - S_o) <= kappa * tol * abs(S_o)
    assert _rel(Ut.grad.cpu().numpy(), Go) <= kappa * tol * 10


def test_stream_copy(dev):
    with P.Lattice((4, 4, 4, 4)) as lat:
        src = torch.randn(1 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        lat.stream_copy(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
        with pytest.raises(P.LgtError):
            lat.stream_copy(src[1:], dst[1:])  # 8-byte offset: misaligned
