"""Batching form on the GPU: the multi-RHS Dslash and the batched CG (one
persistent launch for many right-hand sides and lattices of different sizes),
against the FP64 oracle and against the single-RHS solver."""
import numpy as np
import pytest

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


def _per_element(got, L, U, chi, par, prec, recon, bc, ref, what):
    """FP64: every component within 1e-12 max|ref|; FP32 / BF16 links: every
    output real within the FP32-arithmetic bound against the oracle on the
    stored (rounded) links and input (tests/lowprec.py)."""
    if prec == P.LGT_F64:
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), what
    else:
        lowprec.check_dslash(got, L, U, chi, par, prec, recon, bc, None, what)


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("nrhs", [1, 2, 4, 16])
def test_dslash_mrhs_parity(dev, fmt, nrhs):
    prec, recon, tol = FMTS[fmt]
    L, bc = (6, 4, 6, 8), (1, 1, 1, -1)
    U = li.links(L, "haar", 141)
    chis = li.vectors(L, 142, nrhs)
    vp = P.LGT_F64 if prec == P.LGT_F64 else P.LGT_F32
    with P.Lattice(L, bc) as lat:
        Up = lat.pack_links(_t(U, dev), prec, recon)
        for par in (0, 1):
            x = lat.pack_vec_mrhs(_t(chis, dev), vp)
            got = lat.unpack_vec_mrhs(lat.dslash_mrhs(Up, x, par), vp).cpu().numpy()
            for r in range(nrhs):
                ref = oracle.dslash(L, U, chis[r], par, bc)
                assert _rel(got[r], ref) <= tol, (fmt, nrhs, par, r)
                _per_element(got[r], L, U, chis[r], par, prec, recon, bc, ref, (fmt, nrhs, par, r))


ENGINES = {"lane": 0, "valu4": 1, "mfma": 2}


@pytest.mark.parametrize("engine", sorted(ENGINES))
@pytest.mark.parametrize("fmt", ["f32r18", "f32r12", "bf16r12"])
@pytest.mark.parametrize("nrhs", [4, 8, 16])
@pytest.mark.parametrize("L", [(8, 8, 8, 12), (6, 6, 6, 6)])
def test_dslash_mrhs_engines(dev, engine, fmt, nrhs, L):
    """Every multi-RHS engine against the oracle. 8^3x12 (V/2 = 3072) spans
    48 workgroups of four-lane sites; 6^4 (V/2 = 648, not a multiple of 16)
    leaves a ragged last workgroup, and the MFMA engine falls back to one
    lane per right-hand side there."""
    prec, recon, tol = FMTS[fmt]
    bc = (1, 1, 1, -1)
    U = li.links(L, "haar", 151)
    chis = li.vectors(L, 152, nrhs)
    with P.Lattice(L, bc) as lat:
        lat.set_mrhs_engine(ENGINES[engine])
        assert lat.mrhs_engine() == ENGINES[engine]
        Up = lat.pack_links(_t(U, dev), prec, recon)
        x = lat.pack_vec_mrhs(_t(chis, dev), P.LGT_F32)
        for par in (0, 1):
            got = lat.unpack_vec_mrhs(lat.dslash_mrhs(Up, x, par), P.LGT_F32).cpu().numpy()
            for r in range(nrhs):
                ref = oracle.dslash(L, U, chis[r], par, bc)
                assert _rel(got[r], ref) <= tol, (engine, fmt, nrhs, L, par, r)
                _per_element(got[r], L, U, chis[r], par, prec, recon, bc, ref, (engine, fmt, nrhs, L, par, r))


# every (engine, groups, nrhs) with at least one right-hand side per lane
SHAPES = [(e, g, n) for e in ("valu4", "mfma") for g in (1, 2, 4) for n in (4, 8, 16) if 4 * g <= n]


@pytest.mark.parametrize("engine,groups,nrhs", SHAPES)
@pytest.mark.parametrize("fmt", ["f32r12", "bf16r12"])
def test_dslash_mrhs_groups(dev, engine, groups, fmt, nrhs):
    """Every tile shape (groups of four lanes per site) of both four-lane
    engines against the oracle, at 8^3x12 (48+ workgroups)."""
    prec, recon, tol = FMTS[fmt]
    L, bc = (8, 8, 8, 12), (1, 1, 1, -1)
    U = li.links(L, "haar", 161)
    chis = li.vectors(L, 162, nrhs)
    with P.Lattice(L, bc) as lat:
        lat.set_mrhs_variant(prec, recon, nrhs, ENGINES[engine], groups)
        assert lat.mrhs_variant(prec, recon, nrhs) == (ENGINES[engine], groups)
        Up = lat.pack_links(_t(U, dev), prec, recon)
        x = lat.pack_vec_mrhs(_t(chis, dev), P.LGT_F32)
        for par in (0, 1):
            got = lat.unpack_vec_mrhs(lat.dslash_mrhs(Up, x, par), P.LGT_F32).cpu().numpy()
            for r in range(nrhs):
                ref = oracle.dslash(L, U, chis[r], par, bc)
                assert _rel(got[r], ref) <= tol, (engine, groups, fmt, nrhs, par, r)
                _per_element(got[r], L, U, chis[r], par, prec, recon, bc, ref, (engine, groups, fmt, nrhs, par, r))


@pytest.mark.parametrize("engine,groups,nrhs", SHAPES)
@pytest.mark.parametrize("fmt", ["f32r18", "f32r12", "bf16r12"])
def test_dslash_mrhs_staged(dev, engine, groups, fmt, nrhs):
    """The LDS-staged kernel of every four-lane tile shape: bit-identical to the
    unstaged one (same products in the same order, only the load path differs)
    and within the per-element bound of the oracle, at 8^3x12, at 12x8x8x16
    (z-ordered tiles, x/y neighbourhood split across tiles) and at 6x6x6x8
    (V/2 = 864: a ragged last tile, the MFMA engine running one lane per rhs)."""
    prec, recon, tol = FMTS[fmt]
    bc = (1, 1, 1, -1)
    for L in ((8, 8, 8, 12), (12, 8, 8, 16), (6, 6, 6, 8)):
        U = li.links(L, "haar", 171)
        chis = li.vectors(L, 172, nrhs)
        with P.Lattice(L, bc) as lat:
            lat.set_mrhs_variant(prec, recon, nrhs, ENGINES[engine], groups)
            Up = lat.pack_links(_t(U, dev), prec, recon)
            x = lat.pack_vec_mrhs(_t(chis, dev), P.LGT_F32)
            for par in (0, 1):
                lat.set_mrhs_staging(prec, recon, nrhs, False)
                plain = lat.dslash_mrhs(Up, x, par).clone()
                lat.set_mrhs_staging(prec, recon, nrhs, True)
                four = lat.mrhs_variant(prec, recon, nrhs)[0] != ENGINES["lane"]
                assert lat.mrhs_staging(prec, recon, nrhs) == four, (L, engine)
                staged = lat.dslash_mrhs(Up, x, par)
                assert torch.equal(staged, plain), (engine, groups, fmt, nrhs, L, par)
                got = lat.unpack_vec_mrhs(staged, P.LGT_F32).cpu().numpy()
                for r in range(nrhs):
                    ref = oracle.dslash(L, U, chis[r], par, bc)
                    _per_element(got[r], L, U, chis[r], par, prec, recon, bc, ref, (engine, groups, fmt, L, par, r))


def test_dslash_mrhs_staging_falls_back_when_the_tile_does_not_fit(dev):
    """Lx = 48, 16 rhs, one group: 3 x (128 + 48) sites x 16 x 8 B = 66 KB > 64 KB
    of LDS, so the unstaged kernel runs (and reports so)."""
    L, bc = (48, 4, 4, 4), (1, 1, 1, -1)
    U = li.links(L, "haar", 181)
    chis = li.vectors(L, 182, 16)
    with P.Lattice(L, bc) as lat:
        lat.set_mrhs_variant(P.LGT_F32, P.LGT_R12, 16, ENGINES["mfma"], 1)
        lat.set_mrhs_staging(P.LGT_F32, P.LGT_R12, 16, True)
        assert not lat.mrhs_staging(P.LGT_F32, P.LGT_R12, 16)
        lat.set_mrhs_variant(P.LGT_F32, P.LGT_R12, 16, ENGINES["mfma"], 2)  # 64-site tiles fit
        assert lat.mrhs_staging(P.LGT_F32, P.LGT_R12, 16)
        lat.set_mrhs_variant(P.LGT_F32, P.LGT_R12, 16, ENGINES["mfma"], 1)
        Up = lat.pack_links(_t(U, dev), P.LGT_F32, P.LGT_R12)
        x = lat.pack_vec_mrhs(_t(chis, dev), P.LGT_F32)
        got = lat.unpack_vec_mrhs(lat.dslash_mrhs(Up, x, 0), P.LGT_F32).cpu().numpy()
        for r in range(16):
            ref = oracle.dslash(L, U, chis[r], 0, bc)
            _per_element(got[r], L, U, chis[r], 0, P.LGT_F32, P.LGT_R12, bc, ref, ("fallback", r))
        with pytest.raises(P.LgtError):
            lat.set_mrhs_staging(P.LGT_F32, P.LGT_R12, 6, True)


def test_mrhs_variant_arguments(dev):
    with P.Lattice((4, 4, 4, 4)) as lat:
        for bad in ((P.LGT_F32, P.LGT_R12, 8, ENGINES["mfma"], 4),   # 4 groups need 16 rhs
                    (P.LGT_F32, P.LGT_R12, 16, ENGINES["mfma"], 3),  # groups 1, 2 or 4
                    (P.LGT_F32, P.LGT_R12, 6, ENGINES["mfma"], 1),   # nrhs a power of two <= 16
                    (P.LGT_F32, P.LGT_R12, 16, 5, 1)):               # unknown engine
            with pytest.raises(P.LgtError):
                lat.set_mrhs_variant(*bad)
        # FP64 links and nrhs < 4 always run one lane per (site, rhs)
        lat.set_mrhs_variant(P.LGT_F64, P.LGT_R18, 16, ENGINES["mfma"], 2)
        assert lat.mrhs_variant(P.LGT_F64, P.LGT_R18, 16) == (ENGINES["lane"], 1)
        assert lat.mrhs_variant(P.LGT_F32, P.LGT_R12, 2) == (ENGINES["lane"], 1)


def test_tune_dslash_mrhs(dev, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LGT_TUNE_CACHE", str(cache))
    L = (8, 8, 8, 8)
    U = li.links(L, "haar", 171)
    chis = li.vectors(L, 172, 16)
    with P.Lattice(L) as lat:
        Up = lat.pack_links(_t(U, dev), P.LGT_F32, P.LGT_R12)
        times = lat.tune_dslash_mrhs(Up, 16)
        # all thirteen shapes apply at N = 16 with V/2 a multiple of 16 (staged tiles fit)
        assert set(times) == set(P.Lattice.MRHS_VARIANTS) and all(t > 0 for t in times.values())

        def kept(lt):
            return lt.mrhs_variant(P.LGT_F32, P.LGT_R12, 16) + (int(lt.mrhs_staging(P.LGT_F32, P.LGT_R12, 16)),)
        best = min(times, key=times.get)
        assert kept(lat) == best
        x = lat.pack_vec_mrhs(_t(chis, dev), P.LGT_F32)
        got = lat.unpack_vec_mrhs(lat.dslash_mrhs(Up, x, 1), P.LGT_F32).cpu().numpy()
        for r in range(16):
            assert _rel(got[r], oracle.dslash(L, U, chis[r], 1)) <= 32 * U32
        # N = 4 on a lattice with V/2 = 648 (not a multiple of 16): no MFMA shapes
        lat2 = P.Lattice((6, 6, 6, 6))
        U2 = lat2.pack_links(_t(li.links((6, 6, 6, 6), "haar", 173), dev), P.LGT_F32, P.LGT_R12)
        t2 = lat2.tune_dslash_mrhs(U2, 4)
        assert set(t2) == {(ENGINES["lane"], 1, 0), (ENGINES["valu4"], 1, 0), (ENGINES["valu4"], 1, 1)}
        lat2.close()
    assert "mrhs16" in cache.read_text()
    # a new context picks the cached choice without timing
    with P.Lattice(L) as lat:
        Up = lat.pack_links(_t(U, dev), P.LGT_F32, P.LGT_R12)
        lat.tune_dslash_mrhs(Up, 16, report=False)
        assert kept(lat) == best


def test_mrhs_engine_rejects_unknown(dev):
    with P.Lattice((4, 4, 4, 4)) as lat:
        with pytest.raises(P.LgtError):
            lat.set_mrhs_engine(3)
        assert lat.mrhs_engine() == ENGINES["mfma"]


def test_mrhs_pack_roundtrip(dev):
    L = (4, 4, 4, 4)
    v = li.vectors(L, 7, 8)
    with P.Lattice(L) as lat:
        back = lat.unpack_vec_mrhs(lat.pack_vec_mrhs(_t(v, dev))).cpu().numpy()
    np.testing.assert_array_equal(back, v)


def _check_solution(L, U, mass, b, x, res, tol):
    r = b - oracle.apply_A(L, U, mass, x)
    rr = float(np.linalg.norm(r) / np.linalg.norm(b))
    assert res.status == 0, res
    assert rr <= 1.05 * tol, rr
    assert abs(res.true_rel_resid - rr) <= 1e-3 * tol + 0.05 * rr
    return rr


@pytest.mark.parametrize("scheme,lo", [(P.LGT_CG_FP64, None), (P.LGT_CG_RELIABLE, (P.LGT_F32, P.LGT_R12)),
                                       (P.LGT_CG_RELIABLE, (P.LGT_F32, P.LGT_R18)),
                                       (P.LGT_CG_REFINE, (P.LGT_BF16, P.LGT_R12))],
                         ids=["fp64", "rel_f32r12", "rel_f32r18", "ir_bf16r12"])
def test_batch_heterogeneous(dev, scheme, lo):
    """Three lattices of different sizes, 4 / 2 / 16 right-hand sides, one launch."""
    mass, tol = 0.1, 1e-10
    specs = [((8, 8, 8, 8), 4, 4101), ((6, 4, 6, 8), 2, 4201), ((4, 4, 4, 4), 16, 4301)]
    lats, probs, data = [], [], []
    for L, n, seed in specs:
        U = li.links(L, "haar", seed)
        b = li.vectors(L, seed + 10, n)
        lat = P.Lattice(L)
        Uh = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        Ul = lat.pack_links(_t(U, dev), *lo) if lo else None
        lats.append(lat)
        probs.append((lat, Uh, Ul, _t(b, dev)))
        data.append((L, U, b))
    print("batch", scheme, lo, flush=True)
    xs, res = P.cg_solve_batch(probs, mass, tol=tol, scheme=scheme, ru_interval=50,
                               inner_tol=0.1 if scheme == P.LGT_CG_REFINE else 0.0)
    for (L, U, b), x, rs in zip(data, xs, res):
        xg = x.cpu().numpy()
        for j in range(len(rs)):
            _check_solution(L, U, mass, b[j], xg[j], rs[j], tol)
            st, xo, it_o, rr_o = oracle.cg(L, U, mass, b[j], tol=tol)
            bound = (1.05 * tol + rr_o) * np.linalg.norm(b[j]) / (4 * mass * mass)
            assert np.linalg.norm(xg[j] - xo) <= bound
            if scheme == P.LGT_CG_FP64:
                assert abs(rs[j].iters - it_o) <= 3
    for lat in lats:
        lat.close()


@pytest.mark.parametrize("scheme,lo", [(P.LGT_CG_FP64, None), (P.LGT_CG_RELIABLE, (P.LGT_F32, P.LGT_R12)),
                                       (P.LGT_CG_REFINE, (P.LGT_BF16, P.LGT_R12))],
                         ids=["fp64", "rel_f32r12", "ir_bf16r12"])
def test_batch_ragged_rhs_counts(dev, scheme, lo):
    """1, 3, 5 and 13 right-hand sides (padded inside to 1, 4, 8 and 16 with
    zero sources): every solution meets the tolerance by the oracle's residual,
    and the first three of a 3-RHS problem are bit-identical to the same three
    solved in a 4-RHS problem (right-hand sides never mix)."""
    mass, tol = 0.1, 1e-10
    specs = [((8, 8, 8, 8), 3, 4501), ((6, 4, 6, 8), 5, 4511), ((4, 4, 4, 4), 13, 4521), ((4, 4, 4, 6), 1, 4531)]
    lats, probs, data = [], [], []
    for L, n, seed in specs:
        U = li.links(L, "haar", seed)
        b = li.vectors(L, seed + 1, n)
        lat = P.Lattice(L)
        Uh = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        Ul = lat.pack_links(_t(U, dev), *lo) if lo else None
        lats.append(lat)
        probs.append((lat, Uh, Ul, _t(b, dev)))
        data.append((L, U, b))
    print("batch ragged", scheme, flush=True)
    itol = 0.1 if scheme == P.LGT_CG_REFINE else 0.0
    xs, res = P.cg_solve_batch(probs, mass, tol=tol, scheme=scheme, inner_tol=itol)
    for (L, U, b), x, rs in zip(data, xs, res):
        assert x.shape[0] == b.shape[0] and len(rs) == b.shape[0]
        xg = x.cpu().numpy()
        for j in range(len(rs)):
            _check_solution(L, U, mass, b[j], xg[j], rs[j], tol)
    # the 3-RHS problem again with a fourth right-hand side in place of the padding
    L, U, b = data[0]
    b4 = np.concatenate([b, li.vectors(L, 4509, 1)])
    lat, Uh, Ul, _ = probs[0]
    x4, r4 = P.cg_solve_batch([(lat, Uh, Ul, _t(b4, dev))], mass, tol=tol, scheme=scheme, inner_tol=itol)
    x3, r3 = P.cg_solve_batch([(lat, Uh, Ul, _t(b, dev))], mass, tol=tol, scheme=scheme, inner_tol=itol)
    assert torch.equal(x3[0], x4[0][:3])
    assert [r.iters for r in r3[0]] == [r.iters for r in r4[0][:3]]
    for lat in lats:
        lat.close()


def test_batch_rejects_bad_rhs_counts(dev):
    L = (4, 4, 4, 4)
    U = li.links(L, "haar", 4541)
    with P.Lattice(L) as lat:
        Uh = lat.pack_links(_t(U, dev))
        for n in (0, 17, 20):
            b = _t(li.vectors(L, 4542, n), dev)
            with pytest.raises(P.LgtError) as e:
                P.cg_solve_batch([(lat, Uh, None, b)], 0.1, scheme=P.LGT_CG_FP64)
            assert e.value.status == -1


def test_batch_matches_single_solves_c4_shape(dev):
    """24^3 x 48 is too large for a quick oracle solve: compare the 16-RHS batch
    with the single-RHS solver on the same lattice, right-hand side by right-hand
    side, on a 12^3 x 24 lattice of the same aspect, m = 0.02."""
    L, n, mass, tol = (12, 12, 12, 24), 16, 0.02, 1e-10
    U = li.links(L, "haar", 4001)
    b = li.vectors(L, 4010, n)
    with P.Lattice(L) as lat:
        Uh = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        Ul = lat.pack_links(_t(U, dev), P.LGT_F32, P.LGT_R12)
        xs, res = P.cg_solve_batch([(lat, Uh, Ul, _t(b, dev))], mass, tol=tol)
        xb = xs[0].cpu().numpy()
        for j in (0, 7, 15):
            xj, rj = lat.cg_solve(Uh, _t(b[j], dev), mass, tol=tol, scheme=P.LGT_CG_RELIABLE, U_lo=Ul)
            assert res[0][j].status == 0 and rj.status == 0
            bound = 2.1 * tol * np.linalg.norm(b[j]) / (4 * mass * mass)
            assert np.linalg.norm(xb[j] - xj.cpu().numpy()) <= bound
            assert abs(res[0][j].iters - rj.iters) <= max(10, rj.iters // 20)
        # the oracle's FP64 residual of a few batch solutions
        for j in (0, 15):
            r = b[j] - oracle.apply_A(L, U, mass, xb[j])
            assert np.linalg.norm(r) / np.linalg.norm(b[j]) <= 1.05 * tol


@pytest.mark.parametrize("scheme,lo", [(P.LGT_CG_FP64, None), (P.LGT_CG_RELIABLE, (P.LGT_F32, P.LGT_R12)),
                                       (P.LGT_CG_REFINE, (P.LGT_BF16, P.LGT_R12))],
                         ids=["fp64", "rel_f32r12", "ir_bf16r12"])
def test_batch_two_pass_step1(dev, scheme, lo, monkeypatch):
    """24^4 x 16 (2.65M site-rhs pairs: step 1 runs as two passes, p' and then
    D_oe p') next to 8^4 x 4 in the same persistent launch (forced: two mixed
    problems would run as kernel launches): every right-hand side checked
    against the oracle's FP64 residual, the large lattice's against the single
    solver's solution."""
    monkeypatch.setenv("LGT_BATCH_LAUNCHED", "0")
    mass, tol = 0.05, 1e-10
    Lb, Ls = (24, 24, 24, 24), (8, 8, 8, 8)
    Ub, Us = li.links(Lb, "expih", 4501, c=0.3), li.links(Ls, "haar", 4502)
    bb, bs = li.vectors(Lb, 4503, 16), li.vectors(Ls, 4504, 4)
    with P.Lattice(Lb) as lb, P.Lattice(Ls) as ls:
        probs = []
        for lat, U, b in ((lb, Ub, bb), (ls, Us, bs)):
            Ut = _t(U, dev)
            ul = lat.pack_links(Ut, *lo) if lo else None
            probs.append((lat, lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), ul, _t(b, dev)))
        xs, res = P.cg_solve_batch(probs, mass, tol=tol, scheme=scheme,
                                   inner_tol=0.1 if scheme == P.LGT_CG_REFINE else 0.0)
        xb = xs[0].cpu().numpy()
        xj, rj = lb.cg_solve(probs[0][1], probs[0][3][5], mass, tol=tol, scheme=scheme, U_lo=probs[0][2],
                             inner_tol=0.1 if scheme == P.LGT_CG_REFINE else 0.0)
    assert rj.status == 0
    assert np.linalg.norm(xb[5] - xj.cpu().numpy()) <= 2.1 * tol * np.linalg.norm(bb[5]) / (4 * mass * mass)
    for j in (0, 5, 15):
        _check_solution(Lb, Ub, mass, bb[j], xb[j], res[0][j], tol)
    for j in range(4):
        _check_solution(Ls, Us, mass, bs[j], xs[1].cpu().numpy()[j], res[1][j], tol)


def test_batch_iteration_cap_and_determinism(dev):
    L = (4, 4, 4, 4)
    U = li.links(L, "haar", 4401)
    b = li.vectors(L, 4402, 4)
    with P.Lattice(L) as lat:
        Uh = lat.pack_links(_t(U, dev))
        xs, res = P.cg_solve_batch([(lat, Uh, None, _t(b, dev))], 0.1, scheme=P.LGT_CG_FP64, max_iter=7,
                                   raise_on_fail=False)
        assert all(r.status == -5 and r.iters == 7 for r in res[0])
        x1, r1 = P.cg_solve_batch([(lat, Uh, None, _t(b, dev))], 0.1, scheme=P.LGT_CG_FP64)
        x2, r2 = P.cg_solve_batch([(lat, Uh, None, _t(b, dev))], 0.1, scheme=P.LGT_CG_FP64)
        assert torch.equal(x1[0], x2[0])
        assert [r.iters for r in r1[0]] == [r.iters for r in r2[0]]


@pytest.mark.parametrize("nrhs,engine,groups", [(8, "valu4", 1), (8, "mfma", 2), (16, "valu4", 4),
                                                (16, "mfma", 2), (16, "mfma", 4), (16, "lane", 1)])
def test_batch_inner_shapes(dev, nrhs, engine, groups, monkeypatch):
    """The persistent batched solver with each inner-Dslash shape it runs (forced:
    one mixed problem would run as kernel launches): every right-hand side's
    oracle-recomputed residual within the tolerance."""
    monkeypatch.setenv("LGT_BATCH_LAUNCHED", "0")
    L, mass, tol = (8, 8, 8, 12), 0.1, 1e-10
    U = li.links(L, "haar", 181)
    bs = li.vectors(L, 182, nrhs)
    with P.Lattice(L) as lat:
        lat.set_mrhs_variant(P.LGT_F32, P.LGT_R12, nrhs, ENGINES[engine], groups)
        Ut = _t(U, dev)
        uh, ul = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), lat.pack_links(Ut, P.LGT_F32, P.LGT_R12)
        xs, res = P.cg_solve_batch([(lat, uh, ul, _t(bs, dev))], mass, tol=tol, scheme=P.LGT_CG_RELIABLE)
    xg = xs[0].cpu().numpy()
    for j in range(nrhs):
        _check_solution(L, U, mass, bs[j], xg[j], res[0][j], tol)


def test_batch_barrier_timeout_is_reported(dev, monkeypatch):
    """A grid-barrier wait bounded at one poll (LGT_BATCH_SPIN_LIMIT, set on
    the host) times out: every workgroup leaves the persistent kernel, the call
    returns LGT_ERR_DEVICE naming the barrier, and the next call with the
    normal bound solves the same batch (the persistent launch forced: this
    mixed one-problem batch would run as kernel launches)."""
    monkeypatch.setenv("LGT_BATCH_LAUNCHED", "0")
    L, mass = (8, 8, 8, 8), 0.1
    U = li.links(L, "haar", 181)
    bs = li.vectors(L, 182, 4)
    with P.Lattice(L) as lat:
        Ut = torch.from_numpy(U).to(dev)
        uh, ul = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), lat.pack_links(Ut, P.LGT_F32, P.LGT_R12)
        probs = [(lat, uh, ul, torch.from_numpy(bs).to(dev))]
        monkeypatch.setenv("LGT_BATCH_SPIN_LIMIT", "1")
        with pytest.raises(P.LgtError) as ei:
            P.cg_solve_batch(probs, mass, tol=1e-10, scheme=P.LGT_CG_RELIABLE)
        assert ei.value.status == -4 and "barrier" in str(ei.value)
        torch.cuda.synchronize()
        monkeypatch.setenv("LGT_BATCH_SPIN_LIMIT", "0")
        with pytest.raises(P.LgtError) as ei:                  # out of range: rejected before any launch
            P.cg_solve_batch(probs, mass, tol=1e-10, scheme=P.LGT_CG_RELIABLE)
        assert ei.value.status == -1
        monkeypatch.delenv("LGT_BATCH_SPIN_LIMIT")
        xs, res = P.cg_solve_batch(probs, mass, tol=1e-10, scheme=P.LGT_CG_RELIABLE)
    assert all(r.status == 0 for r in res[0])
    x = xs[0].cpu().numpy()
    for j in range(4):
        r = bs[j] - oracle.apply_A(L, U, mass, x[j])
        assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(bs[j])
