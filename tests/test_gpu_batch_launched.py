"""The batched CG as kernel launches (the form lgt_cg_solve_batch takes for
mixed-precision batches of up to four problems on different contexts, each
with a four-lane inner engine): every right-hand side against the FP64
oracle's residual, against the persistent launch's solution of the same batch
and against the single-RHS solver, at small shapes and at 24^3 x 48 x 16;
several problems at once, also on one shared context."""
import numpy as np
import pytest

import lgt_inputs as li
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1309_0551_amd")

pytestmark = pytest.mark.gpu

ENGINES = {"valu4": 1, "mfma": 2}
LO = {"f32r12": (P.LGT_F32, P.LGT_R12), "f32r18": (P.LGT_F32, P.LGT_R18), "bf16r12": (P.LGT_BF16, P.LGT_R12)}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _check_solution(L, U, mass, b, x, res, tol):
    r = b - oracle.apply_A(L, U, mass, x)
    rr = float(np.linalg.norm(r) / np.linalg.norm(b))
    assert res.status == 0, res
    assert rr <= 1.05 * tol, rr
    assert abs(res.true_rel_resid - rr) <= 1e-3 * tol + 0.05 * rr
    return rr


def _solve(monkeypatch, mode, probs, mass, tol, scheme, **kw):
    monkeypatch.setenv("LGT_BATCH_LAUNCHED", mode)
    try:
        return P.cg_solve_batch(probs, mass, tol=tol, scheme=scheme, **kw)
    finally:
        monkeypatch.delenv("LGT_BATCH_LAUNCHED")


def _is_launched(lat):
    """The launched form leaves no barrier waits in the phase profile and
    times its p = r + beta p pass separately."""
    prof = lat.batch_profile()
    return prof["wait1"] == 0.0 and prof["wait2"] == 0.0 and prof["step1_p"] > 0.0


SHAPES = [(n, e, g) for e in ("valu4", "mfma") for g in (1, 2, 4) for n in (4, 8, 16) if 4 * g <= n]


@pytest.mark.parametrize("nrhs,engine,groups", SHAPES)
@pytest.mark.parametrize("scheme,lo", [(P.LGT_CG_RELIABLE, "f32r12"), (P.LGT_CG_REFINE, "bf16r12")],
                         ids=["rel_f32r12", "ir_bf16r12"])
def test_launched_shapes(dev, monkeypatch, nrhs, engine, groups, scheme, lo):
    """Every inner-Dslash shape (engine, groups of four lanes, N; a request for
    one group at N = 16 runs two, in both forms): each right-hand side within
    the tolerance by the oracle's residual, and within the tolerance's bound of
    the persistent launch's solution of the same batch."""
    L, mass, tol = (8, 8, 8, 12), 0.1, 1e-10
    U = li.links(L, "haar", 6101)
    bs = li.vectors(L, 6102, nrhs)
    itol = 0.1 if scheme == P.LGT_CG_REFINE else 0.0
    print("launched", nrhs, engine, groups, lo, flush=True)
    with P.Lattice(L) as lat:
        lat.set_mrhs_variant(*LO[lo], nrhs, ENGINES[engine], groups)
        Ut = _t(U, dev)
        uh, ul = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), lat.pack_links(Ut, *LO[lo])
        probs = [(lat, uh, ul, _t(bs, dev))]
        lat.set_timing(1)
        xl, rl = _solve(monkeypatch, "1", probs, mass, tol, scheme, inner_tol=itol)
        assert _is_launched(lat)
        xp, rp = _solve(monkeypatch, "0", probs, mass, tol, scheme, inner_tol=itol)
        assert not _is_launched(lat)
        lat.set_timing(0)
    xg, xq = xl[0].cpu().numpy(), xp[0].cpu().numpy()
    for j in range(nrhs):
        _check_solution(L, U, mass, bs[j], xg[j], rl[0][j], tol)
        bound = 2.1 * tol * np.linalg.norm(bs[j]) / (4 * mass * mass)
        assert np.linalg.norm(xg[j] - xq[j]) <= bound
        assert abs(rl[0][j].iters - rp[0][j].iters) <= max(12, rp[0][j].iters // 10)


@pytest.mark.parametrize("lo", ["f32r18", "f32r12", "bf16r12"])
def test_launched_ragged_tail_and_mfma_fallback(dev, monkeypatch, lo):
    """6^4: V/2 = 648 leaves a ragged last tile at every tile size and is not a
    multiple of 16, so a request for the MFMA engine runs the VALU one; each
    right-hand side checked against the oracle's residual."""
    L, mass, tol, nrhs = (6, 6, 6, 6), 0.1, 1e-10, 8
    U = li.links(L, "haar", 6111)
    bs = li.vectors(L, 6112, nrhs)
    scheme = P.LGT_CG_REFINE if lo == "bf16r12" else P.LGT_CG_RELIABLE
    with P.Lattice(L) as lat:
        lat.set_mrhs_variant(*LO[lo], nrhs, ENGINES["mfma"], 2)
        Ut = _t(U, dev)
        probs = [(lat, lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), lat.pack_links(Ut, *LO[lo]), _t(bs, dev))]
        xs, res = _solve(monkeypatch, "1", probs, mass, tol, scheme,
                         inner_tol=0.1 if scheme == P.LGT_CG_REFINE else 0.0)
    xg = xs[0].cpu().numpy()
    for j in range(nrhs):
        _check_solution(L, U, mass, bs[j], xg[j], res[0][j], tol)


def test_launched_ragged_rhs_counts_and_independence(dev, monkeypatch):
    """3 and 13 right-hand sides (padded to 4 and 16 with zero sources) meet the
    tolerance; the 3-RHS solutions are bit-identical to the first three of a
    4-RHS batch (right-hand sides never mix) and to a second run (fixed-order
    sums)."""
    L, mass, tol = (8, 8, 8, 8), 0.1, 1e-10
    U = li.links(L, "haar", 6121)
    b13 = li.vectors(L, 6122, 13)
    with P.Lattice(L) as lat:
        Ut = _t(U, dev)
        uh, ul = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), lat.pack_links(Ut, P.LGT_F32, P.LGT_R12)
        for b in (b13[:3], b13):
            xs, res = _solve(monkeypatch, "1", [(lat, uh, ul, _t(b, dev))], mass, tol, P.LGT_CG_RELIABLE)
            assert xs[0].shape[0] == b.shape[0] and len(res[0]) == b.shape[0]
            xg = xs[0].cpu().numpy()
            for j in range(b.shape[0]):
                _check_solution(L, U, mass, b[j], xg[j], res[0][j], tol)
        x3, r3 = _solve(monkeypatch, "1", [(lat, uh, ul, _t(b13[:3], dev))], mass, tol, P.LGT_CG_RELIABLE)
        x3b, r3b = _solve(monkeypatch, "1", [(lat, uh, ul, _t(b13[:3], dev))], mass, tol, P.LGT_CG_RELIABLE)
        x4, r4 = _solve(monkeypatch, "1", [(lat, uh, ul, _t(b13[:4], dev))], mass, tol, P.LGT_CG_RELIABLE)
    assert torch.equal(x3[0], x3b[0])
    assert torch.equal(x3[0], x4[0][:3])
    assert [r.iters for r in r3[0]] == [r.iters for r in r4[0][:3]] == [r.iters for r in r3b[0]]


def test_launched_iteration_cap(dev, monkeypatch):
    L, mass = (8, 8, 8, 8), 0.1
    U = li.links(L, "haar", 6131)
    bs = li.vectors(L, 6132, 4)
    with P.Lattice(L) as lat:
        Ut = _t(U, dev)
        uh, ul = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), lat.pack_links(Ut, P.LGT_F32, P.LGT_R12)
        probs = [(lat, uh, ul, _t(bs, dev))]
        xs, res = _solve(monkeypatch, "1", probs, mass, 1e-10, P.LGT_CG_RELIABLE, max_iter=7, raise_on_fail=False)
        assert all(r.status == -5 and r.iters == 7 for r in res[0])
        # the capped iterates come back with x_lo folded into x64: the
        # reported residual is the FP64 one of the returned x
        x = xs[0].cpu().numpy()
        for j in range(4):
            r = bs[j] - oracle.apply_A(L, U, mass, x[j])
            rr = np.linalg.norm(r) / np.linalg.norm(bs[j])
            assert abs(res[0][j].true_rel_resid - rr) <= 1e-9 + 1e-6 * rr


def test_launched_rejects_bad_switch(dev, monkeypatch):
    L = (8, 8, 8, 8)
    U = li.links(L, "haar", 6141)
    with P.Lattice(L) as lat:
        Ut = _t(U, dev)
        probs = [(lat, lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), lat.pack_links(Ut, P.LGT_F32, P.LGT_R12),
                  _t(li.vectors(L, 6142, 4), dev))]
        with pytest.raises(P.LgtError) as e:
            _solve(monkeypatch, "yes", probs, 0.1, 1e-10, P.LGT_CG_RELIABLE)
        assert e.value.status == -1


def test_launched_default_at_24x24x24x48_x16(dev):
    """The 16-RHS batch on 24^3 x 48 at m = 0.02 (5.3M site-rhs pairs) takes the
    launched form by default: three right-hand sides checked against the
    oracle's FP64 residual and one against the single-RHS solver."""
    L, n, mass, tol = (24, 24, 24, 48), 16, 0.02, 1e-10
    U = li.links(L, "expih", 6151, c=0.3)
    b = li.vectors(L, 6152, n)
    print("launched 24^3x48 x16", flush=True)
    with P.Lattice(L) as lat:
        Ut = _t(U, dev)
        uh, ul = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), lat.pack_links(Ut, P.LGT_F32, P.LGT_R12)
        del Ut
        lat.set_timing(1)
        xs, res = P.cg_solve_batch([(lat, uh, ul, _t(b, dev))], mass, tol=tol)
        assert _is_launched(lat)
        lat.set_timing(0)
        xb = xs[0].cpu().numpy()
        xj, rj = lat.cg_solve(uh, _t(b[9], dev), mass, tol=tol, scheme=P.LGT_CG_RELIABLE, U_lo=ul)
    assert rj.status == 0
    assert np.linalg.norm(xb[9] - xj.cpu().numpy()) <= 2.1 * tol * np.linalg.norm(b[9]) / (4 * mass * mass)
    assert abs(res[0][9].iters - rj.iters) <= max(12, rj.iters // 10)
    for j in (0, 9, 15):
        _check_solution(L, U, mass, b[j], xb[j], res[0][j], tol)


def _mixed_problems(dev, specs, lo="f32r12", share=False):
    """(L, nrhs, seed) -> problems on their own contexts (or all on the first)."""
    lats, probs, data = [], [], []
    for i, (L, n, seed) in enumerate(specs):
        U = li.links(L, "haar", seed)
        b = li.vectors(L, seed + 1, n)
        lat = P.Lattice(L) if not (share and lats) else lats[0]
        if not (share and lats):
            lats.append(lat)
        Ut = _t(U, dev)
        probs.append((lat, lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), lat.pack_links(Ut, *LO[lo]), _t(b, dev)))
        data.append((L, U, b))
    return lats, probs, data


@pytest.mark.parametrize("scheme,lo", [(P.LGT_CG_RELIABLE, "f32r12"), (P.LGT_CG_REFINE, "bf16r12")],
                         ids=["rel_f32r12", "ir_bf16r12"])
def test_launched_three_lattices(dev, monkeypatch, scheme, lo):
    """8^4, 12^4 and 16^3 x 32 with 4, 8 and 16 right-hand sides on their own
    contexts take the launched form by default (each problem on its own
    stream): every right-hand side against the oracle's residual and within
    the tolerance's bound of the persistent launch's solution."""
    mass, tol = 0.1, 1e-10
    specs = [((8, 8, 8, 8), 4, 6201), ((12, 12, 12, 12), 8, 6211), ((16, 16, 16, 32), 16, 6221)]
    lats, probs, data = _mixed_problems(dev, specs, lo)
    itol = 0.1 if scheme == P.LGT_CG_REFINE else 0.0
    print("launched three lattices", lo, flush=True)
    lats[0].set_timing(1)
    xl, rl = P.cg_solve_batch(probs, mass, tol=tol, scheme=scheme, inner_tol=itol)
    assert _is_launched(lats[0])
    xp, rp = _solve(monkeypatch, "0", probs, mass, tol, scheme, inner_tol=itol)
    assert not _is_launched(lats[0])
    lats[0].set_timing(0)
    for (L, U, b), x1, x2, r1 in zip(data, xl, xp, rl):
        g1, g2 = x1.cpu().numpy(), x2.cpu().numpy()
        for j in range(b.shape[0]):
            _check_solution(L, U, mass, b[j], g1[j], r1[j], tol)
            assert np.linalg.norm(g1[j] - g2[j]) <= 2.1 * tol * np.linalg.norm(b[j]) / (4 * mass * mass)
    for lat in lats:
        lat.close()


def test_launched_problems_sharing_a_context(dev, monkeypatch):
    """Two problems on one context (one stream, the launches of the two
    serialised) and a third on another, forced into the launched form: each
    right-hand side against the oracle's residual; the first problem's
    solutions bit-identical to the same problem solved alone (problems never
    mix)."""
    mass, tol = 0.1, 1e-10
    specs = [((8, 8, 8, 12), 4, 6231), ((8, 8, 8, 12), 8, 6241)]
    lats, probs, data = _mixed_problems(dev, specs, share=True)
    assert probs[0][0] is probs[1][0]
    other = P.Lattice((6, 6, 6, 8))
    U3 = li.links((6, 6, 6, 8), "haar", 6251)
    b3 = li.vectors((6, 6, 6, 8), 6252, 4)
    U3t = _t(U3, dev)
    probs.append((other, other.pack_links(U3t, P.LGT_F64, P.LGT_R18), other.pack_links(U3t, P.LGT_F32, P.LGT_R12),
                  _t(b3, dev)))
    data.append(((6, 6, 6, 8), U3, b3))
    xs, res = _solve(monkeypatch, "1", probs, mass, tol, P.LGT_CG_RELIABLE)
    for (L, U, b), x, rs in zip(data, xs, res):
        g = x.cpu().numpy()
        for j in range(b.shape[0]):
            _check_solution(L, U, mass, b[j], g[j], rs[j], tol)
    x0, r0 = _solve(monkeypatch, "1", probs[:1], mass, tol, P.LGT_CG_RELIABLE)
    assert torch.equal(x0[0], xs[0])
    assert [r.iters for r in r0[0]] == [r.iters for r in res[0]]
    other.close()
    for lat in lats:
        lat.close()


def test_launched_five_problems_forced(dev, monkeypatch):
    """More problems than the automatic rule takes (five, on five contexts)
    run the persistent launch by default and the launched form when forced:
    both within the tolerance by the oracle's residual."""
    mass, tol = 0.1, 1e-10
    specs = [((4, 4, 4, 8), 4, 6261 + 10 * i) for i in range(5)]
    lats, probs, data = _mixed_problems(dev, specs)
    lats[0].set_timing(1)
    for mode, launched in (("1", True), ("0", False)):
        xs, res = _solve(monkeypatch, mode, probs, mass, tol, P.LGT_CG_RELIABLE)
        assert _is_launched(lats[0]) == launched
        for (L, U, b), x, rs in zip(data, xs, res):
            g = x.cpu().numpy()
            for j in range(b.shape[0]):
                _check_solution(L, U, mass, b[j], g[j], rs[j], tol)
    xs, res = P.cg_solve_batch(probs, mass, tol=tol, scheme=P.LGT_CG_RELIABLE)
    assert not _is_launched(lats[0])
    lats[0].set_timing(0)
    for lat in lats:
        lat.close()


def test_launched_graph_replays_match_eager(dev):
    """Without timing each problem's chunk is captured once into a HIP graph and
    replayed every chunk (about 30 replays a solve here); with timing on the
    same launches go out one by one. Both give bit-identical solutions and
    iteration counts, for one problem and for three on their own streams."""
    mass, tol = 0.1, 1e-10
    specs = [((8, 8, 8, 12), 8, 6301), ((6, 6, 6, 8), 4, 6311), ((8, 8, 8, 8), 16, 6321)]
    lats, probs, data = _mixed_problems(dev, specs)
    for sel in (probs[:1], probs):
        lats[0].set_timing(1)
        xe, re_ = P.cg_solve_batch(sel, mass, tol=tol, scheme=P.LGT_CG_RELIABLE)
        assert _is_launched(lats[0])
        lats[0].set_timing(0)
        for rep in range(2):
            xg, rg = P.cg_solve_batch(sel, mass, tol=tol, scheme=P.LGT_CG_RELIABLE)
            for a, b, ra, rb in zip(xe, xg, re_, rg):
                assert torch.equal(a, b)
                assert [r.iters for r in ra] == [r.iters for r in rb]
    for (L, U, b), x, rs in zip(data, xg, rg):
        g = x.cpu().numpy()
        for j in range(b.shape[0]):
            _check_solution(L, U, mass, b[j], g[j], rs[j], tol)
    for lat in lats:
        lat.close()
