"""The CG with p = r + beta p formed inside D_oe (p double-buffered, the pending
x += alpha p applied there too) against the CG with a pass of its own: the
same arithmetic in the same order, so bit-identical solutions, iteration and
update counts, for every scheme, the one-link and the improved operator and
each Dslash variant; and against the oracle's residual."""
import numpy as np
import pytest

import lgt_inputs as li
import oracle

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1309_0551_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _both(monkeypatch, fn):
    out = []
    for mode in ("0", "1"):
        monkeypatch.setenv("LGT_CG_FUSED_XPAY", mode)
        out.append(fn())
    monkeypatch.delenv("LGT_CG_FUSED_XPAY")
    return out


SCHEMES = [("fp64", P.LGT_CG_FP64, None, 0.0), ("rel_f32r12", P.LGT_CG_RELIABLE, (P.LGT_F32, P.LGT_R12), 0.0),
           ("ir_bf16r12", P.LGT_CG_REFINE, (P.LGT_BF16, P.LGT_R12), 0.1)]


@pytest.mark.parametrize("name,scheme,lo,itol", SCHEMES, ids=[s[0] for s in SCHEMES])
@pytest.mark.parametrize("hops,streaming", [(1, 1), (2, 1), (4, 0), (8, 1), (8, 0)])
@pytest.mark.parametrize("L", [(8, 8, 8, 8), (6, 4, 6, 8)])
def test_fused_xpay_matches_separate_pass(dev, monkeypatch, name, scheme, lo, itol, hops, streaming, L):
    mass, tol = 0.1, 1e-10
    U = li.links(L, "haar", 7101)
    b = li.vector(L, 7102)
    with P.Lattice(L) as lat:
        Ut = _t(U, dev)
        uh = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18)
        ul = lat.pack_links(Ut, *lo) if lo else None
        lat.set_dslash_variant(P.LGT_F64, P.LGT_R18, hops, streaming)
        if lo:
            lat.set_dslash_variant(*lo, hops, streaming)
        runs = _both(monkeypatch, lambda: lat.cg_solve(uh, _t(b, dev), mass, tol=tol, scheme=scheme, U_lo=ul,
                                                       inner_tol=itol, ru_interval=20))
    (x0, r0), (x1, r1) = runs
    assert torch.equal(x0, x1)
    assert (r0.iters, r0.updates) == (r1.iters, r1.updates)
    res = b - oracle.apply_A(L, U, mass, x1.cpu().numpy())
    assert np.linalg.norm(res) <= 1.05 * tol * np.linalg.norm(b)


@pytest.mark.parametrize("scheme,prec", [(P.LGT_CG_FP64, P.LGT_F64), (P.LGT_CG_RELIABLE, P.LGT_F32)])
def test_fused_xpay_improved_operator(dev, monkeypatch, scheme, prec):
    """The improved operator's CG (16 hops from the fat and Naik fields)."""
    L, mass, tol = (8, 8, 8, 8), 0.1, 1e-10
    U = li.links(L, "haar", 7111)
    b = li.vector(L, 7112)
    with P.Lattice(L) as lat:
        F, N = lat.fatten_links(_t(U, dev), P.asqtad_coeffs(0.9))
        fh, nh = lat.pack_links(F, P.LGT_F64, P.LGT_R18), lat.pack_links(N, P.LGT_F64, P.LGT_R18)
        kw = {}
        if scheme != P.LGT_CG_FP64:
            kw = dict(F_lo=lat.pack_links(F, prec, P.LGT_R18), N_lo=lat.pack_links(N, prec, P.LGT_R18))
        runs = _both(monkeypatch, lambda: lat.cg_solve_improved(fh, nh, _t(b, dev), mass, tol=tol, scheme=scheme,
                                                                **kw))
    (x0, r0), (x1, r1) = runs
    assert torch.equal(x0, x1)
    assert (r0.iters, r0.updates) == (r1.iters, r1.updates)


def test_fused_xpay_iteration_cap_and_guess(dev, monkeypatch):
    """A capped solve (its last update still pending when the cap ends it) and
    a second solve from that iterate as the initial guess."""
    L, mass = (8, 8, 8, 8), 0.1
    U = li.links(L, "haar", 7121)
    b = li.vector(L, 7122)
    with P.Lattice(L) as lat:
        uh = lat.pack_links(_t(U, dev), P.LGT_F64, P.LGT_R18)
        runs = _both(monkeypatch, lambda: lat.cg_solve(uh, _t(b, dev), mass, tol=1e-10, max_iter=13,
                                                       raise_on_fail=False))
        (x0, r0), (x1, r1) = runs
        assert torch.equal(x0, x1) and r0.iters == r1.iters == 13
        rr = np.linalg.norm(b - oracle.apply_A(L, U, mass, x1.cpu().numpy())) / np.linalg.norm(b)
        assert abs(rr - r1.true_rel_resid) <= 1e-9 + 1e-6 * rr
        again = _both(monkeypatch, lambda: lat.cg_solve(uh, _t(b, dev), mass, tol=1e-10, x0=x1.clone()))
    (y0, q0), (y1, q1) = again
    assert torch.equal(y0, y1) and q0.iters == q1.iters
    res = b - oracle.apply_A(L, U, mass, y1.cpu().numpy())
    assert np.linalg.norm(res) <= 1.05e-10 * np.linalg.norm(b)
