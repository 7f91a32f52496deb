"""Full-size workloads in the launch configuration the benchmark times, checked
against the FP64 oracle.

* 16^4, links exp(0.3 i H), m = 0.05: the FP64 GPU CG against the oracle's own
  CG (solution, residual, iteration count).
* 32^4, Haar links, m = 0.01: FP64, FP32x12 reliable-update and BF16x12
  refinement solves. The oracle recomputes every true residual |b - A x|/|b|
  in FP64; since lambda_min(A) >= 4 m^2, |x - x*| <= |b - A x| / (4 m^2) bounds
  the error against the exact solution. (An oracle solve at this size takes
  minutes on the host, so the solution itself is checked through that bound.)
* 24^3x48 with 16 right-hand sides and the 8^4 / 12^4 / 16^3x32 batch with 4
  each (m = 0.02, FP32x12 + FP64 reliable updates): the oracle's true residual
  of every right-hand side.

Each test prints the error it measured against the oracle.
"""
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


def _oracle_resid(L, U, mass, b, x):
    r = b - oracle.apply_A(L, U, mass, x)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def test_cg_smooth_16x16x16x16_vs_oracle_solve(dev):
    c = li.CONFIGS["c2_16x16x16x16"]
    L, mass, tol = c["L"], c["mass"], c["tol"]
    U = li.links(L, c["kind"], c["link_seed"], c["c"])
    b = li.vector(L, c["src_seed"])
    st, xo, it_o, rr_o = oracle.cg(L, U, mass, b, tol=tol)
    assert st == 0
    with P.Lattice(L) as lat:
        x, res = lat.cg_solve(lat.pack_links(_t(U, dev)), _t(b, dev), mass, tol=tol)
    xg = x.cpu().numpy()
    rr = _oracle_resid(L, U, mass, b, xg)
    err = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
    print(f"\n16^4 FP64 CG: iters gpu {res.iters} oracle {it_o}; oracle-recomputed resid {rr:.3e}; "
          f"|x - x_oracle|/|x_oracle| {err:.3e}", flush=True)
    assert res.status == 0 and rr <= 1.05 * tol
    assert abs(res.iters - it_o) <= 3
    bound = (1.05 * tol + rr_o) * np.linalg.norm(b) / (4 * mass * mass)
    assert np.linalg.norm(xg - xo) <= bound


def test_cg_32x32x32x32_all_schemes(dev):
    c = li.CONFIGS["c3_32x32x32x32"]
    L, mass, tol = c["L"], c["mass"], c["tol"]
    U = li.links(L, c["kind"], c["link_seed"])
    b = li.vector(L, c["src_seed"])
    bn = float(np.linalg.norm(b))
    xs = {}
    with P.Lattice(L) as lat:
        Ut = _t(U, dev)
        Uh = lat.pack_links(Ut, P.LGT_F64, P.LGT_R18)
        lo32 = lat.pack_links(Ut, P.LGT_F32, P.LGT_R12)
        lo16 = lat.pack_links(Ut, P.LGT_BF16, P.LGT_R12)
        del Ut
        bt = _t(b, dev)
        runs = {"fp64": dict(scheme=P.LGT_CG_FP64),
                "f32r12_reliable": dict(scheme=P.LGT_CG_RELIABLE, U_lo=lo32, ru_interval=50),
                "bf16r12_refine": dict(scheme=P.LGT_CG_REFINE, U_lo=lo16, inner_tol=0.1)}
        for name, kw in runs.items():
            x, res = lat.cg_solve(Uh, bt, mass, tol=tol, **kw)
            xg = x.cpu().numpy()
            rr = _oracle_resid(L, U, mass, b, xg)
            # |x - x*| <= |b - A x| / lambda_min(A), lambda_min(A) >= 4 m^2
            bound = rr * bn / (4 * mass * mass) / float(np.linalg.norm(xg))
            print(f"\n32^4 {name}: iters {res.iters} updates {res.updates} dslash {res.dslash_calls}; "
                  f"oracle-recomputed resid {rr:.3e} (gpu {res.true_rel_resid:.3e}); "
                  f"|x - x*|/|x| <= {bound:.3e}", flush=True)
            assert res.status == 0
            assert rr <= 1.05 * tol
            assert abs(res.true_rel_resid - rr) <= 1e-3 * tol + 0.05 * rr
            xs[name] = xg
    for name in ("f32r12_reliable", "bf16r12_refine"):
        d = float(np.linalg.norm(xs[name] - xs["fp64"]) / np.linalg.norm(xs["fp64"]))
        print(f"32^4 |x_{name} - x_fp64|/|x_fp64| = {d:.3e}", flush=True)
        # both within the residual bound of the exact solution
        assert d <= 2 * 1.05 * tol * bn / (4 * mass * mass) / float(np.linalg.norm(xs["fp64"]))


def _batch_problem(Lb, link_seed, src_seed, nrhs, dev):
    lat = P.Lattice(Lb)
    U = li.links(Lb, "haar", link_seed)
    bs = li.vectors(Lb, src_seed, nrhs)
    Ut = _t(U, dev)
    prob = (lat, lat.pack_links(Ut, P.LGT_F64, P.LGT_R18), lat.pack_links(Ut, P.LGT_F32, P.LGT_R12), _t(bs, dev))
    return prob, U, bs


@pytest.mark.parametrize("which", ["24x24x24x48_x16", "mixed_x4"])
def test_batch_full_size_vs_oracle(dev, which):
    c4, c4m = li.CONFIGS["c4_24x24x24x48"], li.CONFIGS["c4_mixed"]
    if which == "24x24x24x48_x16":
        members = [(c4["L"], c4["link_seed"], c4["src_seed"], c4["nrhs"])]
    else:
        members = [(Lm, sd, sd + c4m["src_seed_offset"], c4m["nrhs"]) for Lm, sd in c4m["members"]]
    built = [_batch_problem(*m, dev) for m in members]
    try:
        xs, res = P.cg_solve_batch([p for p, _, _ in built], c4["mass"], tol=c4["tol"],
                                   scheme=P.LGT_CG_RELIABLE, ru_interval=50)
        worst = 0.0
        for (prob, U, bs), x, rs in zip(built, xs, res):
            L = prob[0].L
            xg = x.cpu().numpy()
            for j in range(bs.shape[0]):
                rr = _oracle_resid(L, U, c4["mass"], bs[j], xg[j])
                worst = max(worst, rr)
                assert rs[j].status == 0
                assert rr <= 1.05 * c4["tol"], (L, j, rr)
                assert abs(rs[j].true_rel_resid - rr) <= 1e-3 * c4["tol"] + 0.05 * rr
        print(f"\nbatch {which}: {sum(len(r) for r in res)} right-hand sides, iterations "
              f"{max(r.iters for rr_ in res for r in rr_)}, worst oracle-recomputed resid {worst:.3e}", flush=True)
    finally:
        for prob, _, _ in built:
            prob[0].close()
