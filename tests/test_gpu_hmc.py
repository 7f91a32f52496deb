"""The HMC step on the GPU against the HMC oracle: gauge force, momentum and
link updates, plaquette and kinetic energy element by element, then whole
leapfrog trajectories (FP64 and mixed-precision CG) and the Metropolis test."""
import numpy as np
import pytest

import lgt_inputs as li
import oracle.hmc as hmc

torch = pytest.importorskip("torch")
P_ = pytest.importorskip("paper_1309_0551_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("L", [(4, 2, 6, 4), (8, 8, 8, 8)])
def test_gauge_force_plaquette_vs_oracle(dev, L):
    beta = 5.7
    U = li.links(L, "haar", 601)
    with P_.Lattice(L) as lat:
        Ut = _t(U, dev)
        G = lat.gauge_force(Ut, beta).cpu().numpy()
        ref = hmc.gauge_force_G(L, U, beta)
        assert np.abs(G - ref).max() <= 1e-13 * np.abs(ref).max()
        # accumulate: G0 + 0.5 G_gauge
        G0 = li.links(L, "haar", 602)
        Ga = lat.gauge_force(Ut, beta, scale=0.5, G=_t(G0, dev), accumulate=True).cpu().numpy()
        np.testing.assert_allclose(Ga, G0 + 0.5 * ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        pl = lat.plaquette(Ut)
        assert pl == pytest.approx(hmc.plaquette_sum(L, U), rel=1e-13)


def test_momentum_link_kinetic_vs_oracle(dev):
    L, eps = (4, 4, 6, 4), 0.03
    U = li.links(L, "haar", 611)
    G = li.links(L, "haar", 612)  # any complex field serves as G here
    Pc = li.momenta(L, 613)
    P = hmc.real(Pc)
    with P_.Lattice(L) as lat:
        Ut, Pt = _t(U, dev), _t(P, dev)
        assert lat.kinetic_energy(Pt) == pytest.approx(hmc.kinetic(Pc), rel=1e-13)
        lat.momentum_update(Ut, _t(G, dev), eps, Pt)
        Pref = Pc + eps * hmc.md_force(U, G)
        np.testing.assert_allclose(Pt.cpu().numpy(), hmc.real(Pref), rtol=0, atol=1e-14)
        lat.link_update(_t(hmc.real(Pref), dev), eps, Ut)
        Uref = hmc.real(hmc.expm_su3(eps * Pref) @ hmc.cplx(U))
        np.testing.assert_allclose(Ut.cpu().numpy(), Uref, rtol=0, atol=2e-14)


def _traj_inputs(L, seed):
    U = li.links(L, "expih", seed, c=0.3)
    Pc = li.momenta(L, seed + 1)
    return U, Pc, li.vector(L, seed + 2), li.vector(L, seed + 3)


@pytest.mark.parametrize("scheme", ["fp64", "reliable_f32r12"])
def test_trajectory_vs_oracle(dev, scheme):
    L, beta, mass, eps, nsteps, tol = (4, 4, 4, 4), 5.5, 0.2, 0.025, 8, 1e-12
    U, Pc, Re, Ro = _traj_inputs(L, 621)
    ref = hmc.trajectory(L, U, Pc, Re, Ro, beta, mass, eps, nsteps, tol=tol)
    sch = P_.LGT_CG_FP64 if scheme == "fp64" else P_.LGT_CG_RELIABLE
    with P_.Lattice(L) as lat:
        Ut, Pt = _t(U, dev), _t(hmc.real(Pc), dev)
        r = lat.hmc_trajectory(Ut, Pt, _t(Re, dev), _t(Ro, dev), beta, mass, eps, nsteps, u=0.0, tol=tol,
                               scheme=sch)
        Ug, Pg = Ut.cpu().numpy(), Pt.cpu().numpy()
    print(f"\nhmc {scheme}: dH gpu {r['dH']:.10f} oracle {ref['dH']:.10f}; H0 {r['H0']:.6f}; "
          f"cg {r['cg_solves']} solves {r['cg_iters']} iters", flush=True)
    assert r["accepted"] == 1  # u = 0 accepts every finite trajectory
    for k in ("H0", "Sg0", "Sf0", "K0", "H1", "Sg1", "Sf1", "K1"):
        assert r[k] == pytest.approx(ref[k], rel=1e-9, abs=1e-9), k
    assert abs(r["dH"] - ref["dH"]) <= 1e-8
    assert np.abs(Ug - ref["U"]).max() <= 1e-10
    assert np.abs(Pg - hmc.real(ref["P"])).max() <= 1e-9
    assert r["cg_solves"] == nsteps + 3


def test_trajectory_rejected_restores_fields(dev):
    L, beta, mass, eps, nsteps = (4, 4, 4, 4), 5.5, 0.2, 0.05, 4
    # coarse steps: the first seed whose oracle trajectory raises H by > 0.05,
    # which u close to 1 must reject
    for seed in range(631, 661, 3):
        U, Pc, Re, Ro = _traj_inputs(L, seed)
        if hmc.trajectory(L, U, Pc, Re, Ro, beta, mass, eps, nsteps)["dH"] > 0.05:
            break
    else:
        pytest.fail("no seed with dH > 0.05")
    P = hmc.real(Pc)
    with P_.Lattice(L) as lat:
        Ut, Pt = _t(U, dev), _t(P, dev)
        r = lat.hmc_trajectory(Ut, Pt, _t(Re, dev), _t(Ro, dev), beta, mass, eps, nsteps, u=1.0 - 1e-12)
        assert r["dH"] > 0.05
        assert r["accepted"] == 0
        np.testing.assert_array_equal(Ut.cpu().numpy(), U)
        np.testing.assert_array_equal(Pt.cpu().numpy(), P)
        with pytest.raises(P_.LgtError):
            lat.hmc_trajectory(Ut, Pt, _t(Re, dev), _t(Ro, dev), beta, mass, 0.05, 4, u=1.5)


def _leapfrog_gauge(lat, U, P, beta, eps, n):
    """Pure-gauge leapfrog from the library's kernels: half momentum steps at
    both ends, U = exp(eps P) U in between."""
    lat.momentum_update(U, lat.gauge_force(U, beta), 0.5 * eps, P)
    for k in range(n):
        lat.link_update(P, eps, U)
        lat.momentum_update(U, lat.gauge_force(U, beta), eps if k < n - 1 else 0.5 * eps, P)


def _h_gauge(lat, U, P, beta, V):
    return lat.kinetic_energy(P) + beta * (6 * V - lat.plaquette(U) / 3.0)


def test_gauge_leapfrog_reversible(dev):
    """Integrate, flip the momenta, integrate again: the GPU kernels bring U
    and -P back to the start (a pin independent of the oracle)."""
    L, beta, eps, n = (4, 4, 4, 6), 5.6, 0.02, 10
    U0 = li.links(L, "expih", 641, c=0.3)
    P0 = hmc.real(li.momenta(L, 642))
    with P_.Lattice(L) as lat:
        U, P = _t(U0, dev), _t(P0, dev)
        _leapfrog_gauge(lat, U, P, beta, eps, n)
        assert np.abs(U.cpu().numpy() - U0).max() > 1e-3  # it did move
        P.neg_()
        _leapfrog_gauge(lat, U, P, beta, eps, n)
        np.testing.assert_allclose(U.cpu().numpy(), U0, rtol=0, atol=1e-11)
        np.testing.assert_allclose(P.cpu().numpy(), -P0, rtol=0, atol=1e-11)


def test_gauge_leapfrog_energy_error_is_second_order(dev):
    """Same trajectory length, half the step: |dH| falls by 4 (leapfrog)."""
    L, beta = (8, 8, 8, 8), 5.6
    U0 = li.links(L, "expih", 651, c=0.3)
    P0 = hmc.real(li.momenta(L, 652))
    V = int(np.prod(L))
    dH = []
    with P_.Lattice(L) as lat:
        for eps, n in ((0.02, 10), (0.01, 20)):
            U, P = _t(U0, dev), _t(P0, dev)
            h0 = _h_gauge(lat, U, P, beta, V)
            _leapfrog_gauge(lat, U, P, beta, eps, n)
            dH.append(_h_gauge(lat, U, P, beta, V) - h0)
    print(f"\npure gauge dH: {dH}", flush=True)
    assert 3.5 <= abs(dH[0] / dH[1]) <= 4.5


def test_trajectory_energy_error_is_second_order(dev):
    """Whole trajectories with the fermion force (FP64 CG): same length, half
    the step, |dH| falls by 4."""
    L, beta, mass = (4, 4, 4, 4), 5.5, 0.2
    U, Pc, Re, Ro = _traj_inputs(L, 661)
    dH = []
    with P_.Lattice(L) as lat:
        for eps, n in ((0.04, 5), (0.02, 10)):
            r = lat.hmc_trajectory(_t(U, dev), _t(hmc.real(Pc), dev), _t(Re, dev), _t(Ro, dev), beta, mass, eps, n,
                                   u=0.0, tol=1e-12)
            dH.append(r["dH"])
    print(f"\nhmc dH: {dH}", flush=True)
    assert 3.5 <= abs(dH[0] / dH[1]) <= 4.5


# ------------------------------------------------ improved operator (fat + Naik) ---

@pytest.mark.parametrize("scheme", ["fp64", "reliable_f32r18"])
def test_improved_trajectory_vs_oracle(dev, scheme):
    """lgt_hmc_trajectory_improved against the oracle's improved trajectory
    (fattening, improved CG and force, chain rule through the fattening)"""
    import oracle.fatten as ofat
    L, beta, mass, eps, nsteps, tol = (4, 4, 4, 4), 5.5, 0.2, 0.025, 8, 1e-12
    w = ofat.asqtad_coeffs(0.9)
    U, Pc, Re, Ro = _traj_inputs(L, 671)
    ref = hmc.trajectory(L, U, Pc, Re, Ro, beta, mass, eps, nsteps, tol=tol, coeffs=w)
    sch = P_.LGT_CG_FP64 if scheme == "fp64" else P_.LGT_CG_RELIABLE
    with P_.Lattice(L) as lat:
        Ut, Pt = _t(U, dev), _t(hmc.real(Pc), dev)
        r = lat.hmc_trajectory_improved(Ut, Pt, _t(Re, dev), _t(Ro, dev), beta, mass, eps, nsteps, u=0.0,
                                        coeffs=w, tol=tol, scheme=sch)
        Ug, Pg = Ut.cpu().numpy(), Pt.cpu().numpy()
    print(f"\nhmc improved {scheme}: dH gpu {r['dH']:.10f} oracle {ref['dH']:.10f}; "
          f"cg {r['cg_solves']} solves {r['cg_iters']} iters", flush=True)
    assert r["accepted"] == 1
    for k in ("H0", "Sg0", "Sf0", "K0", "H1", "Sg1", "Sf1", "K1"):
        assert r[k] == pytest.approx(ref[k], rel=1e-9, abs=1e-9), k
    assert abs(r["dH"] - ref["dH"]) <= 1e-8
    assert np.abs(Ug - ref["U"]).max() <= 1e-10
    assert np.abs(Pg - hmc.real(ref["P"])).max() <= 1e-9
    assert r["cg_solves"] == nsteps + 3


def test_improved_trajectory_energy_error_is_second_order(dev):
    L, beta, mass = (4, 4, 4, 4), 5.5, 0.2
    U, Pc, Re, Ro = _traj_inputs(L, 681)
    w = P_.asqtad_coeffs(0.9)
    dH = []
    with P_.Lattice(L) as lat:
        for eps, n in ((0.04, 5), (0.02, 10)):
            r = lat.hmc_trajectory_improved(_t(U, dev), _t(hmc.real(Pc), dev), _t(Re, dev), _t(Ro, dev), beta,
                                            mass, eps, n, u=0.0, coeffs=w, tol=1e-12)
            dH.append(r["dH"])
        with pytest.raises(P_.LgtError):  # non-finite weights
            lat.hmc_trajectory_improved(_t(U, dev), _t(hmc.real(Pc), dev), _t(Re, dev), _t(Ro, dev), beta,
                                        mass, 0.02, 1, u=0.0, coeffs=(1.0, 0, 0, 0, 0, float("nan")))
    print(f"\nhmc improved dH: {dH}", flush=True)
    assert 3.5 <= abs(dH[0] / dH[1]) <= 4.5
