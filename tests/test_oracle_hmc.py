"""Pins for the HMC oracle (oracle/hmc.py): each checks it against something
the mathematics fixes -- finite differences of the action, invariants of the
plaquette, an exponential computed a second way, the momentum distribution,
the leapfrog's O(eps^2) energy error and its reversibility -- and planted
mistakes must fail at least one of them."""
import numpy as np
import pytest

import lgt_inputs as li
import oracle
import oracle.hmc as hmc

L4 = (4, 4, 4, 4)


def test_gauge_force_vs_central_differences():
    L, beta = (4, 2, 4, 6), 5.3
    U = li.links(L, "haar", 501)
    G = hmc.gauge_force_G(L, U, beta)
    g = np.random.default_rng(502)
    for _ in range(6):
        E = g.standard_normal(U.shape)
        h = 1e-5
        fd = (hmc.gauge_action(L, U + h * E, beta) - hmc.gauge_action(L, U - h * E, beta)) / (2 * h)
        an = float(np.sum(G * E))  # sum Re tr(G^dag E) over the real layout
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)


def test_plaquette_unit_links_and_gauge_invariance():
    V = int(np.prod(L4))
    assert hmc.plaquette_sum(L4, li.links(L4, "unit")) == pytest.approx(18 * V, rel=1e-15)
    assert hmc.gauge_action(L4, li.links(L4, "unit"), 5.6) == pytest.approx(0.0, abs=1e-9)
    U = li.links(L4, "haar", 511)
    Gt = li.haar_su3(V, li.rng(512))
    Uc = hmc.cplx(U)
    UG = np.stack([Gt @ Uc[mu] @ hmc.dag(Gt[hmc.shift(L4, mu, 1)]) for mu in range(4)])
    assert hmc.plaquette_sum(L4, hmc.real(UG)) == pytest.approx(hmc.plaquette_sum(L4, U), rel=1e-12)


def test_exponential_second_way_and_su3():
    P = 0.3 * li.momenta((2, 2, 2, 2), 521)
    E = hmc.expm_su3(P)
    # exp(i H) = W exp(i w) W^dag from the eigen-decomposition of H = -i P
    w, W = np.linalg.eigh(-1j * P)
    E2 = W @ (np.exp(1j * w)[..., None] * hmc.dag(W))
    np.testing.assert_allclose(E, E2, atol=1e-13)
    np.testing.assert_allclose(E @ hmc.dag(E), np.broadcast_to(np.eye(3), E.shape), atol=1e-13)
    np.testing.assert_allclose(np.linalg.det(E), 1.0, atol=1e-13)


def test_momenta_are_su3_algebra_with_unit_normal_components():
    P = li.momenta((8, 8, 8, 8), 531)
    assert np.abs(P + hmc.dag(P)).max() == 0.0
    assert np.abs(np.trace(P, axis1=-2, axis2=-1)).max() < 1e-15
    # K = sum_a (p^a)^2 / 2 per link has mean 8 / 2 = 4
    K = -np.trace(P @ P, axis1=-2, axis2=-1).real
    assert abs(K.mean() - 4.0) < 0.1
    assert hmc.kinetic(P) == pytest.approx(K.sum(), rel=1e-12)


def _setup(seed=541):
    L, beta, mass = L4, 5.5, 0.2
    U = li.links(L, "expih", seed, c=0.3)
    P = li.momenta(L, seed + 1)
    Re, Ro = li.vector(L, seed + 2), li.vector(L, seed + 3)
    return L, U, P, Re, Ro, beta, mass


def _dH(eps, nsteps):
    L, U, P, Re, Ro, beta, mass = _setup()
    return hmc.trajectory(L, U, P, Re, Ro, beta, mass, eps, nsteps)["dH"]


def test_leapfrog_energy_error_scales_as_eps_squared():
    # (this field is far from equilibrium, so the forces and dH are large;
    # what matters is that dH vanishes as eps^2)
    tau = 0.2
    d8, d16 = _dH(tau / 8, 8), _dH(tau / 16, 16)
    assert abs(d16) < 0.1
    ratio = d8 / d16
    assert 3.5 < ratio < 4.5, (d8, d16, ratio)


def test_trajectory_reversible():
    L, U, P, Re, Ro, beta, mass = _setup(551)
    fwd = hmc.trajectory(L, U, P, Re, Ro, beta, mass, 0.05, 4)
    back = hmc.trajectory(L, fwd["U"], -fwd["P"], None, None, beta, mass, 0.05, 4, phi=fwd["phi"])
    np.testing.assert_allclose(back["U"], U, atol=1e-10)
    np.testing.assert_allclose(back["P"], -P, atol=1e-9)
    assert back["dH"] == pytest.approx(-fwd["dH"], abs=1e-8)


def test_pseudofermion_heat_bath_covariance():
    """phi = 2m R_e - D_eo R_o has covariance A: for a fixed v,
    E |<v, phi>|^2 = <v, A v> (400 samples, 20 % statistical margin)."""
    L, mass = (4, 2, 2, 4), 0.3
    U = li.links(L, "haar", 561)
    v = li.vector(L, 562)
    vc = li.to_complex(v).reshape(-1)
    Av = li.to_complex(oracle.apply_A(L, U, mass, v)).reshape(-1)
    want = float(np.vdot(vc, Av).real)
    samples = []
    for k in range(400):
        phi = hmc.pseudofermion(L, U, mass, li.vector(L, 10000 + 2 * k), li.vector(L, 10001 + 2 * k))
        samples.append(np.vdot(vc, li.to_complex(phi).reshape(-1)))
    samples = np.array(samples)
    got = float(np.mean(np.abs(samples) ** 2))
    assert abs(got / want - 1.0) < 0.2


MUTANTS = {
    "gauge_force_sign": lambda m: m.setattr(hmc, "gauge_force_G", (lambda f: (lambda L, U, b: -f(L, U, b)))(hmc.gauge_force_G)),
    "md_force_factor": lambda m: m.setattr(hmc, "md_force", (lambda f: (lambda U, G: 2.0 * f(U, G)))(hmc.md_force)),
    "exp_direction": lambda m: m.setattr(hmc, "expm_su3", (lambda f: (lambda A: f(-A)))(hmc.expm_su3)),
    "fermion_force_dropped": lambda m: m.setattr(hmc, "fermion_action_and_G",
                                                 (lambda f: (lambda *a, **k: (lambda r: (r[0], 0 * r[1], r[2]))(f(*a, **k))))(hmc.fermion_action_and_G)),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_energy_pin_catches_mutant(name, monkeypatch):
    MUTANTS[name](monkeypatch)
    with pytest.raises(AssertionError):
        test_leapfrog_energy_error_scales_as_eps_squared()


# ------------------------------------------------ improved operator (fat + Naik) ---

def _dH_imp(eps, nsteps):
    import oracle.fatten as fat
    L, U, P, Re, Ro, beta, mass = _setup()
    return hmc.trajectory(L, U, P, Re, Ro, beta, mass, eps, nsteps, coeffs=fat.asqtad_coeffs(0.9))["dH"]


@pytest.mark.slow
def test_improved_leapfrog_energy_error_scales_as_eps_squared():
    """the improved operator's force (through the fattening's chain rule)
    conserves H to O(eps^2): a wrong force leaves dH of O(eps) or O(1)"""
    tau = 0.2
    d8, d16 = _dH_imp(tau / 8, 8), _dH_imp(tau / 16, 16)
    assert abs(d16) < 0.1
    ratio = d8 / d16
    assert 3.5 < ratio < 4.5, (d8, d16, ratio)


def test_improved_trajectory_reversible():
    import oracle.fatten as fat
    L, beta, mass = (4, 2, 2, 4), 5.5, 0.2
    U, P = li.links(L, "expih", 571, c=0.3), li.momenta(L, 572)
    Re, Ro = li.vector(L, 573), li.vector(L, 574)
    w = fat.asqtad_coeffs(0.9)
    fwd = hmc.trajectory(L, U, P, Re, Ro, beta, mass, 0.05, 3, coeffs=w)
    back = hmc.trajectory(L, fwd["U"], -fwd["P"], None, None, beta, mass, 0.05, 3, phi=fwd["phi"], coeffs=w)
    np.testing.assert_allclose(back["U"], U, atol=1e-10)
    np.testing.assert_allclose(back["P"], -P, atol=1e-9)
    assert back["dH"] == pytest.approx(-fwd["dH"], abs=1e-8)


@pytest.mark.slow
def test_improved_energy_pin_catches_a_chain_rule_that_stops_at_the_fat_field(monkeypatch):
    """G_U = G_F (the fat field taken as the link) must break the eps^2 scaling"""
    import oracle.fatten as fat
    monkeypatch.setattr(fat, "fatten_vjp", lambda L, U, c, GF, GN: GF)
    with pytest.raises(AssertionError):
        test_improved_leapfrog_energy_error_scales_as_eps_squared()
