"""Pins of the link-fattening oracle (CPU only).

* unit links: F = c1 + 6 c3 + 24 c5 + 48 c7 + 6 cL and N = cN (times 1), with
  generic weights so that a wrong path count shows up;
* constant abelian phases U_nu = exp(i theta_nu): every path from x to x+mu
  carries exp(i theta_mu), so F = (the same sum) exp(i theta_mu) and
  N = cN exp(3 i theta_mu); a leg without its adjoint would leave a transverse
  phase behind;
* gauge covariance: F[U^G](x) = G(x) F[U](x) G(x+mu)^dag and
  N[U^G](x) = G(x) N[U](x) G(x+3mu)^dag;
* brute force: at sampled sites, every path written out as its list of steps
  and multiplied link by link with explicit coordinates (an implementation
  that shares nothing with the oracle's whole-lattice staples), on lattices
  with extent 2 (where x + a and x - a coincide) and non-cubic shapes;
* tree-level asqtad weights give the free improved operator, F = 9/8 and
  N = -1/24.
"""
import numpy as np
import pytest

import brute
import lgt_inputs as li
import oracle.fatten as fat
import oracle.hmc as hmc

W = (0.37, -0.11, 0.023, -0.0071, 0.052, -0.29)  # generic weights (c1, c3, c5, c7, cL, cN)


def _unit(L):
    return li.links(L, "unit", 0)


def _gauss_links(L, seed):
    """general complex 3x3 links (the definition does not need SU(3))"""
    g = li.rng(seed)
    V = li.volume(L)
    return g.standard_normal((4, V, 3, 3, 2)) * 0.5


def pin_unit(fatten):
    L = (4, 4, 2, 6)
    F, N = fatten(L, _unit(L), W)
    c1, c3, c5, c7, cL, cN = W
    want = c1 + 6 * c3 + 24 * c5 + 48 * c7 + 6 * cL
    Fc, Nc = hmc.cplx(F), hmc.cplx(N)
    np.testing.assert_allclose(Fc, want * np.broadcast_to(np.eye(3), Fc.shape), atol=1e-15)
    np.testing.assert_allclose(Nc, cN * np.broadcast_to(np.eye(3), Nc.shape), atol=1e-15)


def test_unit_links_count_every_path():
    pin_unit(fat.fatten)


def test_asqtad_weights_give_the_free_improved_operator():
    L = (4, 4, 4, 4)
    F, N = fat.fatten(L, _unit(L), fat.asqtad_coeffs())
    assert np.abs(hmc.cplx(F)[:, :, 0, 0] - 9.0 / 8.0).max() < 1e-15
    assert np.abs(hmc.cplx(N)[:, :, 0, 0] + 1.0 / 24.0).max() < 1e-15
    # tadpole factors: a path of n links is divided by u0^(n-1)
    c = fat.asqtad_coeffs(0.9)
    assert c[1] == pytest.approx(fat.ASQTAD[1] / 0.81) and c[3] == pytest.approx(fat.ASQTAD[3] / 0.9 ** 6)


def pin_abelian(fatten):
    L = (4, 2, 4, 4)
    V = li.volume(L)
    th = np.array([0.3, -0.7, 1.1, 0.45])
    Uc = np.zeros((4, V, 3, 3), complex)
    for mu in range(4):
        Uc[mu] = np.exp(1j * th[mu]) * np.eye(3)
    F, N = fatten(L, hmc.real(Uc), W)
    c1, c3, c5, c7, cL, cN = W
    s = c1 + 6 * c3 + 24 * c5 + 48 * c7 + 6 * cL
    for mu in range(4):
        np.testing.assert_allclose(hmc.cplx(F)[mu], s * Uc[mu], atol=1e-14)
        np.testing.assert_allclose(hmc.cplx(N)[mu], cN * np.exp(3j * th[mu]) * np.broadcast_to(np.eye(3), (V, 3, 3)),
                                   atol=1e-14)


def test_constant_abelian_phases():
    pin_abelian(fat.fatten)


def pin_covariance(fatten):
    L = (4, 4, 4, 6)
    V = li.volume(L)
    U = li.links(L, "haar", 7101)
    G = li.haar_su3(V, li.rng(7102))
    Uc = hmc.cplx(U)
    Ug = np.empty_like(Uc)
    for mu in range(4):
        Ug[mu] = G @ Uc[mu] @ hmc.dag(G[hmc.shift(L, mu, 1)])
    F, N = fatten(L, U, W)
    Fg, Ng = fatten(L, hmc.real(Ug), W)
    for mu in range(4):
        np.testing.assert_allclose(hmc.cplx(Fg)[mu], G @ hmc.cplx(F)[mu] @ hmc.dag(G[hmc.shift(L, mu, 1)]),
                                   atol=1e-13)
        np.testing.assert_allclose(hmc.cplx(Ng)[mu], G @ hmc.cplx(N)[mu] @ hmc.dag(G[hmc.shift(L, mu, 3)]),
                                   atol=1e-13)


def test_gauge_covariance():
    pin_covariance(fat.fatten)


# ---------------------------------------------------------------- brute force ---

def pin_brute(fatten, L):
    U = _gauss_links(L, 7201 + L[0])
    Uc = hmc.cplx(U)
    F, N = fatten(L, U, W)
    Fc, Nc = hmc.cplx(F), hmc.cplx(N)
    V = li.volume(L)
    g = li.rng(7301)
    for eo in g.integers(0, V, 5):
        x = brute.coords_of_eo(L, int(eo))
        for mu in range(4):
            Fb, Nb = brute.fat_link(L, Uc, x, mu, W)
            scale = np.abs(Fb).max()
            assert np.abs(Fc[mu, eo] - Fb).max() <= 1e-13 * scale, (L, eo, mu)
            assert np.abs(Nc[mu, eo] - Nb).max() <= 1e-13 * np.abs(Nb).max(), (L, eo, mu)


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 4, 2, 6), (6, 2, 4, 4)])
def test_brute_force_paths(L):
    pin_brute(fat.fatten, L)


# ------------------------------------------------------------------- mutants ---

MUTANTS = {
    # return leg without its adjoint
    "return_no_adjoint": ("@ dag(La[shift(L, mu, 1)])", "@ La[shift(L, mu, 1)]"),
    # return leg taken at x instead of x + mu
    "return_at_x": ("@ dag(La[shift(L, mu, 1)])", "@ dag(La)"),
    # backward step uses the link at y instead of y - nu
    "backward_unshifted": ("return dag(Uc[nu][shift(L, nu, -1)])", "return dag(Uc[nu])"),
    # legs multiplied in the wrong order
    "leg_order": ("return La @ M[shift(L, a[0], a[1])] @", "return M[shift(L, a[0], a[1])] @ La @"),
    # Lepage term dropped
    "lepage_dropped": ("+ cL * sum(lepage))", ")"),
    # seven-link paths allowed to reuse an axis
    "seven_axis_reuse": ("if len({a[0], b[0], c[0]}) == 3]", "if a[0] != b[0] and b[0] != c[0]]"),
    # Naik field two links long
    "naik_short": ("Uc[mu][shift(L, mu, 2)])", "Uc[mu][shift(L, mu, 1)])"),
    # five-link paths that go out and straight back along one axis
    "five_axis_reuse": ("for b in dirs if a[0] != b[0]}", "for b in dirs if a != b}"),
}


def _mutant(name):
    import types
    src = open(fat.__file__).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle._fatten_mutant_" + name)
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), mod.__name__, "exec"), mod.__dict__)
    return mod.fatten


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutants_fail_a_pin(name):
    f = _mutant(name)
    caught = []
    for pin in (pin_unit, pin_abelian, pin_covariance, lambda g: pin_brute(g, (2, 4, 2, 6))):
        try:
            pin(f)
        except AssertionError:
            caught.append(pin)
    assert caught, name
