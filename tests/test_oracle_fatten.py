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

The chain rule through the fattening (fatten_vjp) is pinned by central
differences of the (already pinned) forward: of a linear functional
sum Re tr(R_F^dag F(U)) + Re tr(R_N^dag N(U)) on general complex links, and of
the composed improved fermion action phi^dag A_imp(F(U), N(U))^-1 phi, whose
derivative runs through the C oracle's improved CG and force first; planted
mistakes in the chain rule must fail the first of these.
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


# ------------------------------------------------------ chain rule (fatten_vjp) ---

def _directional_fd(S, U, E, h):
    return (S(U + h * E) - S(U - h * E)) / (2 * h)


def pin_vjp_linear(fatten_vjp, L=(4, 2, 4, 6), ndir=3):
    """d/dh of sum Re tr(R_F^dag F(U + hE)) + Re tr(R_N^dag N(U + hE)) against
    sum Re tr(G_U^dag E); in the real layout Re tr(A^dag B) is the plain dot."""
    U = _gauss_links(L, 7401 + L[1])
    g = li.rng(7402)
    RF, RN = g.standard_normal(U.shape), g.standard_normal(U.shape)
    GU = fatten_vjp(L, U, W, RF, RN)

    def S(Ux):
        F, N = fat.fatten(L, Ux, W)
        return float(np.sum(RF * F) + np.sum(RN * N))

    for k in range(ndir):
        E = g.standard_normal(U.shape)
        fd = _directional_fd(S, U, E, 1e-5)
        an = float(np.sum(GU * E))
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an)), (L, k, fd, an)


@pytest.mark.parametrize("L", [(4, 2, 4, 6), (2, 4, 2, 4), (4, 4, 4, 4)])
def test_vjp_linear_functional_central_differences(L):
    pin_vjp_linear(fat.fatten_vjp, L)


def test_vjp_one_link_and_naik_alone():
    """only c1: G_U = c1 G_F; only cN: U_mu(z) gets the three positions of the
    three-link product (checked entry by entry against a direct loop)"""
    L = (4, 2, 2, 6)
    U = _gauss_links(L, 7411)
    g = li.rng(7412)
    RF, RN = g.standard_normal(U.shape), g.standard_normal(U.shape)
    np.testing.assert_allclose(fat.fatten_vjp(L, U, (0.7, 0, 0, 0, 0, 0), RF, RN), 0.7 * RF, atol=1e-15)
    GU = hmc.cplx(fat.fatten_vjp(L, U, (0, 0, 0, 0, 0, 1.0), RF, RN))
    Uc, H = hmc.cplx(U), hmc.cplx(RN)
    V = li.volume(L)
    for mu in range(4):
        p1, p2 = hmc.shift(L, mu, 1), hmc.shift(L, mu, 2)
        want = np.zeros((V, 3, 3), complex)
        for x in range(V):
            A, B, C = Uc[mu, x], Uc[mu, p1[x]], Uc[mu, p2[x]]
            want[x] += H[mu, x] @ (B @ C).conj().T
            want[p1[x]] += A.conj().T @ H[mu, x] @ C.conj().T
            want[p2[x]] += (A @ B).conj().T @ H[mu, x]
        np.testing.assert_allclose(GU[mu], want, atol=1e-12)


def test_vjp_composed_improved_action_central_differences():
    """S(U) = phi^dag A_imp^-1 phi with F, N = fatten(U): the gradient from the
    C oracle's improved CG and force, taken back through fatten_vjp, against
    central differences of S (CG to 1e-14)."""
    L, mass, bc = (4, 2, 2, 4), 0.3, (1, 1, 1, -1)
    U = li.links(L, "expih", 7421, c=0.3)
    phi = li.vector(L, 7422)
    w = fat.asqtad_coeffs(0.9)
    S0, GU, _ = hmc.fermion_action_and_G(L, U, mass, phi, 1e-14, bc, w)

    def S(Ux):
        return hmc.fermion_action_and_G(L, Ux, mass, phi, 1e-14, bc, w)[0]

    g = li.rng(7423)
    for k in range(3):
        E = g.standard_normal(U.shape)
        fd = _directional_fd(S, U, E, 1e-5)
        an = float(np.sum(GU * E))
        assert abs(fd - an) <= 1e-7 * abs(an), (k, fd, an)


VJP_MUTANTS = {
    # return leg's gradient without the adjoint of G
    "vjp_return_leg_no_adjoint": ("gC[xm] = dag(G) @ A @ B", "gC[xm] = G @ A @ B"),
    # first leg's gradient with its factors swapped
    "vjp_first_leg_order": ("gA = G @ C @ dag(B)", "gA = G @ dag(B) @ C"),
    # backward link's gradient put at y instead of y - nu
    "vjp_backward_unshifted": ("GU[nu] += dag(y_grad[shift(L, nu, 1)])", "GU[nu] += dag(y_grad)"),
    # inner field's gradient left at x instead of x + a
    "vjp_inner_at_x": ("gM[xa] = dag(A) @ G @ C", "gM[:] = dag(A) @ G @ C"),
    # seven-link gradient not passed on to the five-link fields
    "vjp_seven_not_passed": ("c5 * G + g_two[(a, b)]", "c5 * G"),
    # Lepage term dropped
    "vjp_lepage_dropped": ("one[a], cL * G, GU)", "one[a], 0.0 * G, GU)"),
    # Naik middle link's gradient two sites on
    "vjp_naik_middle_shift": ("gb[x1] = dag(A) @ H @ dag(C)", "gb[x2] = dag(A) @ H @ dag(C)"),
}


def _vjp_mutant(name):
    import types
    src = open(fat.__file__).read()
    old, new = VJP_MUTANTS[name]
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle._fatten_vjp_mutant_" + name)
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), mod.__name__, "exec"), mod.__dict__)
    return mod.fatten_vjp


@pytest.mark.parametrize("name", sorted(VJP_MUTANTS))
def test_vjp_mutants_fail_the_central_difference_pin(name):
    with pytest.raises(AssertionError):
        pin_vjp_linear(_vjp_mutant(name))
