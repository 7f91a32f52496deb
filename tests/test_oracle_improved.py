"""Pins for the oracle's improved (fat one-link + Naik three-link) operator.

Each pin checks it against something fixed independently of its code: the
one-link oracle (already pinned) when the Naik field vanishes, anti-Hermiticity,
a closed-form plane-wave eigenvalue for constant links, gauge covariance
(three-link fields transform like three-step paths), a dense matrix built
entry by entry in Python with its own step-by-step boundary counting, and a
dense solve for the CG.
"""
import math

import numpy as np
import pytest

import brute
import lgt_inputs as li
import oracle

C1, C3 = 9.0 / 8.0, -1.0 / 24.0


def test_improved_reduces_to_one_link_when_naik_vanishes():
    L = (4, 6, 4, 8)
    F, N = li.improved_links(L, 301)
    for par in (0, 1):
        chi = li.vector(L, 302 + par)
        a = oracle.dslash_imp(L, F, np.zeros_like(N), chi, par, (1, 1, 1, -1))
        b = oracle.dslash(L, F, chi, par, (1, 1, 1, -1))
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("L,bc", [((4, 6, 4, 8), (1, 1, 1, 1)), ((8, 4, 6, 4), (1, 1, 1, -1)),
                                  ((2, 4, 2, 6), (-1, 1, 1, -1))])
def test_improved_antihermitian(L, bc):
    F, N = li.improved_links(L, 311)
    phi_e, psi_o = li.vector(L, 312), li.vector(L, 313)
    # <phi_e, D_eo psi_o> = -<D_oe phi_e, psi_o>
    lhs = oracle.cdot(phi_e, oracle.dslash_imp(L, F, N, psi_o, 0, bc))
    rhs = -oracle.cdot(oracle.dslash_imp(L, F, N, phi_e, 1, bc), psi_o)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _plane_wave(L, n):
    Vh = int(np.prod(L)) // 2
    z = np.zeros((Vh, 3), complex)
    col = np.array([0.3 - 1j, 1.0, 0.25j])
    for _, c in brute.sites(L):
        e = brute.eo_index(L, c)
        if e < Vh:
            z[e] = np.exp(1j * sum(2 * math.pi * n[mu] * c[mu] / L[mu] for mu in range(4))) * col
    return li.to_real(z)


@pytest.mark.parametrize("L,n,bc", [
    ((8, 6, 8, 8), (1, 2, 3, 1), (1, 1, 1, 1)),
    ((8, 8, 4, 10), (3, 1, 1, 2), (1, 1, 1, 1)),
    ((8, 8, 8, 8), (1, 2, 0, 1.5), (1, 1, 1, -1)),  # antiperiodic t: p_t = (2k + 1) pi / L_t
    ((6, 4, 4, 8), (1, 1, 1, 3.5), (1, 1, 1, -1)),
])
def test_improved_free_field_plane_wave(L, n, bc):
    """F = c1 1, N = c3 1: D acts on e^{ipx} with symbol 2i (c1 sin p + c3 sin 3p)
    per direction and the phases make the directions anticommute, so
    A e^{ipx} = 4 (m^2 + sum_mu (c1 sin p_mu + c3 sin 3 p_mu)^2) e^{ipx}."""
    U1 = li.links(L, "unit")
    F, N = C1 * U1, C3 * U1
    m = 0.29
    psi = _plane_wave(L, n)
    Apsi = oracle.apply_A_imp(L, F, N, m, psi, bc=bc)
    p = [2 * math.pi * n[mu] / L[mu] for mu in range(4)]
    lam = 4 * (m * m + sum((C1 * math.sin(q) + C3 * math.sin(3 * q)) ** 2 for q in p))
    np.testing.assert_allclose(Apsi, lam * psi, atol=1e-13)


def _transform(L, W, G, steps):
    """W^G_mu(x) = G(x) W_mu(x) G(x + steps mu)^dag."""
    Wc = li.to_complex(W)
    out = np.empty_like(Wc)
    for _, c in brute.sites(L):
        e = brute.eo_index(L, c)
        for mu in range(4):
            f = brute.eo_index(L, brute.shift(L, c, mu, steps))
            out[mu, e] = G[e] @ Wc[mu, e] @ G[f].conj().T
    return li.to_real(out)


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, -1, 1, -1)])
def test_improved_gauge_covariance(bc):
    L = (8, 4, 6, 8)
    V = int(np.prod(L))
    Vh = V // 2
    F, N = li.improved_links(L, 321)
    G = li.haar_su3(V, li.rng(322))
    FG, NG = _transform(L, F, G, 1), _transform(L, N, G, 3)
    for out_par in (0, 1):
        psi = li.vector(L, 323 + out_par)
        psic = li.to_complex(psi)
        Gin = G[(1 - out_par) * Vh:(2 - out_par) * Vh]
        Gout = G[out_par * Vh:(out_par + 1) * Vh]
        lhs = oracle.dslash_imp(L, FG, NG, li.to_real(np.einsum("nij,nj->ni", Gin, psic)), out_par, bc)
        rhs = np.einsum("nij,nj->ni", Gout, li.to_complex(oracle.dslash_imp(L, F, N, psi, out_par, bc)))
        np.testing.assert_allclose(li.to_complex(lhs), rhs, atol=1e-12)


@pytest.mark.parametrize("L,bc", [((2, 4, 2, 6), (1, 1, 1, -1)),   # extents 2, 4, 6: hops coincide
                                  ((4, 2, 6, 4), (-1, 1, -1, 1)),
                                  ((8, 4, 2, 8), (1, 1, 1, -1))])
def test_improved_dense_brute_force(L, bc):
    F, N = li.improved_links(L, 331)
    D = brute.dense_D_imp(L, F, N, bc)
    n = D.shape[0] // 2
    assert np.abs(D + D.conj().T).max() < 1e-14
    assert np.abs(D[:n, :n]).max() == 0 and np.abs(D[n:, n:]).max() == 0
    Deo, Doe = brute.blocks(L, D)
    chi_o, chi_e = li.vector(L, 332), li.vector(L, 333)
    np.testing.assert_allclose(brute.cvec(oracle.dslash_imp(L, F, N, chi_o, 0, bc)),
                               Deo @ brute.cvec(chi_o), atol=1e-13)
    np.testing.assert_allclose(brute.cvec(oracle.dslash_imp(L, F, N, chi_e, 1, bc)),
                               Doe @ brute.cvec(chi_e), atol=1e-13)


def test_improved_cg_vs_dense_solve():
    L, mass, tol = (4, 2, 6, 4), 0.07, 1e-10
    F, N = li.improved_links(L, 341)
    b = li.vector(L, 342)
    st, x, it, rr = oracle.cg_imp(L, F, N, mass, b, tol=tol)
    assert st == 0 and rr <= tol
    xs = np.linalg.solve(brute.dense_A_imp(L, F, N, mass), brute.cvec(b))
    bound = rr * np.linalg.norm(brute.cvec(b)) / (4 * mass * mass)
    assert np.linalg.norm(brute.cvec(x) - xs) <= 1.01 * bound + 1e-12


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, 1, 1, -1)])
def test_improved_force_central_differences(bc):
    """dS/dF and dS/dN of S = Re phi^dag A^-1 phi (improved operator) from
    or_force_imp against central differences of S computed by a dense solve of
    the brute-force matrix, along random directions in F only and in N only.
    Extent 8 in t keeps the Naik hops apart from the one-link hops there."""
    L, mass, h = (4, 2, 2, 8), 0.1, 1e-5
    F, N = li.improved_links(L, 471)
    phi = brute.cvec(li.vector(L, 472))
    Vh = int(np.prod(L)) // 2

    def S(Fx, Nx):
        return float(np.vdot(phi, np.linalg.solve(brute.dense_A_imp(L, Fx, Nx, mass, bc), phi)).real)

    X = brute.rvec(np.linalg.solve(brute.dense_A_imp(L, F, N, mass, bc), phi), Vh)
    GF, GN = oracle.force_imp(L, F, N, X, bc)
    rng = np.random.default_rng(473)
    for which in ("F", "N"):
        for _ in range(3):
            E = rng.standard_normal(F.shape)
            if which == "F":
                fd = (S(F + h * E, N) - S(F - h * E, N)) / (2 * h)
                an = float(np.sum(GF * E))
            else:
                fd = (S(F, N + h * E) - S(F, N - h * E)) / (2 * h)
                an = float(np.sum(GN * E))
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, fd, an)


def test_improved_force_reduces_to_one_link_force():
    """With the Naik field zero the fat-link derivative is the one-link force."""
    L = (4, 4, 6, 4)
    F, N = li.improved_links(L, 481)
    X = li.vector(L, 482)
    GF, GN = oracle.force_imp(L, F, np.zeros_like(N), X)
    np.testing.assert_allclose(GF, oracle.force(L, F, X), rtol=0, atol=1e-13 * np.abs(GF).max())
