"""Pins for the FP64 oracle: closed forms, invariants, brute force, library routines.

None of these re-types the oracle's own formula: each checks it against
something the mathematics fixes independently (numpy linear algebra, a
plane-wave eigenvalue, anti-Hermiticity, gauge covariance, a dense matrix
built entry by entry, finite differences).
"""
import itertools
import math
import os

import numpy as np
import pytest

import brute
import lgt_inputs as li
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    vals = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


# ---------------------------------------------------------------- routines ---

def _rc(g, *shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_table1_routines_vs_numpy(seed):
    g = np.random.default_rng(seed)
    A, B = _rc(g, 3, 3), _rc(g, 3, 3)
    a, b = _rc(g, 3), _rc(g, 3)
    A4, b4 = _rc(g, 4, 3, 3), _rc(g, 4, 3)
    s = float(g.standard_normal())
    r = oracle.routine
    np.testing.assert_allclose(r("add_su3_vector", a, b), a + b, rtol=1e-14)
    np.testing.assert_allclose(r("mult_su3_mat_vec", A, b), A @ b, rtol=1e-13)
    np.testing.assert_allclose(r("mult_adj_su3_mat_vec", A, b), A.conj().T @ b, rtol=1e-13)
    np.testing.assert_allclose(r("mult_adj_su3_mat_vec_4dir", a, A4).reshape(4, 3),
                               np.einsum("kji,j->ki", A4.conj(), a), rtol=1e-13)
    outs = r("mult_adj_su3_mat_4vec", A4, a)
    for k in range(4):
        np.testing.assert_allclose(outs[k], A4[k].conj().T @ a, rtol=1e-13)
    np.testing.assert_allclose(r("mult_su3_an", A, B).reshape(3, 3), A.conj().T @ B, rtol=1e-13)
    np.testing.assert_allclose(r("mult_su3_na", A, B).reshape(3, 3), A @ B.conj().T, rtol=1e-13)
    np.testing.assert_allclose(r("mult_su3_nn", A, B).reshape(3, 3), A @ B, rtol=1e-13)
    np.testing.assert_allclose(r("mult_su3_mat_vec_sum_4dir", A4, b4),
                               np.einsum("kij,kj->i", A4, b4), rtol=1e-13)
    np.testing.assert_allclose(r("scalar_mult_add_su3_matrix", A, B, scalar=s).reshape(3, 3),
                               A + s * B, rtol=1e-13)
    np.testing.assert_allclose(r("scalar_mult_add_su3_vector", a, b, scalar=s), a + s * b,
                               rtol=1e-13)
    np.testing.assert_allclose(r("su3_projector", a, b).reshape(3, 3), np.outer(a, b.conj()),
                               rtol=1e-13)
    np.testing.assert_allclose(r("sub_four_su3_vecs", a, b4), a - b4.sum(0), rtol=1e-13)


def test_adjoint_matvec_first_element_matches_eq_1_2():
    """C_0 of the adjoint product with one nonzero term per line of Eqs (1.1)-(2.3)."""
    A = np.zeros((3, 3), complex)
    b = np.zeros(3, complex)
    A[1, 0] = 2.0 + 3.0j  # A_10
    b[1] = 5.0 - 7.0j     # B_1
    c = oracle.routine("mult_adj_su3_mat_vec", A, b)
    # line (1.2): A10.re*B1.re + A10.im*B1.im ; line (2.2): A10.re*B1.im - A10.im*B1.re
    assert c[0] == complex(2 * 5 + 3 * (-7), 2 * (-7) - 3 * 5)
    assert c[1] == 0 and c[2] == 0


def test_flop_constants_golden():
    g = _golden("op_counts.txt")
    assert g["element_mul"] * 3 == g["matvec_mul"]
    assert g["element_add"] * 3 == g["matvec_add"]
    matvec = g["matvec_mul"] + g["matvec_add"]
    assert matvec == 66
    # 8 mat-vecs (4 forward, 4 adjoint backward) and 7 vector adds per site
    assert 8 * matvec + 7 * g["su3_vector_add_flop"] == g["dslash_flop_per_site"] == 570


# ---------------------------------------------------------------- geometry ---

@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 2, 6, 4), (2, 4, 2, 8), (4, 4, 4, 4)])
def test_index_maps_enumeration(L):
    lex_of_eo, nbr = oracle.index_maps(L)
    V = int(np.prod(L))
    Vh = V // 2
    exp_lex = np.empty(V, np.int32)
    exp_nbr = np.empty((2, 8, Vh), np.int32)
    for lex, c in brute.sites(L):
        e = brute.eo_index(L, c)
        exp_lex[e] = lex
        p, cb = divmod(e, Vh)
        for mu in range(4):
            exp_nbr[p, mu, cb] = brute.eo_index(L, brute.shift(L, c, mu, +1)) - (1 - p) * Vh
            exp_nbr[p, 4 + mu, cb] = brute.eo_index(L, brute.shift(L, c, mu, -1)) - (1 - p) * Vh
    np.testing.assert_array_equal(lex_of_eo, exp_lex)
    np.testing.assert_array_equal(nbr, exp_nbr)
    # invariants: bijection per parity; +mu then -mu returns home
    assert sorted(lex_of_eo.tolist()) == list(range(V))
    for p in range(2):
        for mu in range(4):
            back = nbr[1 - p, 4 + mu][nbr[p, mu]]
            np.testing.assert_array_equal(back, np.arange(Vh))


def test_geometry_rejects_odd_and_small():
    assert oracle.geom_ok((4, 4, 4, 4))
    assert not oracle.geom_ok((3, 4, 4, 4))
    assert not oracle.geom_ok((4, 0, 4, 4))
    assert not oracle.geom_ok((4, 4, 4, 4), bc=(1, 1, 1, 2))


# -------------------------------------------------------------- generators ---

def test_haar_is_su3_and_haar_moments():
    U = li.haar_su3(40000, li.rng(7))
    I = np.eye(3)
    err = np.abs(np.einsum("nji,njk->nik", U.conj(), U) - I).max()
    assert err < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
    tr = np.trace(U, axis1=1, axis2=2)
    # Haar on SU(3): E tr U = 0, E |tr U|^2 = 1 (std of the sample mean ~ 0.005)
    assert abs(tr.mean()) < 0.03
    assert abs((np.abs(tr) ** 2).mean() - 1.0) < 0.03


def test_expih_is_su3():
    U = li.expih_su3(2000, 0.5, li.rng(8))
    assert np.abs(np.einsum("nji,njk->nik", U.conj(), U) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13


def test_inputs_deterministic():
    a = li.links((4, 4, 4, 4), "haar", 1001)
    b = li.links((4, 4, 4, 4), "haar", 1001)
    assert li.sha256(a) == li.sha256(b)
    assert a.shape == (4, 256, 3, 3, 2)


# ---------------------------------------------------------------- operator ---

def _plane_wave(L, n, parity=0, colour=None):
    """e^{i p.x} restricted to one parity, p_mu = 2 pi n_mu / L_mu (n may be half-integer)."""
    V = int(np.prod(L))
    Vh = V // 2
    z = np.zeros((Vh, 3), complex)
    col = np.array([1.0, 0.5 - 0.25j, -0.3j]) if colour is None else colour
    for lex, c in brute.sites(L):
        e = brute.eo_index(L, c)
        if e // Vh != parity:
            continue
        ph = sum(2 * math.pi * n[mu] * c[mu] / L[mu] for mu in range(4))
        z[e % Vh] = np.exp(1j * ph) * col
    return li.to_real(z)


@pytest.mark.parametrize("L,n,bc", [
    ((4, 6, 4, 8), (1, 0, 0, 0), (1, 1, 1, 1)),
    ((4, 6, 4, 8), (1, 2, 3, 1), (1, 1, 1, 1)),
    ((6, 4, 4, 4), (0, 1, 1, 2), (1, 1, 1, 1)),
    ((4, 4, 4, 8), (1, 1, 0, 0.5), (1, 1, 1, -1)),   # antiperiodic t: p_t = (2k+1) pi / L_t
    ((4, 4, 4, 8), (0, 0, 1, 2.5), (1, 1, 1, -1)),
])
def test_free_field_plane_wave_eigenvalue(L, n, bc):
    """Unit links: A e^{ipx} = 4 (m^2 + sum_mu sin^2 p_mu) e^{ipx} on even sites."""
    U = li.links(L, "unit")
    m = 0.37
    psi = _plane_wave(L, n)
    Apsi = oracle.apply_A(L, U, m, psi, bc=bc)
    lam = 4 * (m * m + sum(math.sin(2 * math.pi * n[mu] / L[mu]) ** 2 for mu in range(4)))
    np.testing.assert_allclose(Apsi, lam * psi, atol=1e-13)


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, 1, 1, -1), (-1, 1, -1, 1)])
def test_dslash_antihermitian(bc):
    L = (4, 6, 4, 8)
    U = li.links(L, "haar", 11)
    phi_e, psi_o = li.vector(L, 12), li.vector(L, 13)
    # <phi_e, D_eo psi_o> = -<D_oe phi_e, psi_o>
    lhs = oracle.cdot(phi_e, oracle.dslash(L, U, psi_o, 0, bc))
    rhs = -oracle.cdot(oracle.dslash(L, U, phi_e, 1, bc), psi_o)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _gauge_transform(L, U, G):
    """U^G_mu(x) = G(x) U_mu(x) G(x+mu)^dag, all in eo order."""
    Uc = li.to_complex(U)
    out = np.empty_like(Uc)
    for lex, c in brute.sites(L):
        e = brute.eo_index(L, c)
        for mu in range(4):
            f = brute.eo_index(L, brute.shift(L, c, mu, +1))
            out[mu, e] = G[e] @ Uc[mu, e] @ G[f].conj().T
    return li.to_real(out)


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, 1, 1, -1)])
def test_dslash_gauge_covariance(bc):
    L = (4, 4, 6, 4)
    V = int(np.prod(L))
    Vh = V // 2
    U = li.links(L, "haar", 21)
    G = li.haar_su3(V, li.rng(23))
    UG = _gauge_transform(L, U, G)
    for out_par in (0, 1):
        psi = li.vector(L, 22 + out_par)
        psic = li.to_complex(psi)
        Gin = G[(1 - out_par) * Vh:(2 - out_par) * Vh]
        Gout = G[out_par * Vh:(out_par + 1) * Vh]
        lhs = oracle.dslash(L, UG, li.to_real(np.einsum("nij,nj->ni", Gin, psic)), out_par, bc)
        rhs = np.einsum("nij,nj->ni", Gout, li.to_complex(oracle.dslash(L, U, psi, out_par, bc)))
        np.testing.assert_allclose(li.to_complex(lhs), rhs, atol=1e-12)


@pytest.mark.parametrize("L,bc", [((2, 2, 2, 2), (1, 1, 1, 1)), ((2, 4, 2, 6), (1, 1, 1, -1)),
                                  ((4, 4, 4, 4), (1, 1, 1, 1)), ((4, 2, 2, 4), (-1, 1, 1, -1))])
def test_dslash_dense_brute_force(L, bc):
    U = li.links(L, "haar", 31)
    D = brute.dense_D(L, U, bc)
    n = D.shape[0] // 2
    # the dense operator is anti-Hermitian and parity-off-diagonal
    assert np.abs(D + D.conj().T).max() < 1e-14
    assert np.abs(D[:n, :n]).max() == 0 and np.abs(D[n:, n:]).max() == 0
    Deo, Doe = brute.blocks(L, D)
    Vh = int(np.prod(L)) // 2
    chi_o, chi_e = li.vector(L, 32), li.vector(L, 33)
    np.testing.assert_allclose(brute.cvec(oracle.dslash(L, U, chi_o, 0, bc)),
                               Deo @ brute.cvec(chi_o), atol=1e-13)
    np.testing.assert_allclose(brute.cvec(oracle.dslash(L, U, chi_e, 1, bc)),
                               Doe @ brute.cvec(chi_e), atol=1e-13)
    assert Vh * 3 == n


# ---------------------------------------------------------------------- CG ---

@pytest.mark.parametrize("L,mass,kind", [((4, 4, 4, 4), 0.1, "haar"), ((2, 4, 2, 6), 0.05, "expih")])
def test_cg_vs_dense_solve(L, mass, kind):
    U = li.links(L, kind, 41, c=0.3)
    b = li.vector(L, 42)
    tol = 1e-10
    st, x, it, rr = oracle.cg(L, U, mass, b, tol=tol)
    assert st == 0 and rr <= tol
    A = brute.dense_A(L, U, mass)
    xs = np.linalg.solve(A, brute.cvec(b))
    # lambda_min(A) >= 4 m^2  =>  |x - x*| <= |b - A x| / (4 m^2)
    bound = rr * np.linalg.norm(brute.cvec(b)) / (4 * mass * mass)
    assert np.linalg.norm(brute.cvec(x) - xs) <= 1.01 * bound + 1e-12
    assert np.linalg.norm(brute.cvec(x) - xs) <= 1e-6 * np.linalg.norm(xs)


def test_cg_free_field_plane_wave():
    L = (4, 4, 6, 4)
    m = 0.2
    U = li.links(L, "unit")
    n = (1, 1, 2, 0)
    b = _plane_wave(L, n)
    lam = 4 * (m * m + sum(math.sin(2 * math.pi * n[mu] / L[mu]) ** 2 for mu in range(4)))
    st, x, it, rr = oracle.cg(L, U, m, b, tol=1e-12)
    assert st == 0
    assert it <= 2  # b is an eigenvector: one step, plus at most one for rounding
    np.testing.assert_allclose(x, b / lam, atol=1e-12)


def test_cg_zero_source_and_iteration_cap():
    L = (4, 4, 4, 4)
    U = li.links(L, "haar", 51)
    st, x, it, rr = oracle.cg(L, U, 0.1, np.zeros((128, 3, 2)))
    assert st == 0 and it == 0 and not x.any()
    st, x, it, rr = oracle.cg(L, U, 0.1, li.vector(L, 52), max_iter=3)
    assert st == -5 and it == 3


# ------------------------------------------------------------------- force ---

def _S_dense(L, U, mass, phi, bc=(1, 1, 1, 1)):
    A = brute.dense_A(L, U, mass, bc)
    p = brute.cvec(phi)
    return float(np.real(p.conj() @ np.linalg.solve(A, p)))


@pytest.mark.parametrize("L,bc", [((2, 4, 2, 4), (1, 1, 1, 1)), ((4, 2, 2, 4), (1, 1, 1, -1))])
def test_force_vs_dense_central_differences(L, bc):
    mass = 0.3
    U = li.links(L, "expih", 61, c=0.5)
    phi = li.vector(L, 62)
    st, X, it, rr = oracle.cg(L, U, mass, phi, tol=1e-14, bc=bc)
    G = oracle.force(L, U, X, bc)
    g = li.rng(64)
    V = int(np.prod(L))
    eps = 1e-5
    for _ in range(8):
        mu, s = int(g.integers(4)), int(g.integers(V))
        E = g.standard_normal(18)
        E /= np.linalg.norm(E)
        Up, Um = U.copy(), U.copy()
        Up[mu, s] += eps * E.reshape(3, 3, 2)
        Um[mu, s] -= eps * E.reshape(3, 3, 2)
        fd = (_S_dense(L, Up, mass, phi, bc) - _S_dense(L, Um, mass, phi, bc)) / (2 * eps)
        an = float(np.dot(G[mu, s].reshape(-1), E))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (mu, s, fd, an)


@pytest.mark.parametrize("L,bc", [((2, 4, 2, 4), (1, 1, 1, 1)), ((4, 2, 2, 4), (1, 1, 1, -1))])
def test_phi_grad_vs_dense_central_differences(L, bc):
    """dS/dphi from the oracle's X against central differences of the dense S
    along random directions in the source."""
    mass = 0.3
    U = li.links(L, "expih", 65, c=0.5)
    phi = li.vector(L, 66)
    st, X, it, rr = oracle.cg(L, U, mass, phi, tol=1e-14, bc=bc)
    gphi = oracle.action_phi_grad(X)
    g = li.rng(67)
    eps = 1e-5
    for _ in range(6):
        E = g.standard_normal(phi.shape)
        E /= np.linalg.norm(E)
        fd = (_S_dense(L, U, mass, phi + eps * E, bc) - _S_dense(L, U, mass, phi - eps * E, bc)) / (2 * eps)
        an = float(np.sum(gphi * E))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)
    # a planted factor: X alone (without the 2) misses the central difference
    E = g.standard_normal(phi.shape)
    fd = (_S_dense(L, U, mass, phi + eps * E, bc) - _S_dense(L, U, mass, phi - eps * E, bc)) / (2 * eps)
    assert abs(fd - float(np.sum(X * E))) > 1e-3 * abs(fd)


def test_force_vs_oracle_cg_differences():
    """Same check through the oracle's own CG and the variational S estimate."""
    L = (4, 4, 4, 4)
    mass = 0.2
    U = li.links(L, "expih", 71, c=0.5)
    phi = li.vector(L, 72)
    st, X, it, rr = oracle.cg(L, U, mass, phi, tol=1e-14)
    G = oracle.force(L, U, X)
    g = li.rng(74)
    eps = 1e-6
    for _ in range(4):
        mu, s = int(g.integers(4)), int(g.integers(256))
        E = g.standard_normal(18)
        E /= np.linalg.norm(E)
        vals = []
        for sgn in (+1, -1):
            Uq = U.copy()
            Uq[mu, s] += sgn * eps * E.reshape(3, 3, 2)
            _, xq, _, _ = oracle.cg(L, Uq, mass, phi, tol=1e-14)
            vals.append(oracle.action_variational(L, Uq, mass, phi, xq))
        fd = (vals[0] - vals[1]) / (2 * eps)
        an = float(np.dot(G[mu, s].reshape(-1), E))
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (fd, an)


def test_action_gauge_invariant():
    L = (4, 4, 4, 4)
    V, Vh = 256, 128
    mass = 0.2
    U = li.links(L, "haar", 81)
    phi = li.vector(L, 82)
    G = li.haar_su3(V, li.rng(83))
    UG = _gauge_transform(L, U, G)
    phiG = li.to_real(np.einsum("nij,nj->ni", G[:Vh], li.to_complex(phi)))
    _, x1, _, _ = oracle.cg(L, U, mass, phi, tol=1e-13)
    _, x2, _, _ = oracle.cg(L, UG, mass, phiG, tol=1e-13)
    S1 = oracle.cdot(phi, x1).real
    S2 = oracle.cdot(phiG, x2).real
    assert abs(S1 - S2) <= 1e-10 * abs(S1)
