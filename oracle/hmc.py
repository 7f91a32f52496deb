"""Oracle for the HMC step around the solve (test infrastructure only: only
tests/ and the benchmark's CPU baseline may use it).

Plain FP64 numpy on top of the C oracle's Dslash, CG and fermion force. The
paper's application (Table 4) runs hybrid Monte Carlo with improved staggered
quarks; its gauge part uses the Table 1 matrix products (mult_su3_an / _na /
_nn) for staples and scalar_mult_add_su3_matrix for the momentum and link
updates. The paper does not write these steps out; the reading used here is
the textbook one:

* Wilson gauge action S_g = beta sum_{x, mu<nu} (1 - Re tr U_mu,nu(x) / 3) with
  U_mu,nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag.
* Staple sum Sigma_mu(x) = sum_{nu != mu} [ U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
  + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) ], so that the plaquettes holding
  U_mu(x) sum to Re tr(U_mu(x) Sigma_mu(x)).
* Derivatives in the fermion force's convention dS = sum Re tr(G^dag dU):
  G_gauge = -(beta / 3) Sigma^dag.
* Molecular dynamics: dU/dt = P U with P traceless anti-Hermitian, kinetic
  energy K = -sum tr(P^2) (= sum (p^a)^2 / 2 for P = i p^a lambda^a / 2); H = K + S
  is conserved when dP/dt = TA(U G^dag) / 2, TA = traceless anti-Hermitian part.
* Leapfrog: P += (eps/2) F; then (U = exp(eps P) U; P += eps F) with the last
  momentum step halved; F = TA(U G^dag) / 2 with G = G_gauge + G_fermion.
* Pseudofermion (heat bath): phi_e = (M^dag R)_e = 2m R_e - D_eo R_o for Gaussian
  R on all sites, so phi_e is distributed as exp(-phi^dag A^-1 phi).
* S_f = Re <phi, X>, X = A^-1 phi by CG; its G from the fermion-force oracle.
* Metropolis: accept when u < exp(-dH) for a uniform u given as input.
* Improved operator (the application's action, Table 4): with fattening
  weights given, the Dslash takes the fat and Naik fields F(U), N(U) of the
  fattening oracle. phi_e = 2m R_e - D^imp_eo R_o, S_f = Re <phi, X> with
  X = A_imp^-1 phi, and G_fermion = the fermion-force oracle's derivatives with
  respect to F and N taken back to U by the chain rule through the fattening.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import cg as _cg
from . import cg_imp as _cg_imp
from . import dslash as _dslash
from . import dslash_imp as _dslash_imp
from . import force as _force
from . import force_imp as _force_imp

_SHIFT_CACHE: dict = {}


def _coords(L):
    """eo-ordered coordinates [V][4] (lex = x + Lx (y + Ly (z + Lz t)))."""
    V = int(np.prod(L))
    lex = np.arange(V)
    c = np.stack([lex % L[0], (lex // L[0]) % L[1], (lex // (L[0] * L[1])) % L[2], lex // (L[0] * L[1] * L[2])], 1)
    par = c.sum(1) % 2
    eo = par * (V // 2) + lex // 2
    out = np.empty_like(c)
    out[eo] = c
    return out


def shift(L, mu, d):
    """eo index of x + d mu for every eo site x (periodic)."""
    key = (tuple(L), mu, d)
    if key not in _SHIFT_CACHE:
        c = _coords(L).copy()
        c[:, mu] = (c[:, mu] + d) % L[mu]
        lex = c[:, 0] + L[0] * (c[:, 1] + L[1] * (c[:, 2] + L[2] * c[:, 3]))
        par = c.sum(1) % 2
        V = int(np.prod(L))
        _SHIFT_CACHE[key] = par * (V // 2) + lex // 2
    return _SHIFT_CACHE[key]


def cplx(U):
    """canonical real [4][V][3][3][2] -> complex [4][V][3][3]."""
    return U[..., 0] + 1j * U[..., 1]


def real(Uc):
    return np.ascontiguousarray(np.stack([Uc.real, Uc.imag], -1))


def dag(X):
    return np.conj(np.swapaxes(X, -1, -2))


def plaquette_sum(L, U):
    """sum over x and mu < nu of Re tr U_mu,nu(x)."""
    Uc = cplx(U)
    s = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = Uc[mu] @ Uc[nu][shift(L, mu, 1)] @ dag(Uc[mu][shift(L, nu, 1)]) @ dag(Uc[nu])
            s += float(np.trace(P, axis1=1, axis2=2).real.sum())
    return s


def gauge_action(L, U, beta):
    V = int(np.prod(L))
    return beta * (6 * V - plaquette_sum(L, U) / 3.0)


def staples(L, U):
    """Sigma_mu(x), complex [4][V][3][3]."""
    Uc = cplx(U)
    S = np.zeros_like(Uc)
    for mu in range(4):
        for nu in range(4):
            if nu == mu:
                continue
            up = Uc[nu][shift(L, mu, 1)] @ dag(Uc[mu][shift(L, nu, 1)]) @ dag(Uc[nu])
            xmn = shift(L, nu, -1)
            dn = dag(Uc[nu][shift(L, mu, 1)][xmn]) @ dag(Uc[mu][xmn]) @ Uc[nu][xmn]
            S[mu] += up + dn
    return S


def gauge_force_G(L, U, beta):
    """G of S_g: dS_g = sum Re tr(G^dag dU); real canonical layout."""
    return real(-(beta / 3.0) * dag(staples(L, U)))


def ta(X):
    """traceless anti-Hermitian part (X - X^dag)/2 - tr(X - X^dag)/6."""
    A = 0.5 * (X - dag(X))
    tr = np.trace(A, axis1=-2, axis2=-1)
    return A - (tr / 3.0)[..., None, None] * np.eye(3)


def md_force(U, G):
    """dP/dt = TA(U G^dag) / 2 (complex [4][V][3][3])."""
    return 0.5 * ta(cplx(U) @ dag(cplx(G)))


def kinetic(P):
    """K = -sum tr(P^2) for complex anti-Hermitian P."""
    return float(-np.trace(P @ P, axis1=-2, axis2=-1).real.sum())


def expm_su3(A):
    """exp of each 3x3 matrix of A (library routine)."""
    flat = A.reshape(-1, 3, 3)
    return np.stack([scipy.linalg.expm(m) for m in flat]).reshape(A.shape)


def pseudofermion(L, U, mass, R_e, R_o, bc=None, coeffs=None):
    """phi_e = 2m R_e - D_eo R_o (the improved D_eo of F(U), N(U) with coeffs)."""
    if coeffs is None:
        return 2.0 * mass * R_e - _dslash(L, U, R_o, 0, bc)
    from .fatten import fatten
    F, N = fatten(L, U, coeffs)
    return 2.0 * mass * R_e - _dslash_imp(L, F, N, R_o, 0, bc)


def fermion_action_and_G(L, U, mass, phi, tol, bc=None, coeffs=None):
    """(S_f, G_fermion, CG iterations) at links U; with coeffs the improved
    operator of the fattened fields, G taken back to U through the fattening."""
    if coeffs is None:
        st, X, it, rr = _cg(L, U, mass, phi, tol=tol, bc=bc)
    else:
        from .fatten import fatten, fatten_vjp
        F, N = fatten(L, U, coeffs)
        st, X, it, rr = _cg_imp(L, F, N, mass, phi, tol=tol, bc=bc)
    if st != 0:
        raise RuntimeError(f"oracle CG failed ({st})")
    S = float(np.sum(phi * X))  # Re <phi, X> over the real layout
    if coeffs is None:
        return S, _force(L, U, X, bc), it
    GF, GN = _force_imp(L, F, N, X, bc)
    return S, fatten_vjp(L, U, coeffs, GF, GN), it


def trajectory(L, U0, P0, R_e, R_o, beta, mass, eps, nsteps, tol=1e-12, bc=None, phi=None, coeffs=None):
    """One leapfrog trajectory. U0 real canonical, P0 complex [4][V][3][3]
    (traceless anti-Hermitian). The pseudofermion comes from R_e, R_o at U0
    unless phi is given. coeffs: fattening weights (c1, c3, c5, c7, cL, cN) for
    the improved operator, None for the one-link one. Returns dict with U, P,
    phi, H0, H1, dH and parts."""
    U = U0.copy()
    P = P0.copy()
    if phi is None:
        phi = pseudofermion(L, U, mass, R_e, R_o, bc, coeffs)

    def force(U):
        Sf, Gf, it = fermion_action_and_G(L, U, mass, phi, tol, bc, coeffs)
        return md_force(U, Gf + gauge_force_G(L, U, beta)), Sf, it

    Sf0, _, _ = fermion_action_and_G(L, U, mass, phi, tol, bc, coeffs)
    Sg0, K0 = gauge_action(L, U, beta), kinetic(P)
    F, _, its = force(U)
    P = P + 0.5 * eps * F
    for k in range(nsteps):
        Uc = expm_su3(eps * P) @ cplx(U)
        U = real(Uc)
        F, _, it = force(U)
        its += it
        P = P + (eps if k < nsteps - 1 else 0.5 * eps) * F
    Sf1, _, _ = fermion_action_and_G(L, U, mass, phi, tol, bc, coeffs)
    Sg1, K1 = gauge_action(L, U, beta), kinetic(P)
    H0, H1 = K0 + Sg0 + Sf0, K1 + Sg1 + Sf1
    return dict(U=U, P=P, phi=phi, H0=H0, H1=H1, dH=H1 - H0, Sg0=Sg0, Sg1=Sg1, Sf0=Sf0, Sf1=Sf1, K0=K0, K1=K1,
                cg_iters=its)
