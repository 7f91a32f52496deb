"""Link fattening for the improved staggered operator (test infrastructure only:
only tests/, the smoke check and the benchmark's CPU baseline may use it).

The application the paper times (Table 4, an improved staggered code) uses a
one-link field smeared over paths built with the Table 1 matrix products
(mult_su3_nn, mult_su3_na, mult_su3_an) and a three-link (Naik) field that is a
product of three links. The paper gives neither the paths nor their weights;
the reading used here is the asqtad one:

  F_mu(x) = c1 U_mu(x) + c3 sum_a S_a[U_mu](x) + c5 sum_{a,b} S_a[S_b[U_mu]](x)
          + c7 sum_{a,b,c} S_a[S_b[S_c[U_mu]]](x) + cL sum_a S_a[S_a[U_mu]](x)
  N_mu(x) = cN U_mu(x) U_mu(x+mu) U_mu(x+2mu)

a, b, c run over the six signed directions +-nu, nu != mu, on pairwise
different axes within one term (6, 24 and 48 terms; 6 for the cL term). The
staple of a field M along the signed direction a is

  S_a[M](x) = L_a(x) M(x+a) L_a(x+mu)^dag,

with L_{+nu}(y) = U_nu(y) and L_{-nu}(y) = U_nu(y-nu)^dag the link of one step
from y, so every term is the ordered product of the links along a path from x
to x+mu: out along a (and b, c), one mu step, back along -c, -b, -a. The gauge
field is periodic; fermion boundary signs belong to the Dslash, not here.

Weights are inputs. The tree-level asqtad values (divide each by u0 to the
power of its path length minus one for tadpole improvement) are
c1 = 5/8, c3 = 1/16, c5 = 1/64, c7 = 1/384, cL = -1/16, cN = -1/24; for unit
links they give F = 9/8 and N = -1/24, the free improved operator.

Arrays use the canonical layout: real float64 [4][V][3][3][2], eo site order.
"""
from __future__ import annotations

import numpy as np

from .hmc import cplx, dag, real, shift

ASQTAD = (5.0 / 8.0, 1.0 / 16.0, 1.0 / 64.0, 1.0 / 384.0, -1.0 / 16.0, -1.0 / 24.0)


def asqtad_coeffs(u0: float = 1.0):
    """(c1, c3, c5, c7, cL, cN) with tadpole factor u0 (path length n: / u0^(n-1))."""
    c1, c3, c5, c7, cL, cN = ASQTAD
    return (c1, c3 / u0 ** 2, c5 / u0 ** 4, c7 / u0 ** 6, cL / u0 ** 4, cN / u0 ** 2)


def _step_link(L, Uc, a):
    """L_a(y) for every eo site y; a = (axis, +1 | -1)."""
    nu, sg = a
    if sg > 0:
        return Uc[nu]
    return dag(Uc[nu][shift(L, nu, -1)])


def _staple(L, Uc, mu, a, M):
    """S_a[M](x) = L_a(x) M(x + a) L_a(x + mu)^dag for every x."""
    La = _step_link(L, Uc, a)
    return La @ M[shift(L, a[0], a[1])] @ dag(La[shift(L, mu, 1)])


def _levels(L, Uc, mu):
    """The six signed directions orthogonal to mu, the three-link staples
    S_a[U_mu] (keyed by a) and the five-link ones S_a[S_b[U_mu]] (keyed by (a, b),
    a and b on different axes)."""
    dirs = [(nu, sg) for nu in range(4) if nu != mu for sg in (1, -1)]
    one = {a: _staple(L, Uc, mu, a, Uc[mu]) for a in dirs}
    two = {(a, b): _staple(L, Uc, mu, a, one[b]) for a in dirs for b in dirs if a[0] != b[0]}
    return dirs, one, two


def fatten(L, U, coeffs):
    """(F, N) from the gauge field U (canonical real layout in and out)."""
    c1, c3, c5, c7, cL, cN = (float(c) for c in coeffs)
    Uc = cplx(np.asarray(U, dtype=np.float64))
    F = np.empty_like(Uc)
    N = np.empty_like(Uc)
    for mu in range(4):
        M0 = Uc[mu]
        dirs, one, two = _levels(L, Uc, mu)
        three = [_staple(L, Uc, mu, a, two[(b, c)]) for a in dirs for b in dirs for c in dirs
                 if len({a[0], b[0], c[0]}) == 3]
        lepage = [_staple(L, Uc, mu, a, one[a]) for a in dirs]
        F[mu] = (c1 * M0 + c3 * sum(one.values()) + c5 * sum(two.values()) + c7 * sum(three)
                 + cL * sum(lepage))
        N[mu] = cN * (Uc[mu] @ Uc[mu][shift(L, mu, 1)] @ Uc[mu][shift(L, mu, 2)])
    return real(F), real(N)


# ---- the chain rule through the fattening -------------------------------------
#
# With S depending on U through F(U) and N(U) and the derivative convention of
# the fermion force, dS = sum Re tr(G_F^dag dF) + Re tr(G_N^dag dN), the field
# G_U with dS = sum Re tr(G_U^dag dU) follows from the product rule. For a
# product P = A B C^dag and dS = Re tr(G^dag dP):
#   A receives G C B^dag,   B receives A^dag G C,   C receives G^dag A B,
# and a link entering as its adjoint (L_{-nu}(y) = U_nu(y - nu)^dag) passes the
# adjoint of what it receives to U_nu(y - nu). The nested staple sums of
# fatten() are taken back level by level in that way.


def _add_to_step_link(L, GU, a, y_grad):
    """Add the gradient of L_a(y), given for every y, to the gradient of U."""
    nu, sg = a
    if sg > 0:
        GU[nu] += y_grad
    else:
        # L_{-nu}(y) = U_nu(y - nu)^dag: U_nu(z) receives (grad at z + nu)^dag
        GU[nu] += dag(y_grad[shift(L, nu, 1)])


def _staple_vjp(L, Uc, mu, a, M, G, GU):
    """For P = S_a[M] with dS = Re tr(G^dag P) summed over x: return the
    gradient of M (as a field over y = x + a) and add the link gradients to GU."""
    La = _step_link(L, Uc, a)
    xa = shift(L, a[0], a[1])
    xm = shift(L, mu, 1)
    A, B, C = La, M[xa], La[xm]
    gM = np.empty_like(M)
    gM[xa] = dag(A) @ G @ C
    gA = G @ C @ dag(B)
    gC = np.empty_like(M)
    gC[xm] = dag(G) @ A @ B
    _add_to_step_link(L, GU, a, gA + gC)
    return gM


def fatten_vjp(L, U, coeffs, GF, GN):
    """G_U (canonical real layout) from G_F and G_N (same layout) for the
    fattening of fatten(L, U, coeffs): dS = sum Re tr(G_U^dag dU)."""
    c1, c3, c5, c7, cL, cN = (float(c) for c in coeffs)
    Uc = cplx(np.asarray(U, dtype=np.float64))
    gF, gN = cplx(np.asarray(GF, dtype=np.float64)), cplx(np.asarray(GN, dtype=np.float64))
    GU = np.zeros_like(Uc)
    for mu in range(4):
        M0 = Uc[mu]
        G = gF[mu]
        dirs, one, two = _levels(L, Uc, mu)
        g_two = {k: np.zeros_like(M0) for k in two}
        g_one = {a: np.zeros_like(M0) for a in dirs}
        # c1 U_mu; then the seven-link and Lepage staples pass their gradient
        # to the five- and three-link fields under them, those to U_mu
        GU[mu] += c1 * G
        for a in dirs:
            for b in dirs:
                for c in dirs:
                    if len({a[0], b[0], c[0]}) == 3:
                        g_two[(b, c)] += _staple_vjp(L, Uc, mu, a, two[(b, c)], c7 * G, GU)
            g_one[a] += _staple_vjp(L, Uc, mu, a, one[a], cL * G, GU)
        for (a, b) in two:
            g_one[b] += _staple_vjp(L, Uc, mu, a, one[b], c5 * G + g_two[(a, b)], GU)
        for b in dirs:
            GU[mu] += _staple_vjp(L, Uc, mu, b, M0, c3 * G + g_one[b], GU)
        # Naik: N = cN A B C with A = U_mu(x), B = U_mu(x+mu), C = U_mu(x+2mu)
        x1, x2 = shift(L, mu, 1), shift(L, mu, 2)
        A, B, C = M0, M0[x1], M0[x2]
        H = cN * gN[mu]
        GU[mu] += H @ dag(B @ C)
        gb = np.empty_like(M0)
        gb[x1] = dag(A) @ H @ dag(C)
        GU[mu] += gb
        gc = np.empty_like(M0)
        gc[x2] = dag(A @ B) @ H
        GU[mu] += gc
    return real(GU)
