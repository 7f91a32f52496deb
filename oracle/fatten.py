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


def fatten(L, U, coeffs):
    """(F, N) from the gauge field U (canonical real layout in and out)."""
    c1, c3, c5, c7, cL, cN = (float(c) for c in coeffs)
    Uc = cplx(np.asarray(U, dtype=np.float64))
    F = np.empty_like(Uc)
    N = np.empty_like(Uc)
    for mu in range(4):
        M0 = Uc[mu]
        dirs = [(nu, sg) for nu in range(4) if nu != mu for sg in (1, -1)]
        one = {a: _staple(L, Uc, mu, a, M0) for a in dirs}
        two = {(a, b): _staple(L, Uc, mu, a, one[b]) for a in dirs for b in dirs if a[0] != b[0]}
        three = [_staple(L, Uc, mu, a, two[(b, c)]) for a in dirs for b in dirs for c in dirs
                 if len({a[0], b[0], c[0]}) == 3]
        lepage = [_staple(L, Uc, mu, a, one[a]) for a in dirs]
        F[mu] = (c1 * M0 + c3 * sum(one.values()) + c5 * sum(two.values()) + c7 * sum(three)
                 + cL * sum(lepage))
        N[mu] = cN * (Uc[mu] @ Uc[mu][shift(L, mu, 1)] @ Uc[mu][shift(L, mu, 2)])
    return real(F), real(N)
