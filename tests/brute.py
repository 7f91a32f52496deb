"""Brute-force dense staggered operator, built entry by entry in Python.

Used only to pin the oracle on tiny lattices (2^4, 4^4 and small non-cubic
shapes). It is written independently of the C oracle: its own coordinate
enumeration, its own neighbour arithmetic, and a dense matrix instead of a
matrix-free site loop. On lattices with an extent of 2 the forward and
backward neighbours coincide and both hops add into the same matrix block,
which a site loop that overwrote instead of accumulating would get wrong.
"""
from __future__ import annotations

import itertools

import numpy as np


def sites(L):
    """Yield (lex, coords) in lexicographic order (x fastest)."""
    Lx, Ly, Lz, Lt = L
    lex = 0
    for t, z, y, x in itertools.product(range(Lt), range(Lz), range(Ly), range(Lx)):
        yield lex, (x, y, z, t)
        lex += 1


def eo_index(L, c):
    Lx, Ly, Lz, Lt = L
    x, y, z, t = c
    lex = x + Lx * (y + Ly * (z + Lz * t))
    V = Lx * Ly * Lz * Lt
    par = (x + y + z + t) % 2
    return par * (V // 2) + lex // 2


def shift(L, c, mu, d):
    c = list(c)
    c[mu] = (c[mu] + d) % L[mu]
    return tuple(c)


def eta(c, mu):
    return -1.0 if sum(c[:mu]) % 2 else 1.0


def dense_D(L, U, bc=(1, 1, 1, 1)):
    """Dense D over all sites, rows/cols ordered (eo, colour): shape (3V, 3V), complex.

    U: canonical float64 [4][V][3][3][2] (eo order).
    """
    V = int(np.prod(L))
    Uc = U[..., 0] + 1j * U[..., 1]
    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    for _, c in sites(L):
        i = eo_index(L, c)
        for mu in range(4):
            e = eta(c, mu)
            sp = bc[mu] if c[mu] == L[mu] - 1 else 1
            sm = bc[mu] if c[mu] == 0 else 1
            jf = eo_index(L, shift(L, c, mu, +1))
            cm = shift(L, c, mu, -1)
            jb = eo_index(L, cm)
            D[3 * i:3 * i + 3, 3 * jf:3 * jf + 3] += e * sp * Uc[mu, i]
            D[3 * i:3 * i + 3, 3 * jb:3 * jb + 3] -= e * sm * Uc[mu, jb].conj().T
    return D


def shift_signed(L, c, mu, steps, bc):
    """Site reached by |steps| single steps along +-mu, and the product of the
    boundary signs picked up each time a step wraps around."""
    c = list(c)
    sign = 1.0
    d = 1 if steps > 0 else -1
    for _ in range(abs(steps)):
        n = c[mu] + d
        if n == L[mu] or n < 0:
            sign *= bc[mu]
        c[mu] = n % L[mu]
    return tuple(c), sign


def dense_D_imp(L, F, N, bc=(1, 1, 1, 1)):
    """Dense improved operator: one-link hops with F, three-link hops with N
    (N_mu(x) joins x to x + 3 mu), both canonical [4][V][3][3][2]."""
    V = int(np.prod(L))
    Fc = F[..., 0] + 1j * F[..., 1]
    Nc = N[..., 0] + 1j * N[..., 1]
    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    for _, c in sites(L):
        i = eo_index(L, c)
        for mu in range(4):
            e = eta(c, mu)
            for steps, W in ((1, Fc), (3, Nc)):
                cf, sf = shift_signed(L, c, mu, +steps, bc)
                cb, sb = shift_signed(L, c, mu, -steps, bc)
                jf, jb = eo_index(L, cf), eo_index(L, cb)
                D[3 * i:3 * i + 3, 3 * jf:3 * jf + 3] += e * sf * W[mu, i]
                D[3 * i:3 * i + 3, 3 * jb:3 * jb + 3] -= e * sb * W[mu, jb].conj().T
    return D


def blocks(L, D):
    """(D_eo, D_oe) blocks of the dense D: D_eo maps odd -> even, D_oe even -> odd."""
    n = 3 * int(np.prod(L)) // 2
    return D[:n, n:], D[n:, :n]


def dense_A(L, U, mass, bc=(1, 1, 1, 1)):
    Deo, Doe = blocks(L, dense_D(L, U, bc))
    n = Deo.shape[0]
    return 4.0 * mass * mass * np.eye(n) - Deo @ Doe


def dense_A_imp(L, F, N, mass, bc=(1, 1, 1, 1)):
    Deo, Doe = blocks(L, dense_D_imp(L, F, N, bc))
    n = Deo.shape[0]
    return 4.0 * mass * mass * np.eye(n) - Deo @ Doe


def cvec(v):
    """canonical [V/2][3][2] -> flat complex (3 V/2)."""
    v = np.asarray(v)
    return (v[..., 0] + 1j * v[..., 1]).reshape(-1)


def rvec(z, Vh):
    out = np.empty((Vh, 3, 2))
    z = z.reshape(Vh, 3)
    out[..., 0] = z.real
    out[..., 1] = z.imag
    return out


# ---- link fattening, path by path ------------------------------------------

def walk(L, Uc, x, steps):
    """Ordered product of the links along a path from x given as signed steps
    (axis, +1 | -1): a forward step from y uses U_nu(y), a backward step the
    adjoint of the link that ends at y. Uc: complex [4][V][3][3], eo order."""
    c = list(x)
    P = np.eye(3, dtype=complex)
    for nu, sg in steps:
        if sg > 0:
            P = P @ Uc[nu][eo_index(L, c)]
            c[nu] = (c[nu] + 1) % L[nu]
        else:
            c[nu] = (c[nu] - 1) % L[nu]
            P = P @ Uc[nu][eo_index(L, c)].conj().T
    return P


def fat_link(L, Uc, x, mu, w):
    """(F_mu(x), N_mu(x)) summed path by path: the link, the 3-, 5- and 7-link
    staples (out along transverse directions on different axes, one mu step,
    back in reverse order), the 5-link Lepage path, and the Naik product."""
    c1, c3, c5, c7, cL, cN = w
    dirs = [(nu, sg) for nu in range(4) if nu != mu for sg in (1, -1)]
    back = lambda a: (a[0], -a[1])
    M = (mu, 1)
    F = c1 * walk(L, Uc, x, [M])
    for a in dirs:
        F = F + c3 * walk(L, Uc, x, [a, M, back(a)])
        F = F + cL * walk(L, Uc, x, [a, a, M, back(a), back(a)])
    for a, b in itertools.permutations(dirs, 2):
        if a[0] != b[0]:
            F = F + c5 * walk(L, Uc, x, [a, b, M, back(b), back(a)])
    for a, b, c in itertools.permutations(dirs, 3):
        if len({a[0], b[0], c[0]}) == 3:
            F = F + c7 * walk(L, Uc, x, [a, b, c, M, back(c), back(b), back(a)])
    return F, cN * walk(L, Uc, x, [M, M, M])


def coords_of_eo(L, eo):
    """Coordinates of the site with eo index eo: lex is 2 cb or 2 cb + 1,
    whichever has the site's parity; checked against eo_index."""
    Lx, Ly, Lz, Lt = L
    Vh = Lx * Ly * Lz * Lt // 2
    par, cb = divmod(int(eo), Vh)
    for lex in (2 * cb, 2 * cb + 1):
        c = (lex % Lx, (lex // Lx) % Ly, (lex // (Lx * Ly)) % Lz, lex // (Lx * Ly * Lz))
        if sum(c) % 2 == par:
            assert eo_index(L, c) == eo
            return c
    raise ValueError(eo)
