"""Seeded synthetic inputs for the staggered Dslash / even-odd CG workloads.

This module only draws random numbers and shapes them into gauge fields and
colour vectors. It holds none of the operator's arithmetic (no Dslash, no CG,
no force) and is the one module that both the FP64 oracle tests and the GPU
path use, so that both sides see bit-identical inputs.

Conventions (shared with the library header):

* Lattice dims ``L = (Lx, Ly, Lz, Lt)``, all even; lexicographic site index
  ``lex = x + Lx*(y + Ly*(z + Lz*t))``; parity ``(x+y+z+t) & 1``; checkerboard
  index ``cb = lex >> 1``; even-odd index ``eo = parity*V/2 + cb``.
* Canonical link field: float64 array ``[4][V][3][3][2]`` -- direction mu,
  eo site, row, column, (re, im). No staggered phases or boundary signs are
  folded in.
* Canonical colour vector on one parity: float64 ``[V/2][3][2]``, cb order.

Distributions (the paper's workloads are lattices of SU(3) links, Sec. 1 and
Sec. 4; the random ensembles below are synthetic stand-ins):

* ``haar``: Haar-random SU(3). A complex Gaussian 3x3 matrix is orthonormalised
  column by column (Gram-Schmidt, i.e. a QR factorisation whose R has a
  positive real diagonal, which makes Q Haar on U(3)); dividing by the
  principal cube root of det(Q) lands in SU(3) and keeps left invariance.
* ``expih``: exp(i c H) with H = (A + A^dag)/2 - tr(.)/3, A complex Gaussian
  with Re, Im ~ N(0, 1/2); computed as V diag(exp(i c w)) V^dag from eigh.
* ``haar_pool``: every link an independent uniform draw from a seeded pool of
  2^16 Haar matrices (each link is Haar-distributed; for lattices whose
  per-link QR would take minutes on the host).
* ``gaussian`` vectors: Re, Im ~ N(0, 1/2) per component.

Seeds: numpy ``Generator(PCG64(seed))``; whole arrays are drawn in canonical
array order.
"""
from __future__ import annotations

import hashlib

import numpy as np

__all__ = [
    "volume",
    "rng",
    "haar_su3",
    "expih_su3",
    "gaussian_cvec",
    "links",
    "improved_links",
    "momenta",
    "uniform",
    "fd_directions",
    "vector",
    "vectors",
    "to_real",
    "to_complex",
    "sha256",
    "CONFIGS",
]


def volume(L) -> int:
    v = 1
    for d in L:
        v *= int(d)
    return v


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _complex_gaussian(g: np.random.Generator, shape) -> np.ndarray:
    """Complex normal with Re, Im ~ N(0, 1/2) (so E|z|^2 = 1)."""
    a = g.standard_normal(tuple(shape) + (2,))
    a *= np.sqrt(0.5)
    return a[..., 0] + 1j * a[..., 1]


def haar_su3(n: int, g: np.random.Generator) -> np.ndarray:
    """n Haar-random SU(3) matrices, complex128 (n, 3, 3)."""
    z = _complex_gaussian(g, (n, 3, 3))
    q = np.empty_like(z)
    # modified Gram-Schmidt on the columns == QR with diag(R) > 0
    for j in range(3):
        v = z[:, :, j].copy()
        for k in range(j):
            proj = np.einsum("ni,ni->n", q[:, :, k].conj(), v)
            v -= proj[:, None] * q[:, :, k]
        nrm = np.sqrt(np.einsum("ni,ni->n", v.conj(), v).real)
        q[:, :, j] = v / nrm[:, None]
    det = np.linalg.det(q)
    root = np.exp(1j * np.angle(det) / 3.0)  # principal cube root of a unit complex
    q /= root[:, None, None]
    return q


def expih_su3(n: int, c: float, g: np.random.Generator) -> np.ndarray:
    """n matrices exp(i c H), H random traceless Hermitian; complex128 (n,3,3)."""
    a = _complex_gaussian(g, (n, 3, 3))
    h = 0.5 * (a + np.conj(np.swapaxes(a, 1, 2)))
    tr = np.trace(h, axis1=1, axis2=2).real / 3.0
    h[:, 0, 0] -= tr
    h[:, 1, 1] -= tr
    h[:, 2, 2] -= tr
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * c * w)
    return np.einsum("nij,nj,nkj->nik", v, ph, v.conj())


def gaussian_cvec(n: int, g: np.random.Generator) -> np.ndarray:
    """n colour vectors, complex128 (n, 3)."""
    return _complex_gaussian(g, (n, 3))


def to_real(a: np.ndarray) -> np.ndarray:
    """complex (...) -> float64 (..., 2), contiguous."""
    out = np.empty(a.shape + (2,), dtype=np.float64)
    out[..., 0] = a.real
    out[..., 1] = a.imag
    return out


def to_complex(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    return a[..., 0] + 1j * a[..., 1]


def links(L, kind: str = "haar", seed: int = 1, c: float = 0.3) -> np.ndarray:
    """Canonical float64 link field [4][V][3][3][2] in eo site order.

    kind: 'haar' | 'expih' | 'unit' | 'haar_pool'.
    """
    V = volume(L)
    if kind == "haar_pool":
        g = rng(seed)
        pool = to_real(haar_su3(1 << 16, g))
        idx = g.integers(0, pool.shape[0], size=4 * V)
        out = np.empty((4 * V, 3, 3, 2), dtype=np.float64)
        np.take(pool, idx, axis=0, out=out)
        return out.reshape(4, V, 3, 3, 2)
    if kind == "unit":
        u = np.zeros((4 * V, 3, 3), dtype=np.complex128)
        u[:, 0, 0] = u[:, 1, 1] = u[:, 2, 2] = 1.0
    elif kind == "haar":
        u = haar_su3(4 * V, rng(seed))
    elif kind == "expih":
        u = expih_su3(4 * V, c, rng(seed))
    else:
        raise ValueError(f"unknown link kind {kind!r}")
    return to_real(u).reshape(4, V, 3, 3, 2)


def improved_links(L, seed: int, c1: float = 9.0 / 8.0, c3: float = -1.0 / 24.0, w: float = 0.1):
    """Link fields of the improved operator, canonical float64 [4][V][3][3][2] each:
    fat one-link F = c1 U + w Z (U Haar SU(3), Z complex Gaussian: a general
    complex 3x3 matrix, as a sum of smeared paths is) and Naik three-link
    N = c3 W (W Haar SU(3)); the tree-level coefficients c1 = 9/8, c3 = -1/24
    by default. One stream: U, then Z, then W."""
    V = volume(L)
    g = rng(seed)
    U = haar_su3(4 * V, g)
    Z = _complex_gaussian(g, (4 * V, 3, 3))
    W = haar_su3(4 * V, g)
    F = (c1 * U + w * Z).reshape(4, V, 3, 3)
    N = (c3 * W).reshape(4, V, 3, 3)
    return to_real(F), to_real(N)


def momenta(L, seed: int) -> np.ndarray:
    """Gaussian HMC momenta, complex [4][V][3][3]: P = i H with H the traceless
    part of (Z + Z^dag)/2, Z complex Gaussian with E|Z_ij|^2 = 1. H then has the
    distribution of sum_a p^a lambda^a / 2 with p^a ~ N(0, 1) (off-diagonal
    parts N(0, 1/4) each, diagonal covariance (delta_ij - 1/3)/2)."""
    V = volume(L)
    Z = _complex_gaussian(rng(seed), (4, V, 3, 3))
    H = 0.5 * (Z + np.conj(np.swapaxes(Z, -1, -2)))
    H = H - (np.trace(H, axis1=-2, axis2=-1) / 3.0)[..., None, None] * np.eye(3)
    return 1j * H


def uniform(seed: int) -> float:
    """One uniform number in [0, 1) (the Metropolis test's)."""
    return float(rng(seed).random())


def fd_directions(L, seed: int, n: int):
    """n random link directions for finite differences: per direction a uniform
    mu in 0..3, a uniform eo site, and a Gaussian E in R^18 scaled to unit norm
    (drawn in that order from one stream). Returns (mu[n], site[n], E[n][3][3][2])."""
    g = rng(seed)
    V = volume(L)
    mus, sites, Es = [], [], []
    for _ in range(n):
        mus.append(int(g.integers(4)))
        sites.append(int(g.integers(V)))
        e = g.standard_normal(18)
        Es.append((e / np.linalg.norm(e)).reshape(3, 3, 2))
    return mus, sites, np.array(Es)


def vector(L, seed: int) -> np.ndarray:
    """Canonical float64 colour vector on one parity, [V/2][3][2]."""
    Vh = volume(L) // 2
    return to_real(gaussian_cvec(Vh, rng(seed)))


def vectors(L, seed: int, n: int) -> np.ndarray:
    """n independent parity vectors drawn from one stream, [n][V/2][3][2]."""
    Vh = volume(L) // 2
    return to_real(gaussian_cvec(n * Vh, rng(seed))).reshape(n, Vh, 3, 2)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# The five workloads: lattice, link ensemble, mass, seeds (seed = 1000*k + role;
# role 1 links, 2 source, 3 gauge transform, 4 FD directions, 10+j member j).
CONFIGS = {
    "c1_4x4x4x4": dict(L=(4, 4, 4, 4), kind="haar", c=None, mass=0.1,
                       link_seed=1001, src_seed=1002, tol=1e-10),
    "c2_16x16x16x16": dict(L=(16, 16, 16, 16), kind="expih", c=0.3, mass=0.05,
                           link_seed=2001, src_seed=2002, tol=1e-10),
    "c3_32x32x32x32": dict(L=(32, 32, 32, 32), kind="haar", c=None, mass=0.01,
                           link_seed=3001, src_seed=3002, tol=1e-10),
    "c4_24x24x24x48": dict(L=(24, 24, 24, 48), kind="haar", c=None, mass=0.02,
                           link_seed=4001, src_seed=4010, nrhs=16, tol=1e-10),
    "c4_mixed": dict(members=[((8, 8, 8, 8), 4101), ((12, 12, 12, 12), 4201),
                              ((16, 16, 16, 32), 4301)],
                     kind="haar", mass=0.02, nrhs=4, src_seed_offset=10, tol=1e-10),
    "c5_16x16x16x32": dict(L=(16, 16, 16, 32), kind="expih", c=0.5, mass=0.05,
                           link_seed=5001, src_seed=5002, fd_seed=5004, tol=1e-10),
    # HMC trajectory around the solve (links, momenta, pseudofermion R_e, R_o, Metropolis u)
    # trajectory length 0.2 in 80 leapfrog steps: |dH| of order 1 from these
    # (non-equilibrium) links, so the Metropolis test can go either way
    "hmc_16x16x16x16": dict(L=(16, 16, 16, 16), kind="expih", c=0.3, beta=5.6, mass=0.05, eps=0.0025,
                            nsteps=80, link_seed=8001, mom_seed=8002, re_seed=8003, ro_seed=8004,
                            u_seed=8005, tol=1e-10),
    # improved (fat + Naik) operator at the headline lattice size
    "imp_32x32x32x32": dict(L=(32, 32, 32, 32), mass=0.01, link_seed=6001, src_seed=6002, tol=1e-10),
}
