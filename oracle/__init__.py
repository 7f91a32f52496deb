"""FP64 CPU oracle for the staggered Dslash, the even-odd CG and the fermion force.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg. The library never imports it.

Thin numpy wrappers over ``liblgt_oracle.so`` (plain C, see lgt_oracle.c for
the formulas and the passages they follow). Arrays use the canonical layouts:
links float64 ``[4][V][3][3][2]`` (eo order), parity vectors ``[V/2][3][2]``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import SO, build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            build()
        _lib = C.CDLL(SO)
        _setup(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


def _setup(l):
    l.or_geom_ok.restype = C.c_int
    l.or_geom_ok.argtypes = [_ip, _ip]
    l.or_index_maps.argtypes = [_ip, _ip, _ip]
    l.or_set_threads.argtypes = [C.c_int]
    l.or_get_threads.restype = C.c_int
    l.or_dslash.argtypes = [_ip, _ip, _dp, _dp, _dp, C.c_int]
    l.or_apply_A.argtypes = [_ip, _ip, _dp, C.c_double, _dp, _dp]
    l.or_cdot.argtypes = [C.c_int64, _dp, _dp, _dp, _dp]
    l.or_norm2.restype = C.c_double
    l.or_norm2.argtypes = [C.c_int64, _dp]
    l.or_cg.restype = C.c_int
    l.or_cg.argtypes = [_ip, _ip, _dp, C.c_double, _dp, _dp, C.c_double, C.c_int,
                        C.POINTER(C.c_int), _dp]
    l.or_force.argtypes = [_ip, _ip, _dp, _dp, _dp]
    l.or_dslash_imp.argtypes = [_ip, _ip, _dp, _dp, _dp, _dp, C.c_int]
    l.or_apply_A_imp.argtypes = [_ip, _ip, _dp, _dp, C.c_double, _dp, _dp]
    l.or_cg_imp.restype = C.c_int
    l.or_cg_imp.argtypes = [_ip, _ip, _dp, _dp, C.c_double, _dp, _dp, C.c_double, C.c_int,
                            C.POINTER(C.c_int), C.POINTER(C.c_double)]
    l.or_force_imp.argtypes = [_ip, _ip, _dp, _dp, _dp, _dp, _dp]
    l.or_action_variational.restype = C.c_double
    l.or_action_variational.argtypes = [_ip, _ip, _dp, C.c_double, _dp, _dp]
    cx = C.c_void_p
    for name in ("or_add_su3_vector", "or_mult_su3_mat_vec", "or_mult_adj_su3_mat_vec",
                 "or_mult_adj_su3_mat_vec_4dir", "or_mult_su3_an", "or_mult_su3_na",
                 "or_mult_su3_nn", "or_mult_su3_mat_vec_sum_4dir", "or_su3_projector"):
        getattr(l, name).argtypes = [cx, cx, cx]
    l.or_mult_adj_su3_mat_4vec.argtypes = [cx, cx, cx, cx, cx, cx]
    l.or_scalar_mult_add_su3_matrix.argtypes = [cx, cx, C.c_double, cx]
    l.or_scalar_mult_add_su3_vector.argtypes = [cx, cx, C.c_double, cx]
    l.or_sub_four_su3_vecs.argtypes = [cx, cx]


def _i4(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(4))


def _dptr(a):
    return a.ctypes.data_as(_dp)


def _iptr(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _bc(bc):
    return _i4((1, 1, 1, 1) if bc is None else bc)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def threads() -> int:
    return int(lib().or_get_threads())


def geom_ok(L, bc=None) -> bool:
    return bool(lib().or_geom_ok(_iptr(_i4(L)), _iptr(_bc(bc))))


def index_maps(L):
    L = _i4(L)
    V = int(np.prod(L.astype(np.int64)))
    lex_of_eo = np.empty(V, np.int32)
    nbr = np.empty((2, 8, V // 2), np.int32)
    lib().or_index_maps(_iptr(L), _iptr(lex_of_eo), _iptr(nbr))
    return lex_of_eo, nbr


def dslash(L, U, chi, out_parity: int, bc=None):
    """out (parity out_parity) = D chi; chi on the other parity, [V/2][3][2]."""
    L = _i4(L)
    U = _f64(U)
    chi = _f64(chi)
    out = np.empty_like(chi)
    lib().or_dslash(_iptr(L), _iptr(_bc(bc)), _dptr(U), _dptr(chi), _dptr(out), int(out_parity))
    return out


def apply_A(L, U, mass, v, bc=None):
    L = _i4(L)
    U = _f64(U)
    v = _f64(v)
    out = np.empty_like(v)
    lib().or_apply_A(_iptr(L), _iptr(_bc(bc)), _dptr(U), float(mass), _dptr(v), _dptr(out))
    return out


def cdot(a, b):
    a = _f64(a)
    b = _f64(b)
    re, im = C.c_double(), C.c_double()
    lib().or_cdot(a.size, _dptr(a), _dptr(b), C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def norm2(a):
    a = _f64(a)
    return float(lib().or_norm2(a.size, _dptr(a)))


def cg(L, U, mass, b, tol=1e-10, max_iter=100000, bc=None):
    """Returns (status, x, iters, true_rel_resid)."""
    L = _i4(L)
    U = _f64(U)
    b = _f64(b)
    x = np.empty_like(b)
    it = C.c_int()
    rr = C.c_double()
    st = lib().or_cg(_iptr(L), _iptr(_bc(bc)), _dptr(U), float(mass), _dptr(b), _dptr(x),
                     float(tol), int(max_iter), C.byref(it), C.byref(rr))
    return int(st), x, int(it.value), float(rr.value)


def dslash_imp(L, F, N, chi, out_parity: int, bc=None):
    """Improved operator: fat one-link field F plus Naik three-link field N."""
    L = _i4(L)
    F = _f64(F)
    N = _f64(N)
    chi = _f64(chi)
    out = np.empty_like(chi)
    lib().or_dslash_imp(_iptr(L), _iptr(_bc(bc)), _dptr(F), _dptr(N), _dptr(chi), _dptr(out), int(out_parity))
    return out


def apply_A_imp(L, F, N, mass, v, bc=None):
    L = _i4(L)
    F = _f64(F)
    N = _f64(N)
    v = _f64(v)
    out = np.empty_like(v)
    lib().or_apply_A_imp(_iptr(L), _iptr(_bc(bc)), _dptr(F), _dptr(N), float(mass), _dptr(v), _dptr(out))
    return out


def cg_imp(L, F, N, mass, b, tol=1e-10, max_iter=100000, bc=None):
    """CG with the improved operator. Returns (status, x, iters, true_rel_resid)."""
    L = _i4(L)
    F = _f64(F)
    N = _f64(N)
    b = _f64(b)
    x = np.empty_like(b)
    it = C.c_int()
    rr = C.c_double()
    st = lib().or_cg_imp(_iptr(L), _iptr(_bc(bc)), _dptr(F), _dptr(N), float(mass), _dptr(b), _dptr(x),
                         float(tol), int(max_iter), C.byref(it), C.byref(rr))
    return int(st), x, int(it.value), float(rr.value)


def force(L, U, X, bc=None):
    """G[4][V][3][3][2] = dS/d(Re U, Im U) for S = phi^dag A^-1 phi, given X = A^-1 phi."""
    L = _i4(L)
    U = _f64(U)
    X = _f64(X)
    G = np.empty_like(U)
    lib().or_force(_iptr(L), _iptr(_bc(bc)), _dptr(U), _dptr(X), _dptr(G))
    return G


def force_imp(L, F, N, X, bc=None):
    """(GF, GN) = dS/d(Re, Im) of the fat and Naik fields for the improved
    operator's S = phi^dag A^-1 phi, given X = A^-1 phi (or_force_imp)."""
    L = _i4(L)
    F, N, X = _f64(F), _f64(N), _f64(X)
    GF, GN = np.empty_like(F), np.empty_like(N)
    lib().or_force_imp(_iptr(L), _iptr(_bc(bc)), _dptr(F), _dptr(N), _dptr(X), _dptr(GF), _dptr(GN))
    return GF, GN


def action_phi_grad(X):
    """dS/d(Re phi, Im phi) for S = phi^dag A^-1 phi, given X = A^-1 phi.

    A^-1 is Hermitian, so S(phi + d) - S(phi) = 2 Re <X, d> + O(d^2): the
    derivative along the real and imaginary parts of each component is twice
    the real and imaginary part of X there. [V/2][3][2]."""
    return 2.0 * np.asarray(X, dtype=np.float64)


def action_variational(L, U, mass, phi, x, bc=None):
    L = _i4(L)
    return float(lib().or_action_variational(_iptr(L), _iptr(_bc(bc)), _dptr(_f64(U)),
                                             float(mass), _dptr(_f64(phi)), _dptr(_f64(x))))


# --- single-object Table 1 routines on numpy complex arrays (for the routine tests) ---

def _cx(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    assert a.size == n
    return a


def routine(name, *args, scalar=None):
    """Call one Table 1 routine on complex arrays; returns the output array(s)."""
    l = lib()
    f = getattr(l, "or_" + name)
    if name == "mult_adj_su3_mat_4vec":
        B4 = _cx(args[0], 36)
        a = _cx(args[1], 3)
        outs = [np.empty(3, np.complex128) for _ in range(4)]
        f(B4.ctypes.data, a.ctypes.data, *[o.ctypes.data for o in outs])
        return outs
    if name == "sub_four_su3_vecs":
        a = _cx(args[0], 3).copy()
        b4 = _cx(args[1], 12)
        f(a.ctypes.data, b4.ctypes.data)
        return a
    shapes_out = {
        "add_su3_vector": 3, "mult_su3_mat_vec": 3, "mult_adj_su3_mat_vec": 3,
        "mult_adj_su3_mat_vec_4dir": 12, "mult_su3_an": 9, "mult_su3_na": 9,
        "mult_su3_nn": 9, "mult_su3_mat_vec_sum_4dir": 3, "su3_projector": 9,
        "scalar_mult_add_su3_matrix": 9, "scalar_mult_add_su3_vector": 3,
    }
    n_in = {
        "add_su3_vector": (3, 3), "mult_su3_mat_vec": (9, 3), "mult_adj_su3_mat_vec": (9, 3),
        "mult_adj_su3_mat_vec_4dir": (3, 36), "mult_su3_an": (9, 9), "mult_su3_na": (9, 9),
        "mult_su3_nn": (9, 9), "mult_su3_mat_vec_sum_4dir": (36, 12), "su3_projector": (3, 3),
        "scalar_mult_add_su3_matrix": (9, 9), "scalar_mult_add_su3_vector": (3, 3),
    }[name]
    a = _cx(args[0], n_in[0])
    b = _cx(args[1], n_in[1])
    out = np.empty(shapes_out[name], np.complex128)
    if scalar is not None:
        f(a.ctypes.data, b.ctypes.data, float(scalar), out.ctypes.data)
    else:
        f(a.ctypes.data, b.ctypes.data, out.ctypes.data)
    return out
