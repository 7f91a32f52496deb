"""ctypes binding of liblgt.so with torch tensors as device memory.

Names follow include/lgt.h. Tensors passed in must be CUDA (HIP) tensors on
the context's device, contiguous, in the canonical layouts of lgt.h:
links float64 [4][V][3][3][2] (eo order), parity vectors float64 [V/2][3][2].
Native vectors are held as tensors of shape [3][V/2][2] (float64 for F64
fields, float32 otherwise); packed links as uint8 tensors.
"""
from __future__ import annotations

import atexit
import ctypes as C
import dataclasses
import os
import re
import weakref

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "liblgt.so")

LGT_F64, LGT_F32, LGT_BF16 = 0, 1, 2
LGT_R18, LGT_R12 = 18, 12
LGT_EVEN, LGT_ODD = 0, 1
LGT_CG_FP64, LGT_CG_RELIABLE, LGT_CG_REFINE = 0, 1, 2
LGT_MRHS_LANE, LGT_MRHS_VALU4, LGT_MRHS_MFMA = 0, 1, 2

STATUS = {
    0: "LGT_OK", -1: "LGT_ERR_ARG", -2: "LGT_ERR_GEOMETRY", -3: "LGT_ERR_ALIGN",
    -4: "LGT_ERR_DEVICE", -5: "LGT_ERR_NOT_CONVERGED", -6: "LGT_ERR_NONFINITE",
    -7: "LGT_ERR_OOM", -8: "LGT_ERR_UNSUPPORTED",
}

# 8 complex 3x3 mat-vecs of 66 flop (36 mul + 30 add) and 7 three-complex vector
# additions of 6 flop per output site
DSLASH_FLOP_PER_SITE = 8 * 66 + 7 * 6
IMPROVED_FLOP_PER_SITE = 16 * 66 + 15 * 6  # one-link and Naik hops: 1146


def link_bytes_per_dir(prec: int, recon: int) -> int:
    return {(0, 18): 144, (0, 12): 96, (1, 18): 72, (1, 12): 48, (2, 12): 24}[(prec, recon)]


def vec_bytes_per_site(prec: int) -> int:
    return 48 if prec == LGT_F64 else 24


class LgtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Geom(C.Structure):
    _fields_ = [("L", C.c_int32 * 4), ("bc", C.c_int32 * 4)]


class _Links(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("prec", C.c_int32), ("recon", C.c_int32)]


class _CgParams(C.Structure):
    _fields_ = [("mass", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("scheme", C.c_int32), ("ru_interval", C.c_int32), ("x0_is_guess", C.c_int32),
                ("inner_tol", C.c_double), ("check_interval", C.c_int32), ("reserved", C.c_int32)]


class _CgResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("updates", C.c_int32),
                ("dslash_calls", C.c_int32), ("true_rel_resid", C.c_double), ("seconds", C.c_double),
                ("dslash_ms_hi", C.c_double), ("dslash_ms_lo", C.c_double),
                ("dslash_timed_hi", C.c_int32), ("dslash_timed_lo", C.c_int32)]


class _CgProblem(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("U_hi", C.POINTER(_Links)), ("U_lo", C.POINTER(_Links)),
                ("nrhs", C.c_int32), ("b", C.c_void_p), ("x", C.c_void_p), ("res", C.POINTER(_CgResult))]


_lib = None


def lib_path() -> str:
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise ImportError(f"{_SO} is missing: build it with `python -c 'import __graft_entry__ as g; "
                              "g.build()'` (there is no fallback path)")
        _lib = C.CDLL(_SO)
        _setup(_lib)
    return _lib


class _HmcParams(C.Structure):
    _fields_ = [("beta", C.c_double), ("mass", C.c_double), ("eps", C.c_double), ("tol", C.c_double),
                ("u", C.c_double), ("nsteps", C.c_int32), ("scheme", C.c_int32), ("reserved", C.c_int32 * 2)]


class _HmcResult(C.Structure):
    _fields_ = [("H0", C.c_double), ("H1", C.c_double), ("dH", C.c_double), ("Sg0", C.c_double),
                ("Sg1", C.c_double), ("Sf0", C.c_double), ("Sf1", C.c_double), ("K0", C.c_double),
                ("K1", C.c_double), ("seconds", C.c_double), ("accepted", C.c_int32), ("cg_iters", C.c_int32),
                ("cg_solves", C.c_int32), ("reserved", C.c_int32)]


class _FatCoeffs(C.Structure):
    _fields_ = [("one_link", C.c_double), ("staple3", C.c_double), ("staple5", C.c_double),
                ("staple7", C.c_double), ("lepage", C.c_double), ("naik", C.c_double)]


def asqtad_coeffs(u0: float = 1.0) -> tuple:
    """Tree-level asqtad weights (one link, 3-, 5-, 7-link staples, Lepage, Naik)
    with tadpole improvement by u0, from the library (lgt_asqtad_coeffs)."""
    w = _FatCoeffs()
    _check(lib().lgt_asqtad_coeffs(float(u0), C.byref(w)))
    return (w.one_link, w.staple3, w.staple5, w.staple7, w.lepage, w.naik)


def _setup(l):
    vp, i32, st = C.c_void_p, C.c_int32, C.c_int32
    sig = {
        "lgt_status_string": (C.c_char_p, [st]),
        "lgt_last_error": (C.c_char_p, []),
        "lgt_geom_check": (st, [C.POINTER(_Geom)]),
        "lgt_links_bytes": (st, [C.POINTER(_Geom), i32, i32, C.POINTER(C.c_size_t)]),
        "lgt_vec_bytes": (st, [C.POINTER(_Geom), i32, C.POINTER(C.c_size_t)]),
        "lgt_create": (st, [C.POINTER(_Geom), i32, vp, C.POINTER(vp)]),
        "lgt_destroy": (st, [vp]),
        "lgt_set_timing": (st, [vp, i32]),
        "lgt_index_maps": (st, [vp, vp, vp]),
        "lgt_pack_links": (st, [vp, vp, i32, i32, vp]),
        "lgt_unpack_links": (st, [vp, vp, i32, i32, vp]),
        "lgt_pack_vec": (st, [vp, i32, vp, vp]),
        "lgt_unpack_vec": (st, [vp, i32, vp, vp]),
        "lgt_dslash": (st, [vp, C.POINTER(_Links), i32, vp, vp]),
        "lgt_cg_solve": (st, [vp, C.POINTER(_Links), C.POINTER(_Links), C.POINTER(_CgParams), vp, vp,
                              C.POINTER(_CgResult)]),
        "lgt_cdot": (st, [vp, C.c_int64, vp, vp, C.POINTER(C.c_double)]),
        "lgt_force": (st, [vp, C.POINTER(_Links), vp, C.c_double, vp]),
        "lgt_force_noalloc": (st, [vp, C.POINTER(_Links), vp, C.c_double, vp]),
        "lgt_set_dslash_variant": (st, [vp, i32, i32, i32, i32]),
        "lgt_get_dslash_variant": (st, [vp, i32, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "lgt_set_dslash_workgroup": (st, [vp, i32, i32, i32]),
        "lgt_get_dslash_workgroup": (st, [vp, i32, i32, C.POINTER(C.c_int32)]),
        "lgt_tune_dslash": (st, [vp, C.POINTER(_Links), C.POINTER(C.c_double)]),
        "lgt_set_dslash_improved_variant": (st, [vp, i32, i32, i32]),
        "lgt_get_dslash_improved_variant": (st, [vp, i32, C.POINTER(i32), C.POINTER(i32)]),
        "lgt_tune_dslash_improved": (st, [vp, C.POINTER(_Links), C.POINTER(_Links), C.POINTER(C.c_double)]),
        "lgt_apply_normal": (st, [vp, C.POINTER(_Links), C.c_double, vp, vp, C.POINTER(C.c_double)]),
        "lgt_stream_copy": (st, [vp, vp, vp, C.c_size_t]),
        "lgt_stream_read": (st, [vp, vp, C.c_size_t, vp]),
        "lgt_stream_read_links": (st, [vp, C.POINTER(_Links), i32, i32, vp]),
        "lgt_pack_vec_mrhs": (st, [vp, i32, i32, vp, vp]),
        "lgt_unpack_vec_mrhs": (st, [vp, i32, i32, vp, vp]),
        "lgt_dslash_mrhs": (st, [vp, C.POINTER(_Links), i32, i32, vp, vp]),
        "lgt_set_mrhs_engine": (st, [vp, i32]),
        "lgt_get_mrhs_engine": (st, [vp, C.POINTER(C.c_int32)]),
        "lgt_set_mrhs_variant": (st, [vp, i32, i32, i32, i32, i32]),
        "lgt_set_mrhs_staging": (st, [vp, i32, i32, i32, i32]),
        "lgt_get_mrhs_staging": (st, [vp, i32, i32, i32, C.POINTER(i32)]),
        "lgt_get_mrhs_variant": (st, [vp, i32, i32, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "lgt_tune_dslash_mrhs": (st, [vp, C.POINTER(_Links), i32, C.POINTER(C.c_double)]),
        "lgt_cg_solve_batch": (st, [C.POINTER(_CgProblem), i32, C.POINTER(_CgParams)]),
        "lgt_batch_profile": (st, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
        "lgt_cg_dslash_profile": (st, [vp, C.POINTER(C.c_double), C.POINTER(i32)]),
        "lgt_cg_profile": (st, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
        "lgt_dslash_improved": (st, [vp, C.POINTER(_Links), C.POINTER(_Links), i32, vp, vp]),
        "lgt_force_improved": (st, [vp, C.POINTER(_Links), C.POINTER(_Links), vp, C.c_double, vp, vp]),
        "lgt_routine": (st, [vp, i32, i32, C.c_int64, vp, vp, vp, C.c_double]),
        "lgt_gauge_force": (st, [vp, vp, C.c_double, C.c_double, i32, vp]),
        "lgt_fatten_links": (st, [vp, vp, C.POINTER(_FatCoeffs), vp, vp]),
        "lgt_fatten_links_vjp": (st, [vp, vp, C.POINTER(_FatCoeffs), vp, vp, C.c_double, i32, vp]),
        "lgt_asqtad_coeffs": (st, [C.c_double, C.POINTER(_FatCoeffs)]),
        "lgt_action_phi_grad": (st, [vp, vp, C.c_double, vp]),
        "lgt_momentum_update": (st, [vp, vp, vp, C.c_double, vp]),
        "lgt_link_update": (st, [vp, vp, C.c_double, vp]),
        "lgt_plaquette": (st, [vp, vp, C.POINTER(C.c_double)]),
        "lgt_kinetic_energy": (st, [vp, vp, C.POINTER(C.c_double)]),
        "lgt_hmc_trajectory": (st, [vp, vp, vp, vp, vp, C.POINTER(_HmcParams), C.POINTER(_HmcResult)]),
        "lgt_hmc_trajectory_improved": (st, [vp, vp, vp, vp, vp, C.POINTER(_HmcParams), C.POINTER(_FatCoeffs),
                                             C.POINTER(_HmcResult)]),
        "lgt_cg_solve_improved": (st, [vp, C.POINTER(_Links), C.POINTER(_Links), C.POINTER(_Links),
                                       C.POINTER(_Links), C.POINTER(_CgParams), vp, vp, C.POINTER(_CgResult)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(l, name)
        f.restype = res
        f.argtypes = args


def exported_symbols_declared(header: str | None = None) -> list[str]:
    header = header or os.path.join(os.path.dirname(HERE), "include", "lgt.h")
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lgt_[a-z0-9_]+)\s*\(", text)))


def exported_symbols() -> list[str]:
    """Names declared in include/lgt.h that the loaded library exports."""
    l = lib()
    return [n for n in exported_symbols_declared() if hasattr(l, n)]


def _check(status: int):
    if status != 0:
        msg = lib().lgt_last_error().decode()
        raise LgtError(status, msg)


def _geom(L, bc) -> _Geom:
    g = _Geom()
    for i in range(4):
        g.L[i] = int(L[i])
        g.bc[i] = int(bc[i])
    return g


def geom_check(L, bc=(1, 1, 1, 1)) -> int:
    return int(lib().lgt_geom_check(C.byref(_geom(L, bc))))


def links_bytes(L, prec, recon, bc=(1, 1, 1, 1)) -> int:
    n = C.c_size_t()
    _check(lib().lgt_links_bytes(C.byref(_geom(L, bc)), prec, recon, C.byref(n)))
    return int(n.value)


def vec_bytes(L, prec, bc=(1, 1, 1, 1)) -> int:
    n = C.c_size_t()
    _check(lib().lgt_vec_bytes(C.byref(_geom(L, bc)), prec, C.byref(n)))
    return int(n.value)


def _ptr(t: torch.Tensor) -> int:
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


@dataclasses.dataclass
class PackedLinks:
    data: torch.Tensor  # uint8, lgt_links_bytes
    prec: int
    recon: int

    def desc(self) -> _Links:
        return _Links(self.data.data_ptr(), self.prec, self.recon)


@dataclasses.dataclass
class CgResult:
    status: int
    iters: int
    updates: int
    dslash_calls: int
    true_rel_resid: float
    seconds: float
    dslash_ms_hi: float
    dslash_ms_lo: float
    dslash_timed_hi: int
    dslash_timed_lo: int


# Contexts still open when the interpreter exits are destroyed from an atexit
# hook, in order, while the HIP runtime is fully alive: left to garbage
# collection at shutdown, lgt_destroy (a stream synchronise and hipFree of the
# workspace) could run after the runtime or a profiler attached to it has
# begun tearing down.
_live = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    for lat in list(_live):
        try:
            lat.close()
        except Exception:
            pass


class Lattice:
    """One lattice geometry on one GPU: an lgt_ctx bound to torch's current stream."""

    def __init__(self, L, bc=(1, 1, 1, 1), device: int = 0, stream: torch.cuda.Stream | None = None):
        self.L = tuple(int(x) for x in L)
        self.bc = tuple(int(x) for x in bc)
        self.V = self.L[0] * self.L[1] * self.L[2] * self.L[3]
        self.Vh = self.V // 2
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = C.c_void_p()
        _check(lib().lgt_create(C.byref(_geom(self.L, self.bc)), device, C.c_void_p(self.stream.cuda_stream),
                                C.byref(self._ctx)))
        _live.add(self)

    def close(self):
        if self._ctx:
            lib().lgt_destroy(self._ctx)
            self._ctx = C.c_void_p()
        _live.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_timing(self, every):
        """Time the Dslash launches of every `every`-th CG iteration (True = every one, 0/False = off)."""
        _check(lib().lgt_set_timing(self._ctx, int(every)))

    def set_dslash_variant(self, prec: int, recon: int, hops: int, streaming: int = 1):
        _check(lib().lgt_set_dslash_variant(self._ctx, prec, recon, hops, streaming))

    def dslash_variant(self, prec: int, recon: int) -> tuple[int, int]:
        """(hops per load group, streaming link loads) used for this link format."""
        h, s = C.c_int32(), C.c_int32()
        _check(lib().lgt_get_dslash_variant(self._ctx, prec, recon, C.byref(h), C.byref(s)))
        return int(h.value), int(s.value)

    def set_dslash_workgroup(self, prec: int, recon: int, threads: int):
        """Dslash workgroup size for this link format: 64, 128 or 256 sites."""
        _check(lib().lgt_set_dslash_workgroup(self._ctx, prec, recon, int(threads)))

    def dslash_workgroup(self, prec: int, recon: int) -> int:
        w = C.c_int32()
        _check(lib().lgt_get_dslash_workgroup(self._ctx, prec, recon, C.byref(w)))
        return int(w.value)

    # (streaming, workgroup size) in the order lgt_tune_dslash_improved reports them
    TUNE_IMPROVED_VARIANTS = ((1, 256), (0, 256), (1, 128), (0, 128), (1, 64), (0, 64))

    def set_dslash_improved_variant(self, prec: int, streaming: int, threads: int = 256):
        """The improved operator's Dslash for 18-real links of precision prec:
        streaming (1) or cached (0) link loads, 64/128/256-site workgroups."""
        _check(lib().lgt_set_dslash_improved_variant(self._ctx, prec, int(streaming), int(threads)))

    def dslash_improved_variant(self, prec: int) -> tuple:
        st, w = C.c_int32(), C.c_int32()
        _check(lib().lgt_get_dslash_improved_variant(self._ctx, prec, C.byref(st), C.byref(w)))
        return int(st.value), int(w.value)

    def tune_dslash_improved(self, F: "PackedLinks", N: "PackedLinks") -> dict:
        """Time the improved operator's variants on (F, N) and keep the fastest;
        returns {(streaming, workgroup size): us} for the timed ones."""
        df, dn = F.desc(), N.desc()
        t = (C.c_double * len(self.TUNE_IMPROVED_VARIANTS))()
        _check(lib().lgt_tune_dslash_improved(self._ctx, C.byref(df), C.byref(dn), t))
        return {v: t[i] for i, v in enumerate(self.TUNE_IMPROVED_VARIANTS) if t[i] >= 0}

    def cg_profile(self) -> dict:
        """Mean times (ms) of the vector kernels of the timed iterations of the last CG with timing on."""
        ms = (C.c_double * 4)()
        n = C.c_int32()
        _check(lib().lgt_cg_profile(self._ctx, ms, C.byref(n)))
        return {"xpay": ms[0], "update": ms[1], "beta_step": ms[2], "alpha_step": ms[3], "iters_timed": int(n.value)}

    def cg_dslash_profile(self) -> dict:
        """Mean kernel times (ms) and counts of the timed Dslash launches of the
        last CG with timing on, by kind (iteration D_oe / D_eo, update D_oe / D_eo)."""
        ms = (C.c_double * 4)()
        n = (C.c_int32 * 4)()
        _check(lib().lgt_cg_dslash_profile(self._ctx, ms, n))
        keys = ("iter_doe", "iter_deo_update", "ru_doe", "ru_deo_residual")
        return {k: {"ms": ms[i], "n": int(n[i])} for i, k in enumerate(keys)}

    BATCH_PHASES = ("setup_and_final", "step1_doe", "wait1", "step2_deo_update", "wait2", "step1_p", "wait1_p",
                    "scalar", "fp64_updates")

    def batch_profile(self) -> dict:
        """Phase times (ms) of the last batched solve launched with timing on from this context."""
        ms = (C.c_double * len(self.BATCH_PHASES))()
        it = C.c_int32()
        _check(lib().lgt_batch_profile(self._ctx, ms, C.byref(it)))
        out = {k: ms[i] for i, k in enumerate(self.BATCH_PHASES)}
        out["iters"] = int(it.value)
        return out

    def set_mrhs_engine(self, engine: int):
        """Multi-RHS Dslash engine: LGT_MRHS_LANE, LGT_MRHS_VALU4 or LGT_MRHS_MFMA."""
        _check(lib().lgt_set_mrhs_engine(self._ctx, int(engine)))

    def mrhs_engine(self) -> int:
        e = C.c_int32()
        _check(lib().lgt_get_mrhs_engine(self._ctx, C.byref(e)))
        return int(e.value)

    def set_mrhs_variant(self, prec: int, recon: int, nrhs: int, engine: int, groups: int = 1):
        _check(lib().lgt_set_mrhs_variant(self._ctx, prec, recon, int(nrhs), int(engine), int(groups)))

    def set_mrhs_staging(self, prec: int, recon: int, nrhs: int, staged: bool):
        """LDS-staged multi-RHS Dslash (four-lane engines) for this format and nrhs."""
        _check(lib().lgt_set_mrhs_staging(self._ctx, prec, recon, int(nrhs), int(bool(staged))))

    def mrhs_staging(self, prec: int, recon: int, nrhs: int) -> bool:
        """Whether lgt_dslash_mrhs runs the staged kernel for this format and nrhs."""
        st = C.c_int32()
        _check(lib().lgt_get_mrhs_staging(self._ctx, prec, recon, int(nrhs), C.byref(st)))
        return bool(st.value)

    def mrhs_variant(self, prec: int, recon: int, nrhs: int) -> tuple[int, int]:
        """(engine, groups of four lanes per site) that lgt_dslash_mrhs runs for this format and nrhs."""
        e, g = C.c_int32(), C.c_int32()
        _check(lib().lgt_get_mrhs_variant(self._ctx, prec, recon, int(nrhs), C.byref(e), C.byref(g)))
        return int(e.value), int(g.value)

    # (engine, groups, LDS-staged) in the order lgt_tune_dslash_mrhs reports them
    MRHS_VARIANTS = tuple((e, g, 0) for e, g in ((LGT_MRHS_LANE, 1), (LGT_MRHS_VALU4, 1), (LGT_MRHS_VALU4, 2),
                                                 (LGT_MRHS_VALU4, 4), (LGT_MRHS_MFMA, 1), (LGT_MRHS_MFMA, 2),
                                                 (LGT_MRHS_MFMA, 4))) + \
        tuple((e, g, 1) for e in (LGT_MRHS_VALU4, LGT_MRHS_MFMA) for g in (1, 2, 4))

    def tune_dslash_mrhs(self, U: "PackedLinks", nrhs: int, report: bool = True):
        """Time every multi-RHS variant on U for nrhs and keep the fastest;
        returns {(engine, groups, staged): us} (variants that do not apply omitted) or None."""
        d = U.desc()
        if not report:
            _check(lib().lgt_tune_dslash_mrhs(self._ctx, C.byref(d), int(nrhs), None))
            return None
        t = (C.c_double * len(self.MRHS_VARIANTS))()
        _check(lib().lgt_tune_dslash_mrhs(self._ctx, C.byref(d), int(nrhs), t))
        return {v: t[i] for i, v in enumerate(self.MRHS_VARIANTS) if t[i] >= 0}

    TUNE_VARIANTS = tuple((h, st, w) for w in (256, 128, 64)
                          for h, st in ((8, 1), (2, 1), (1, 1), (4, 1), (8, 0), (2, 0), (1, 0), (4, 0)))

    def tune_dslash(self, U: "PackedLinks", report: bool = True):
        """Time every variant on U and keep the fastest; returns
        {(hops, streaming, workgroup size): us} or None."""
        d = U.desc()
        if not report:
            _check(lib().lgt_tune_dslash(self._ctx, C.byref(d), None))
            return None
        t = (C.c_double * len(self.TUNE_VARIANTS))()
        _check(lib().lgt_tune_dslash(self._ctx, C.byref(d), t))
        return {v: t[i] for i, v in enumerate(self.TUNE_VARIANTS) if t[i] >= 0}

    # -- helpers
    def _dev(self, t: torch.Tensor, dtype=None, shape=None, what="tensor"):
        if t.device != self.device:
            raise ValueError(f"{what} must be on {self.device}")
        if dtype is not None and t.dtype != dtype:
            raise ValueError(f"{what} must be {dtype}")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        return _ptr(t)

    def vec_shape(self):
        return (self.Vh, 3, 2)

    def native_vec(self, prec: int) -> torch.Tensor:
        dt = torch.float64 if prec == LGT_F64 else torch.float32
        return torch.empty((3, self.Vh, 2), dtype=dt, device=self.device)

    # -- entry points
    def index_maps(self):
        lex = torch.empty(self.V, dtype=torch.int32, device=self.device)
        nbr = torch.empty((2, 8, self.Vh), dtype=torch.int32, device=self.device)
        _check(lib().lgt_index_maps(self._ctx, lex.data_ptr(), nbr.data_ptr()))
        return lex, nbr

    def pack_links(self, U: torch.Tensor, prec: int = LGT_F64, recon: int = LGT_R18) -> PackedLinks:
        p = self._dev(U, torch.float64, (4, self.V, 3, 3, 2), "U")
        out = torch.empty(links_bytes(self.L, prec, recon, self.bc), dtype=torch.uint8, device=self.device)
        _check(lib().lgt_pack_links(self._ctx, p, prec, recon, out.data_ptr()))
        return PackedLinks(out, prec, recon)

    def unpack_links(self, Up: PackedLinks) -> torch.Tensor:
        """The links a packed field holds, canonical float64 [4][V][3][3][2]
        (12-real formats: row 2 rebuilt as the Dslash rebuilds it)."""
        if Up.data.device != self.device:
            raise ValueError(f"packed links must be on {self.device}")
        out = torch.empty((4, self.V, 3, 3, 2), dtype=torch.float64, device=self.device)
        _check(lib().lgt_unpack_links(self._ctx, _ptr(Up.data), Up.prec, Up.recon, out.data_ptr()))
        return out

    def pack_vec(self, v: torch.Tensor, prec: int = LGT_F64) -> torch.Tensor:
        p = self._dev(v, torch.float64, self.vec_shape(), "v")
        out = self.native_vec(prec)
        _check(lib().lgt_pack_vec(self._ctx, prec, p, out.data_ptr()))
        return out

    def unpack_vec(self, n: torch.Tensor, prec: int = LGT_F64) -> torch.Tensor:
        dt = torch.float64 if prec == LGT_F64 else torch.float32
        p = self._dev(n, dt, (3, self.Vh, 2), "native vector")
        out = torch.empty(self.vec_shape(), dtype=torch.float64, device=self.device)
        _check(lib().lgt_unpack_vec(self._ctx, prec, p, out.data_ptr()))
        return out

    def dslash(self, U: PackedLinks, x: torch.Tensor, out_parity: int, out: torch.Tensor | None = None):
        """out = D x for native vectors (precision of U's vectors)."""
        dt = torch.float64 if U.prec == LGT_F64 else torch.float32
        p = self._dev(x, dt, (3, self.Vh, 2), "input vector")
        if out is None:
            out = torch.empty_like(x)
        q = self._dev(out, dt, (3, self.Vh, 2), "output vector")
        d = U.desc()
        _check(lib().lgt_dslash(self._ctx, C.byref(d), int(out_parity), p, q))
        return out

    def apply_normal(self, U: PackedLinks, x: torch.Tensor, mass: float, out: torch.Tensor | None = None):
        """(A x, Re <x, A x>) with A = 4 mass^2 - D_eo D_oe on native even vectors."""
        dt = torch.float64 if U.prec == LGT_F64 else torch.float32
        p = self._dev(x, dt, (3, self.Vh, 2), "input vector")
        if out is None:
            out = torch.empty_like(x)
        q = self._dev(out, dt, (3, self.Vh, 2), "output vector")
        d = U.desc()
        pap = C.c_double()
        _check(lib().lgt_apply_normal(self._ctx, C.byref(d), float(mass), p, q, C.byref(pap)))
        return out, float(pap.value)

    def cg_solve(self, U_hi: PackedLinks, b: torch.Tensor, mass: float, tol: float = 1e-10,
                 scheme: int = LGT_CG_FP64, U_lo: PackedLinks | None = None, ru_interval: int = 50,
                 inner_tol: float = 0.0, max_iter: int = 100000, x0: torch.Tensor | None = None,
                 check_interval: int = 0, raise_on_fail: bool = True):
        pb = self._dev(b, torch.float64, self.vec_shape(), "b")
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        px = self._dev(x, torch.float64, self.vec_shape(), "x")
        prm = _CgParams(float(mass), float(tol), int(max_iter), int(scheme), int(ru_interval),
                        int(x0 is not None), float(inner_tol), int(check_interval), 0)
        res = _CgResult()
        dhi = U_hi.desc()
        dlo = U_lo.desc() if U_lo is not None else None
        st = lib().lgt_cg_solve(self._ctx, C.byref(dhi), C.byref(dlo) if dlo is not None else None,
                                C.byref(prm), pb, px, C.byref(res))
        r = CgResult(*(getattr(res, f[0]) for f in _CgResult._fields_))
        if st != 0 and (raise_on_fail or st not in (-5, -6)):
            _check(st)
        return x, r

    # -- HMC step: fields are canonical [4][V][3][3][2] float64 tensors
    def _field(self, t, what):
        return self._dev(t, torch.float64, (4, self.V, 3, 3, 2), what)

    def gauge_force(self, U: torch.Tensor, beta: float, scale: float = 1.0, G: torch.Tensor | None = None,
                    accumulate: bool = False) -> torch.Tensor:
        """G (+)= scale * dS_g/dU for the Wilson action with coupling beta."""
        pu = self._field(U, "U")
        if G is None:
            G = torch.zeros_like(U) if accumulate else torch.empty_like(U)
        pg = self._field(G, "G")
        _check(lib().lgt_gauge_force(self._ctx, pu, float(beta), float(scale), int(bool(accumulate)), pg))
        return G

    def momentum_update(self, U: torch.Tensor, G: torch.Tensor, eps: float, P: torch.Tensor) -> torch.Tensor:
        _check(lib().lgt_momentum_update(self._ctx, self._field(U, "U"), self._field(G, "G"), float(eps),
                                         self._field(P, "P")))
        return P

    def link_update(self, P: torch.Tensor, eps: float, U: torch.Tensor) -> torch.Tensor:
        _check(lib().lgt_link_update(self._ctx, self._field(P, "P"), float(eps), self._field(U, "U")))
        return U

    def fatten_links(self, U: torch.Tensor, coeffs=None, F: torch.Tensor | None = None,
                     N: torch.Tensor | None = None):
        """(F, N), the fat one-link and Naik fields of the improved operator, from
        the canonical gauge field U; coeffs = (one link, 3-, 5-, 7-link staples,
        Lepage, Naik), asqtad_coeffs() by default."""
        w = _FatCoeffs(*(float(c) for c in (coeffs if coeffs is not None else asqtad_coeffs())))
        pu = self._field(U, "U")
        F = torch.empty_like(U) if F is None else F
        N = torch.empty_like(U) if N is None else N
        _check(lib().lgt_fatten_links(self._ctx, pu, C.byref(w), self._field(F, "F"), self._field(N, "N")))
        return F, N

    def fatten_links_vjp(self, U: torch.Tensor, G_fat: torch.Tensor, G_naik: torch.Tensor, coeffs=None,
                         scale: float = 1.0, G: torch.Tensor | None = None, accumulate: bool = False):
        """G (+)= scale * dS/dU from G_fat = dS/dF and G_naik = dS/dN through the
        fattening with coeffs (asqtad_coeffs() by default); canonical fields."""
        w = _FatCoeffs(*(float(c) for c in (coeffs if coeffs is not None else asqtad_coeffs())))
        if G is None:
            G = torch.zeros_like(U) if accumulate else torch.empty_like(U)
        _check(lib().lgt_fatten_links_vjp(self._ctx, self._field(U, "U"), C.byref(w), self._field(G_fat, "G_fat"),
                                          self._field(G_naik, "G_naik"), float(scale), int(bool(accumulate)),
                                          self._field(G, "G")))
        return G

    def plaquette(self, U: torch.Tensor) -> float:
        out = C.c_double()
        _check(lib().lgt_plaquette(self._ctx, self._field(U, "U"), C.byref(out)))
        return float(out.value)

    def kinetic_energy(self, P: torch.Tensor) -> float:
        out = C.c_double()
        _check(lib().lgt_kinetic_energy(self._ctx, self._field(P, "P"), C.byref(out)))
        return float(out.value)

    def hmc_trajectory(self, U: torch.Tensor, P: torch.Tensor, R_e: torch.Tensor, R_o: torch.Tensor, beta: float,
                       mass: float, eps: float, nsteps: int, u: float, tol: float = 1e-10,
                       scheme: int = LGT_CG_FP64) -> dict:
        """One HMC trajectory; U and P are updated in place (restored if rejected)."""
        prm = _HmcParams(float(beta), float(mass), float(eps), float(tol), float(u), int(nsteps), int(scheme))
        res = _HmcResult()
        _check(lib().lgt_hmc_trajectory(self._ctx, self._field(U, "U"), self._field(P, "P"),
                                        self._dev(R_e, torch.float64, self.vec_shape(), "R_e"),
                                        self._dev(R_o, torch.float64, self.vec_shape(), "R_o"),
                                        C.byref(prm), C.byref(res)))
        return {f[0]: getattr(res, f[0]) for f in _HmcResult._fields_ if f[0] != "reserved"}

    def hmc_trajectory_improved(self, U: torch.Tensor, P: torch.Tensor, R_e: torch.Tensor, R_o: torch.Tensor,
                                beta: float, mass: float, eps: float, nsteps: int, u: float, coeffs=None,
                                tol: float = 1e-10, scheme: int = LGT_CG_FP64) -> dict:
        """hmc_trajectory with the improved operator of the fattened fields
        (coeffs: asqtad_coeffs() by default)."""
        w = _FatCoeffs(*(float(c) for c in (coeffs if coeffs is not None else asqtad_coeffs())))
        prm = _HmcParams(float(beta), float(mass), float(eps), float(tol), float(u), int(nsteps), int(scheme))
        res = _HmcResult()
        _check(lib().lgt_hmc_trajectory_improved(self._ctx, self._field(U, "U"), self._field(P, "P"),
                                                 self._dev(R_e, torch.float64, self.vec_shape(), "R_e"),
                                                 self._dev(R_o, torch.float64, self.vec_shape(), "R_o"),
                                                 C.byref(prm), C.byref(w), C.byref(res)))
        return {f[0]: getattr(res, f[0]) for f in _HmcResult._fields_ if f[0] != "reserved"}

    # -- improved (fat + Naik) operator
    def dslash_improved(self, F: PackedLinks, N: PackedLinks, x: torch.Tensor, out_parity: int,
                        out: torch.Tensor | None = None):
        """out = D x with the improved operator (fat F, Naik N: same 18-real format)."""
        dt = torch.float64 if F.prec == LGT_F64 else torch.float32
        p = self._dev(x, dt, (3, self.Vh, 2), "input vector")
        if out is None:
            out = torch.empty_like(x)
        q = self._dev(out, dt, (3, self.Vh, 2), "output vector")
        df, dn = F.desc(), N.desc()
        _check(lib().lgt_dslash_improved(self._ctx, C.byref(df), C.byref(dn), int(out_parity), p, q))
        return out

    def cg_solve_improved(self, F_hi: PackedLinks, N_hi: PackedLinks, b: torch.Tensor, mass: float,
                          tol: float = 1e-10, scheme: int = LGT_CG_FP64, F_lo: PackedLinks | None = None,
                          N_lo: PackedLinks | None = None, ru_interval: int = 50, inner_tol: float = 0.0,
                          max_iter: int = 100000, raise_on_fail: bool = True):
        pb = self._dev(b, torch.float64, self.vec_shape(), "b")
        x = torch.zeros_like(b)
        px = self._dev(x, torch.float64, self.vec_shape(), "x")
        prm = _CgParams(float(mass), float(tol), int(max_iter), int(scheme), int(ru_interval), 0,
                        float(inner_tol), 0, 0)
        res = _CgResult()
        dfh, dnh = F_hi.desc(), N_hi.desc()
        dfl = F_lo.desc() if F_lo is not None else None
        dnl = N_lo.desc() if N_lo is not None else None
        st = lib().lgt_cg_solve_improved(self._ctx, C.byref(dfh), C.byref(dnh),
                                         C.byref(dfl) if dfl is not None else None,
                                         C.byref(dnl) if dnl is not None else None, C.byref(prm), pb, px,
                                         C.byref(res))
        r = CgResult(*(getattr(res, f[0]) for f in _CgResult._fields_))
        if st != 0 and (raise_on_fail or st not in (-5, -6)):
            _check(st)
        return x, r

    # -- many right-hand sides
    def pack_vec_mrhs(self, v: torch.Tensor, prec: int = LGT_F64) -> torch.Tensor:
        """canonical [N][V/2][3][2] float64 -> native multi-RHS [3][V/2][N][2]."""
        n = int(v.shape[0])
        p = self._dev(v, torch.float64, (n,) + self.vec_shape(), "v")
        dt = torch.float64 if prec == LGT_F64 else torch.float32
        out = torch.empty((3, self.Vh, n, 2), dtype=dt, device=self.device)
        _check(lib().lgt_pack_vec_mrhs(self._ctx, prec, n, p, out.data_ptr()))
        return out

    def unpack_vec_mrhs(self, nv: torch.Tensor, prec: int = LGT_F64) -> torch.Tensor:
        n = int(nv.shape[2])
        dt = torch.float64 if prec == LGT_F64 else torch.float32
        p = self._dev(nv, dt, (3, self.Vh, n, 2), "native vector")
        out = torch.empty((n,) + self.vec_shape(), dtype=torch.float64, device=self.device)
        _check(lib().lgt_unpack_vec_mrhs(self._ctx, prec, n, p, out.data_ptr()))
        return out

    def dslash_mrhs(self, U: PackedLinks, x: torch.Tensor, out_parity: int, out: torch.Tensor | None = None):
        """out = D x for every right-hand side of a native multi-RHS vector."""
        dt = torch.float64 if U.prec == LGT_F64 else torch.float32
        n = int(x.shape[2])
        p = self._dev(x, dt, (3, self.Vh, n, 2), "input vector")
        if out is None:
            out = torch.empty_like(x)
        q = self._dev(out, dt, (3, self.Vh, n, 2), "output vector")
        d = U.desc()
        _check(lib().lgt_dslash_mrhs(self._ctx, C.byref(d), int(out_parity), n, p, q))
        return out

    def stream_copy(self, src: torch.Tensor, dst: torch.Tensor):
        """dst[:] = src[:] with the library's streaming copy kernel (bandwidth probe)."""
        n = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() < n:
            raise ValueError("dst too small")
        _check(lib().lgt_stream_copy(self._ctx, self._dev(src, None, None, "src"),
                                     self._dev(dst, None, None, "dst"), n))

    def stream_read(self, src: torch.Tensor, sink: torch.Tensor):
        """Read all of src with streaming loads (read-bandwidth probe); sink: >= 16 bytes."""
        if sink.numel() * sink.element_size() < 16:
            raise ValueError("sink must hold 16 bytes")
        _check(lib().lgt_stream_read(self._ctx, self._dev(src, None, None, "src"),
                                     src.numel() * src.element_size(), self._dev(sink, None, None, "sink")))

    def stream_read_links(self, U: PackedLinks, out_parity: int, streaming: int, sink: torch.Tensor):
        """Read the 8 links of every site of out_parity as the Dslash does, nothing else (probe)."""
        if sink.numel() * sink.element_size() < 8:
            raise ValueError("sink must hold 8 bytes")
        d = U.desc()
        _check(lib().lgt_stream_read_links(self._ctx, C.byref(d), int(out_parity), int(streaming),
                                           self._dev(sink, None, None, "sink")))

    def cdot(self, a: torch.Tensor, b: torch.Tensor) -> complex:
        if a.numel() != b.numel() or a.numel() % 2:
            raise ValueError("cdot needs two float64 tensors of equal even size")
        pa = self._dev(a, torch.float64, None, "a")
        pb = self._dev(b, torch.float64, None, "b")
        out = (C.c_double * 2)()
        _check(lib().lgt_cdot(self._ctx, a.numel() // 2, pa, pb, out))
        return complex(out[0], out[1])

    def force(self, U: PackedLinks, X: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
        px = self._dev(X, torch.float64, self.vec_shape(), "X")
        G = torch.empty((4, self.V, 3, 3, 2), dtype=torch.float64, device=self.device)
        d = U.desc()
        _check(lib().lgt_force(self._ctx, C.byref(d), px, float(scale), G.data_ptr()))
        return G

    def action_phi_grad(self, X: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
        """scale * dS/d(Re phi, Im phi) = 2 scale X for S = phi^dag A^-1 phi, X = A^-1 phi."""
        px = self._dev(X, torch.float64, self.vec_shape(), "X")
        g = torch.empty_like(X)
        _check(lib().lgt_action_phi_grad(self._ctx, px, float(scale), g.data_ptr()))
        return g

    def force_improved(self, F: PackedLinks, N: PackedLinks, X: torch.Tensor, scale: float = 1.0):
        """(G_fat, G_naik) = scale * dS/d(Re, Im) of the improved operator's two link fields."""
        px = self._dev(X, torch.float64, self.vec_shape(), "X")
        GF = torch.empty((4, self.V, 3, 3, 2), dtype=torch.float64, device=self.device)
        GN = torch.empty_like(GF)
        df, dn = F.desc(), N.desc()
        _check(lib().lgt_force_improved(self._ctx, C.byref(df), C.byref(dn), px, float(scale), GF.data_ptr(),
                                        GN.data_ptr()))
        return GF, GN


# Table 1 routines: id, operand kinds (a, b, c) and flop per call (a mat-vec
# is 36 multiplications + 30 additions = 66 flop, Sec. 4)
ROUTINES = {
    "add_su3_vector": (1, "vec", "vec", "vec", 6),
    "mult_adj_su3_mat_vec": (3, "mat", "vec", "vec", 66),
    "mult_adj_su3_mat_vec_4dir": (4, "vec", "mat4", "vec4", 264),
    "mult_adj_su3_mat_4vec": (5, "mat4", "vec", "vec4", 264),
    "mult_su3_an": (6, "mat", "mat", "mat", 198),
    "mult_su3_na": (8, "mat", "mat", "mat", 198),
    "mult_su3_nn": (9, "mat", "mat", "mat", 198),
    "mult_su3_mat_vec": (10, "mat", "vec", "vec", 66),
    "mult_su3_mat_vec_sum_4dir": (11, "mat4", "vec4", "vec", 282),
    "scalar_mult_add_su3_matrix": (12, "mat", "mat", "mat", 36),
    "scalar_mult_add_su3_vector": (13, "vec", "vec", "vec", 12),
    "su3_projector": (14, "vec", "vec", "mat", 54),
    "sub_four_su3_vecs": (15, "vec", "vec4", "vec", 24),
}
# complex numbers per call of each operand kind
PLANES = {"vec": 3, "mat": 9, "vec4": 12, "mat4": 36}


def routine(lat: "Lattice", name: str, a: torch.Tensor, b: torch.Tensor, s: float = 0.0,
            out: torch.Tensor | None = None) -> torch.Tensor:
    """One Table 1 routine over n calls: operands are [planes][n][2] real tensors
    (float64 or float32) on the lattice's device; returns c."""
    rid, ka, kb, kc, _ = ROUTINES[name]
    n = int(a.shape[1])
    dt = a.dtype
    if dt not in (torch.float64, torch.float32):
        raise LgtError(-1, "operands must be float64 or float32")
    pa = lat._dev(a, dt, (PLANES[ka], n, 2), "a")
    pb = lat._dev(b, dt, (PLANES[kb], n, 2), "b")
    if out is None:
        out = torch.empty((PLANES[kc], n, 2), dtype=dt, device=lat.device)
    pc = lat._dev(out, dt, (PLANES[kc], n, 2), "c")
    prec = LGT_F64 if dt == torch.float64 else LGT_F32
    _check(lib().lgt_routine(lat._ctx, rid, prec, n, pa, pb, pc, float(s)))
    return out


def cg_solve_batch(problems, mass: float, tol: float = 1e-10, scheme: int = LGT_CG_RELIABLE,
                   ru_interval: int = 50, inner_tol: float = 0.0, max_iter: int = 100000,
                   raise_on_fail: bool = True):
    """Independent CGs for every right-hand side of every problem: one persistent launch, or
    (mixed precision, four-lane inner engines, one problem or up to four on different
    contexts) the same iteration as kernel launches, problems on their own streams.

    problems: list of (lattice, U_hi, U_lo, b) with b a float64 tensor [N][V/2][3][2]
    (1 <= N <= 16). Returns ([x per problem], [[CgResult per rhs] per problem]).
    """
    keep, descs, xs, results = [], [], [], []
    arr = (_CgProblem * len(problems))()
    for i, (lat, U_hi, U_lo, b) in enumerate(problems):
        n = int(b.shape[0])
        lat._dev(b, torch.float64, (n,) + lat.vec_shape(), "b")
        x = torch.zeros_like(b)
        dh = U_hi.desc()
        dl = U_lo.desc() if U_lo is not None else None
        res = (_CgResult * n)()
        keep += [dh, dl, res]
        arr[i].ctx = lat._ctx
        arr[i].U_hi = C.pointer(dh)
        arr[i].U_lo = C.pointer(dl) if dl is not None else None
        arr[i].nrhs = n
        arr[i].b = b.data_ptr()
        arr[i].x = x.data_ptr()
        arr[i].res = res
        xs.append(x)
        results.append(res)
    prm = _CgParams(float(mass), float(tol), int(max_iter), int(scheme), int(ru_interval), 0,
                    float(inner_tol), 0, 0)
    st = lib().lgt_cg_solve_batch(arr, len(problems), C.byref(prm))
    out = [[CgResult(*(getattr(r, f[0]) for f in _CgResult._fields_)) for r in res] for res in results]
    if st != 0 and (raise_on_fail or st not in (-5, -6)):
        _check(st)
    return xs, out


class PseudofermionAction(torch.autograd.Function):
    """S = phi^dag A^-1 phi with A = 4 m^2 - D_eo D_oe, differentiable in U (and phi).

    forward: X = A^-1 phi by the library's CG, S = Re <phi, X>; the FP64 CG by
    default, or with mixed=True the FP32 x 12 inner CG with FP64 reliable
    updates (same FP64 true-residual stop, so S and dS/dU agree to O(tol)).
    backward: dS/dU from the fermion-force kernel, reusing the saved X.
    U: float64 [4][V][3][3][2] (real view of the complex links), phi: [V/2][3][2].
    """

    @staticmethod
    def forward(ctx, U, phi, lat: Lattice, mass: float, tol: float = 1e-12, max_iter: int = 100000,
                mixed: bool = False):
        Up = lat.pack_links(U.detach(), LGT_F64, LGT_R18)
        if mixed:
            Ul = lat.pack_links(U.detach(), LGT_F32, LGT_R12)
            X, res = lat.cg_solve(Up, phi.detach(), mass, tol=tol, max_iter=max_iter, scheme=LGT_CG_RELIABLE,
                                  U_lo=Ul)
            del Ul
        else:
            X, res = lat.cg_solve(Up, phi.detach(), mass, tol=tol, max_iter=max_iter)
        S = lat.cdot(phi.detach(), X).real
        ctx.lat = lat
        ctx.Up = Up
        ctx.res = res
        ctx.save_for_backward(X)
        return torch.tensor(S, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, gS):
        (X,) = ctx.saved_tensors
        g = float(gS.item())
        gU = ctx.lat.force(ctx.Up, X, scale=g) if ctx.needs_input_grad[0] else None
        gphi = ctx.lat.action_phi_grad(X, scale=g) if ctx.needs_input_grad[1] else None
        return gU, gphi, None, None, None, None, None


class ImprovedPseudofermionAction(torch.autograd.Function):
    """S = phi^dag A^-1 phi for the improved operator (fat F + Naik N),
    differentiable in F, N (and phi): the forward solve by the library's FP64
    improved CG, the backward from its improved fermion-force kernel with the
    saved X. F, N: float64 [4][V][3][3][2]; phi: [V/2][3][2]."""

    @staticmethod
    def forward(ctx, F, N, phi, lat: Lattice, mass: float, tol: float = 1e-12, max_iter: int = 100000):
        Fp = lat.pack_links(F.detach(), LGT_F64, LGT_R18)
        Np = lat.pack_links(N.detach(), LGT_F64, LGT_R18)
        X, res = lat.cg_solve_improved(Fp, Np, phi.detach(), mass, tol=tol, max_iter=max_iter)
        S = lat.cdot(phi.detach(), X).real
        ctx.lat, ctx.Fp, ctx.Np, ctx.res = lat, Fp, Np, res
        ctx.save_for_backward(X)
        return torch.tensor(S, dtype=torch.float64, device=F.device)

    @staticmethod
    def backward(ctx, gS):
        (X,) = ctx.saved_tensors
        g = float(gS.item())
        gF = gN = None
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            gF, gN = ctx.lat.force_improved(ctx.Fp, ctx.Np, X, scale=g)
            gF = gF if ctx.needs_input_grad[0] else None
            gN = gN if ctx.needs_input_grad[1] else None
        gphi = ctx.lat.action_phi_grad(X, scale=g) if ctx.needs_input_grad[2] else None
        return gF, gN, gphi, None, None, None, None
