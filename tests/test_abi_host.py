"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad arguments on the host before launching anything."""
import ctypes as C

import pytest

import paper_1309_0551_amd as P
from paper_1309_0551_amd import lgt as B


def test_library_exports_every_declared_symbol():
    declared = B.exported_symbols_declared()
    assert "lgt_dslash" in declared and "lgt_cg_solve" in declared and "lgt_force" in declared
    missing = [n for n in declared if not hasattr(P.lib(), n)]
    assert not missing, missing


def test_status_strings():
    l = P.lib()
    for code in range(-8, 1):
        s = l.lgt_status_string(code).decode()
        assert s and s != "unknown status"
    assert l.lgt_status_string(-99).decode() == "unknown status"


@pytest.mark.parametrize("L,bc,ok", [
    ((4, 4, 4, 4), (1, 1, 1, 1), True),
    ((2, 2, 2, 2), (1, 1, 1, -1), True),
    ((32, 32, 32, 32), (1, 1, 1, 1), True),
    ((3, 4, 4, 4), (1, 1, 1, 1), False),
    ((4, 4, 0, 4), (1, 1, 1, 1), False),
    ((4, 4, 4, 4), (1, 1, 1, 0), False),
    ((2048, 2048, 2048, 2), (1, 1, 1, 1), False),  # > 2^31 sites
])
def test_geometry_validation(L, bc, ok):
    assert (P.geom_check(L, bc) == 0) == ok
    if not ok:
        assert P.geom_check(L, bc) == -2


def test_sizes():
    L = (32, 32, 32, 32)
    V = 32 ** 4
    assert P.links_bytes(L, P.LGT_F64, P.LGT_R18) == V * 4 * 144
    assert P.links_bytes(L, P.LGT_F32, P.LGT_R12) == V * 4 * 48
    assert P.links_bytes(L, P.LGT_BF16, P.LGT_R12) == V * 4 * 24
    assert P.vec_bytes(L, P.LGT_F64) == V // 2 * 48
    assert P.vec_bytes(L, P.LGT_BF16) == V // 2 * 24
    with pytest.raises(P.LgtError) as e:
        P.links_bytes(L, P.LGT_BF16, P.LGT_R18)
    assert e.value.status == -8


def _geom(L):
    return B._geom(L, (1, 1, 1, 1))


def test_create_checks_geometry_before_device():
    ctx = C.c_void_p()
    st = P.lib().lgt_create(C.byref(_geom((5, 4, 4, 4))), 0, None, C.byref(ctx))
    assert st == -2
    assert "even" in P.lib().lgt_last_error().decode()


def test_create_without_gpu_reports_device_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = C.c_void_p()
    st = P.lib().lgt_create(C.byref(_geom((4, 4, 4, 4))), 0, None, C.byref(ctx))
    assert st == -4
    assert not ctx


def test_null_context_and_args_rejected():
    l = P.lib()
    assert l.lgt_destroy(None) == -1
    assert l.lgt_set_timing(None, 1) == -1
    assert l.lgt_dslash(None, None, 0, None, None) == -1
    assert l.lgt_cg_solve(None, None, None, None, None, None, None) == -1
    assert l.lgt_force(None, None, None, 1.0, None) == -1
    assert l.lgt_cdot(None, 1, None, None, None) == -1
    assert l.lgt_links_bytes(C.byref(_geom((4, 4, 4, 4))), 0, 18, None) == -1


def test_param_struct_layout_matches_header():
    assert C.sizeof(B._CgParams) == 48
    assert C.sizeof(B._CgResult) == 56
    assert C.sizeof(B._Links) == 16
    assert C.sizeof(B._Geom) == 32


def test_flop_constant():
    assert P.DSLASH_FLOP_PER_SITE == 570


def test_build_entry_resolves_both_builders():
    """build() compiles the library and the oracle; its two steps are the
    build scripts' functions, loaded without importing the package (which
    would load a possibly missing or stale liblgt.so before rebuilding it)."""
    import importlib
    import os
    import subprocess
    import sys
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..")
    sys.path.insert(0, root)
    ge = importlib.import_module("__graft_entry__")
    lib_b, or_b = ge._builders()
    assert callable(lib_b) and callable(or_b)
    assert lib_b.__globals__["__file__"].endswith(os.path.join("paper_1309_0551_amd", "build.py"))
    assert or_b.__globals__["__file__"].endswith(os.path.join("oracle", "build.py"))
    assert callable(ge.smoke)
    code = ("import sys, __graft_entry__ as g; g._builders(); "
            "print('paper_1309_0551_amd' in sys.modules, 'oracle' in sys.modules)")
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, check=True)
    assert out.stdout.split() == ["False", "False"]


def test_every_context_call_rejects_a_null_context():
    """Every entry point that takes a context returns LGT_ERR_ARG for NULL,
    on the host, before any device work."""
    l = P.lib()
    d = C.c_double()
    i = C.c_int32()
    calls = {
        "lgt_index_maps": (None, None, None),
        "lgt_pack_links": (None, None, 0, 18, None),
        "lgt_pack_vec": (None, 0, None, None),
        "lgt_unpack_vec": (None, 0, None, None),
        "lgt_set_dslash_variant": (None, 0, 18, 8, 1),
        "lgt_get_dslash_variant": (None, 0, 18, C.byref(i), C.byref(i)),
        "lgt_tune_dslash": (None, None, None),
        "lgt_apply_normal": (None, None, 0.1, None, None, C.byref(d)),
        "lgt_stream_copy": (None, None, None, 16),
        "lgt_stream_read": (None, None, 16, None),
        "lgt_pack_vec_mrhs": (None, 1, 4, None, None),
        "lgt_unpack_vec_mrhs": (None, 1, 4, None, None),
        "lgt_dslash_mrhs": (None, None, 0, 4, None, None),
        "lgt_set_mrhs_engine": (None, 0),
        "lgt_get_mrhs_engine": (None, C.byref(i)),
        "lgt_set_mrhs_variant": (None, 1, 12, 4, 0, 1),
        "lgt_get_mrhs_variant": (None, 1, 12, 4, C.byref(i), C.byref(i)),
        "lgt_tune_dslash_mrhs": (None, None, 4, None),
        "lgt_dslash_improved": (None, None, None, 0, None, None),
        "lgt_cg_solve_improved": (None, None, None, None, None, None, None, None, None),
        "lgt_routine": (None, 1, 0, 16, None, None, None, 1.0),
        "lgt_gauge_force": (None, None, 5.6, 1.0, 0, None),
        "lgt_momentum_update": (None, None, None, 0.1, None),
        "lgt_link_update": (None, None, 0.1, None),
        "lgt_plaquette": (None, None, C.byref(d)),
        "lgt_kinetic_energy": (None, None, C.byref(d)),
        "lgt_hmc_trajectory": (None, None, None, None, None, None, None),
        "lgt_fatten_links": (None, None, None, None, None),
        "lgt_fatten_links_vjp": (None, None, None, None, None, 1.0, 0, None),
        "lgt_set_dslash_improved_variant": (None, 0, 1, 256),
        "lgt_set_mrhs_staging": (None, 1, 12, 16, 1),
        "lgt_get_mrhs_staging": (None, 1, 12, 16, C.byref(i)),
        "lgt_get_dslash_improved_variant": (None, 0, C.byref(i), C.byref(i)),
        "lgt_tune_dslash_improved": (None, None, None, None),
        "lgt_hmc_trajectory_improved": (None, None, None, None, None, None, None, None),
        "lgt_unpack_links": (None, None, 0, 18, None),
        "lgt_action_phi_grad": (None, None, 1.0, None),
        "lgt_force_noalloc": (None, None, None, 1.0, None),
        "lgt_stream_read_links": (None, None, 1, 1, None),
        "lgt_set_dslash_workgroup": (None, 0, 18, 64),
        "lgt_get_dslash_workgroup": (None, 0, 18, C.byref(i)),
        "lgt_batch_profile": (None, (C.c_double * 9)(), C.byref(i)),
        "lgt_cg_profile": (None, (C.c_double * 4)(), C.byref(i)),
        "lgt_cg_dslash_profile": (None, (C.c_double * 4)(), (C.c_int32 * 4)()),
    }
    for name, args in calls.items():
        assert getattr(l, name)(*args) == -1, name
    # no problems / a NULL problem list
    assert l.lgt_cg_solve_batch(None, 0, None) == -1


def test_asqtad_coeffs_from_the_library():
    """lgt_asqtad_coeffs: the tree-level weights at u0 = 1 exactly, a path of n
    links divided by u0^(n-1) otherwise (against the oracle's table), and bad
    u0 rejected on the host."""
    from oracle import fatten as ofat

    assert P.asqtad_coeffs(1.0) == (5.0 / 8.0, 1.0 / 16.0, 1.0 / 64.0, 1.0 / 384.0, -1.0 / 16.0, -1.0 / 24.0)
    for u0 in (0.9, 0.8751, 1.3):
        got, want = P.asqtad_coeffs(u0), ofat.asqtad_coeffs(u0)
        for a, b in zip(got, want):
            assert abs(a - b) <= 4e-16 * abs(b), (u0, got, want)
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(P.LgtError):
            P.asqtad_coeffs(bad)
