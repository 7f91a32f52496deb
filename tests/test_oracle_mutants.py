"""Plant plausible mistakes in a copy of the oracle and check that the pins catch each.

Every mutant is a one-line textual change of oracle/lgt_oracle.c compiled into
a temporary library (CPU only). The test passes when at least one pin fails on
every mutant, i.e. the pins are strong enough to notice a dropped term, a wrong
sign, a wrong index or a transposed operand.
"""
import ctypes
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
import test_oracle_improved as ipins
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "lgt_oracle.c")

MUTANTS = {
    # transposed operand in the forward mat-vec
    "transpose_fwd": ("const or_cx a = A[3 * i + j];", "const or_cx a = A[3 * j + i];"),
    # sign error in Eq (2.x): + instead of -
    "adj_sign": ("im += a.re * b[j].im - a.im * b[j].re; /* (2.1)-(2.3) */",
                 "im += a.re * b[j].im + a.im * b[j].re; /* (2.1)-(2.3) */"),
    # dropped backward half
    "drop_backward": ("or_sub_four_su3_vecs(fwd, back);", "(void)back;"),
    # backward link taken from the output site instead of x - mu
    "bwd_link_index": ("link_at(U, V, mu, in_par * Vh + cbm)", "link_at(U, V, mu, out_par * Vh + cb)"),
    # staggered phase includes its own direction
    "eta_index": ("for (int nu = 0; nu < mu; nu++) s += c[nu];",
                  "for (int nu = 0; nu <= mu; nu++) s += c[nu];"),
    # lower-boundary sign tested on the wrong face
    "bc_face": ("return (c[mu] == 0) ? (double)bc[mu] : 1.0;",
                "return (c[mu] == 1) ? (double)bc[mu] : 1.0;"),
    # neighbour in the wrong direction for the forward hop
    "fwd_dir": ("chi + 3 * nbr_cb(L, c, mu, +1)", "chi + 3 * nbr_cb(L, c, mu, -1)"),
    # mass term with the wrong factor
    "mass_factor": ("const double m4 = 4.0 * mass * mass;", "const double m4 = 2.0 * mass * mass;"),
    # force: sign of the odd-site term
    "force_sign": ("const double sg = par == 0 ? s : -s;", "const double sg = s;"),
    # improved operator: Naik backward link taken at the output site
    "naik_bwd_link": ("link_at(N, V, mu, in_par * Vh + cbm3)", "link_at(N, V, mu, out_par * Vh + cb)"),
    # improved operator: one crossing too few counted for the forward three-step hop
    "naik_crossings": ("(c[mu] + 3) / L[mu]", "(c[mu] + 2) / L[mu]"),
    # improved operator: dropped Naik backward hop
    "naik_drop_bwd": ("or_scalar_mult_add_su3_vector(acc, t, -e * s3(L, bc, c, mu, -1), acc);",
                      "or_scalar_mult_add_su3_vector(acc, t, 0.0 * e, acc);"),
    # improved operator: two-step instead of three-step neighbours
    "naik_distance": ("d[mu] = ((d[mu] + 3 * dir) % L[mu] + L[mu]) % L[mu];",
                      "d[mu] = ((d[mu] + 2 * dir) % L[mu] + L[mu]) % L[mu];"),
    # improved operator: backward Naik hop without the adjoint
    "naik_force_sign": ("const double s = 2.0 * eta(c, mu) * (naik ? s3(L, bc, c, mu, +1) : s_plus(L, bc, c, mu));",
                        "const double s = 2.0 * eta(c, mu) * (naik ? -s3(L, bc, c, mu, +1) : s_plus(L, bc, c, mu));"),
    "naik_force_distance": ("const int64_t cbp = naik ? nbr3_cb(L, c, mu, +1) : nbr_cb(L, c, mu, +1);",
                            "const int64_t cbp = nbr_cb(L, c, mu, +1);"),
    "naik_no_adjoint": ("or_mult_adj_su3_mat_vec(link_at(N, V", "or_mult_su3_mat_vec(link_at(N, V"),
}


def _build_mutant(tmp, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = os.path.join(tmp, f"m_{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    shutil.copy(os.path.join(os.path.dirname(SRC), "lgt_oracle.h"), tmp)
    so = os.path.join(tmp, f"m_{name}.so")
    subprocess.run(["gcc", "-std=c99", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", so, path, "-lm"],
                   check=True)
    lib = ctypes.CDLL(so)
    oracle._setup(lib)
    return lib


def _pins():
    yield lambda: pins.test_table1_routines_vs_numpy(0)
    yield lambda: pins.test_free_field_plane_wave_eigenvalue((4, 6, 4, 8), (1, 2, 3, 1), (1, 1, 1, 1))
    yield lambda: pins.test_free_field_plane_wave_eigenvalue((4, 4, 4, 8), (1, 1, 0, 0.5), (1, 1, 1, -1))
    yield lambda: pins.test_dslash_antihermitian((1, 1, 1, -1))
    yield lambda: pins.test_dslash_gauge_covariance((1, 1, 1, 1))
    yield lambda: pins.test_dslash_dense_brute_force((2, 4, 2, 6), (1, 1, 1, -1))
    yield lambda: pins.test_cg_vs_dense_solve((2, 4, 2, 6), 0.05, "expih")
    yield lambda: pins.test_force_vs_dense_central_differences((2, 4, 2, 4), (1, 1, 1, 1))
    yield lambda: ipins.test_improved_antihermitian((8, 4, 6, 4), (1, 1, 1, -1))
    yield lambda: ipins.test_improved_free_field_plane_wave((8, 8, 8, 8), (1, 2, 0, 1.5), (1, 1, 1, -1))
    yield lambda: ipins.test_improved_gauge_covariance((1, -1, 1, -1))
    yield lambda: ipins.test_improved_dense_brute_force((8, 4, 2, 8), (1, 1, 1, -1))
    yield ipins.test_improved_cg_vs_dense_solve
    yield lambda: ipins.test_improved_force_central_differences((1, 1, 1, -1))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, monkeypatch):
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(tmp, name, *MUTANTS[name])
        monkeypatch.setattr(oracle, "_lib", lib)
        caught = 0
        for pin in _pins():
            try:
                pin()
            except AssertionError:
                caught += 1
        assert caught >= 1, f"no pin noticed mutant {name}"


def test_unmutated_copy_passes_all_pins(monkeypatch):
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(tmp, "none", "or_set_threads(int n)", "or_set_threads(int n)")
        monkeypatch.setattr(oracle, "_lib", lib)
        for pin in _pins():
            pin()
