"""Host check of the z-blocked XCD tile order of the multi-RHS kernels: for
every lattice, tile size and XCD grid (kz z ranges x 8/kz t ranges) it applies
to, the blocks of the eight XCDs cover each tile exactly once, each XCD's
tiles of a t-slice are one contiguous range of positions (a range of z
planes), and its slices one contiguous t range, walked t-major. Compiles the
header's host path."""
import shutil
import subprocess

import pytest

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

PROG = r"""
#include <cstdio>
#include <vector>
#include "geom.hpp"
using namespace lgt;
int main() {
    const int Ls[][4] = {{24, 24, 24, 48}, {32, 32, 32, 32}, {16, 16, 16, 32}, {12, 12, 12, 12},
                         {8, 8, 8, 8}, {6, 10, 14, 18}, {4, 4, 4, 4}, {64, 2, 2, 30}, {2, 2, 2, 2}};
    int applied = 0;
    for (auto &L : Ls) {
        Geom g{};
        for (int m = 0; m < 4; m++) { g.L[m] = L[m]; g.bc[m] = 1; }
        g.hx = L[0] / 2;
        g.Vh = L[0] * L[1] * L[2] * L[3] / 2;
        for (int kz = 8; kz >= 1; kz /= 2)
        for (int T = 1; T <= 256; T *= 2) {
            const TileOrder o = tile_order(g, T, kz);
            const int kt = 8 / kz;
            if (!o.n_ts) {
                if ((g.Vh / L[3]) % T == 0 && (g.Vh / L[3]) / T >= 8) { printf("FAIL not applied\n"); return 1; }
                continue;
            }
            applied++;
            const int ntiles = g.Vh / T;
            std::vector<int> seen(ntiles, 0);
            for (int x = 0; x < 8; x++) {
                int lo = 1 << 30, hi = -1, tlo = 1 << 30, thi = -1;
                for (int k = 0; k < o.per; k++) {
                    const int t = zorder_tile(o, x, k);
                    if (t < -1 || t >= ntiles) { printf("FAIL range\n"); return 1; }
                    if (t < 0) continue;
                    seen[t]++;
                    const int pos = t % o.n_ts, ts = t / o.n_ts;
                    lo = pos < lo ? pos : lo;
                    hi = pos > hi ? pos : hi;
                    tlo = ts < tlo ? ts : tlo;
                    thi = ts > thi ? ts : thi;
                    if (k > 0 && zorder_tile(o, x, k - 1) >= 0 && zorder_tile(o, x, k - 1) / o.n_ts > t / o.n_ts) {
                        printf("FAIL not t-major\n"); return 1;
                    }
                }
                const int zx = x % kz, tx = x / kz;
                if (hi >= 0 && (lo != (zx * o.n_ts) / kz || hi != ((zx + 1) * o.n_ts) / kz - 1)) { printf("FAIL z range\n"); return 1; }
                if (thi >= 0 && (tlo != (tx * L[3]) / kt || thi != ((tx + 1) * L[3]) / kt - 1)) { printf("FAIL t range\n"); return 1; }
            }
            for (int t = 0; t < ntiles; t++)
                if (seen[t] != 1) { printf("FAIL tile %d seen %d (L %d %d %d %d T %d kz %d)\n", t, seen[t], L[0], L[1], L[2], L[3], T, kz); return 1; }
        }
    }
    printf("OK %d\n", applied);
    return 0;
}
"""


def test_tile_order_is_a_bijection(tmp_path):
    if not shutil.which(HIPCC) and not __import__("os").path.exists(HIPCC):
        pytest.skip("hipcc not available")
    import os
    src = tmp_path / "tile_order.cpp"
    src.write_text(PROG)
    exe = tmp_path / "tile_order"
    inc = os.path.join(os.path.dirname(__file__), "..", "paper_1309_0551_amd", "csrc")
    subprocess.run([HIPCC, "-std=c++17", "-O1", "-I", inc, str(src), "-o", str(exe)], check=True,
                   capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    assert out.startswith("OK") and int(out.split()[1]) > 80, out
