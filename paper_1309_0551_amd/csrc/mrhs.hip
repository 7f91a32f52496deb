// mrhs.hip -- many right-hand sides: the standalone multi-RHS staggered
// Dslash and the multi-RHS vector packing.
//
// One lane per (site, rhs) or four lanes per site (VALU or MFMA products):
// either way a link is fetched from memory once per site for all N
// right-hand sides, so the HBM bytes per site and RHS fall from 8 links + 2
// vectors to 8/N links + 2 vectors.
#include "batch.hpp"
#include "fields.hpp"
#include "mrhs_dev.hpp"

namespace lgt {

// ------------------------------------------------------- standalone ---

// XCD grid of the standalone four-lane kernels' tile order: 4 z ranges x 2 t
// ranges, which halves the gathers across the z boundary of an XCD's share
// (at 24^3 x 48 with 16 right-hand sides, FP32 x 12, pseudo-random input, on
// one GPU: VALU engine 81.8-82.1 us against 83.0-83.4 with 8 z ranges, MFMA
// engine 91.9-93.3 against 95.7-96.7). The batched CG keeps 8 z ranges,
// which its kernels run about 1 % faster on.
constexpr int kMrhsKz = 4;

template <class LF>
__global__ __launch_bounds__(kBS) void k_dslash_mrhs(const void *__restrict__ U, const void *__restrict__ in,
                                                     void *__restrict__ out, Geom g, int par, int logN, int nblk_pad,
                                                     TileOrder o)
{
    using T = typename LF::real;
    const int blk = mrhs_block(o, nblk_pad);
    if (blk < 0) return;
    const unsigned idx = (unsigned)blk * kBS + threadIdx.x;
    const unsigned site = idx >> logN, rhs = idx & ((1u << logN) - 1u);
    if (site >= (unsigned)g.Vh) return;
    const size_t Vh = (size_t)g.Vh;
    auto IN = [=](int s, cx<T> v[3]) __attribute__((always_inline)) { ldm<T>(in, Vh, logN, s, rhs, v); };
    cx<T> acc[3];
    dslash_mrhs<LF>(g, par, U, site, IN, acc);
    stm<T, true>(out, Vh, logN, site, rhs, acc);
}

// GPS groups of four lanes per site, R right-hand sides per lane (N = 4 GPS R),
// VALU or MFMA engine. Lane l of a site's 4 GPS lanes owns right-hand sides
// l R .. l R + R - 1; each group of four is one MFMA block.
template <class LF, int R, int GPS, bool MFMA>
__global__ __launch_bounds__(kBS) void k_dslash_mrhs4(const void *__restrict__ U, const void *__restrict__ in,
                                                      void *__restrict__ out, Geom g, int par, int logN, int nblk_pad,
                                                      TileOrder o)
{
    constexpr unsigned LPS = 4 * GPS;
    const int blk = mrhs_block(o, nblk_pad);
    if (blk < 0) return;
    const unsigned idx = (unsigned)blk * kBS + threadIdx.x;
    const unsigned site = idx / LPS, lane4 = idx & 3u;
    // the lanes of a site and the 64 / LPS sites of a wavefront stay together,
    // and a wavefront is never split by the bound below (Vh is a multiple of 16
    // whenever the MFMA engine is used: checked on the host)
    if (site >= (unsigned)g.Vh) return;
    const size_t Vh = (size_t)g.Vh;
    const unsigned rhs0 = (idx % LPS) * R;
    auto IN = [=](int s, cx<float> v[R][3]) __attribute__((always_inline)) { ldm_r<float, R>(in, Vh, logN, s, rhs0, v); };
    cx<float> acc[R][3];
    // two directions per trip of the direction loop, four hops' loads in
    // flight (same hop order, so the same sums): at 24^3 x 48 with 16
    // right-hand sides, FP32 x 12, the VALU engine with two groups 81.1-81.8
    // -> 76.9-77.6 us, one group 96.3-97.2 -> 82.8-84.0; MFMA a tie
    dslash_site4<LF, R, MFMA, 2>(g, par, U, site, lane4, IN, acc);
    stm_r<float, R, true>(out, Vh, logN, site, rhs0, acc);
}

// Staged variant: kStageBS lanes per workgroup, a tile of TS = kStageBS /
// (4 GPS) consecutive sites. The workgroup first copies the input of the
// tile's x and y neighbourhood -- the input-parity cb range [first - Lx/2,
// last + Lx/2], which holds every x and y neighbour of the tile except across
// the y boundary -- into LDS as [3][ns][N] complex with 16-byte coalesced
// loads, each element once; the x and y hops then read it there, so only the
// z and t hops (and the y-boundary ones) gather through the vector-memory
// path, which limits the unstaged kernel (texture units busy 83-91 %, HBM at
// 54 %). The range costs (TS + Lx) / TS loads of each element against the
// four x/y gathers per site it replaces.
template <class LF, int R, int GPS, bool MFMA>
__global__ __launch_bounds__(kStageBS) void k_dslash_mrhs4s(const void *__restrict__ U, const void *__restrict__ in,
                                                            void *__restrict__ out, Geom g, int par, int logN,
                                                            int nblk_pad, TileOrder o)
{
    extern __shared__ __align__(16) unsigned char mrhs_lds[];
    constexpr unsigned LPS = 4 * GPS;
    constexpr int TS = kStageBS / LPS;
    const int blk = mrhs_block(o, nblk_pad);
    if (blk < 0) return; // the whole workgroup
    const size_t Vh = (size_t)g.Vh;
    const int s0 = blk * TS - g.hx, ns = TS + 2 * g.hx;
    // stage: two complex numbers (one right-hand-side pair) per 16-byte load
    const int hlog = logN - 1, per = ns << hlog; // fv4 per colour plane
    const fv4 *in4 = (const fv4 *)in;
    fv4 *lds4 = (fv4 *)mrhs_lds;
    for (int i = threadIdx.x; i < 3 * per; i += kStageBS) {
        const int c = i / per, rem = i - c * per;
        const int n = s0 + (rem >> hlog);
        if (n >= 0 && n < g.Vh) lds4[i] = in4[(((size_t)c * Vh + (size_t)n) << hlog) + (rem & ((1 << hlog) - 1))];
    }
    __syncthreads();
    const unsigned idx = (unsigned)blk * kStageBS + threadIdx.x;
    const unsigned site = idx / LPS, lane4 = idx & 3u;
    // whole wavefronts leave together (V/2 % 16 == 0 for MFMA); no barrier follows
    if (site >= (unsigned)g.Vh) return;
    const unsigned rhs0 = (threadIdx.x % LPS) * R;
    const fv2 *lds = (const fv2 *)mrhs_lds;
    auto IN = [=](int n, cx<float> v[R][3]) __attribute__((always_inline)) {
        const unsigned j = (unsigned)(n - s0);
        if (j < (unsigned)ns) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const fv2 *q = lds + (((size_t)c * ns + j) << logN) + rhs0;
                if constexpr (R % 2 == 0) {
#pragma unroll
                    for (int r = 0; r < R; r += 2) {
                        const fv4 w = *(const fv4 *)(q + r);
                        v[r][c] = cx<float>{w.x, w.y};
                        v[r + 1][c] = cx<float>{w.z, w.w};
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < R; r++) v[r][c] = cx<float>{q[r].x, q[r].y};
                }
            }
            return;
        }
        ldm_r<float, R>(in, Vh, logN, n, rhs0, v);
    };
    cx<float> acc[R][3];
    dslash_site4<LF, R, MFMA>(g, par, U, site, lane4, IN, acc);
    stm_r<float, R, true>(out, Vh, logN, site, rhs0, acc);
}

template <class LF, int R, int GPS>
static void launch_mrhs4_rg(bool mf, bool staged, const void *U, const void *in, void *out, const Geom &g, int par,
                            int logN, hipStream_t s)
{
    const int lanes = staged ? kStageBS : kBS, TS = lanes / (4 * GPS);
    const int nblk = (int)(((int64_t)g.Vh + TS - 1) / TS);
    const int pad = (nblk + 7) / 8 * 8;
    const TileOrder o = tile_order(g, TS, kMrhsKz);
    const dim3 grid(mrhs_grid(o, nblk)), block(lanes);
    if (staged) {
        const size_t lds = mrhs_stage_bytes(TS, g.hx, logN);
        if (mf) hipLaunchKernelGGL((k_dslash_mrhs4s<LF, R, GPS, true>), grid, block, lds, s, U, in, out, g, par, logN, pad, o);
        else hipLaunchKernelGGL((k_dslash_mrhs4s<LF, R, GPS, false>), grid, block, lds, s, U, in, out, g, par, logN, pad, o);
        return;
    }
    if (mf) hipLaunchKernelGGL((k_dslash_mrhs4<LF, R, GPS, true>), grid, block, 0, s, U, in, out, g, par, logN, pad, o);
    else hipLaunchKernelGGL((k_dslash_mrhs4<LF, R, GPS, false>), grid, block, 0, s, U, in, out, g, par, logN, pad, o);
}

template <class LF>
static hipError_t launch_mrhs4(int engine, int gps, bool st, const void *U, const void *in, void *out, const Geom &g,
                               int par, int logN, hipStream_t s)
{
    const bool mf = engine == MRHS_MFMA;
    const int key = logN * 8 + gps;
    switch (key) {
    case 2 * 8 + 1: launch_mrhs4_rg<LF, 1, 1>(mf, st, U, in, out, g, par, logN, s); break;
    case 3 * 8 + 1: launch_mrhs4_rg<LF, 2, 1>(mf, st, U, in, out, g, par, logN, s); break;
    case 3 * 8 + 2: launch_mrhs4_rg<LF, 1, 2>(mf, st, U, in, out, g, par, logN, s); break;
    case 4 * 8 + 1: launch_mrhs4_rg<LF, 4, 1>(mf, st, U, in, out, g, par, logN, s); break;
    case 4 * 8 + 2: launch_mrhs4_rg<LF, 2, 2>(mf, st, U, in, out, g, par, logN, s); break;
    case 4 * 8 + 4: launch_mrhs4_rg<LF, 1, 4>(mf, st, U, in, out, g, par, logN, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool mrhs_staging_fits(const Geom &g, int logN, int gps)
{
    return mrhs_stage_bytes(kStageBS / (4 * gps), g.hx, logN) <= kMrhsStageMax;
}

bool mrhs_engine_applies(Fmt f, int logN, int Vh, int engine)
{
    if (engine == MRHS_LANE || logN < 2 || fmt_is_f64_fmt(f)) return false;
    return engine == MRHS_VALU4 || (Vh % 16) == 0;
}

bool mrhs_groups_valid(int logN, int gps)
{
    return (gps == 1 || gps == 2 || gps == 4) && 4 * gps <= (1 << logN);
}

hipError_t launch_dslash_mrhs(Fmt f, const void *U, const void *in, void *out, const Geom &g, int par, int logN,
                              hipStream_t s, int engine, int gps, bool staged)
{
    if (mrhs_engine_applies(f, logN, g.Vh, engine)) {
        if (!mrhs_groups_valid(logN, gps)) gps = 1;
        const bool st = staged && mrhs_staging_fits(g, logN, gps);
        switch (f) {
        case F32R18: return launch_mrhs4<LinkF32R18>(engine, gps, st, U, in, out, g, par, logN, s);
        case F32R12: return launch_mrhs4<LinkF32R12>(engine, gps, st, U, in, out, g, par, logN, s);
        case BF16R12: return launch_mrhs4<LinkBF16R12>(engine, gps, st, U, in, out, g, par, logN, s);
        default: break;
        }
    }
    const int64_t n = (int64_t)g.Vh << logN;
    const int nblk = (int)((n + kBS - 1) / kBS);
    const int pad = (nblk + 7) / 8 * 8;
    const TileOrder o = tile_order(g, kBS >> logN);
    const dim3 grid(mrhs_grid(o, nblk)), block(kBS);
    switch (f) {
    case F64R18: hipLaunchKernelGGL(k_dslash_mrhs<LinkF64R18>, grid, block, 0, s, U, in, out, g, par, logN, pad, o); break;
    case F64R12: hipLaunchKernelGGL(k_dslash_mrhs<LinkF64R12>, grid, block, 0, s, U, in, out, g, par, logN, pad, o); break;
    case F32R18: hipLaunchKernelGGL(k_dslash_mrhs<LinkF32R18>, grid, block, 0, s, U, in, out, g, par, logN, pad, o); break;
    case F32R12: hipLaunchKernelGGL(k_dslash_mrhs<LinkF32R12>, grid, block, 0, s, U, in, out, g, par, logN, pad, o); break;
    case BF16R12: hipLaunchKernelGGL(k_dslash_mrhs<LinkBF16R12>, grid, block, 0, s, U, in, out, g, par, logN, pad, o); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// canonical [nsrc][V/2][3][2] float64 <-> multi-RHS [3][V/2][N] of T, N =
// 2^logN >= nsrc: packing fills right-hand sides nsrc..N-1 with zeros, and
// unpacking writes only the first nsrc
template <typename T>
__global__ __launch_bounds__(kBS) void k_pack_mrhs(const double *__restrict__ src, void *__restrict__ dst, int Vh,
                                                   int logN, int nsrc)
{
    const int64_t idx = (int64_t)blockIdx.x * kBS + threadIdx.x; // (site << logN) + rhs
    if (idx >= ((int64_t)Vh << logN)) return;
    const unsigned site = (unsigned)(idx >> logN), rhs = (unsigned)(idx & ((1 << logN) - 1));
    cx<T> v[3];
    if (rhs < (unsigned)nsrc) {
        const dv2 *p = (const dv2 *)src + ((size_t)rhs * Vh + site) * 3;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const dv2 w = p[c];
            v[c].re = (T)w.x;
            v[c].im = (T)w.y;
        }
    } else {
#pragma unroll
        for (int c = 0; c < 3; c++) v[c].re = v[c].im = T(0);
    }
    stm<T>(dst, (size_t)Vh, logN, site, rhs, v);
}

template <typename T>
__global__ __launch_bounds__(kBS) void k_unpack_mrhs(const void *__restrict__ src, double *__restrict__ dst, int Vh,
                                                     int logN, int nsrc)
{
    const int64_t idx = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (idx >= ((int64_t)Vh << logN)) return;
    const unsigned site = (unsigned)(idx >> logN), rhs = (unsigned)(idx & ((1 << logN) - 1));
    if (rhs >= (unsigned)nsrc) return;
    cx<T> v[3];
    ldm<T>(src, (size_t)Vh, logN, site, rhs, v);
    dv2 *p = (dv2 *)dst + ((size_t)rhs * Vh + site) * 3;
#pragma unroll
    for (int c = 0; c < 3; c++) p[c] = dv2{(double)v[c].re, (double)v[c].im};
}

hipError_t launch_pack_mrhs(bool f64, const double *src, void *dst, const Geom &g, int logN, hipStream_t s, int nsrc)
{
    const int64_t n = (int64_t)g.Vh << logN;
    if (nsrc < 0 || nsrc > (1 << logN)) nsrc = 1 << logN;
    const dim3 grid((unsigned)((n + kBS - 1) / kBS)), block(kBS);
    if (f64) hipLaunchKernelGGL(k_pack_mrhs<double>, grid, block, 0, s, src, dst, g.Vh, logN, nsrc);
    else hipLaunchKernelGGL(k_pack_mrhs<float>, grid, block, 0, s, src, dst, g.Vh, logN, nsrc);
    return hipGetLastError();
}

hipError_t launch_unpack_mrhs(bool f64, const void *src, double *dst, const Geom &g, int logN, hipStream_t s,
                              int nsrc)
{
    const int64_t n = (int64_t)g.Vh << logN;
    if (nsrc < 0 || nsrc > (1 << logN)) nsrc = 1 << logN;
    const dim3 grid((unsigned)((n + kBS - 1) / kBS)), block(kBS);
    if (f64) hipLaunchKernelGGL(k_unpack_mrhs<double>, grid, block, 0, s, src, dst, g.Vh, logN, nsrc);
    else hipLaunchKernelGGL(k_unpack_mrhs<float>, grid, block, 0, s, src, dst, g.Vh, logN, nsrc);
    return hipGetLastError();
}

} // namespace lgt
