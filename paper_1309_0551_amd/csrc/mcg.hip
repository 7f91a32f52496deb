// mcg.hip -- the batched CG of one lattice with N right-hand sides as a
// sequence of kernel launches: the form for large batches.
//
// The persistent batched solver (batch_cg.hip) holds one 1024-lane
// workgroup per CU for the whole solve; its register budget (set by the FP64
// and control paths in the same kernel) leaves 16 waves per CU, and its
// multi-RHS Dslash steps run about a third slower than the standalone
// kernels, which keep twice as many waves in flight. On a large batch that
// outweighs the launches it saves, so there each iteration runs as launches,
// with the same algorithm: independent CGs, one state per right-hand side
// (reduce.hpp), per right-hand-side FP64 sums in a fixed order.
//   xpay   p = r + beta p (right-hand sides that iterate), partials of 4m^2 |p|^2
//   doe    t = D_oe p, partials of |t|^2
//   fin    alpha = rho / <p, A p> from both rows of partials
//   deo    D_eo t; x += alpha p, r -= alpha (4m^2 p - D_eo t), partials of |r|^2
//   fin    beta, stop tests
// (D_eo = -D_oe^dag makes <p, A p> = 4m^2 |p|^2 + |D_oe p|^2.) The FP64 steps
// (reliable updates, refinement residuals, the final residual) run between
// chunks of iterations for the right-hand sides whose state asks for one,
// with x64 += x_lo folded into the residual pass.
//
// Partial sums: a reducing kernel leaves, per workgroup, one FP64 sum per
// right-hand side in row rhs of a [N][stride] array (plain stores of N
// lanes); the finalize kernel runs one workgroup per right-hand side, which
// reads its row contiguously and sums it in a fixed order.
#include "batch.hpp"
#include "fields.hpp"
#include "mrhs_dev.hpp"
#include "reduce.hpp"

namespace lgt {

namespace {

// Sizes measured at 24^3 x 48 x 16 (the iteration in us, against 416): 512-lane
// workgroups +3, finalize workgroups of 256 / 512 lanes +6 / +1.5, 2 or 8
// pairs per lane in the p pass +3, workgroups that walk several tiles (fewer
// partials) +4 to +37, one partial per wavefront instead of per workgroup +18.
constexpr int kMB = kBS;      // lanes per workgroup of the vector, Dslash and FP64 kernels
constexpr int kFinBS = 1024;  // lanes of a finalize workgroup
constexpr int kXpayPairs = 4; // (site, rhs) pairs per lane of the p = r + beta p pass
// directions per trip of the inner Dslash's direction loop: two (four hops'
// loads in flight, 84 VGPRs at R = 2) took the iteration from 416 to 407 us
// with the VALU engine and left the MFMA one unchanged; four spills the update
// kernel at R = 2
constexpr int kUnr = 2;

// Whether any right-hand side's gate is open (uniform over the workgroup:
// every lane reads the same N states, written by an earlier launch)
__device__ __forceinline__ bool any_open(const CgState *st, int N, int gate)
{
    bool a = false;
    for (int q = 0; q < N; q++) a |= gate_open(gate, &st[q]);
    return a;
}

// Per right-hand-side sums of a workgroup whose lane li holds v[r] for
// right-hand side (li % LPS) R + r: a butterfly over the lanes of a wavefront
// that share (li % LPS), then the wavefronts in index order. Writes
// out[rhs * stride] for the N = LPS R right-hand sides. Every lane of the
// workgroup calls it.
template <int R, int LPS>
__device__ __forceinline__ void wg_rhs_sums(double v[R], double *out, size_t stride)
{
    for (int o = LPS; o < 64; o <<= 1) {
#pragma unroll
        for (int r = 0; r < R; r++) v[r] += __shfl_xor(v[r], o, 64);
    }
    __shared__ double red[kMB / 64][kMaxRhs];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane < LPS) {
#pragma unroll
        for (int r = 0; r < R; r++) red[w][lane * R + r] = v[r];
    }
    __syncthreads();
    if ((int)threadIdx.x < LPS * R) {
        double s = 0.0;
        for (int k = 0; k < kMB / 64; k++) s += red[k][threadIdx.x];
        out[threadIdx.x * stride] = s;
    }
}

// the same for one lane per (site, rhs), rhs = li % N
__device__ __forceinline__ void wg_rhs_sums_lane(double v, int N, double *out, size_t stride)
{
    for (int o = N; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    __shared__ double red[kMB / 64][kMaxRhs];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane < N) red[w][lane] = v;
    __syncthreads();
    if ((int)threadIdx.x < N) {
        double s = 0.0;
        for (int k = 0; k < kMB / 64; k++) s += red[k][threadIdx.x];
        out[threadIdx.x * stride] = s;
    }
}

__global__ void k_mcg_init(CgState *st, int N, int scheme, int ru_fixed, int max_iter, double tol, double inner)
{
    const int q = threadIdx.x;
    if (q >= N) return;
    CgState &s = st[q];
    s.rho = s.rho_prev = s.alpha = s.beta = s.pAp = 0.0;
    s.bnorm2 = 0.0;
    s.stop_outer = tol * tol; // multiplied by |b|^2 in FIN_INIT
    s.stop_inner = 0.0;
    s.inner2 = scheme == SCH_REFINE ? inner * inner : (inner * tol) * (inner * tol);
    s.last_true = 0.0;
    s.iter = 0;
    s.updates = 0;
    s.state = ST_INIT;
    s.max_iter = max_iter;
    s.scheme = scheme;
    s.ru_fixed = ru_fixed;
    s.pend = s.pcur = 0;
}

// partials of |b|^2
__global__ __launch_bounds__(kMB) void k_mcg_norm(const double *__restrict__ b64, int Vh, int logN,
                                                  double *__restrict__ parts, size_t stride)
{
    const unsigned idx = blockIdx.x * kMB + threadIdx.x;
    const unsigned site = idx >> logN, rhs = idx & ((1u << logN) - 1u);
    double v = 0.0;
    if (site < (unsigned)Vh) {
        cx<double> bb[3];
        ldm<double>(b64, (size_t)Vh, logN, site, rhs, bb);
#pragma unroll
        for (int c = 0; c < 3; c++) v += bb[c].re * bb[c].re + bb[c].im * bb[c].im;
    }
    wg_rhs_sums_lane(v, 1 << logN, parts + blockIdx.x, stride);
}

// sum of row[0..n) by lane t: entries t, t + kFinBS, ... into four
// accumulators in a fixed order, four loads in flight
__device__ __forceinline__ double lane_row_sum(const double *__restrict__ row, int n)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * kFinBS < n; b += 4 * kFinBS) {
        s0 += row[b];
        s1 += row[b + kFinBS];
        s2 += row[b + 2 * kFinBS];
        s3 += row[b + 3 * kFinBS];
    }
    for (; b < n; b += kFinBS) s0 += row[b];
    return (s0 + s1) + (s2 + s3);
}

// Workgroup q: the sum of row q's first n partials (and of the first n2 of
// row q of parts2 when n2 > 0; lanes in block_sum's order), then the scalar
// step fin where right-hand side q's gate is open.
__global__ __launch_bounds__(kFinBS) void k_mcg_fin(const double *__restrict__ parts, size_t stride, int n,
                                                    const double *__restrict__ parts2, size_t stride2, int n2,
                                                    CgState *st, int fin, int gate)
{
    const int q = blockIdx.x;
    if (!gate_open(gate, &st[q])) return; // uniform
    double s = lane_row_sum(parts + (size_t)q * stride, n);
    if (n2 > 0) s += lane_row_sum(parts2 + (size_t)q * stride2, n2);
    __shared__ double lds[kFinBS / 64];
    const double tot = block_sum(s, lds);
    if (threadIdx.x == 0) finalize(fin, &st[q], tot);
}

// p = r + beta p for the right-hand sides that iterate (the others keep p),
// four (site, rhs) pairs per lane kMB apart, and the partials of 4m^2 |p|^2,
// the first term of <p, A p> = 4m^2 |p|^2 + |D_oe p|^2
__global__ __launch_bounds__(kMB) void k_mcg_xpay(const void *__restrict__ r, void *__restrict__ p, int Vh, int logN,
                                                  double m4, const CgState *st, double *__restrict__ parts,
                                                  size_t stride)
{
    const int N = 1 << logN;
    if (!any_open(st, N, GATE_ITER)) return;
    const unsigned rhs = threadIdx.x & (unsigned)(N - 1); // kMB is a multiple of N
    const bool run = st[rhs].state == ST_RUN;
    const float beta = (float)st[rhs].beta;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kXpayPairs; k++) {
        const unsigned idx = (blockIdx.x * kXpayPairs + k) * kMB + threadIdx.x;
        const unsigned site = idx >> logN;
        if (site >= (unsigned)Vh || !run) continue;
        cx<float> rr[3], pp[3];
        // streaming accesses (392 -> 388 us an iteration for the loads, 380
        // with the store): r is not read again before D_eo; the new p is
        // gathered by D_oe next, yet stored non-temporally it leaves the
        // caches to the gathers' own reuse
        ldm<float, true>(r, (size_t)Vh, logN, site, rhs, rr);
        ldm<float, true>(p, (size_t)Vh, logN, site, rhs, pp);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            pp[c].re = fmaf(beta, pp[c].re, rr[c].re);
            pp[c].im = fmaf(beta, pp[c].im, rr[c].im);
            v += (double)pp[c].re * (double)pp[c].re + (double)pp[c].im * (double)pp[c].im;
        }
        stm<float, true>(p, (size_t)Vh, logN, site, rhs, pp);
    }
    wg_rhs_sums_lane(m4 * v, N, parts + blockIdx.x, stride);
}

// t = D_oe p (four lanes per site), partials of |t|^2, the second term of
// <p, A p>
template <class LF, int R, int GPS, bool MFMA>
__global__ __launch_bounds__(kMB) void k_mcg_doe(const void *__restrict__ U, const void *__restrict__ p,
                                                 void *__restrict__ t, Geom g, int logN, int nblk_pad, TileOrder o,
                                                 const CgState *st, double *__restrict__ parts, size_t stride)
{
    constexpr unsigned LPS = 4 * GPS;
    if (!any_open(st, LPS * R, GATE_ITER)) return;
    const int blk = mrhs_block(o, nblk_pad);
    if (blk < 0) return; // the whole workgroup
    const unsigned idx = (unsigned)blk * kMB + threadIdx.x;
    const unsigned site = idx / LPS, lane4 = idx & 3u;
    const size_t Vh = (size_t)g.Vh;
    const unsigned r0 = (threadIdx.x % LPS) * R;
    double v[R];
#pragma unroll
    for (int r = 0; r < R; r++) v[r] = 0.0;
    // whole quads are in or out of range; the MFMA engine needs whole
    // wavefronts, which V/2 % 16 == 0 gives it
    if (site < (unsigned)g.Vh) {
        auto IN = [=](int n, cx<float> u[R][3]) __attribute__((always_inline)) { ldm_r<float, R>(p, Vh, logN, n, r0, u); };
        cx<float> acc[R][3];
        dslash_site4<LF, R, MFMA, kUnr, true>(g, kOdd, U, site, lane4, IN, acc);
        // non-temporal: write-allocating t would evict the p that the
        // neighbouring sites' gathers reuse (1.4 % of the iteration)
        stm_r<float, R, true>(t, Vh, logN, site, r0, acc);
#pragma unroll
        for (int r = 0; r < R; r++) {
            double tt = 0.0;
#pragma unroll
            for (int c = 0; c < 3; c++)
                tt += (double)acc[r][c].re * (double)acc[r][c].re + (double)acc[r][c].im * (double)acc[r][c].im;
            v[r] = tt;
        }
    }
    wg_rhs_sums<R, LPS>(v, parts + blk, stride);
}

// D_eo t with the update: x += alpha p, r -= alpha (4m^2 p - D_eo t) for the
// right-hand sides that iterate (the others' x and r are stored back as they
// were), partials of |r|^2
template <class LF, int R, int GPS, bool MFMA>
__global__ __launch_bounds__(kMB) void k_mcg_deo(const void *__restrict__ U, const void *__restrict__ t,
                                                 const void *__restrict__ p, void *__restrict__ x, void *__restrict__ r,
                                                 Geom g, int logN, int nblk_pad, TileOrder o, double m4,
                                                 const CgState *st, double *__restrict__ parts, size_t stride)
{
    constexpr unsigned LPS = 4 * GPS;
    if (!any_open(st, LPS * R, GATE_ITER)) return;
    const int blk = mrhs_block(o, nblk_pad);
    if (blk < 0) return;
    const unsigned idx = (unsigned)blk * kMB + threadIdx.x;
    const unsigned site = idx / LPS, lane4 = idx & 3u;
    const size_t Vh = (size_t)g.Vh;
    const unsigned r0 = (threadIdx.x % LPS) * R;
    double v[R];
#pragma unroll
    for (int q = 0; q < R; q++) v[q] = 0.0;
    if (site < (unsigned)g.Vh) {
        auto IN = [=](int n, cx<float> u[R][3]) __attribute__((always_inline)) { ldm_r<float, R>(t, Vh, logN, n, r0, u); };
        cx<float> acc[R][3], pp[R][3], xx[R][3], rr[R][3];
        dslash_site4<LF, R, MFMA, kUnr, true>(g, kEven, U, site, lane4, IN, acc);
        // x and p with streaming (non-temporal) accesses: neither is read
        // again before the next p pass, and keeping them out of the caches
        // leaves room for the t gathers and for r (407 -> 391 us an iteration)
        ldm_r<float, R, true>(p, Vh, logN, site, r0, pp);
        ldm_r<float, R, true>(x, Vh, logN, site, r0, xx);
        ldm_r<float, R>(r, Vh, logN, site, r0, rr);
        const float m4f = (float)m4;
#pragma unroll
        for (int q = 0; q < R; q++) {
            if (st[r0 + q].state != ST_RUN) continue; // x and r stay as they are
            const float alpha = (float)st[r0 + q].alpha;
            double d = 0.0;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const float apr = m4f * pp[q][c].re - acc[q][c].re;
                const float api = m4f * pp[q][c].im - acc[q][c].im;
                xx[q][c].re = fmaf(alpha, pp[q][c].re, xx[q][c].re);
                xx[q][c].im = fmaf(alpha, pp[q][c].im, xx[q][c].im);
                rr[q][c].re = fmaf(-alpha, apr, rr[q][c].re);
                rr[q][c].im = fmaf(-alpha, api, rr[q][c].im);
                d += (double)rr[q][c].re * (double)rr[q][c].re + (double)rr[q][c].im * (double)rr[q][c].im;
            }
            v[q] = d;
        }
        stm_r<float, R, true>(x, Vh, logN, site, r0, xx);
        stm_r<float, R>(r, Vh, logN, site, r0, rr);
    }
    wg_rhs_sums<R, LPS>(v, parts + blk, stride);
}

// FP64 step, first half: t64 = D_oe (x64 + x_lo) for the right-hand sides
// whose gate is open (one lane per (site, rhs), FP64 links)
__global__ __launch_bounds__(kMB) void k_mcg_fp64_doe(const void *__restrict__ Uhi, const double *__restrict__ x64,
                                                      const void *__restrict__ xlo, double *__restrict__ t64, Geom g,
                                                      int logN, int nblk_pad, TileOrder o, const CgState *st,
                                                      int gate)
{
    const int blk = mrhs_block(o, nblk_pad);
    if (blk < 0) return;
    const unsigned idx = (unsigned)blk * kMB + threadIdx.x;
    const unsigned site = idx >> logN, rhs = idx & ((1u << logN) - 1u);
    if (site >= (unsigned)g.Vh || !gate_open(gate, &st[rhs])) return;
    const size_t Vh = (size_t)g.Vh;
    auto IN = [=](int n, cx<double> u[3]) __attribute__((always_inline)) {
        cx<float> e[3];
        ldm<double>(x64, Vh, logN, n, rhs, u);
        ldm<float>(xlo, Vh, logN, n, rhs, e);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            u[c].re += (double)e[c].re;
            u[c].im += (double)e[c].im;
        }
    };
    cx<double> acc[3];
    dslash_mrhs<LinkF64R18>(g, kOdd, Uhi, site, IN, acc);
    stm<double>(t64, Vh, logN, site, rhs, acc);
}

// FP64 step, second half: x64 += x_lo, x_lo = 0, r = b - (4m^2 x64 - D_eo t64)
// in FP64, rounded into r_lo; partials of |r|^2
__global__ __launch_bounds__(kMB) void k_mcg_fp64_res(const void *__restrict__ Uhi, const double *__restrict__ t64,
                                                      double *__restrict__ x64, void *__restrict__ xlo,
                                                      const double *__restrict__ b64, void *__restrict__ rlo, Geom g,
                                                      int logN, int nblk_pad, TileOrder o, double m4,
                                                      const CgState *st, int gate, double *__restrict__ parts,
                                                      size_t stride)
{
    const int N = 1 << logN;
    if (!any_open(st, N, gate)) return; // uniform; no partial of a closed gate is read
    const int blk = mrhs_block(o, nblk_pad);
    if (blk < 0) return;
    const unsigned idx = (unsigned)blk * kMB + threadIdx.x;
    const unsigned site = idx >> logN, rhs = idx & ((1u << logN) - 1u);
    double v = 0.0;
    if (site < (unsigned)g.Vh && gate_open(gate, &st[rhs])) {
        const size_t Vh = (size_t)g.Vh;
        auto IN = [=](int n, cx<double> u[3]) __attribute__((always_inline)) { ldm<double>(t64, Vh, logN, n, rhs, u); };
        cx<double> acc[3], x[3], bb[3];
        cx<float> e[3], lo[3];
        dslash_mrhs<LinkF64R18>(g, kEven, Uhi, site, IN, acc);
        ldm<double>(x64, Vh, logN, site, rhs, x);
        ldm<double>(b64, Vh, logN, site, rhs, bb);
        ldm<float>(xlo, Vh, logN, site, rhs, e);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            x[c].re += (double)e[c].re;
            x[c].im += (double)e[c].im;
            e[c].re = e[c].im = 0.f;
            acc[c].re = bb[c].re - (m4 * x[c].re - acc[c].re);
            acc[c].im = bb[c].im - (m4 * x[c].im - acc[c].im);
            v += acc[c].re * acc[c].re + acc[c].im * acc[c].im;
            lo[c].re = (float)acc[c].re;
            lo[c].im = (float)acc[c].im;
        }
        stm<double>(x64, Vh, logN, site, rhs, x);
        stm<float>(xlo, Vh, logN, site, rhs, e);
        stm<float>(rlo, Vh, logN, site, rhs, lo);
    }
    wg_rhs_sums_lane(v, N, parts + blk, stride);
}

template <class LF, int R, int GPS>
hipError_t launch_iter_rg(const McgArgs &a, bool mf, int which, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const int TS = kMB / (4 * GPS), nblk = (a.g.Vh + TS - 1) / TS, pad = (nblk + 7) / 8 * 8;
    const TileOrder o = tile_order(a.g, TS);
    const dim3 grid(mrhs_grid(o, nblk)), block(kMB);
    if (e0) (void)hipEventRecord(e0, s);
    if (which == 0) {
        if (mf)
            hipLaunchKernelGGL((k_mcg_doe<LF, R, GPS, true>), grid, block, 0, s, a.Ulo, a.p, a.t, a.g, a.logN, pad, o,
                               a.st, a.parts, a.stride);
        else
            hipLaunchKernelGGL((k_mcg_doe<LF, R, GPS, false>), grid, block, 0, s, a.Ulo, a.p, a.t, a.g, a.logN, pad,
                               o, a.st, a.parts, a.stride);
    } else {
        if (mf)
            hipLaunchKernelGGL((k_mcg_deo<LF, R, GPS, true>), grid, block, 0, s, a.Ulo, a.t, a.p, a.xlo, a.r, a.g,
                               a.logN, pad, o, a.m4, a.st, a.parts, a.stride);
        else
            hipLaunchKernelGGL((k_mcg_deo<LF, R, GPS, false>), grid, block, 0, s, a.Ulo, a.t, a.p, a.xlo, a.r, a.g,
                               a.logN, pad, o, a.m4, a.st, a.parts, a.stride);
    }
    if (e1) (void)hipEventRecord(e1, s);
    return hipGetLastError();
}

// (N = 16 runs two or four groups: see batch_groups)
template <class LF>
hipError_t launch_iter_fmt(const McgArgs &a, int which, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const bool mf = a.engine == MRHS_MFMA;
    switch (a.logN * 8 + a.gps) {
    case 2 * 8 + 1: return launch_iter_rg<LF, 1, 1>(a, mf, which, s, e0, e1);
    case 3 * 8 + 1: return launch_iter_rg<LF, 2, 1>(a, mf, which, s, e0, e1);
    case 3 * 8 + 2: return launch_iter_rg<LF, 1, 2>(a, mf, which, s, e0, e1);
    case 4 * 8 + 2: return launch_iter_rg<LF, 2, 2>(a, mf, which, s, e0, e1);
    case 4 * 8 + 4: return launch_iter_rg<LF, 1, 4>(a, mf, which, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

} // namespace

int mcg_iter_parts(const Geom &g, int gps, bool padded)
{
    const int TS = kMB / (4 * gps), nblk = (g.Vh + TS - 1) / TS;
    return padded ? (nblk + 7) / 8 * 8 : nblk;
}
int mcg_lane_blocks(const Geom &g, int logN) { return (int)((((int64_t)g.Vh << logN) + kMB - 1) / kMB); }
int mcg_xpay_blocks(const Geom &g, int logN)
{
    return (int)((((int64_t)g.Vh << logN) + kMB * kXpayPairs - 1) / (kMB * kXpayPairs));
}

hipError_t launch_mcg_init(const McgArgs &a, int scheme, int ru_fixed, int max_iter, double tol, double inner,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_mcg_init, dim3(1), dim3(64), 0, s, a.st, 1 << a.logN, scheme, ru_fixed, max_iter, tol,
                       inner);
    return hipGetLastError();
}

hipError_t launch_mcg_norm(const McgArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_mcg_norm, dim3(mcg_lane_blocks(a.g, a.logN)), dim3(kMB), 0, s, a.b64, a.g.Vh, a.logN,
                       a.parts, a.stride);
    return hipGetLastError();
}

hipError_t launch_mcg_fin(const McgArgs &a, int n, int fin, int gate, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                          int n_p)
{
    if (e0) (void)hipEventRecord(e0, s);
    hipLaunchKernelGGL(k_mcg_fin, dim3(1 << a.logN), dim3(kFinBS), 0, s, a.parts, a.stride, n, a.parts_p,
                       a.stride_p, n_p, a.st, fin, gate);
    if (e1) (void)hipEventRecord(e1, s);
    return hipGetLastError();
}

hipError_t launch_mcg_xpay(const McgArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (e0) (void)hipEventRecord(e0, s);
    hipLaunchKernelGGL(k_mcg_xpay, dim3(mcg_xpay_blocks(a.g, a.logN)), dim3(kMB), 0, s, a.r, a.p, a.g.Vh, a.logN,
                       a.m4, a.st, a.parts_p, a.stride_p);
    if (e1) (void)hipEventRecord(e1, s);
    return hipGetLastError();
}

hipError_t launch_mcg_dslash(Fmt lo, const McgArgs &a, int which, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    switch (lo) {
    case F32R18: return launch_iter_fmt<LinkF32R18>(a, which, s, e0, e1);
    case F32R12: return launch_iter_fmt<LinkF32R12>(a, which, s, e0, e1);
    case BF16R12: return launch_iter_fmt<LinkBF16R12>(a, which, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mcg_fp64(const McgArgs &a, int gate, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    // tiles of kMB (site, rhs) pairs in the XCD-aware order of the
    // standalone lane engine: a workgroup's neighbours stay in its XCD's L2
    // (in plain block order the FP64 step fetched 4.2 x its bytes)
    const int nblk = mcg_lane_blocks(a.g, a.logN), pad = (nblk + 7) / 8 * 8;
    const TileOrder o = tile_order(a.g, kMB >> a.logN);
    const dim3 grid(mrhs_grid(o, nblk)), block(kMB);
    if (e0) (void)hipEventRecord(e0, s);
    hipLaunchKernelGGL(k_mcg_fp64_doe, grid, block, 0, s, a.Uhi, a.x64, a.xlo, a.t64, a.g, a.logN, pad, o, a.st,
                       gate);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mcg_fp64_res, grid, block, 0, s, a.Uhi, a.t64, a.x64, a.xlo, a.b64, a.r, a.g, a.logN, pad,
                       o, a.m4, a.st, gate, a.parts, a.stride);
    if (e1) (void)hipEventRecord(e1, s);
    return hipGetLastError();
}

} // namespace lgt
