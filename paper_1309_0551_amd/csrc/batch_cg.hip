// batch_cg.hip -- the persistent batched CG.
//
// Independent even-odd CGs (own alpha, beta and state per right-hand side;
// not block CG) for every right-hand side of every problem -- lattices of
// different sizes included -- run in lock-step in one cooperative launch of
// one kBB-thread workgroup per CU.
//
// An iteration takes two grid barriers (D_eo needs all of D_oe's output, and
// beta is a global sum):
//   1. t = D_oe p', where p' = r + beta p is formed at the neighbours from r
//      and the previous p, and written by the owner of each even index into
//      the other of two p buffers; partial <p', A p'> = 4m^2 |p'|^2 + |t|^2
//      (D_eo = -D_oe^dag, so -<p', D_eo D_oe p'> = |D_oe p'|^2)  -> alpha;
//   2. Ap = 4m^2 p' - D_eo t, used at once: x += alpha p', r -= alpha Ap,
//      partial |r|^2                                           -> beta, stop tests.
// Knowing alpha before D_eo saves the third barrier and a pass over x, r, p'
// and Ap that a separate update step would take.
// Each workgroup adds its partial sums per right-hand side into one row.
// After the barrier EVERY workgroup sums all rows in the same fixed order and
// runs the scalar step on its own copy of the states, kept in LDS: the copies
// stay bit-identical, so all workgroups take the same branches and meet the
// same barriers, and no barrier is spent on publishing scalars. FP64 reliable
// updates and refinement steps (two more barriers) run in the same launch for
// the right-hand sides that need them.
#include <type_traits>

#include "batch.hpp"
#include "mrhs_dev.hpp"
#include "reduce.hpp"

namespace lgt {

namespace {

constexpr int kWaves = kBB / 64;

struct Shared {
    CgState st[kMaxTotalRhs];
    double coef[kMaxTotalRhs];         // beta before step 1, alpha before step 3; 0 unless iterating
    double acc[kMaxTotalRhs];          // this workgroup's partial sums
    double red[kBB];                   // reduction scratch
    double tot[kMaxTotalRhs];          // row sums (sum_rows)
    unsigned char run[kMaxTotalRhs];   // state == ST_RUN
    unsigned char sel[kMaxTotalRhs];   // selected for the current FP64 step
    int prun[kMaxProblems], psel[kMaxProblems];
    int any_run, any_sel, ok, pad;
    unsigned long long prof[kBatchPhases]; // phase profile of workgroup 0 (thread 0 only)
    unsigned long long prof_last;
};

// Phase profile (when BatchArgs::prof is set): workgroup 0's thread 0 adds the
// constant-rate clock ticks since its previous mark to phase k. Its marks
// after each barrier make a phase's time the slowest workgroup's work on it
// plus the barrier; the marks before a barrier separate its own work from the
// wait, which is then imbalance plus barrier latency.
__device__ __forceinline__ void mark(const BatchArgs *A, Shared &S, int k)
{
    if (A->prof && blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long now = __builtin_amdgcn_s_memrealtime();
        if (k >= 0) S.prof[k] += now - S.prof_last;
        S.prof_last = now;
    }
}

__device__ __forceinline__ double ld_f64(const double *p)
{
    return __longlong_as_double((long long)__hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ unsigned int ld_u32(const unsigned int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Two-level grid barrier. Workgroups arrive on the counter of their XCD
// (blockIdx % 8 under round-robin dispatch), the last of each XCD on the top
// counter, and the last of those opens the next generation. A device-scope
// fence before arriving publishes the workgroup's writes; one after leaving
// makes the others' writes visible. A wait longer than `limit` polls, or an
// error raised by another workgroup, ends the wait and returns false, so
// every wave always reaches the end of the kernel.
__device__ bool grid_sync(BatchCtl *ctl, unsigned int limit, Shared &S)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = ld_u32(&ctl->err) == 0;
        if (ok) {
            const unsigned int gen = ld_u32(&ctl->gen);
            __threadfence();
            const unsigned int G = gridDim.x, x = blockIdx.x & 7u;
            const unsigned int ng = G < 8u ? G : 8u, nx = (G - x + 7u) / 8u;
            bool last = false;
            if ((atomicAdd(&ctl->grp[x][0], 1u) + 1u) % nx == 0u) last = (atomicAdd(&ctl->top, 1u) + 1u) % ng == 0u;
            if (last) {
                atomicAdd(&ctl->gen, 1u);
            } else {
                unsigned int n = 0;
                while (ld_u32(&ctl->gen) == gen) {
                    __builtin_amdgcn_s_sleep(2);
                    ++n;
                    if (n > limit || ((n & 63u) == 0u && ld_u32(&ctl->err) != 0u)) {
                        atomicOr(&ctl->err, 1u);
                        ok = 0;
                        break;
                    }
                }
            }
            __threadfence();
        }
        S.ok = ok;
    }
    __syncthreads();
    return S.ok != 0;
}

// Tiles of the problems whose mask is set. The workgroups of XCD x take the
// x-th contiguous eighth of the tile list, so the lattice neighbours of a
// tile mostly lie in tiles served by the same L2. flush(p) runs whenever the
// workgroup leaves problem p. Everything here is uniform over the workgroup.
template <bool DT, class Body, class Flush>
__device__ __forceinline__ void tiles(const BatchArgs *A, const int *pmask, Body body, Flush flush)
{
    const int total = DT ? A->total_dt : A->total_lt;
    const int G = gridDim.x;
    int begin = 0, end = total, j = blockIdx.x, step = G;
    if (G >= 8) {
        const int x = blockIdx.x & 7, per = (total + 7) / 8;
        begin = min(total, x * per);
        end = min(total, begin + per);
        j = blockIdx.x >> 3;
        step = (G - x + 7) / 8;
    }
    int p = 0, cur = -1;
    for (int w = begin + j; w < end; w += step) {
        while (p + 1 < A->nprob && w >= (DT ? A->prob[p + 1].dt0 : A->prob[p + 1].lt0)) p++;
        if (!pmask[p]) continue;
        if (p != cur) {
            if (cur >= 0) flush(cur);
            cur = p;
        }
        body(A->prob[p], w - (DT ? A->prob[p].dt0 : A->prob[p].lt0));
    }
    if (cur >= 0) flush(cur);
}

// Add the per-thread sums v[r] (right-hand side (lane % LG) * R + r; LG * R =
// N) into S.acc[rhs0 ..]: butterfly across the lane groups of a wavefront,
// then the wavefronts in index order -- a fixed order.
template <int R> __device__ __forceinline__ void flush_acc(Shared &S, double v[4], int LG, int rhs0)
{
    for (int o = 32; o >= LG; o >>= 1) {
#pragma unroll
        for (int r = 0; r < R; r++) v[r] += __shfl_xor(v[r], o, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane < LG) {
#pragma unroll
        for (int r = 0; r < R; r++) S.red[w * kMaxRhs + lane * R + r] = v[r];
    }
    __syncthreads();
    if ((int)threadIdx.x < LG * R) {
        double s = 0.0;
        for (int k = 0; k < kWaves; k++) s += S.red[k * kMaxRhs + threadIdx.x];
        S.acc[rhs0 + threadIdx.x] += s;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; r++) v[r] = 0.0;
}

// flush for problem P: groups of four lanes (R = N / (4 gps) right-hand sides
// per lane, N / R lanes per site) or one lane per rhs
__device__ __forceinline__ void flush_prob(Shared &S, double v[4], const BatchProb &P, bool four)
{
    const int N = 1 << P.logN;
    if (!four || N == 4 * P.gps) flush_acc<1>(S, v, N, P.rhs0);
    else flush_acc<2>(S, v, N / 2, P.rhs0);
}

// this workgroup's sums -> its row of `rows`; S.acc cleared
__device__ __forceinline__ void write_row(const BatchArgs *A, double *rows, Shared &S)
{
    const int Q = A->total_rhs;
    for (int q = threadIdx.x; q < Q; q += kBB) {
        rows[(size_t)blockIdx.x * Q + q] = S.acc[q];
        S.acc[q] = 0.0;
    }
}

// Sum of all workgroups' rows for right-hand side threadIdx.x (valid below
// total_rhs), in an order that is the same in every workgroup: C = kBB / Q
// chunk sums per right-hand side, then those C by one wavefront per
// right-hand side (lane l adds chunks l, l + 64, ..., then a butterfly),
// which keeps the serial part short (summing the chunks in one lane took
// C dependent LDS reads, 85 at Q = 12).
__device__ double sum_rows(const BatchArgs *A, const double *rows, Shared &S)
{
    const int Q = A->total_rhs, G = gridDim.x, C = kBB / Q;
    const int t = threadIdx.x, q = t % Q, c = t / Q;
    double s = 0.0;
    if (c < C)
        for (int b = c; b < G; b += C) s += ld_f64(rows + (size_t)b * Q + q);
    S.red[t] = s;
    __syncthreads();
    const int w = t >> 6, lane = t & 63;
    for (int r = w; r < Q; r += kBB / 64) {
        double x = 0.0;
        for (int k = lane; k < C; k += 64) x += S.red[k * Q + r];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0) S.tot[r] = x;
    }
    __syncthreads();
    return t < Q ? S.tot[t] : 0.0;
}

// After a scalar step: run flags, step coefficients (alpha after FIN_ALPHA,
// beta otherwise), per-problem masks. `sel_mode`: 0 keep sel, 1 select the
// right-hand sides due an FP64 update (`fixed`: interval reached).
__device__ void refresh(const BatchArgs *A, Shared &S, bool alpha, int sel_mode, bool fixed)
{
    const int Q = A->total_rhs, np = A->nprob;
    const int t = threadIdx.x;
    if (t < Q) {
        const CgState &s = S.st[t];
        const bool r = s.state == ST_RUN;
        S.run[t] = r;
        S.coef[t] = r ? (alpha ? s.alpha : s.beta) : 0.0;
        if (sel_mode) S.sel[t] = s.state == ST_INNER || (fixed && r);
    }
    __syncthreads();
    if (t < np) {
        const BatchProb &P = A->prob[t];
        int ar = 0, as = 0;
        for (int k = 0; k < (1 << P.logN); k++) {
            ar |= S.run[P.rhs0 + k];
            as |= S.sel[P.rhs0 + k];
        }
        S.prun[t] = ar;
        S.psel[t] = as;
    }
    __syncthreads();
    if (t == 0) {
        int ar = 0, as = 0;
        for (int p = 0; p < np; p++) {
            ar |= S.prun[p];
            as |= S.psel[p];
        }
        S.any_run = ar;
        S.any_sel = as;
    }
    __syncthreads();
}

// ---- inner-precision steps, four lanes per site
//
// Step 1 (odd sites): t = D_oe p', with p' = r + beta p formed from r and the
// previous p; the owner of each even index writes p' into the other p buffer.
// Where it fits in the workgroup's LDS (kBatchStageBytes), p' is formed once
// per site over the tile's x/y neighbourhood and staged there, so those hops
// read one staged vector instead of gathering two; z and t hops gather r and
// p from memory. Measured at 24^3 x 48 x 16: step 1 280 -> 235 us. Partial m4 |p'|^2 + |t|^2 = <p', A p'> (A =
// 4m^2 - D_eo D_oe and D_eo = -D_oe^dag), from which alpha follows before
// step 2. Step 2 (even sites): Ap = m4 p' - D_eo t, then at once x += alpha
// p', r -= alpha Ap and the partial |r|^2 for beta; Ap is never stored.

// LDS staging of one tile's multi-RHS input (the tile's sites and their x and
// y neighbours: the cb range [first - Lx/2, last + Lx/2]), FP32 complex in
// the layout [3][ns][N]; `get(e)` yields element e of the [3][V/2][N] global
// layout. Called by every thread of the workgroup (it holds two barriers).
template <class Get>
__device__ __forceinline__ void stage_tile(const BatchProb &P, int s0, int ns, fv2 *lds, Get get)
{
    const int logN = P.logN, N = 1 << logN, plane = ns << logN, Vh = P.g.Vh;
    __syncthreads(); // the previous tile's reads of lds are done
    for (int i = threadIdx.x; i < 3 * plane; i += kBB) {
        const int c = i / plane, rem = i - c * plane, n = s0 + (rem >> logN);
        if (n >= 0 && n < Vh) lds[i] = get((((size_t)c * Vh + n) << logN) + (rem & (N - 1)), rem & (N - 1));
    }
    __syncthreads();
}

template <class LF, int R, int GPS, bool MFMA>
__device__ __forceinline__ void step1_four(const BatchProb &P, const Shared &S, int dt, const void *pold, void *pnew,
                                           double v[4], fv2 *lds)
{
    constexpr int LPS = 4 * GPS; // lanes per site
    constexpr int TS = kBB / LPS; // sites per tile
    const size_t Vh = (size_t)P.g.Vh;
    const int logN = P.logN;
    const void *rv = P.r;
    // p' = r + beta p over the tile's staged range, formed once per site
    const int s0 = dt * TS - P.g.hx, ns = P.stage ? TS + 2 * P.g.hx : 0;
    if (P.stage)
        stage_tile(P, s0, ns, lds, [&](size_t e, int rhs) __attribute__((always_inline)) {
            const fv2 a = ((const fv2 *)rv)[e], b = ((const fv2 *)pold)[e];
            const float be = (float)S.coef[P.rhs0 + rhs];
            return fv2{fmaf(be, b.x, a.x), fmaf(be, b.y, a.y)};
        });
    const unsigned s = (unsigned)dt * TS + threadIdx.x / LPS, lane4 = threadIdx.x & 3u;
    // whole wavefronts leave together: V/2 is a multiple of 16 for MFMA
    if (s >= (unsigned)P.g.Vh) return;
    const unsigned r0 = (threadIdx.x % LPS) * R; // group g, lane l: rhs (4 g + l) R + r
    float beta[R];
#pragma unroll
    for (int r = 0; r < R; r++) beta[r] = (float)S.coef[P.rhs0 + r0 + r];
    auto IN = [=](int n, cx<float> v[R][3]) __attribute__((always_inline)) {
        const unsigned j = (unsigned)(n - s0);
        if (j < (unsigned)ns) { // staged: x and y neighbours, and the site itself
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const fv2 *q = lds + (((size_t)c * ns + j) << logN) + r0;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    v[r][c].re = q[r].x;
                    v[r][c].im = q[r].y;
                }
            }
            return;
        }
        cx<float> pp[R][3];
        ldm_r<float, R>(rv, Vh, logN, n, r0, v);
        ldm_r<float, R>(pold, Vh, logN, n, r0, pp);
#pragma unroll
        for (int r = 0; r < R; r++) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                v[r][c].re = fmaf(beta[r], pp[r][c].re, v[r][c].re);
                v[r][c].im = fmaf(beta[r], pp[r][c].im, v[r][c].im);
            }
        }
    };
    cx<float> acc[R][3], pp[R][3];
    dslash_site4<LF, R, MFMA>(P.g, kOdd, P.Ulo, s, lane4, IN, acc);
    stm_r<float, R>(P.t, Vh, logN, s, r0, acc);
    IN(s, pp);
    stm_r<float, R>(pnew, Vh, logN, s, r0, pp);
    const double m4 = P.m4;
#pragma unroll
    for (int r = 0; r < R; r++) {
        double tt = 0.0, qq = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            tt += (double)acc[r][c].re * (double)acc[r][c].re + (double)acc[r][c].im * (double)acc[r][c].im;
            qq += (double)pp[r][c].re * (double)pp[r][c].re + (double)pp[r][c].im * (double)pp[r][c].im;
        }
        if (S.run[P.rhs0 + r0 + r]) v[r] += m4 * qq + tt;
    }
}

// (Staging t as step 1 stages p' was measured and not kept: t is one vector
// read once per neighbour, and the staging barriers and registers cost more
// than the cache hits it replaces.)
template <class LF, int R, int GPS, bool MFMA>
__device__ __forceinline__ void step2_four(const BatchProb &P, const Shared &S, int dt, const void *pnew, double v[4])
{
    constexpr int LPS = 4 * GPS; // lanes per site
    const unsigned s = (unsigned)dt * (kBB / LPS) + threadIdx.x / LPS, lane4 = threadIdx.x & 3u;
    if (s >= (unsigned)P.g.Vh) return;
    const size_t Vh = (size_t)P.g.Vh;
    const int logN = P.logN;
    const unsigned r0 = (threadIdx.x % LPS) * R; // group g, lane l: rhs (4 g + l) R + r
    const void *tv = P.t;
    auto IN = [=](int n, cx<float> u[R][3]) __attribute__((always_inline)) { ldm_r<float, R>(tv, Vh, logN, n, r0, u); };
    cx<float> acc[R][3], pp[R][3], x[R][3], rr[R][3];
    dslash_site4<LF, R, MFMA>(P.g, kEven, P.Ulo, s, lane4, IN, acc);
    ldm_r<float, R>(pnew, Vh, logN, s, r0, pp);
    ldm_r<float, R>(P.xlo, Vh, logN, s, r0, x);
    ldm_r<float, R>(P.r, Vh, logN, s, r0, rr);
    const float m4 = (float)P.m4;
#pragma unroll
    for (int r = 0; r < R; r++) {
        // alpha is 0 for right-hand sides that are not iterating: x and r stay
        const float alpha = (float)S.coef[P.rhs0 + r0 + r];
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const float apr = m4 * pp[r][c].re - acc[r][c].re;
            const float api = m4 * pp[r][c].im - acc[r][c].im;
            x[r][c].re = fmaf(alpha, pp[r][c].re, x[r][c].re);
            x[r][c].im = fmaf(alpha, pp[r][c].im, x[r][c].im);
            rr[r][c].re = fmaf(-alpha, apr, rr[r][c].re);
            rr[r][c].im = fmaf(-alpha, api, rr[r][c].im);
            d += (double)rr[r][c].re * (double)rr[r][c].re + (double)rr[r][c].im * (double)rr[r][c].im;
        }
        if (S.run[P.rhs0 + r0 + r]) v[r] += d;
    }
    stm_r<float, R>(P.xlo, Vh, logN, s, r0, x);
    stm_r<float, R>(P.r, Vh, logN, s, r0, rr);
}

// ---- inner-precision steps, one lane per (site, rhs)

template <class LF>
__device__ __forceinline__ void step1_lane(const BatchProb &P, const Shared &S, int lt, const void *pold, void *pnew,
                                           double v[4])
{
    using T = typename LF::real;
    const unsigned idx = (unsigned)lt * kBB + threadIdx.x;
    const unsigned site = idx >> P.logN, rhs = idx & ((1u << P.logN) - 1u);
    if (site >= (unsigned)P.g.Vh) return;
    const size_t Vh = (size_t)P.g.Vh;
    const int logN = P.logN;
    const void *rv = P.r;
    const T beta = (T)S.coef[P.rhs0 + rhs];
    auto IN = [=](int n, cx<T> v[3]) __attribute__((always_inline)) {
        cx<T> pp[3];
        ldm<T>(rv, Vh, logN, n, rhs, v);
        ldm<T>(pold, Vh, logN, n, rhs, pp);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            v[c].re = fma(beta, pp[c].re, v[c].re);
            v[c].im = fma(beta, pp[c].im, v[c].im);
        }
    };
    cx<T> acc[3], pp[3];
    dslash_mrhs<LF>(P.g, kOdd, P.Ulo, site, IN, acc);
    stm<T>(P.t, Vh, logN, site, rhs, acc);
    IN(site, pp);
    stm<T>(pnew, Vh, logN, site, rhs, pp);
    double tt = 0.0, qq = 0.0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        tt += (double)acc[c].re * (double)acc[c].re + (double)acc[c].im * (double)acc[c].im;
        qq += (double)pp[c].re * (double)pp[c].re + (double)pp[c].im * (double)pp[c].im;
    }
    if (S.run[P.rhs0 + rhs]) v[0] += P.m4 * qq + tt;
}

template <class LF>
__device__ __forceinline__ void step2_lane(const BatchProb &P, const Shared &S, int lt, const void *pnew, double v[4])
{
    using T = typename LF::real;
    const unsigned idx = (unsigned)lt * kBB + threadIdx.x;
    const unsigned site = idx >> P.logN, rhs = idx & ((1u << P.logN) - 1u);
    if (site >= (unsigned)P.g.Vh) return;
    const size_t Vh = (size_t)P.g.Vh;
    const int logN = P.logN;
    const void *tv = P.t;
    auto IN = [=](int n, cx<T> u[3]) __attribute__((always_inline)) { ldm<T>(tv, Vh, logN, n, rhs, u); };
    cx<T> acc[3], pp[3], x[3], rr[3];
    dslash_mrhs<LF>(P.g, kEven, P.Ulo, site, IN, acc);
    ldm<T>(pnew, Vh, logN, site, rhs, pp);
    ldm<T>(P.xlo, Vh, logN, site, rhs, x);
    ldm<T>(P.r, Vh, logN, site, rhs, rr);
    const T m4 = (T)P.m4;
    const T alpha = (T)S.coef[P.rhs0 + rhs]; // 0 unless iterating: x and r stay
    double d = 0.0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const T apr = m4 * pp[c].re - acc[c].re;
        const T api = m4 * pp[c].im - acc[c].im;
        x[c].re = fma(alpha, pp[c].re, x[c].re);
        x[c].im = fma(alpha, pp[c].im, x[c].im);
        rr[c].re = fma(-alpha, apr, rr[c].re);
        rr[c].im = fma(-alpha, api, rr[c].im);
        d += (double)rr[c].re * (double)rr[c].re + (double)rr[c].im * (double)rr[c].im;
    }
    if (S.run[P.rhs0 + rhs]) v[0] += d;
    stm<T>(P.xlo, Vh, logN, site, rhs, x);
    stm<T>(P.r, Vh, logN, site, rhs, rr);
}

// ---- step 1 split in two passes (BatchArgs::split): (a) p' = r + beta p over
// the even sites, elementwise, with the partial m4 |p'|^2; a grid barrier;
// (b) t = D_oe p' gathering one vector, with the partial |t|^2. Same
// arithmetic per element as the fused step 1.

template <typename T>
__device__ __forceinline__ void step1_p(const BatchProb &P, const Shared &S, int lt, const void *pold, void *pnew,
                                        double v[4])
{
    const unsigned idx = (unsigned)lt * kBB + threadIdx.x;
    const unsigned site = idx >> P.logN, rhs = idx & ((1u << P.logN) - 1u);
    if (site >= (unsigned)P.g.Vh) return;
    const size_t Vh = (size_t)P.g.Vh;
    const T beta = (T)S.coef[P.rhs0 + rhs];
    cx<T> r[3], p[3];
    ldm<T>(P.r, Vh, P.logN, site, rhs, r);
    ldm<T>(pold, Vh, P.logN, site, rhs, p);
    double qq = 0.0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        r[c].re = fma(beta, p[c].re, r[c].re);
        r[c].im = fma(beta, p[c].im, r[c].im);
        qq += (double)r[c].re * (double)r[c].re + (double)r[c].im * (double)r[c].im;
    }
    stm<T>(pnew, Vh, P.logN, site, rhs, r);
    if (S.run[P.rhs0 + rhs]) v[0] += P.m4 * qq;
}

template <class LF, int R, int GPS, bool MFMA>
__device__ __forceinline__ void step1_d_four(const BatchProb &P, const Shared &S, int dt, const void *pnew, double v[4])
{
    constexpr int LPS = 4 * GPS;
    const unsigned s = (unsigned)dt * (kBB / LPS) + threadIdx.x / LPS, lane4 = threadIdx.x & 3u;
    if (s >= (unsigned)P.g.Vh) return;
    const size_t Vh = (size_t)P.g.Vh;
    const int logN = P.logN;
    const unsigned r0 = (threadIdx.x % LPS) * R;
    auto IN = [=](int n, cx<float> u[R][3]) __attribute__((always_inline)) { ldm_r<float, R>(pnew, Vh, logN, n, r0, u); };
    cx<float> acc[R][3];
    dslash_site4<LF, R, MFMA>(P.g, kOdd, P.Ulo, s, lane4, IN, acc);
    stm_r<float, R>(P.t, Vh, logN, s, r0, acc);
#pragma unroll
    for (int r = 0; r < R; r++) {
        double tt = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++)
            tt += (double)acc[r][c].re * (double)acc[r][c].re + (double)acc[r][c].im * (double)acc[r][c].im;
        if (S.run[P.rhs0 + r0 + r]) v[r] += tt;
    }
}

template <class LF>
__device__ __forceinline__ void step1_d_lane(const BatchProb &P, const Shared &S, int lt, const void *pnew, double v[4])
{
    using T = typename LF::real;
    const unsigned idx = (unsigned)lt * kBB + threadIdx.x;
    const unsigned site = idx >> P.logN, rhs = idx & ((1u << P.logN) - 1u);
    if (site >= (unsigned)P.g.Vh) return;
    const size_t Vh = (size_t)P.g.Vh;
    const int logN = P.logN;
    auto IN = [=](int n, cx<T> u[3]) __attribute__((always_inline)) { ldm<T>(pnew, Vh, logN, n, rhs, u); };
    cx<T> acc[3];
    dslash_mrhs<LF>(P.g, kOdd, P.Ulo, site, IN, acc);
    stm<T>(P.t, Vh, logN, site, rhs, acc);
    double tt = 0.0;
#pragma unroll
    for (int c = 0; c < 3; c++) tt += (double)acc[c].re * (double)acc[c].re + (double)acc[c].im * (double)acc[c].im;
    if (S.run[P.rhs0 + rhs]) v[0] += tt;
}

// engine dispatch for the inner steps (four-lane engines for F32/BF16 links only)
template <class LF>
__device__ __forceinline__ void step1_d(const BatchProb &P, const Shared &S, int dt, const void *pnew, double v[4])
{
    if constexpr (!std::is_same<typename LF::real, double>::value) {
        if (P.eng != MRHS_LANE) {
            const bool mf = P.eng == MRHS_MFMA;
#define LGT_STEP1D(R, G) (mf ? step1_d_four<LF, R, G, true>(P, S, dt, pnew, v) : step1_d_four<LF, R, G, false>(P, S, dt, pnew, v))
            if (P.logN == 2) LGT_STEP1D(1, 1);
            else if (P.logN == 3) P.gps == 2 ? LGT_STEP1D(1, 2) : LGT_STEP1D(2, 1);
            else P.gps == 4 ? LGT_STEP1D(1, 4) : LGT_STEP1D(2, 2);
#undef LGT_STEP1D
            return;
        }
    }
    step1_d_lane<LF>(P, S, dt, pnew, v);
}

template <class LF>
__device__ __forceinline__ void step1(const BatchProb &P, const Shared &S, int dt, const void *pold, void *pnew,
                                      double v[4], fv2 *lds)
{
    if constexpr (!std::is_same<typename LF::real, double>::value) {
        if (P.eng != MRHS_LANE) {
            const bool mf = P.eng == MRHS_MFMA;
#define LGT_STEP1(R, G) (mf ? step1_four<LF, R, G, true>(P, S, dt, pold, pnew, v, lds) : step1_four<LF, R, G, false>(P, S, dt, pold, pnew, v, lds))
            if (P.logN == 2) LGT_STEP1(1, 1);
            else if (P.logN == 3) P.gps == 2 ? LGT_STEP1(1, 2) : LGT_STEP1(2, 1);
            else P.gps == 4 ? LGT_STEP1(1, 4) : LGT_STEP1(2, 2);
#undef LGT_STEP1
            return;
        }
    }
    step1_lane<LF>(P, S, dt, pold, pnew, v);
}

template <class LF>
__device__ __forceinline__ void step2(const BatchProb &P, const Shared &S, int dt, const void *pnew, double v[4])
{
    if constexpr (!std::is_same<typename LF::real, double>::value) {
        if (P.eng != MRHS_LANE) {
            const bool mf = P.eng == MRHS_MFMA;
#define LGT_STEP2(R, G) (mf ? step2_four<LF, R, G, true>(P, S, dt, pnew, v) : step2_four<LF, R, G, false>(P, S, dt, pnew, v))
            if (P.logN == 2) LGT_STEP2(1, 1);
            else if (P.logN == 3) P.gps == 2 ? LGT_STEP2(1, 2) : LGT_STEP2(2, 1);
            else P.gps == 4 ? LGT_STEP2(1, 4) : LGT_STEP2(2, 2);
#undef LGT_STEP2
            return;
        }
    }
    step2_lane<LF>(P, S, dt, pnew, v);
}

} // namespace

template <class LF>
__global__ __launch_bounds__(kBB) void k_batch_cg(const BatchArgs *__restrict__ A)
{
    using T = typename LF::real;
    using LH = LinkF64R18;
    constexpr bool mixed = !std::is_same<T, double>::value;
    __shared__ Shared S;
    extern __shared__ __align__(16) unsigned char batch_lds[]; // staged tiles (kBatchStageBytes)
    fv2 *lds = (fv2 *)batch_lds;
    BatchCtl *ctl = A->ctl;
    const unsigned int lim = A->spin_limit;
    const int Q = A->total_rhs, np = A->nprob;
    double v[4] = {0.0, 0.0, 0.0, 0.0};

    // every workgroup keeps its own copy of the states
    for (int q = threadIdx.x; q < Q; q += kBB) {
        CgState &s = S.st[q];
        s.rho = s.rho_prev = s.alpha = s.beta = s.pAp = 0.0;
        s.bnorm2 = 0.0;
        s.stop_outer = A->tol * A->tol;
        s.stop_inner = 0.0;
        s.inner2 = A->scheme == SCH_REFINE ? A->inner * A->inner : (A->inner * A->tol) * (A->inner * A->tol);
        s.last_true = 0.0;
        s.iter = 0;
        s.updates = 0;
        s.state = ST_INIT;
        s.max_iter = A->max_iter;
        s.scheme = A->scheme;
        s.ru_fixed = A->scheme == SCH_RELIABLE;
        s.pend = s.pcur = 0;
        S.acc[q] = 0.0;
        S.coef[q] = 0.0;
        S.run[q] = 0;
        S.sel[q] = 1;
    }
    for (int p = threadIdx.x; p < np; p += kBB) {
        S.prun[p] = 0;
        S.psel[p] = 1;
    }
    if (threadIdx.x < kBatchPhases) S.prof[threadIdx.x] = 0ull;
    __syncthreads();
    mark(A, S, -1);

    auto flush_lane = [&](int p) { flush_prob(S, v, A->prob[p], false); };
    auto no_flush = [](int) {};

    // FP64 step on the selected right-hand sides: x64 += xlo, xlo = 0,
    // r = b - A x64 (rounded to the inner precision), scalar step `fin` on
    // |b - A x64|^2
    auto fp64_step = [&](int fin) -> bool {
        tiles<false>(
            A, S.psel,
            [&](const BatchProb &P, int lt) {
                const unsigned idx = (unsigned)lt * kBB + threadIdx.x;
                const unsigned site = idx >> P.logN, rhs = idx & ((1u << P.logN) - 1u);
                if (site >= (unsigned)P.g.Vh || !S.sel[P.rhs0 + rhs]) return;
                const size_t Vh = (size_t)P.g.Vh;
                const int logN = P.logN;
                const double *x64 = P.x64;
                const void *xlo = P.xlo;
                auto IN = [=](int n, cx<double> u[3]) __attribute__((always_inline)) {
                    ldm<double>(x64, Vh, logN, n, rhs, u);
                    if constexpr (mixed) {
                        cx<T> e[3];
                        ldm<T>(xlo, Vh, logN, n, rhs, e);
#pragma unroll
                        for (int c = 0; c < 3; c++) {
                            u[c].re += (double)e[c].re;
                            u[c].im += (double)e[c].im;
                        }
                    }
                };
                cx<double> acc[3];
                dslash_mrhs<LH>(P.g, kOdd, P.Uhi, site, IN, acc);
                stm<double>(P.t64, Vh, logN, site, rhs, acc);
            },
            no_flush);
        if (!grid_sync(ctl, lim, S)) return false;
        tiles<false>(
            A, S.psel,
            [&](const BatchProb &P, int lt) {
                const unsigned idx = (unsigned)lt * kBB + threadIdx.x;
                const unsigned site = idx >> P.logN, rhs = idx & ((1u << P.logN) - 1u);
                if (site >= (unsigned)P.g.Vh || !S.sel[P.rhs0 + rhs]) return;
                const size_t Vh = (size_t)P.g.Vh;
                const int logN = P.logN;
                const double *t64 = P.t64;
                auto IN = [=](int n, cx<double> u[3]) __attribute__((always_inline)) { ldm<double>(t64, Vh, logN, n, rhs, u); };
                cx<double> acc[3], x[3], bb[3];
                dslash_mrhs<LH>(P.g, kEven, P.Uhi, site, IN, acc);
                ldm<double>(P.x64, Vh, logN, site, rhs, x);
                ldm<double>(P.b64, Vh, logN, site, rhs, bb);
                if constexpr (mixed) {
                    cx<T> e[3];
                    ldm<T>(P.xlo, Vh, logN, site, rhs, e);
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        x[c].re += (double)e[c].re;
                        x[c].im += (double)e[c].im;
                        e[c].re = e[c].im = T(0);
                    }
                    stm<double>(P.x64, Vh, logN, site, rhs, x);
                    stm<T>(P.xlo, Vh, logN, site, rhs, e);
                }
                cx<T> lo[3];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    acc[c].re = bb[c].re - (P.m4 * x[c].re - acc[c].re);
                    acc[c].im = bb[c].im - (P.m4 * x[c].im - acc[c].im);
                    v[0] += acc[c].re * acc[c].re + acc[c].im * acc[c].im;
                    lo[c].re = (T)acc[c].re;
                    lo[c].im = (T)acc[c].im;
                }
                stm<T>(P.r, Vh, logN, site, rhs, lo);
            },
            flush_lane);
        write_row(A, A->rows[1], S);
        if (!grid_sync(ctl, lim, S)) return false;
        const double tot = sum_rows(A, A->rows[1], S);
        if ((int)threadIdx.x < Q && S.sel[threadIdx.x]) finalize(fin, &S.st[threadIdx.x], tot);
        __syncthreads();
        refresh(A, S, false, 0, false);
        return true;
    };

    bool ok = true;
    // ---- set-up: |b|^2, then r = b - A x0 (beta = 0)
    tiles<false>(
        A, S.psel,
        [&](const BatchProb &P, int lt) {
            const unsigned idx = (unsigned)lt * kBB + threadIdx.x;
            const unsigned site = idx >> P.logN, rhs = idx & ((1u << P.logN) - 1u);
            if (site >= (unsigned)P.g.Vh) return;
            cx<double> bb[3];
            ldm<double>(P.b64, (size_t)P.g.Vh, P.logN, site, rhs, bb);
#pragma unroll
            for (int c = 0; c < 3; c++) v[0] += bb[c].re * bb[c].re + bb[c].im * bb[c].im;
        },
        flush_lane);
    write_row(A, A->rows[0], S);
    ok = grid_sync(ctl, lim, S);
    if (ok) {
        const double tot = sum_rows(A, A->rows[0], S);
        if ((int)threadIdx.x < Q) finalize(FIN_INIT, &S.st[threadIdx.x], tot);
        __syncthreads();
        ok = fp64_step(FIN_RU);
    }
    mark(A, S, PH_SETUP);

    // ---- iterations, all right-hand sides of all problems in lock-step
    const int cap = A->max_iter + 2;
    for (int it = 0; ok && S.any_run && it < cap; it++) {
        // 1. t = D_oe p', p' = r + beta p (written to the other p buffer),
        //    <p', A p'> = m4 |p'|^2 + |t|^2  -> alpha
        if (A->split) {
            tiles<false>(
                A, S.prun,
                [&](const BatchProb &P, int lt) {
                    step1_p<T>(P, S, lt, (it & 1) ? P.pb : P.pa, (it & 1) ? P.pa : P.pb, v);
                },
                flush_lane);
            mark(A, S, PH_STEP1P);
            if (!(ok = grid_sync(ctl, lim, S))) break;
            mark(A, S, PH_WAIT1P);
            tiles<true>(
                A, S.prun, [&](const BatchProb &P, int dt) { step1_d<LF>(P, S, dt, (it & 1) ? P.pa : P.pb, v); },
                [&](int p) { flush_prob(S, v, A->prob[p], mixed && A->prob[p].eng != MRHS_LANE); });
        } else {
            tiles<true>(
                A, S.prun,
                [&](const BatchProb &P, int dt) {
                    const void *po = (it & 1) ? P.pb : P.pa;
                    void *pn = (it & 1) ? P.pa : P.pb;
                    step1<LF>(P, S, dt, po, pn, v, lds);
                },
                [&](int p) { flush_prob(S, v, A->prob[p], mixed && A->prob[p].eng != MRHS_LANE); });
        }
        write_row(A, A->rows[0], S);
        mark(A, S, PH_STEP1);
        if (!(ok = grid_sync(ctl, lim, S))) break;
        mark(A, S, PH_WAIT1);
        {
            const double tot = sum_rows(A, A->rows[0], S);
            if ((int)threadIdx.x < Q && S.run[threadIdx.x]) finalize(FIN_ALPHA, &S.st[threadIdx.x], tot);
            __syncthreads();
            refresh(A, S, true, 0, false);
        }
        mark(A, S, PH_SCALAR);
        // 2. Ap = m4 p' - D_eo t ; x += alpha p', r -= alpha Ap ; |r|^2  -> beta, stop tests
        tiles<true>(
            A, S.prun,
            [&](const BatchProb &P, int dt) { step2<LF>(P, S, dt, (it & 1) ? P.pa : P.pb, v); },
            [&](int p) { flush_prob(S, v, A->prob[p], mixed && A->prob[p].eng != MRHS_LANE); });
        write_row(A, A->rows[1], S);
        mark(A, S, PH_STEP2);
        if (!(ok = grid_sync(ctl, lim, S))) break;
        mark(A, S, PH_WAIT2);
        {
            const double tot = sum_rows(A, A->rows[1], S);
            if ((int)threadIdx.x < Q && S.run[threadIdx.x]) finalize(FIN_UPDATE, &S.st[threadIdx.x], tot);
            __syncthreads();
            const bool fixed = A->scheme == SCH_RELIABLE && (it + 1) % A->ru_interval == 0;
            refresh(A, S, false, 1, fixed);
        }
        mark(A, S, PH_SCALAR);
        if (S.any_sel) ok = fp64_step(FIN_RU);
        mark(A, S, PH_FP64);
        if (blockIdx.x == 0 && threadIdx.x == 0) ctl->iters_done = it + 1;
    }

    // ---- final: accumulate x, FP64 true residual of every right-hand side
    if (ok) {
        for (int q = threadIdx.x; q < Q; q += kBB) S.sel[q] = 1;
        for (int p = threadIdx.x; p < np; p += kBB) S.psel[p] = 1;
        __syncthreads();
        ok = fp64_step(FIN_FINAL);
    }
    mark(A, S, PH_SETUP);
    if (blockIdx.x == 0) {
        for (int q = threadIdx.x; q < Q; q += kBB) A->states[q] = S.st[q];
        if (A->prof && threadIdx.x < kBatchPhases) A->prof[threadIdx.x] = S.prof[threadIdx.x];
    }
}

template <class LF> static int max_blocks_per_cu()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_cg<LF>, kBB, kBatchStageBytes) != hipSuccess)
        return 0;
    return n;
}

int batch_cg_max_blocks_per_cu(Fmt lo)
{
    switch (lo) {
    case F64R18: return max_blocks_per_cu<LinkF64R18>();
    case F32R18: return max_blocks_per_cu<LinkF32R18>();
    case F32R12: return max_blocks_per_cu<LinkF32R12>();
    case BF16R12: return max_blocks_per_cu<LinkBF16R12>();
    default: return 0;
    }
}

hipError_t launch_batch_cg(Fmt lo, const BatchArgs *a_dev, int grid, hipStream_t s)
{
    void *args[] = {(void *)&a_dev};
    const void *fn;
    switch (lo) {
    case F64R18: fn = (const void *)k_batch_cg<LinkF64R18>; break;
    case F32R18: fn = (const void *)k_batch_cg<LinkF32R18>; break;
    case F32R12: fn = (const void *)k_batch_cg<LinkF32R12>; break;
    case BF16R12: fn = (const void *)k_batch_cg<LinkBF16R12>; break;
    default: return hipErrorInvalidValue;
    }
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBB), args, kBatchStageBytes, s);
}

} // namespace lgt
