// mrhs.hip -- many right-hand sides: the multi-RHS staggered Dslash and the
// persistent batched CG.
//
// Thread = (site, right-hand side). With the RHS fastest in the vector layout
// [3][V/2][N], the N lanes of a site read one contiguous run of each input
// and output, and issue the same link address, which the load unit serves
// once: a link is fetched from memory once per site for all N right-hand
// sides, so the HBM bytes per site and RHS fall from 8 links + 2 vectors to
// 8/N links + 2 vectors.
//
// The batched solver runs independent CGs (one alpha, beta and state per
// right-hand side; not block CG) for every right-hand side of every problem
// -- lattices of different sizes included -- in one cooperative launch. Its
// phases are separated by a grid barrier; p = r + beta p is folded into the
// next D_oe (which reads r and the previous p at the neighbours and also
// writes the new p, into the other of two p buffers), and the FP64 reliable
// updates run inside the same launch.
#include "batch.hpp"
#include "fields.hpp"
#include "mrhs4.hpp"
#include "reduce.hpp"

namespace lgt {

constexpr int kEven = 0, kOdd = 1; // output parity of a half-Dslash

template <typename T> struct V2of;
template <> struct V2of<double> { using type = dv2; };
template <> struct V2of<float> { using type = fv2; };

// element (colour c, site, rhs) of a multi-RHS vector; the plane base is uniform
template <typename T>
__device__ __forceinline__ void ldm(const void *v, size_t Vh, int logN, unsigned site, unsigned rhs, cx<T> o[3])
{
    using V2 = typename V2of<T>::type;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const V2 w = ld<false>((const V2 *)v + ((size_t)c * Vh << logN), (site << logN) + rhs);
        o[c].re = w.x;
        o[c].im = w.y;
    }
}

template <typename T>
__device__ __forceinline__ void stm(void *v, size_t Vh, int logN, unsigned site, unsigned rhs, const cx<T> o[3])
{
    using V2 = typename V2of<T>::type;
#pragma unroll
    for (int c = 0; c < 3; c++) st<false>((V2 *)v + ((size_t)c * Vh << logN), (site << logN) + rhs, V2{o[c].re, o[c].im});
}

// D on one (site, rhs): the input at a neighbour comes from `in(site, v)`.
template <class LF, class In>
__device__ __forceinline__ void dslash_mrhs(const Geom &g, int par, const void *U, int cb, In in,
                                            cx<typename LF::real> acc[3])
{
    using T = typename LF::real;
    const size_t Vh = (size_t)g.Vh;
    int c[4];
    decode(g, par, cb, c);
#pragma unroll
    for (int i = 0; i < 3; i++) acc[i].re = acc[i].im = T(0);
#pragma unroll 1
    for (int mu = 0; mu < 4; mu++) {
        const Hop h = hop_rt(g, c, cb, mu);
        cx<T> u[9], v[3];
        LF::template load<false>(U, Vh, par * 4 + mu, cb, u);
        in(h.f, v);
        negate_if(h.fneg, v);
        mv_add(u, v, acc);
        LF::template load<false>(U, Vh, (1 - par) * 4 + mu, h.b, u);
        in(h.b, v);
        negate_if(h.bneg, v);
        amv_sub(u, v, acc);
    }
}

// ------------------------------------------------------- standalone ---

template <class LF>
__global__ __launch_bounds__(kBS) void k_dslash_mrhs(const void *__restrict__ U, const void *__restrict__ in,
                                                     void *__restrict__ out, Geom g, int par, int logN, int nblk_pad)
{
    using T = typename LF::real;
    const unsigned idx = (unsigned)xcd_block(blockIdx.x, nblk_pad) * kBS + threadIdx.x;
    const unsigned site = idx >> logN, rhs = idx & ((1u << logN) - 1u);
    if (site >= (unsigned)g.Vh) return;
    const size_t Vh = (size_t)g.Vh;
    auto IN = [=](int s, cx<T> v[3]) __attribute__((always_inline)) { ldm<T>(in, Vh, logN, s, rhs, v); };
    cx<T> acc[3];
    dslash_mrhs<LF>(g, par, U, site, IN, acc);
    stm<T>(out, Vh, logN, site, rhs, acc);
}

// four lanes per site, R right-hand sides per lane, VALU or MFMA engine
template <class LF, int R, bool MFMA>
__global__ __launch_bounds__(kBS) void k_dslash_mrhs4(const void *__restrict__ U, const void *__restrict__ in,
                                                      void *__restrict__ out, Geom g, int par, int logN, int nblk_pad)
{
    const unsigned idx = (unsigned)xcd_block(blockIdx.x, nblk_pad) * kBS + threadIdx.x;
    const unsigned site = idx >> 2, lane4 = idx & 3u;
    // the 4 lanes of a site and the 16 sites of a wavefront stay together, and
    // a wavefront is never split by the bound below (Vh is a multiple of 16
    // whenever the MFMA engine is used: checked on the host)
    if (site >= (unsigned)g.Vh) return;
    const size_t Vh = (size_t)g.Vh;
    const unsigned rhs0 = lane4 * R;
    auto IN = [=](int s, cx<float> v[R][3]) __attribute__((always_inline)) { ldm_r<float, R>(in, Vh, logN, s, rhs0, v); };
    cx<float> acc[R][3];
    dslash_site4<LF, R, MFMA>(g, par, U, site, lane4, IN, acc);
    stm_r<float, R>(out, Vh, logN, site, rhs0, acc);
}

template <class LF>
static hipError_t launch_mrhs4(int engine, const void *U, const void *in, void *out, const Geom &g, int par, int logN,
                               hipStream_t s)
{
    const int64_t n = (int64_t)g.Vh * 4;
    const int nblk = (int)((n + kBS - 1) / kBS);
    const int pad = (nblk + 7) / 8 * 8;
    const dim3 grid(pad), block(kBS);
    const bool mf = engine == MRHS_MFMA;
    switch (logN) {
    case 2:
        if (mf) hipLaunchKernelGGL((k_dslash_mrhs4<LF, 1, true>), grid, block, 0, s, U, in, out, g, par, logN, pad);
        else hipLaunchKernelGGL((k_dslash_mrhs4<LF, 1, false>), grid, block, 0, s, U, in, out, g, par, logN, pad);
        break;
    case 3:
        if (mf) hipLaunchKernelGGL((k_dslash_mrhs4<LF, 2, true>), grid, block, 0, s, U, in, out, g, par, logN, pad);
        else hipLaunchKernelGGL((k_dslash_mrhs4<LF, 2, false>), grid, block, 0, s, U, in, out, g, par, logN, pad);
        break;
    case 4:
        if (mf) hipLaunchKernelGGL((k_dslash_mrhs4<LF, 4, true>), grid, block, 0, s, U, in, out, g, par, logN, pad);
        else hipLaunchKernelGGL((k_dslash_mrhs4<LF, 4, false>), grid, block, 0, s, U, in, out, g, par, logN, pad);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool mrhs_engine_applies(Fmt f, int logN, int Vh, int engine)
{
    if (engine == MRHS_LANE || logN < 2 || fmt_is_f64_fmt(f)) return false;
    return engine == MRHS_VALU4 || (Vh % 16) == 0;
}

hipError_t launch_dslash_mrhs(Fmt f, const void *U, const void *in, void *out, const Geom &g, int par, int logN,
                              hipStream_t s, int engine)
{
    if (mrhs_engine_applies(f, logN, g.Vh, engine)) {
        switch (f) {
        case F32R18: return launch_mrhs4<LinkF32R18>(engine, U, in, out, g, par, logN, s);
        case F32R12: return launch_mrhs4<LinkF32R12>(engine, U, in, out, g, par, logN, s);
        case BF16R12: return launch_mrhs4<LinkBF16R12>(engine, U, in, out, g, par, logN, s);
        default: break;
        }
    }
    const int64_t n = (int64_t)g.Vh << logN;
    const int nblk = (int)((n + kBS - 1) / kBS);
    const int pad = (nblk + 7) / 8 * 8;
    const dim3 grid(pad), block(kBS);
    switch (f) {
    case F64R18: hipLaunchKernelGGL(k_dslash_mrhs<LinkF64R18>, grid, block, 0, s, U, in, out, g, par, logN, pad); break;
    case F64R12: hipLaunchKernelGGL(k_dslash_mrhs<LinkF64R12>, grid, block, 0, s, U, in, out, g, par, logN, pad); break;
    case F32R18: hipLaunchKernelGGL(k_dslash_mrhs<LinkF32R18>, grid, block, 0, s, U, in, out, g, par, logN, pad); break;
    case F32R12: hipLaunchKernelGGL(k_dslash_mrhs<LinkF32R12>, grid, block, 0, s, U, in, out, g, par, logN, pad); break;
    case BF16R12: hipLaunchKernelGGL(k_dslash_mrhs<LinkBF16R12>, grid, block, 0, s, U, in, out, g, par, logN, pad); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// canonical [N][V/2][3][2] float64 <-> multi-RHS [3][V/2][N] of T
template <typename T>
__global__ __launch_bounds__(kBS) void k_pack_mrhs(const double *__restrict__ src, void *__restrict__ dst, int Vh,
                                                   int logN)
{
    const int64_t idx = (int64_t)blockIdx.x * kBS + threadIdx.x; // (site << logN) + rhs
    if (idx >= ((int64_t)Vh << logN)) return;
    const unsigned site = (unsigned)(idx >> logN), rhs = (unsigned)(idx & ((1 << logN) - 1));
    const dv2 *p = (const dv2 *)src + ((size_t)rhs * Vh + site) * 3;
    cx<T> v[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const dv2 w = p[c];
        v[c].re = (T)w.x;
        v[c].im = (T)w.y;
    }
    stm<T>(dst, (size_t)Vh, logN, site, rhs, v);
}

template <typename T>
__global__ __launch_bounds__(kBS) void k_unpack_mrhs(const void *__restrict__ src, double *__restrict__ dst, int Vh,
                                                     int logN)
{
    const int64_t idx = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (idx >= ((int64_t)Vh << logN)) return;
    const unsigned site = (unsigned)(idx >> logN), rhs = (unsigned)(idx & ((1 << logN) - 1));
    cx<T> v[3];
    ldm<T>(src, (size_t)Vh, logN, site, rhs, v);
    dv2 *p = (dv2 *)dst + ((size_t)rhs * Vh + site) * 3;
#pragma unroll
    for (int c = 0; c < 3; c++) p[c] = dv2{(double)v[c].re, (double)v[c].im};
}

hipError_t launch_pack_mrhs(bool f64, const double *src, void *dst, const Geom &g, int logN, hipStream_t s)
{
    const int64_t n = (int64_t)g.Vh << logN;
    const dim3 grid((unsigned)((n + kBS - 1) / kBS)), block(kBS);
    if (f64) hipLaunchKernelGGL(k_pack_mrhs<double>, grid, block, 0, s, src, dst, g.Vh, logN);
    else hipLaunchKernelGGL(k_pack_mrhs<float>, grid, block, 0, s, src, dst, g.Vh, logN);
    return hipGetLastError();
}

hipError_t launch_unpack_mrhs(bool f64, const void *src, double *dst, const Geom &g, int logN, hipStream_t s)
{
    const int64_t n = (int64_t)g.Vh << logN;
    const dim3 grid((unsigned)((n + kBS - 1) / kBS)), block(kBS);
    if (f64) hipLaunchKernelGGL(k_unpack_mrhs<double>, grid, block, 0, s, src, dst, g.Vh, logN);
    else hipLaunchKernelGGL(k_unpack_mrhs<float>, grid, block, 0, s, src, dst, g.Vh, logN);
    return hipGetLastError();
}

// --------------------------------------------------- persistent batch ---

// State words written by other workgroups in earlier phases are read with
// device-scope atomic loads, so no stale cached copy can be used.
__device__ __forceinline__ int ld_i32(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ double ld_f64(const double *p)
{
    return __longlong_as_double((long long)__hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT));
}

__device__ __forceinline__ CgState ld_state(const CgState *p)
{
    CgState s;
    s.rho = ld_f64(&p->rho);
    s.rho_prev = ld_f64(&p->rho_prev);
    s.alpha = ld_f64(&p->alpha);
    s.beta = ld_f64(&p->beta);
    s.pAp = ld_f64(&p->pAp);
    s.bnorm2 = ld_f64(&p->bnorm2);
    s.stop_outer = ld_f64(&p->stop_outer);
    s.stop_inner = ld_f64(&p->stop_inner);
    s.inner2 = ld_f64(&p->inner2);
    s.last_true = ld_f64(&p->last_true);
    s.iter = ld_i32(&p->iter);
    s.updates = ld_i32(&p->updates);
    s.state = ld_i32(&p->state);
    s.max_iter = ld_i32(&p->max_iter);
    s.scheme = ld_i32(&p->scheme);
    s.ru_fixed = ld_i32(&p->ru_fixed);
    s.pad0 = s.pad1 = 0;
    return s;
}

__device__ __forceinline__ bool gate_state(int gate, int state, int ru_fixed)
{
    if (gate == GATE_NONE) return true;
    if (gate == GATE_ITER) return state == ST_RUN;
    return state == ST_INIT || state == ST_INNER || (state == ST_RUN && ru_fixed);
}

// Grid barrier: device-scope release before arriving, acquire after leaving.
// A wait longer than `limit` polls gives up and raises ctl->err, so every
// wave of the launch always reaches the end of the kernel.
__device__ void grid_barrier(BatchCtl *ctl, unsigned int limit)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int gen = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned int arrived = atomicAdd(&ctl->bar_count, 1u);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(&ctl->bar_gen, 1u);
        } else {
            unsigned int n = 0;
            while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++n > limit) {
                    atomicOr(&ctl->err, 1u);
                    break;
                }
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// tiles of all problems, round-robin over the workgroups of the grid
template <class F> __device__ __forceinline__ void for_tiles(const BatchArgs *A, F f)
{
    for (int w = blockIdx.x; w < A->total_tiles; w += gridDim.x) {
        int p = 0;
        while (p + 1 < A->nprob && w >= A->prob[p + 1].tile0) p++;
        const BatchProb &P = A->prob[p];
        const unsigned idx = (unsigned)(w - P.tile0) * kBS + threadIdx.x;
        const unsigned site = idx >> P.logN, rhs = idx & ((1u << P.logN) - 1u);
        f(P, w, site, rhs, site < (unsigned)P.g.Vh);
    }
}

// per-tile partial sums, one per right-hand side, summed in a fixed order
__device__ __forceinline__ void tile_partial(double v, double *row, int logN)
{
    __shared__ double lds[kBS];
    lds[threadIdx.x] = v;
    __syncthreads();
    const int N = 1 << logN;
    if ((int)threadIdx.x < N) {
        double s = 0.0;
        for (int k = threadIdx.x; k < kBS; k += N) s += lds[k];
        row[threadIdx.x] = s;
    }
    __syncthreads();
}

// scalar step for every (problem, rhs) whose gate is open; counts the
// right-hand sides that keep iterating and those that need an FP64 update
__device__ void finalize_all(const BatchArgs *A, int fin, int gate, unsigned int *active, unsigned int *need_ru)
{
    __shared__ double lds[kBS / 64];
    for (int q = blockIdx.x; q < A->total_rhs; q += gridDim.x) {
        int p = 0;
        while (p + 1 < A->nprob && q >= A->prob[p + 1].rhs0) p++;
        const BatchProb &P = A->prob[p];
        const int rhs = q - P.rhs0;
        CgState *stp = P.st + rhs;
        const CgState s0 = ld_state(stp);
        if (!gate_state(gate, s0.state, s0.ru_fixed)) {
            if (threadIdx.x == 0 && active && (s0.state == ST_RUN || s0.state == ST_INNER)) {
                atomicAdd(active, 1u);
                if (s0.state == ST_INNER) atomicAdd(need_ru, 1u);
            }
            continue;
        }
        double acc = 0.0;
        for (int t = threadIdx.x; t < P.ntiles; t += kBS) acc += A->partials[(size_t)(P.tile0 + t) * kMaxRhs + rhs];
        const double tot = block_sum(acc, lds);
        if (threadIdx.x == 0) {
            CgState s = s0;
            finalize(fin, &s, tot);
            *stp = s;
            if (active && (s.state == ST_RUN || s.state == ST_INNER)) {
                atomicAdd(active, 1u);
                if (s.state == ST_INNER) atomicAdd(need_ru, 1u);
            }
        }
    }
}

__global__ void k_state_init_batch(const BatchArgs *A, double tol, double inner)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= A->total_rhs) return;
    int p = 0;
    while (p + 1 < A->nprob && q >= A->prob[p + 1].rhs0) p++;
    CgState *st = A->prob[p].st + (q - A->prob[p].rhs0);
    st->rho = st->rho_prev = st->alpha = st->beta = st->pAp = 0.0;
    st->bnorm2 = 0.0;
    st->stop_outer = tol * tol;
    st->stop_inner = 0.0;
    st->inner2 = A->scheme == SCH_REFINE ? inner * inner : (inner * tol) * (inner * tol);
    st->last_true = 0.0;
    st->iter = 0;
    st->updates = 0;
    st->state = ST_INIT;
    st->max_iter = A->max_iter;
    st->scheme = A->scheme;
    st->ru_fixed = A->scheme == SCH_RELIABLE;
    st->pad0 = st->pad1 = 0;
}

template <class LF>
__global__ __launch_bounds__(kBS) void k_batch_cg(const BatchArgs *__restrict__ A)
{
    using T = typename LF::real;
    using LH = LinkF64R18;
    constexpr bool mixed = !std::is_same<T, double>::value;
    BatchCtl *ctl = A->ctl;
    const unsigned int lim = A->spin_limit;
    double *part = A->partials;

    // FP64 update: x64 += x_lo ; t64 = D_oe x64 ; r = b - A64 x64 (rounded to the inner precision)
    auto reliable = [&](int gate, int fin, unsigned int *act, unsigned int *nru) {
        if (mixed) {
            for_tiles(A, [&](const BatchProb &P, int, unsigned site, unsigned rhs, bool ok) {
                if (!ok) return;
                const CgState *s = P.st + rhs;
                if (!gate_state(gate, ld_i32(&s->state), ld_i32(&s->ru_fixed))) return;
                cx<double> x[3];
                cx<T> e[3];
                const size_t Vh = (size_t)P.g.Vh;
                ldm<double>(P.x64, Vh, P.logN, site, rhs, x);
                ldm<T>(P.xlo, Vh, P.logN, site, rhs, e);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    x[c].re += (double)e[c].re;
                    x[c].im += (double)e[c].im;
                    e[c].re = e[c].im = T(0);
                }
                stm<double>(P.x64, Vh, P.logN, site, rhs, x);
                stm<T>(P.xlo, Vh, P.logN, site, rhs, e);
            });
            grid_barrier(ctl, lim);
        }
        for_tiles(A, [&](const BatchProb &P, int, unsigned site, unsigned rhs, bool ok) {
            if (!ok) return;
            const CgState *s = P.st + rhs;
            if (!gate_state(gate, ld_i32(&s->state), ld_i32(&s->ru_fixed))) return;
            const size_t Vh = (size_t)P.g.Vh;
            auto IN = [=](int n, cx<double> v[3]) __attribute__((always_inline)) { ldm<double>(P.x64, Vh, P.logN, n, rhs, v); };
            cx<double> acc[3];
            dslash_mrhs<LH>(P.g, kOdd, P.Uhi, site, IN, acc);
            stm<double>(P.t64, Vh, P.logN, site, rhs, acc);
        });
        grid_barrier(ctl, lim);
        for_tiles(A, [&](const BatchProb &P, int w, unsigned site, unsigned rhs, bool ok) {
            double v = 0.0;
            const CgState *s = P.st + rhs;
            if (ok && gate_state(gate, ld_i32(&s->state), ld_i32(&s->ru_fixed))) {
                const size_t Vh = (size_t)P.g.Vh;
                auto IN = [=](int n, cx<double> u[3]) __attribute__((always_inline)) { ldm<double>(P.t64, Vh, P.logN, n, rhs, u); };
                cx<double> acc[3], x[3], bb[3];
                dslash_mrhs<LH>(P.g, kEven, P.Uhi, site, IN, acc);
                ldm<double>(P.x64, Vh, P.logN, site, rhs, x);
                ldm<double>(P.b64, Vh, P.logN, site, rhs, bb);
                cx<T> lo[3];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    acc[c].re = bb[c].re - (P.m4 * x[c].re - acc[c].re);
                    acc[c].im = bb[c].im - (P.m4 * x[c].im - acc[c].im);
                    v += acc[c].re * acc[c].re + acc[c].im * acc[c].im;
                    lo[c].re = (T)acc[c].re;
                    lo[c].im = (T)acc[c].im;
                }
                if (fin == FIN_FINAL) stm<double>(P.q64, Vh, P.logN, site, rhs, acc);
                else stm<T>(P.r, Vh, P.logN, site, rhs, lo);
            }
            tile_partial(v, part + (size_t)w * kMaxRhs, P.logN);
        });
        grid_barrier(ctl, lim);
        finalize_all(A, fin, gate, act, nru);
        grid_barrier(ctl, lim);
    };

    // ---- set-up: |b|^2, then r = b - A x0 (rho, beta = 0)
    for_tiles(A, [&](const BatchProb &P, int w, unsigned site, unsigned rhs, bool ok) {
        double v = 0.0;
        if (ok) {
            cx<double> bb[3];
            ldm<double>(P.b64, (size_t)P.g.Vh, P.logN, site, rhs, bb);
#pragma unroll
            for (int c = 0; c < 3; c++) v += bb[c].re * bb[c].re + bb[c].im * bb[c].im;
        }
        tile_partial(v, part + (size_t)w * kMaxRhs, P.logN);
    });
    grid_barrier(ctl, lim);
    finalize_all(A, FIN_INIT, GATE_NONE, nullptr, nullptr);
    grid_barrier(ctl, lim);
    reliable(GATE_RU, FIN_RU, nullptr, nullptr);

    // ---- iterations, all right-hand sides of all problems in lock-step
    const int loop_cap = A->max_iter + 2;
    for (int it = 0; it < loop_cap; it++) {
        const int sl = it & 1;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl->active[sl] = 0;
            ctl->need_ru[sl] = 0;
        }
        // t = D_oe (r + beta p_old) ; p_new = r + beta p_old on the even sites
        for_tiles(A, [&](const BatchProb &P, int, unsigned site, unsigned rhs, bool ok) {
            if (!ok) return;
            const CgState *s = P.st + rhs;
            if (ld_i32(&s->state) != ST_RUN) return;
            const size_t Vh = (size_t)P.g.Vh;
            const T beta = (T)ld_f64(&s->beta);
            const void *pold = sl ? P.pb : P.pa;
            void *pnew = sl ? P.pa : P.pb;
            auto IN = [=](int n, cx<T> v[3]) __attribute__((always_inline)) {
                cx<T> rr[3], pp[3];
                ldm<T>(P.r, Vh, P.logN, n, rhs, rr);
                ldm<T>(pold, Vh, P.logN, n, rhs, pp);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    v[c].re = fma(beta, pp[c].re, rr[c].re);
                    v[c].im = fma(beta, pp[c].im, rr[c].im);
                }
            };
            cx<T> acc[3], pn[3];
            dslash_mrhs<LF>(P.g, kOdd, P.Ulo, site, IN, acc);
            stm<T>(P.t, Vh, P.logN, site, rhs, acc);
            IN(site, pn);
            stm<T>(pnew, Vh, P.logN, site, rhs, pn);
        });
        grid_barrier(ctl, lim);
        // Ap = m4 p - D_eo t ; partial <p, Ap>
        for_tiles(A, [&](const BatchProb &P, int w, unsigned site, unsigned rhs, bool ok) {
            double v = 0.0;
            const CgState *s = P.st + rhs;
            if (ok && ld_i32(&s->state) == ST_RUN) {
                const size_t Vh = (size_t)P.g.Vh;
                const void *pnew = sl ? P.pa : P.pb;
                auto IN = [=](int n, cx<T> u[3]) __attribute__((always_inline)) { ldm<T>(P.t, Vh, P.logN, n, rhs, u); };
                cx<T> acc[3], pp[3];
                dslash_mrhs<LF>(P.g, kEven, P.Ulo, site, IN, acc);
                ldm<T>(pnew, Vh, P.logN, site, rhs, pp);
                const T m4 = (T)P.m4;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    acc[c].re = m4 * pp[c].re - acc[c].re;
                    acc[c].im = m4 * pp[c].im - acc[c].im;
                    v += (double)pp[c].re * (double)acc[c].re + (double)pp[c].im * (double)acc[c].im;
                }
                stm<T>(P.Ap, Vh, P.logN, site, rhs, acc);
            }
            tile_partial(v, part + (size_t)w * kMaxRhs, P.logN);
        });
        grid_barrier(ctl, lim);
        finalize_all(A, FIN_ALPHA, GATE_ITER, nullptr, nullptr);
        grid_barrier(ctl, lim);
        // x_lo += alpha p ; r -= alpha Ap ; partial |r|^2
        for_tiles(A, [&](const BatchProb &P, int w, unsigned site, unsigned rhs, bool ok) {
            double v = 0.0;
            const CgState *s = P.st + rhs;
            if (ok && ld_i32(&s->state) == ST_RUN) {
                const size_t Vh = (size_t)P.g.Vh;
                const void *pnew = sl ? P.pa : P.pb;
                const T alpha = (T)ld_f64(&s->alpha);
                cx<T> x[3], rr[3], pp[3], q[3];
                ldm<T>(P.xlo, Vh, P.logN, site, rhs, x);
                ldm<T>(P.r, Vh, P.logN, site, rhs, rr);
                ldm<T>(pnew, Vh, P.logN, site, rhs, pp);
                ldm<T>(P.Ap, Vh, P.logN, site, rhs, q);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    x[c].re = fma(alpha, pp[c].re, x[c].re);
                    x[c].im = fma(alpha, pp[c].im, x[c].im);
                    rr[c].re = fma(-alpha, q[c].re, rr[c].re);
                    rr[c].im = fma(-alpha, q[c].im, rr[c].im);
                    v += (double)rr[c].re * (double)rr[c].re + (double)rr[c].im * (double)rr[c].im;
                }
                stm<T>(P.xlo, Vh, P.logN, site, rhs, x);
                stm<T>(P.r, Vh, P.logN, site, rhs, rr);
            }
            tile_partial(v, part + (size_t)w * kMaxRhs, P.logN);
        });
        grid_barrier(ctl, lim);
        finalize_all(A, FIN_UPDATE, GATE_ITER, &ctl->active[sl], &ctl->need_ru[sl]);
        grid_barrier(ctl, lim);
        const unsigned int nru = __hip_atomic_load(&ctl->need_ru[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool fixed = A->scheme == SCH_RELIABLE && (it + 1) % A->ru_interval == 0;
        unsigned int act = __hip_atomic_load(&ctl->active[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (fixed || nru > 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                ctl->active[sl ^ 1] = 0;
                ctl->need_ru[sl ^ 1] = 0;
            }
            grid_barrier(ctl, lim);
            reliable(GATE_RU, FIN_RU, &ctl->active[sl ^ 1], &ctl->need_ru[sl ^ 1]);
            act = __hip_atomic_load(&ctl->active[sl ^ 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) ctl->iters_done = it + 1;
        if (act == 0 || __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        grid_barrier(ctl, lim);
    }
    grid_barrier(ctl, lim);
    // ---- final: accumulate, FP64 true residual of every right-hand side
    reliable(GATE_NONE, FIN_FINAL, nullptr, nullptr);
}

template <class LF> static int max_blocks_per_cu()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_cg<LF>, kBS, 0) != hipSuccess) return 0;
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

hipError_t launch_batch_cg_init(const BatchArgs *a_dev, int total_rhs, double tol, double inner, hipStream_t s)
{
    hipLaunchKernelGGL(k_state_init_batch, dim3((total_rhs + 63) / 64), dim3(64), 0, s, a_dev, tol, inner);
    return hipGetLastError();
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
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBS), args, 0, s);
}

} // namespace lgt
