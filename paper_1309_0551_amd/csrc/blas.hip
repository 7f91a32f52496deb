// blas.hip -- the CG vector updates (Table 1: scalar_mult_add_su3_vector,
// add_su3_vector) with fused FP64 partial sums, the one-workgroup finalize
// kernel that turns partial sums into the solver's scalars, and the solver's
// small kernels. The vector kernels are one thread per site (three complex
// numbers) and HBM-bound.
#include "fields.hpp"
#include "kernels.hpp"
#include "reduce.hpp"

#include <hip/hip_ext.h>

namespace lgt {

// Launch with optional start / stop events carried on the kernel's own
// dispatch packet (they time the kernel alone, as a kernel trace does).
template <class K, class... Args>
static void launch_ev(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args)
{
    if (e0 || e1) hipExtLaunchKernelGGL(kernel, grid, block, 0u, s, e0, e1, 0u, args...);
    else hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// x += alpha p (the previous update's, while pending) ; p = r + beta p.
// Adding alpha p here rather than in the update saves one vector pass per
// iteration: this kernel reads p anyway, and the update then touches only r.
template <typename T>
__global__ __launch_bounds__(kBS) void k_xpay(VecArgs a)
{
    if (!gate_open(a.gate, a.st)) return;
    const int cb = blockIdx.x * kBS + threadIdx.x;
    if (cb >= a.Vh) return;
    const T beta = (T)a.st->beta;
    const bool pend = a.st->pend != 0;
    cx<T> r[3], p[3];
    VecFmt<T>::template load<false>(a.r, (size_t)a.Vh, cb, r);
    VecFmt<T>::template load<false>(a.p, (size_t)a.Vh, cb, p);
    if (pend) {
        const T alpha = (T)a.st->alpha;
        cx<T> x[3];
        VecFmt<T>::template load<false>(a.x, (size_t)a.Vh, cb, x);
#pragma unroll
        for (int i = 0; i < 3; i++) {
            x[i].re = fma(alpha, p[i].re, x[i].re);
            x[i].im = fma(alpha, p[i].im, x[i].im);
        }
        VecFmt<T>::template store<false>(a.x, (size_t)a.Vh, cb, x);
    }
#pragma unroll
    for (int i = 0; i < 3; i++) {
        p[i].re = fma(beta, p[i].re, r[i].re);
        p[i].im = fma(beta, p[i].im, r[i].im);
    }
    VecFmt<T>::template store<false>(a.p, (size_t)a.Vh, cb, p);
}

// FP32: two neighbouring sites per thread, so each colour plane moves in
// 16-byte accesses (V/2 is a multiple of 8; the solver's vectors are workspace
// allocations, 256-byte aligned); the same operations per element as k_xpay,
// so the same results (32^4: 11.5 -> 10.3 us a pass, the FP32 x 12 and
// BF16 x 12 solves 1.7 and 2.6 % faster)
__global__ __launch_bounds__(kBS) void k_xpay2(VecArgs a)
{
    if (!gate_open(a.gate, a.st)) return;
    const int cb2 = blockIdx.x * kBS + threadIdx.x; // sites 2 cb2, 2 cb2 + 1
    if (2 * cb2 >= a.Vh) return;
    const float beta = (float)a.st->beta;
    const bool pend = a.st->pend != 0;
    const size_t P = (size_t)a.Vh / 2; // fv4 per plane
    const fv4 *rv = (const fv4 *)a.r;
    fv4 *pv = (fv4 *)a.p;
    fv4 r[3], p[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        r[i] = rv[i * P + cb2];
        p[i] = pv[i * P + cb2];
    }
    if (pend) {
        const float alpha = (float)a.st->alpha;
        fv4 *xv = (fv4 *)a.x;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            fv4 x = xv[i * P + cb2];
            x.x = fmaf(alpha, p[i].x, x.x);
            x.y = fmaf(alpha, p[i].y, x.y);
            x.z = fmaf(alpha, p[i].z, x.z);
            x.w = fmaf(alpha, p[i].w, x.w);
            xv[i * P + cb2] = x;
        }
    }
#pragma unroll
    for (int i = 0; i < 3; i++) {
        fv4 q;
        q.x = fmaf(beta, p[i].x, r[i].x);
        q.y = fmaf(beta, p[i].y, r[i].y);
        q.z = fmaf(beta, p[i].z, r[i].z);
        q.w = fmaf(beta, p[i].w, r[i].w);
        pv[i * P + cb2] = q;
    }
}

hipError_t launch_xpay(bool f64, const VecArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (f64) launch_ev(k_xpay<double>, dim3(a.l.nblk), dim3(kBS), s, e0, e1, a);
    else launch_ev(k_xpay2, dim3((unsigned)((a.Vh / 2 + kBS - 1) / kBS)), dim3(kBS), s, e0, e1, a);
    return hipGetLastError();
}

// x += alpha p if an update is pending (before a reliable update or the final
// residual, which use x); the finalize step that follows clears the flag
template <typename T>
__global__ __launch_bounds__(kBS) void k_x_pending(VecArgs a)
{
    if (!gate_open(a.gate, a.st)) return;
    if (a.st->pend == 0) return;
    const int cb = blockIdx.x * kBS + threadIdx.x;
    if (cb >= a.Vh) return;
    const T alpha = (T)a.st->alpha;
    const void *pc = a.p2 && a.st->pcur ? a.p2 : a.p; // the p alpha belongs to
    cx<T> x[3], p[3];
    VecFmt<T>::template load<false>(a.x, (size_t)a.Vh, cb, x);
    VecFmt<T>::template load<false>(pc, (size_t)a.Vh, cb, p);
#pragma unroll
    for (int i = 0; i < 3; i++) {
        x[i].re = fma(alpha, p[i].re, x[i].re);
        x[i].im = fma(alpha, p[i].im, x[i].im);
    }
    VecFmt<T>::template store<false>(a.x, (size_t)a.Vh, cb, x);
}

hipError_t launch_x_pending(bool f64, const VecArgs &a, hipStream_t s)
{
    if (f64) hipLaunchKernelGGL(k_x_pending<double>, dim3(a.l.nblk), dim3(kBS), 0, s, a);
    else hipLaunchKernelGGL(k_x_pending<float>, dim3(a.l.nblk), dim3(kBS), 0, s, a);
    return hipGetLastError();
}

// Sum n partials in a fixed order (four strided accumulators per thread, so
// four loads are in flight, then a fixed tree inside one workgroup: the
// result is bit-reproducible) and run the scalar step `fin`. Gated exactly
// like the kernel that wrote the partials. (One accumulator left each
// thread's loads one after another: the 32^4 solves took 0.4-3.9 % longer.)
__global__ __launch_bounds__(kBS) void k_finalize(const double *__restrict__ partials, int n, CgState *st, int fin,
                                                  int gate)
{
    if (!gate_open(gate, st)) return;
    __shared__ double lds[kBS / 64];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * kBS < n; i += 4 * kBS) {
        s0 += partials[i];
        s1 += partials[i + kBS];
        s2 += partials[i + 2 * kBS];
        s3 += partials[i + 3 * kBS];
    }
    for (; i < n; i += kBS) s0 += partials[i];
    const double tot = block_sum((s0 + s1) + (s2 + s3), lds);
    if (threadIdx.x == 0) finalize(fin, st, tot);
}

hipError_t launch_finalize(const double *partials, int n, CgState *st, int fin, int gate, hipStream_t s,
                           hipEvent_t e0, hipEvent_t e1)
{
    launch_ev(k_finalize, dim3(1), dim3(kBS), s, e0, e1, partials, n, st, fin, gate);
    return hipGetLastError();
}

// x64 += x_lo ; x_lo = 0   (solution accumulation in FP64)
__global__ __launch_bounds__(kBS) void k_ru_accum(double *__restrict__ x64, void *__restrict__ xlo, int Vh,
                                                  CgState *st, int gate)
{
    if (!gate_open(gate, st)) return;
    const int cb = blockIdx.x * kBS + threadIdx.x;
    if (cb >= Vh) return;
    cx<double> x[3];
    cx<float> e[3];
    VecFmt<double>::load<false>(x64, (size_t)Vh, cb, x);
    VecFmt<float>::load<false>(xlo, (size_t)Vh, cb, e);
#pragma unroll
    for (int i = 0; i < 3; i++) {
        x[i].re += (double)e[i].re;
        x[i].im += (double)e[i].im;
        e[i].re = 0.0f;
        e[i].im = 0.0f;
    }
    VecFmt<double>::store<false>(x64, (size_t)Vh, cb, x);
    VecFmt<float>::store<false>(xlo, (size_t)Vh, cb, e);
}

hipError_t launch_ru_accum(double *x64, void *xlo, int Vh, CgState *st, int gate, hipStream_t s)
{
    hipLaunchKernelGGL(k_ru_accum, dim3((Vh + kBS - 1) / kBS), dim3(kBS), 0, s, x64, xlo, Vh, st, gate);
    return hipGetLastError();
}

// zero fill with a kernel (safe inside captured graphs, unlike memset nodes)
__global__ __launch_bounds__(kBS) void k_zero(uv4 *__restrict__ p, size_t n16)
{
    const size_t i = (size_t)blockIdx.x * kBS + threadIdx.x;
    if (i < n16) p[i] = uv4{0u, 0u, 0u, 0u};
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16; // every buffer here is a multiple of 16 bytes
    if (n16 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n16 + kBS - 1) / kBS)), dim3(kBS), 0, s, (uv4 *)p, n16);
    return hipGetLastError();
}

// Pseudo-random reals in [-1, 1) from a 32-bit integer hash of the index
// (two xorshift-multiply rounds), for buffers that only carry timing traffic:
// kernels timed on all-zero data ran up to a fifth faster than on data like a
// solver's (the multi-RHS Dslash at 24^3 x 48, 16 right-hand sides: 74
// against 84-88 us).
template <typename T> __global__ __launch_bounds__(kBS) void k_fill_noise(T *__restrict__ p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBS + threadIdx.x;
    if (i >= n) return;
    unsigned h = (unsigned)i ^ (unsigned)(i >> 32) * 0x9E3779B9u;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    p[i] = (T)((double)(h >> 8) * (1.0 / 8388608.0) - 1.0);
}

hipError_t launch_fill_noise(void *p, size_t n, bool f64, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kBS - 1) / kBS)), block(kBS);
    if (f64) hipLaunchKernelGGL(k_fill_noise<double>, grid, block, 0, s, (double *)p, n);
    else hipLaunchKernelGGL(k_fill_noise<float>, grid, block, 0, s, (float *)p, n);
    return hipGetLastError();
}

__global__ void k_state_init(CgState *st, int scheme, int ru_fixed, int max_iter, double tol, double inner)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->rho = st->rho_prev = st->alpha = st->beta = st->pAp = 0.0;
    st->bnorm2 = 0.0;
    st->stop_outer = tol * tol; // multiplied by |b|^2 in FIN_INIT
    st->stop_inner = 0.0;
    st->inner2 = scheme == SCH_REFINE ? inner * inner : (inner * tol) * (inner * tol);
    st->last_true = 0.0;
    st->iter = 0;
    st->updates = 0;
    st->state = ST_INIT;
    st->max_iter = max_iter;
    st->scheme = scheme;
    st->ru_fixed = ru_fixed;
    st->pend = st->pcur = 0;
}

hipError_t launch_state_init(CgState *st, int scheme, int ru_fixed, int max_iter, double tol, double inner,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, scheme, ru_fixed, max_iter, tol, inner);
    return hipGetLastError();
}

// |b|^2 partials (the FIN_INIT step sets the stop thresholds)
__global__ __launch_bounds__(kBS) void k_norm_parts(const double *__restrict__ b, int Vh, double *partials)
{
    const int cb = blockIdx.x * kBS + threadIdx.x;
    double part = 0.0;
    if (cb < Vh) {
        cx<double> v[3];
        VecFmt<double>::load<false>(b, (size_t)Vh, cb, v);
#pragma unroll
        for (int i = 0; i < 3; i++) part += v[i].re * v[i].re + v[i].im * v[i].im;
    }
    write_partial(part, partials, blockIdx.x);
}

hipError_t launch_norm_init(const double *b64, int Vh, double *partials, CgState *st, hipStream_t s)
{
    const int nblk = (Vh + kBS - 1) / kBS;
    hipLaunchKernelGGL(k_norm_parts, dim3(nblk), dim3(kBS), 0, s, b64, Vh, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(partials, nblk, st, FIN_INIT, GATE_NONE, s);
}

// generic complex dot product sum conj(a) b, FP64, fixed order: partials per
// workgroup, then one workgroup sums them
__global__ __launch_bounds__(kBS) void k_cdot_parts(int64_t n, const dv2 *__restrict__ a, const dv2 *__restrict__ b,
                                                    double *partials, int nblk)
{
    __shared__ double lds[kBS / 64];
    double re = 0.0, im = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)nblk * kBS) {
        const dv2 x = a[i], y = b[i];
        re += x.x * y.x + x.y * y.y;
        im += x.x * y.y - x.y * y.x;
    }
    const double sr = block_sum(re, lds);
    const double si = block_sum(im, lds);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = sr;
        partials[2 * blockIdx.x + 1] = si;
    }
}

__global__ __launch_bounds__(kBS) void k_cdot_final(const double *__restrict__ partials, int nblk, double *result)
{
    __shared__ double lds[kBS / 64];
    double ar = 0.0, ai = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kBS) {
        ar += partials[2 * i];
        ai += partials[2 * i + 1];
    }
    const double tr = block_sum(ar, lds);
    const double ti = block_sum(ai, lds);
    if (threadIdx.x == 0) {
        result[0] = tr;
        result[1] = ti;
    }
}

hipError_t launch_cdot(int64_t n, const double *a, const double *b, double *partials, double *result, hipStream_t s)
{
    int nblk = (int)((n + kBS - 1) / kBS);
    if (nblk > 1024) nblk = 1024;
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(k_cdot_parts, dim3(nblk), dim3(kBS), 0, s, n, (const dv2 *)a, (const dv2 *)b, partials, nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cdot_final, dim3(1), dim3(kBS), 0, s, partials, nblk, result);
    return hipGetLastError();
}

} // namespace lgt
