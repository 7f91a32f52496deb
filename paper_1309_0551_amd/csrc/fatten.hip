// fatten.hip -- the link fields of the improved staggered operator from the
// gauge field: the fat one-link field F (the link plus its 3-, 5- and 7-link
// staples and the 5-link Lepage path) and the Naik three-link field N, built
// from the Table 1 matrix products (mult_su3_nn / _na / _an).
//
// With the staple of a field M along a signed direction a,
//   S_a[M](x) = L_a(x) M(x+a) L_a(x+mu)^dag,  L_{+nu}(y) = U_nu(y),
//                                               L_{-nu}(y) = U_nu(y-nu)^dag,
//   F_mu = c1 U_mu + c3 sum_a S_a[U_mu] + c5 sum_{a,b} S_a[S_b[U_mu]]
//        + c7 sum_{a,b,c} S_a[S_b[S_c[U_mu]]] + cL sum_a S_a[S_a[U_mu]]
//   N_mu(x) = cN U_mu(x) U_mu(x+mu) U_mu(x+2mu)
// (a, b, c signed directions orthogonal to mu on pairwise different axes). The
// staple is linear in M, so one thread per link evaluates F nested:
//   F = c1 U + sum_a S_a[ c3 U + cL S_a[U] + sum_b S_b[ c5 U + c7 sum_c S_c[U] ] ]
// 168 products of 3x3 complex matrices per link; all link reads come from the
// caches (each link is read by many threads), so the kernel is bound by FP64
// arithmetic, not by HBM.
#include "fields.hpp"
#include "kernels.hpp"
#include "su3.hpp"

namespace lgt {

namespace {

// y = x + d * axis, periodic (selects only, no dynamic indexing of private arrays)
__device__ __forceinline__ void step(const Geom &g, const int x[4], int axis, int d, int y[4])
{
#pragma unroll
    for (int k = 0; k < 4; k++) {
        int v = x[k] + (axis == k ? d : 0);
        v = v < 0 ? v + g.L[k] : (v >= g.L[k] ? v - g.L[k] : v);
        y[k] = v;
    }
}

// the k-th axis other than mu (k = 0, 1, 2)
__device__ __forceinline__ int other_axis(int mu, int k) { return k + (k >= mu ? 1 : 0); }

__device__ __forceinline__ M3 adj(const M3 &A)
{
    M3 B;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) B.e[3 * i + j] = cx<double>{A.e[3 * j + i].re, -A.e[3 * j + i].im};
    return B;
}

// L_a(y): the link of one step from y along axis a in direction s
__device__ __forceinline__ M3 step_link(const double *U, int64_t V, const Geom &g, const int y[4], int a, int s)
{
    if (s > 0) return ldm3(U, V, a, eo_of(g, y));
    int ym[4];
    step(g, y, a, -1, ym);
    return adj(ldm3(U, V, a, eo_of(g, ym)));
}

__device__ __forceinline__ void axpy(M3 &A, double f, const M3 &B)
{
#pragma unroll
    for (int k = 0; k < 9; k++) {
        A.e[k].re = fma(f, B.e[k].re, A.e[k].re);
        A.e[k].im = fma(f, B.e[k].im, A.e[k].im);
    }
}

__device__ __forceinline__ M3 scaled(double f, const M3 &B)
{
    M3 A;
#pragma unroll
    for (int k = 0; k < 9; k++) A.e[k] = cx<double>{f * B.e[k].re, f * B.e[k].im};
    return A;
}

// S_a[M](y) with M(y+a) given: L_a(y) M L_a(y+mu)^dag
__device__ __forceinline__ M3 staple(const double *U, int64_t V, const Geom &g, const int y[4], int mu, int a, int s,
                                     const M3 &M)
{
    int ymu[4];
    step(g, y, mu, 1, ymu);
    return mul<false, true>(mul<false, false>(step_link(U, V, g, y, a, s), M), step_link(U, V, g, ymu, a, s));
}

__global__ __launch_bounds__(kBS) void k_fatten(const double *__restrict__ U, double *__restrict__ F,
                                                double *__restrict__ N, Geom g, FatCoeffs w)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t l = (int64_t)blockIdx.x * kBS + threadIdx.x; // mu * V + x
    if (l >= 4 * V) return;
    const int mu = (int)(l / V);
    const int64_t ex = l - mu * V;
    int x[4];
    site_coords(g, ex, x);

    M3 acc = scaled(w.c1, ldm3(U, V, mu, ex));
#pragma unroll 1
    for (int ia = 0; ia < 6; ia++) {
        const int a = other_axis(mu, ia >> 1), sa = (ia & 1) ? -1 : 1;
        int xa[4], xaa[4];
        step(g, x, a, sa, xa);
        step(g, xa, a, sa, xaa);
        // inner1 at x + a: c3 U + cL S_a[U] + sum_b S_b[inner2]
        M3 in1 = scaled(w.c3, ldm3(U, V, mu, eo_of(g, xa)));
        axpy(in1, w.cL, staple(U, V, g, xa, mu, a, sa, ldm3(U, V, mu, eo_of(g, xaa))));
#pragma unroll 1
        for (int ib = 0; ib < 6; ib++) {
            const int b = other_axis(mu, ib >> 1), sb = (ib & 1) ? -1 : 1;
            if (b == a) continue;
            int xab[4];
            step(g, xa, b, sb, xab);
            // inner2 at x + a + b: c5 U + c7 sum_c S_c[U]
            M3 in2 = scaled(w.c5, ldm3(U, V, mu, eo_of(g, xab)));
#pragma unroll 1
            for (int ic = 0; ic < 6; ic++) {
                const int c = other_axis(mu, ic >> 1), sc = (ic & 1) ? -1 : 1;
                if (c == a || c == b) continue;
                int xabc[4];
                step(g, xab, c, sc, xabc);
                axpy(in2, w.c7, staple(U, V, g, xab, mu, c, sc, ldm3(U, V, mu, eo_of(g, xabc))));
            }
            axpy(in1, 1.0, staple(U, V, g, xa, mu, b, sb, in2));
        }
        axpy(acc, 1.0, staple(U, V, g, x, mu, a, sa, in1));
    }
    stm3(F, V, mu, ex, acc);

    int x1[4], x2[4];
    step(g, x, mu, 1, x1);
    step(g, x1, mu, 1, x2);
    const M3 n = mul<false, false>(mul<false, false>(ldm3(U, V, mu, ex), ldm3(U, V, mu, eo_of(g, x1))),
                                   ldm3(U, V, mu, eo_of(g, x2)));
    stm3(N, V, mu, ex, scaled(w.cN, n));
}

} // namespace

hipError_t launch_fatten(const double *U, double *F, double *N, const Geom &g, const FatCoeffs &w, hipStream_t s)
{
    const int64_t n = 8 * (int64_t)g.Vh;
    hipLaunchKernelGGL(k_fatten, dim3((unsigned)((n + kBS - 1) / kBS)), dim3(kBS), 0, s, U, F, N, g, w);
    return hipGetLastError();
}

} // namespace lgt
