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
// staple is linear in M, so F nests:
//   F = c1 U + sum_a S_a[ c3 U + cL S_a[U] + sum_b S_b[ W_rho ] ],
//   W_rho = c5 U + c7 (S_{+rho}[U] + S_{-rho}[U]),
// where rho is the one axis other than mu, a and b: the innermost sum depends
// on the axis pair only, so per direction mu a first kernel stores the three
// fields W_rho (4 products per site each) and a second evaluates the outer
// levels per link from them (72 products, plus 2 for N) instead of
// recomputing W at every (a, b) of every link (168 products). Link and W
// reads come from the caches; the kernels are bound by the latency of those
// gathers (one wave per SIMD) and FP64 arithmetic, not by HBM. Workgroups are
// dispatched round-robin over the 8 XCDs, so both kernels remap the block
// index: each XCD walks one contiguous range of checkerboard indices, the two
// parities of a block of sites back to back (and in the first kernel its
// three fields W_r), which keeps the y and z neighbours in that XCD's L2.
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

// eo index of thread t of the k-th block taken by XCD xcd: checkerboard block
// xcd * nbh_pad / 8 + k / 2 of parity k % 2, or -1 past the Vh sites of a
// parity (nbh_pad: blocks per parity, rounded up to a multiple of 8)
__device__ __forceinline__ int64_t xcd_site(const Geom &g, int xcd, int k, int nbh_pad, int t)
{
    const int64_t cb = (int64_t)(xcd * (nbh_pad >> 3) + (k >> 1)) * kBS + t;
    return cb < g.Vh ? (k & 1) * (int64_t)g.Vh + cb : -1;
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

// W_r(y) = c5 U_mu(y) + c7 (S_{+rho}[U_mu](y) + S_{-rho}[U_mu](y)), rho = the r-th
// axis other than mu; W is [3][V][3][3][2]; 6 * nbh_pad blocks
__global__ __launch_bounds__(kBS) void k_fat_inner(const double *__restrict__ U, double *__restrict__ W, Geom g,
                                                   int mu, double c5, double c7, int nbh_pad)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int k = (int)(blockIdx.x >> 3);
    const int r = k % 3; // the three fields of one block of sites on one XCD in a row
    const int64_t ey = xcd_site(g, (int)(blockIdx.x & 7), k / 3, nbh_pad, (int)threadIdx.x);
    if (ey < 0) return;
    const int rho = other_axis(mu, r);
    int y[4], yp[4], ym[4];
    site_coords(g, ey, y);
    step(g, y, rho, 1, yp);
    step(g, y, rho, -1, ym);
    M3 w = scaled(c5, ldm3(U, V, mu, ey));
    axpy(w, c7, staple(U, V, g, y, mu, rho, 1, ldm3(U, V, mu, eo_of(g, yp))));
    axpy(w, c7, staple(U, V, g, y, mu, rho, -1, ldm3(U, V, mu, eo_of(g, ym))));
    stm3(W, V, r, ey, w);
}

// F_mu(x) and N_mu(x) for every site x of direction mu, the innermost level from
// W; 2 * nbh_pad blocks
__global__ __launch_bounds__(kBS) void k_fat_outer(const double *__restrict__ U, const double *__restrict__ W,
                                                   double *__restrict__ F, double *__restrict__ N, Geom g, int mu,
                                                   FatCoeffs w, int nbh_pad)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t ex = xcd_site(g, (int)(blockIdx.x & 7), (int)(blockIdx.x >> 3), nbh_pad, (int)threadIdx.x);
    if (ex < 0) return;
    int x[4];
    site_coords(g, ex, x);

    M3 acc = scaled(w.c1, ldm3(U, V, mu, ex));
#pragma unroll 1
    for (int ia = 0; ia < 6; ia++) {
        const int ka = ia >> 1, a = other_axis(mu, ka), sa = (ia & 1) ? -1 : 1;
        int xa[4], xaa[4];
        step(g, x, a, sa, xa);
        step(g, xa, a, sa, xaa);
        // the field under the outer staple, at x + a: c3 U + cL S_a[U] + sum_b S_b[W]
        M3 in1 = scaled(w.c3, ldm3(U, V, mu, eo_of(g, xa)));
        axpy(in1, w.cL, staple(U, V, g, xa, mu, a, sa, ldm3(U, V, mu, eo_of(g, xaa))));
#pragma unroll 1
        for (int ib = 0; ib < 6; ib++) {
            const int kb = ib >> 1;
            if (kb == ka) continue;
            const int b = other_axis(mu, kb), sb = (ib & 1) ? -1 : 1;
            int xab[4];
            step(g, xa, b, sb, xab);
            // rho: the third axis other than mu (index 3 - ka - kb among mu's others)
            axpy(in1, 1.0, staple(U, V, g, xa, mu, b, sb, ldm3(W, V, 3 - ka - kb, eo_of(g, xab))));
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

hipError_t launch_fatten(const double *U, double *F, double *N, double *W, const Geom &g, const FatCoeffs &w,
                         hipStream_t s)
{
    const int nbh = (int)(((int64_t)g.Vh + kBS - 1) / kBS), nbh_pad = (nbh + 7) / 8 * 8;
    for (int mu = 0; mu < 4; mu++) {
        hipLaunchKernelGGL(k_fat_inner, dim3(6u * (unsigned)nbh_pad), dim3(kBS), 0, s, U, W, g, mu, w.c5, w.c7,
                           nbh_pad);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_fat_outer, dim3(2u * (unsigned)nbh_pad), dim3(kBS), 0, s, U, W, F, N, g, mu, w,
                           nbh_pad);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

} // namespace lgt
