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

// The field under the outer staple along the signed direction ia (axis index
// ia / 2 among mu's others, sign - for odd ia), at y:
//   I_a(y) = c3 U_mu(y) + cL S_a[U_mu](y) + sum_b S_b[W_rho](y),
// b over the four signed directions on the other two axes, rho the third axis
// other than mu, a and b (index 3 - ka - kb among mu's others).
__device__ __forceinline__ M3 mid_field(const double *U, const double *W, const Geom &g, const int y[4], int mu,
                                        int ia, const FatCoeffs &w)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int ka = ia >> 1, a = other_axis(mu, ka), sa = (ia & 1) ? -1 : 1;
    int ya[4];
    step(g, y, a, sa, ya);
    M3 in1 = scaled(w.c3, ldm3(U, V, mu, eo_of(g, y)));
    axpy(in1, w.cL, staple(U, V, g, y, mu, a, sa, ldm3(U, V, mu, eo_of(g, ya))));
#pragma unroll 1
    for (int ib = 0; ib < 6; ib++) {
        const int kb = ib >> 1;
        if (kb == ka) continue;
        const int b = other_axis(mu, kb), sb = (ib & 1) ? -1 : 1;
        int yb[4];
        step(g, y, b, sb, yb);
        axpy(in1, 1.0, staple(U, V, g, y, mu, b, sb, ldm3(W, V, 3 - ka - kb, eo_of(g, yb))));
    }
    return in1;
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
// W; with I set, also the six fields I_a(x + a) under the outer staples
// (slot a; each (a, y) is reached from exactly one x), which the chain rule
// needs again; 2 * nbh_pad blocks
__global__ __launch_bounds__(kBS) void k_fat_outer(const double *__restrict__ U, const double *__restrict__ W,
                                                   double *__restrict__ F, double *__restrict__ N, Geom g, int mu,
                                                   FatCoeffs w, int nbh_pad, double *__restrict__ I)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t ex = xcd_site(g, (int)(blockIdx.x & 7), (int)(blockIdx.x >> 3), nbh_pad, (int)threadIdx.x);
    if (ex < 0) return;
    int x[4];
    site_coords(g, ex, x);

    M3 acc = scaled(w.c1, ldm3(U, V, mu, ex));
#pragma unroll 1
    for (int ia = 0; ia < 6; ia++) {
        const int a = other_axis(mu, ia >> 1), sa = (ia & 1) ? -1 : 1;
        int xa[4];
        step(g, x, a, sa, xa);
        const M3 m = mid_field(U, W, g, xa, mu, ia, w);
        if (I) stm3(I, V, ia, eo_of(g, xa), m);
        axpy(acc, 1.0, staple(U, V, g, x, mu, a, sa, m));
    }
    stm3(F, V, mu, ex, acc);

    int x1[4], x2[4];
    step(g, x, mu, 1, x1);
    step(g, x1, mu, 1, x2);
    const M3 n = mul<false, false>(mul<false, false>(ldm3(U, V, mu, ex), ldm3(U, V, mu, eo_of(g, x1))),
                                   ldm3(U, V, mu, eo_of(g, x2)));
    stm3(N, V, mu, ex, scaled(w.cN, n));
}

// ---- the chain rule through the fattening -----------------------------------
// dS = sum Re tr(G_F^dag dF) + Re tr(G_N^dag dN) is taken back to
// dS = sum Re tr(G_U^dag dU) over the nested form above. A staple
// P(x) = L(x) M(x+a) L(x+mu)^dag whose output receives Gp(x) passes
//   L(x)^dag Gp(x) L(x+mu)      to M(x+a),
//   Gp(x) L(x+mu) M(x+a)^dag    to its first leg L(x),
//   Gp(x)^dag L(x) M(x+a)       to its return leg L(x+mu),
// and L_{-nu}(y) = U_nu(y-nu)^dag passes the adjoint of what it receives to
// U_nu(y-nu). Per direction mu, with I_a the field under the outer staple
// (mid_field) and W_r as in the forward, every kernel gathers what reaches its
// output site (no atomics; a fixed order of summation):
//   Q_a(y) = L_a(y-a)^dag G(y-a) L_a(y-a+mu)                        (of I_a)
//   R_r(z) = sum_b L_b(z-b)^dag (Q_{+k} + Q_{-k})(z-b) L_b(z-b+mu)    (of W_r)
//            b over the two axes other than r, k the third axis
//   G_U,mu(x) += c1 G + c3 sum_a Q_a + c5 sum_r R_r
//              + sum_a L_a(x-a)^dag (cL Q_a + c7 R_{axis of a})(x-a) L_a(x-a+mu)
//              + the three places of U_mu(x) in the Naik products
//   G_U,nu(z) += the legs through U_nu(z) of every staple along +-nu (nu != mu).
// A leg along a (axis index r) collects four staples: the outer one (Gp = G,
// M = I_a), the Lepage and innermost ones together (Gp = cL Q_a + c7 R_r,
// M = U_mu) and the two middle ones (Gp = Q_{+k} + Q_{-k}, M = W_rho, k each
// of the two other axes, rho the remaining one). G is scale * G_F,mu.
// Fields I and Q hold six matrices per site (slot = signed direction ia), R
// three (slot = axis index r); block mapping as in the forward.

// I_a(y) for the six signed directions; 12 * nbh_pad blocks
__global__ __launch_bounds__(kBS) void k_vjp_mid(const double *__restrict__ U, const double *__restrict__ W,
                                                 double *__restrict__ I, Geom g, int mu, FatCoeffs w, int nbh_pad)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int k = (int)(blockIdx.x >> 3);
    const int ia = k % 6;
    const int64_t ey = xcd_site(g, (int)(blockIdx.x & 7), k / 6, nbh_pad, (int)threadIdx.x);
    if (ey < 0) return;
    int y[4];
    site_coords(g, ey, y);
    stm3(I, V, ia, ey, mid_field(U, W, g, y, mu, ia, w));
}

// Q_a(y) = L_a(x)^dag G(x) L_a(x+mu), x = y - a; 12 * nbh_pad blocks
__global__ __launch_bounds__(kBS) void k_vjp_q(const double *__restrict__ U, const double *__restrict__ GF,
                                               double *__restrict__ Q, Geom g, int mu, double scale, int nbh_pad)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int k = (int)(blockIdx.x >> 3);
    const int ia = k % 6;
    const int64_t ey = xcd_site(g, (int)(blockIdx.x & 7), k / 6, nbh_pad, (int)threadIdx.x);
    if (ey < 0) return;
    const int a = other_axis(mu, ia >> 1), sa = (ia & 1) ? -1 : 1;
    int y[4], x[4], xm[4];
    site_coords(g, ey, y);
    step(g, y, a, -sa, x);
    step(g, x, mu, 1, xm);
    const M3 Gx = scaled(scale, ldm3(GF, V, mu, eo_of(g, x)));
    stm3(Q, V, ia, ey, mul<true, false>(step_link(U, V, g, x, a, sa), mul<false, false>(Gx, step_link(U, V, g, xm, a, sa))));
}

// (Q_{+k} + Q_{-k})(x) for the axis index k
__device__ __forceinline__ M3 q_pair(const double *Q, int64_t V, int k, int64_t ex)
{
    M3 h = ldm3(Q, V, 2 * k, ex);
    acc(h, ldm3(Q, V, 2 * k + 1, ex));
    return h;
}

// R_r(z); 6 * nbh_pad blocks
__global__ __launch_bounds__(kBS) void k_vjp_r(const double *__restrict__ U, const double *__restrict__ Q,
                                               double *__restrict__ R, Geom g, int mu, int nbh_pad)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int k = (int)(blockIdx.x >> 3);
    const int r = k % 3;
    const int64_t ez = xcd_site(g, (int)(blockIdx.x & 7), k / 3, nbh_pad, (int)threadIdx.x);
    if (ez < 0) return;
    int z[4];
    site_coords(g, ez, z);
    M3 out{};
#pragma unroll 1
    for (int ib = 0; ib < 6; ib++) {
        const int kb = ib >> 1;
        if (kb == r) continue;
        const int b = other_axis(mu, kb), sb = (ib & 1) ? -1 : 1;
        int x[4], xm[4];
        step(g, z, b, -sb, x);
        step(g, x, mu, 1, xm);
        const M3 h = q_pair(Q, V, 3 - r - kb, eo_of(g, x));
        acc(out, mul<true, false>(step_link(U, V, g, x, b, sb), mul<false, false>(h, step_link(U, V, g, xm, b, sb))));
    }
    stm3(R, V, r, ez, out);
}

// G_U,mu(x) += its share from direction mu's own fields; 2 * nbh_pad blocks
__global__ __launch_bounds__(kBS) void k_vjp_mu(const double *__restrict__ U, const double *__restrict__ GF,
                                                const double *__restrict__ GN, const double *__restrict__ Q,
                                                const double *__restrict__ R, double *__restrict__ GU, Geom g, int mu,
                                                FatCoeffs w, double scale, int nbh_pad)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t ex = xcd_site(g, (int)(blockIdx.x & 7), (int)(blockIdx.x >> 3), nbh_pad, (int)threadIdx.x);
    if (ex < 0) return;
    int x[4];
    site_coords(g, ex, x);
    M3 out = ldm3(GU, V, mu, ex);
    axpy(out, scale * w.c1, ldm3(GF, V, mu, ex));
#pragma unroll 1
    for (int ia = 0; ia < 6; ia++) axpy(out, w.c3, ldm3(Q, V, ia, ex));
#pragma unroll 1
    for (int r = 0; r < 3; r++) axpy(out, w.c5, ldm3(R, V, r, ex));
#pragma unroll 1
    for (int ia = 0; ia < 6; ia++) {
        const int a = other_axis(mu, ia >> 1), sa = (ia & 1) ? -1 : 1;
        int y[4], ym[4];
        step(g, x, a, -sa, y);
        step(g, y, mu, 1, ym);
        const int64_t ey = eo_of(g, y);
        M3 t = scaled(w.cL, ldm3(Q, V, ia, ey));
        axpy(t, w.c7, ldm3(R, V, ia >> 1, ey));
        acc(out, mul<true, false>(step_link(U, V, g, y, a, sa), mul<false, false>(t, step_link(U, V, g, ym, a, sa))));
    }
    // Naik: N(y) = cN U(y) U(y+mu) U(y+2mu) holds U_mu(x) at y = x, x - mu, x - 2mu
    int x1[4], x2[4], xm1[4], xm2[4];
    step(g, x, mu, 1, x1);
    step(g, x1, mu, 1, x2);
    step(g, x, mu, -1, xm1);
    step(g, xm1, mu, -1, xm2);
    const double h = scale * w.cN;
    const int64_t e1 = eo_of(g, x1), em1 = eo_of(g, xm1), em2 = eo_of(g, xm2);
    const M3 u1 = ldm3(U, V, mu, e1), um1 = ldm3(U, V, mu, em1);
    acc(out, mul<false, true>(scaled(h, ldm3(GN, V, mu, ex)), mul<false, false>(u1, ldm3(U, V, mu, eo_of(g, x2)))));
    acc(out, mul<true, false>(um1, mul<false, true>(scaled(h, ldm3(GN, V, mu, em1)), u1)));
    acc(out, mul<true, false>(mul<false, false>(ldm3(U, V, mu, em2), um1), scaled(h, ldm3(GN, V, mu, em2))));
    stm3(GU, V, mu, ex, out);
}

// What the legs along the signed direction (axis index r, sign s) of the
// staples of direction mu that start at x receive: FIRST, the first leg L(x),
// sum_t Gp_t(x) L(x+mu) M_t(x+a)^dag; else the return leg L(x+mu),
// sum_t Gp_t(x)^dag L(x) M_t(x+a).
template <bool FIRST>
__device__ __forceinline__ M3 legs(const double *U, const double *GF, const double *I, const double *Q,
                                   const double *R, const double *W, const Geom &g, int mu, int r, int s,
                                   const int x[4], const FatCoeffs &w, double scale)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int nu = other_axis(mu, r), ia = 2 * r + (s < 0 ? 1 : 0);
    int xa[4], xm[4];
    step(g, x, nu, s, xa);
    step(g, x, mu, 1, xm);
    const int64_t ex = eo_of(g, x), exa = eo_of(g, xa);
    const M3 L = FIRST ? step_link(U, V, g, xm, nu, s) : step_link(U, V, g, x, nu, s);
    // Gp op(L, M): first leg Gp L M^dag, return leg Gp^dag L M
    auto term = [&](const M3 &Gp, const M3 &M) {
        return FIRST ? mul<false, false>(Gp, mul<false, true>(L, M)) : mul<true, false>(Gp, mul<false, false>(L, M));
    };
    M3 out = term(scaled(scale, ldm3(GF, V, mu, ex)), ldm3(I, V, ia, exa));
    M3 t = scaled(w.cL, ldm3(Q, V, ia, ex));
    axpy(t, w.c7, ldm3(R, V, r, ex));
    acc(out, term(t, ldm3(U, V, mu, exa)));
#pragma unroll 1
    for (int k = 0; k < 3; k++) {
        if (k == r) continue;
        acc(out, term(q_pair(Q, V, k, ex), ldm3(W, V, 3 - r - k, exa)));
    }
    return out;
}

// G_U,nu(z) += the legs through U_nu(z), nu the r-th axis other than mu:
// L_{+nu}(z) as a first leg (staples at z) and a return leg (at z - mu),
// L_{-nu}(z + nu) = U_nu(z)^dag as a first leg (at z + nu) and a return leg
// (at z + nu - mu); 6 * nbh_pad blocks
__global__ __launch_bounds__(kBS) void k_vjp_tr(const double *__restrict__ U, const double *__restrict__ GF,
                                                const double *__restrict__ I, const double *__restrict__ Q,
                                                const double *__restrict__ R, const double *__restrict__ W,
                                                double *__restrict__ GU, Geom g, int mu, FatCoeffs w, double scale,
                                                int nbh_pad)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int k = (int)(blockIdx.x >> 3);
    const int r = k % 3;
    const int64_t ez = xcd_site(g, (int)(blockIdx.x & 7), k / 3, nbh_pad, (int)threadIdx.x);
    if (ez < 0) return;
    const int nu = other_axis(mu, r);
    int z[4], zm[4], zn[4], znm[4];
    site_coords(g, ez, z);
    step(g, z, mu, -1, zm);
    step(g, z, nu, 1, zn);
    step(g, zn, mu, -1, znm);
    M3 back = legs<true>(U, GF, I, Q, R, W, g, mu, r, -1, zn, w, scale);
    acc(back, legs<false>(U, GF, I, Q, R, W, g, mu, r, -1, znm, w, scale));
    M3 out = ldm3(GU, V, nu, ez);
    acc(out, adj(back));
    acc(out, legs<true>(U, GF, I, Q, R, W, g, mu, r, 1, z, w, scale));
    acc(out, legs<false>(U, GF, I, Q, R, W, g, mu, r, 1, zm, w, scale));
    stm3(GU, V, nu, ez, out);
}

} // namespace

hipError_t launch_fatten(const double *U, double *F, double *N, double *W, const Geom &g, const FatCoeffs &w,
                         hipStream_t s, double *I)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int nbh = (int)(((int64_t)g.Vh + kBS - 1) / kBS), nbh_pad = (nbh + 7) / 8 * 8;
    for (int mu = 0; mu < 4; mu++) {
        // with I: the fields of every direction kept (W per direction, I after them)
        double *Wm = I ? W + (size_t)mu * 3 * V * 18 : W;
        double *Im = I ? I + (size_t)mu * 6 * V * 18 : nullptr;
        hipLaunchKernelGGL(k_fat_inner, dim3(6u * (unsigned)nbh_pad), dim3(kBS), 0, s, U, Wm, g, mu, w.c5, w.c7,
                           nbh_pad);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_fat_outer, dim3(2u * (unsigned)nbh_pad), dim3(kBS), 0, s, U, Wm, F, N, g, mu, w,
                           nbh_pad, Im);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fatten_vjp(const double *U, const double *GF, const double *GN, double *GU, double *ws,
                             const Geom &g, const FatCoeffs &w, double scale, bool accumulate, hipStream_t s,
                             const double *Wk, const double *Ik)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int nbh = (int)(((int64_t)g.Vh + kBS - 1) / kBS), nbh_pad = (nbh + 7) / 8 * 8;
    double *W = ws, *I = W + 3 * V * 18, *Q = I + 6 * V * 18, *R = Q + 6 * V * 18;
    hipError_t e;
    if (!accumulate && (e = launch_zero(GU, (size_t)4 * V * 18 * sizeof(double), s)) != hipSuccess) return e;
    const dim3 b(kBS), g2(2u * (unsigned)nbh_pad), g6(6u * (unsigned)nbh_pad), g12(12u * (unsigned)nbh_pad);
    for (int mu = 0; mu < 4; mu++) {
        if (Wk) { // the forward's fields of this direction
            W = (double *)Wk + (size_t)mu * 3 * V * 18;
            I = (double *)Ik + (size_t)mu * 6 * V * 18;
        } else {
            hipLaunchKernelGGL(k_fat_inner, g6, b, 0, s, U, W, g, mu, w.c5, w.c7, nbh_pad);
            hipLaunchKernelGGL(k_vjp_mid, g12, b, 0, s, U, W, I, g, mu, w, nbh_pad);
        }
        hipLaunchKernelGGL(k_vjp_q, g12, b, 0, s, U, GF, Q, g, mu, scale, nbh_pad);
        hipLaunchKernelGGL(k_vjp_r, g6, b, 0, s, U, Q, R, g, mu, nbh_pad);
        hipLaunchKernelGGL(k_vjp_mu, g2, b, 0, s, U, GF, GN, Q, R, GU, g, mu, w, scale, nbh_pad);
        hipLaunchKernelGGL(k_vjp_tr, g6, b, 0, s, U, GF, I, Q, R, W, GU, g, mu, w, scale, nbh_pad);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

} // namespace lgt
