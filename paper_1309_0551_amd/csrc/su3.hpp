// su3.hpp -- 3x3 complex matrices in the canonical link layout
// ([4][V][3][3][2] float64, eo site order) for the per-link kernels: loads,
// stores, products with either factor adjoint (the Table 1 products
// mult_su3_nn / _na / _an), accumulation, and site arithmetic for paths.
#pragma once
#include "fields.hpp"
#include "geom.hpp"

namespace lgt {

struct M3 {
    cx<double> e[9];
};

__device__ __forceinline__ M3 ldm3(const double *F, int64_t V, int mu, int64_t eo)
{
    const dv2 *p = (const dv2 *)(F + ((int64_t)mu * V + eo) * 18);
    M3 m;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const dv2 v = p[k];
        m.e[k] = cx<double>{v.x, v.y};
    }
    return m;
}
__device__ __forceinline__ void stm3(double *F, int64_t V, int mu, int64_t eo, const M3 &m)
{
    dv2 *p = (dv2 *)(F + ((int64_t)mu * V + eo) * 18);
#pragma unroll
    for (int k = 0; k < 9; k++) p[k] = dv2{m.e[k].re, m.e[k].im};
}

// C = op(A) op(B) with op = identity or adjoint
template <bool DA, bool DB> __device__ __forceinline__ M3 mul(const M3 &A, const M3 &B)
{
    M3 C;
#pragma unroll
    for (int i = 0; i < 3; i++) {
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const cx<double> a = DA ? cx<double>{A.e[3 * k + i].re, -A.e[3 * k + i].im} : A.e[3 * i + k];
                const cx<double> b = DB ? cx<double>{B.e[3 * j + k].re, -B.e[3 * j + k].im} : B.e[3 * k + j];
                re += a.re * b.re - a.im * b.im;
                im += a.re * b.im + a.im * b.re;
            }
            C.e[3 * i + j] = cx<double>{re, im};
        }
    }
    return C;
}

__device__ __forceinline__ void acc(M3 &A, const M3 &B)
{
#pragma unroll
    for (int k = 0; k < 9; k++) {
        A.e[k].re += B.e[k].re;
        A.e[k].im += B.e[k].im;
    }
}

// eo index of the site with coordinates c
__device__ __forceinline__ int64_t eo_of(const Geom &g, const int c[4])
{
    const int64_t lex = c[0] + (int64_t)g.L[0] * (c[1] + (int64_t)g.L[1] * (c[2] + (int64_t)g.L[2] * c[3]));
    const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
    return par * (int64_t)g.Vh + (lex >> 1);
}

// eo index of c + d mu + e nu for directions known only at run time (selects
// only: no indexed access to a private array)
__device__ __forceinline__ int64_t eo_shift(const Geom &g, const int c[4], int mu, int d, int nu, int e)
{
    int s[4];
    s[0] = c[0] + (mu == 0 ? d : 0) + (nu == 0 ? e : 0);
    s[1] = c[1] + (mu == 1 ? d : 0) + (nu == 1 ? e : 0);
    s[2] = c[2] + (mu == 2 ? d : 0) + (nu == 2 ? e : 0);
    s[3] = c[3] + (mu == 3 ? d : 0) + (nu == 3 ? e : 0);
    s[0] = s[0] < 0 ? s[0] + g.L[0] : (s[0] >= g.L[0] ? s[0] - g.L[0] : s[0]);
    s[1] = s[1] < 0 ? s[1] + g.L[1] : (s[1] >= g.L[1] ? s[1] - g.L[1] : s[1]);
    s[2] = s[2] < 0 ? s[2] + g.L[2] : (s[2] >= g.L[2] ? s[2] - g.L[2] : s[2]);
    s[3] = s[3] < 0 ? s[3] + g.L[3] : (s[3] >= g.L[3] ? s[3] - g.L[3] : s[3]);
    return eo_of(g, s);
}

__device__ __forceinline__ void site_coords(const Geom &g, int64_t eo, int c[4])
{
    const int par = eo >= g.Vh;
    decode(g, par, (int)(eo - par * (int64_t)g.Vh), c);
}

} // namespace lgt
