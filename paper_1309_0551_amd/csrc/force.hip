// force.hip -- fermion force of S = phi^dag A^-1 phi (the outer product
// su3_projector of Table 1, C_ij = a_i conj(b_j)).
//
// With X = A^-1 phi on even sites and Y = D_oe X on odd sites, dS =
// 2 Re(X^dag dD_eo Y), which per link gives
//   x even: G_mu(x) = +2 eta_mu(x) s+_mu(x) X(x) Y(x+mu)^dag
//   x odd : G_mu(x) = -2 eta_mu(x) s+_mu(x) Y(x) X(x+mu)^dag
// and dS/dRe U_ij = Re G_ij, dS/dIm U_ij = Im G_ij. One thread per link; the
// kernel is bound by the 144-byte gradient write per link.
#include "fields.hpp"
#include "kernels.hpp"

namespace lgt {

// NAIK: the derivative for the three-link field of the improved operator:
// the link N_mu(x) joins x to x + 3 mu, with that hop's sign.
template <bool NAIK>
__global__ __launch_bounds__(kBS) void k_force(const double *__restrict__ X, const double *__restrict__ Y,
                                               double scale, double *__restrict__ G, Geom g)
{
    // A workgroup's 256 links are consecutive in [4][V], so its gradients are
    // one contiguous 36 KB run: each thread writes its 3x3 matrix into LDS,
    // and the workgroup then stores the run with fully coalesced 16-byte
    // stores (a direct store of 144 bytes per thread spreads every store
    // instruction of a wavefront over 64 places 144 bytes apart).
    __shared__ dv2 buf[kBS * 9];
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t first = (int64_t)blockIdx.x * kBS;
    const int64_t idx = first + threadIdx.x; // mu*V + eo
    if (idx < 4 * V) {
        const int mu = (int)(idx / V);
        const int64_t eo = idx - mu * V;
        const int par = eo >= g.Vh;
        const int cb = (int)(eo - par * (int64_t)g.Vh);
        int c[4];
        decode(g, par, cb, c);
        int f;
        bool hop_neg;
        if constexpr (NAIK) {
            const Hop h = hop3_rt(g, c, cb, mu);
            f = h.f;
            hop_neg = h.fneg; // eta_mu(x) times the boundary sign of the three-step hop
        } else {
            f = nbr_fwd(g, c, cb, mu);
            hop_neg = fwd_neg(g, c, mu);
        }
        // a: the vector at x, b: the vector at x+mu (other parity)
        cx<double> a[3], b[3];
        if (par == 0) {
            VecFmt<double>::load<false>(X, (size_t)g.Vh, cb, a);
            VecFmt<double>::load<false>(Y, (size_t)g.Vh, f, b);
        } else {
            VecFmt<double>::load<false>(Y, (size_t)g.Vh, cb, a);
            VecFmt<double>::load<false>(X, (size_t)g.Vh, f, b);
        }
        const bool neg = hop_neg ^ (par == 1);
        const double s = neg ? -2.0 * scale : 2.0 * scale;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const double re = a[i].re * b[j].re + a[i].im * b[j].im;
                const double im = a[i].im * b[j].re - a[i].re * b[j].im;
                buf[threadIdx.x * 9 + 3 * i + j] = dv2{s * re, s * im};
            }
    }
    __syncthreads();
    const int64_t left = 4 * V - first;
    const int n = 9 * (int)(left < kBS ? left : kBS);
    dv2 *out = (dv2 *)G + first * 9;
    for (int k = threadIdx.x; k < n; k += kBS) st<true>(out, (unsigned)k, buf[k]); // streamed: no reuse
}

hipError_t launch_force(const double *Xnat, const double *Ynat, double scale, double *G, const Geom &g,
                        hipStream_t s, bool naik)
{
    const int64_t n = 8 * (int64_t)g.Vh;
    const dim3 grid((unsigned)((n + kBS - 1) / kBS)), block(kBS);
    if (naik) hipLaunchKernelGGL(k_force<true>, grid, block, 0, s, Xnat, Ynat, scale, G, g);
    else hipLaunchKernelGGL(k_force<false>, grid, block, 0, s, Xnat, Ynat, scale, G, g);
    return hipGetLastError();
}

// dS/dphi of S = phi^dag A^-1 phi: A^-1 is Hermitian, so dS = 2 Re <X, dphi>
// with X = A^-1 phi, i.e. dS/dRe phi = 2 Re X, dS/dIm phi = 2 Im X. One thread
// per pair of reals of the canonical even vector (bound by its read and write).
__global__ __launch_bounds__(kBS) void k_phi_grad(const dv2 *__restrict__ X, double s2, dv2 *__restrict__ g,
                                                  int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i >= n) return;
    const dv2 v = X[i];
    g[i] = dv2{s2 * v.x, s2 * v.y};
}

hipError_t launch_phi_grad(const double *X, double scale, double *gphi, const Geom &g, hipStream_t s)
{
    const int64_t n = 3 * (int64_t)g.Vh; // complex numbers of one parity vector
    const dim3 grid((unsigned)((n + kBS - 1) / kBS)), block(kBS);
    hipLaunchKernelGGL(k_phi_grad, grid, block, 0, s, (const dv2 *)X, 2.0 * scale, (dv2 *)gphi, n);
    return hipGetLastError();
}

} // namespace lgt
