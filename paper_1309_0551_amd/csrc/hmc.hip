// hmc.hip -- the gauge-field side of the HMC step around the solve.
//
// Fields in the canonical layout [4][V][3][3][2] (float64, eo site order):
// links U, momenta P (traceless anti-Hermitian) and derivatives G with
// dS = sum Re tr(G^dag dU) (the fermion force's convention). One thread per
// link (per site for the plaquette). Kernels:
//   gauge force  G (+)= scale * (-(beta/3)) Sigma^dag, Sigma = staple sum
//                (the Table 1 products mult_su3_nn / _na / _an)
//   momentum     P += eps * TA(U G^dag) / 2   (dP/dt that conserves
//                H = -sum tr P^2 + S for dU/dt = P U)
//   links        U = exp(eps P) U, exp by a degree-12 Taylor series in
//                Horner form (|eps P| <= 1 gives a remainder below 1e-9 and
//                far below that for molecular-dynamics steps)
//   plaquette    sum_{x, mu<nu} Re tr U_mu,nu(x)      (FP64 partials, fixed order)
//   kinetic      -sum tr P^2                           (FP64 partials, fixed order)
#include "fields.hpp"
#include "kernels.hpp"
#include "reduce.hpp"
#include "su3.hpp"

namespace lgt {

namespace {

// G_mu(x) (+)= f Sigma_mu(x)^dag, one thread per link, runtime loop over nu
__global__ __launch_bounds__(kBS) void k_gauge_force(const double *__restrict__ U, double *__restrict__ G, Geom g,
                                                     double f, int accumulate)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t l = (int64_t)blockIdx.x * kBS + threadIdx.x; // mu * V + x
    if (l >= 4 * V) return;
    const int mu = (int)(l / V);
    const int64_t x = l - mu * V;
    int c[4];
    site_coords(g, x, c);
    M3 S;
#pragma unroll
    for (int k = 0; k < 9; k++) S.e[k] = cx<double>{0.0, 0.0};
#pragma unroll 1
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        const int64_t xpm = eo_shift(g, c, mu, 1, nu, 0), xpn = eo_shift(g, c, nu, 1, mu, 0);
        const int64_t xmn = eo_shift(g, c, nu, -1, mu, 0), xpmmn = eo_shift(g, c, mu, 1, nu, -1);
        // U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
        const M3 a = mul<false, true>(ldm3(U, V, nu, xpm), ldm3(U, V, mu, xpn));
        acc(S, mul<false, true>(a, ldm3(U, V, nu, x)));
        // U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
        const M3 b = mul<true, true>(ldm3(U, V, nu, xpmmn), ldm3(U, V, mu, xmn));
        acc(S, mul<false, false>(b, ldm3(U, V, nu, xmn)));
    }
    M3 out;
    if (accumulate) out = ldm3(G, V, mu, x);
#pragma unroll
    for (int i = 0; i < 3; i++) {
#pragma unroll
        for (int j = 0; j < 3; j++) {
            // (Sigma^dag)_ij = conj(Sigma_ji)
            const cx<double> s = S.e[3 * j + i];
            const cx<double> v{f * s.re, -f * s.im};
            if (accumulate) {
                out.e[3 * i + j].re += v.re;
                out.e[3 * i + j].im += v.im;
            } else {
                out.e[3 * i + j] = v;
            }
        }
    }
    stm3(G, V, mu, x, out);
}

// P += eps * TA(U G^dag) / 2, per link
__global__ __launch_bounds__(kBS) void k_momentum(const double *__restrict__ U, const double *__restrict__ G,
                                                  double *__restrict__ P, int64_t V, double eps)
{
    const int64_t l = (int64_t)blockIdx.x * kBS + threadIdx.x; // mu * V + x
    if (l >= 4 * V) return;
    const int mu = (int)(l / V);
    const int64_t x = l - mu * V;
    const M3 X = mul<false, true>(ldm3(U, V, mu, x), ldm3(G, V, mu, x));
    M3 p = ldm3(P, V, mu, x);
    // A = (X - X^dag)/2, then minus tr(A)/3 on the diagonal
    double tr_im = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++) tr_im += X.e[4 * i].im; // tr A = i Im tr X
    const double h = 0.5 * eps;
#pragma unroll
    for (int i = 0; i < 3; i++) {
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const cx<double> a = X.e[3 * i + j], b = X.e[3 * j + i];
            double re = 0.5 * (a.re - b.re), im = 0.5 * (a.im + b.im);
            if (i == j) im -= tr_im / 3.0;
            p.e[3 * i + j].re += h * re;
            p.e[3 * i + j].im += h * im;
        }
    }
    stm3(P, V, mu, x, p);
}

// U = exp(eps P) U with exp(A) = I + A (I + A/2 (I + ... (I + A/12)))
__global__ __launch_bounds__(kBS) void k_links(const double *__restrict__ P, double *__restrict__ U, int64_t V,
                                               double eps)
{
    const int64_t l = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (l >= 4 * V) return;
    const int mu = (int)(l / V);
    const int64_t x = l - mu * V;
    M3 A = ldm3(P, V, mu, x);
#pragma unroll
    for (int k = 0; k < 9; k++) {
        A.e[k].re *= eps;
        A.e[k].im *= eps;
    }
    M3 R;
#pragma unroll
    for (int k = 0; k < 9; k++) R.e[k] = cx<double>{(k % 4 == 0) ? 1.0 : 0.0, 0.0};
#pragma unroll 1
    for (int n = 12; n >= 1; n--) {
        M3 T = mul<false, false>(A, R);
        const double s = 1.0 / n;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            R.e[k].re = T.e[k].re * s + ((k % 4 == 0) ? 1.0 : 0.0);
            R.e[k].im = T.e[k].im * s;
        }
    }
    stm3(U, V, mu, x, mul<false, false>(R, ldm3(U, V, mu, x)));
}

// per-workgroup partial sums of Re tr U_mu,nu(x) over mu < nu
__global__ __launch_bounds__(kBS) void k_plaquette(const double *__restrict__ U, Geom g, double *partials)
{
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t x = (int64_t)blockIdx.x * kBS + threadIdx.x;
    double s = 0.0;
    if (x < V) {
        int c[4];
        site_coords(g, x, c);
#pragma unroll 1
        for (int k = 0; k < 6; k++) {
            // planes (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
            const int mu = k < 3 ? 0 : (k < 5 ? 1 : 2);
            const int nu = k < 3 ? k + 1 : (k < 5 ? k - 1 : 3);
            const M3 a = mul<false, false>(ldm3(U, V, mu, x), ldm3(U, V, nu, eo_shift(g, c, mu, 1, nu, 0)));
            const M3 b = mul<false, true>(a, ldm3(U, V, mu, eo_shift(g, c, nu, 1, mu, 0)));
            const M3 d = mul<false, true>(b, ldm3(U, V, nu, x));
            s += d.e[0].re + d.e[4].re + d.e[8].re;
        }
    }
    write_partial(s, partials, blockIdx.x);
}

__global__ __launch_bounds__(kBS) void k_kinetic(const double *__restrict__ P, int64_t nlinks, double *partials)
{
    const int64_t l = (int64_t)blockIdx.x * kBS + threadIdx.x;
    double s = 0.0;
    if (l < nlinks) {
        const dv2 *p = (const dv2 *)(P + l * 18);
        // -tr(P^2) = -sum_ij P_ij P_ji
#pragma unroll
        for (int i = 0; i < 3; i++) {
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const dv2 a = p[3 * i + j], b = p[3 * j + i];
                s -= a.x * b.x - a.y * b.y;
            }
        }
    }
    write_partial(s, partials, blockIdx.x);
}

// sum of n partials in index order (one workgroup) into *out
__global__ __launch_bounds__(kBS) void k_sum_partials(const double *__restrict__ partials, int n, double *out)
{
    __shared__ double lds[kBS / 64];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += kBS) a += partials[i];
    const double t = block_sum(a, lds);
    if (threadIdx.x == 0) *out = t;
}

// phi = 2m R_e - t (canonical even vectors)
__global__ __launch_bounds__(kBS) void k_phi(const double *__restrict__ Re, const double *__restrict__ t,
                                             double *__restrict__ phi, int64_t n, double m2)
{
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i < n) phi[i] = m2 * Re[i] - t[i];
}

} // namespace

static unsigned nblocks(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

hipError_t launch_gauge_force(const double *U, double *G, const Geom &g, double beta, double scale, int accumulate,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_gauge_force, dim3(nblocks(8 * (int64_t)g.Vh)), dim3(kBS), 0, s, U, G, g,
                       -scale * beta / 3.0, accumulate);
    return hipGetLastError();
}

hipError_t launch_momentum(const double *U, const double *G, double *P, int64_t V, double eps, hipStream_t s)
{
    hipLaunchKernelGGL(k_momentum, dim3(nblocks(4 * V)), dim3(kBS), 0, s, U, G, P, V, eps);
    return hipGetLastError();
}

hipError_t launch_links(const double *P, double *U, int64_t V, double eps, hipStream_t s)
{
    hipLaunchKernelGGL(k_links, dim3(nblocks(4 * V)), dim3(kBS), 0, s, P, U, V, eps);
    return hipGetLastError();
}

hipError_t launch_plaquette(const double *U, const Geom &g, double *partials, double *out, hipStream_t s)
{
    const unsigned nb = nblocks(2 * (int64_t)g.Vh);
    hipLaunchKernelGGL(k_plaquette, dim3(nb), dim3(kBS), 0, s, U, g, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBS), 0, s, partials, (int)nb, out);
    return hipGetLastError();
}

hipError_t launch_kinetic(const double *P, int64_t V, double *partials, double *out, hipStream_t s)
{
    const unsigned nb = nblocks(4 * V);
    hipLaunchKernelGGL(k_kinetic, dim3(nb), dim3(kBS), 0, s, P, 4 * V, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBS), 0, s, partials, (int)nb, out);
    return hipGetLastError();
}

hipError_t launch_phi(const double *Re, const double *t, double *phi, int64_t n, double m2, hipStream_t s)
{
    hipLaunchKernelGGL(k_phi, dim3(nblocks(n)), dim3(kBS), 0, s, Re, t, phi, n, m2);
    return hipGetLastError();
}

} // namespace lgt
