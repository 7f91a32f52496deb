// hmc_abi.cpp -- C ABI of the HMC step: the gauge-side kernels one by one and a
// native driver for one leapfrog trajectory with a Metropolis test, built on
// the library's own CG (FP64 or mixed precision) and fermion force.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "ctx.hpp"

namespace lgt {
hipError_t launch_gauge_force(const double *U, double *G, const Geom &g, double beta, double scale, int accumulate,
                              hipStream_t s);
hipError_t launch_momentum(const double *U, const double *G, double *P, int64_t V, double eps, hipStream_t s);
hipError_t launch_links(const double *P, double *U, int64_t V, double eps, hipStream_t s);
hipError_t launch_plaquette(const double *U, const Geom &g, double *partials, double *out, hipStream_t s);
hipError_t launch_kinetic(const double *P, int64_t V, double *partials, double *out, hipStream_t s);
hipError_t launch_phi(const double *Re, const double *t, double *phi, int64_t n, double m2, hipStream_t s);
} // namespace lgt

using namespace lgt;

namespace {

#define CHECK(c)                                                     \
    do {                                                             \
        clear_error();                                               \
        if (!(c)) return fail(LGT_ERR_ARG, "context is NULL");       \
    } while (0)

int64_t volume(const lgt_ctx *c) { return 2 * (int64_t)c->g.Vh; }

// scalar reduction result of a launch_* kernel pair, read back synchronously
lgt_status reduce_to_host(lgt_ctx *c, double *dev_out, double *host_out)
{
    double *h = (double *)pinned(c, 3 * sizeof(CgState));
    if (!h) return fail(LGT_ERR_OOM, "cannot allocate pinned staging");
    LGT_HIP(hipMemcpyAsync(h, dev_out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LGT_HIP(hipStreamSynchronize(c->stream));
    *host_out = h[0];
    return LGT_OK;
}

lgt_status plaquette(lgt_ctx *c, const double *U, double *sum)
{
    const int64_t nb = (volume(c) + kBS - 1) / kBS;
    double *part = (double *)workspace(c, "hmc.partials", sizeof(double) * (size_t)(4 * nb + 8));
    double *out = (double *)workspace(c, "hmc.scalar", 64);
    if (!part || !out) return fail(LGT_ERR_OOM, "cannot allocate the reduction workspace");
    LGT_HIP(launch_plaquette(U, c->g, part, out, c->stream));
    return reduce_to_host(c, out, sum);
}

lgt_status kinetic(lgt_ctx *c, const double *P, double *K)
{
    const int64_t nb = (4 * volume(c) + kBS - 1) / kBS;
    double *part = (double *)workspace(c, "hmc.partials", sizeof(double) * (size_t)(nb + 8));
    double *out = (double *)workspace(c, "hmc.scalar", 64);
    if (!part || !out) return fail(LGT_ERR_OOM, "cannot allocate the reduction workspace");
    LGT_HIP(launch_kinetic(P, volume(c), part, out, c->stream));
    return reduce_to_host(c, out, K);
}

lgt_status fat_coeffs(const lgt_fat_coeffs *w, FatCoeffs *fc)
{
    if (!w) return fail(LGT_ERR_ARG, "coefficients are NULL");
    const double cs[6] = {w->one_link, w->staple3, w->staple5, w->staple7, w->lepage, w->naik};
    for (double v : cs)
        if (!std::isfinite(v)) return fail(LGT_ERR_ARG, "coefficients must be finite");
    *fc = FatCoeffs{w->one_link, w->staple3, w->staple5, w->staple7, w->lepage, w->naik};
    return LGT_OK;
}

// [p, p + bytes) and [q, q + bytes) overlap
bool overlap(const void *p, const void *q, size_t bytes)
{
    const char *a = (const char *)p, *b = (const char *)q;
    return a < b + bytes && b < a + bytes;
}

// Wk, Ik: the fields a launch_fatten at the same U kept, or null
lgt_status fatten_vjp(lgt_ctx *c, const double *U, const FatCoeffs &fc, const double *GF, const double *GN,
                      double scale, bool accumulate, double *GU, const double *Wk = nullptr,
                      const double *Ik = nullptr)
{
    double *ws = (double *)workspace(c, "fatten.vjp", (size_t)kFatVjpMatrices * volume(c) * 18 * sizeof(double));
    if (!ws) return fail(LGT_ERR_OOM, "cannot allocate the fattening workspace");
    LGT_HIP(launch_fatten_vjp(U, GF, GN, GU, ws, c->g, fc, scale, accumulate, c->stream, Wk, Ik));
    return LGT_OK;
}

// One trajectory; fc = null: the one-link operator of U, else the improved
// operator of the fields F(U), N(U) fattened with fc (its fermion force taken
// back to U through the fattening).
lgt_status hmc_trajectory(lgt_ctx *c, double *U, double *P, const double *R_e, const double *R_o,
                          const lgt_hmc_params *hp, const FatCoeffs *fc, lgt_hmc_result *hr)
{
    CHECK(c);
    lgt_status s;
    if (!hp || !hr) return fail(LGT_ERR_ARG, "params or result is NULL");
    if ((s = check_ptr(U, "U")) != LGT_OK) return s;
    if ((s = check_ptr(P, "P")) != LGT_OK) return s;
    if ((s = check_ptr(R_e, "R_e")) != LGT_OK) return s;
    if ((s = check_ptr(R_o, "R_o")) != LGT_OK) return s;
    if (!(hp->mass > 0.0) || !std::isfinite(hp->beta) || !(hp->eps > 0.0) || hp->nsteps < 1 || !(hp->tol > 0.0))
        return fail(LGT_ERR_ARG, "need mass > 0, finite beta, eps > 0, nsteps >= 1, tol > 0");
    if (hp->scheme != LGT_CG_FP64 && hp->scheme != LGT_CG_RELIABLE)
        return fail(LGT_ERR_ARG, "scheme must be LGT_CG_FP64 or LGT_CG_RELIABLE");
    if (!(hp->u >= 0.0 && hp->u < 1.0)) return fail(LGT_ERR_ARG, "u must be in [0, 1)");
    DeviceScope ds(c->device);
    const auto t0 = std::chrono::steady_clock::now();
    const hipStream_t st = c->stream;
    const int64_t V = volume(c);
    const size_t fb = (size_t)4 * V * 18 * sizeof(double);
    const size_t v64 = (size_t)c->g.Vh * 48;
    const bool mixed = hp->scheme == LGT_CG_RELIABLE, imp = fc != nullptr;
    // one-link: U packed F64 x 18 (+ F32 x 12 inner); improved: F and N packed
    // F64 x 18 (+ F32 x 18 inner: fattened fields are not unitary)
    const int32_t lo_recon = imp ? LGT_R18 : LGT_R12;
    size_t lb_hi = 0, lb_lo = 0;
    (void)lgt_links_bytes(&c->geom, LGT_F64, LGT_R18, &lb_hi);
    if (mixed) (void)lgt_links_bytes(&c->geom, LGT_F32, lo_recon, &lb_lo);
    double *U0 = (double *)workspace(c, "hmc.U0", fb);
    double *P0 = (double *)workspace(c, "hmc.P0", fb);
    double *G = (double *)workspace(c, "hmc.G", fb);
    void *Uhi = workspace(c, "hmc.Uhi", lb_hi);
    void *Ulo = mixed ? workspace(c, "hmc.Ulo", lb_lo) : nullptr;
    double *phi = (double *)workspace(c, "hmc.phi", v64);
    double *X = (double *)workspace(c, "hmc.X", v64);
    double *t = (double *)workspace(c, "hmc.t", v64);
    void *nv_in = workspace(c, "hmc.nv_in", v64);
    void *nv_out = workspace(c, "hmc.nv_out", v64);
    if (!U0 || !P0 || !G || !Uhi || (mixed && !Ulo) || !phi || !X || !t || !nv_in || !nv_out)
        return fail(LGT_ERR_OOM, "cannot allocate the HMC workspace");
    // improved: canonical F, N and their derivatives, packed Naik fields, and
    // the fattening's intermediate fields of every direction (12 V and 24 V
    // matrices), kept by each fattening for the chain rule at the same U,
    // which then skips a third of its products
    double *Fc = nullptr, *Nc = nullptr, *GF = nullptr, *GN = nullptr, *Wk = nullptr, *Ik = nullptr;
    void *Nhi = nullptr, *Nlo = nullptr;
    if (imp) {
        Fc = (double *)workspace(c, "hmc.F", fb);
        Nc = (double *)workspace(c, "hmc.N", fb);
        GF = (double *)workspace(c, "hmc.GF", fb);
        GN = (double *)workspace(c, "hmc.GN", fb);
        Nhi = workspace(c, "hmc.Nhi", lb_hi);
        Nlo = mixed ? workspace(c, "hmc.Nlo", lb_lo) : nullptr;
        Wk = (double *)workspace(c, "hmc.fatW", (size_t)12 * V * 18 * sizeof(double));
        Ik = (double *)workspace(c, "hmc.fatI", (size_t)24 * V * 18 * sizeof(double));
        if (!Fc || !Nc || !GF || !GN || !Nhi || (mixed && !Nlo) || !Wk || !Ik)
            return fail(LGT_ERR_OOM, "cannot allocate the HMC workspace");
    }
    LGT_HIP(hipMemcpyAsync(U0, U, fb, hipMemcpyDeviceToDevice, st));
    LGT_HIP(hipMemcpyAsync(P0, P, fb, hipMemcpyDeviceToDevice, st));

    lgt_links lhi{Uhi, LGT_F64, LGT_R18}, llo{Ulo, LGT_F32, lo_recon};
    lgt_links nhi{Nhi, LGT_F64, LGT_R18}, nlo{Nlo, LGT_F32, LGT_R18};
    lgt_fat_coeffs w{};
    if (imp) w = lgt_fat_coeffs{fc->c1, fc->c3, fc->c5, fc->c7, fc->cL, fc->cN};
    // the operator's link fields at the current U
    auto pack = [&]() -> lgt_status {
        lgt_status r;
        if (!imp) {
            r = lgt_pack_links(c, U, LGT_F64, LGT_R18, Uhi);
            if (r == LGT_OK && mixed) r = lgt_pack_links(c, U, LGT_F32, LGT_R12, Ulo);
            return r;
        }
        LGT_HIP(launch_fatten(U, Fc, Nc, Wk, c->g, *fc, st, Ik));
        if ((r = lgt_pack_links(c, Fc, LGT_F64, LGT_R18, Uhi)) != LGT_OK) return r;
        if ((r = lgt_pack_links(c, Nc, LGT_F64, LGT_R18, Nhi)) != LGT_OK) return r;
        if (mixed && (r = lgt_pack_links(c, Fc, LGT_F32, LGT_R18, Ulo)) != LGT_OK) return r;
        if (mixed && (r = lgt_pack_links(c, Nc, LGT_F32, LGT_R18, Nlo)) != LGT_OK) return r;
        return LGT_OK;
    };
    lgt_cg_params cp;
    std::memset(&cp, 0, sizeof(cp));
    cp.mass = hp->mass;
    cp.tol = hp->tol;
    cp.max_iter = 100000;
    cp.scheme = hp->scheme;
    cp.ru_interval = 50;
    std::memset(hr, 0, sizeof(*hr));
    // X = A^-1 phi from x0 = 0; S_f = Re <phi, X>
    auto solve = [&](double *Sf) -> lgt_status {
        lgt_cg_result r;
        lgt_status q = imp ? cg_solve(c, &lhi, mixed ? &llo : nullptr, &cp, phi, X, &r, &nhi, mixed ? &nlo : nullptr)
                           : cg_solve(c, &lhi, mixed ? &llo : nullptr, &cp, phi, X, &r);
        hr->cg_iters += r.iters;
        hr->cg_solves += 1;
        if (q != LGT_OK) return q;
        if (Sf) {
            double d[2];
            // V/2 sites x 3 colours complex numbers
            if ((q = lgt_cdot(c, (int64_t)c->g.Vh * 3, phi, X, d)) != LGT_OK) return q;
            *Sf = d[0];
        }
        return LGT_OK;
    };
    // P += h * TA(U G^dag) / 2 with G = G_fermion + G_gauge at the current U
    auto kick = [&](double h) -> lgt_status {
        lgt_status q = solve(nullptr);
        if (q != LGT_OK) return q;
        if (!imp) {
            if ((q = lgt_force(c, &lhi, X, 1.0, G)) != LGT_OK) return q;
        } else {
            if ((q = lgt_force_improved(c, &lhi, &nhi, X, 1.0, GF, GN)) != LGT_OK) return q;
            // the last fattening ran at this U (pack() before the solve)
            if ((q = fatten_vjp(c, U, *fc, GF, GN, 1.0, false, G, Wk, Ik)) != LGT_OK) return q;
        }
        LGT_HIP(launch_gauge_force(U, G, c->g, hp->beta, 1.0, 1, st));
        LGT_HIP(launch_momentum(U, G, P, V, h, st));
        return LGT_OK;
    };
    auto energy = [&](double *Sg, double *Sf, double *K) -> lgt_status {
        double pl;
        lgt_status q;
        if ((q = plaquette(c, U, &pl)) != LGT_OK) return q;
        *Sg = hp->beta * (6.0 * (double)V - pl / 3.0);
        if ((q = kinetic(c, P, K)) != LGT_OK) return q;
        return solve(Sf);
    };

    // pseudofermion phi_e = 2m R_e - D_eo R_o at the starting links
    if ((s = pack()) != LGT_OK) return s;
    if ((s = lgt_pack_vec(c, LGT_F64, R_o, nv_in)) != LGT_OK) return s;
    s = imp ? lgt_dslash_improved(c, &lhi, &nhi, LGT_EVEN, nv_in, nv_out) : lgt_dslash(c, &lhi, LGT_EVEN, nv_in, nv_out);
    if (s != LGT_OK) return s;
    if ((s = lgt_unpack_vec(c, LGT_F64, nv_out, t)) != LGT_OK) return s;
    LGT_HIP(launch_phi(R_e, t, phi, (int64_t)c->g.Vh * 6, 2.0 * hp->mass, st));

    if ((s = energy(&hr->Sg0, &hr->Sf0, &hr->K0)) != LGT_OK) return s;
    // leapfrog: half kick, (drift, kick) x nsteps with the last kick halved
    if ((s = kick(0.5 * hp->eps)) != LGT_OK) return s;
    for (int k = 0; k < hp->nsteps; k++) {
        LGT_HIP(launch_links(P, U, V, hp->eps, st));
        if ((s = pack()) != LGT_OK) return s;
        if ((s = kick(k < hp->nsteps - 1 ? hp->eps : 0.5 * hp->eps)) != LGT_OK) return s;
    }
    if ((s = energy(&hr->Sg1, &hr->Sf1, &hr->K1)) != LGT_OK) return s;
    hr->H0 = hr->K0 + hr->Sg0 + hr->Sf0;
    hr->H1 = hr->K1 + hr->Sg1 + hr->Sf1;
    hr->dH = hr->H1 - hr->H0;
    if (!std::isfinite(hr->dH)) return fail(LGT_ERR_NONFINITE, "non-finite energy change");
    hr->accepted = hp->u < std::exp(-hr->dH) ? 1 : 0;
    if (!hr->accepted) {
        LGT_HIP(hipMemcpyAsync(U, U0, fb, hipMemcpyDeviceToDevice, st));
        LGT_HIP(hipMemcpyAsync(P, P0, fb, hipMemcpyDeviceToDevice, st));
    }
    LGT_HIP(hipStreamSynchronize(st));
    hr->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return LGT_OK;
}

} // namespace

extern "C" {

lgt_status lgt_gauge_force(lgt_ctx *c, const double *U, double beta, double scale, int32_t accumulate, double *G)
{
    CHECK(c);
    lgt_status s;
    if ((s = check_ptr(U, "U")) != LGT_OK) return s;
    if ((s = check_ptr(G, "G")) != LGT_OK) return s;
    if (U == G) return fail(LGT_ERR_ARG, "U and G alias");
    if (!std::isfinite(beta) || !std::isfinite(scale)) return fail(LGT_ERR_ARG, "beta and scale must be finite");
    DeviceScope ds(c->device);
    LGT_HIP(launch_gauge_force(U, G, c->g, beta, scale, accumulate != 0, c->stream));
    return LGT_OK;
}

lgt_status lgt_momentum_update(lgt_ctx *c, const double *U, const double *G, double eps, double *P)
{
    CHECK(c);
    lgt_status s;
    if ((s = check_ptr(U, "U")) != LGT_OK) return s;
    if ((s = check_ptr(G, "G")) != LGT_OK) return s;
    if ((s = check_ptr(P, "P")) != LGT_OK) return s;
    if (P == U || P == G) return fail(LGT_ERR_ARG, "P aliases U or G");
    if (!std::isfinite(eps)) return fail(LGT_ERR_ARG, "eps must be finite");
    DeviceScope ds(c->device);
    LGT_HIP(launch_momentum(U, G, P, volume(c), eps, c->stream));
    return LGT_OK;
}

lgt_status lgt_link_update(lgt_ctx *c, const double *P, double eps, double *U)
{
    CHECK(c);
    lgt_status s;
    if ((s = check_ptr(U, "U")) != LGT_OK) return s;
    if ((s = check_ptr(P, "P")) != LGT_OK) return s;
    if (P == U) return fail(LGT_ERR_ARG, "P and U alias");
    if (!std::isfinite(eps)) return fail(LGT_ERR_ARG, "eps must be finite");
    DeviceScope ds(c->device);
    LGT_HIP(launch_links(P, U, volume(c), eps, c->stream));
    return LGT_OK;
}

lgt_status lgt_asqtad_coeffs(double u0, lgt_fat_coeffs *w)
{
    clear_error();
    if (!w) return fail(LGT_ERR_ARG, "coefficients are NULL");
    if (!(u0 > 0.0) || !std::isfinite(u0)) return fail(LGT_ERR_ARG, "u0 must be positive and finite");
    // tree-level weights, each divided by u0^(path length - 1)
    const double u2 = u0 * u0, u4 = u2 * u2, u6 = u4 * u2;
    w->one_link = 5.0 / 8.0;
    w->staple3 = 1.0 / 16.0 / u2;
    w->staple5 = 1.0 / 64.0 / u4;
    w->staple7 = 1.0 / 384.0 / u6;
    w->lepage = -1.0 / 16.0 / u4;
    w->naik = -1.0 / 24.0 / u2;
    return LGT_OK;
}

lgt_status lgt_fatten_links(lgt_ctx *c, const double *U, const lgt_fat_coeffs *w, double *F, double *N)
{
    CHECK(c);
    lgt_status s;
    if ((s = check_ptr(U, "U")) != LGT_OK) return s;
    if ((s = check_ptr(F, "F")) != LGT_OK) return s;
    if ((s = check_ptr(N, "N")) != LGT_OK) return s;
    FatCoeffs fc;
    if ((s = fat_coeffs(w, &fc)) != LGT_OK) return s;
    // the kernel reads U around every link while it writes F and N: no overlap
    const size_t bytes = (size_t)volume(c) * 4 * 18 * sizeof(double);
    if (overlap(U, F, bytes) || overlap(U, N, bytes) || overlap(F, N, bytes))
        return fail(LGT_ERR_ARG, "U, F and N must not overlap");
    DeviceScope ds(c->device);
    double *W = (double *)workspace(c, "fatten.inner", 3 * (size_t)volume(c) * 18 * sizeof(double));
    if (!W) return fail(LGT_ERR_OOM, "cannot allocate the fattening workspace");
    LGT_HIP(launch_fatten(U, F, N, W, c->g, fc, c->stream));
    return LGT_OK;
}

lgt_status lgt_fatten_links_vjp(lgt_ctx *c, const double *U, const lgt_fat_coeffs *w, const double *G_fat,
                                const double *G_naik, double scale, int32_t accumulate, double *G_U)
{
    CHECK(c);
    lgt_status s;
    if ((s = check_ptr(U, "U")) != LGT_OK) return s;
    if ((s = check_ptr(G_fat, "G_fat")) != LGT_OK) return s;
    if ((s = check_ptr(G_naik, "G_naik")) != LGT_OK) return s;
    if ((s = check_ptr(G_U, "G_U")) != LGT_OK) return s;
    FatCoeffs fc;
    if ((s = fat_coeffs(w, &fc)) != LGT_OK) return s;
    if (!std::isfinite(scale)) return fail(LGT_ERR_ARG, "scale must be finite");
    // G_U is written while U, G_fat and G_naik are read around every link
    const size_t bytes = (size_t)volume(c) * 4 * 18 * sizeof(double);
    if (overlap(G_U, U, bytes) || overlap(G_U, G_fat, bytes) || overlap(G_U, G_naik, bytes))
        return fail(LGT_ERR_ARG, "G_U must not overlap U, G_fat or G_naik");
    DeviceScope ds(c->device);
    return fatten_vjp(c, U, fc, G_fat, G_naik, scale, accumulate != 0, G_U);
}

lgt_status lgt_plaquette(lgt_ctx *c, const double *U, double *sum)
{
    CHECK(c);
    lgt_status s;
    if ((s = check_ptr(U, "U")) != LGT_OK) return s;
    if (!sum) return fail(LGT_ERR_ARG, "sum is NULL");
    DeviceScope ds(c->device);
    return plaquette(c, U, sum);
}

lgt_status lgt_kinetic_energy(lgt_ctx *c, const double *P, double *K)
{
    CHECK(c);
    lgt_status s;
    if ((s = check_ptr(P, "P")) != LGT_OK) return s;
    if (!K) return fail(LGT_ERR_ARG, "K is NULL");
    DeviceScope ds(c->device);
    return kinetic(c, P, K);
}

lgt_status lgt_hmc_trajectory(lgt_ctx *c, double *U, double *P, const double *R_e, const double *R_o,
                              const lgt_hmc_params *hp, lgt_hmc_result *hr)
{
    return hmc_trajectory(c, U, P, R_e, R_o, hp, nullptr, hr);
}

lgt_status lgt_hmc_trajectory_improved(lgt_ctx *c, double *U, double *P, const double *R_e, const double *R_o,
                                       const lgt_hmc_params *hp, const lgt_fat_coeffs *w, lgt_hmc_result *hr)
{
    CHECK(c);
    FatCoeffs fc;
    lgt_status s;
    if ((s = fat_coeffs(w, &fc)) != LGT_OK) return s;
    return hmc_trajectory(c, U, P, R_e, R_o, hp, &fc, hr);
}

} // extern "C"
