// solver.cpp -- even-odd CG on A = 4 m^2 - D_eo D_oe (host driver).
//
// Textbook CG (alpha = rho/<p,Ap>, x += alpha p, r -= alpha Ap,
// beta = rho'/rho, p = r + beta p) with every scalar kept in device memory:
// the kernels compute alpha and beta themselves from FP64 reductions, and a
// solver state word makes every later kernel of a finished solve exit at
// once. Since D_eo = -D_oe^dag, <p, A p> = 4m^2 |p|^2 + |D_oe p|^2, so alpha is
// known once D_oe has run, and D_eo can apply the update itself. An iteration
// is four launches: x += alpha p (the previous update's) and p = r + beta p;
// t = D_oe p with the partials of <p, A p>; D_eo t with r -= alpha (4m^2 p -
// D_eo t) (Ap is never stored; every workgroup sums D_oe's partials itself for
// alpha) and the partials of |r|^2; and the one-workgroup step for beta and the
// stop tests. On lattices with more than kFuseAlphaMaxParts Dslash workgroups
// a one-workgroup alpha step runs between the two Dslash launches instead,
// since the redundant sums grow with the square of the lattice size. Where an
// inner-precision vector fits in about one XCD's L2 (kFusedXpayMaxBytes),
// p = r + beta p (with the pending x += alpha p) is formed inside D_oe
// instead, three launches an iteration: D_oe gathers r and the old p at every
// neighbour and writes the new p into the other of two p buffers (the state's
// pcur says which is current; the beta step flips it). On larger lattices the
// second gathered vector costs more cache misses than the pass it saves.
// The host enqueues iterations in chunks and reads the state back once per
// chunk, one chunk behind, so the GPU never waits for the host.
//
// Precision forms (single precision gains more than double, Sec. 4):
//  FP64      all in FP64; at inner convergence the true residual b - A x is
//            recomputed and replaces r (a reliable update).
//  RELIABLE  inner CG in FP32 vectors with F32 or BF16 links; every
//            ru_interval iterations and at inner convergence x64 += x_lo,
//            r = b - A64 x64 in FP64 (rounded into r_lo), beta from the
//            FP64 rho, p kept.
//  REFINE    iterative refinement: the inner CG restarts from 0 (beta = 0)
//            after each FP64 residual and stops when its residual has dropped
//            by inner_tol.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ctx.hpp"

namespace lgt {

namespace {

struct Events {
    std::vector<hipEvent_t> ev;
    ~Events()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipError_t make(size_t n)
    {
        ev.resize(n, nullptr);
        for (auto &e : ev) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
};

// Largest partial count for which the update kernel sums the <p, Ap>
// partials itself; LGT_FUSE_ALPHA_MAX overrides the built-in value (both
// paths give the same bits, so this only moves work between launches).
// p = r + beta p inside D_oe (EPI_PAPX, p double-buffered) instead of a pass
// of its own: one launch less per iteration, two vectors gathered at every
// neighbour instead of one. It pays while an inner-precision vector fits in
// about one XCD's L2, kFusedXpayMaxBytes (measured, us an iteration, separate
// -> fused: FP32 x 12 8^4 22.4 -> 18.7, 16^4 23.2 -> 21.4, 24^4 41.3 -> 37.9,
// 32^4 100.8 -> 105.8; BF16 x 12 16^4 50.1 -> 39.3, 24^4 52.5 -> 49.0; FP64
// 8^4 22.0 -> 20.6, 20^4 51.0 -> 47.5, 24^4 90.2 -> 98.9, 32^4 261 -> 292).
// The results are bit-identical either way. LGT_CG_FUSED_XPAY = 1 / 0
// forces it on / off; else `dflt`.
constexpr size_t kFusedXpayMaxBytes = (size_t)4 << 20;
bool fused_xpay(bool dflt)
{
    const char *e = std::getenv("LGT_CG_FUSED_XPAY");
    if (e && !std::strcmp(e, "1")) return true;
    if (e && !std::strcmp(e, "0")) return false;
    return dflt;
}

int fuse_alpha_max()
{
    const char *e = std::getenv("LGT_FUSE_ALPHA_MAX");
    if (!e || !*e) return kFuseAlphaMaxParts;
    char *end = nullptr;
    const long v = std::strtol(e, &end, 10);
    return (end && *end == 0 && v >= 0 && v <= (1L << 30)) ? (int)v : kFuseAlphaMaxParts;
}

} // namespace

lgt_status cg_solve(lgt_ctx *c, const lgt_links *Uhi, const lgt_links *Ulo, const lgt_cg_params *p,
                    const double *b, double *x, lgt_cg_result *res, const lgt_links *U3hi,
                    const lgt_links *U3lo)
{
    const Geom g = c->g;
    const int Vh = g.Vh;
    const hipStream_t s = c->stream;
    const Launch l = site_launch(Vh); // vector kernels
    const int scheme = p->scheme;
    const bool mixed = scheme != SCH_FP64;

    Fmt fhi, flo;
    lgt_status st = check_links(Uhi, true, &fhi);
    if (st != LGT_OK) return st;
    flo = fhi;
    if (mixed) {
        st = check_links(Ulo, false, &flo);
        if (st != LGT_OK) return st;
        if (fmt_is_f64(flo)) return fail(LGT_ERR_ARG, "U_lo must be F32 or BF16 links for a mixed scheme");
    }
    const size_t v64 = (size_t)Vh * 48;
    const size_t vlo = mixed ? (size_t)Vh * 24 : v64;
    const int chunk = scheme == SCH_RELIABLE ? p->ru_interval : (p->check_interval > 0 ? p->check_interval : 50);
    const double inner = scheme == SCH_REFINE ? p->inner_tol : (p->inner_tol > 0 ? p->inner_tol : 1.0);
    const double m4 = 4.0 * p->mass * p->mass;

    // workspace
    double *b64 = (double *)workspace(c, "cg.b64", v64);
    double *x64 = (double *)workspace(c, "cg.x64", v64);
    double *t64 = (double *)workspace(c, "cg.t64", v64);
    double *q64 = (double *)workspace(c, "cg.q64", v64); // scratch FP64 residual
    void *r = workspace(c, "cg.r", vlo);
    void *pp = workspace(c, "cg.p", vlo);
    const bool fx = fused_xpay(vlo <= kFusedXpayMaxBytes);
    void *pp2 = fx ? workspace(c, "cg.p2", vlo) : nullptr;
    void *t = workspace(c, "cg.t", vlo);
    void *xlo = mixed ? workspace(c, "cg.xlo", vlo) : x64;
    // Dslash launches of the two link formats (their workgroup sizes are
    // per-format choices, so their partial-sum counts may differ)
    const bool imp = U3hi != nullptr;
    const Launch lhi = imp ? dslash_launch_improved(c, fhi) : dslash_launch(c, fhi);
    const Launch llo = imp ? dslash_launch_improved(c, flo) : dslash_launch(c, flo);
    // two partial-sum buffers: D_eo reads D_oe's while writing its own
    const size_t np1 = (size_t)std::max(std::max(lhi.nblk_pad, llo.nblk_pad), l.nblk_pad);
    double *partials = (double *)workspace(c, "cg.partials", sizeof(double) * 2 * np1);
    double *partials2 = partials ? partials + np1 : nullptr;
    CgState *dst = (CgState *)workspace(c, "cg.state", sizeof(CgState));
    CgState *host = (CgState *)pinned(c, 3 * sizeof(CgState));
    if (!b64 || !x64 || !t64 || !q64 || !r || !pp || (fx && !pp2) || !t || !xlo || !partials || !dst || !host)
        return fail(LGT_ERR_OOM, "cannot allocate the solver workspace");

    const bool timing = c->timing > 0;
    const int every = timing ? c->timing : 1; // iterations of a chunk whose Dslash pair is timed: i % every == 0
    const int pairs = 2 * chunk + 2; // event pairs per chunk: 2 Dslash per iteration + 2 in the update
    Events evs, tev, vev;
    LGT_HIP(evs.make(4)); // 0 start, 1 end, 2/3 chunk slots
    if (timing) LGT_HIP(tev.make((size_t)2 * 2 * pairs));
    // the vector kernels of the timed iterations: xpay, (update: inside D_eo), beta step, alpha step
    constexpr int kVec = 4;
    if (timing) LGT_HIP(vev.make((size_t)2 * chunk * kVec * 2));

    // Dslash launch; the reducing epilogues (EPI_PAP, EPI_UPD, EPI_RES*) leave
    // one partial sum per workgroup for the kernel that follows.
    auto D = [&](Fmt f, int epi, int par, const void *U, const void *in, void *out, int gate, const void *aux0,
                 const void *aux1, void *out_lo, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                 void *rw = nullptr, double *parts = nullptr, const double *parts_in = nullptr, int nparts_in = 0,
                 void *pb = nullptr, const void *rin = nullptr, void *xw = nullptr) {
        DslashArgs a;
        a.U = U;
        // the improved operator's Naik field that goes with this fat field
        a.U3 = !U3hi ? nullptr : (U == Uhi->ptr ? U3hi->ptr : U3lo->ptr);
        a.in = in;
        a.out = out;
        a.g = g;
        a.par = par;
        a.gate = gate;
        a.l = f == fhi ? lhi : llo;
        a.aux0 = aux0;
        a.aux1 = aux1;
        a.out_lo = out_lo;
        a.m4 = m4;
        a.partials = parts ? parts : partials;
        a.rw = rw;
        a.pb = pb;
        a.rin = rin;
        a.xw = xw;
        a.parts_in = parts_in;
        a.nparts_in = nparts_in;
        a.st = dst;
        a.hpi = c->hpi[f];
        a.ntl = imp ? c->intl[f] : c->ntl[f];
        return launch_dslash(f, epi, a, s, e0, e1);
    };
    auto F = [&](const double *parts, int fin, int gate, int nparts) {
        return launch_finalize(parts, nparts, dst, fin, gate, s);
    };
    // start / stop events of timed Dslash launch idx of a chunk slot (null: untimed)
    auto ev = [&](int slot, int idx, bool begin) -> hipEvent_t {
        if (!timing || slot < 0) return nullptr;
        return tev.ev[((size_t)slot * pairs + idx) * 2 + (begin ? 0 : 1)];
    };
    // events of vector kernel k of iteration i of a chunk slot (null: untimed)
    auto vv = [&](int slot, int i, int k, bool begin) -> hipEvent_t {
        if (!timing || slot < 0) return nullptr;
        return vev.ev[(((size_t)slot * chunk + i) * kVec + k) * 2 + (begin ? 0 : 1)];
    };
    double vms[kVec] = {0.0, 0.0, 0.0, 0.0};
    int vn = 0;
    VecArgs va;
    va.x = xlo;
    va.r = r;
    va.p = pp;
    va.p2 = pp2;
    va.Vh = Vh;
    va.l = l;
    // partial slots from nblk on belong to idle workgroups (zeros): sum nblk
    // (the iteration's Dslash pair runs in the inner format's launch geometry)
    const bool fuse_alpha = llo.nblk <= fuse_alpha_max();
    va.st = dst;
    va.gate = GATE_ITER;

    const int lo_is_f64 = !mixed;
    // FP64 update step: x64 += x_lo ; r = b - A64 x64 (rounded into r_lo when mixed)
    auto reliable = [&](int gate, int slot, int fin) -> hipError_t {
        hipError_t e = hipSuccess;
        // the last update's x += alpha p, if no p = r + beta p has added it yet
        VecArgs vp = va;
        vp.gate = gate;
        if ((e = launch_x_pending(lo_is_f64, vp, s)) != hipSuccess) return e;
        if (mixed && (e = launch_ru_accum(x64, xlo, Vh, dst, gate, s)) != hipSuccess) return e;
        if ((e = D(fhi, EPI_PLAIN, LGT_ODD, Uhi->ptr, x64, t64, gate, nullptr, nullptr, nullptr,
                   ev(slot, 2 * chunk, true), ev(slot, 2 * chunk, false))) != hipSuccess)
            return e;
        hipEvent_t r0 = ev(slot, 2 * chunk + 1, true), r1 = ev(slot, 2 * chunk + 1, false);
        if (fin == FIN_FINAL)
            e = D(fhi, EPI_RES, LGT_EVEN, Uhi->ptr, t64, q64, gate, x64, b64, nullptr, r0, r1);
        else if (mixed)
            e = D(fhi, EPI_RES_LO, LGT_EVEN, Uhi->ptr, t64, nullptr, gate, x64, b64, r, r0, r1);
        else
            e = D(fhi, EPI_RES, LGT_EVEN, Uhi->ptr, t64, r, gate, x64, b64, nullptr, r0, r1);
        if (e != hipSuccess) return e;
        return F(partials, fin, gate, lhi.nblk);
    };

    LGT_HIP(hipEventRecord(evs.ev[0], s));
    // ---- setup
    LGT_HIP(launch_pack_vec(true, b, b64, g, s));
    if (p->x0_is_guess) LGT_HIP(launch_pack_vec(true, x, x64, g, s));
    else LGT_HIP(launch_zero(x64, v64, s));
    if (mixed) LGT_HIP(launch_zero(xlo, vlo, s));
    LGT_HIP(launch_zero(pp, vlo, s));
    LGT_HIP(launch_state_init(dst, scheme, scheme == SCH_RELIABLE, p->max_iter, p->tol, inner, s));
    LGT_HIP(launch_norm_init(b64, Vh, partials, dst, s));
    LGT_HIP(reliable(GATE_RU, -1, FIN_RU)); // r = b - A x0, rho, beta = 0

    // ---- iterations, `chunk` at a time
    int k = 0;
    int prev_iter = 0, prev_upd = 0;
    double ms_hi = 0.0, ms_lo = 0.0;
    int n_hi = 0, n_lo = 0;
    double dsl_ms[4] = {0.0, 0.0, 0.0, 0.0}; // by kind: iteration D_oe, D_eo; update D_oe, D_eo
    int dsl_n[4] = {0, 0, 0, 0};
    // every chunk that starts running does at least one iteration, and the
    // kernels stop at max_iter, so this bound is never the one that ends the loop
    const int max_chunks = p->max_iter + 4;
    auto harvest = [&](int slot, const CgState &end) -> hipError_t {
        if (!timing) return hipSuccess;
        const int nreal = std::min(end.iter - prev_iter, chunk);
        for (int i = 0; i < nreal; i += every) {
            for (int k = 0; k < kVec; k++) {
                if (k == 1 || (k == 3 && fuse_alpha)) continue; // the update runs inside D_eo
                if (k == 0 && fx) continue;                      // p = r + beta p runs inside D_oe
                float ms = 0.f;
                hipError_t e = hipEventElapsedTime(&ms, vv(slot, i, k, true), vv(slot, i, k, false));
                if (e != hipSuccess) return e;
                vms[k] += ms;
            }
            vn++;
        }
        for (int i = 0; i < 2 * nreal; i++) {
            if ((i / 2) % every != 0) continue;
            float ms = 0.f;
            hipError_t e = hipEventElapsedTime(&ms, tev.ev[((size_t)slot * pairs + i) * 2],
                                               tev.ev[((size_t)slot * pairs + i) * 2 + 1]);
            if (e != hipSuccess) return e;
            if (lo_is_f64) {
                ms_hi += ms;
                n_hi++;
            } else {
                ms_lo += ms;
                n_lo++;
            }
            dsl_ms[i & 1] += ms;
            dsl_n[i & 1]++;
        }
        if (end.updates > prev_upd) {
            for (int i = 2 * chunk; i < 2 * chunk + 2; i++) {
                float ms = 0.f;
                hipError_t e = hipEventElapsedTime(&ms, tev.ev[((size_t)slot * pairs + i) * 2],
                                                   tev.ev[((size_t)slot * pairs + i) * 2 + 1]);
                if (e != hipSuccess) return e;
                ms_hi += ms;
                n_hi++;
                dsl_ms[2 + (i & 1)] += ms;
                dsl_n[2 + (i & 1)]++;
            }
        }
        return hipSuccess;
    };
    bool finished = false;
    while (!finished) {
        const int slot = k & 1;
        for (int i = 0; i < chunk; i++) {
            const int ts = i % every == 0 ? slot : -1;
            const void *Ui = mixed ? Ulo->ptr : Uhi->ptr;
            if (fx) {
                // p' = r + beta p (and the pending x += alpha p) inside D_oe, p' into
                // the other p buffer; t = D_oe p' with the partials of <p', A p'>
                LGT_HIP(D(flo, EPI_PAPX, LGT_ODD, Ui, pp, t, GATE_ITER, nullptr, nullptr, nullptr,
                          ev(ts, 2 * i, true), ev(ts, 2 * i, false), nullptr, nullptr, nullptr, 0, pp2, r, xlo));
            } else {
                LGT_HIP(launch_xpay(lo_is_f64, va, s, vv(ts, i, 0, true), vv(ts, i, 0, false)));
                // t = D_oe p with the partials of <p, A p> = m4 |p|^2 + |t|^2
                LGT_HIP(D(flo, EPI_PAP, LGT_ODD, Ui, pp, t, GATE_ITER, pp, nullptr, nullptr, ev(ts, 2 * i, true),
                          ev(ts, 2 * i, false)));
            }
            if (!fuse_alpha)
                LGT_HIP(launch_finalize(partials, llo.nblk, dst, FIN_ALPHA, GATE_ITER, s, vv(ts, i, 3, true),
                                        vv(ts, i, 3, false)));
            // r -= alpha (m4 p - D_eo t) with the partials of |r|^2 (alpha summed
            // from D_oe's partials in every workgroup when fused)
            LGT_HIP(D(flo, EPI_UPD, LGT_EVEN, Ui, t, nullptr, GATE_ITER, pp, nullptr, nullptr, ev(ts, 2 * i + 1, true),
                      ev(ts, 2 * i + 1, false), r, partials2, fuse_alpha ? partials : nullptr,
                      fuse_alpha ? llo.nblk : 0, pp2));
            LGT_HIP(launch_finalize(partials2, llo.nblk, dst, FIN_UPDATE, GATE_ITER, s, vv(ts, i, 2, true),
                                    vv(ts, i, 2, false)));
        }
        LGT_HIP(reliable(GATE_RU, timing ? slot : -1, FIN_RU));
        LGT_HIP(hipMemcpyAsync(host + slot, dst, sizeof(CgState), hipMemcpyDeviceToHost, s));
        LGT_HIP(hipEventRecord(evs.ev[2 + slot], s));
        if (k > 0) {
            const int ps = (k - 1) & 1;
            LGT_HIP(hipEventSynchronize(evs.ev[2 + ps]));
            const CgState e = host[ps];
            LGT_HIP(harvest(ps, e));
            prev_iter = e.iter;
            prev_upd = e.updates;
            if (e.state == ST_DONE || e.state == ST_FAIL || e.state == ST_MAXIT) finished = true;
        }
        k++;
        if (k > max_chunks) break;
    }
    {
        const int ls = (k - 1) & 1;
        LGT_HIP(hipEventSynchronize(evs.ev[2 + ls]));
        LGT_HIP(harvest(ls, host[ls]));
    }
    // ---- final: accumulate, FP64 true residual, unpack
    LGT_HIP(reliable(GATE_NONE, -1, FIN_FINAL));
    LGT_HIP(launch_unpack_vec(true, x64, x, g, s));
    LGT_HIP(hipMemcpyAsync(host + 2, dst, sizeof(CgState), hipMemcpyDeviceToHost, s));
    LGT_HIP(hipEventRecord(evs.ev[1], s));
    LGT_HIP(hipEventSynchronize(evs.ev[1]));
    const CgState e = host[2];
    float ms = 0.f;
    LGT_HIP(hipEventElapsedTime(&ms, evs.ev[0], evs.ev[1]));

    lgt_cg_result out;
    std::memset(&out, 0, sizeof(out));
    out.iters = e.iter;
    out.updates = e.updates;
    out.dslash_calls = 2 * (e.iter + e.updates + 2);
    out.true_rel_resid = e.bnorm2 > 0.0 ? std::sqrt(e.last_true / e.bnorm2) : 0.0;
    out.seconds = 1e-3 * ms;
    out.dslash_ms_hi = ms_hi;
    out.dslash_ms_lo = ms_lo;
    out.dslash_timed_hi = n_hi;
    out.dslash_timed_lo = n_lo;
    if (timing) {
        for (int k = 0; k < kVec; k++) c->cg_prof_ms[k] = vn ? vms[k] / vn : 0.0;
        c->cg_prof_n = vn;
        for (int k = 0; k < 4; k++) {
            c->cg_dsl_ms[k] = dsl_n[k] ? dsl_ms[k] / dsl_n[k] : 0.0;
            c->cg_dsl_n[k] = dsl_n[k];
        }
    }
    lgt_status ret;
    if (e.state == ST_DONE) ret = LGT_OK;
    else if (e.state == ST_FAIL || !std::isfinite(e.last_true)) ret = LGT_ERR_NONFINITE;
    else ret = LGT_ERR_NOT_CONVERGED;
    out.status = ret;
    if (res) *res = out;
    if (ret == LGT_ERR_NONFINITE) return fail(ret, "CG breakdown or non-finite residual after %d iterations", e.iter);
    if (ret == LGT_ERR_NOT_CONVERGED)
        return fail(ret, "CG not converged: %d iterations, true relative residual %.3e", e.iter, out.true_rel_resid);
    return LGT_OK;
}

} // namespace lgt
