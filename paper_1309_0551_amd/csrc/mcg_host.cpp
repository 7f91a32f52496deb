// mcg_host.cpp -- host driver of the batched CG of one lattice as kernel launches
// (kernels in mcg.hip): the form lgt_cg_solve_batch takes for one large
// mixed-precision problem.
//
// Per iteration five launches (p = r + beta p with the partials of
// 4m^2 |p|^2; t = D_oe p with those of |t|^2; alpha; D_eo t with the update
// of x and r and the |r|^2 partials; beta and the stop tests), every
// right-hand side with its own scalars and its own gate. Iterations are
// enqueued in chunks of ru_interval (reliable updates) or check_interval
// (refinement; 10 when 0) iterations, each chunk ending with the FP64 step
// for the right-hand sides that ask for one; the host reads the states back
// once per chunk, one chunk behind, so the GPU never waits for the host. A
// right-hand side that meets its inner stop test inside a chunk idles (its
// kernels skip it) until the FP64 step at the end of the chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"

namespace lgt {

namespace {

struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool()
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

bool terminal(int s) { return s == ST_DONE || s == ST_FAIL || s == ST_MAXIT; }

} // namespace

lgt_status mcg_solve(const lgt_cg_problem &q, const lgt_cg_params *p, Fmt flo, int logN, int engine, int gps)
{
    lgt_ctx *c = q.ctx;
    const Geom g = c->g;
    const hipStream_t s = c->stream;
    const int N = 1 << logN;
    const size_t n = (size_t)g.Vh << logN;
    const int scheme = p->scheme;
    const int chunk = scheme == SCH_RELIABLE ? p->ru_interval : (p->check_interval > 0 ? p->check_interval : 10);
    const double inner = scheme == SCH_REFINE ? p->inner_tol : (p->inner_tol > 0 ? p->inner_tol : 1.0);
    const int nit = mcg_iter_parts(g, gps, false), nlane = mcg_lane_blocks(g, logN);
    const int nxp = mcg_xpay_blocks(g, logN);
    const size_t stride = (size_t)std::max(mcg_iter_parts(g, gps, true), (nlane + 7) / 8 * 8);

    McgArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = g;
    a.logN = logN;
    a.engine = engine;
    a.gps = gps;
    a.m4 = 4.0 * p->mass * p->mass;
    a.Ulo = q.U_lo->ptr;
    a.Uhi = q.U_hi->ptr;
    a.stride = stride;
    double *b64 = (double *)workspace(c, "mcg.b64", n * 48);
    a.x64 = (double *)workspace(c, "mcg.x64", n * 48);
    a.t64 = (double *)workspace(c, "mcg.t64", n * 48);
    a.xlo = workspace(c, "mcg.xlo", n * 24);
    a.r = workspace(c, "mcg.r", n * 24);
    a.p = workspace(c, "mcg.p", n * 24);
    a.t = workspace(c, "mcg.t", n * 24);
    a.st = (CgState *)workspace(c, "mcg.states", sizeof(CgState) * N);
    a.parts = (double *)workspace(c, "mcg.parts", sizeof(double) * stride * N);
    a.stride_p = (size_t)nxp;
    a.parts_p = (double *)workspace(c, "mcg.parts_p", sizeof(double) * a.stride_p * N);
    a.b64 = b64;
    CgState *host = (CgState *)pinned(c, 3 * sizeof(CgState) * N);
    if (!b64 || !a.x64 || !a.t64 || !a.xlo || !a.r || !a.p || !a.t || !a.st || !a.parts || !a.parts_p || !host)
        return fail(LGT_ERR_OOM, "cannot allocate the batch workspace");

    // phase events when timing is on: per iteration of a chunk slot xpay,
    // D_oe, alpha, D_eo, beta; per slot the FP64 step with its scalar step;
    // set-up and final step
    const bool timing = c->timing > 0;
    constexpr int kK = 5;
    const int per_slot = chunk * kK + 1;
    EventPool evs, tev;
    LGT_HIP(evs.make(8)); // 0 start, 1 end of set-up, 2/3 chunk slots, 4 start of final, 5 end
    if (timing) LGT_HIP(tev.make((size_t)2 * per_slot * 2));
    auto ev = [&](int slot, int idx, bool begin) -> hipEvent_t {
        if (!timing) return nullptr;
        return tev.ev[((size_t)slot * per_slot + idx) * 2 + (begin ? 0 : 1)];
    };
    double ph[kBatchPhases] = {};
    auto span = [&](hipEvent_t e0, hipEvent_t e1, double &acc) -> hipError_t {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) acc += ms;
        return e;
    };
    auto harvest = [&](int slot) -> hipError_t {
        if (!timing) return hipSuccess;
        static const int kPhase[kK] = {PH_STEP1P, PH_STEP1, PH_SCALAR, PH_STEP2, PH_SCALAR};
        hipError_t e;
        for (int i = 0; i < chunk; i++)
            for (int k = 0; k < kK; k++)
                if ((e = span(ev(slot, i * kK + k, true), ev(slot, i * kK + k, false), ph[kPhase[k]])) != hipSuccess)
                    return e;
        return span(ev(slot, chunk * kK, true), ev(slot, chunk * kK, false), ph[PH_FP64]);
    };

    LGT_HIP(hipEventRecord(evs.ev[0], s));
    // ---- set-up: right-hand sides q.nrhs..N-1 get zero sources (converged at once)
    LGT_HIP(launch_pack_mrhs(true, q.b, b64, g, logN, s, q.nrhs));
    if (p->x0_is_guess) LGT_HIP(launch_pack_mrhs(true, q.x, a.x64, g, logN, s, q.nrhs));
    else LGT_HIP(launch_zero(a.x64, n * 48, s));
    LGT_HIP(launch_zero(a.xlo, n * 24, s));
    LGT_HIP(launch_zero(a.p, n * 24, s));
    LGT_HIP(launch_mcg_init(a, scheme, scheme == SCH_RELIABLE, p->max_iter, p->tol, inner, s));
    LGT_HIP(launch_mcg_norm(a, s));
    LGT_HIP(launch_mcg_fin(a, nlane, FIN_INIT, GATE_NONE, s));
    LGT_HIP(launch_mcg_fp64(a, GATE_RU, s)); // r = b - A x0, rho, beta = 0
    LGT_HIP(launch_mcg_fin(a, nlane, FIN_RU, GATE_RU, s));
    LGT_HIP(hipEventRecord(evs.ev[1], s));

    // ---- iterations, `chunk` at a time
    int k = 0;
    bool finished = false;
    // a right-hand side that still runs at the start of a chunk does at least
    // one iteration in it, and the kernels stop it at max_iter
    const int max_chunks = p->max_iter + 4;
    while (!finished) {
        const int slot = k & 1;
        for (int i = 0; i < chunk; i++) {
            const int b = i * kK;
            LGT_HIP(launch_mcg_xpay(a, s, ev(slot, b, true), ev(slot, b, false)));
            LGT_HIP(launch_mcg_dslash(flo, a, 0, s, ev(slot, b + 1, true), ev(slot, b + 1, false)));
            LGT_HIP(launch_mcg_fin(a, nit, FIN_ALPHA, GATE_ITER, s, ev(slot, b + 2, true), ev(slot, b + 2, false),
                                   nxp));
            LGT_HIP(launch_mcg_dslash(flo, a, 1, s, ev(slot, b + 3, true), ev(slot, b + 3, false)));
            LGT_HIP(launch_mcg_fin(a, nit, FIN_UPDATE, GATE_ITER, s, ev(slot, b + 4, true), ev(slot, b + 4, false)));
        }
        LGT_HIP(launch_mcg_fp64(a, GATE_RU, s, ev(slot, chunk * kK, true)));
        LGT_HIP(launch_mcg_fin(a, nlane, FIN_RU, GATE_RU, s, nullptr, ev(slot, chunk * kK, false)));
        LGT_HIP(hipMemcpyAsync(host + (size_t)slot * N, a.st, sizeof(CgState) * N, hipMemcpyDeviceToHost, s));
        LGT_HIP(hipEventRecord(evs.ev[2 + slot], s));
        if (k > 0) {
            const int ps = (k - 1) & 1;
            LGT_HIP(hipEventSynchronize(evs.ev[2 + ps]));
            LGT_HIP(harvest(ps));
            finished = true;
            for (int j = 0; j < N; j++) finished = finished && terminal(host[(size_t)ps * N + j].state);
        }
        k++;
        if (k > max_chunks) break;
    }
    {
        const int ls = (k - 1) & 1;
        LGT_HIP(hipEventSynchronize(evs.ev[2 + ls]));
        LGT_HIP(harvest(ls));
    }
    // ---- final: x64 += x_lo and the FP64 true residual of every right-hand side
    LGT_HIP(hipEventRecord(evs.ev[4], s));
    LGT_HIP(launch_mcg_fp64(a, GATE_NONE, s));
    LGT_HIP(launch_mcg_fin(a, nlane, FIN_FINAL, GATE_NONE, s));
    LGT_HIP(launch_unpack_mrhs(true, a.x64, q.x, g, logN, s, q.nrhs));
    LGT_HIP(hipMemcpyAsync(host + (size_t)2 * N, a.st, sizeof(CgState) * N, hipMemcpyDeviceToHost, s));
    LGT_HIP(hipEventRecord(evs.ev[5], s));
    LGT_HIP(hipEventSynchronize(evs.ev[5]));
    float ms = 0.f;
    LGT_HIP(hipEventElapsedTime(&ms, evs.ev[0], evs.ev[5]));
    const CgState *fin = host + (size_t)2 * N;
    if (timing) {
        double setup = 0.0;
        LGT_HIP(span(evs.ev[0], evs.ev[1], setup));
        LGT_HIP(span(evs.ev[4], evs.ev[5], setup));
        ph[PH_SETUP] = setup;
        int its = 0;
        for (int j = 0; j < N; j++) its = std::max(its, fin[j].iter);
        for (int j = 0; j < kBatchPhases; j++) c->batch_prof_ms[j] = ph[j];
        c->batch_prof_iters = its;
    }

    lgt_status ret = LGT_OK;
    for (int j = 0; j < q.nrhs; j++) {
        const CgState &e = fin[j];
        lgt_cg_result r;
        std::memset(&r, 0, sizeof(r));
        r.iters = e.iter;
        r.updates = e.updates;
        r.dslash_calls = 2 * (e.iter + e.updates + 2);
        r.true_rel_resid = e.bnorm2 > 0.0 ? std::sqrt(e.last_true / e.bnorm2) : 0.0;
        r.seconds = 1e-3 * ms;
        if (e.state == ST_DONE) r.status = LGT_OK;
        else if (e.state == ST_FAIL || !std::isfinite(e.last_true)) r.status = LGT_ERR_NONFINITE;
        else r.status = LGT_ERR_NOT_CONVERGED;
        q.res[j] = r;
        if (r.status != LGT_OK && ret == LGT_OK) ret = r.status;
    }
    if (ret != LGT_OK) return fail(ret, "batched CG: at least one right-hand side did not converge");
    return LGT_OK;
}

} // namespace lgt
