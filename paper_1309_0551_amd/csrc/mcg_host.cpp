// mcg_host.cpp -- host driver of the batched CG as kernel launches (kernels
// in mcg.hip): the form lgt_cg_solve_batch takes for a few mixed-precision
// problems that all run a four-lane inner engine.
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
//
// A single problem runs on its context's stream. Several problems run each on
// its context's auxiliary stream, after the work already queued on the
// context's own stream and on the first problem's, so the launches of
// different problems overlap on the GPU (problems that share a context share
// its auxiliary stream and run one after the other); at the end each
// context's stream waits for its problems, and the batch's time is taken on
// the first problem's stream. (Auxiliary streams only where they serve
// overlap: HIP maps streams onto four hardware queues by default, and
// streams beyond that share queues and serialise.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
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

constexpr int kK = 5; // launches of an iteration: xpay, D_oe, alpha, D_eo, beta

// One problem of the batch: its launch arguments, stream, partial counts,
// state read-back slots and events.
struct Run {
    const lgt_cg_problem *q = nullptr;
    Fmt flo = F32R12;
    hipStream_t s = nullptr;  // the problem's work: the context's stream, or its auxiliary one
    hipStream_t cs = nullptr; // the context's stream
    McgArgs a;
    int N = 0, nit = 0, nlane = 0, nxp = 0;
    size_t n = 0;
    CgState *host = nullptr; // pinned: slots 0 and 1 (chunks), 2 (final), N states each
    EventPool evs;           // 0 set-up end, 1/2 chunk slots, 3 final start, 4 end, 5 inputs ready
    EventPool tev;           // timing: per slot, kK per iteration + the FP64 step
    hipGraphExec_t chunk = nullptr; // one chunk's launches, captured (timing off)
    bool done = false;
    int enq = 0;             // chunks enqueued
    ~Run()
    {
        // an error return may leave launches of this problem queued: let them
        // finish before its graph and events go
        if (s) (void)hipStreamSynchronize(s);
        if (chunk) (void)hipGraphExecDestroy(chunk);
    }
};

} // namespace

lgt_status mcg_solve(const McgProblem *mp, int nprob, const lgt_cg_params *p)
{
    lgt_ctx *c0 = mp[0].q->ctx;
    const hipStream_t s0 = c0->stream;
    const int scheme = p->scheme;
    const int chunk = scheme == SCH_RELIABLE ? p->ru_interval : (p->check_interval > 0 ? p->check_interval : 10);
    const double inner = scheme == SCH_REFINE ? p->inner_tol : (p->inner_tol > 0 ? p->inner_tol : 1.0);
    const bool timing = c0->timing > 0;
    const int per_slot = chunk * kK + 1;

    int total_n = 0;
    for (int i = 0; i < nprob; i++) total_n += 1 << mp[i].logN;
    CgState *host = (CgState *)pinned(c0, 3 * sizeof(CgState) * (size_t)total_n);
    if (!host) return fail(LGT_ERR_OOM, "cannot allocate pinned staging");

    std::vector<std::unique_ptr<Run>> runs;
    int off = 0;
    for (int i = 0; i < nprob; i++) {
        const McgProblem &m = mp[i];
        auto run = std::make_unique<Run>();
        Run &R = *run;
        lgt_ctx *c = m.q->ctx;
        const Geom g = c->g;
        R.q = m.q;
        R.flo = m.flo;
        if (nprob > 1 && !c->aux && hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) {
            c->aux = nullptr;
            return fail(LGT_ERR_DEVICE, "cannot create the auxiliary stream of problem %d", i);
        }
        R.s = nprob > 1 ? c->aux : c->stream;
        R.cs = c->stream;
        R.N = 1 << m.logN;
        R.n = (size_t)g.Vh << m.logN;
        R.nit = mcg_iter_parts(g, m.gps, false);
        R.nlane = mcg_lane_blocks(g, m.logN);
        R.nxp = mcg_xpay_blocks(g, m.logN);
        R.host = host + (size_t)3 * off;
        off += R.N;
        McgArgs &a = R.a;
        std::memset(&a, 0, sizeof(a));
        a.g = g;
        a.logN = m.logN;
        a.engine = m.engine;
        a.gps = m.gps;
        a.m4 = 4.0 * p->mass * p->mass;
        a.Ulo = m.q->U_lo->ptr;
        a.Uhi = m.q->U_hi->ptr;
        a.stride = (size_t)std::max(mcg_iter_parts(g, m.gps, true), (R.nlane + 7) / 8 * 8);
        a.stride_p = (size_t)R.nxp;
        // named per problem index: one context may serve several problems
        auto ws = [&](const char *what, size_t bytes) {
            char name[48];
            std::snprintf(name, sizeof(name), "mcg.%s.%d", what, i);
            return workspace(c, name, bytes);
        };
        a.b64 = (const double *)ws("b64", R.n * 48);
        a.x64 = (double *)ws("x64", R.n * 48);
        a.t64 = (double *)ws("t64", R.n * 48);
        a.xlo = ws("xlo", R.n * 24);
        a.r = ws("r", R.n * 24);
        a.p = ws("p", R.n * 24);
        a.t = ws("t", R.n * 24);
        a.st = (CgState *)ws("states", sizeof(CgState) * R.N);
        a.parts = (double *)ws("parts", sizeof(double) * a.stride * R.N);
        a.parts_p = (double *)ws("parts_p", sizeof(double) * a.stride_p * R.N);
        if (!a.b64 || !a.x64 || !a.t64 || !a.xlo || !a.r || !a.p || !a.t || !a.st || !a.parts || !a.parts_p)
            return fail(LGT_ERR_OOM, "cannot allocate the batch workspace of problem %d", i);
        LGT_HIP(R.evs.make(6));
        if (timing) LGT_HIP(R.tev.make((size_t)2 * per_slot * 2));
        runs.push_back(std::move(run));
    }

    // phase times summed over the problems' own kernels (they overlap in time)
    double ph[kBatchPhases] = {};
    auto span = [](hipEvent_t e0, hipEvent_t e1, double &acc) -> hipError_t {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) acc += ms;
        return e;
    };
    auto ev = [&](Run &R, int slot, int idx, bool begin) -> hipEvent_t {
        if (!timing) return nullptr;
        return R.tev.ev[((size_t)slot * per_slot + idx) * 2 + (begin ? 0 : 1)];
    };
    auto harvest = [&](Run &R, int slot) -> hipError_t {
        if (!timing) return hipSuccess;
        static const int kPhase[kK] = {PH_STEP1P, PH_STEP1, PH_SCALAR, PH_STEP2, PH_SCALAR};
        hipError_t e;
        for (int i = 0; i < chunk; i++)
            for (int k = 0; k < kK; k++)
                if ((e = span(ev(R, slot, i * kK + k, true), ev(R, slot, i * kK + k, false), ph[kPhase[k]])) !=
                    hipSuccess)
                    return e;
        return span(ev(R, slot, chunk * kK, true), ev(R, slot, chunk * kK, false), ph[PH_FP64]);
    };

    // one chunk: `chunk` iterations and the FP64 step for the right-hand
    // sides that ask for one (events only with timing on)
    auto enqueue_chunk = [&](Run &R, int slot) -> hipError_t {
        McgArgs &a = R.a;
        hipError_t e;
        for (int i = 0; i < chunk; i++) {
            const int b = i * kK;
            if ((e = launch_mcg_xpay(a, R.s, ev(R, slot, b, true), ev(R, slot, b, false))) != hipSuccess) return e;
            if ((e = launch_mcg_dslash(R.flo, a, 0, R.s, ev(R, slot, b + 1, true), ev(R, slot, b + 1, false))) !=
                hipSuccess)
                return e;
            if ((e = launch_mcg_fin(a, R.nit, FIN_ALPHA, GATE_ITER, R.s, ev(R, slot, b + 2, true),
                                    ev(R, slot, b + 2, false), R.nxp)) != hipSuccess)
                return e;
            if ((e = launch_mcg_dslash(R.flo, a, 1, R.s, ev(R, slot, b + 3, true), ev(R, slot, b + 3, false))) !=
                hipSuccess)
                return e;
            if ((e = launch_mcg_fin(a, R.nit, FIN_UPDATE, GATE_ITER, R.s, ev(R, slot, b + 4, true),
                                    ev(R, slot, b + 4, false))) != hipSuccess)
                return e;
        }
        if ((e = launch_mcg_fp64(a, GATE_RU, R.s, ev(R, slot, chunk * kK, true))) != hipSuccess) return e;
        return launch_mcg_fin(a, R.nlane, FIN_RU, GATE_RU, R.s, nullptr, ev(R, slot, chunk * kK, false));
    };
    EventPool top;
    LGT_HIP(top.make(2)); // 0 start, 1 end
    LGT_HIP(hipEventRecord(top.ev[0], s0));
    // ---- set-up: right-hand sides nrhs..N-1 get zero sources (converged at once)
    for (auto &run : runs) {
        Run &R = *run;
        McgArgs &a = R.a;
        const Geom &g = a.g;
        // after what the caller queued on the first problem's stream and on
        // this problem's context stream (b and x are read there)
        if (R.s != s0) LGT_HIP(hipStreamWaitEvent(R.s, top.ev[0], 0));
        if (R.cs != s0 && R.cs != R.s) {
            LGT_HIP(hipEventRecord(R.evs.ev[5], R.cs));
            LGT_HIP(hipStreamWaitEvent(R.s, R.evs.ev[5], 0));
        }
        LGT_HIP(launch_pack_mrhs(true, R.q->b, (void *)a.b64, g, a.logN, R.s, R.q->nrhs));
        if (p->x0_is_guess) LGT_HIP(launch_pack_mrhs(true, R.q->x, a.x64, g, a.logN, R.s, R.q->nrhs));
        else LGT_HIP(launch_zero(a.x64, R.n * 48, R.s));
        LGT_HIP(launch_zero(a.xlo, R.n * 24, R.s));
        LGT_HIP(launch_zero(a.p, R.n * 24, R.s));
        LGT_HIP(launch_mcg_init(a, scheme, scheme == SCH_RELIABLE, p->max_iter, p->tol, inner, R.s));
        LGT_HIP(launch_mcg_norm(a, R.s));
        LGT_HIP(launch_mcg_fin(a, R.nlane, FIN_INIT, GATE_NONE, R.s));
        LGT_HIP(launch_mcg_fp64(a, GATE_RU, R.s)); // r = b - A x0, rho, beta = 0
        LGT_HIP(launch_mcg_fin(a, R.nlane, FIN_RU, GATE_RU, R.s));
        LGT_HIP(hipEventRecord(R.evs.ev[0], R.s));
    }

    // Without timing, each problem's chunk is captured once into a graph (while
    // the GPU runs the set-up; the time counts in the batch's) and
    // replayed: one launch call per chunk instead of 5 per iteration, which
    // left the host issuing launches as fast as small lattices ran them. The
    // chunk holds kernels only (no memset nodes); its arguments never change
    // within a solve, the kernels read their gates from the device states.
    if (!timing) {
        // captured on a stream of its own (the context's stream may be the
        // null stream, which cannot be captured), replayed on the problem's
        struct CaptureStream {
            hipStream_t s = nullptr;
            ~CaptureStream()
            {
                if (s) (void)hipStreamDestroy(s);
            }
        } cap;
        LGT_HIP(hipStreamCreateWithFlags(&cap.s, hipStreamNonBlocking));
        for (auto &run : runs) {
            Run &R = *run;
            hipGraph_t gr = nullptr;
            const hipStream_t exec = R.s;
            R.s = cap.s; // enqueue_chunk launches on R.s
            LGT_HIP(hipStreamBeginCapture(R.s, hipStreamCaptureModeThreadLocal));
            const hipError_t e = enqueue_chunk(R, 0);
            const hipError_t e2 = hipStreamEndCapture(R.s, &gr);
            R.s = exec;
            if (e != hipSuccess || e2 != hipSuccess) {
                if (gr) (void)hipGraphDestroy(gr);
                return fail(LGT_ERR_DEVICE, "capturing the batched CG chunk failed: %s",
                            hipGetErrorString(e != hipSuccess ? e : e2));
            }
            const hipError_t e3 = hipGraphInstantiate(&R.chunk, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (e3 != hipSuccess) {
                R.chunk = nullptr;
                return fail(LGT_ERR_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
            }
        }
    }

    // ---- iterations, `chunk` at a time per problem, problems interleaved
    // A right-hand side that still runs at the start of a chunk does at least
    // one iteration in it, and the kernels stop it at max_iter.
    const int max_chunks = p->max_iter + 4;
    for (;;) {
        bool any = false;
        for (auto &run : runs) {
            Run &R = *run;
            if (R.done) continue;
            if (R.enq > max_chunks) { // not reached: see above
                R.done = true;
                continue;
            }
            const int slot = R.enq & 1;
            McgArgs &a = R.a;
            if (R.chunk) LGT_HIP(hipGraphLaunch(R.chunk, R.s));
            else LGT_HIP(enqueue_chunk(R, slot));
            LGT_HIP(hipMemcpyAsync(R.host + (size_t)slot * R.N, a.st, sizeof(CgState) * R.N, hipMemcpyDeviceToHost,
                                   R.s));
            LGT_HIP(hipEventRecord(R.evs.ev[1 + slot], R.s));
            R.enq++;
            any = true;
        }
        if (!any) break;
        // the previous chunk of every problem still running: finished?
        for (auto &run : runs) {
            Run &R = *run;
            if (R.done || R.enq < 2) continue;
            const int ps = (R.enq - 2) & 1;
            LGT_HIP(hipEventSynchronize(R.evs.ev[1 + ps]));
            LGT_HIP(harvest(R, ps));
            bool fin = true;
            for (int j = 0; j < R.N; j++) fin = fin && terminal(R.host[(size_t)ps * R.N + j].state);
            if (fin) R.done = true;
        }
    }
    for (auto &run : runs) {
        Run &R = *run;
        if (R.enq == 0) continue;
        const int ls = (R.enq - 1) & 1;
        LGT_HIP(hipEventSynchronize(R.evs.ev[1 + ls]));
        LGT_HIP(harvest(R, ls));
    }
    // ---- final: x64 += x_lo and the FP64 true residual of every right-hand side
    for (auto &run : runs) {
        Run &R = *run;
        McgArgs &a = R.a;
        LGT_HIP(hipEventRecord(R.evs.ev[3], R.s));
        LGT_HIP(launch_mcg_fp64(a, GATE_NONE, R.s));
        LGT_HIP(launch_mcg_fin(a, R.nlane, FIN_FINAL, GATE_NONE, R.s));
        LGT_HIP(launch_unpack_mrhs(true, a.x64, R.q->x, a.g, a.logN, R.s, R.q->nrhs));
        LGT_HIP(hipMemcpyAsync(R.host + (size_t)2 * R.N, a.st, sizeof(CgState) * R.N, hipMemcpyDeviceToHost, R.s));
        LGT_HIP(hipEventRecord(R.evs.ev[4], R.s));
        if (R.s != s0) LGT_HIP(hipStreamWaitEvent(s0, R.evs.ev[4], 0));
        if (R.cs != s0 && R.cs != R.s) LGT_HIP(hipStreamWaitEvent(R.cs, R.evs.ev[4], 0));
    }
    LGT_HIP(hipEventRecord(top.ev[1], s0));
    LGT_HIP(hipEventSynchronize(top.ev[1]));
    for (auto &run : runs) LGT_HIP(hipEventSynchronize(run->evs.ev[4]));
    float ms = 0.f;
    LGT_HIP(hipEventElapsedTime(&ms, top.ev[0], top.ev[1]));
    if (timing) {
        int its = 0;
        for (auto &run : runs) {
            Run &R = *run;
            LGT_HIP(span(top.ev[0], R.evs.ev[0], ph[PH_SETUP]));
            LGT_HIP(span(R.evs.ev[3], R.evs.ev[4], ph[PH_SETUP]));
            for (int j = 0; j < R.N; j++) its = std::max(its, R.host[(size_t)2 * R.N + j].iter);
        }
        for (int j = 0; j < kBatchPhases; j++) c0->batch_prof_ms[j] = ph[j];
        c0->batch_prof_iters = its;
    }

    lgt_status ret = LGT_OK;
    for (auto &run : runs) {
        Run &R = *run;
        for (int j = 0; j < R.q->nrhs; j++) {
            const CgState &e = R.host[(size_t)2 * R.N + j];
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
            R.q->res[j] = r;
            if (r.status != LGT_OK && ret == LGT_OK) ret = r.status;
        }
    }
    if (ret != LGT_OK) return fail(ret, "batched CG: at least one right-hand side did not converge");
    return LGT_OK;
}

} // namespace lgt
