// batch.cpp -- C ABI of the multi-RHS Dslash and of the batched CG (one
// cooperative launch for every right-hand side of every problem).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"

using namespace lgt;

namespace {

int log2_rhs(int32_t n)
{
    for (int l = 0; l <= 4; l++)
        if (n == (1 << l)) return l;
    return -1;
}

// the batched solver pads 1..16 right-hand sides to the next power of two
int log2_rhs_padded(int32_t n)
{
    for (int l = 0; l <= 4; l++)
        if (n >= 1 && n <= (1 << l)) return l;
    return -1;
}

} // namespace

extern "C" {

lgt_status lgt_pack_vec_mrhs(lgt_ctx *c, int32_t prec, int32_t nrhs, const double *src, void *dst)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    const int logN = log2_rhs(nrhs);
    if (logN < 0) return fail(LGT_ERR_ARG, "nrhs must be 1, 2, 4, 8 or 16");
    if (!mrhs_size_ok(c->g.Vh)) return fail(LGT_ERR_UNSUPPORTED, "lattice too large for multi-RHS vectors");
    if (prec != LGT_F64 && prec != LGT_F32 && prec != LGT_BF16) return fail(LGT_ERR_ARG, "bad precision %d", prec);
    lgt_status s;
    if ((s = check_ptr(src, "src")) != LGT_OK) return s;
    if ((s = check_ptr(dst, "dst")) != LGT_OK) return s;
    DeviceScope ds(c->device);
    LGT_HIP(launch_pack_mrhs(prec == LGT_F64, src, dst, c->g, logN, c->stream));
    return LGT_OK;
}

lgt_status lgt_unpack_vec_mrhs(lgt_ctx *c, int32_t prec, int32_t nrhs, const void *src, double *dst)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    const int logN = log2_rhs(nrhs);
    if (logN < 0) return fail(LGT_ERR_ARG, "nrhs must be 1, 2, 4, 8 or 16");
    if (!mrhs_size_ok(c->g.Vh)) return fail(LGT_ERR_UNSUPPORTED, "lattice too large for multi-RHS vectors");
    if (prec != LGT_F64 && prec != LGT_F32 && prec != LGT_BF16) return fail(LGT_ERR_ARG, "bad precision %d", prec);
    lgt_status s;
    if ((s = check_ptr(src, "src")) != LGT_OK) return s;
    if ((s = check_ptr(dst, "dst")) != LGT_OK) return s;
    DeviceScope ds(c->device);
    LGT_HIP(launch_unpack_mrhs(prec == LGT_F64, src, dst, c->g, logN, c->stream));
    return LGT_OK;
}

lgt_status lgt_set_mrhs_engine(lgt_ctx *c, int32_t engine)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    if (engine < LGT_MRHS_LANE || engine > LGT_MRHS_MFMA) return fail(LGT_ERR_ARG, "bad engine %d", engine);
    c->mrhs_engine = engine;
    for (int f = 0; f < FMT_COUNT; f++)
        for (int l = 0; l < 5; l++) {
            c->mrhs_eng[f][l] = engine;
            c->mrhs_gps[f][l] = 1;
        }
    return LGT_OK;
}

lgt_status lgt_set_mrhs_variant(lgt_ctx *c, int32_t prec, int32_t recon, int32_t nrhs, int32_t engine,
                                int32_t groups)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    const int logN = log2_rhs(nrhs);
    if (logN < 0) return fail(LGT_ERR_ARG, "nrhs must be 1, 2, 4, 8 or 16");
    if (engine < LGT_MRHS_LANE || engine > LGT_MRHS_MFMA) return fail(LGT_ERR_ARG, "bad engine %d", engine);
    if (engine != LGT_MRHS_LANE && !mrhs_groups_valid(logN, groups))
        return fail(LGT_ERR_ARG, "groups must be 1, 2 or 4 with 4 * groups <= nrhs");
    c->mrhs_eng[f][logN] = engine;
    c->mrhs_gps[f][logN] = engine == LGT_MRHS_LANE ? 1 : groups;
    return LGT_OK;
}

lgt_status lgt_get_mrhs_variant(lgt_ctx *c, int32_t prec, int32_t recon, int32_t nrhs, int32_t *engine,
                                int32_t *groups)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    if (!engine || !groups) return fail(LGT_ERR_ARG, "output pointer is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    const int logN = log2_rhs(nrhs);
    if (logN < 0) return fail(LGT_ERR_ARG, "nrhs must be 1, 2, 4, 8 or 16");
    // the variant lgt_dslash_mrhs runs on this lattice
    const int e = c->mrhs_eng[f][logN];
    const bool four = mrhs_engine_applies(f, logN, c->g.Vh, e);
    *engine = four ? e : LGT_MRHS_LANE;
    *groups = four && mrhs_groups_valid(logN, c->mrhs_gps[f][logN]) ? c->mrhs_gps[f][logN] : 1;
    return LGT_OK;
}

lgt_status lgt_get_mrhs_engine(lgt_ctx *c, int32_t *engine)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    if (!engine) return fail(LGT_ERR_ARG, "engine is NULL");
    *engine = c->mrhs_engine;
    return LGT_OK;
}

lgt_status lgt_dslash_mrhs(lgt_ctx *c, const lgt_links *U, int32_t out_parity, int32_t nrhs, const void *in,
                           void *out)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    lgt_status s;
    if ((s = check_links(U, false, &f)) != LGT_OK) return s;
    if (out_parity != LGT_EVEN && out_parity != LGT_ODD) return fail(LGT_ERR_ARG, "bad parity %d", out_parity);
    const int logN = log2_rhs(nrhs);
    if (logN < 0) return fail(LGT_ERR_ARG, "nrhs must be 1, 2, 4, 8 or 16");
    if (!mrhs_size_ok(c->g.Vh)) return fail(LGT_ERR_UNSUPPORTED, "lattice too large for multi-RHS vectors");
    if ((s = check_ptr(in, "in")) != LGT_OK) return s;
    if ((s = check_ptr(out, "out")) != LGT_OK) return s;
    if (in == out) return fail(LGT_ERR_ARG, "in and out alias");
    DeviceScope ds(c->device);
    LGT_HIP(launch_dslash_mrhs(f, U->ptr, in, out, c->g, out_parity, logN, c->stream, c->mrhs_eng[f][logN],
                               c->mrhs_gps[f][logN], c->mrhs_stage[f][logN] != 0));
    return LGT_OK;
}

lgt_status lgt_set_mrhs_staging(lgt_ctx *c, int32_t prec, int32_t recon, int32_t nrhs, int32_t staged)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    const int logN = log2_rhs(nrhs);
    if (logN < 0) return fail(LGT_ERR_ARG, "nrhs must be 1, 2, 4, 8 or 16");
    if (staged != 0 && staged != 1) return fail(LGT_ERR_ARG, "staged must be 0 or 1");
    c->mrhs_stage[f][logN] = staged;
    return LGT_OK;
}

lgt_status lgt_get_mrhs_staging(lgt_ctx *c, int32_t prec, int32_t recon, int32_t nrhs, int32_t *staged)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    if (!staged) return fail(LGT_ERR_ARG, "output pointer is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    const int logN = log2_rhs(nrhs);
    if (logN < 0) return fail(LGT_ERR_ARG, "nrhs must be 1, 2, 4, 8 or 16");
    // whether lgt_dslash_mrhs runs the staged kernel on this lattice
    const int e = c->mrhs_eng[f][logN];
    const int gps = mrhs_groups_valid(logN, c->mrhs_gps[f][logN]) ? c->mrhs_gps[f][logN] : 1;
    *staged = c->mrhs_stage[f][logN] && mrhs_engine_applies(f, logN, c->g.Vh, e) && mrhs_staging_fits(c->g, logN, gps);
    return LGT_OK;
}

lgt_status lgt_cg_solve_batch(const lgt_cg_problem *probs, int32_t nprob, const lgt_cg_params *p)
{
    clear_error();
    if (!probs) return fail(LGT_ERR_ARG, "problems is NULL");
    if (nprob < 1 || nprob > kMaxProblems) return fail(LGT_ERR_ARG, "nprob must be in [1, %d]", kMaxProblems);
    if (!p) return fail(LGT_ERR_ARG, "params is NULL");
    if (!(p->mass > 0.0)) return fail(LGT_ERR_ARG, "mass must be > 0");
    if (!(p->tol > 0.0)) return fail(LGT_ERR_ARG, "tol must be > 0");
    if (p->max_iter <= 0) return fail(LGT_ERR_ARG, "max_iter must be > 0");
    if (p->scheme < LGT_CG_FP64 || p->scheme > LGT_CG_REFINE) return fail(LGT_ERR_ARG, "bad scheme %d", p->scheme);
    if (p->scheme == LGT_CG_RELIABLE && p->ru_interval <= 0) return fail(LGT_ERR_ARG, "ru_interval must be > 0");
    if (p->scheme == LGT_CG_REFINE && !(p->inner_tol > 0.0 && p->inner_tol < 1.0))
        return fail(LGT_ERR_ARG, "inner_tol must be in (0, 1) for refinement");
    if (p->scheme != LGT_CG_REFINE && (p->inner_tol < 0.0 || p->inner_tol > 1.0))
        return fail(LGT_ERR_ARG, "inner_tol must be in [0, 1]");
    const bool mixed = p->scheme != LGT_CG_FP64;
    lgt_ctx *c0 = probs[0].ctx;
    if (!c0) return fail(LGT_ERR_ARG, "problem 0 has no context");
    Fmt flo = F64R18;
    int total_rhs = 0;
    for (int i = 0; i < nprob; i++) {
        const lgt_cg_problem &q = probs[i];
        if (!q.ctx) return fail(LGT_ERR_ARG, "problem %d has no context", i);
        if (q.ctx->device != c0->device) return fail(LGT_ERR_ARG, "problem %d is on another device", i);
        const int logN = log2_rhs_padded(q.nrhs);
        if (logN < 0) return fail(LGT_ERR_ARG, "problem %d: nrhs must be in 1..16", i);
        if (!mrhs_size_ok(q.ctx->g.Vh)) return fail(LGT_ERR_UNSUPPORTED, "problem %d: lattice too large", i);
        Fmt fh, fl;
        lgt_status s = check_links(q.U_hi, true, &fh);
        if (s != LGT_OK) return s;
        if (fh != F64R18) return fail(LGT_ERR_UNSUPPORTED, "problem %d: batched solves take F64 x 18 links", i);
        if (mixed) {
            if ((s = check_links(q.U_lo, false, &fl)) != LGT_OK) return s;
            if (fmt_is_f64(fl)) return fail(LGT_ERR_ARG, "problem %d: U_lo must be F32 or BF16 links", i);
            if (i == 0) flo = fl;
            else if (fl != flo) return fail(LGT_ERR_UNSUPPORTED, "every problem must use the same U_lo format");
        }
        if ((s = check_ptr(q.b, "b")) != LGT_OK) return s;
        if ((s = check_ptr(q.x, "x")) != LGT_OK) return s;
        if (!q.res) return fail(LGT_ERR_ARG, "problem %d: res is NULL", i);
        total_rhs += 1 << logN; // padding right-hand sides (zero sources) included
    }
    if (total_rhs > kMaxTotalRhs)
        return fail(LGT_ERR_ARG, "at most %d right-hand sides per batch (each nrhs rounded up to a power of two)",
                    kMaxTotalRhs);
    DeviceScope ds(c0->device);
    const hipStream_t s = c0->stream;

    // Mixed precision with a four-lane inner engine in every problem: the
    // iteration as kernel launches (mcg_host.cpp), each problem on its own
    // context's stream. Its Dslash steps keep more waves in flight than the
    // persistent launch can, and a single problem of any size, or up to
    // kMcgMaxProblems on different contexts (each context's auxiliary stream;
    // HIP's default of four hardware queues), solves faster that way.
    // LGT_BATCH_LAUNCHED = 1 takes that form whenever every problem has a
    // four-lane engine, 0 never.
    if (mixed) {
        int mode = -1;
        if (const char *e = std::getenv("LGT_BATCH_LAUNCHED")) {
            if (!std::strcmp(e, "0")) mode = 0;
            else if (!std::strcmp(e, "1")) mode = 1;
            else if (*e) return fail(LGT_ERR_ARG, "LGT_BATCH_LAUNCHED must be 0 or 1");
        }
        std::vector<McgProblem> mp((size_t)nprob);
        bool four = true, distinct = true;
        for (int i = 0; i < nprob; i++) {
            const lgt_cg_problem &q = probs[i];
            lgt_ctx *c = q.ctx;
            const int logN = log2_rhs_padded(q.nrhs);
            int eng = c->mrhs_eng[flo][logN];
            if (eng == MRHS_MFMA && !mrhs_engine_applies(flo, logN, c->g.Vh, eng)) eng = MRHS_VALU4; // V/2 % 16 != 0
            // groups as in the persistent launch: at N = 16 one group (R = 4)
            // costs the update kernel's occupancy (24^3x48 x16: 450 against
            // 416 us an iteration with 2 groups, VALU), so a request for it runs two
            mp[i] = McgProblem{&q, flo, logN, eng, batch_groups(logN, c->mrhs_gps[flo][logN])};
            four = four && mrhs_engine_applies(flo, logN, c->g.Vh, eng);
            for (int j = 0; j < i; j++) distinct = distinct && probs[j].ctx != c;
        }
        const bool suits = nprob == 1 || (nprob <= kMcgMaxProblems && distinct);
        if (four && (mode == 1 || (mode < 0 && suits))) return mcg_solve(mp.data(), nprob, p);
    }

    // grid: one workgroup per CU, all resident at once (cooperative launch)
    int coop = 0, ncu = 0;
    LGT_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c0->device));
    if (!coop) return fail(LGT_ERR_UNSUPPORTED, "device does not support cooperative launches");
    LGT_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c0->device));
    if (batch_cg_max_blocks_per_cu(mixed ? flo : F64R18) < 1) return fail(LGT_ERR_DEVICE, "cannot size the batched launch");

    BatchArgs *ha = (BatchArgs *)pinned(c0, sizeof(BatchArgs));
    if (!ha) return fail(LGT_ERR_OOM, "cannot allocate pinned staging");
    std::memset(ha, 0, sizeof(BatchArgs));
    int lt = 0, dt = 0, rhs0 = 0;
    size_t split_pairs = 0; // (site, rhs) pairs of all problems
    for (int i = 0; i < nprob; i++) {
        const lgt_cg_problem &q = probs[i];
        lgt_ctx *c = q.ctx;
        const int logN = log2_rhs_padded(q.nrhs);
        const size_t n = (size_t)c->g.Vh << logN;
        const size_t v64 = n * 48, vlo = mixed ? n * 24 : n * 48;
        BatchProb &P = ha->prob[i];
        P.g = c->g;
        P.logN = logN;
        // inner Dslash engine: four-lane groups for F32/BF16 links and N >= 4
        // (the variant this problem's context keeps for the inner format and N)
        P.eng = MRHS_LANE;
        P.gps = 1;
        if (mixed && mrhs_engine_applies(flo, logN, c->g.Vh, c->mrhs_eng[flo][logN])) {
            P.eng = c->mrhs_eng[flo][logN];
            P.gps = batch_groups(logN, c->mrhs_gps[flo][logN]);
        } else if (mixed && c->mrhs_eng[flo][logN] == MRHS_MFMA &&
                   mrhs_engine_applies(flo, logN, c->g.Vh, MRHS_VALU4)) {
            P.eng = MRHS_VALU4; // MFMA needs V/2 % 16 == 0
            P.gps = batch_groups(logN, c->mrhs_gps[flo][logN]);
        }
        // LDS staging of the inner Dslash's x/y neighbourhood (four-lane engines)
        P.stage = P.eng != MRHS_LANE && batch_stage_fits(kBB / (4 * P.gps), c->g.hx, logN);
        P.lt0 = lt;
        P.nlt = (int)((n + kBB - 1) / kBB);
        P.dt0 = dt;
        if (P.eng == MRHS_LANE) P.ndt = P.nlt;
        else {
            const int sites = kBB / (4 * P.gps);
            P.ndt = (c->g.Vh + sites - 1) / sites;
        }
        P.rhs0 = rhs0;
        P.m4 = 4.0 * p->mass * p->mass;
        P.Uhi = q.U_hi->ptr;
        P.Ulo = mixed ? q.U_lo->ptr : q.U_hi->ptr;
        // buffers are named per problem index: one context may serve several problems
        auto ws = [&](const char *what, size_t bytes) {
            char name[48];
            std::snprintf(name, sizeof(name), "batch.%s.%d", what, i);
            return workspace(c, name, bytes);
        };
        P.b64 = (const double *)ws("b64", v64);
        P.x64 = (double *)ws("x64", v64);
        P.t64 = (double *)ws("t64", v64);
        P.r = ws("r", vlo);
        P.pa = ws("pa", vlo);
        P.pb = ws("pb", vlo);
        P.Ap = ws("Ap", vlo);
        P.t = ws("t", vlo);
        P.xlo = mixed ? ws("xlo", vlo) : (void *)P.x64;
        if (!P.b64 || !P.x64 || !P.t64 || !P.r || !P.pa || !P.pb || !P.Ap || !P.t || !P.xlo)
            return fail(LGT_ERR_OOM, "cannot allocate the batch workspace of problem %d", i);
        lt += P.nlt;
        dt += P.ndt;
        rhs0 += 1 << logN;
        split_pairs += n;
    }
    int grid = ncu;
    const int most = lt > dt ? lt : dt;
    if (grid > most) grid = most; // more workgroups than tiles only add barrier arrivals
    if (grid < 1) grid = 1;
    ha->nprob = nprob;
    ha->total_lt = lt;
    ha->total_dt = dt;
    ha->total_rhs = total_rhs;
    ha->scheme = p->scheme;
    ha->ru_interval = p->scheme == LGT_CG_RELIABLE ? p->ru_interval : 1 << 30;
    ha->max_iter = p->max_iter;
    // Step 1 as two passes (p' elementwise, a barrier, then D_oe p' gathering
    // one vector) where the p' pass outweighs the extra barrier: at 24^3x48
    // x16 (5.3M site-rhs pairs) 264 -> 236 us an iteration, while the mixed
    // 8^4/12^4/16^3x32 x4 batch (0.31M) got 13 % slower.
    ha->split = split_pairs >= kBatchSplitPairs;
    ha->tol = p->tol;
    ha->inner = p->scheme == LGT_CG_REFINE ? p->inner_tol : (p->inner_tol > 0 ? p->inner_tol : 1.0);
    // Bound on the polls of one grid-barrier wait: seconds of polling, far
    // beyond any phase of a valid launch. LGT_BATCH_SPIN_LIMIT overrides it (a
    // tiny limit makes the barriers time out: every workgroup then leaves the
    // kernel and the call reports LGT_ERR_DEVICE, which tests of that path use).
    ha->spin_limit = 1u << 21;
    if (const char *e = std::getenv("LGT_BATCH_SPIN_LIMIT")) {
        char *end = nullptr;
        const long v = std::strtol(e, &end, 10);
        if (!end || *end || v < 1 || v > (1L << 30)) return fail(LGT_ERR_ARG, "LGT_BATCH_SPIN_LIMIT must be in [1, 2^30]");
        ha->spin_limit = (unsigned int)v;
    }
    CgState *states = (CgState *)workspace(c0, "batch.states", sizeof(CgState) * (size_t)total_rhs);
    double *rows = (double *)workspace(c0, "batch.rows", 2 * sizeof(double) * (size_t)grid * total_rhs);
    BatchCtl *ctl = (BatchCtl *)workspace(c0, "batch.ctl", sizeof(BatchCtl));
    BatchArgs *da = (BatchArgs *)workspace(c0, "batch.args", sizeof(BatchArgs));
    if (!states || !rows || !ctl || !da) return fail(LGT_ERR_OOM, "cannot allocate the batch control buffers");
    // phase profile of the launch while timing is on for the first problem's context
    unsigned long long *prof = nullptr;
    if (c0->timing > 0) {
        prof = (unsigned long long *)workspace(c0, "batch.prof", sizeof(unsigned long long) * kBatchPhases);
        if (!prof) return fail(LGT_ERR_OOM, "cannot allocate the batch profile");
    }
    ha->prof = prof;
    ha->states = states;
    ha->rows[0] = rows;
    ha->rows[1] = rows + (size_t)grid * total_rhs;
    ha->ctl = ctl;

    hipEvent_t e0, e1;
    LGT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(LGT_ERR_DEVICE, "hipEventCreate failed");
    }
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard()
        {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};

    LGT_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < nprob; i++) {
        const lgt_cg_problem &q = probs[i];
        const BatchProb &P = ha->prob[i];
        const size_t n = (size_t)q.ctx->g.Vh << P.logN;
        const size_t vlo = mixed ? n * 24 : n * 48;
        // right-hand sides q.nrhs..2^logN-1 get zero sources: converged at the start
        LGT_HIP(launch_pack_mrhs(true, q.b, (void *)P.b64, q.ctx->g, P.logN, s, q.nrhs));
        if (p->x0_is_guess) LGT_HIP(launch_pack_mrhs(true, q.x, P.x64, q.ctx->g, P.logN, s, q.nrhs));
        else LGT_HIP(launch_zero(P.x64, n * 48, s));
        if (mixed) LGT_HIP(launch_zero(P.xlo, vlo, s));
        LGT_HIP(launch_zero(P.pa, vlo, s));
        LGT_HIP(launch_zero(P.pb, vlo, s));
    }
    LGT_HIP(launch_zero(ctl, sizeof(BatchCtl), s));
    LGT_HIP(hipMemcpyAsync(da, ha, sizeof(BatchArgs), hipMemcpyHostToDevice, s));
    LGT_HIP(launch_batch_cg(mixed ? flo : F64R18, da, grid, s));
    for (int i = 0; i < nprob; i++) {
        const lgt_cg_problem &q = probs[i];
        LGT_HIP(launch_unpack_mrhs(true, ha->prob[i].x64, q.x, q.ctx->g, ha->prob[i].logN, s, q.nrhs));
    }
    LGT_HIP(hipEventRecord(e1, s));
    std::vector<CgState> st((size_t)total_rhs);
    LGT_HIP(hipMemcpyAsync(st.data(), states, sizeof(CgState) * (size_t)total_rhs, hipMemcpyDeviceToHost, s));
    BatchCtl hc;
    LGT_HIP(hipMemcpyAsync(&hc, ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, s));
    unsigned long long hp[kBatchPhases] = {};
    if (prof) LGT_HIP(hipMemcpyAsync(hp, prof, sizeof(hp), hipMemcpyDeviceToHost, s));
    LGT_HIP(hipStreamSynchronize(s));
    if (prof) {
        // ticks of the constant 100 MHz clock -> milliseconds
        for (int k = 0; k < kBatchPhases; k++) c0->batch_prof_ms[k] = 1e-5 * (double)hp[k];
        c0->batch_prof_iters = (int)hc.iters_done;
    }
    float ms = 0.f;
    LGT_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (hc.err) return fail(LGT_ERR_DEVICE, "batched CG: a grid barrier timed out");

    lgt_status ret = LGT_OK;
    for (int i = 0; i < nprob; i++) {
        for (int j = 0; j < probs[i].nrhs; j++) {
            const CgState &e = st[(size_t)ha->prob[i].rhs0 + j];
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
            probs[i].res[j] = r;
            if (r.status != LGT_OK && ret == LGT_OK) ret = r.status;
        }
    }
    if (ret != LGT_OK) return fail(ret, "batched CG: at least one right-hand side did not converge");
    return LGT_OK;
}

lgt_status lgt_batch_profile(lgt_ctx *c, double ms[9], int32_t *iters)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    if (!ms || !iters) return fail(LGT_ERR_ARG, "output pointer is NULL");
    for (int k = 0; k < kBatchPhases; k++) ms[k] = c->batch_prof_ms[k];
    *iters = c->batch_prof_iters;
    return LGT_OK;
}

} // extern "C"
