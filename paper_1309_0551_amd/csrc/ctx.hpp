// ctx.hpp -- the library context: geometry, device, stream and workspace.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <map>
#include <string>

#include "../../include/lgt.h"
#include "kernels.hpp"

struct lgt_ctx {
    lgt_geom geom;
    lgt::Geom g;
    int device = 0;
    hipStream_t stream = nullptr;
    int timing = 0; // Dslash timing inside CG: every n-th iteration (0 = off)
    // Dslash variant per link format: hops whose loads are issued together
    // (8 = fully unrolled, 2 = one direction per loop trip, 1 = one hop).
    // and whether link loads stream past the caches (1) or are cached (0).
    // Set by lgt_set_dslash_variant or lgt_tune_dslash.
    // Defaults measured on MI355X: FP64 fields (604 / 403 MB at 32^4) stream;
    // FP32 and BF16 fields are cached while they (mostly) fit in the 256 MB
    // Infinity Cache (32^4 12-real: FP32x12 42 -> 34 us, BF16x12 25 -> 20 us)
    // and stream beyond 384 MB (lgt_create sets ntl from the field size).
    int hpi[lgt::FMT_COUNT] = {2, 2, 8, 8, 8};
    int ntl[lgt::FMT_COUNT] = {1, 1, 0, 0, 0};
    // Dslash workgroup size per link format (64, 128 or 256 sites): small
    // lattices have too few 256-site workgroups to reach every CU
    int dbs[lgt::FMT_COUNT] = {256, 256, 256, 256, 256};
    // the improved operator's Dslash (fat + Naik fields, 18-real formats):
    // workgroup size and streaming link loads per format, kept apart from the
    // one-link choices above (twice the link traffic, 16 neighbours). Set by
    // lgt_set_dslash_improved_variant or lgt_tune_dslash_improved; lgt_create
    // streams when the two fields exceed the Infinity Cache by half.
    int ibs[lgt::FMT_COUNT] = {256, 256, 256, 256, 256};
    int intl[lgt::FMT_COUNT] = {0, 0, 0, 0, 0};
    // multi-RHS Dslash: engine (0 lane per RHS, 1 four-lane VALU, 2 four-lane
    // MFMA) last set for all cases, and the variant per (link format, log2 N):
    // engine and groups of four lanes per site. Set by lgt_set_mrhs_engine,
    // lgt_set_mrhs_variant or lgt_tune_dslash_mrhs.
    int mrhs_engine = 2;
    int mrhs_eng[lgt::FMT_COUNT][5] = {{2, 2, 2, 2, 2}, {2, 2, 2, 2, 2}, {2, 2, 2, 2, 2}, {2, 2, 2, 2, 2},
                                       {2, 2, 2, 2, 2}};
    int mrhs_gps[lgt::FMT_COUNT][5] = {{1, 1, 1, 1, 1}, {1, 1, 1, 1, 1}, {1, 1, 1, 1, 1}, {1, 1, 1, 1, 1},
                                       {1, 1, 1, 1, 1}};
    // standalone multi-RHS Dslash: 1 = the four-lane engines' LDS-staged
    // variant, per (link format, log2 N); lgt_set_mrhs_staging or the tuner
    int mrhs_stage[lgt::FMT_COUNT][5] = {};
    struct Buf {
        void *ptr = nullptr;
        size_t bytes = 0;
    };
    std::map<std::string, Buf> ws; // named device workspace, grown on demand
    void *pinned = nullptr;        // host pinned staging for state read-back
    size_t pinned_bytes = 0;
    // the batched CG's launched form runs each problem on its context's own
    // auxiliary stream (default priority, created on first use), ordered
    // against `stream` by events, so that problems overlap even when every
    // context was given the same stream
    hipStream_t aux = nullptr;
    // phase profile of the last batched solve launched from this context with
    // timing on (lgt_batch_profile), ms per phase and iterations
    double batch_prof_ms[9] = {};
    int batch_prof_iters = 0;
    // mean kernel times (ms) of the vector kernels of the timed iterations of
    // the last lgt_cg_solve* with timing on: xpay, update, beta step, alpha
    // step (0 when fused into the update), and the number of those iterations
    double cg_prof_ms[4] = {};
    int cg_prof_n = 0;
    // mean kernel times (ms) of the timed Dslash launches of that solve by
    // kind: iteration D_oe (with the <p, A p> partials), iteration D_eo (with
    // the update of r), FP64-update D_oe, FP64-update D_eo (the residual)
    double cg_dsl_ms[4] = {};
    int cg_dsl_n[4] = {};
};

namespace lgt {

lgt_status fail(lgt_status s, const char *fmt, ...);
void clear_error();

// device workspace buffer `name` of at least `bytes` (contents undefined)
void *workspace(lgt_ctx *c, const char *name, size_t bytes);
void *pinned(lgt_ctx *c, size_t bytes);

// (prec, recon) -> storage format; returns false if unsupported
bool fmt_of(int32_t prec, int32_t recon, Fmt *f);
inline bool fmt_is_f64(Fmt f) { return f == F64R18 || f == F64R12; }
size_t link_bytes_per_site_dir(Fmt f);

lgt_status check_links(const lgt_links *U, bool need_f64, Fmt *f);
// fat and Naik fields of the improved operator: one 18-real format (F64, or F32 unless need_f64)
lgt_status check_improved(const lgt_links *F, const lgt_links *N, bool need_f64, Fmt *f);
lgt_status check_ptr(const void *p, const char *what);

// make ctx's device current for the scope, restoring the previous one
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceScope()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Even-odd CG. With U3hi (and U3lo for the mixed schemes) set, the operator is
// the improved one: Uhi/Ulo are its fat fields and U3hi/U3lo its Naik fields.
lgt_status cg_solve(lgt_ctx *c, const lgt_links *Uhi, const lgt_links *Ulo, const lgt_cg_params *p,
                    const double *b, double *x, lgt_cg_result *res, const lgt_links *U3hi = nullptr,
                    const lgt_links *U3lo = nullptr);

// The batched CG as kernel launches (mcg_host.cpp), for mixed schemes: each
// problem with N = 2^logN >= 4 right-hand sides (nrhs of them real), a
// four-lane inner engine with gps groups, q->U_hi F64 x 18 and q->U_lo in
// format flo; every problem on its own context's stream.
struct McgProblem {
    const lgt_cg_problem *q;
    Fmt flo;
    int logN, engine, gps;
};
lgt_status mcg_solve(const McgProblem *mp, int nprob, const lgt_cg_params *p);

// launch geometry of the one-link / improved Dslash for link format f
inline Launch dslash_launch(const lgt_ctx *c, Fmt f) { return site_launch(c->g.Vh, c->dbs[f]); }
inline Launch dslash_launch_improved(const lgt_ctx *c, Fmt f) { return site_launch(c->g.Vh, c->ibs[f]); }

// the fermion force given its two native scratch vectors (X and Y = D_oe X)
lgt_status force_run(lgt_ctx *c, const lgt_links *U, Fmt f, const double *X, double scale, double *G, double *Xn,
                     double *Yn);

// Fixed scratch array of the library (noalloc.hip), kScratchBytes per device:
// scratch_init looks up its address on `device` (which must be current) once
// per device; scratch_ptr returns it (null before scratch_init succeeded).
// 64 MiB: the two FP64 parity vectors of the force up to V/2 = 699050 sites
// (a 32^4 lattice needs 50 MB).
constexpr size_t kScratchBytes = (size_t)64 << 20;
lgt_status scratch_init(int device);
void *scratch_ptr(int device);

} // namespace lgt

#define LGT_HIP(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return lgt::fail(LGT_ERR_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                                \
    } while (0)
