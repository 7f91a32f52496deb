// batch.hpp -- many right-hand sides and lattices: multi-RHS vector layout,
// the per-problem descriptor of the batched solver, and launch interfaces.
//
// Multi-RHS vectors hold N right-hand sides of one parity as planes
// [3][V/2][N] of complex (RHS fastest), so the N lanes that work on one site
// read one contiguous run and share every link load of that site.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "kernels.hpp"

namespace lgt {

constexpr int kMaxRhs = 16;        // right-hand sides per problem (power of two)
constexpr int kMaxProblems = 64;   // problems per batched launch
constexpr int kMaxTotalRhs = 256;  // right-hand sides per batched launch
constexpr int kBB = 1024;          // threads per workgroup of the batched solver
// (site, rhs) pairs of a batch from which its step 1 runs as two passes
constexpr size_t kBatchSplitPairs = (size_t)1 << 21;
// problems (each on its own stream) up to which a mixed-precision batch runs
// as kernel launches (mcg.hip) instead of the persistent launch
constexpr int kMcgMaxProblems = 4;
// LDS per workgroup of the batched solver for the staged input tiles of its
// four-lane Dslash steps: 3 colours x (sites of a tile + Lx) x N right-hand
// sides of FP32 complex (8 B) must fit
constexpr int kBatchStageBytes = 64 * 1024;
inline bool batch_stage_fits(int tile_sites, int hx, int logN)
{
    return (size_t)3 * (tile_sites + 2 * hx) * ((size_t)8 << logN) <= (size_t)kBatchStageBytes;
}
// Groups of four lanes per site the batched solver can run for N = 2^logN
// right-hand sides (R = N / (4 groups) per lane): N = 4: 1; N = 8: 1 or 2;
// N = 16: 2 or 4 (R = 4 needs more registers than its 1024-thread
// workgroups leave, so a request for 1 group at N = 16 becomes 2).
inline int batch_groups(int logN, int gps)
{
    if (logN <= 2) return 1;
    if (logN == 3) return gps == 2 ? 2 : 1;
    return gps == 4 ? 4 : 2;
}

// One problem of a batched solve. Two tilings of its (site, rhs) pairs:
// lane tiles of kBB pairs (BLAS steps, FP64 Dslash, inner Dslash of the lane
// engine) and, for the four-lane engines, inner-Dslash tiles of
// kBB / (4 gps) sites.
struct BatchProb {
    Geom g;
    int logN;    // log2 of the number of right-hand sides
    int eng;     // inner Dslash engine (MrhsEngine)
    int gps;     // four-lane engines: groups of four lanes per site (batch_groups)
    int lt0, nlt; // first global lane tile, lane tiles
    int dt0, ndt; // first global inner-Dslash tile, inner-Dslash tiles
    int rhs0;    // first global right-hand-side index
    int stage;   // four-lane engines: 1 if a tile's x/y neighbourhood is staged in LDS
    double m4;   // 4 m^2
    const void *Ulo, *Uhi;
    const double *b64;          // FP64 multi-RHS vectors
    double *x64, *t64;
    void *r, *pa, *pb, *Ap, *t, *xlo; // inner-precision multi-RHS vectors (xlo = x64 for FP64)
};

// Control words of a persistent launch (device memory, zeroed by the host).
// Arrival counters only grow: the last arrival of a barrier is the one that
// brings a counter to a multiple of its group size.
struct BatchCtl {
    unsigned int gen;        // barrier generation
    unsigned int top;        // group leaders arrived
    unsigned int err;        // 1: a barrier wait exceeded its spin limit
    unsigned int iters_done; // outer loop trips performed
    unsigned int pad[12];
    unsigned int grp[8][16]; // per-XCD arrival counters, one 64-byte line each
};

// Phases of the batched solver's profile (BatchArgs::prof, clock ticks of
// workgroup 0 at the constant 100 MHz rate): set-up and final step, the inner
// steps 1 (D_oe with p' and <p', A p'>) and 2 (D_eo with the update of x and r
// and |r|^2) as this workgroup's own work, the waits at the barriers after
// them (imbalance + barrier), the scalar steps after the barriers, and the
// FP64 reliable updates / refinement steps; with step 1 split (BatchArgs::split),
// its first pass (p' = r + beta p) and the wait after it.
enum BatchPhase {
    PH_SETUP = 0, PH_STEP1, PH_WAIT1, PH_STEP2, PH_WAIT2, PH_STEP1P, PH_WAIT1P, PH_SCALAR, PH_FP64, kBatchPhases
};

struct BatchArgs {
    BatchProb prob[kMaxProblems];
    int nprob;
    int total_lt, total_dt;
    int total_rhs;
    int scheme;
    int ru_interval;
    int max_iter;
    int split;          // 1: step 1 as two passes (p' elementwise, then D_oe p') with a barrier between
    double tol, inner;  // relative tolerance; REFINE inner tolerance or RELIABLE factor
    CgState *states;    // [total_rhs], written at the end of the launch
    double *rows[2];    // partial-sum rows [grid][total_rhs], two buffers
    BatchCtl *ctl;
    unsigned int spin_limit;
    unsigned long long *prof; // [kBatchPhases] phase profile, or null (off)
};

// Multi-RHS Dslash engines: one lane per (site, rhs); four lanes per site
// with R = N/4 right-hand sides each, products on the VALU or on MFMA.
// The four-lane engines serve FP32/BF16 links with N >= 4 (MFMA also needs
// V/2 to be a multiple of 16); other cases use one lane per (site, rhs).
enum MrhsEngine { MRHS_LANE = 0, MRHS_VALU4 = 1, MRHS_MFMA = 2 };
inline bool fmt_is_f64_fmt(Fmt f) { return f == F64R18 || f == F64R12; }
bool mrhs_engine_applies(Fmt f, int logN, int Vh, int engine);
// groups of four lanes per site for the four-lane engines: 1, 2 or 4, with
// R = N / (4 groups) >= 1 right-hand sides per lane
bool mrhs_groups_valid(int logN, int gps);
// The multi-RHS kernels index (site, rhs) and (site, lane) pairs, up to 16 per
// site, in 32 bits: lattices with V/2 * 16 >= 2^31 are rejected.
inline bool mrhs_size_ok(int Vh) { return (int64_t)Vh * 16 < ((int64_t)1 << 31); }

// Standalone multi-RHS Dslash (plain epilogue): out = D in, N right-hand sides.
// staged: the four-lane engines' LDS-staged variant (kStageBS-lane
// workgroups) where its tile fits kMrhsStageMax of LDS; ignored otherwise.
constexpr int kStageBS = 512;
constexpr size_t kMrhsStageMax = 64 * 1024;
// LDS of a staged tile of ts sites: 3 colours x (ts + Lx) sites x N FP32 complex
inline size_t mrhs_stage_bytes(int ts, int hx, int logN) { return (size_t)3 * (ts + 2 * hx) * ((size_t)8 << logN); }
bool mrhs_staging_fits(const Geom &g, int logN, int gps);
hipError_t launch_dslash_mrhs(Fmt f, const void *U, const void *in, void *out, const Geom &g, int par, int logN,
                              hipStream_t s, int engine, int gps, bool staged = false);
// nsrc: canonical right-hand sides present (the rest of the 2^logN are zero-padded / not written); -1: all
hipError_t launch_pack_mrhs(bool f64, const double *src, void *dst, const Geom &g, int logN, hipStream_t s,
                            int nsrc = -1);
hipError_t launch_unpack_mrhs(bool f64, const void *src, double *dst, const Geom &g, int logN, hipStream_t s,
                              int nsrc = -1);
// Persistent batched CG (cooperative launch of `grid` workgroups of kBB
// threads). lo = inner link format; a_dev = BatchArgs in device memory.
hipError_t launch_batch_cg(Fmt lo, const BatchArgs *a_dev, int grid, hipStream_t s);
int batch_cg_max_blocks_per_cu(Fmt lo);

// ---- the batched CG of one lattice as kernel launches (mcg.hip) -------------
// Mixed precision, a four-lane inner engine, N = 2^logN >= 4 right-hand sides.
struct McgArgs {
    Geom g;
    int logN;
    int engine, gps;   // inner multi-RHS engine (MRHS_VALU4 or MRHS_MFMA), groups of four lanes
    double m4;         // 4 m^2
    const void *Ulo, *Uhi; // inner links (F32/BF16), F64 x 18 links
    const double *b64; // FP64 multi-RHS vectors
    double *x64, *t64;
    void *xlo, *r, *p, *t; // FP32 multi-RHS vectors
    CgState *st;       // [N]
    double *parts;     // partial sums [N][stride]
    size_t stride;     // >= the workgroups of every reducing launch
    double *parts_p;   // partials of 4m^2 |p|^2 from the p = r + beta p pass [N][stride_p]
    size_t stride_p;   // >= its workgroups (mcg_xpay_blocks)
};
// partials per right-hand side that the inner Dslash launches write (padded:
// including their idle workgroups), and workgroups of the one-lane-per-(site,
// rhs) launches and of the p = r + beta p pass
int mcg_iter_parts(const Geom &g, int gps, bool padded);
int mcg_lane_blocks(const Geom &g, int logN);
int mcg_xpay_blocks(const Geom &g, int logN);
hipError_t launch_mcg_init(const McgArgs &a, int scheme, int ru_fixed, int max_iter, double tol, double inner,
                           hipStream_t s);
// partials of |b|^2 (mcg_lane_blocks of them per right-hand side)
hipError_t launch_mcg_norm(const McgArgs &a, hipStream_t s);
// per right-hand side: the sum of the first n partials of its row (and of
// the first n_p of its row of parts_p), then the scalar step fin where its
// gate is open (one workgroup per right-hand side)
hipError_t launch_mcg_fin(const McgArgs &a, int n, int fin, int gate, hipStream_t s, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr, int n_p = 0);
// p = r + beta p with the partials of 4m^2 |p|^2 into parts_p
hipError_t launch_mcg_xpay(const McgArgs &a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// which = 0: t = D_oe p with the |t|^2 partials; 1: D_eo t with the update
// of x and r and the |r|^2 partials
hipError_t launch_mcg_dslash(Fmt lo, const McgArgs &a, int which, hipStream_t s, hipEvent_t e0 = nullptr,
                             hipEvent_t e1 = nullptr);
// FP64 step for the right-hand sides whose gate is open: x64 += x_lo, x_lo = 0,
// r = b - A x64 rounded into r, partials of |b - A x64|^2
hipError_t launch_mcg_fp64(const McgArgs &a, int gate, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);

} // namespace lgt
