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

constexpr int kMaxRhs = 16;       // right-hand sides per problem (power of two)
constexpr int kMaxProblems = 64;  // problems per batched launch

struct BatchProb {
    Geom g;
    int logN;     // log2 of the number of right-hand sides
    int tile0;    // first global tile of this problem (a tile = 256 threads)
    int ntiles;   // tiles of this problem: ceil(V/2 * N / 256)
    int rhs0;     // first global right-hand-side index
    double m4;    // 4 m^2
    const void *Ulo, *Uhi;
    // FP64 multi-RHS vectors
    const double *b64;
    double *x64, *t64, *q64;
    // inner-precision multi-RHS vectors (FP32 for F32/BF16 links, FP64 otherwise)
    void *r, *pa, *pb, *Ap, *t, *xlo;
    CgState *st; // N states
};

// Control words of a persistent launch (device memory, zeroed by the host).
struct BatchCtl {
    unsigned int bar_count;
    unsigned int bar_gen;
    unsigned int err;         // 1: a barrier wait exceeded its spin limit
    unsigned int iters_done;  // outer loop trips performed
    unsigned int active[2];   // right-hand sides still iterating, per loop parity
    unsigned int need_ru[2];  // right-hand sides waiting for an FP64 update
};

struct BatchArgs {
    BatchProb prob[kMaxProblems];
    int nprob;
    int total_tiles;
    int total_rhs;
    int scheme;
    int ru_interval;
    int max_iter;
    double *partials; // [total_tiles][kMaxRhs]
    BatchCtl *ctl;
    unsigned int spin_limit;
};

// Multi-RHS Dslash engines: one lane per (site, rhs); four lanes per site
// with R = N/4 right-hand sides each, products on the VALU or on MFMA.
// The four-lane engines serve FP32/BF16 links with N >= 4 (MFMA also needs
// V/2 to be a multiple of 16); other cases use one lane per (site, rhs).
enum MrhsEngine { MRHS_LANE = 0, MRHS_VALU4 = 1, MRHS_MFMA = 2 };
inline bool fmt_is_f64_fmt(Fmt f) { return f == F64R18 || f == F64R12; }
bool mrhs_engine_applies(Fmt f, int logN, int Vh, int engine);

// Standalone multi-RHS Dslash (plain epilogue): out = D in, N right-hand sides.
hipError_t launch_dslash_mrhs(Fmt f, const void *U, const void *in, void *out, const Geom &g, int par, int logN,
                              hipStream_t s, int engine);
hipError_t launch_pack_mrhs(bool f64, const double *src, void *dst, const Geom &g, int logN, hipStream_t s);
hipError_t launch_unpack_mrhs(bool f64, const void *src, double *dst, const Geom &g, int logN, hipStream_t s);
// Persistent batched CG (cooperative launch). lo = inner link format.
hipError_t launch_batch_cg(Fmt lo, const BatchArgs *a_host, int grid, hipStream_t s);
int batch_cg_max_blocks_per_cu(Fmt lo);

} // namespace lgt
