// kernels.hpp -- launch interfaces shared by the host code of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "geom.hpp"

namespace lgt {

constexpr int kBS = 256; // threads per workgroup of the site-parallel kernels
// LDS-staged Dslash: at most this many input sites per workgroup (48 KB at FP64)
constexpr int kMaxStagedSites = 1024;
// MI355X Infinity Cache (memory-side, shared by the 8 XCDs)
constexpr size_t kMallBytes = (size_t)256 << 20;
// CG: up to this many <p, Ap> partials (one per Dslash workgroup), every
// workgroup of the update kernel sums them itself, which saves a launch per
// iteration; the work of those redundant sums grows with the square of the
// workgroup count, so on larger lattices one finalize workgroup computes
// alpha once instead. Both give the same bits. Measured on MI355X: the fused
// sums win at 2048 workgroups (32^4), the extra launch from 5000 (40^4) on,
// by 7 % (FP64) and 17 % (FP32) of the iteration at 64^4.
#ifndef LGT_FUSE_ALPHA_MAX
#define LGT_FUSE_ALPHA_MAX 3584
#endif
constexpr int kFuseAlphaMaxParts = LGT_FUSE_ALPHA_MAX;

// Link storage formats (see fields.hpp)
enum Fmt { F64R18 = 0, F64R12 = 1, F32R18 = 2, F32R12 = 3, BF16R12 = 4, FMT_COUNT = 5 };

// Solver state in device memory, read and written only by the kernels of one
// solve; the host reads it back with an asynchronous copy.
enum State { ST_RUN = 0, ST_INNER = 1, ST_DONE = 2, ST_FAIL = 3, ST_MAXIT = 4, ST_INIT = 5 };
enum Scheme { SCH_FP64 = 0, SCH_RELIABLE = 1, SCH_REFINE = 2 };

struct CgState {
    double rho;        // |r|^2 of the iterated residual
    double rho_prev;   // previous rho (beta after a reliable update)
    double alpha, beta, pAp;
    double bnorm2;     // |b|^2
    double stop_outer; // tol^2 |b|^2 on the FP64 true residual
    double stop_inner; // threshold on the iterated residual
    double inner2;     // REFINE: inner_tol^2 (relative); else absolute threshold
    double last_true;  // last FP64 true |r|^2
    int iter, updates, state, max_iter;
    int scheme, ru_fixed;
    int pend; // 1 while x still lacks alpha p of the last update: the next
              // p = r + beta p adds it (it reads p anyway), else the reliable
              // update or the final residual does, before using x
    int pcur; // double-buffered p (the CG with p = r + beta p inside D_oe):
              // the buffer holding the current p; the beta step flips it
};

// Early-exit rule of a solver kernel, read from CgState at kernel start
enum Gate { GATE_NONE = 0, GATE_ITER = 1, GATE_RU = 2 };
// Scalar step that k_finalize runs on the partial sums of a reducing kernel
enum Fin { FIN_NONE = 0, FIN_ALPHA = 1, FIN_UPDATE = 2, FIN_RU = 3, FIN_INIT = 4, FIN_FINAL = 5 };

struct Launch {
    int nblk;     // workgroups doing work
    int nblk_pad; // launched (multiple of 8 for the XCD remap)
    int bs;       // threads (sites) per workgroup: 64, 128 or 256
};

// one thread per site, bs sites per workgroup (the Dslash's workgroup size is a
// tuned choice per link format; the vector kernels use kBS)
inline Launch site_launch(int Vh, int bs = kBS)
{
    Launch l;
    l.bs = bs;
    l.nblk = (Vh + bs - 1) / bs;
    l.nblk_pad = (l.nblk + 7) / 8 * 8;
    return l;
}
inline bool dslash_bs_ok(int bs) { return bs == 64 || bs == 128 || bs == 256; }

// ---- Dslash family ------------------------------------------------------
enum Epi { EPI_PLAIN = 0, EPI_A = 1, EPI_RES = 2, EPI_RES_LO = 3, EPI_PAP = 4, EPI_UPD = 5, EPI_PAPX = 6 };

struct DslashArgs {
    const void *U;   // packed links (the fat one-link field of the improved operator)
    const void *U3;  // improved operator: packed Naik three-link field, same format; else null
    const void *in;  // vector on parity 1-par
    void *out;       // vector on parity par
    Geom g;
    int par;
    int gate;
    Launch l;
    // EPI_A:   out = m4*aux0 - D in, partial <aux0, out>
    // EPI_RES: r = aux1 - (m4*aux0 - D in) in FP64 into out (or out_lo), partial |r|^2
    // EPI_PAP: out = D in (D_oe p), partial m4 |aux0|^2 + |out|^2 at the same cb,
    //          which sums to <p, A p> (A = m4 - D_eo D_oe, D_eo = -D_oe^dag)
    // EPI_UPD: rw -= alpha (m4*aux0 - D in) (D_eo t, Ap never stored), partial
    //          |rw|^2; alpha = rho / (sum of the nparts_in partials parts_in of the
    //          preceding EPI_PAP), every workgroup summing them in the same order
    //          (workgroup 0 records it in st), or st->alpha when nparts_in == 0;
    //          with pb set, p is double-buffered and aux0 / pb are buffers 0 / 1:
    //          the update reads the new p, buffer 1 - st->pcur
    // EPI_PAPX: EPI_PAP with p' = r + beta p formed here: in / pb are the p
    //          buffers 0 / 1 (the old p is buffer st->pcur), rin is r; every
    //          gathered input is r + beta p_old; at its own index each thread
    //          writes p' to the other buffer and, with st->pend, x += alpha
    //          p_old into xw; partials m4 |p'|^2 + |out|^2
    const void *aux0;
    const void *aux1;
    void *out_lo;
    void *rw;
    void *pb;        // second p buffer (double-buffered p), else null
    const void *rin; // EPI_PAPX: r
    void *xw;        // EPI_PAPX: x
    const double *parts_in;
    int nparts_in;
    double m4;
    double *partials;
    CgState *st;
    int hpi; // hops whose loads are issued together: 1, 2 or 8; 4 = 2 with the input staged in LDS
    int ntl; // 1: streaming (non-temporal) link loads, 0: cached
};

// e0 / e1 (may be null): events set to the start and end of the kernel itself
hipError_t launch_dslash(Fmt f, int epi, const DslashArgs &a, hipStream_t s, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
hipError_t launch_pack_links(Fmt f, const double *Ucanon, void *Upacked, const Geom &g, hipStream_t s);
hipError_t launch_unpack_links(Fmt f, const void *Upacked, double *Ucanon, const Geom &g, hipStream_t s);
hipError_t launch_pack_vec(bool f64, const double *src, void *dst, const Geom &g, hipStream_t s);
hipError_t launch_unpack_vec(bool f64, const void *src, double *dst, const Geom &g, hipStream_t s);
hipError_t launch_index_maps(int32_t *lex_of_eo, int32_t *nbr, const Geom &g, hipStream_t s);

// ---- vector kernels (solver.hip) -----------------------------------------
struct VecArgs {
    void *x, *r, *p;
    void *p2; // double-buffered p: the second buffer (the current p is p2 when st->pcur), else null
    int Vh;
    Launch l;
    CgState *st;
    int gate;
};
// e0 / e1 (may be null): events on the kernel's own dispatch packet
hipError_t launch_xpay(bool f64, const VecArgs &a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// x += alpha p when the state holds a pending update (gate: a.gate)
hipError_t launch_x_pending(bool f64, const VecArgs &a, hipStream_t s);
hipError_t launch_ru_accum(double *x64, void *xlo, int Vh, CgState *st, int gate, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
// n reals (double if f64, else float) of pseudo-random values in [-1, 1)
hipError_t launch_fill_noise(void *p, size_t n, bool f64, hipStream_t s);
hipError_t launch_state_init(CgState *st, int scheme, int ru_fixed, int max_iter, double tol,
                             double inner, hipStream_t s);
hipError_t launch_norm_init(const double *b64, int Vh, double *partials, CgState *st, hipStream_t s);
hipError_t launch_cdot(int64_t n, const double *a, const double *b, double *partials, double *result,
                       hipStream_t s);
// sum n partials in order and run the scalar step `fin` (one workgroup)
hipError_t launch_finalize(const double *partials, int n, CgState *st, int fin, int gate, hipStream_t s,
                           hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// ---- link fattening (fatten.hip) --------------------------------------------
struct FatCoeffs {
    double c1, c3, c5, c7, cL, cN; // one link, 3-, 5-, 7-link staples, Lepage, Naik
};
// F, N (canonical [4][V][3][3][2] float64) from U in the same layout; W: workspace
// of 3 V matrices (the innermost staple fields of one direction at a time).
// With I set, W must hold 4 * 3 V and I 4 * 6 V matrices: every direction's
// innermost fields and the fields under its outer staples are kept there for
// launch_fatten_vjp at the same U.
hipError_t launch_fatten(const double *U, double *F, double *N, double *W, const Geom &g, const FatCoeffs &w,
                         hipStream_t s, double *I = nullptr);
// GU (+)= scale * dS/dU from GF = dS/dF and GN = dS/dN (all canonical); ws:
// workspace of kFatVjpMatrices * V matrices (18 doubles each). Wk, Ik: the
// fields launch_fatten kept at this U (then not recomputed), or null.
constexpr int kFatVjpMatrices = 18;
hipError_t launch_fatten_vjp(const double *U, const double *GF, const double *GN, double *GU, double *ws,
                             const Geom &g, const FatCoeffs &w, double scale, bool accumulate, hipStream_t s,
                             const double *Wk = nullptr, const double *Ik = nullptr);

// ---- Table 1 routines (routines.hip) ---------------------------------------
hipError_t launch_routine(int routine, bool f64, const void *a, const void *b, void *c, int64_t n, double s,
                          hipStream_t st);

// ---- force (force.hip) -----------------------------------------------------
// fermion force of one link field (naik: the three-link field of the improved operator)
hipError_t launch_force(const double *Xnat, const double *Ynat, double scale, double *G, const Geom &g,
                        hipStream_t s, bool naik = false);
// gphi = 2 scale X over one canonical parity vector (dS/dphi of phi^dag A^-1 phi)
hipError_t launch_phi_grad(const double *X, double scale, double *gphi, const Geom &g, hipStream_t s);

} // namespace lgt
