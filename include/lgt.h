/*
 * lgt.h -- C ABI of the MI355X (gfx950) staggered Dslash / even-odd CG library.
 *
 * The operation. On a 4-D lattice every site has eight neighbours, two per
 * dimension, joined by SU(3) link matrices (Sec. 1); the work is SU(3)
 * matrix-vector products over those links (Table 1, Sec. 4; the adjoint
 * product element by element is Eqs (1.1)-(2.3)). The library applies the
 * naive staggered operator
 *
 *   (D chi)(x) = sum_mu eta_mu(x) [ s+_mu(x) U_mu(x) chi(x+mu)
 *                                  - s-_mu(x) U_mu(x-mu)^dag chi(x-mu) ]
 *
 * (eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z);
 * s+ = bc_mu on the upper face, s- = bc_mu on the lower face, else 1), i.e.
 * four forward products, four adjoint products and the vector sums: 570 flop
 * per site. M = 2m + D; the solver works on the even-site normal operator
 * A = (M^dag M)_ee = 4 m^2 - D_eo D_oe.
 *
 * Geometry. dims L = (Lx, Ly, Lz, Lt), all even and >= 2, V = prod L <= 2^31.
 * lex = x + Lx*(y + Ly*(z + Lz*t)); parity = (x+y+z+t) & 1; cb = lex >> 1
 * (a bijection onto [0, V/2) for each parity); eo = parity*V/2 + cb.
 *
 * Canonical (user-facing) layouts, float64, little endian:
 *   links    U[4][V][3][3][2]   direction mu, eo site, row, column, (re, im);
 *                               no eta or boundary sign folded in
 *   vectors  v[V/2][3][2]       one parity, cb order
 *   force    G[4][V][3][3][2]   same as links
 * Native (library) layouts are opaque; their sizes come from lgt_links_bytes
 * and lgt_vec_bytes, and lgt_pack_* / lgt_unpack_vec convert.
 *
 * Memory and ownership. Every array argument of a compute call is a device
 * pointer owned by the caller; the library never frees caller memory. Device
 * pointers must be 16-byte aligned (256 recommended). A context owns only its
 * workspace. Calls are ordered on the context's stream; lgt_dslash*,
 * lgt_pack_*, lgt_unpack_vec*, lgt_index_maps, lgt_force*, lgt_fatten_links,
 * lgt_routine and the HMC field updates are asynchronous, as is lgt_apply_normal without its
 * dot product; the solves (lgt_cg_solve*, lgt_hmc_trajectory), the tuners and
 * every call that returns a number to the host (lgt_cdot, lgt_plaquette,
 * lgt_kinetic_energy, lgt_apply_normal with pAp) return after the work is
 * complete.
 *
 * Errors. Every entry point returns an lgt_status; arguments are validated on
 * the host before anything is launched, and a failed call launches nothing.
 * lgt_last_error() gives a thread-local message for the last failure.
 * One context per host thread.
 */
#ifndef LGT_H
#define LGT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lgt_status;
enum {
    LGT_OK = 0,
    LGT_ERR_ARG = -1,           /* null pointer, bad enum, bad parameter value */
    LGT_ERR_GEOMETRY = -2,      /* odd or < 2 dimension, bad bc, volume too large */
    LGT_ERR_ALIGN = -3,         /* device pointer not 16-byte aligned */
    LGT_ERR_DEVICE = -4,        /* no usable GPU, or a HIP runtime error */
    LGT_ERR_NOT_CONVERGED = -5, /* solver hit max_iter; x holds the best iterate */
    LGT_ERR_NONFINITE = -6,     /* NaN/Inf residual, or p.Ap <= 0 (breakdown) */
    LGT_ERR_OOM = -7,           /* workspace allocation failed */
    LGT_ERR_UNSUPPORTED = -8    /* precision/compression pair or device not supported */
};

/* arithmetic / storage precision of a link field or vector */
enum { LGT_F64 = 0, LGT_F32 = 1, LGT_BF16 = 2 };
/* link compression: 18 reals, or 12 reals (rows 0 and 1; row 2 = conj(row0 x row1)) */
enum { LGT_R18 = 18, LGT_R12 = 12 };
enum { LGT_EVEN = 0, LGT_ODD = 1 };

typedef struct {
    int32_t L[4];  /* x, y, z, t extents: even, >= 2 */
    int32_t bc[4]; /* +1 periodic, -1 antiperiodic, per direction */
} lgt_geom;

/* A packed link field in device memory, as written by lgt_pack_links.
 * Supported (prec, recon): (F64,18) (F64,12) (F32,18) (F32,12) (BF16,12).
 * Vectors paired with F64 links are F64; with F32 or BF16 links they are F32. */
typedef struct {
    const void *ptr;
    int32_t prec;
    int32_t recon;
} lgt_links;

typedef struct lgt_ctx lgt_ctx;

/* ---- status and host-only helpers (no device needed) ---------------------- */

const char *lgt_status_string(lgt_status s);
/* message for the last failed call on this thread ("" if none) */
const char *lgt_last_error(void);
/* LGT_OK or LGT_ERR_GEOMETRY */
lgt_status lgt_geom_check(const lgt_geom *g);
/* bytes of a packed link field / of one parity vector in native layout */
lgt_status lgt_links_bytes(const lgt_geom *g, int32_t prec, int32_t recon, size_t *bytes);
lgt_status lgt_vec_bytes(const lgt_geom *g, int32_t prec, size_t *bytes);

/* ---- context ---------------------------------------------------------------- */

/* Create a context on HIP device `device`, ordering work on `hip_stream`
 * (a hipStream_t; NULL = the null stream). Checks the geometry first
 * (LGT_ERR_GEOMETRY), then that the device exists (LGT_ERR_DEVICE) and is a
 * gfx950 part (LGT_ERR_UNSUPPORTED). */
lgt_status lgt_create(const lgt_geom *g, int32_t device, void *hip_stream, lgt_ctx **out);
lgt_status lgt_destroy(lgt_ctx *ctx);
/* Dslash kernel timing inside lgt_cg_solve: with every > 0, the two Dslash
 * launches of every `every`-th iteration of each chunk and every FP64
 * update's Dslash pair carry start and stop events on their own dispatch
 * packets (the kernel's execution alone, as a kernel trace reports it), and
 * the summed times and counts are reported in lgt_cg_result. Sampling
 * (every = 16, say) keeps the host's event bookkeeping small. 0 = off (the
 * default); negative is LGT_ERR_ARG. */
lgt_status lgt_set_timing(lgt_ctx *ctx, int32_t every);
/* The rest of a timed CG iteration: for the last lgt_cg_solve* on this context
 * with timing on, ms[4] receives the mean kernel time (ms) per timed iteration
 * of the vector kernels around the Dslash pair -- (0) x += alpha p with
 * p = r + beta p, (1) always 0: the update r -= alpha Ap runs inside the D_eo
 * launch (its time is in lgt_cg_result's Dslash figures), (2) the
 * one-workgroup step for beta and the stop tests, (3) the one-workgroup alpha
 * step (0 where D_eo sums D_oe's <p, A p> partials itself) -- and n the number
 * of iterations timed (their Dslash pairs are in lgt_cg_result). Host only. */
lgt_status lgt_cg_profile(lgt_ctx *ctx, double ms[4], int32_t *n);
/* The timed Dslash launches of that solve by kind: ms[k] receives the mean
 * kernel time (ms) and n[k] the number timed of (0) the iteration's D_oe
 * (t = D_oe p with the <p, A p> partials), (1) the iteration's D_eo (with the
 * update r -= alpha (4m^2 p - D_eo t) and the |r|^2 partials), (2) and (3) the
 * D_oe and D_eo of the FP64 updates (the residual b - A x). Host only. */
lgt_status lgt_cg_dslash_profile(lgt_ctx *ctx, double ms[4], int32_t n[4]);

/* ---- kernel variants and autotuning ---------------------------------------- */

/* The Dslash comes in variants that issue the loads of 8, 2 or 1 hops
 * together (more loads in flight per thread against more waves per SIMD), with
 * link loads that either stream past the caches (streaming = 1, the default)
 * or are cached (0: a link field that fits in the Infinity Cache may be served
 * from it on the next call). hops_per_group = 4 (LGT_HOPS_LDS) is the 2-hop
 * variant with the input vector's sites around each workgroup's own (its x and
 * y neighbours) copied once into LDS and read from there; where that range
 * would exceed 1024 sites (Lx > 768) it runs as 2. The choice is per link format
 * and per context; it changes speed only, never results. hops_per_group must
 * be 1, 2, 4 or 8. */
#define LGT_HOPS_LDS 4
lgt_status lgt_set_dslash_variant(lgt_ctx *ctx, int32_t prec, int32_t recon, int32_t hops_per_group,
                                  int32_t streaming);
lgt_status lgt_get_dslash_variant(lgt_ctx *ctx, int32_t prec, int32_t recon, int32_t *hops_per_group,
                                  int32_t *streaming);
/* Workgroup size of the Dslash for one link format: 64, 128 or 256 sites
 * (default 256; LGT_ERR_ARG otherwise). A lattice with fewer 256-site
 * workgroups than the chip has CUs (16^4: 128 for 256 CUs) reaches more CUs
 * with smaller ones. Speed only: the operator is the same; the per-workgroup
 * partial sums of the CG's dot products then group differently, so solves
 * agree to rounding rather than bit for bit across sizes. */
lgt_status lgt_set_dslash_workgroup(lgt_ctx *ctx, int32_t prec, int32_t recon, int32_t threads);
lgt_status lgt_get_dslash_workgroup(lgt_ctx *ctx, int32_t prec, int32_t recon, int32_t *threads);
/* Time every variant on U as the CG runs it (1 warm-up and 5 timed pairs of a
 * plain D_oe and a D_eo with the 4m^2 p epilogue and its partial sums, on the
 * context's stream, on pseudo-random vectors in [-1, 1), after about 40 ms of
 * the first variant so the GPU is out of idle; synchronises) and keep, for
 * U's format, the first variant
 * in the order below whose time is within 1 % of the fastest. times_us (host,
 * may be NULL; 24 entries) receives the mean launch time of the variants
 * (hops, streaming) = (8,1) (2,1) (1,1) (4,1) (8,0) (2,0) (1,0) (4,0), first
 * with 256-site workgroups, then 128, then 64; the smaller workgroups are
 * timed only on lattices with fewer than 1024 workgroups of 256 sites (-1
 * elsewhere: there they only add partial sums to the CG). When the environment variable
 * LGT_TUNE_CACHE names a file and times_us is NULL, a cached choice for
 * (device architecture, lattice, format) is used without timing unless
 * LGT_TUNE=force; new results are appended to that file. */
lgt_status lgt_tune_dslash(lgt_ctx *ctx, const lgt_links *U, double times_us[24]);
/* The improved operator's Dslash (lgt_dslash_improved, lgt_cg_solve_improved,
 * lgt_force_improved) keeps its own choice per precision (LGT_F64 or LGT_F32,
 * 18 reals): streaming (1) or cached (0) link loads and the workgroup size (64,
 * 128 or 256 sites; LGT_ERR_ARG otherwise), apart from the one-link
 * operator's choice for the same format. Default: 256 sites, streaming when
 * the fat and Naik fields together exceed 1.5 times the 256 MB Infinity Cache.
 * Speed only, as for the one-link variants. */
lgt_status lgt_set_dslash_improved_variant(lgt_ctx *ctx, int32_t prec, int32_t streaming, int32_t threads);
lgt_status lgt_get_dslash_improved_variant(lgt_ctx *ctx, int32_t prec, int32_t *streaming, int32_t *threads);
/* Time the improved operator's CG pair (as lgt_tune_dslash does, warm-up and
 * pseudo-random vectors included) on fat and
 * naik (one 18-real format) for streaming and cached link loads with 256-,
 * 128- and 64-site workgroups (the smaller ones only below 1024 workgroups of
 * 256 sites) and keep the first within 1 % of the fastest. times_us (host, may
 * be NULL; 6 entries, -1 for untimed): (streaming, 256), (cached, 256),
 * (streaming, 128), (cached, 128), (streaming, 64), (cached, 64). Synchronises. */
lgt_status lgt_tune_dslash_improved(lgt_ctx *ctx, const lgt_links *fat, const lgt_links *naik, double times_us[6]);

/* ---- geometry export (Sec. 1: unique 4-tuple per site, 8 neighbours) ------- */

/* lex_of_eo[V] (int32): lexicographic index of eo site e.
 * nbr[2][8][V/2] (int32): for output parity p, hop h (0..3 = +mu, 4..7 = -mu)
 * and cb, the cb index of the neighbour (it has parity 1-p). Device buffers. */
lgt_status lgt_index_maps(lgt_ctx *ctx, int32_t *lex_of_eo, int32_t *nbr);

/* ---- packing ---------------------------------------------------------------- */

/* Canonical float64 links (device) -> native packed field of (prec, recon).
 * The paper's complex numbers have FP32 or FP64 real and imaginary parts
 * (Sec. 4) and the links are SU(3) (Sec. 1); BF16 storage and the 12-real
 * form (rows 0 and 1 kept, row 2 = conj(row0 x row1) rebuilt, exact for SU(3))
 * are this library's reading, not the paper's. Rounding to F32 / BF16 is
 * round-to-nearest-even from the float64 value (one rounding step).
 * U_packed must hold lgt_links_bytes bytes. */
lgt_status lgt_pack_links(lgt_ctx *ctx, const double *U_canon, int32_t prec, int32_t recon,
                          void *U_packed);
/* The inverse view: a packed field of (prec, recon) -> canonical float64 links
 * [4][V][3][3][2] (device, caller-owned, U_canon must not overlap U_packed).
 * Every stored real is widened exactly (FP32 and BF16 values are exact in
 * float64), so unpacking a packed field shows the rounding of lgt_pack_links
 * element by element; for 12-real formats row 2 is rebuilt as
 * conj(row0 x row1) in the field's arithmetic precision (FP64 for F64 fields,
 * FP32 for F32 and BF16 fields), the matrix the Dslash applies. Unsupported
 * pair: LGT_ERR_UNSUPPORTED. Asynchronous. */
lgt_status lgt_unpack_links(lgt_ctx *ctx, const void *U_packed, int32_t prec, int32_t recon,
                            double *U_canon);
/* Canonical float64 parity vector [V/2][3][2] <-> native vector of `prec`
 * (LGT_F64 or LGT_F32; BF16 fields use F32 vectors). */
lgt_status lgt_pack_vec(lgt_ctx *ctx, int32_t prec, const double *src, void *dst);
lgt_status lgt_unpack_vec(lgt_ctx *ctx, int32_t prec, const void *src, double *dst);

/* ---- Dslash (Sec. 4; Table 1 routines composed over the 8 hops) ------------- */

/* out = D_{out_parity, 1-out_parity} in: in is a native vector on parity
 * 1 - out_parity, out a native vector on out_parity, both in the vector
 * precision that goes with U->prec. No mass term. in and out must not alias. */
lgt_status lgt_dslash(lgt_ctx *ctx, const lgt_links *U, int32_t out_parity,
                      const void *in, void *out);

/* The even-site normal operator the CG solves with, applied once:
 * out = A in = 4 mass^2 in - D_eo D_oe in (M = 2m + D, A = (M^dag M)_ee).
 * in and out are native even-parity vectors in the vector precision of
 * U->prec and must not alias; mass >= 0. When pAp is not NULL it receives
 * Re <in, A in>, summed in FP64 in a fixed order (deterministic), and the call
 * synchronises the context's stream; otherwise it only enqueues. */
lgt_status lgt_apply_normal(lgt_ctx *ctx, const lgt_links *U, double mass, const void *in, void *out,
                            double *pAp);

/* ---- even-odd CG on A = 4 m^2 - D_eo D_oe ------------------------------------ */

enum {
    LGT_CG_FP64 = 0,     /* FP64 links, vectors and arithmetic throughout */
    LGT_CG_RELIABLE = 1, /* low-precision inner CG, FP64 reliable update every
                            ru_interval iterations and at inner convergence */
    LGT_CG_REFINE = 2    /* iterative refinement: FP64 outer residual, inner
                            low-precision CG restarted from 0 to inner_tol */
};

typedef struct {
    double mass;          /* > 0 */
    double tol;           /* target true relative residual |b - A x| / |b|, > 0 */
    int32_t max_iter;     /* > 0, counts inner iterations */
    int32_t scheme;       /* LGT_CG_* */
    int32_t ru_interval;  /* RELIABLE: iterations between FP64 updates (e.g. 50) */
    int32_t x0_is_guess;  /* 1: x holds an initial guess on entry; 0: start from 0 */
    double inner_tol;     /* REFINE: inner relative reduction (e.g. 0.1);
                             RELIABLE/FP64: inner stop as a fraction of tol (<= 1; 0 -> 1) */
    int32_t check_interval; /* iterations between host polls (0 -> 50) */
    int32_t reserved;
} lgt_cg_params;

typedef struct {
    int32_t status;          /* LGT_OK, LGT_ERR_NOT_CONVERGED or LGT_ERR_NONFINITE */
    int32_t iters;           /* inner CG iterations */
    int32_t updates;         /* FP64 reliable updates / refinement steps */
    int32_t dslash_calls;    /* half-Dslash applications, all precisions */
    double true_rel_resid;   /* |b - A x| / |b| recomputed in FP64 at the end */
    double seconds;          /* wall time of the solve on the stream (HIP events) */
    double dslash_ms_hi;     /* with timing on: summed FP64 Dslash kernel time */
    double dslash_ms_lo;     /*                 summed low-precision Dslash time */
    int32_t dslash_timed_hi; /*                 number of launches summed */
    int32_t dslash_timed_lo;
} lgt_cg_result;

/* Solve A x = b on even sites. The paper names the solver only through the
 * routines it spends its time in (Table 1: the vector updates
 * scalar_mult_add_su3_vector / add_su3_vector around the Dslash) and prints no
 * algorithm; the library runs the textbook conjugate-gradient iteration on the
 * Hermitian positive definite A (the even-odd reduction of M^dag M, M = 2m + D)
 * with the stop test on the FP64 true residual, and the mixed-precision
 * schemes of its own reading (reliable updates, iterative refinement), none of
 * them from the paper. U_hi: F64 links (recon 18 or 12). U_lo: the
 * low-precision links for RELIABLE / REFINE (F32 or BF16), ignored (may be
 * NULL) for FP64. b, x: canonical float64 even-parity vectors (device).
 * NOT_CONVERGED and NONFINITE still write the best x and fill *res.
 * An iteration is five launches while the Dslash has at most 3584
 * workgroups of 256 sites (the update kernel then sums the <p, Ap> partials
 * in every workgroup), six beyond (one workgroup computes alpha first); the
 * environment variable LGT_FUSE_ALPHA_MAX moves that limit. The results are
 * the same bit for bit either way. */
lgt_status lgt_cg_solve(lgt_ctx *ctx, const lgt_links *U_hi, const lgt_links *U_lo,
                        const lgt_cg_params *p, const double *b, double *x,
                        lgt_cg_result *res);

/* ---- improved (fat + Naik) operator ----------------------------------------
 * The improved staggered action of the paper's application (Table 4), with
 * its path coefficients folded into two link fields, both general complex
 * 3x3 and packed with lgt_pack_links in one 18-real format (F64 or F32):
 *   (D chi)(x) = sum_mu eta_mu(x) [ s+ F_mu(x) chi(x+mu) - s- F_mu(x-mu)^dag chi(x-mu)
 *                    + s3+ N_mu(x) chi(x+3mu) - s3- N_mu(x-3mu)^dag chi(x-3mu) ]
 * with N_mu(x) the Naik link joining x to x+3mu and s3+- the boundary sign
 * raised to the number of boundary crossings of the three-step hop. 16
 * neighbours, 1146 flop per site; still anti-Hermitian, so A = 4m^2 - D_eo D_oe
 * and the solver are unchanged. Other formats: LGT_ERR_UNSUPPORTED; fat and
 * Naik in different formats: LGT_ERR_ARG. */
lgt_status lgt_dslash_improved(lgt_ctx *ctx, const lgt_links *fat, const lgt_links *naik, int32_t out_parity,
                               const void *in, void *out);
/* lgt_cg_solve for the improved operator: fat_hi and naik_hi F64 x 18; for
 * RELIABLE and REFINE, fat_lo and naik_lo F32 x 18 (ignored for FP64). */
lgt_status lgt_cg_solve_improved(lgt_ctx *ctx, const lgt_links *fat_hi, const lgt_links *naik_hi,
                                 const lgt_links *fat_lo, const lgt_links *naik_lo, const lgt_cg_params *p,
                                 const double *b, double *x, lgt_cg_result *res);

/* The fermion force of the improved operator, for both link fields: with
 * X = A^-1 phi (A built from fat and naik, both F64 x 18), G_fat and G_naik
 * (canonical [4][V][3][3][2], device) receive scale * dS/d(Re, Im) of each
 * field, dS = sum Re tr(G_fat^dag dF) + Re tr(G_naik^dag dN). The Naik link
 * N_mu(x) joins x to x + 3 mu, so its derivative is the one-link formula of
 * lgt_force with x + mu replaced by x + 3 mu and that hop's sign. X is a
 * canonical even vector. Asynchronous. */
lgt_status lgt_force_improved(lgt_ctx *ctx, const lgt_links *fat, const lgt_links *naik, const double *X,
                              double scale, double *G_fat, double *G_naik);

/* ---- link fattening for the improved operator -------------------------------- *
 * The application the paper times (Table 4) uses improved staggered quarks: a
 * fat one-link field smeared over staple paths built with the Table 1 matrix
 * products (mult_su3_nn / _na / _an) and a three-link (Naik) field. The paper
 * gives neither paths nor weights; this library uses the asqtad paths. With
 * L_{+nu}(y) = U_nu(y), L_{-nu}(y) = U_nu(y-nu)^dag and the staple
 * S_a[M](x) = L_a(x) M(x+a) L_a(x+mu)^dag along a signed direction a:
 *   F_mu = one_link U_mu + staple3 sum_a S_a[U_mu] + staple5 sum_{a,b} S_a[S_b[U_mu]]
 *        + staple7 sum_{a,b,c} S_a[S_b[S_c[U_mu]]] + lepage sum_a S_a[S_a[U_mu]]
 *   N_mu(x) = naik U_mu(x) U_mu(x+mu) U_mu(x+2mu)
 * with a, b, c orthogonal to mu on pairwise different axes (6, 24, 48 and 6
 * terms). Tree-level asqtad weights: 5/8, 1/16, 1/64, 1/384, -1/16, -1/24
 * (divide each by u0^(path length - 1) for tadpole improvement); unit links
 * then give F = 9/8, N = -1/24. F and N are the fields lgt_dslash_improved and
 * lgt_cg_solve_improved take (after lgt_pack_links). */
typedef struct {
    double one_link, staple3, staple5, staple7, lepage, naik;
} lgt_fat_coeffs;

/* The asqtad weights above with tadpole improvement: each tree-level weight
 * divided by u0^(path length - 1), i.e. one_link 5/8, staple3 1/16 / u0^2,
 * staple5 1/64 / u0^4, staple7 1/384 / u0^6, lepage -1/16 / u0^4, naik
 * -1/24 / u0^2 (u0 = 1: the tree-level weights). The paper's application uses
 * an improved action without printing its weights (Table 4); this is the
 * reading the library takes. u0 must be positive and finite (LGT_ERR_ARG).
 * Host only: no context or device needed. */
lgt_status lgt_asqtad_coeffs(double u0, lgt_fat_coeffs *out);

/* F, N from U: canonical [4][V][3][3][2] float64 device fields (periodic gauge
 * field; fermion boundary signs stay in the Dslash). U, F and N must not
 * overlap (LGT_ERR_ARG). Per direction, the innermost staple sums go to a
 * context workspace of 3 V matrices (allocated on first use), then the outer
 * levels run per link: 86 products of 3x3 complex matrices per link in all.
 * Asynchronous. */
lgt_status lgt_fatten_links(lgt_ctx *ctx, const double *U, const lgt_fat_coeffs *coeffs, double *F, double *N);

/* The chain rule through lgt_fatten_links, for the molecular-dynamics force of
 * the improved operator: given G_fat and G_naik with
 * dS = sum Re tr(G_fat^dag dF) + Re tr(G_naik^dag dN) (what lgt_force_improved
 * writes), G_U receives scale * the G with dS = sum Re tr(G^dag dU) (added to
 * it when accumulate != 0, else overwriting it). Every staple
 * P(x) = L(x) M(x+a) L(x+mu)^dag whose output receives Gp(x) passes
 * L(x)^dag Gp(x) L(x+mu) to M(x+a), Gp(x) L(x+mu) M(x+a)^dag to L(x) and
 * Gp(x)^dag L(x) M(x+a) to L(x+mu); a backward link L_{-nu}(y) passes the
 * adjoint of its share to U_nu(y-nu); the nested sums are taken back level by
 * level, as gathers at each receiving site (no atomics: the result does not
 * depend on scheduling). All fields canonical [4][V][3][3][2] float64 device
 * memory; G_U must not overlap U, G_fat or G_naik (LGT_ERR_ARG); coefficients
 * and scale finite (LGT_ERR_ARG). Needs a context workspace of 18 V matrices
 * (2.6 kB per site; allocated on first use, LGT_ERR_OOM if that fails).
 * Asynchronous. */
lgt_status lgt_fatten_links_vjp(lgt_ctx *ctx, const double *U, const lgt_fat_coeffs *coeffs, const double *G_fat,
                                const double *G_naik, double scale, int32_t accumulate, double *G_U);

/* ---- the HMC step around the solve ----------------------------------------- *
 * Fields in the canonical layout [4][V][3][3][2] float64, eo site order, device
 * memory: links U, momenta P (traceless anti-Hermitian), derivatives G with
 * dS = sum Re tr(G^dag dU) (lgt_force's convention). Wilson gauge action
 * S_g = beta sum_{x, mu<nu} (1 - Re tr U_mu,nu(x)/3); molecular dynamics
 * dU/dt = P U, dP/dt = TA(U G^dag)/2 with TA the traceless anti-Hermitian part,
 * which conserves H = -sum tr P^2 + S_g + S_f. The paper's application runs
 * this (Table 4); its gauge side uses the Table 1 matrix products. */
/* G (+)= scale * dS_g/dU = scale * (-(beta/3)) Sigma^dag, Sigma_mu(x) the staple
 * sum; accumulate = 0 overwrites G. Asynchronous. */
lgt_status lgt_gauge_force(lgt_ctx *ctx, const double *U, double beta, double scale, int32_t accumulate, double *G);
/* P += eps TA(U G^dag) / 2. Asynchronous. */
lgt_status lgt_momentum_update(lgt_ctx *ctx, const double *U, const double *G, double eps, double *P);
/* U = exp(eps P) U (degree-12 Taylor series; accurate to rounding for
 * |eps P| of a molecular-dynamics step). Asynchronous. */
lgt_status lgt_link_update(lgt_ctx *ctx, const double *P, double eps, double *U);
/* sum over x and mu < nu of Re tr U_mu,nu(x) (FP64, fixed summation order); synchronous */
lgt_status lgt_plaquette(lgt_ctx *ctx, const double *U, double *sum);
/* K = -sum tr P^2 (FP64, fixed order); synchronous */
lgt_status lgt_kinetic_energy(lgt_ctx *ctx, const double *P, double *K);

typedef struct {
    double beta, mass;
    double eps;       /* leapfrog step */
    double tol;       /* CG relative residual for the action and every force */
    double u;         /* uniform in [0, 1) for the Metropolis test */
    int32_t nsteps;   /* leapfrog steps */
    int32_t scheme;   /* LGT_CG_FP64, or LGT_CG_RELIABLE with F32 x 12 inner links
                         (F32 x 18 fat and Naik fields for the improved trajectory) */
    int32_t reserved[2];
} lgt_hmc_params;

typedef struct {
    double H0, H1, dH;          /* H = K + S_g + S_f at the start and end */
    double Sg0, Sg1, Sf0, Sf1, K0, K1;
    double seconds;             /* wall time of the call */
    int32_t accepted;           /* 1: u < exp(-dH) */
    int32_t cg_iters, cg_solves;
    int32_t reserved;
} lgt_hmc_result;

/* One HMC trajectory: pseudofermion phi_e = 2m R_e - D_eo R_o from the Gaussian
 * canonical vectors R_e (even) and R_o (odd) at the starting links; leapfrog
 * with nsteps steps of eps (half momentum steps at both ends), every force
 * from a fresh CG (x0 = 0) and lgt_force plus lgt_gauge_force; Metropolis test
 * with u. U and P (device, canonical) are updated in place, or restored when
 * the trajectory is rejected. Uses context workspace; synchronous. */
lgt_status lgt_hmc_trajectory(lgt_ctx *ctx, double *U, double *P, const double *R_e, const double *R_o,
                              const lgt_hmc_params *p, lgt_hmc_result *res);

/* lgt_hmc_trajectory with the improved operator of the application the paper
 * times (Table 4): at every step the fat and Naik fields F(U), N(U) come from
 * lgt_fatten_links with coeffs and are packed F64 x 18 (LGT_CG_RELIABLE: also
 * F32 x 18 for the inner solver); the pseudofermion, action and CG use
 * lgt_dslash_improved's operator, and the fermion force is lgt_force_improved
 * taken back to U with lgt_fatten_links_vjp. Same arguments, workspace and
 * errors as lgt_hmc_trajectory, plus coeffs (non-NULL, finite: LGT_ERR_ARG). */
lgt_status lgt_hmc_trajectory_improved(lgt_ctx *ctx, double *U, double *P, const double *R_e, const double *R_o,
                                       const lgt_hmc_params *p, const lgt_fat_coeffs *coeffs,
                                       lgt_hmc_result *res);

/* ---- Table 1 routines, one at a time --------------------------------------- *
 * lgt_routine applies one SU(3) routine of Table 1 to n independent operand
 * sets (one GPU thread per call), for microbenchmarks of each routine on its
 * own and for checking each against its definition. Operands are
 * structure-of-arrays planes of complex numbers in the precision prec
 * (LGT_F64: double pairs, LGT_F32: float pairs), device memory:
 *   vec = [3][n], mat = [9][n] (element 3 i + j), vec4 = [4][3][n], mat4 = [4][9][n].
 * Operands in the routine's argument order (c is the output):
 *   1 add_su3_vector             a vec, b vec          -> c vec  = a + b
 *   3 mult_adj_su3_mat_vec       a mat, b vec          -> c vec  = a^dag b (Eqs (1.1)-(2.3))
 *   4 mult_adj_su3_mat_vec_4dir  a vec, b mat4         -> c vec4 = b_k^dag a
 *   5 mult_adj_su3_mat_4vec      a mat4, b vec         -> c vec4 = a_k^dag b
 *   6 mult_su3_an                a mat, b mat          -> c mat  = a^dag b
 *   8 mult_su3_na                a mat, b mat          -> c mat  = a b^dag
 *   9 mult_su3_nn                a mat, b mat          -> c mat  = a b
 *  10 mult_su3_mat_vec           a mat, b vec          -> c vec  = a b
 *  11 mult_su3_mat_vec_sum_4dir  a mat4, b vec4        -> c vec  = sum_k a_k b_k
 *  12 scalar_mult_add_su3_matrix a mat, b mat, s       -> c mat  = a + s b
 *  13 scalar_mult_add_su3_vector a vec, b vec, s       -> c vec  = a + s b
 *  14 su3_projector              a vec, b vec          -> c mat, c_ij = a_i conj(b_j)
 *  15 sub_four_su3_vecs          a vec, b vec4         -> c vec  = a - sum_k b_k
 * (2 and 7, the Wilson half-vector routines, are not built: LGT_ERR_UNSUPPORTED.)
 * c must not overlap a or b, except that c may be a for 1, 12, 13 and 15.
 * n = 0 does nothing. Asynchronous on the context's stream. */
enum {
    LGT_R_ADD_SU3_VECTOR = 1,
    LGT_R_MULT_ADJ_SU3_MAT_VEC = 3,
    LGT_R_MULT_ADJ_SU3_MAT_VEC_4DIR = 4,
    LGT_R_MULT_ADJ_SU3_MAT_4VEC = 5,
    LGT_R_MULT_SU3_AN = 6,
    LGT_R_MULT_SU3_NA = 8,
    LGT_R_MULT_SU3_NN = 9,
    LGT_R_MULT_SU3_MAT_VEC = 10,
    LGT_R_MULT_SU3_MAT_VEC_SUM_4DIR = 11,
    LGT_R_SCALAR_MULT_ADD_SU3_MATRIX = 12,
    LGT_R_SCALAR_MULT_ADD_SU3_VECTOR = 13,
    LGT_R_SU3_PROJECTOR = 14,
    LGT_R_SUB_FOUR_SU3_VECS = 15
};
lgt_status lgt_routine(lgt_ctx *ctx, int32_t routine, int32_t prec, int64_t n, const void *a, const void *b,
                       void *c, double s);

/* ---- many right-hand sides and lattices ------------------------------------ */

/* Multi-RHS native vectors hold nrhs (1, 2, 4, 8 or 16) right-hand sides of
 * one parity, right-hand side fastest; canonical multi-RHS vectors are
 * float64 [nrhs][V/2][3][2]. Byte size: nrhs * lgt_vec_bytes. Every multi-RHS
 * call (and lgt_cg_solve_batch) needs V/2 * 16 < 2^31, else
 * LGT_ERR_UNSUPPORTED. */
lgt_status lgt_pack_vec_mrhs(lgt_ctx *ctx, int32_t prec, int32_t nrhs, const double *src, void *dst);
lgt_status lgt_unpack_vec_mrhs(lgt_ctx *ctx, int32_t prec, int32_t nrhs, const void *src, double *dst);
/* out = D in for nrhs right-hand sides at once (native multi-RHS vectors in
 * the vector precision of U): each link is read once per site for all of
 * them. Asynchronous. */
lgt_status lgt_dslash_mrhs(lgt_ctx *ctx, const lgt_links *U, int32_t out_parity, int32_t nrhs, const void *in,
                           void *out);
/* How lgt_dslash_mrhs and the batched solver compute with F32/BF16 links and
 * nrhs >= 4: LGT_MRHS_MFMA (default) puts 16 sites of a wavefront in the 16
 * blocks of 4x4 MFMA outer products over the real embedding of each hop
 * (right-hand sides x output reals, one input real per step);
 * LGT_MRHS_VALU4 does the same products with FMAs; LGT_MRHS_LANE uses one lane
 * per (site, right-hand side). FP64 links and nrhs < 4 always use
 * LGT_MRHS_LANE. Speed only: results agree to rounding. */
enum { LGT_MRHS_LANE = 0, LGT_MRHS_VALU4 = 1, LGT_MRHS_MFMA = 2 };
/* Sets the engine for every link format and nrhs, with one group of four
 * lanes per site (R = nrhs / 4 right-hand sides per lane). */
lgt_status lgt_set_mrhs_engine(lgt_ctx *ctx, int32_t engine);
lgt_status lgt_get_mrhs_engine(lgt_ctx *ctx, int32_t *engine);
/* Variant for one (link format, nrhs): the engine and, for the four-lane
 * engines, `groups` = 1, 2 or 4 groups of four lanes per site, each lane then
 * holding R = nrhs / (4 groups) >= 1 right-hand sides (otherwise LGT_ERR_ARG).
 * The get call reports the variant lgt_dslash_mrhs actually runs on this
 * lattice (LGT_MRHS_LANE, groups 1, where the engine does not apply). The
 * batched solver runs the four-lane engines with 1 group for nrhs = 4, 1 or 2
 * for 8, and 2 or 4 for 16 (a request for 1 group at 16 runs 2). */
lgt_status lgt_set_mrhs_variant(lgt_ctx *ctx, int32_t prec, int32_t recon, int32_t nrhs, int32_t engine,
                                int32_t groups);
lgt_status lgt_get_mrhs_variant(lgt_ctx *ctx, int32_t prec, int32_t recon, int32_t nrhs, int32_t *engine,
                                int32_t *groups);
/* LDS staging for lgt_dslash_mrhs with the four-lane engines (staged = 1, per
 * format and nrhs; default 0): 512-lane workgroups each copy the input of
 * their tile's x and y neighbourhood (the tile's cb range widened by Lx/2 on
 * each side) into LDS once, with 16-byte coalesced loads, and read the x and y
 * hops from there; only the z and t hops gather from memory. Applies where
 * the staged tile (3 x (sites + Lx) x nrhs FP32 complex) fits 64 KB of LDS,
 * else the unstaged kernel runs; lgt_get_mrhs_staging reports what runs. Not
 * used by the batched solver (its persistent launch stages its own inner
 * Dslash; its launched form does not stage). Speed only:
 * results are bit-identical to the unstaged kernel of the same engine and
 * groups. */
lgt_status lgt_set_mrhs_staging(lgt_ctx *ctx, int32_t prec, int32_t recon, int32_t nrhs, int32_t staged);
lgt_status lgt_get_mrhs_staging(lgt_ctx *ctx, int32_t prec, int32_t recon, int32_t nrhs, int32_t *staged);
/* Autotuner of the multi-RHS tile shape: times every variant that applies to
 * U's format and nrhs on this lattice (10 launches each after 2 untimed,
 * alternating output parity, pseudo-random input in [-1, 1), the first
 * variant first run for about 40 ms so the GPU is out of idle), keeps the
 * fastest for that (format, nrhs) in the
 * context (engine, groups and staging), and with LGT_TUNE_CACHE set caches it
 * like lgt_tune_dslash. times_us: NULL, or 13 doubles in this order: lane;
 * VALU with 1, 2, 4 groups; MFMA with 1, 2, 4 groups; then the same six
 * LDS-staged (-1 where a variant does not apply). Uses scratch vectors of the
 * context; synchronous. */
lgt_status lgt_tune_dslash_mrhs(lgt_ctx *ctx, const lgt_links *U, int32_t nrhs, double times_us[13]);

typedef struct {
    lgt_ctx *ctx;          /* the problem's lattice; all problems on one device */
    const lgt_links *U_hi; /* F64 x 18 links */
    const lgt_links *U_lo; /* inner links, one format for all problems; ignored for FP64 */
    int32_t nrhs;          /* 1..16 (padded inside to 1, 2, 4, 8 or 16 with zero sources) */
    const double *b;       /* canonical multi-RHS even vectors [nrhs][V/2][3][2], device */
    double *x;             /* same layout; initial guess when x0_is_guess */
    lgt_cg_result *res;    /* host array of nrhs results */
} lgt_cg_problem;

/* Independent even-odd CGs (own alpha, beta and stop test per right-hand
 * side; not block CG) for every right-hand side of every problem, lattices of
 * different sizes included. Not from the paper, which solves one system at a
 * time: each right-hand side runs the CG iteration of lgt_cg_solve, with
 * <p, A p> taken as 4m^2 |p|^2 + |D_oe p|^2 (the same number, since D_eo =
 * -D_oe^dag) so that alpha is known before D_eo, and batching shares each
 * link load among the right-hand sides of a lattice. Two forms, the same
 * iteration and results to rounding:
 *  - kernel launches, when the scheme is mixed, every problem has a four-lane
 *    inner engine (F32/BF16 links, nrhs > 2), and there is one problem or up
 *    to four problems on different contexts: five launches per iteration per
 *    problem; one problem runs on its context's stream, several each on an
 *    auxiliary stream of its context (created on first use, default
 *    priority, ordered against the context's stream and probs[0].ctx's
 *    stream by events, so that the problems overlap); chunks
 *    of ru_interval iterations (refinement: check_interval, 10 when 0) go out
 *    ahead of the host's read-back of the states, as one replay of a HIP
 *    graph captured at the start of the call (timing off) or as single
 *    launches (timing on), the FP64 steps between chunks; a right-hand side
 *    that meets its inner stop test inside a chunk waits for the chunk's end.
 *  - otherwise ONE cooperative persistent launch (one workgroup per CU) on
 *    the stream of probs[0].ctx: two grid barriers an iteration, every
 *    workgroup summing the per-workgroup partial sums itself, FP64 reliable
 *    updates / refinement steps inside the same launch. Every grid-barrier
 *    wait is bounded (about 2^21 polls, seconds; the environment variable
 *    LGT_BATCH_SPIN_LIMIT sets another bound in [1, 2^30]): a wait that runs
 *    out ends the launch in every workgroup and the call returns
 *    LGT_ERR_DEVICE.
 * The environment variable LGT_BATCH_LAUNCHED = 1 takes the launched form
 * whenever the scheme and engines allow it (any number of problems), 0 never
 * (other values: LGT_ERR_ARG). Sums are taken in a fixed order in both forms,
 * so results are bit-reproducible for a given device and form. The inner
 * Dslash of each problem uses the multi-RHS variant of that problem's own
 * context (lgt_set_mrhs_engine / lgt_set_mrhs_variant / lgt_tune_dslash_mrhs).
 * Schemes and parameters as lgt_cg_solve (shared by all problems); res[j].seconds
 * is the time of the whole batch. Returns LGT_OK when every right-hand side
 * converged, else the first failing status (every res is filled either way).
 * nprob <= 64; the sum over problems of nrhs rounded up to a power of two
 * is <= 256 (a padding right-hand side costs the work of a real one but
 * converges at once and is never reported); a context may appear in several
 * problems. Synchronous. */
lgt_status lgt_cg_solve_batch(const lgt_cg_problem *probs, int32_t nprob, const lgt_cg_params *p);

/* Phase profile of the last lgt_cg_solve_batch whose first problem's context
 * had timing on (lgt_set_timing > 0): ms[9] receives the milliseconds that
 * workgroup 0 of the persistent launch spent in (0) set-up and the final FP64
 * step, (1) the inner D_oe step with <p, A p> (and p = r + beta p unless
 * that runs as a pass of its own), (2) the wait at the barrier after it, (3)
 * the inner D_eo step with the update of x and r and |r|^2, (4) its barrier
 * wait, (5) the pass p = r + beta p where it runs on its own (batches of at
 * least 2^21 (site, rhs) pairs), (6) the wait after it, (7) the scalar steps,
 * (8) the FP64 reliable updates / refinement steps; iters the iterations run
 * (the most of any right-hand side, for the launched form). A wait is the
 * slowest workgroup's extra time plus the barrier itself. For the launched
 * form (lgt_cg_solve_batch) the entries are the kernel times of each kind,
 * measured with events around every launch and summed over the problems
 * (which overlap in time), and the waits are zero.
 * Zeros before any such solve. Host only. */
lgt_status lgt_batch_profile(lgt_ctx *ctx, double ms[9], int32_t *iters);

/* ---- reductions ------------------------------------------------------------ */

/* out[0] + i out[1] = sum conj(a) b over n_complex complex numbers (device
 * float64 arrays), accumulated in FP64 in a fixed order; out is host memory. */
lgt_status lgt_cdot(lgt_ctx *ctx, int64_t n_complex, const double *a, const double *b,
                    double out[2]);

/* ---- fermion force (Table 1 su3_projector) ------------------------------------ */

/* Given X = A^-1 phi (canonical even vector, device) and F64 links, write
 * G = scale * F (canonical [4][V][3][3][2], device) where dS = sum Re tr(F^dag dU)
 * for S = phi^dag A^-1 phi, i.e. F_ij = dS/dRe U_ij + i dS/dIm U_ij:
 *   x even: G_mu(x) = +2 eta_mu(x) s+_mu(x) X(x) Y(x+mu)^dag
 *   x odd : G_mu(x) = -2 eta_mu(x) s+_mu(x) Y(x) X(x+mu)^dag,  Y = D_oe X. */
lgt_status lgt_force(lgt_ctx *ctx, const lgt_links *U, const double *X, double scale, double *G);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lgt_force
 * with its two scratch vectors (X and Y = D_oe X in native layout, 96 bytes per
 * even site) in a fixed 64 MiB device array of the library instead of context
 * workspace. Same arguments and results as lgt_force, bit for bit; the call
 * allocates nothing (the array's address on each device is looked up once, by
 * lgt_create). Limit: V/2 <= 699050 sites (a 32^4 lattice fits), else
 * LGT_ERR_UNSUPPORTED before anything runs. Every call on one GPU shares that
 * GPU's single array: calls that overlap on one device (other streams, other
 * contexts, other threads) race and must be ordered by the caller. Nothing in
 * the array needs to start at zero. Asynchronous. */
lgt_status lgt_force_noalloc(lgt_ctx *ctx, const lgt_links *U, const double *X, double scale, double *G);

/* The derivative of the same action in the source: A^-1 is Hermitian, so
 * dS = 2 Re <X, dphi> and dS/d(Re phi, Im phi) = 2 (Re X, Im X). gphi
 * (canonical even vector, device) receives 2 scale X; X and gphi may be the
 * same buffer. The improved operator's action has the same derivative with its
 * own X. Asynchronous. */
lgt_status lgt_action_phi_grad(lgt_ctx *ctx, const double *X, double scale, double *gphi);

/* ---- measurement aid ---------------------------------------------------------- */

/* Copy `bytes` (a multiple of 16; src and dst device buffers that do not
 * overlap) with a plain streaming kernel on the context's stream. Its rate is
 * the achievable HBM ceiling that the Dslash's bandwidth is compared with
 * (the paper ties the routines' speed to memory bandwidth, Sec. 5); it also
 * calibrates hardware byte counters. Asynchronous. */
lgt_status lgt_stream_copy(lgt_ctx *ctx, const void *src, void *dst, size_t bytes);
/* Read `bytes` (a multiple of 16) of src with the same streaming loads and
 * write nothing (sink: 16 bytes of device memory that is written only for one
 * improbable data pattern). The read-only ceiling for read-dominated kernels
 * such as the Dslash. Asynchronous. */
lgt_status lgt_stream_read(lgt_ctx *ctx, const void *src, size_t bytes, void *sink);

/* The Dslash's link reads alone: for every site of out_parity, its four
 * forward links and the four backward links U_mu(x - mu), with the Dslash's
 * workgroup order and load grouping (all of a site's loads issued together),
 * streaming (1) or cached (0) loads, and no vector reads, arithmetic or output
 * (sink: 8 bytes of device memory written only for one improbable sum). Its
 * rate, 8 links per site over the time, is the read ceiling of the Dslash's
 * own link-access pattern, which the Dslash's bandwidth is compared with
 * (Sec. 5: the routines are bound by memory traffic). Asynchronous. */
lgt_status lgt_stream_read_links(lgt_ctx *ctx, const lgt_links *U, int32_t out_parity, int32_t streaming,
                                 void *sink);

#ifdef __cplusplus
}
#endif
#endif /* LGT_H */
