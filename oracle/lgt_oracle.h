/*
 * lgt_oracle.h -- plain FP64 CPU oracle for the staggered Dslash, the even-odd
 * CG on M^dag M and the fermion force.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library path may include, link or
 * call this code; only the test suite, the smoke check and the CPU baseline of
 * the benchmark do. It shares no source with the HIP library.
 *
 * Layouts (all float64, caller-owned host memory):
 *   links  U[4][V][3][3][2]  direction, eo site, row, column, (re,im);
 *                            no staggered phase or boundary sign folded in
 *   vector v[V/2][3][2]      one parity, checkerboard (cb) order
 *   index maps: lex_of_eo[V], nbr[2][8][V/2] (parity, hop 0..3 = +mu,
 *               4..7 = -mu, cb of the output site) -> cb of the neighbour
 *
 * Geometry: lex = x + Lx*(y + Ly*(z + Lz*t)), parity = (x+y+z+t)&1,
 * cb = lex>>1, eo = parity*V/2 + cb. All dims even and >= 2.
 */
#ifndef LGT_ORACLE_H
#define LGT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } or_cx;

/* --- Table 1 routines (Sec. 4): su3 vector = 3 complex, matrix = 3x3 row-major --- */
void or_add_su3_vector(const or_cx *a, const or_cx *b, or_cx *c);
void or_mult_su3_mat_vec(const or_cx *A, const or_cx *b, or_cx *c);
void or_mult_adj_su3_mat_vec(const or_cx *A, const or_cx *b, or_cx *c);
void or_mult_adj_su3_mat_vec_4dir(const or_cx *a, const or_cx *B4, or_cx *c4);
void or_mult_adj_su3_mat_4vec(const or_cx *B4, const or_cx *a,
                              or_cx *c0, or_cx *c1, or_cx *c2, or_cx *c3);
void or_mult_su3_an(const or_cx *A, const or_cx *B, or_cx *C);
void or_mult_su3_na(const or_cx *A, const or_cx *B, or_cx *C);
void or_mult_su3_nn(const or_cx *A, const or_cx *B, or_cx *C);
void or_mult_su3_mat_vec_sum_4dir(const or_cx *A4, const or_cx *b4, or_cx *c);
void or_scalar_mult_add_su3_matrix(const or_cx *A, const or_cx *B, double s, or_cx *C);
void or_scalar_mult_add_su3_vector(const or_cx *a, const or_cx *b, double s, or_cx *c);
void or_su3_projector(const or_cx *a, const or_cx *b, or_cx *C);
void or_sub_four_su3_vecs(or_cx *a, const or_cx *b4);

/* --- geometry --- */
int  or_geom_ok(const int32_t L[4], const int32_t bc[4]);       /* 1 if valid */
void or_index_maps(const int32_t L[4], int32_t *lex_of_eo, int32_t *nbr);
void or_set_threads(int n);
int  or_get_threads(void);

/* --- operator --- */
/* out (parity out_par) = D in (parity 1-out_par); D = sum_mu eta_mu [s+ U fwd - s- U^dag bwd] */
void or_dslash(const int32_t L[4], const int32_t bc[4], const double *U,
               const double *in, double *out, int out_par);
/* out = A in = 4 m^2 in - D_eo D_oe in, even sites */
void or_apply_A(const int32_t L[4], const int32_t bc[4], const double *U, double mass,
                const double *in, double *out);
/* dot products in cb order: re/im of sum conj(a) b */
void or_cdot(int64_t n_real, const double *a, const double *b, double *re, double *im);
double or_norm2(int64_t n_real, const double *a);

/* --- solver: textbook CG on A x = b (even sites), x0 = 0.
 * Stops when |r|^2 <= tol^2 |b|^2 on the iterated residual, then checks the
 * true residual b - A x and continues from it when it fails.
 * Returns 0 converged, -5 not converged after max_iter, -6 breakdown. */
int or_cg(const int32_t L[4], const int32_t bc[4], const double *U, double mass,
          const double *b, double *x, double tol, int max_iter,
          int *iters, double *true_rel_resid);

/* --- improved operator: fat one-link field F plus Naik three-link field N,
 * both canonical [4][V][3][3][2], general complex 3x3 (coefficients folded in):
 * D = sum_mu eta_mu [s+ F fwd - s- F^dag bwd + s3+ N fwd3 - s3- N^dag bwd3] */
void or_dslash_imp(const int32_t L[4], const int32_t bc[4], const double *F, const double *N,
                   const double *in, double *out, int out_par);
void or_apply_A_imp(const int32_t L[4], const int32_t bc[4], const double *F, const double *N,
                    double mass, const double *in, double *out);
int or_cg_imp(const int32_t L[4], const int32_t bc[4], const double *F, const double *N, double mass,
              const double *b, double *x, double tol, int max_iter, int *iters, double *true_rel_resid);

/* --- force: G[4][V][3][3][2] = dS/d(Re U, Im U) of S = phi^dag A^-1 phi, from X = A^-1 phi */
void or_force(const int32_t L[4], const int32_t bc[4], const double *U,
              const double *X, double *G);
/* S estimate 2 Re<phi,x> - <x, A x>: error is -r^dag A^-1 r, quadratic in the residual */
/* dS/dF and dS/dN for the improved operator (GF, GN: [4][V][3][3][2]) */
void or_force_imp(const int32_t L[4], const int32_t bc[4], const double *F, const double *N,
                  const double *X, double *GF, double *GN);
double or_action_variational(const int32_t L[4], const int32_t bc[4], const double *U,
                             double mass, const double *phi, const double *x);

#ifdef __cplusplus
}
#endif
#endif
