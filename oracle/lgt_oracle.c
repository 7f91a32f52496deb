/*
 * lgt_oracle.c -- plain FP64 CPU oracle (test infrastructure only; see
 * lgt_oracle.h). Slow on purpose: every step is written the obvious way so it
 * can be read against its source.
 *
 * Sources for each part:
 *  - SU(3) routines: the routine descriptions of Table 1 (Sec. 4). The adjoint
 *    matrix-vector product follows Eqs (1.1)-(2.3) element by element:
 *      C_i.re = sum_j A_ji.re B_j.re + A_ji.im B_j.im
 *      C_i.im = sum_j A_ji.re B_j.im - A_ji.im B_j.re
 *  - Lattice: a 4-D lattice, every site has a unique 4-tuple and eight
 *    neighbours, two per dimension, joined by SU(3) links (Sec. 1, MILC).
 *  - The staggered operator itself is not written out in the paper; the
 *    reading used here (MILC convention) is
 *      (D chi)(x) = sum_mu eta_mu(x) [ s+_mu(x) U_mu(x) chi(x+mu)
 *                                     - s-_mu(x) U_mu(x-mu)^dag chi(x-mu) ]
 *    with eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z),
 *    s+ = bc_mu on the upper boundary, s- = bc_mu on the lower boundary, else 1.
 *    It is composed from the Table 1 routines: the forward half is
 *    mult_su3_mat_vec_sum_4dir, each backward hop is mult_adj_su3_mat_vec,
 *    and sub_four_su3_vecs assembles them (8*66 + 7*6 = 570 flop per site).
 *  - M = 2m + D, D anti-Hermitian, A = (M^dag M)_ee = 4 m^2 - D_eo D_oe.
 *  - CG: textbook Hestenes-Stiefel on A x = b.
 *  - Force: the outer product su3_projector (Table 1) of X and Y = D_oe X.
 *  - Improved operator: the paper's application uses the improved staggered
 *    action (Table 4), whose operator the paper does not write out either.
 *    Reading used (fat one-link plus Naik three-link hops, path coefficients
 *    folded into the two link fields F and N, general complex 3x3):
 *      (D chi)(x) = sum_mu eta_mu(x) [ s+ F_mu(x) chi(x+mu) - s- F_mu(x-mu)^dag chi(x-mu)
 *                       + s3+ N_mu(x) chi(x+3mu) - s3- N_mu(x-3mu)^dag chi(x-3mu) ]
 *    with s3+- = bc_mu to the number of boundary crossings of the three-step
 *    hop; 16 mat-vecs and 15 vector sums, 16*66 + 15*6 = 1146 flop per site.
 */
#include "lgt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Table 1 routines                                                          */
/* ------------------------------------------------------------------------ */

/* add_su3_vector: c = a + b */
void or_add_su3_vector(const or_cx *a, const or_cx *b, or_cx *c)
{
    for (int i = 0; i < 3; i++) {
        c[i].re = a[i].re + b[i].re;
        c[i].im = a[i].im + b[i].im;
    }
}

/* mult_su3_mat_vec: c = A b, c_i = sum_j A_ij b_j */
void or_mult_su3_mat_vec(const or_cx *A, const or_cx *b, or_cx *c)
{
    for (int i = 0; i < 3; i++) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < 3; j++) {
            const or_cx a = A[3 * i + j];
            re += a.re * b[j].re - a.im * b[j].im;
            im += a.re * b[j].im + a.im * b[j].re;
        }
        c[i].re = re;
        c[i].im = im;
    }
}

/* mult_adj_su3_mat_vec: c = A^dag b, element by element as Eqs (1.1)-(2.3) */
void or_mult_adj_su3_mat_vec(const or_cx *A, const or_cx *b, or_cx *c)
{
    for (int i = 0; i < 3; i++) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < 3; j++) {
            const or_cx a = A[3 * j + i];          /* A_ji */
            re += a.re * b[j].re + a.im * b[j].im; /* (1.1)-(1.3) */
            im += a.re * b[j].im - a.im * b[j].re; /* (2.1)-(2.3) */
        }
        c[i].re = re;
        c[i].im = im;
    }
}

/* mult_adj_su3_mat_vec_4dir: one vector a times four adjoint matrices -> four vectors */
void or_mult_adj_su3_mat_vec_4dir(const or_cx *a, const or_cx *B4, or_cx *c4)
{
    for (int k = 0; k < 4; k++)
        or_mult_adj_su3_mat_vec(B4 + 9 * k, a, c4 + 3 * k);
}

/* mult_adj_su3_mat_4vec: the adjoint of each of four matrices times one vector,
 * into four separate vectors */
void or_mult_adj_su3_mat_4vec(const or_cx *B4, const or_cx *a,
                              or_cx *c0, or_cx *c1, or_cx *c2, or_cx *c3)
{
    or_mult_adj_su3_mat_vec(B4 + 0, a, c0);
    or_mult_adj_su3_mat_vec(B4 + 9, a, c1);
    or_mult_adj_su3_mat_vec(B4 + 18, a, c2);
    or_mult_adj_su3_mat_vec(B4 + 27, a, c3);
}

/* mult_su3_an: C = A^dag B */
void or_mult_su3_an(const or_cx *A, const or_cx *B, or_cx *C)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < 3; k++) {
                const or_cx a = A[3 * k + i], b = B[3 * k + j]; /* conj(A_ki) B_kj */
                re += a.re * b.re + a.im * b.im;
                im += a.re * b.im - a.im * b.re;
            }
            C[3 * i + j].re = re;
            C[3 * i + j].im = im;
        }
}

/* mult_su3_na: C = A B^dag */
void or_mult_su3_na(const or_cx *A, const or_cx *B, or_cx *C)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < 3; k++) {
                const or_cx a = A[3 * i + k], b = B[3 * j + k]; /* A_ik conj(B_jk) */
                re += a.re * b.re + a.im * b.im;
                im += a.im * b.re - a.re * b.im;
            }
            C[3 * i + j].re = re;
            C[3 * i + j].im = im;
        }
}

/* mult_su3_nn: C = A B */
void or_mult_su3_nn(const or_cx *A, const or_cx *B, or_cx *C)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < 3; k++) {
                const or_cx a = A[3 * i + k], b = B[3 * k + j];
                re += a.re * b.re - a.im * b.im;
                im += a.re * b.im + a.im * b.re;
            }
            C[3 * i + j].re = re;
            C[3 * i + j].im = im;
        }
}

/* mult_su3_mat_vec_sum_4dir: c = sum_k A_k b_k over four matrices and four vectors */
void or_mult_su3_mat_vec_sum_4dir(const or_cx *A4, const or_cx *b4, or_cx *c)
{
    or_cx t[3];
    or_mult_su3_mat_vec(A4, b4, c);
    for (int k = 1; k < 4; k++) {
        or_mult_su3_mat_vec(A4 + 9 * k, b4 + 3 * k, t);
        or_add_su3_vector(c, t, c);
    }
}

/* scalar_mult_add_su3_matrix: C = A + s B */
void or_scalar_mult_add_su3_matrix(const or_cx *A, const or_cx *B, double s, or_cx *C)
{
    for (int k = 0; k < 9; k++) {
        C[k].re = A[k].re + s * B[k].re;
        C[k].im = A[k].im + s * B[k].im;
    }
}

/* scalar_mult_add_su3_vector: c = a + s b */
void or_scalar_mult_add_su3_vector(const or_cx *a, const or_cx *b, double s, or_cx *c)
{
    for (int i = 0; i < 3; i++) {
        c[i].re = a[i].re + s * b[i].re;
        c[i].im = a[i].im + s * b[i].im;
    }
}

/* su3_projector: outer product C_ij = a_i conj(b_j) */
void or_su3_projector(const or_cx *a, const or_cx *b, or_cx *C)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            C[3 * i + j].re = a[i].re * b[j].re + a[i].im * b[j].im;
            C[3 * i + j].im = a[i].im * b[j].re - a[i].re * b[j].im;
        }
}

/* sub_four_su3_vecs: a -= b0 + b1 + b2 + b3 */
void or_sub_four_su3_vecs(or_cx *a, const or_cx *b4)
{
    for (int k = 0; k < 4; k++)
        for (int i = 0; i < 3; i++) {
            a[i].re -= b4[3 * k + i].re;
            a[i].im -= b4[3 * k + i].im;
        }
}

/* ------------------------------------------------------------------------ */
/* geometry                                                                  */
/* ------------------------------------------------------------------------ */

static int g_threads = 0;

void or_set_threads(int n) { g_threads = n; }

int or_get_threads(void)
{
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

int or_geom_ok(const int32_t L[4], const int32_t bc[4])
{
    int64_t V = 1;
    for (int mu = 0; mu < 4; mu++) {
        if (L[mu] < 2 || (L[mu] & 1)) return 0;
        if (bc && bc[mu] != 1 && bc[mu] != -1) return 0;
        V *= L[mu];
    }
    return V <= ((int64_t)1 << 31);
}

static int64_t vol(const int32_t L[4])
{
    return (int64_t)L[0] * L[1] * L[2] * L[3];
}

static void coords_of_lex(const int32_t L[4], int64_t lex, int c[4])
{
    for (int mu = 0; mu < 4; mu++) {
        c[mu] = (int)(lex % L[mu]);
        lex /= L[mu];
    }
}

static int64_t lex_of_coords(const int32_t L[4], const int c[4])
{
    return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}

static int parity_of(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

/* coordinates of the site with the given parity and checkerboard index */
static void coords_of_cb(const int32_t L[4], int par, int64_t cb, int c[4])
{
    coords_of_lex(L, 2 * cb, c);
    if (parity_of(c) != par) coords_of_lex(L, 2 * cb + 1, c);
}

/* cb index of the neighbour of c one step along +mu (dir=+1) or -mu (dir=-1), periodic */
static int64_t nbr_cb(const int32_t L[4], const int c[4], int mu, int dir)
{
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[mu] = (d[mu] + dir + L[mu]) % L[mu];
    return lex_of_coords(L, d) >> 1;
}

static double eta(const int c[4], int mu)
{
    int s = 0;
    for (int nu = 0; nu < mu; nu++) s += c[nu];
    return (s & 1) ? -1.0 : 1.0;
}

/* boundary sign for the forward hop (x_mu = L-1) and the backward hop (x_mu = 0) */
static double s_plus(const int32_t L[4], const int32_t bc[4], const int c[4], int mu)
{
    return (c[mu] == L[mu] - 1) ? (double)bc[mu] : 1.0;
}
static double s_minus(const int32_t bc[4], const int c[4], int mu)
{
    return (c[mu] == 0) ? (double)bc[mu] : 1.0;
}

void or_index_maps(const int32_t L[4], int32_t *lex_of_eo, int32_t *nbr)
{
    const int64_t V = vol(L), Vh = V / 2;
    for (int64_t lex = 0; lex < V; lex++) {
        int c[4];
        coords_of_lex(L, lex, c);
        const int p = parity_of(c);
        const int64_t cb = lex >> 1;
        lex_of_eo[p * Vh + cb] = (int32_t)lex;
        for (int mu = 0; mu < 4; mu++) {
            nbr[((int64_t)p * 8 + mu) * Vh + cb] = (int32_t)nbr_cb(L, c, mu, +1);
            nbr[((int64_t)p * 8 + 4 + mu) * Vh + cb] = (int32_t)nbr_cb(L, c, mu, -1);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* operator                                                                  */
/* ------------------------------------------------------------------------ */

static const or_cx *link_at(const double *U, int64_t V, int mu, int64_t eo)
{
    return (const or_cx *)(U + ((int64_t)mu * V + eo) * 18);
}

static void scale3(or_cx *v, double s)
{
    for (int i = 0; i < 3; i++) {
        v[i].re *= s;
        v[i].im *= s;
    }
}

/* one-link part of the operator at output site (out_par, cb) with coordinates c */
static void onelink_site(const int32_t L[4], const int32_t bc[4], const double *U, const or_cx *chi,
                         int out_par, int64_t cb, const int c[4], or_cx fwd[3])
{
    const int64_t V = vol(L), Vh = V / 2;
    const int in_par = 1 - out_par;
    or_cx A4[36], b4[12], back[12];
    for (int mu = 0; mu < 4; mu++) {
        const double e = eta(c, mu);
        /* forward hop: U_mu(x) chi(x+mu) */
        memcpy(A4 + 9 * mu, link_at(U, V, mu, out_par * Vh + cb), 9 * sizeof(or_cx));
        memcpy(b4 + 3 * mu, chi + 3 * nbr_cb(L, c, mu, +1), 3 * sizeof(or_cx));
        scale3(b4 + 3 * mu, e * s_plus(L, bc, c, mu));
        /* backward hop: U_mu(x-mu)^dag chi(x-mu), the link lives on the neighbour */
        const int64_t cbm = nbr_cb(L, c, mu, -1);
        or_mult_adj_su3_mat_vec(link_at(U, V, mu, in_par * Vh + cbm), chi + 3 * cbm,
                                back + 3 * mu);
        scale3(back + 3 * mu, e * s_minus(bc, c, mu));
    }
    or_mult_su3_mat_vec_sum_4dir(A4, b4, fwd);
    or_sub_four_su3_vecs(fwd, back);
}

void or_dslash(const int32_t L[4], const int32_t bc[4], const double *U,
               const double *in, double *out, int out_par)
{
    const int64_t Vh = vol(L) / 2;
    const or_cx *chi = (const or_cx *)in;
    or_cx *res = (or_cx *)out;
#pragma omp parallel for schedule(static) num_threads(or_get_threads())
    for (int64_t cb = 0; cb < Vh; cb++) {
        int c[4];
        coords_of_cb(L, out_par, cb, c);
        onelink_site(L, bc, U, chi, out_par, cb, c, res + 3 * cb);
    }
}

/* cb index of x + 3 mu (dir = +1) or x - 3 mu (dir = -1), periodic */
static int64_t nbr3_cb(const int32_t L[4], const int c[4], int mu, int dir)
{
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[mu] = ((d[mu] + 3 * dir) % L[mu] + L[mu]) % L[mu];
    return lex_of_coords(L, d) >> 1;
}

/* bc_mu to the number of times a three-step hop from c along dir crosses the boundary */
static double s3(const int32_t L[4], const int32_t bc[4], const int c[4], int mu, int dir)
{
    const int crossings = dir > 0 ? (c[mu] + 3) / L[mu] : (L[mu] - 1 - c[mu] + 3) / L[mu];
    return ((crossings & 1) && bc[mu] < 0) ? -1.0 : 1.0;
}

void or_dslash_imp(const int32_t L[4], const int32_t bc[4], const double *F, const double *N,
                   const double *in, double *out, int out_par)
{
    const int64_t V = vol(L), Vh = V / 2;
    const int in_par = 1 - out_par;
    const or_cx *chi = (const or_cx *)in;
    or_cx *res = (or_cx *)out;
#pragma omp parallel for schedule(static) num_threads(or_get_threads())
    for (int64_t cb = 0; cb < Vh; cb++) {
        int c[4];
        coords_of_cb(L, out_par, cb, c);
        or_cx acc[3], t[3];
        onelink_site(L, bc, F, chi, out_par, cb, c, acc);
        for (int mu = 0; mu < 4; mu++) {
            const double e = eta(c, mu);
            /* Naik forward hop: N_mu(x) chi(x+3mu) */
            or_mult_su3_mat_vec(link_at(N, V, mu, out_par * Vh + cb), chi + 3 * nbr3_cb(L, c, mu, +1), t);
            or_scalar_mult_add_su3_vector(acc, t, e * s3(L, bc, c, mu, +1), acc);
            /* Naik backward hop: N_mu(x-3mu)^dag chi(x-3mu), the link lives at x-3mu */
            const int64_t cbm3 = nbr3_cb(L, c, mu, -1);
            or_mult_adj_su3_mat_vec(link_at(N, V, mu, in_par * Vh + cbm3), chi + 3 * cbm3, t);
            or_scalar_mult_add_su3_vector(acc, t, -e * s3(L, bc, c, mu, -1), acc);
        }
        memcpy(res + 3 * cb, acc, 3 * sizeof(or_cx));
    }
}

/* D with the one-link field U, plus the Naik field N when N != NULL */
static void dslash_op(const int32_t L[4], const int32_t bc[4], const double *U, const double *N,
                      const double *in, double *out, int out_par)
{
    if (N) or_dslash_imp(L, bc, U, N, in, out, out_par);
    else or_dslash(L, bc, U, in, out, out_par);
}

static void apply_A_op(const int32_t L[4], const int32_t bc[4], const double *U, const double *N,
                       double mass, const double *in, double *out)
{
    const int64_t n = vol(L) / 2 * 6;
    double *tmp = (double *)malloc(sizeof(double) * n);
    dslash_op(L, bc, U, N, in, tmp, 1);  /* D_oe: even -> odd */
    dslash_op(L, bc, U, N, tmp, out, 0); /* D_eo: odd -> even */
    const double m4 = 4.0 * mass * mass;
    for (int64_t k = 0; k < n; k++) out[k] = m4 * in[k] - out[k];
    free(tmp);
}

void or_apply_A(const int32_t L[4], const int32_t bc[4], const double *U, double mass,
                const double *in, double *out)
{
    apply_A_op(L, bc, U, NULL, mass, in, out);
}

void or_apply_A_imp(const int32_t L[4], const int32_t bc[4], const double *F, const double *N,
                    double mass, const double *in, double *out)
{
    apply_A_op(L, bc, F, N, mass, in, out);
}

void or_cdot(int64_t n_real, const double *a, const double *b, double *re, double *im)
{
    double sr = 0.0, si = 0.0;
    for (int64_t k = 0; k < n_real; k += 2) {
        sr += a[k] * b[k] + a[k + 1] * b[k + 1];
        si += a[k] * b[k + 1] - a[k + 1] * b[k];
    }
    *re = sr;
    *im = si;
}

double or_norm2(int64_t n_real, const double *a)
{
    double s = 0.0;
    for (int64_t k = 0; k < n_real; k++) s += a[k] * a[k];
    return s;
}

/* ------------------------------------------------------------------------ */
/* CG                                                                        */
/* ------------------------------------------------------------------------ */

static int cg_op(const int32_t L[4], const int32_t bc[4], const double *U, const double *N,
                 double mass, const double *b, double *x, double tol, int max_iter,
                 int *iters, double *true_rel_resid)
{
    const int64_t n = vol(L) / 2 * 6;
    double *r = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *Ap = (double *)malloc(sizeof(double) * n);
    int status = -5, k = 0;
    const double bb = or_norm2(n, b);
    const double stop = tol * tol * bb;
    memset(x, 0, sizeof(double) * n);
    memcpy(r, b, sizeof(double) * n);
    memcpy(p, b, sizeof(double) * n);
    double rho = bb;
    if (bb == 0.0) {
        status = 0;
        goto done;
    }
    while (k < max_iter) {
        apply_A_op(L, bc, U, N, mass, p, Ap);
        double pAp, im;
        or_cdot(n, p, Ap, &pAp, &im);
        if (!(pAp > 0.0) || !isfinite(pAp)) {
            status = -6;
            break;
        }
        const double alpha = rho / pAp;
        for (int64_t i = 0; i < n; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * Ap[i];
        }
        k++;
        double rho_new = or_norm2(n, r);
        if (!isfinite(rho_new)) {
            status = -6;
            break;
        }
        if (rho_new <= stop) {
            /* true residual r = b - A x */
            apply_A_op(L, bc, U, N, mass, x, Ap);
            for (int64_t i = 0; i < n; i++) r[i] = b[i] - Ap[i];
            rho_new = or_norm2(n, r);
            if (rho_new <= stop) {
                status = 0;
                break;
            }
        }
        const double beta = rho_new / rho;
        for (int64_t i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
done:
    apply_A_op(L, bc, U, N, mass, x, Ap);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - Ap[i];
    if (iters) *iters = k;
    if (true_rel_resid) *true_rel_resid = bb > 0.0 ? sqrt(or_norm2(n, r) / bb) : 0.0;
    free(r);
    free(p);
    free(Ap);
    return status;
}

int or_cg(const int32_t L[4], const int32_t bc[4], const double *U, double mass,
          const double *b, double *x, double tol, int max_iter,
          int *iters, double *true_rel_resid)
{
    return cg_op(L, bc, U, NULL, mass, b, x, tol, max_iter, iters, true_rel_resid);
}

int or_cg_imp(const int32_t L[4], const int32_t bc[4], const double *F, const double *N, double mass,
              const double *b, double *x, double tol, int max_iter, int *iters, double *true_rel_resid)
{
    return cg_op(L, bc, F, N, mass, b, x, tol, max_iter, iters, true_rel_resid);
}

/* ------------------------------------------------------------------------ */
/* force                                                                     */
/* ------------------------------------------------------------------------ */

/*
 * S = phi^dag A^-1 phi. With X = A^-1 phi and Y = D_oe X, dS = 2 Re(X^dag dD_eo Y)
 * (D^dag = -D for any links). Collecting the terms of each link:
 *   x even: G_mu(x) = +2 eta_mu(x) s+_mu(x) X(x) Y(x+mu)^dag
 *   x odd : G_mu(x) = -2 eta_mu(x) s+_mu(x) Y(x) X(x+mu)^dag
 * and dS = sum Re tr(G^dag dU), i.e. dS/dRe U_ij = Re G_ij, dS/dIm U_ij = Im G_ij.
 */
void or_force(const int32_t L[4], const int32_t bc[4], const double *U,
              const double *X, double *G)
{
    const int64_t V = vol(L), Vh = V / 2;
    double *Y = (double *)malloc(sizeof(double) * Vh * 6);
    or_dslash(L, bc, U, X, Y, 1);
    const or_cx *Xe = (const or_cx *)X, *Yo = (const or_cx *)Y;
#pragma omp parallel for schedule(static) num_threads(or_get_threads())
    for (int64_t eo = 0; eo < V; eo++) {
        const int par = eo >= Vh;
        const int64_t cb = eo - par * Vh;
        int c[4];
        coords_of_cb(L, par, cb, c);
        for (int mu = 0; mu < 4; mu++) {
            const int64_t cbp = nbr_cb(L, c, mu, +1);
            const double s = 2.0 * eta(c, mu) * s_plus(L, bc, c, mu);
            or_cx P[9];
            if (par == 0) {
                or_su3_projector(Xe + 3 * cb, Yo + 3 * cbp, P);
            } else {
                or_su3_projector(Yo + 3 * cb, Xe + 3 * cbp, P);
            }
            const double sg = par == 0 ? s : -s;
            double *g = G + ((int64_t)mu * V + eo) * 18;
            for (int k = 0; k < 9; k++) {
                g[2 * k] = sg * P[k].re;
                g[2 * k + 1] = sg * P[k].im;
            }
        }
    }
    free(Y);
}

/* The same derivative for the improved operator, with respect to both link
 * fields: dS = sum Re tr(GF^dag dF) + Re tr(GN^dag dN). Y = D_oe X now has
 * the Naik hops too; a Naik link N_mu(x) joins x to x + 3 mu with the sign
 * eta_mu(x) s3 of that hop, so its term is the one-link term with x + mu
 * replaced by x + 3 mu. */
void or_force_imp(const int32_t L[4], const int32_t bc[4], const double *F, const double *N,
                  const double *X, double *GF, double *GN)
{
    const int64_t V = vol(L), Vh = V / 2;
    double *Y = (double *)malloc(sizeof(double) * Vh * 6);
    or_dslash_imp(L, bc, F, N, X, Y, 1);
    const or_cx *Xe = (const or_cx *)X, *Yo = (const or_cx *)Y;
#pragma omp parallel for schedule(static) num_threads(or_get_threads())
    for (int64_t eo = 0; eo < V; eo++) {
        const int par = eo >= Vh;
        const int64_t cb = eo - par * Vh;
        int c[4];
        coords_of_cb(L, par, cb, c);
        for (int mu = 0; mu < 4; mu++) {
            for (int naik = 0; naik < 2; naik++) {
                const int64_t cbp = naik ? nbr3_cb(L, c, mu, +1) : nbr_cb(L, c, mu, +1);
                const double s = 2.0 * eta(c, mu) * (naik ? s3(L, bc, c, mu, +1) : s_plus(L, bc, c, mu));
                or_cx P[9];
                if (par == 0) or_su3_projector(Xe + 3 * cb, Yo + 3 * cbp, P);
                else or_su3_projector(Yo + 3 * cb, Xe + 3 * cbp, P);
                const double sgn = par == 0 ? s : -s; /* odd sites: the D_oe half */
                double *g = (naik ? GN : GF) + ((int64_t)mu * V + eo) * 18;
                for (int k = 0; k < 9; k++) {
                    g[2 * k] = sgn * P[k].re;
                    g[2 * k + 1] = sgn * P[k].im;
                }
            }
        }
    }
    free(Y);
}

double or_action_variational(const int32_t L[4], const int32_t bc[4], const double *U,
                             double mass, const double *phi, const double *x)
{
    const int64_t n = vol(L) / 2 * 6;
    double *Ax = (double *)malloc(sizeof(double) * n);
    or_apply_A(L, bc, U, mass, x, Ax);
    double px, pim, xAx, xim;
    or_cdot(n, phi, x, &px, &pim);
    or_cdot(n, x, Ax, &xAx, &xim);
    free(Ax);
    return 2.0 * px - xAx;
}
