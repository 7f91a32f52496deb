/* Runs every entry point of the C oracle on small lattices (extent 2, where a
 * site's +mu and -mu neighbours coincide, and a non-cubic one with an
 * antiperiodic direction) so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks its memory accesses and arithmetic. The
 * values are not checked here (the oracle's pins do that); a sanitizer report
 * or a non-finite result fails the run. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "lgt_oracle.h"

static unsigned long long g_state = 0x9e3779b97f4a7c15ull;

static double unif(void)
{
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

static double *rnd(size_t n)
{
    double *p = malloc(n * sizeof(double));
    if (!p) exit(3);
    for (size_t i = 0; i < n; i++) p[i] = unif();
    return p;
}

static int finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; i++)
        if (!isfinite(p[i])) return 0;
    return 1;
}

static int run(const int32_t L[4], const int32_t bc[4])
{
    const size_t V = (size_t)L[0] * L[1] * L[2] * L[3], Vh = V / 2;
    const size_t nl = 4 * V * 18, nv = Vh * 6;
    if (!or_geom_ok(L, bc)) return 1;
    int32_t *lex = malloc(V * sizeof(int32_t)), *nbr = malloc(2 * 8 * Vh * sizeof(int32_t));
    double *U = rnd(nl), *N = rnd(nl), *a = rnd(nv), *b = rnd(nv), *o = malloc(nv * sizeof(double));
    double *x = malloc(nv * sizeof(double)), *G = malloc(nl * sizeof(double)), *G2 = malloc(nl * sizeof(double));
    if (!lex || !nbr || !o || !x || !G || !G2) return 3;
    or_index_maps(L, lex, nbr);
    int bad = 0;
    for (int par = 0; par < 2; par++) {
        or_dslash(L, bc, U, a, o, par);
        bad |= !finite_all(o, nv);
        or_dslash_imp(L, bc, U, N, a, o, par);
        bad |= !finite_all(o, nv);
    }
    or_apply_A(L, bc, U, 0.3, a, o);
    or_apply_A_imp(L, bc, U, N, 0.3, a, o);
    double re, im;
    or_cdot((int64_t)nv, a, b, &re, &im);
    bad |= !isfinite(re) || !isfinite(im) || !isfinite(or_norm2((int64_t)nv, a));
    int it = 0;
    double rr = 0.0;
    int st = or_cg(L, bc, U, 0.5, b, x, 1e-10, 5000, &it, &rr);
    bad |= st != 0 || !finite_all(x, nv);
    or_force(L, bc, U, x, G);
    bad |= !finite_all(G, nl);
    bad |= !isfinite(or_action_variational(L, bc, U, 0.5, b, x));
    st = or_cg_imp(L, bc, U, N, 0.5, b, x, 1e-10, 5000, &it, &rr);
    bad |= st != 0;
    or_force_imp(L, bc, U, N, x, G, G2);
    bad |= !finite_all(G, nl) || !finite_all(G2, nl);
    /* Table 1 routines on one operand set each */
    or_cx *A = (or_cx *)U, *B = (or_cx *)N, *c = (or_cx *)o;
    or_cx c4[4][3];
    or_add_su3_vector(A, B, c);
    or_mult_su3_mat_vec(A, B, c);
    or_mult_adj_su3_mat_vec(A, B, c);
    or_mult_adj_su3_mat_vec_4dir(A, B, &c4[0][0]);
    or_mult_adj_su3_mat_4vec(B, A, c4[0], c4[1], c4[2], c4[3]);
    or_mult_su3_an(A, B, (or_cx *)G);
    or_mult_su3_na(A, B, (or_cx *)G);
    or_mult_su3_nn(A, B, (or_cx *)G);
    or_mult_su3_mat_vec_sum_4dir(A, B, c);
    or_scalar_mult_add_su3_matrix(A, B, 0.5, (or_cx *)G);
    or_scalar_mult_add_su3_vector(A, B, 0.5, c);
    or_su3_projector(A, B, (or_cx *)G);
    or_sub_four_su3_vecs(c, B);
    free(lex); free(nbr); free(U); free(N); free(a); free(b); free(o); free(x); free(G); free(G2);
    return bad ? 2 : 0;
}

int main(void)
{
    const int32_t L1[4] = {2, 2, 2, 2}, bc1[4] = {1, 1, 1, 1};
    const int32_t L2[4] = {2, 4, 2, 6}, bc2[4] = {1, -1, 1, -1};
    const int32_t L3[4] = {4, 4, 4, 4}, bc3[4] = {1, 1, 1, -1};
    int r = run(L1, bc1) | run(L2, bc2) | run(L3, bc3);
    or_set_threads(1);
    r |= run(L2, bc2);
    printf("oracle driver: %s\n", r ? "FAILED" : "ok");
    return r;
}
