/* Host-side checks of the C ABI under AddressSanitizer and
 * UndefinedBehaviorSanitizer, with no GPU needed: the host-only helpers with
 * valid and invalid geometries, formats and pointers; every entry point that
 * takes a context with a NULL context; context creation, which must fail
 * cleanly (LGT_ERR_DEVICE) where no GPU is present and otherwise be destroyed
 * again; and the status strings. Exit status 0 only if every call returned what
 * the header says. */
#include <stdio.h>
#include <string.h>

#include "lgt.h"

static int fails = 0;
#define EXPECT(call, want)                                                                              \
    do {                                                                                                \
        const lgt_status got_ = (call);                                                                 \
        if (got_ != (want)) {                                                                           \
            fprintf(stderr, "%s:%d: %s returned %d, expected %d (%s)\n", __FILE__, __LINE__, #call, got_, \
                    (int)(want), lgt_last_error());                                                     \
            fails++;                                                                                    \
        }                                                                                               \
    } while (0)

int main(void)
{
    const lgt_geom good = {{4, 4, 6, 8}, {1, 1, 1, -1}};
    const lgt_geom odd = {{4, 5, 6, 8}, {1, 1, 1, 1}};
    const lgt_geom small = {{4, 0, 6, 8}, {1, 1, 1, 1}};
    const lgt_geom badbc = {{4, 4, 6, 8}, {1, 2, 1, 1}};
    const lgt_geom huge = {{65536, 65536, 2, 2}, {1, 1, 1, 1}};
    size_t n = 0;
    EXPECT(lgt_geom_check(&good), LGT_OK);
    EXPECT(lgt_geom_check(&odd), LGT_ERR_GEOMETRY);
    EXPECT(lgt_geom_check(&small), LGT_ERR_GEOMETRY);
    EXPECT(lgt_geom_check(&badbc), LGT_ERR_GEOMETRY);
    EXPECT(lgt_geom_check(&huge), LGT_ERR_GEOMETRY);
    EXPECT(lgt_geom_check(NULL), LGT_ERR_ARG);
    const int fmts[5][2] = {{LGT_F64, LGT_R18}, {LGT_F64, LGT_R12}, {LGT_F32, LGT_R18}, {LGT_F32, LGT_R12},
                            {LGT_BF16, LGT_R12}};
    const size_t per[5] = {144, 96, 72, 48, 24};
    for (int i = 0; i < 5; i++) {
        EXPECT(lgt_links_bytes(&good, fmts[i][0], fmts[i][1], &n), LGT_OK);
        if (n != (size_t)4 * 4 * 4 * 6 * 8 * per[i]) fails++;
    }
    EXPECT(lgt_links_bytes(&good, LGT_BF16, LGT_R18, &n), LGT_ERR_UNSUPPORTED);
    EXPECT(lgt_links_bytes(&good, 7, LGT_R18, &n), LGT_ERR_UNSUPPORTED);
    EXPECT(lgt_links_bytes(&good, LGT_F64, LGT_R18, NULL), LGT_ERR_ARG);
    EXPECT(lgt_links_bytes(&odd, LGT_F64, LGT_R18, &n), LGT_ERR_GEOMETRY);
    EXPECT(lgt_vec_bytes(&good, LGT_F64, &n), LGT_OK);
    if (n != (size_t)4 * 6 * 8 * 4 / 2 * 48) fails++;
    EXPECT(lgt_vec_bytes(&good, 9, &n), LGT_ERR_ARG);
    lgt_fat_coeffs w;
    EXPECT(lgt_asqtad_coeffs(1.0, &w), LGT_OK);
    if (w.one_link != 5.0 / 8.0 || w.naik != -1.0 / 24.0) fails++;
    EXPECT(lgt_asqtad_coeffs(0.0, &w), LGT_ERR_ARG);
    EXPECT(lgt_asqtad_coeffs(1.0, NULL), LGT_ERR_ARG);
    for (int s = 1; s >= -9; s--)
        if (!lgt_status_string(s) || !*lgt_status_string(s)) fails++;
    /* every context call rejects a NULL context before anything else */
    double d[24];
    int32_t i32;
    lgt_links Ul = {NULL, LGT_F64, LGT_R18};
    lgt_cg_params prm;
    memset(&prm, 0, sizeof(prm));
    lgt_cg_result res;
    EXPECT(lgt_destroy(NULL), LGT_ERR_ARG);
    EXPECT(lgt_set_timing(NULL, 1), LGT_ERR_ARG);
    EXPECT(lgt_cg_profile(NULL, d, &i32), LGT_ERR_ARG);
    {
        int32_t n4[4];
        EXPECT(lgt_cg_dslash_profile(NULL, d, n4), LGT_ERR_ARG);
    }
    EXPECT(lgt_set_dslash_variant(NULL, 0, 18, 8, 1), LGT_ERR_ARG);
    EXPECT(lgt_get_dslash_variant(NULL, 0, 18, &i32, &i32), LGT_ERR_ARG);
    EXPECT(lgt_set_dslash_workgroup(NULL, 0, 18, 64), LGT_ERR_ARG);
    EXPECT(lgt_get_dslash_workgroup(NULL, 0, 18, &i32), LGT_ERR_ARG);
    EXPECT(lgt_tune_dslash(NULL, &Ul, d), LGT_ERR_ARG);
    EXPECT(lgt_index_maps(NULL, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_pack_links(NULL, NULL, 0, 18, NULL), LGT_ERR_ARG);
    EXPECT(lgt_unpack_links(NULL, NULL, 0, 18, NULL), LGT_ERR_ARG);
    EXPECT(lgt_pack_vec(NULL, 0, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_unpack_vec(NULL, 0, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_dslash(NULL, &Ul, 0, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_apply_normal(NULL, &Ul, 0.1, NULL, NULL, d), LGT_ERR_ARG);
    EXPECT(lgt_cg_solve(NULL, &Ul, NULL, &prm, NULL, NULL, &res), LGT_ERR_ARG);
    EXPECT(lgt_dslash_improved(NULL, &Ul, &Ul, 0, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_cg_solve_improved(NULL, &Ul, &Ul, NULL, NULL, &prm, NULL, NULL, &res), LGT_ERR_ARG);
    EXPECT(lgt_force_improved(NULL, &Ul, &Ul, NULL, 1.0, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_fatten_links(NULL, NULL, &w, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_fatten_links_vjp(NULL, NULL, &w, NULL, NULL, 1.0, 0, NULL), LGT_ERR_ARG);
    EXPECT(lgt_set_dslash_improved_variant(NULL, 0, 1, 256), LGT_ERR_ARG);
    EXPECT(lgt_set_mrhs_staging(NULL, 1, 12, 16, 1), LGT_ERR_ARG);
    EXPECT(lgt_get_mrhs_staging(NULL, 1, 12, 16, &i32), LGT_ERR_ARG);
    EXPECT(lgt_get_dslash_improved_variant(NULL, 0, &i32, &i32), LGT_ERR_ARG);
    EXPECT(lgt_tune_dslash_improved(NULL, &Ul, &Ul, d), LGT_ERR_ARG);
    EXPECT(lgt_gauge_force(NULL, NULL, 5.6, 1.0, 0, NULL), LGT_ERR_ARG);
    EXPECT(lgt_momentum_update(NULL, NULL, NULL, 0.1, NULL), LGT_ERR_ARG);
    EXPECT(lgt_link_update(NULL, NULL, 0.1, NULL), LGT_ERR_ARG);
    EXPECT(lgt_plaquette(NULL, NULL, d), LGT_ERR_ARG);
    EXPECT(lgt_kinetic_energy(NULL, NULL, d), LGT_ERR_ARG);
    EXPECT(lgt_hmc_trajectory(NULL, NULL, NULL, NULL, NULL, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_hmc_trajectory_improved(NULL, NULL, NULL, NULL, NULL, NULL, &w, NULL), LGT_ERR_ARG);
    EXPECT(lgt_routine(NULL, 1, 0, 16, NULL, NULL, NULL, 1.0), LGT_ERR_ARG);
    EXPECT(lgt_pack_vec_mrhs(NULL, 1, 4, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_unpack_vec_mrhs(NULL, 1, 4, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_dslash_mrhs(NULL, &Ul, 0, 4, NULL, NULL), LGT_ERR_ARG);
    EXPECT(lgt_set_mrhs_engine(NULL, 0), LGT_ERR_ARG);
    EXPECT(lgt_get_mrhs_engine(NULL, &i32), LGT_ERR_ARG);
    EXPECT(lgt_set_mrhs_variant(NULL, 1, 12, 4, 0, 1), LGT_ERR_ARG);
    EXPECT(lgt_get_mrhs_variant(NULL, 1, 12, 4, &i32, &i32), LGT_ERR_ARG);
    EXPECT(lgt_tune_dslash_mrhs(NULL, &Ul, 4, d), LGT_ERR_ARG);
    EXPECT(lgt_cg_solve_batch(NULL, 0, NULL), LGT_ERR_ARG);
    EXPECT(lgt_batch_profile(NULL, d, &i32), LGT_ERR_ARG);
    EXPECT(lgt_cdot(NULL, 4, NULL, NULL, d), LGT_ERR_ARG);
    EXPECT(lgt_force(NULL, &Ul, NULL, 1.0, NULL), LGT_ERR_ARG);
    EXPECT(lgt_force_noalloc(NULL, &Ul, NULL, 1.0, NULL), LGT_ERR_ARG);
    EXPECT(lgt_action_phi_grad(NULL, NULL, 1.0, NULL), LGT_ERR_ARG);
    EXPECT(lgt_stream_copy(NULL, NULL, NULL, 16), LGT_ERR_ARG);
    EXPECT(lgt_stream_read(NULL, NULL, 16, NULL), LGT_ERR_ARG);
    EXPECT(lgt_stream_read_links(NULL, &Ul, 1, 1, NULL), LGT_ERR_ARG);
    /* context creation: geometry first, then the device */
    lgt_ctx *c = NULL;
    EXPECT(lgt_create(&odd, 0, NULL, &c), LGT_ERR_GEOMETRY);
    EXPECT(lgt_create(&good, 0, NULL, NULL), LGT_ERR_ARG);
    const lgt_status s = lgt_create(&good, 0, NULL, &c);
    if (s == LGT_OK) {
        EXPECT(lgt_set_dslash_workgroup(c, 0, 18, 96), LGT_ERR_ARG);
        EXPECT(lgt_dslash(c, NULL, 0, NULL, NULL), LGT_ERR_ARG);
        EXPECT(lgt_destroy(c), LGT_OK);
    } else if (s != LGT_ERR_DEVICE && s != LGT_ERR_UNSUPPORTED) {
        fprintf(stderr, "lgt_create returned %d (%s)\n", s, lgt_last_error());
        fails++;
    }
    printf("abi driver: %s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
