/* A plain C99 caller of the library's host-side entry points: the public
 * header compiles as C, the exports link, and the calls that need no GPU
 * (model constants, equation counts, context creation and sizes, argument
 * validation) return what the header documents.  Exit status 0 on success;
 * every failed check prints one line. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "lbm.h"

static int failures = 0;

static void check(int ok, const char* what) {
    if (!ok) {
        printf("FAILED: %s\n", what);
        ++failures;
    }
}

int main(void) {
    int32_t e[LBM_MAX_Q * 3];
    double w[LBM_MAX_Q], c = 0.0, sum = 0.0;
    int count = 0, i;

    /* status strings */
    check(lbm_status_str(LBM_OK) != NULL && strlen(lbm_status_str(LBM_OK)) > 0, "status string");
    check(lbm_status_str(LBM_E_INVALID) != NULL, "error status string");

    /* Table 1: Omega(4, 2) = 9, Omega(4, 3) = 11, Omega(2, 3) = 4 */
    check(lbm_equation_count(4, 2, &count) == LBM_OK && count == 9, "Omega(4, 2) = 9");
    check(lbm_equation_count(4, 3, &count) == LBM_OK && count == 11, "Omega(4, 3) = 11");
    check(lbm_equation_count(2, 3, &count) == LBM_OK && count == 4, "Omega(2, 3) = 4");
    check(lbm_equation_count(-1, 3, &count) == LBM_E_INVALID, "Omega with m < 0 is refused");

    /* D3Q95: c of Table 3 to the printed digits, weights summing to one */
    check(lbm_velocity_set(3, 95, e, w, &c) == LBM_OK, "D3Q95 velocity set");
    check(fabs(c - 0.421803) < 5e-7, "D3Q95 speed c = .421803");
    for (i = 0; i < 95; ++i) sum += w[i];
    check(fabs(sum - 1.0) < 1e-13, "D3Q95 weights sum to one");
    check(e[0] == 0 && e[1] == 0 && e[2] == 0, "D3Q95 starts with the rest velocity");

    /* D3Q19: the closed-form weights 1/3, 1/18, 1/36 */
    check(lbm_velocity_set(3, 19, e, w, &c) == LBM_OK, "D3Q19 velocity set");
    check(fabs(w[0] - 1.0 / 3.0) < 1e-15 && fabs(w[1] - 1.0 / 18.0) < 1e-15 &&
              fabs(w[18] - 1.0 / 36.0) < 1e-15,
          "D3Q19 weights 1/3, 1/18, 1/36");
    check(lbm_velocity_set(3, 27, e, w, &c) == LBM_E_UNSUPPORTED, "D3Q27 is not a compiled model");

    /* a context needs no device until lbm_bind */
    {
        lbm_ctx* ctx = NULL;
        const int64_t extent[3] = {64, 32, 16};
        size_t pop = 0, scratch = 0, ck = 0;
        check(lbm_velocity_set(3, 95, e, w, &c) == LBM_OK, "D3Q95 velocity set again");
        check(lbm_create(&ctx, 3, 95, e, w, c, extent, 1.5, LBM_FP32_SHIFTED, 1.0, NULL) == LBM_OK &&
                  ctx != NULL,
              "lbm_create D3Q95 64x32x16 FP32-shifted");
        if (ctx) {
            check(lbm_workspace_bytes(ctx, &pop, &scratch) == LBM_OK, "lbm_workspace_bytes");
            check(pop == (size_t)64 * 32 * 16 * 95 * 4, "population bytes = N Q 4");
            check(scratch > 0, "scratch bytes > 0");
            check(lbm_checkpoint_bytes(ctx, 20, 5, 1, &ck) == LBM_OK && ck > 4 * pop,
                  "checkpoint bytes hold the snapshots");
            check(lbm_step(ctx, 1) == LBM_E_STATE, "lbm_step before lbm_bind is refused");
            {
                int order = -1;
                check(lbm_tune_step(ctx, 8, &order) == LBM_E_STATE && order == -1,
                      "lbm_tune_step before lbm_bind is refused");
                check(lbm_set_block_order(ctx, 1) == LBM_OK, "lbm_set_block_order 1");
                check(lbm_set_block_order(ctx, 2) == LBM_E_INVALID, "block order 2 is refused");
            }
            check(strlen(lbm_last_error(ctx)) > 0, "the refusal is explained");
            check(lbm_destroy(ctx) == LBM_OK, "lbm_destroy");
        }
        ctx = NULL;
        check(lbm_create(&ctx, 3, 95, e, w, c, extent, 2.5, LBM_FP64, 1.0, NULL) == LBM_E_INVALID &&
                  ctx == NULL,
              "omega outside [0, 2) is refused");
        check(strlen(lbm_last_error(NULL)) > 0, "the refusal is explained without a context");
        w[3] *= 1.01;
        check(lbm_create(&ctx, 3, 95, e, w, c, extent, 1.5, LBM_FP64, 1.0, NULL) == LBM_E_INVALID,
              "weights that break the group symmetry are refused");
    }
    if (failures == 0) printf("all host-side checks passed\n");
    return failures == 0 ? 0 : 1;
}
