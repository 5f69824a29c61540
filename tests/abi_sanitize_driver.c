/* Test driver: the library's host-side entry points from C, for a build of
 * the host code under AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py).  No device: descriptions are validated, grids
 * and contexts set up and torn down, tunings validated, and every call that
 * needs a bound workspace must answer TK_E_STATE. */
#include "tk.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#define CHECK(cond)                                                     \
    do {                                                                \
        if (!(cond)) {                                                  \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                   \
        }                                                               \
    } while (0)

static tk_instance_desc desc(double a, int m, int n_r, int n_theta)
{
    tk_instance_desc d;
    memset(&d, 0, sizeof d);
    d.M = 1.0;
    d.a = a;
    d.s = -2;
    d.m = m;
    d.n_r = n_r;
    d.n_theta = n_theta;
    d.rstar_min = -30.0;
    d.rstar_max = 40.0;
    d.rstar_obs = 30.0;
    d.extract_every = 4;
    tk_stable_dt(&d, &d.dt);
    return d;
}

int main(void)
{
    CHECK(tk_abi_version() == TK_ABI_VERSION);
    tk_instance_desc ds[3] = {desc(0.9, 2, 301, 17), desc(0.0, 1, 123, 33), desc(0.99, 8, 77, 9)};
    for (int k = 0; k < 3; ++k) CHECK(ds[k].dt > 0);

    /* invalid descriptions, each refused without a context */
    tk_ctx *ctx = NULL;
    tk_instance_desc bad = ds[0];
    bad.n_r = 4;
    CHECK(tk_init_grid(&bad, 1, TK_FP64, NULL, &ctx) == TK_E_INVALID && ctx == NULL);
    bad = ds[0];
    bad.a = 1.0;
    CHECK(tk_init_grid(&bad, 1, TK_FP64, NULL, &ctx) == TK_E_INVALID);
    bad = ds[0];
    bad.rstar_max = NAN;
    CHECK(tk_init_grid(&bad, 1, TK_FP64, NULL, &ctx) == TK_E_INVALID);
    bad = ds[0];
    bad.dt *= 10;
    CHECK(tk_init_grid(&bad, 1, TK_FP64, NULL, &ctx) == TK_E_UNSTABLE);
    bad.flags = TK_FLAG_FORCE_DT;
    CHECK(tk_init_grid(&bad, 1, TK_FP64, NULL, &ctx) == TK_OK && ctx != NULL);
    CHECK(tk_destroy(ctx) == TK_OK);
    /* hyperboloidal layer: accepted on s = -2 inside the grid, refused otherwise */
    bad = ds[0];
    bad.layer_start = 20.0;
    CHECK(tk_init_grid(&bad, 1, TK_FP64, NULL, &ctx) == TK_OK && ctx != NULL);
    CHECK(tk_destroy(ctx) == TK_OK);
    CHECK(tk_init_grid(&bad, 1, TK_FP32_COMP, NULL, &ctx) == TK_OK && ctx != NULL);
    CHECK(tk_destroy(ctx) == TK_OK);
    bad.layer_start = 45.0;
    CHECK(tk_init_grid(&bad, 1, TK_FP64, NULL, &ctx) == TK_E_INVALID);
    ctx = NULL;
    CHECK(tk_init_grid(ds, 0, TK_FP64, NULL, &ctx) == TK_E_INVALID);
    CHECK(tk_init_grid(ds, 3, (tk_precision)7, NULL, &ctx) == TK_E_INVALID);

    for (int prec = 0; prec <= 1; ++prec) {
        ctx = NULL;
        CHECK(tk_init_grid(ds, 3, (tk_precision)prec, NULL, &ctx) == TK_OK);
        size_t bytes = 0;
        CHECK(tk_workspace_bytes(ctx, &bytes) == TK_OK && bytes > 0);
        /* tunings: valid ones accepted, invalid ones refused (no workspace yet) */
        tk_tuning t;
        memset(&t, 0, sizeof t);
        const int rows[] = {0, 3, 8, 64};
        for (int k = 0; k < 4; ++k) {
            t.kernel = rows[k] ? TK_KERNEL_FUSED : TK_KERNEL_FUSED2;
            t.rows_per_tile = rows[k];
            t.prefetch_rows = 1;
            CHECK(tk_set_tuning(ctx, &t) == TK_OK);
        }
        t.kernel = TK_KERNEL_TILED;
        t.rows_per_tile = 8;
        CHECK(tk_set_tuning(ctx, &t) == TK_OK);
        t.rows_per_tile = 5;
        CHECK(tk_set_tuning(ctx, &t) == TK_E_INVALID);
        t.kernel = 9;
        CHECK(tk_set_tuning(ctx, &t) == TK_E_INVALID);
        /* the NULL stream cannot be captured: no graphs on it */
        t.kernel = TK_KERNEL_FUSED2;
        t.rows_per_tile = 0;
        t.graph_steps = 10;
        CHECK(tk_set_tuning(ctx, &t) == TK_E_INVALID);
        t.kernel = TK_KERNEL_TILED;
        t.rows_per_tile = 8;
        t.graph_steps = 0;
        tk_tuning got;
        CHECK(tk_get_tuning(ctx, &got) == TK_OK && got.kernel == TK_KERNEL_TILED && got.rows_per_tile == 8);
        /* calls that need the workspace */
        CHECK(tk_step(ctx, 1) == TK_E_STATE);
        double buf[64];
        long n = -1;
        CHECK(tk_extract(ctx, 0, buf, 1, &n) == TK_E_STATE);
        CHECK(tk_autotune(ctx, 1, 1, NULL, 0, NULL, NULL) == TK_E_STATE);
        CHECK(tk_prepare(ctx, 10) == TK_E_STATE);
        size_t save_bytes = 0;
        CHECK(tk_autotune_bytes(ctx, &save_bytes) == TK_OK && save_bytes > 0);
        tk_counters cnt;
        CHECK(tk_get_counters(ctx, &cnt) == TK_OK && cnt.graphs_instantiated == 0 && cnt.graph_launches == 0 &&
              cnt.eager_launches == 0);
        CHECK(tk_get_fields(ctx, 0, buf, buf) == TK_E_STATE);
        tk_source_desc src;
        memset(&src, 0, sizeof src);
        src.kind = TK_SRC_CIRCULAR_LINEAR_DELTA;
        src.r0 = 8.0;
        src.amplitude = 1.0;
        src.ramp = 50.0;
        CHECK(tk_set_source(ctx, 5, &src) == TK_E_INVALID);
        CHECK(tk_last_error(ctx) != NULL);
        CHECK(tk_destroy(ctx) == TK_OK);
    }

    /* Richardson on complex samples (re, im pairs): values, and argument errors */
    double w1[6] = {1, 0, 2, 0, 3, 0}, w2[6] = {1.5, 0, 2.5, 0, 3.5, 0}, w3[6] = {1.625, 0, 2.625, 0, 3.625, 0};
    double ex[6], err[3];
    CHECK(tk_richardson(w1, w2, w3, 3, 2, ex, err) == TK_OK);
    CHECK(fabs(ex[0] - (4 * 1.625 - 1.5) / 3) < 1e-15 && ex[1] == 0);
    CHECK(tk_richardson(w1, w2, w3, 3, 0, ex, err) == TK_E_INVALID);
    CHECK(tk_richardson(NULL, w2, w3, 3, 2, ex, err) == TK_E_INVALID);
    printf("ok\n");
    return 0;
}
