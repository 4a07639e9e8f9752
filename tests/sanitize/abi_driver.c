/* Calls every host-side path of libmpfc that needs no GPU: the validation of
 * parameters, options and grid sizes (2-D, 3-D, batches), creation requests
 * that are rejected before any HIP call, NULL handles, the operator entry
 * points' argument checks and the error strings.  Built against a host-only,
 * sanitizer-instrumented build of the library (tests/test_sanitizers_cpu.py);
 * prints "abi driver ok" when every call returned what the header states. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "mpfc.h"

static int bad = 0;
#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            printf("failed: %s (line %d)\n", #cond, __LINE__);        \
            bad = 1;                                                   \
        }                                                              \
    } while (0)

static mpfc_params params(void) {
    mpfc_params p;
    memset(&p, 0, sizeof p);
    p.eps = 0.025; p.beta = 0.9; p.M = 1.0; p.h = 0.785398; p.dt = 0.05; p.scheme = 2; p.bc = 0;
    return p;
}

int main(void) {
    mpfc_opts o;
    mpfc_params p = params();
    mpfc_default_opts(&o);
    EXPECT(mpfc_version() == MPFC_VERSION);
    for (int c = 0; c >= -6; --c) EXPECT(mpfc_strerror(c) && strlen(mpfc_strerror(c)) > 0);
    EXPECT(strcmp(mpfc_strerror(-99), "unknown error") == 0);

    /* grid sizes */
    EXPECT(mpfc_validate(1024, 1024, &p, &o) == MPFC_OK);
    EXPECT(mpfc_validate(2048, 1024, &p, &o) == MPFC_OK);
    EXPECT(mpfc_validate(512, 400, &p, &o) == MPFC_OK);
    EXPECT(mpfc_validate(8, 8, &p, &o) == MPFC_OK);
    EXPECT(mpfc_validate(0, 64, &p, &o) == MPFC_EINVAL);
    EXPECT(mpfc_validate(64, -4, &p, &o) == MPFC_EINVAL);
    EXPECT(mpfc_validate(63, 64, &p, &o) == MPFC_EINVAL);
    EXPECT(mpfc_validate(1 << 30, 1 << 30, &p, &o) == MPFC_EINVAL);
    EXPECT(mpfc_validate(64, 64, NULL, &o) == MPFC_EINVAL);
    EXPECT(mpfc_validate(64, 64, &p, NULL) == MPFC_EINVAL);

    /* parameters */
    const double bad_values[] = {0.0, -1.0, NAN, INFINITY};
    for (int k = 0; k < 4; ++k) {
        mpfc_params q = params(); q.h = bad_values[k];
        EXPECT(mpfc_validate(64, 64, &q, &o) == MPFC_EINVAL);
        q = params(); q.dt = bad_values[k];
        EXPECT(mpfc_validate(64, 64, &q, &o) == MPFC_EINVAL);
        q = params(); q.M = bad_values[k];
        EXPECT(mpfc_validate(64, 64, &q, &o) == MPFC_EINVAL);
    }
    { mpfc_params q = params(); q.scheme = 3; EXPECT(mpfc_validate(64, 64, &q, &o) == MPFC_EINVAL); }
    { mpfc_params q = params(); q.eps = 1.5; EXPECT(mpfc_validate(64, 64, &q, &o) == MPFC_EINVAL); }
    { mpfc_params q = params(); q.beta = -0.1; EXPECT(mpfc_validate(64, 64, &q, &o) == MPFC_EINVAL); }
    { mpfc_params q = params(); q.bc = 4; EXPECT(mpfc_validate(64, 64, &q, &o) == MPFC_EINVAL); }
    { mpfc_params q = params(); q.bc = MPFC_BC_NEUMANN_Y; EXPECT(mpfc_validate(64, 64, &q, &o) == MPFC_OK); }

    /* options */
    { mpfc_opts q = o; q.nu1 = 5; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.nu2 = -1; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.tol = 0.0; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.tol = NAN; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.max_cycles = 0; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.precision = 7; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.guess = 9; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.coarsest = 4; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.coarse_sweeps = 65; EXPECT(mpfc_validate(512, 400, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.precision = MPFC_MIXED; EXPECT(mpfc_validate(512, 400, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.precision = MPFC_MIXED; EXPECT(mpfc_validate(512, 512, &p, &q) == MPFC_OK); }
    { mpfc_opts q = o; q.omega = 0.0; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.omega = 2.0; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.omega = NAN; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_EINVAL); }
    { mpfc_opts q = o; q.omega = 0.8; EXPECT(mpfc_validate(64, 64, &p, &q) == MPFC_OK); }
    { mpfc_opts q = o; q.omega = 0.8; EXPECT(mpfc3d_validate(64, 64, 64, &p, &q) == MPFC_EINVAL); }

    /* three dimensions */
    EXPECT(mpfc3d_validate(64, 64, 64, &p, &o) == MPFC_OK);
    EXPECT(mpfc3d_validate(64, 64, 63, &p, &o) == MPFC_EINVAL);
    EXPECT(mpfc3d_validate(64, 64, 64, NULL, &o) == MPFC_EINVAL);

    /* creation rejected on the host, before any HIP call */
    {
        mpfc_ctx *ctx = (mpfc_ctx *)&o;
        mpfc_params q = params(); q.dt = -1.0;
        EXPECT(mpfc_create(&ctx, 64, 64, &q, &o, NULL) == MPFC_EINVAL);
        EXPECT(ctx == NULL);
        EXPECT(strstr(mpfc_last_error(), "dt") != NULL);
        EXPECT(mpfc_create(NULL, 64, 64, &p, &o, NULL) == MPFC_EINVAL);
        mpfc3d_ctx *c3 = NULL;
        EXPECT(mpfc3d_create(&c3, 64, 64, 63, &p, &o, NULL) == MPFC_EINVAL && c3 == NULL);
        mpfc_batch *b = NULL;
        mpfc_sim_desc d[2];
        d[0].m = 64; d[0].n = 64; d[0].p = p;
        d[1].m = 64; d[1].n = 64; d[1].p = p; d[1].p.scheme = 1;  /* schemes differ */
        EXPECT(mpfc_batch_create(&b, 2, d, &o, NULL) == MPFC_EINVAL && b == NULL);
        EXPECT(mpfc_batch_create(&b, 0, d, &o, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_batch_create(&b, MPFC_BATCH_MAX + 1, d, &o, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_batch_create(&b, 1, NULL, &o, NULL) == MPFC_EINVAL);
    }

    /* NULL handles */
    {
        double x[4] = {0, 0, 0, 0};
        mpfc_info info;
        EXPECT(mpfc_step(NULL, x, x, x, x + 1, NULL, NULL, &info) == MPFC_EINVAL);
        EXPECT(mpfc_energies(NULL, x, x, x, x) == MPFC_EINVAL);
        EXPECT(mpfc_set_pinning(NULL, x, x) == MPFC_EINVAL);
        EXPECT(mpfc_prof_enable(NULL, 1) == MPFC_EINVAL);
        EXPECT(mpfc_tile_shape(NULL, 0, 0, NULL, NULL, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_cnn_load(NULL, NULL, 0) == MPFC_EINVAL);
        EXPECT(mpfc_cnn_counts(NULL, NULL, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_cnn_predict(NULL, NULL, NULL, NULL, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_cnn_trainer_set_lr(NULL, 0.1f) == MPFC_EINVAL);
        EXPECT(mpfc_cnn_trainer_blob(NULL, NULL, 0) == MPFC_EINVAL);
        EXPECT(mpfc_cnn_trainer_create(NULL, 64, 64, 1, NULL, 0, NULL, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_cnn_blob_size() > 0);
        EXPECT(mpfc_batch_size(NULL) == 0);
        EXPECT(mpfc_batch_step(NULL, NULL, NULL, NULL, NULL, NULL) == MPFC_EINVAL);
        EXPECT(mpfc3d_step(NULL, x, x, x, x + 1, NULL, NULL, &info) == MPFC_EINVAL);
        EXPECT(mpfc3d_prof_enable(NULL, 1) == MPFC_EINVAL);
        mpfc_destroy(NULL);
        mpfc3d_destroy(NULL);
        mpfc_batch_destroy(NULL);
        mpfc_cnn_trainer_destroy(NULL);
    }

    /* operator entry points: argument checks before any launch */
    {
        double *z = NULL, x[4] = {0, 0, 0, 0};
        mpfc_params q = params(); q.h = -1.0;
        EXPECT(mpfc_op_smooth(&q, MPFC_NEWTON, 64, 64, x, x, x, x, x, x, x, 1, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_op_smooth(&p, 5, 64, 64, x, x, x, x, x, x, x, 1, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_op_smooth(&p, MPFC_NEWTON, 63, 64, x, x, x, x, x, x, x, 1, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_op_smooth(&p, MPFC_NEWTON, 64, 64, z, x, x, x, x, x, x, 1, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_op_smooth_noalloc(&p, MPFC_NEWTON, 1024, 1024, x, x, x, x, x, x, x, 1, NULL)
               == MPFC_EINVAL);
        EXPECT(mpfc_op_smooth_noalloc(&p, MPFC_NEWTON, 64, 64, x, x, x, x, x, x, x, -1, NULL)
               == MPFC_EINVAL);
        EXPECT(mpfc_op_residual(&q, 64, 64, x, x, x, x, x, x, x, x, x, x, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_op_residual(&p, 64, 64, x, x, x, x, x, x, x, z, x, x, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_op_source(&p, 64, 64, x, x, z, x, x, x, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_op_source(&p, 3, 64, x, x, x, x, x, x, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_op_restrict(64, 65, x, x, NULL) == MPFC_EINVAL);
        EXPECT(mpfc_op_restrict(64, 64, x, z, NULL) == MPFC_EINVAL);
        EXPECT(strlen(mpfc_last_error()) > 0);
    }
    if (bad) return 1;
    printf("abi driver ok\n");
    return 0;
}
