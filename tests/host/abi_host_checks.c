/* Host-side checks of the libtm C ABI that need no GPU: status strings, argument validation before any
 * device work, workspace size formulas, NULL contexts.  Built and run under AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only) by tests/test_host_sanitizers.py; exits non-zero on the
 * first failed check. */
#include <stdio.h>
#include <string.h>

#include "tm.h"

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static tm_problem base_problem(void) {
    tm_problem p;
    memset(&p, 0, sizeof p);
    p.n_species = 4;
    p.n_rays = 10;
    p.n_zones = 540;
    p.n_groups = 20;
    p.c_dt = 3e4;
    p.inner_bc = TM_BC_ZERO_FLUX;
    p.outer_bc = TM_BC_FREE_STREAM;
    p.terms = TM_TERMS_ALL;
    p.limiter = TM_LIMITER_INTRP;
    p.psi_floor = 1e-300;
    p.precision = TM_PREC_FP64;
    return p;
}

int main(void) {
    /* status strings, including an unknown code */
    for (int s = 0; s <= 6; ++s) CHECK(strncmp(tm_status_string((tm_status)s), "TM_", 3) == 0);
    CHECK(strcmp(tm_status_string((tm_status)42), "TM_UNKNOWN_STATUS") == 0);
    CHECK(strcmp(tm_last_error(NULL), "context is NULL") == 0);

    /* invalid problems are rejected before any device work */
    tm_ctx* h = (tm_ctx*)0x1;
    CHECK(tm_create(NULL, NULL, &h) == TM_ERR_INVALID_ARG && h == NULL);
    tm_problem p = base_problem();
    CHECK(tm_create(&p, NULL, NULL) == TM_ERR_INVALID_ARG);
    tm_problem bad[12];
    for (int j = 0; j < 12; ++j) bad[j] = base_problem();
    bad[0].n_groups = 0;
    bad[1].n_groups = 33;
    bad[2].n_zones = 0;
    bad[3].n_rays = 0;
    bad[4].n_species = 0;
    bad[5].c_dt = 0.0;
    bad[6].c_dt = -1.0;
    bad[7].outer_bc = 7;
    bad[8].terms = 8u;
    bad[9].limiter = 3;
    bad[10].psi_floor = 0.0;
    bad[11].precision = 3;
    for (int j = 0; j < 12; ++j) {
        h = (tm_ctx*)0x1;
        CHECK(tm_create(&bad[j], NULL, &h) == TM_ERR_INVALID_ARG && h == NULL);
        CHECK(tm_workspace_bytes(&bad[j], 0) == 0);
        CHECK(tm_ye_workspace_bytes(&bad[j], 0) == 0);
    }
    tm_problem huge = base_problem();
    huge.n_species = 1 << 20;
    huge.n_rays = 1 << 20;                     /* 2^40 systems: beyond the supported count */
    CHECK(tm_workspace_bytes(&huge, 0) == 0);

    /* workspace formulas: (b + 15) slots of I * NT * (NT + 1) values; coupled: b slots of I (2NT+1)^2 doubles */
    CHECK(tm_workspace_bytes(&p, 0) == (size_t)(40 + 15) * 540 * 20 * 21 * 8);
    CHECK(tm_workspace_bytes(&p, 3) == (size_t)(3 + 15) * 540 * 20 * 21 * 8);
    CHECK(tm_workspace_bytes(&p, -1) == 0);
    CHECK(tm_ye_workspace_bytes(&p, 0) == (size_t)10 * 540 * (41 * 41 + 1) * 8);
    tm_problem pm = base_problem();
    pm.n_groups = 13;
    pm.precision = TM_PREC_MIXED;
    CHECK(tm_workspace_bytes(&pm, 1) == (size_t)(1 + 15) * 540 * 16 * 17 * 4);

    /* every entry point rejects a NULL context */
    CHECK(tm_destroy(NULL) == TM_ERR_INVALID_ARG);
    CHECK(tm_set_workspace(NULL, NULL, 0) == TM_ERR_INVALID_ARG);
    CHECK(tm_assemble(NULL, NULL, NULL, NULL, NULL, NULL) == TM_ERR_INVALID_ARG);
    CHECK(tm_factor_solve(NULL, NULL, NULL, NULL, NULL, 0) == TM_ERR_INVALID_ARG);
    CHECK(tm_newton_step(NULL, NULL, NULL, NULL, 1, 0.0, NULL) == TM_ERR_INVALID_ARG);
    CHECK(tm_adjoint_step(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == TM_ERR_INVALID_ARG);
    CHECK(tm_luminosity_seed(NULL, NULL, NULL, NULL) == TM_ERR_INVALID_ARG);
    CHECK(tm_ye_newton_step(NULL, NULL, NULL, NULL, NULL, NULL, 1, 0.0, NULL) == TM_ERR_INVALID_ARG);
    CHECK(tm_temperature_update(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == TM_ERR_INVALID_ARG);
    CHECK(tm_energy_advect(NULL, NULL, NULL, NULL, NULL, NULL) == TM_ERR_INVALID_ARG);

    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("abi host checks passed\n");
    return 0;
}
