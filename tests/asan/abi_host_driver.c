/* Host-only exercise of the C ABI for a sanitizer build (no GPU needed): options, plan creation
 * and validation errors, batch plans, region-mode plans, workspace sizes, the launch-bounds
 * check, the allocation-free entry point's host-side rejections, status strings, destruction.
 * Every path that touches device memory is left out. Exit status 0 when every call returned
 * what the header documents. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ptsolve.h"

static int failures = 0;
#define EXPECT(cond)                                                         \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "FAILED line %d: %s (%s)\n", __LINE__, #cond, pt_last_error()); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

static pt_problem base_problem(int n, int N) {
    pt_problem p;
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.N = N;
    p.T = 1.0;
    p.sigma_in = 1.0;
    p.sigma_rect = (pt_rect){0.25, 0.25, 0.75, 0.75};
    p.nu_a = 1.0;
    p.nu_b = 9.0;
    p.nu_out = 1.0;
    p.nu_rect = (pt_rect){0.3, 0.05, 0.7, 0.95};
    p.J0 = 10.0;
    p.coil_rect = (pt_rect){0.1, 0.3, 0.2, 0.7};
    p.waveform = PT_WAVE_SIN;
    p.nu_max = 10.0;
    return p;
}

int main(void) {
    pt_options o;
    pt_options_default(&o);
    char msg[256];
    for (int prec = 0; prec < 2; ++prec) {
        for (int inner = 0; inner < 2; ++inner) {
            pt_problem p = base_problem(64, 64);
            o.precision = prec;
            o.inner = inner;
            o.inner_iters = inner ? 4 : 1;
            pt_plan* plan = NULL;
            EXPECT(pt_plan_create(&p, &o, &plan) == PT_OK && plan);
            size_t bytes = 0;
            EXPECT(pt_plan_workspace_bytes(plan, &bytes) == PT_OK && bytes > 0);
            EXPECT(pt_plan_check_bounds(plan, msg, sizeof(msg)) == PT_OK);
            int32_t count = 0;
            EXPECT(pt_plan_batch_size(plan, &count) == PT_OK && count == 1);
            pt_plan_destroy(plan);
        }
    }
    /* invalid problems and options are rejected with a message, and nothing leaks */
    {
        pt_problem p = base_problem(30, 64);
        pt_plan* plan = (pt_plan*)1;
        pt_options_default(&o);
        EXPECT(pt_plan_create(&p, &o, &plan) == PT_ERR_INVALID && plan == NULL && strlen(pt_last_error()) > 0);
        p = base_problem(32, 32);
        o.tol = 0.0;
        EXPECT(pt_plan_create(&p, &o, &plan) == PT_ERR_INVALID);
        pt_options_default(&o);
        o.inner_rtol = 2.0;
        EXPECT(pt_plan_create(&p, &o, &plan) == PT_ERR_INVALID);
    }
    /* batches of up to 64 instances */
    {
        pt_options_default(&o);
        pt_problem ps[64];
        for (int b = 0; b < 64; ++b) {
            ps[b] = base_problem(32, 64);
            ps[b].J0 = 1.0 + b;
        }
        pt_plan* plan = NULL;
        EXPECT(pt_plan_create_batch(ps, 64, &o, &plan) == PT_OK);
        EXPECT(pt_plan_check_bounds(plan, msg, sizeof(msg)) == PT_OK);
        pt_plan_destroy(plan);
        ps[3].n = 64; /* instances must share the grid */
        EXPECT(pt_plan_create_batch(ps, 64, &o, &plan) == PT_ERR_INVALID);
        EXPECT(pt_plan_create_batch(ps, 3, &o, &plan) == PT_ERR_INVALID);
    }
    /* region mode with the exp-capped law: the plan copies the caller's region array */
    {
        pt_region* regs = (pt_region*)malloc(2 * sizeof(pt_region));
        regs[0] = (pt_region){0.0, 0.0, 0.0, 1.0, 795774.7, 0.0};
        regs[1] = (pt_region){1e7, 5.85, 2.196, 136026.0, 23.15, 1.9e4};
        pt_problem p = base_problem(32, 16);
        p.law = PT_NU_EXPCAP;
        p.nregions = 2;
        p.d_region = (const uint8_t*)regs; /* never dereferenced by plan creation */
        p.regions = regs;
        pt_options_default(&o);
        pt_plan* plan = NULL;
        EXPECT(pt_plan_create(&p, &o, &plan) == PT_OK);
        free(regs); /* the plan holds its own copy */
        EXPECT(pt_plan_check_bounds(plan, msg, sizeof(msg)) == PT_OK);
        pt_plan_destroy(plan);
        p = base_problem(32, 16);
        p.law = PT_NU_EXPCAP; /* the exp-capped law needs regions */
        EXPECT(pt_plan_create(&p, &o, &plan) == PT_ERR_INVALID);
    }
    /* the allocation-free solve rejects plans above its scratch size before touching d_u */
    {
        pt_problem p = base_problem(256, 64);
        pt_options_default(&o);
        pt_plan* plan = NULL;
        double dummy = 0.0;
        EXPECT(pt_plan_create(&p, &o, &plan) == PT_OK);
        EXPECT(pt_solve_noalloc(plan, &dummy, NULL, NULL) == PT_ERR_WORKSPACE);
        pt_plan_destroy(plan);
    }
    EXPECT(strcmp(pt_status_string(PT_ERR_BREAKDOWN), "PT_ERR_BREAKDOWN") == 0);
    EXPECT(pt_kernel_class_name(PT_KERNEL_CLASSES) == NULL);
    pt_plan_destroy(NULL);
    if (failures) fprintf(stderr, "%d check(s) failed\n", failures);
    else printf("abi host driver: all checks passed\n");
    return failures ? 1 : 0;
}
