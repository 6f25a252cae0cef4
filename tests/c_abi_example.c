/* A C program that drives the library through include/sdc.h alone: the
 * trajectory of an 8x8x8 sc antiferromagnet (seeded uniform start, LL RK4),
 * one split-BF16 plan, the finalised outputs, and checks of values the
 * method fixes: every displacement of a periodic box holds exactly N ordered
 * pairs, C(0, 0) = 1 for unit spins (within the split form's bound), the
 * FP64 self term at lag 0 is 1.  Exit status 0 when all hold. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "sdc.h"

#define CHECK(x)                                                                                  \
    do {                                                                                          \
        sdc_status s_ = (x);                                                                      \
        if (s_ != SDC_OK) {                                                                       \
            fprintf(stderr, "%s: %s (%s)\n", #x, sdc_status_string(s_), sdc_last_error());        \
            return 1;                                                                             \
        }                                                                                         \
    } while (0)

enum { L = 8, N = L * L * L, NO = 16, NL = 32, T = NO + NL - 1 };

int main(void) {
    static float pos[3 * N];
    for (int x = 0; x < L; ++x)
        for (int y = 0; y < L; ++y)
            for (int z = 0; z < L; ++z) {
                const int i = (x * L + y) * L + z;
                pos[3 * i] = (float)x;
                pos[3 * i + 1] = (float)y;
                pos[3 * i + 2] = (float)z;
            }
    sdc_traj_spec ts = {0};
    ts.kind = SDC_BINS_PERIODIC_SC;
    ts.cells[0] = ts.cells[1] = ts.cells[2] = L;
    ts.coupling = SDC_COUPLING_NN_UNIFORM;
    ts.J = 1.0;
    ts.dt = 0.01;
    ts.init = SDC_INIT_UNIFORM;
    ts.seed = 7;
    float* frames = NULL;
    if (hipMalloc((void**)&frames, sizeof(float) * 3 * (size_t)N * T) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    CHECK(sdc_traj_generate(pos, N, &ts, frames, T, 0, NULL));

    sdc_bin_spec bs = {SDC_BINS_PERIODIC_SC, {L, L, L}, 0, 0.0f};
    sdc_corr_spec cs = {NO, NL, 1, SDC_PREC_SPLIT_BF16, 0};
    sdc_plan* plan = NULL;
    CHECK(sdc_plan_create(pos, N, &bs, &cs, 0, &plan));
    int64_t nb = 0;
    CHECK(sdc_plan_n_bins(plan, &nb));
    CHECK(sdc_accumulate(plan, frames, T, NULL, 0, NULL));
    double* C = malloc(sizeof(double) * NL * (size_t)nb);
    uint64_t* count = malloc(sizeof(uint64_t) * (size_t)nb);
    double csum[NL], cself[NL];
    if (!C || !count) return 1;
    CHECK(sdc_finalize(plan, C, count, csum, cself, NULL, NULL, NULL));

    int bad = 0;
    if (nb != N) {
        fprintf(stderr, "n_bins %lld, expected %d\n", (long long)nb, N);
        bad = 1;
    }
    for (int64_t b = 0; b < nb; ++b)
        if (count[b] != (uint64_t)N) {
            fprintf(stderr, "count[%lld] = %llu, expected %d\n", (long long)b, (unsigned long long)count[b], N);
            bad = 1;
            break;
        }
    for (int64_t x = 0; x < (int64_t)NL * nb; ++x)
        if (!isfinite(C[x])) {
            fprintf(stderr, "C not finite at %lld\n", (long long)x);
            bad = 1;
            break;
        }
    /* bin 0 is the zero displacement; 4.6e-5 is the split-BF16 bound per product */
    if (fabs(C[0] - 1.0) > 1e-4) {
        fprintf(stderr, "C(0, 0) = %.9f\n", C[0]);
        bad = 1;
    }
    if (fabs(cself[0] - 1.0) > 1e-6) {
        fprintf(stderr, "Cself(0) = %.12f\n", cself[0]);
        bad = 1;
    }
    printf("c abi example: N=%d, %lld bins, C(0,0)=%.9f, Cself(0)=%.12f, Csum(0)=%.6e: %s\n", N, (long long)nb, C[0],
           cself[0], csum[0], bad ? "FAILED" : "ok");
    CHECK(sdc_plan_destroy(plan));
    free(C);
    free(count);
    if (hipFree(frames) != hipSuccess) return 1;
    return bad;
}
