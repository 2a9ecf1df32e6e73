/*
 * c_client.c -- a plain C program that uses the integrator through its C
 * ABI only (no Python, no torch): it allocates the device arena itself,
 * initialises the library with a serving stream, integrates the 4-D Gaussian
 * synchronously, submits the same request to the serving thread, and prints
 * both results.
 *
 * Output (one line each):  sync <integral> <std> <levels> <samples>
 *                          served <integral> <std> <levels> <samples>
 * Exit status 0 on success, 1 on any library or HIP error.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <string.h>

#include "zmc.h"

static int check(int rc, const char* what)
{
    if (rc != ZMC_OK) {
        fprintf(stderr, "%s: %d (%s)\n", what, rc, zmc_strerror(rc));
        return 1;
    }
    return 0;
}

int main(void)
{
    const size_t arena_bytes = (size_t)256 << 20;
    void* arena = NULL;
    hipStream_t st = NULL;
    if (hipMalloc(&arena, arena_bytes) != hipSuccess || hipStreamCreate(&st) != hipSuccess) {
        fprintf(stderr, "HIP allocation failed\n");
        return 1;
    }
    zmc_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.arena = arena;
    cfg.arena_bytes = arena_bytes;
    cfg.serve_stream = st;
    if (check(zmc_init(&cfg), "zmc_init")) return 1;

    /* exp(-|x|^2 / (2 * 0.2^2)) on [-1,1]^4, 4 divisions per axis, 4096
     * points per cube, 5 trials, one refinement, sigma 1, seed 1, FP64 */
    const double params[6] = {0.2, 1.0, 0.0, 0.0, 0.0, 0.0};
    const double lower[4] = {-1.0, -1.0, -1.0, -1.0};
    const double upper[4] = {1.0, 1.0, 1.0, 1.0};
    zmc_result r;
    /* cfg.default_eval = 0: FP64 evaluation */
    if (check(zmc_integrate(ZMC_GAUSS, params, 4, lower, upper, 4, 4096, 5, 1, 1.0, 1, NULL, &r), "zmc_integrate"))
        return 1;
    printf("sync %.17g %.17g %d %llu\n", r.integral, r.std, r.levels_run, (unsigned long long)r.n_samples);

    zmc_request q;
    memset(&q, 0, sizeof(q));
    q.integrand = ZMC_GAUSS;
    q.dim = 4;
    q.divisions_per_axis = 4;
    q.trials = 5;
    q.max_depth = 1;
    q.eval = ZMC_EVAL_FP64;
    q.n_params = 6;
    q.samples_per_cube = 4096;
    q.sigma_mult = 1.0;
    q.seed = 1;
    for (int i = 0; i < 4; ++i) {
        q.lower[i] = lower[i];
        q.upper[i] = upper[i];
    }
    for (int j = 0; j < 6; ++j) q.params[j] = params[j];
    uint64_t ticket = 0;
    if (check(zmc_submit(&q, &ticket), "zmc_submit")) return 1;
    zmc_result s;
    if (check(zmc_poll(ticket, &s, 1), "zmc_poll")) return 1;
    printf("served %.17g %.17g %d %llu\n", s.integral, s.std, s.levels_run, (unsigned long long)s.n_samples);

    if (check(zmc_shutdown(), "zmc_shutdown")) return 1;
    (void)hipStreamDestroy(st);
    (void)hipFree(arena);
    return 0;
}
