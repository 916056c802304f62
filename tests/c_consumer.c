/*
 * A plain C99 consumer of the library's C ABI (include/gracedg.h), used by
 * tests/test_c_consumer.py.  It builds a collision tensor (ballistic kernel,
 * power-law fragmentation, 8 bins, order 2, conservative flux on [1e-4, 1e8]),
 * prints its sizes, checks that an invalid order is rejected, and with the
 * argument "gpu" evaluates the right-hand side of three cells on the device
 * (HIP runtime API from C) and prints their raw flux vectors.
 *
 * The states are g_{c,j,0} = 1 / (1 + j + c) and g_{c,j,i} = 0.05 i / (1 + j) for
 * i >= 1; the test evaluates the same states with the oracle.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gracedg.h"

#define BINS 8
#define ORDER 2
#define CELLS 3

static int run_gpu(const gd_tensor* t, int n_out)
{
    const int P = BINS * (ORDER + 1);
    double g[CELLS * P];
    for (int c = 0; c < CELLS; ++c)
        for (int j = 0; j < BINS; ++j)
            for (int i = 0; i <= ORDER; ++i)
                g[c * P + j * (ORDER + 1) + i] = i == 0 ? 1.0 / (1 + j + c) : 0.05 * i / (1 + j);
    const int cells = CELLS;
    gd_plan* plan = NULL;
    if (gd_plan_create(&t, &cells, 1, GD_PREC_FP64, NULL, NULL, &plan) != GD_OK) {
        fprintf(stderr, "plan: %s\n", gd_last_error());
        return 1;
    }
    double *dg = NULL, *drhs = NULL, *draw = NULL;
    if (hipMalloc((void**)&dg, sizeof g) != hipSuccess || hipMalloc((void**)&drhs, sizeof g) != hipSuccess ||
        hipMalloc((void**)&draw, sizeof(double) * CELLS * n_out) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    if (hipMemcpy(dg, g, sizeof g, hipMemcpyHostToDevice) != hipSuccess) return 1;
    if (gd_collision_rhs(plan, dg, NULL, drhs, draw) != GD_OK) {
        fprintf(stderr, "rhs: %s\n", gd_last_error());
        return 1;
    }
    double* raw = malloc(sizeof(double) * CELLS * n_out);
    if (!raw || hipMemcpy(raw, draw, sizeof(double) * CELLS * n_out, hipMemcpyDeviceToHost) != hipSuccess) return 1;
    for (int c = 0; c < CELLS; ++c) {
        printf("raw");
        for (int o = 0; o < n_out; ++o) printf(" %.17g", raw[c * n_out + o]);
        printf("\n");
    }
    free(raw);
    (void)hipFree(dg);
    (void)hipFree(drhs);
    (void)hipFree(draw);
    gd_plan_destroy(plan);
    return 0;
}

int main(int argc, char** argv)
{
    const gd_kernel kernel = {GD_KERNEL_BALLISTIC, 1.0, 0.0};
    const double levels[1] = {0.5};
    const gd_frag_law frag = {GD_FRAG_POWERLAW, -11.0 / 6.0, 1, levels};
    const gd_grid grid = {1e-4, 1e8, 1, 0};
    gd_tensor* t = NULL;
    if (gd_init_tensor(&kernel, &frag, BINS, ORDER, &grid, &t) != GD_OK) {
        fprintf(stderr, "init: %s\n", gd_last_error());
        return 1;
    }
    gd_tensor_info_t info;
    if (gd_tensor_info(t, &info) != GD_OK) return 1;
    printf("info %d %d %lld\n", info.P, info.n_out, info.nnz_folded);
    gd_tensor* bad = NULL;
    const int rc = gd_init_tensor(&kernel, &frag, BINS, 5, &grid, &bad);
    printf("invalid %d %s\n", rc, gd_last_error());
    int status = 0;
    if (argc > 1 && strcmp(argv[1], "gpu") == 0) status = run_gpu(t, info.n_out);
    gd_free_tensor(t);
    return status;
}
