/* A C program that uses libsuppcg through its C ABI only (no Python, no
 * PyTorch): device memory from the HIP runtime, a 64 x 64 disk phantom, R and
 * R^T of it, then 10 loop bodies of SupPCG (K = 1, a = gamma = 0.5, the
 * ramp-Hamming preconditioner with mu = 1e-5, rho = 0.8) from x0 = 0 with the
 * disk's data.  Writes R x [90][91], R^T R x [64][64] and x_{k-1/2} [64][64]
 * as float32 to the file named by argv[1] and prints k and the status. */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "suppcg.h"

#define HIP_OK(expr)                                                              \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s: %s\n", #expr, hipGetErrorString(e_));           \
            return 2;                                                             \
        }                                                                         \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s OUT\n", argv[0]);
        return 1;
    }
    const int rows = 64, cols = 64, A = 90, B = 91;
    const size_t n = (size_t)rows * cols, m = (size_t)A * B;
    sp_geometry g = {rows, cols, 1.0, A, 0.0, -1.0, B, 1.0, 0.0};
    float* hx = (float*)malloc(n * sizeof(float));
    float* hout = (float*)malloc((m + 2 * n) * sizeof(float));
    if (!hx || !hout) return 2;
    for (int i = 0; i < rows; ++i)
        for (int j = 0; j < cols; ++j) {
            const double y = 31.5 - i, x = j - 31.5;
            hx[i * cols + j] = (x * x + y * y <= 20.0 * 20.0) ? 1.0f : 0.0f;
        }
    float *dx, *dy, *dg, *dxh;
    HIP_OK(hipMalloc((void**)&dx, n * sizeof(float)));
    HIP_OK(hipMalloc((void**)&dy, m * sizeof(float)));
    HIP_OK(hipMalloc((void**)&dg, n * sizeof(float)));
    HIP_OK(hipMalloc((void**)&dxh, n * sizeof(float)));
    HIP_OK(hipMemcpy(dx, hx, n * sizeof(float), hipMemcpyHostToDevice));

    sp_ctx* ctx = NULL;
    int rc = sp_ctx_create(0, NULL, &ctx);
    if (rc != SP_OK) {
        fprintf(stderr, "sp_ctx_create: %d\n", rc);
        return 3;
    }
    if ((rc = sp_project(ctx, &g, dx, dy)) != SP_OK || (rc = sp_backproject(ctx, &g, dy, dg)) != SP_OK) {
        fprintf(stderr, "operators: %d %s\n", rc, sp_ctx_last_error(ctx));
        return 3;
    }
    sp_tv_params tv = {1, 0.5, 0.5, 0};
    sp_precond pc = {SP_PRECOND_RAMP, 1e-5, 0.8, NULL};
    sp_solve_params sp = {0.0, 10, SP_FLAG_GRAPH, NULL};
    int32_t k = 0;
    rc = sp_suppcg_solve(ctx, &g, dy, NULL, &tv, &pc, &sp, dxh, NULL, &k, NULL);
    if (rc != SP_MAXITER) {
        fprintf(stderr, "sp_suppcg_solve: %d %s\n", rc, sp_ctx_last_error(ctx));
        return 3;
    }
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(hout, dy, m * sizeof(float), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hout + m, dg, n * sizeof(float), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hout + m + n, dxh, n * sizeof(float), hipMemcpyDeviceToHost));
    FILE* f = fopen(argv[1], "wb");
    if (!f || fwrite(hout, sizeof(float), m + 2 * n, f) != m + 2 * n) return 4;
    fclose(f);
    printf("k %d status %d\n", (int)k, rc);
    sp_ctx_destroy(ctx);
    hipFree(dx);
    hipFree(dy);
    hipFree(dg);
    hipFree(dxh);
    free(hx);
    free(hout);
    return 0;
}
