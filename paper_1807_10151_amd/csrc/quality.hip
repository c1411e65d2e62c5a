// The selective error SE of Section 4.2, eq. (4.1): C times the root of the
// squared difference between an image and the phantom, summed over the pixels
// whose centres lie in a centred ellipse (closed; horizontal semi-axis along a
// row).  C <= 0 selects 1 / (root of the phantom's own sum of squares over the
// same pixels), i.e. the relative error inside the ellipse.
//
// Two launches: per-workgroup float64 partial sums of (x - ref)^2 and ref^2
// in a fixed order, then one workgroup that sums them in a fixed order and
// writes SE.  Inside a solve the second launch writes the trace entry of the
// current loop body, so the pair can sit in a captured loop body.
#include "sp_internal.h"
#include "sp_reduce.h"

namespace sp {

// Whether pixel (i, j) of a rows x cols image of square pixels centred at the
// origin has its centre inside the ellipse with semi-axes (ah, av).
__device__ __forceinline__ bool in_ellipse(int i, int j, int rows, int cols, double pixel,
                                           double ah, double av) {
    const double y = ((rows - 1) * 0.5 - i) * pixel;
    const double x = (j - (cols - 1) * 0.5) * pixel;
    const double u = x / ah, v = y / av;
    return u * u + v * v <= 1.0;
}

template <class T>
__global__ __launch_bounds__(256) void k_se_partial(int rows, int cols, double pixel, double ah,
                                                    double av, const T* __restrict__ x,
                                                    const float* __restrict__ ref,
                                                    double* __restrict__ partials,
                                                    const int* __restrict__ halt) {
    if (halt && *halt) return;
    __shared__ double red[8];
    const int n = rows * cols;
    double v[2] = {0.0, 0.0};
    for (int q = blockIdx.x * 256 + threadIdx.x; q < n; q += gridDim.x * 256) {
        const int i = q / cols;
        const int j = q - i * cols;
        if (in_ellipse(i, j, rows, cols, pixel, ah, av)) {
            const double r = (double)ref[q];
            const double d = (double)x[q] - r;
            v[0] += d * d;
            v[1] += r * r;
        }
    }
    block_sum_n<2>(v, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = v[0];
        partials[2 * blockIdx.x + 1] = v[1];
    }
}

// dst_body != nullptr: write to dst_body[sc->iter - 1] (the loop body that has
// just formed its iterate) if that entry is below cap; else to *dst.
__global__ __launch_bounds__(256) void k_se_commit(const double* __restrict__ partials, int np,
                                                   double C, double* __restrict__ dst,
                                                   double* __restrict__ dst_body, int cap,
                                                   const Scalars* __restrict__ sc,
                                                   const int* __restrict__ halt) {
    if (halt && *halt) return;
    __shared__ double red[8];
    double v[2] = {0.0, 0.0};
    for (int q = threadIdx.x; q < np; q += 256) {
        v[0] += partials[2 * q];
        v[1] += partials[2 * q + 1];
    }
    block_sum_n<2>(v, red);
    if (threadIdx.x != 0) return;
    const double c = C > 0.0 ? C : 1.0 / sqrt(v[1]);
    const double se = c * sqrt(v[0]);
    if (dst_body) {
        const int it = sc->iter - 1;
        if (it >= 0 && it < cap) dst_body[it] = se;
    } else {
        *dst = se;
    }
}

template <class T>
static void launch_se_t(hipStream_t st, int rows, int cols, double pixel, double ah, double av,
                        const T* x, const float* ref, double C, double* partials, double* dst,
                        double* dst_body, int cap, const Scalars* sc, const int* halt) {
    const int nb = vec_blocks(rows * cols);
    hipLaunchKernelGGL(k_se_partial<T>, dim3(nb), dim3(256), 0, st, rows, cols, pixel, ah, av, x,
                       ref, partials, halt);
    hipLaunchKernelGGL(k_se_commit, dim3(1), dim3(256), 0, st, partials, nb, C, dst, dst_body, cap,
                       sc, halt);
}

void launch_se(hipStream_t st, int rows, int cols, double pixel, double ah, double av,
               const float* x, const float* ref, double C, double* partials, double* dst) {
    launch_se_t(st, rows, cols, pixel, ah, av, x, ref, C, partials, dst, nullptr, 0, nullptr,
                nullptr);
}

void launch_se(hipStream_t st, int rows, int cols, double pixel, double ah, double av,
               const double* x, const float* ref, double C, double* partials, double* dst,
               double* dst_body, int cap, const Scalars* sc, const int* halt) {
    launch_se_t(st, rows, cols, pixel, ah, av, x, ref, C, partials, dst, dst_body, cap, sc, halt);
}

}  // namespace sp
