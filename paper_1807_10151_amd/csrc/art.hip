// ART for the Bayesian criterion of eq. (2.3) and its superiorized form
// (Section 3.4): row projections of (x, u) onto the hyperplanes of the
// consistent system r R (x - mu) + u = r (b - R mu), one ray at a time,
//
//   c = lambda (r (b_i - <R_i, x>) - u_i) / (1 + r^2 ||R_i||^2),
//   u_i += c,   x += r c R_i^T.
//
// Rays of one angle whose bins are q apart touch disjoint pixels
// (art_phases), so the rays of one phase of one angle are projected
// concurrently, one workgroup per ray, with exactly the result of taking them one
// after another; phases and angles follow each other launch by launch.  The
// weights are those of the stored matrices (stored_weight).
#include <algorithm>

#include "sp_internal.h"
#include "sp_reduce.h"
#include "sp_stored.h"

namespace sp {

// ||R_i||^2 of every ray (thread per ray, in the enumeration order).
__global__ __launch_bounds__(256) void k_art_norms(GeomDev G, const AngleDev* __restrict__ nat,
                                                   double* __restrict__ nrm2) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= G.nA * G.nB) return;
    double s = 0.0;
    ray_nonzeros(G, nat[r / G.nB], r % G.nB, [&](int, double w) { s = fma(w, w, s); });
    nrm2[r] = s;
}

// x = mu (the data's mean gray, from the sum of b in *sum_b) and u = 0.
__global__ __launch_bounds__(256) void k_art_init(int n, int m, double coef, const double* __restrict__ sum_b,
                                                  const float* __restrict__ x0, double* __restrict__ x,
                                                  double* __restrict__ u) {
    const double mu = coef * *sum_b;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < n; q += gridDim.x * 256)
        x[q] = x0 ? (double)x0[q] : mu;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < m; q += gridDim.x * 256) u[q] = 0.0;
}

// Partial sums of b (float64) per workgroup.
__global__ __launch_bounds__(256) void k_sum_f(int m, const float* __restrict__ b, double* __restrict__ partials) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < m; q += gridDim.x * 256) acc += (double)b[q];
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// One phase of angle A (row a of the sinogram): workgroup j projects ray
// k = ph + q j.  Its 256 threads take the ray's major lines m = t, t + 256,
// ... for <R_i, x> (summed over the workgroup in a fixed order) and then
// update those pixels.  With at most two lines per thread (LINES = 2: images
// of up to 512 rows and columns) a thread keeps its pixels, weights and the
// values it read in registers (up to 6 per line; a band |s_k - t| < e meets
// at most 3 pixels of a line) and writes x + r c w without a second walk;
// otherwise (LINES = 0, or more entries than that) it walks its lines again.
template <int LINES>
__global__ __launch_bounds__(256) void k_art_phase(GeomDev G, AngleDev A, int a, int ph, int q, int nr,
                                                   const double* __restrict__ nrm2,
                                                   const float* __restrict__ b, double* __restrict__ x,
                                                   double* __restrict__ u, double r, double lam,
                                                   const int* __restrict__ halt) {
    if (halt && *halt) return;
    const int j = blockIdx.x;
    if (j >= nr) return;
    const int k = ph + q * j;
    const int i = a * G.nB + k;
    const double n2 = nrm2[i];
    const double bi = (double)b[i];
    const double ui = u[i];
    if (n2 == 0.0) return;
    __shared__ double red[4];
    const double sk = bin_pos((double)k, G);
    const int nl = ray_lines(G, A);
    double dot = 0.0;
    constexpr int CAP = LINES * 6;
    int pp[CAP > 0 ? CAP : 1];
    double ww[CAP > 0 ? CAP : 1], xv[CAP > 0 ? CAP : 1];
    int cnt = 0;
    for (int m = threadIdx.x; m < nl; m += 256)
        ray_line_nonzeros(G, A, sk, m, [&](int p, double w) {
            const double v = x[p];
            dot = fma(w, v, dot);
            if (LINES > 0) {
                if (cnt < CAP) {
                    pp[cnt] = p;
                    ww[cnt] = w;
                    xv[cnt] = v;
                }
                ++cnt;
            }
        });
    dot = block_sum(dot, red);
    const double c = lam * (r * (bi - dot) - ui) / (1.0 + r * r * n2);
    if (threadIdx.x == 0) u[i] = ui + c;
    const double rc = r * c;
    if (LINES > 0 && cnt <= CAP) {
#pragma unroll
        for (int e = 0; e < CAP; ++e)
            if (e < cnt) x[pp[e]] = fma(rc, ww[e], xv[e]);
    } else {   // (a line with more nonzeros than the registers hold: walk again)
        for (int m = threadIdx.x; m < nl; m += 256)
            ray_line_nonzeros(G, A, sk, m, [&](int p, double w) { x[p] = fma(rc, w, x[p]); });
    }
}

void launch_art_norms(hipStream_t st, const GeomDev& G, const AngleDev* nat, double* nrm2) {
    const int nb = (G.nA * G.nB + 255) / 256;
    hipLaunchKernelGGL(k_art_norms, dim3(nb), dim3(256), 0, st, G, nat, nrm2);
}

void launch_art_init(hipStream_t st, const GeomDev& G, const float* b, const float* x0, double* partials,
                     double* sum_b, double* x, double* u) {
    const int m = G.nA * G.nB, n = G.rows * G.cols;
    const int nb = vec_blocks(m);
    hipLaunchKernelGGL(k_sum_f, dim3(nb), dim3(256), 0, st, m, b, partials);
    launch_reduce(st, partials, nb, sum_b);
    // mu = ds * sum(b) / (A * n * pixel^2), with ds in the geometry's unit
    const double coef = (G.ds * G.pixel) / ((double)G.nA * (double)n * G.pixel * G.pixel);
    hipLaunchKernelGGL(k_art_init, dim3(vec_blocks(std::max(n, m))), dim3(256), 0, st, n, m, coef, sum_b, x0, x,
                       u);
}

void launch_art_sweep(hipStream_t st, const GeomDev& G, const AngleDev* nat_h, const double* nrm2,
                      const float* b, double* x, double* u, double r, double lam, const int* halt) {
    for (int a = 0; a < G.nA; ++a) {
        const AngleDev& A = nat_h[a];
        const int q = art_phases(G, A);
        for (int ph = 0; ph < q && ph < G.nB; ++ph) {
            const int nr = (G.nB - ph + q - 1) / q;
            if (ray_lines(G, A) <= 512)
                hipLaunchKernelGGL(k_art_phase<2>, dim3(nr), dim3(256), 0, st, G, A, a, ph, q, nr, nrm2, b, x, u,
                                   r, lam, halt);
            else
                hipLaunchKernelGGL(k_art_phase<0>, dim3(nr), dim3(256), 0, st, G, A, a, ph, q, nr, nrm2, b, x, u,
                                   r, lam, halt);
        }
    }
}

}  // namespace sp
