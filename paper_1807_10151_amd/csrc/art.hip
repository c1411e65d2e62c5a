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
// pixel basis uses the weights of the stored matrices (stored_weight);
// BlobART (blob basis) uses the projection of a Kaiser-Bessel blob centred on
// each pixel centre at the ray's distance from that centre, and the image is
// the blobs' sum sampled at the pixel centres.
#include <algorithm>
#include <cmath>

#include "sp_blob.h"
#include "sp_internal.h"
#include "sp_reduce.h"
#include "sp_stored.h"

namespace sp {

// ---- blob basis -----------------------------------------------------------------
BlobDev blob_constants() {
    BlobDev B{};
    B.a = BLOB_RADIUS;
    B.alpha = BLOB_ALPHA;
    B.ntab = BLOB_TAB_N;
    B.inv_h = BLOB_TAB_N / B.a;
    const double i2a = blob_bessel_i(2.0, B.alpha);
    B.cproj = B.a * std::sqrt(2.0 * M_PI / B.alpha) / i2a;
    for (int di = -2; di <= 2; ++di)
        for (int dj = -2; dj <= 2; ++dj) {
            const double r = std::sqrt((double)(di * di + dj * dj));
            const double t = 1.0 - (r / B.a) * (r / B.a);
            double v = 0.0;
            if (t > 0.0) {
                const double w = std::sqrt(t);
                v = w * w * blob_bessel_i(2.0, B.alpha * w) / i2a;
            }
            B.stencil[di + 2][dj + 2] = v;
        }
    return B;
}

// p(d): the integral of the blob along a line at distance d (pixel units),
// from its table (sp_blob.h).
__device__ __forceinline__ double blob_proj(const BlobDev& B, double d) {
    return blob_interp(B.tab, B.ntab, B.inv_h, d);
}

// The blobs met by ray k of angle A on major line m (their centres on that
// image row or column within the blob radius of the ray), in increasing
// order, with weight p(d) times the pixel size.
template <class F>
__device__ __forceinline__ void blob_line_nonzeros(const GeomDev& G, const AngleDev& A, const BlobDev& B,
                                                   double sk, int m, F&& emit) {
    if (!(A.flags & ANG_HORIZ)) {
        const double hw = B.a / fabs(A.c);
        const double yi = G.yoff - (double)m;
        const double xs = (sk - yi * A.s) / A.c + G.xoff;
        const int lo = imax((int)floor(xs - hw) - 1, 0);
        const int hi = imin((int)ceil(xs + hw) + 1, G.cols - 1);
        for (int j = lo; j <= hi; ++j) {
            const double xj = (double)j - G.xoff;
            const double w = blob_proj(B, sk - fma(xj, A.c, yi * A.s)) * G.pixel;
            if (w > 0.0) emit(m * G.cols + j, w);
        }
    } else {
        const double hw = B.a / fabs(A.s);
        const double xj = (double)m - G.xoff;
        const double ys = G.yoff - (sk - xj * A.c) / A.s;
        const int lo = imax((int)floor(ys - hw) - 1, 0);
        const int hi = imin((int)ceil(ys + hw) + 1, G.rows - 1);
        for (int i = lo; i <= hi; ++i) {
            const double yi = G.yoff - (double)i;
            const double w = blob_proj(B, sk - fma(yi, A.s, xj * A.c)) * G.pixel;
            if (w > 0.0) emit(i * G.cols + m, w);
        }
    }
}

// The nonzeros of ray k on line m in the chosen basis.
template <bool BLOB, class F>
__device__ __forceinline__ void basis_line_nonzeros(const GeomDev& G, const AngleDev& A, const BlobDev& B,
                                                    double sk, int m, F&& emit) {
    if (BLOB) blob_line_nonzeros(G, A, B, sk, m, emit);
    else ray_line_nonzeros(G, A, sk, m, emit);
}

// img = sum of the blobs with coefficients c, at the pixel centres.
__global__ __launch_bounds__(256) void k_blob_synth(int rows, int cols, BlobDev B, const double* __restrict__ c,
                                                    double* __restrict__ img, const int* __restrict__ halt) {
    if (halt && *halt) return;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < rows * cols; q += gridDim.x * 256) {
        const int i = q / cols, j = q - i * cols;
        double acc = 0.0;
        for (int di = -2; di <= 2; ++di) {
            const int ii = i + di;
            if (ii < 0 || ii >= rows) continue;
            for (int dj = -2; dj <= 2; ++dj) {
                const int jj = j + dj;
                if (jj < 0 || jj >= cols) continue;
                acc = fma(B.stencil[di + 2][dj + 2], c[ii * cols + jj], acc);
            }
        }
        img[q] = acc;
    }
}

void launch_blob_synth(hipStream_t st, int rows, int cols, const BlobDev& B, const double* c, double* img,
                       const int* halt) {
    hipLaunchKernelGGL(k_blob_synth, dim3(vec_blocks(rows * cols)), dim3(256), 0, st, rows, cols, B, c, img, halt);
}

// ||R_i||^2 of every ray (thread per ray, in the enumeration order).
template <bool BLOB>
__global__ __launch_bounds__(256) void k_art_norms(GeomDev G, const AngleDev* __restrict__ nat, BlobDev B,
                                                   double* __restrict__ nrm2) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= G.nA * G.nB) return;
    const AngleDev A = nat[r / G.nB];
    const double sk = bin_pos((double)(r % G.nB), G);
    const int nl = ray_lines(G, A);
    double s = 0.0;
    for (int m = 0; m < nl; ++m)
        basis_line_nonzeros<BLOB>(G, A, B, sk, m, [&](int, double w) { s = fma(w, w, s); });
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
// k = ph + q j.  Its NT threads take the ray's major lines m = t, t + NT,
// ... for <R_i, x> (summed over the workgroup in a fixed order) and then
// update those pixels.  With at most LINES lines per thread a thread keeps
// its pixels, weights and the values it read in registers (up to 6 per line;
// a band |s_k - t| < e meets at most 3 pixels of a line; 10 blobs, of at most
// 6 met) and writes x + r c w without a second walk; otherwise (LINES = 0, or
// more entries than that) it walks its lines again.  A phase holds few rays
// (nB / q workgroups), so 512 threads per ray halve each thread's chain of
// dependent weight evaluations and gathers.
template <bool BLOB, int LINES, int NT>
__global__ __launch_bounds__(NT) void k_art_phase(GeomDev G, AngleDev A, BlobDev B, int a, int ph, int q, int nr,
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
    __shared__ double red[NT / 64];
    const double sk = bin_pos((double)k, G);
    const int nl = ray_lines(G, A);
    double dot = 0.0;
    constexpr int CAP = LINES * (BLOB ? 10 : 6);
    int pp[CAP > 0 ? CAP : 1];
    double ww[CAP > 0 ? CAP : 1], xv[CAP > 0 ? CAP : 1];
    int cnt = 0;
    for (int m = threadIdx.x; m < nl; m += NT)
        basis_line_nonzeros<BLOB>(G, A, B, sk, m, [&](int p, double w) {
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
    dot = block_sum_w<NT / 64>(dot, red);
    // a ray without nonzeros (n2 = 0) gathered nothing and changes nothing; the
    // test sits after the walk so its load overlaps the gathers
    if (n2 == 0.0) return;
    const double c = lam * (r * (bi - dot) - ui) / (1.0 + r * r * n2);
    if (threadIdx.x == 0) u[i] = ui + c;
    const double rc = r * c;
    if (LINES > 0 && cnt <= CAP) {
#pragma unroll
        for (int e = 0; e < CAP; ++e)
            if (e < cnt) x[pp[e]] = fma(rc, ww[e], xv[e]);
    } else {   // (a line with more nonzeros than the registers hold: walk again)
        for (int m = threadIdx.x; m < nl; m += NT)
            basis_line_nonzeros<BLOB>(G, A, B, sk, m, [&](int p, double w) { x[p] = fma(rc, w, x[p]); });
    }
}

void launch_art_norms(hipStream_t st, const GeomDev& G, const AngleDev* nat, const BlobDev* blob, double* nrm2) {
    const int nb = (G.nA * G.nB + 255) / 256;
    const BlobDev B = blob ? *blob : BlobDev{};
    if (blob) hipLaunchKernelGGL(k_art_norms<true>, dim3(nb), dim3(256), 0, st, G, nat, B, nrm2);
    else hipLaunchKernelGGL(k_art_norms<false>, dim3(nb), dim3(256), 0, st, G, nat, B, nrm2);
}

void launch_art_init(hipStream_t st, const GeomDev& G, const float* b, const float* x0, double divisor,
                     double* partials, double* sum_b, double* x, double* u) {
    const int m = G.nA * G.nB, n = G.rows * G.cols;
    const int nb = vec_blocks(m);
    hipLaunchKernelGGL(k_sum_f, dim3(nb), dim3(256), 0, st, m, b, partials);
    launch_reduce(st, partials, nb, sum_b);
    // mu = ds * sum(b) / (A * n * pixel^2), with ds in the geometry's unit;
    // the blob basis starts at the coefficients whose image is mu (divisor:
    // the image of a unit coefficient field)
    const double coef = (G.ds * G.pixel) / ((double)G.nA * (double)n * G.pixel * G.pixel) / divisor;
    hipLaunchKernelGGL(k_art_init, dim3(vec_blocks(std::max(n, m))), dim3(256), 0, st, n, m, coef, sum_b, x0, x,
                       u);
}

int art_blob_phases(const GeomDev& G, const BlobDev& B) { return (int)std::floor(2.0 * B.a / G.ds + 1e-9) + 1; }

void launch_art_sweep(hipStream_t st, const GeomDev& G, const AngleDev* nat_h, const BlobDev* blob,
                      const double* nrm2, const float* b, double* x, double* u, double r, double lam,
                      const int* halt) {
    const BlobDev B = blob ? *blob : BlobDev{};
    for (int a = 0; a < G.nA; ++a) {
        const AngleDev& A = nat_h[a];
        const int q = blob ? art_blob_phases(G, B) : art_phases(G, A);
        constexpr int NT = 512;
        const bool regs = ray_lines(G, A) <= NT;
        for (int ph = 0; ph < q && ph < G.nB; ++ph) {
            const int nr = (G.nB - ph + q - 1) / q;
            const dim3 grid(nr), blk(NT);
            if (blob && regs)
                hipLaunchKernelGGL((k_art_phase<true, 1, NT>), grid, blk, 0, st, G, A, B, a, ph, q, nr, nrm2, b, x,
                                   u, r, lam, halt);
            else if (blob)
                hipLaunchKernelGGL((k_art_phase<true, 0, NT>), grid, blk, 0, st, G, A, B, a, ph, q, nr, nrm2, b, x,
                                   u, r, lam, halt);
            else if (regs)
                hipLaunchKernelGGL((k_art_phase<false, 1, NT>), grid, blk, 0, st, G, A, B, a, ph, q, nr, nrm2, b,
                                   x, u, r, lam, halt);
            else
                hipLaunchKernelGGL((k_art_phase<false, 0, NT>), grid, blk, 0, st, G, A, B, a, ph, q, nr, nrm2, b,
                                   x, u, r, lam, halt);
        }
    }
}

}  // namespace sp
