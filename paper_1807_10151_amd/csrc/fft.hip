// The paper's preconditioner M = F^-1 D F (Section 3.2), applied to an l x c
// image zero-embedded in a P x P grid, with D = h(|omega|) of eq. (3.2) on the
// radial frequency.  Three kernels, all LDS-resident radix-2 FFTs:
//
//  1. rows forward: two real rows are packed as one complex row (real and
//     imaginary parts), transformed, and split into the two half spectra
//     u = 0..P/2 (Hermitian symmetry) -> scratch S[l][P/2+1];
//  2. columns: CB half-spectrum columns per workgroup; forward FFT over the P
//     rows (rows >= l are the zero embedding), multiply by D(u, v), inverse FFT,
//     keep rows < l;
//  3. rows inverse: two rows rebuilt from their half spectra as one complex
//     row, inverse FFT; real part -> row r, imaginary part -> row r+1; crop to c
//     columns.  Optionally the float64 partial dot of the result with `dotv`.
//
// The output is real because D is real and even in both frequencies.
// Arithmetic and scratch are float64 (input and output float32): with mu = 1e-5
// the window spans five decades, and a float32 transform's rounding swamps the
// low-frequency part of z.
#include "sp_internal.h"
#include "sp_reduce.h"

namespace sp {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ int bitrev(int v, int logP) {
    return (int)(__builtin_bitreverse32((unsigned)v) >> (32 - logP));
}

// In-place decimation-in-time FFTs of `ncol` length-P arrays stored back to
// back in LDS, input in bit-reversed order, output in natural order.
// sign = -1: forward (exp(-2 pi i ...)); +1: inverse, unscaled.
__device__ void fft_dit(double2* buf, int P, int logP, int ncol, const double2* __restrict__ tw,
                        float sign) {
    const int half_total = ncol * (P >> 1);
    for (int s = 1; s <= logP; ++s) {
        const int half = 1 << (s - 1);
        const int tstride = P >> s;
        for (int bidx = threadIdx.x; bidx < half_total; bidx += blockDim.x) {
            const int col = bidx >> (logP - 1);
            const int bb = bidx & ((P >> 1) - 1);
            const int grp = bb >> (s - 1);
            const int pos = bb & (half - 1);
            const int i0 = col * P + grp * (half << 1) + pos;
            const int i1 = i0 + half;
            double2 w = tw[pos * tstride];   // exp(-2 pi i pos / len)
            if (sign > 0.0f) w.y = -w.y;    // inverse: conjugate twiddle
            const double2 u = buf[i0];
            const double2 v = cmul(buf[i1], w);
            buf[i0] = make_double2(u.x + v.x, u.y + v.y);
            buf[i1] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

// In-place decimation-in-frequency FFTs, input natural order, output
// bit-reversed.
__device__ void fft_dif(double2* buf, int P, int logP, int ncol, const double2* __restrict__ tw,
                        float sign) {
    const int half_total = ncol * (P >> 1);
    for (int s = logP; s >= 1; --s) {
        const int half = 1 << (s - 1);
        const int tstride = P >> s;
        for (int bidx = threadIdx.x; bidx < half_total; bidx += blockDim.x) {
            const int col = bidx >> (logP - 1);
            const int bb = bidx & ((P >> 1) - 1);
            const int grp = bb >> (s - 1);
            const int pos = bb & (half - 1);
            const int i0 = col * P + grp * (half << 1) + pos;
            const int i1 = i0 + half;
            double2 w = tw[pos * tstride];
            if (sign > 0.0f) w.y = -w.y;
            const double2 u = buf[i0];
            const double2 v = buf[i1];
            buf[i0] = make_double2(u.x + v.x, u.y + v.y);
            buf[i1] = cmul(make_double2(u.x - v.x, u.y - v.y), w);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void rows_fwd_body(const FFTPlan& F, const float* __restrict__ g,
                                              double2* buf, int bx) {
    const int r0 = 2 * bx, r1 = r0 + 1;
    for (int nidx = threadIdx.x; nidx < F.P; nidx += blockDim.x) {
        float re = 0.0f, im = 0.0f;
        if (nidx < F.cols) {
            re = g[(size_t)r0 * F.cols + nidx];
            if (r1 < F.rows) im = g[(size_t)r1 * F.cols + nidx];
        }
        buf[bitrev(nidx, F.logP)] = make_double2(re, im);
    }
    __syncthreads();
    fft_dit(buf, F.P, F.logP, 1, F.tw, -1.0f);
    for (int u = threadIdx.x; u <= F.P / 2; u += blockDim.x) {
        const double2 Z = buf[u];
        const double2 W = buf[(F.P - u) & (F.P - 1)];   // Z(-u); conj taken below
        // X0 = (Z + conj W) / 2 ;  X1 = (Z - conj W) / (2i)
        const double2 X0 = make_double2(0.5f * (Z.x + W.x), 0.5f * (Z.y - W.y));
        const double2 X1 = make_double2(0.5f * (Z.y + W.y), -0.5f * (Z.x - W.x));
        F.S[(size_t)r0 * F.SP + u] = X0;
        if (r1 < F.rows) F.S[(size_t)r1 * F.SP + u] = X1;
    }
}

__global__ __launch_bounds__(256) void k_rows_fwd(FFTPlan F, const float* __restrict__ g, const int* __restrict__ run,
                                                  const int* __restrict__ halt) {
    if (halt && *halt) return;
    if (run && !*run) return;
    extern __shared__ double2 buf[];
    rows_fwd_body(F, g, buf, blockIdx.x);
}

__device__ __forceinline__ double window_h(double w, double mu, double rho) {
    return (w + mu) * (rho + (1.0 - rho) * cos(w));
}

__device__ __forceinline__ void cols_body(const FFTPlan& F, double mu, double rho, double2* buf,
                                          int bx) {
    const int u0 = bx * F.CB;
    const int total = F.CB * F.P;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int r = idx / F.CB, cc = idx - r * F.CB;
        double2 v = make_double2(0.0f, 0.0f);
        if (r < F.rows && u0 + cc < F.SP) v = F.S[(size_t)r * F.SP + u0 + cc];
        buf[cc * F.P + bitrev(r, F.logP)] = v;
    }
    __syncthreads();
    fft_dit(buf, F.P, F.logP, F.CB, F.tw, -1.0f);
    const double two_pi_over_P = 6.283185307179586 / (double)F.P;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int cc = idx / F.P, v = idx - cc * F.P;
        const int u = u0 + cc;
        const int vv = v < F.P / 2 ? v : v - F.P;
        const double wu = two_pi_over_P * (double)u, wv = two_pi_over_P * (double)vv;
        const double h = window_h(sqrt(wu * wu + wv * wv), mu, rho);
        const double2 z = buf[idx];
        buf[idx] = make_double2(z.x * h, z.y * h);
    }
    __syncthreads();
    fft_dif(buf, F.P, F.logP, F.CB, F.tw, 1.0f);
    for (int idx = threadIdx.x; idx < F.rows * F.CB; idx += blockDim.x) {
        const int r = idx / F.CB, cc = idx - r * F.CB;
        if (u0 + cc < F.SP) F.S[(size_t)r * F.SP + u0 + cc] = buf[cc * F.P + bitrev(r, F.logP)];
    }
}

__global__ __launch_bounds__(256) void k_cols(FFTPlan F, double mu, double rho, const int* __restrict__ run,
                                              const int* __restrict__ halt) {
    if (halt && *halt) return;
    if (run && !*run) return;
    extern __shared__ double2 buf[];
    cols_body(F, mu, rho, buf, blockIdx.x);
}

__device__ __forceinline__ void rows_inv_body(const FFTPlan& F, float* __restrict__ z,
                                              const float* __restrict__ dotv,
                                              double* __restrict__ partials, double2* buf, int bx) {
    double* red = reinterpret_cast<double*>(buf);   // reused after the transform is read
    const int r0 = 2 * bx, r1 = r0 + 1;
    const bool has1 = r1 < F.rows;
    for (int u = threadIdx.x; u < F.P; u += blockDim.x) {
        double2 X0, X1 = make_double2(0.0f, 0.0f);
        if (u <= F.P / 2) {
            X0 = F.S[(size_t)r0 * F.SP + u];
            if (has1) X1 = F.S[(size_t)r1 * F.SP + u];
        } else {
            const double2 a = F.S[(size_t)r0 * F.SP + (F.P - u)];
            X0 = make_double2(a.x, -a.y);
            if (has1) {
                const double2 b = F.S[(size_t)r1 * F.SP + (F.P - u)];
                X1 = make_double2(b.x, -b.y);
            }
        }
        // Z = X0 + i X1
        buf[bitrev(u, F.logP)] = make_double2(X0.x - X1.y, X0.y + X1.x);
    }
    __syncthreads();
    fft_dit(buf, F.P, F.logP, 1, F.tw, 1.0f);
    const double scale = 1.0 / ((double)F.P * (double)F.P);
    double dot = 0.0;
    for (int j = threadIdx.x; j < F.cols; j += blockDim.x) {
        const double2 v = buf[j];
        const float a = (float)(v.x * scale);
        z[(size_t)r0 * F.cols + j] = a;
        if (dotv) dot += (double)a * (double)dotv[(size_t)r0 * F.cols + j];
        if (has1) {
            const float bv = (float)(v.y * scale);
            z[(size_t)r1 * F.cols + j] = bv;
            if (dotv) dot += (double)bv * (double)dotv[(size_t)r1 * F.cols + j];
        }
    }
    if (dotv) {
        const double tot = block_sum(dot, red);
        if (threadIdx.x == 0) partials[bx] = tot;
    }
}

__global__ __launch_bounds__(256) void k_rows_inv(FFTPlan F, float* __restrict__ z, const int* __restrict__ run,
                                                  const float* __restrict__ dotv,
                                                  double* __restrict__ partials,
                                                  const int* __restrict__ halt) {
    if (halt && *halt) return;
    if (run && !*run) return;
    extern __shared__ double2 buf[];
    rows_inv_body(F, z, dotv, partials, buf, blockIdx.x);
}

// Batched: z = M g per slice, partials of z^T h into pzh.
__global__ __launch_bounds__(256) void kb_rows_fwd(const SliceDev* __restrict__ sl, ItemTable t) {
    extern __shared__ double2 buf[];
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        FFTPlan F = S.F;
        F.S = gmem(F.S);
        F.tw = cmem(F.tw);
        rows_fwd_body(F, gmem(S.g), buf, lin);
    });
}

__global__ __launch_bounds__(256) void kb_cols(const SliceDev* __restrict__ sl, ItemTable t, double mu,
                                               double rho) {
    extern __shared__ double2 buf[];
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        FFTPlan F = S.F;
        F.S = gmem(F.S);
        F.tw = cmem(F.tw);
        cols_body(F, mu, rho, buf, lin);
    });
}

__global__ __launch_bounds__(256) void kb_rows_inv(const SliceDev* __restrict__ sl, ItemTable t) {
    extern __shared__ double2 buf[];
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        FFTPlan F = S.F;
        F.S = gmem(F.S);
        F.tw = cmem(F.tw);
        rows_inv_body(F, gmem(S.z), gmem(S.h), gmem(S.pzh), buf, lin);
    });
}

void launch_precond_b(hipStream_t st, const SliceDev* sl, ItemTable rows, ItemTable cols,
                      size_t lds_rows, size_t lds_cols, double mu, double rho) {
    hipLaunchKernelGGL(kb_rows_fwd, dim3(rows.grid), dim3(256), lds_rows, st, sl, rows);
    hipLaunchKernelGGL(kb_cols, dim3(cols.grid), dim3(256), lds_cols, st, sl, cols, mu, rho);
    hipLaunchKernelGGL(kb_rows_inv, dim3(rows.grid), dim3(256), lds_rows, st, sl, rows);
}

int precond_dot_blocks(const FFTPlan& F) { return (F.rows + 1) / 2; }

void launch_precond(hipStream_t st, const FFTPlan& F, double mu, double rho, const float* g,
                    float* z, const float* dotv, double* partials, const int* halt, const int* run) {
    const int nrow = (F.rows + 1) / 2;
    const size_t row_lds = (size_t)F.P * sizeof(double2);
    hipLaunchKernelGGL(k_rows_fwd, dim3(nrow), dim3(256), row_lds, st, F, g, run, halt);
    const int ncb = (F.SP + F.CB - 1) / F.CB;
    hipLaunchKernelGGL(k_cols, dim3(ncb), dim3(256), (size_t)F.CB * row_lds, st, F, mu, rho, run, halt);
    hipLaunchKernelGGL(k_rows_inv, dim3(nrow), dim3(256), row_lds, st, F, z, run, dotv, partials, halt);
}

}  // namespace sp
