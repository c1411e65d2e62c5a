// The paper's preconditioner M = F^-1 D F (Section 3.2), applied to an l x c
// image zero-embedded in a P x P grid, with D = h(|omega|) of eq. (3.2) on the
// radial frequency.  Three kernels, all LDS-resident radix-2 FFTs (two stages per LDS pass):
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

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
    return make_double2(a.x - b.x, a.y - b.y);
}

// LDS layout of the transform entries: logical entry i of the ncol * P
// entries sits at i + (i >> sh).  With sh = 3 (one spare 16-byte slot after
// every 8 entries, used when the padded buffer fits in 64 KB) the
// power-of-two strides of the butterflies and of the bit-reversed scatter
// spread over the LDS banks instead of piling onto a few; sh = 30 leaves the
// layout dense.
__host__ __device__ __forceinline__ int fft_lds_shift(int P, int ncol) {
    const size_t n = (size_t)ncol * P;
    return (n + (n >> 3)) * sizeof(double2) <= 65536 ? 3 : 30;
}

__host__ __device__ __forceinline__ size_t fft_data_len(int P, int ncol) {
    const size_t n = (size_t)ncol * P;
    return n + (n >> fft_lds_shift(P, ncol));
}

struct LdsBuf {
    double2* p;
    int sh;
    __device__ __forceinline__ double2& operator[](int i) const { return p[i + (i >> sh)]; }
};

// In-place decimation-in-time FFTs of `ncol` length-P arrays stored back to
// back in LDS, input in bit-reversed order, output in natural order.
// sign = -1: forward (exp(-2 pi i ...)); +1: inverse, unscaled.  tw[k] =
// exp(-2 pi i k / P), k < P/2 (LDS or global).
//
// Radix-2 stages s = 1..logP, taken two per pass: a thread loads the four
// elements i0 + {0, h, 2h, 3h} (h = 2^(s-1)) and applies to them exactly the
// butterflies of stages s and s+1, so every value is the one the stage-by-
// stage sequence produces, with half the LDS round trips and barriers.
template <class TW>
__device__ __forceinline__ void fft_dit(LdsBuf buf, int P, int logP, int ncol, TW tw, float sign) {
    const bool inv = sign > 0.0f;
    auto twd = [&](int k) {
        double2 w = tw[k];
        if (inv) w.y = -w.y;   // inverse: conjugate twiddle
        return w;
    };
    int s = 1;
    for (; s + 1 <= logP; s += 2) {
        const int half = 1 << (s - 1);
        const int ts0 = P >> s, ts1 = P >> (s + 1);
        const int quads = ncol * (P >> 2);
        for (int q = threadIdx.x; q < quads; q += blockDim.x) {
            const int col = q >> (logP - 2);
            const int qq = q & ((P >> 2) - 1);
            const int pos = qq & (half - 1);
            const int e0 = col * P + (qq >> (s - 1)) * (half << 2) + pos;
            const int e1 = e0 + half, e2 = e1 + half, e3 = e2 + half;
            const double2 wa = twd(pos * ts0), wb = twd(pos * ts1), wc = twd((pos + half) * ts1);
            const double2 x0 = buf[e0], x1 = buf[e1], x2 = buf[e2], x3 = buf[e3];
            double2 v = cmul(x1, wa);                       // stage s: (e0, e1), (e2, e3)
            const double2 y0 = cadd(x0, v), y1 = csub(x0, v);
            v = cmul(x3, wa);
            const double2 y2 = cadd(x2, v), y3 = csub(x2, v);
            v = cmul(y2, wb);                               // stage s+1: (e0, e2), (e1, e3)
            buf[e0] = cadd(y0, v);
            buf[e2] = csub(y0, v);
            v = cmul(y3, wc);
            buf[e1] = cadd(y1, v);
            buf[e3] = csub(y1, v);
        }
        __syncthreads();
    }
    if (s == logP) {   // odd logP: the last stage alone
        const int half = 1 << (s - 1);
        const int tstride = P >> s;
        for (int bidx = threadIdx.x; bidx < ncol * (P >> 1); bidx += blockDim.x) {
            const int col = bidx >> (logP - 1);
            const int bb = bidx & ((P >> 1) - 1);
            const int pos = bb & (half - 1);
            const int i0 = col * P + (bb >> (s - 1)) * (half << 1) + pos;
            const int i1 = i0 + half;
            const double2 u = buf[i0];
            const double2 v = cmul(buf[i1], twd(pos * tstride));
            buf[i0] = cadd(u, v);
            buf[i1] = csub(u, v);
        }
        __syncthreads();
    }
}

// In-place decimation-in-frequency FFTs, input natural order, output
// bit-reversed.  Stages s = logP..1, two per pass (s and s-1 on the four
// elements i0 + {0, q, 2q, 3q}, q = 2^(s-2)).
template <class TW>
__device__ __forceinline__ void fft_dif(LdsBuf buf, int P, int logP, int ncol, TW tw, float sign) {
    const bool inv = sign > 0.0f;
    auto twd = [&](int k) {
        double2 w = tw[k];
        if (inv) w.y = -w.y;
        return w;
    };
    int s = logP;
    for (; s >= 2; s -= 2) {
        const int q4 = 1 << (s - 2);
        const int ts0 = P >> s, ts1 = P >> (s - 1);
        const int quads = ncol * (P >> 2);
        for (int q = threadIdx.x; q < quads; q += blockDim.x) {
            const int col = q >> (logP - 2);
            const int qq = q & ((P >> 2) - 1);
            const int pos = qq & (q4 - 1);
            const int a = col * P + (qq >> (s - 2)) * (q4 << 2) + pos;
            const int b = a + q4, c = b + q4, d = c + q4;
            const double2 w0 = twd(pos * ts0), w1 = twd((pos + q4) * ts0), w2 = twd(pos * ts1);
            const double2 xa = buf[a], xb = buf[b], xc = buf[c], xd = buf[d];
            const double2 ya = cadd(xa, xc), yc = cmul(csub(xa, xc), w0);   // stage s
            const double2 yb = cadd(xb, xd), yd = cmul(csub(xb, xd), w1);
            buf[a] = cadd(ya, yb);                                          // stage s-1
            buf[b] = cmul(csub(ya, yb), w2);
            buf[c] = cadd(yc, yd);
            buf[d] = cmul(csub(yc, yd), w2);
        }
        __syncthreads();
    }
    if (s == 1) {   // odd logP: stage 1 alone
        for (int bidx = threadIdx.x; bidx < ncol * (P >> 1); bidx += blockDim.x) {
            const int col = bidx >> (logP - 1);
            const int bb = bidx & ((P >> 1) - 1);
            const int i0 = col * P + bb * 2;
            const int i1 = i0 + 1;
            const double2 u = buf[i0];
            const double2 v = buf[i1];
            buf[i0] = cadd(u, v);
            buf[i1] = cmul(csub(u, v), twd(0));
        }
        __syncthreads();
    }
}

// The twiddles go to LDS after the (padded) transform entries when both fit
// in 64 KB (stage_twiddles returns the LDS copy), else they are read from
// global memory.
__host__ __device__ __forceinline__ bool tw_in_lds(int P, int ncol) {
    return (fft_data_len(P, ncol) + P / 2) * sizeof(double2) <= 65536;
}

__device__ __forceinline__ const double2* stage_twiddles(const FFTPlan& F, double2* raw, int ncol) {
    double2* t = raw + fft_data_len(F.P, ncol);
    for (int k = threadIdx.x; k < F.P / 2; k += blockDim.x) t[k] = F.tw[k];
    return t;   // visible after the caller's next barrier
}

#define SP_FFT(kind, ncol, sign)                                                  \
    do {                                                                          \
        if (twl) kind(buf, F.P, F.logP, ncol, (const double2*)(raw + fft_data_len(F.P, ncol)), sign); \
        else kind(buf, F.P, F.logP, ncol, F.tw, sign);                            \
    } while (0)

__device__ __forceinline__ void rows_fwd_body(const FFTPlan& F, const float* __restrict__ g,
                                              double2* raw, int bx) {
    const LdsBuf buf{raw, fft_lds_shift(F.P, 1)};
    const int r0 = 2 * bx, r1 = r0 + 1;
    const bool twl = tw_in_lds(F.P, 1);
    if (twl) stage_twiddles(F, raw, 1);
    for (int nidx = threadIdx.x; nidx < F.P; nidx += blockDim.x) {
        float re = 0.0f, im = 0.0f;
        if (nidx < F.cols) {
            re = g[(size_t)r0 * F.cols + nidx];
            if (r1 < F.rows) im = g[(size_t)r1 * F.cols + nidx];
        }
        buf[bitrev(nidx, F.logP)] = make_double2(re, im);
    }
    __syncthreads();
    SP_FFT(fft_dit, 1, -1.0f);
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

__global__ __launch_bounds__(512) void k_rows_fwd(FFTPlan F, const float* __restrict__ g, const int* __restrict__ run,
                                                  const int* __restrict__ halt) {
    if (halt && *halt) return;
    if (run && !*run) return;
    extern __shared__ double2 buf[];
    rows_fwd_body(F, g, buf, blockIdx.x);
}

__device__ __forceinline__ double window_h(double w, double mu, double rho) {
    return (w + mu) * (rho + (1.0 - rho) * cos(w));
}

__device__ __forceinline__ void cols_body(const FFTPlan& F, double mu, double rho, double2* raw,
                                          int bx) {
    const LdsBuf buf{raw, fft_lds_shift(F.P, F.CB)};
    const int u0 = bx * F.CB;
    const int total = F.CB * F.P;
    const bool twl = tw_in_lds(F.P, F.CB);
    if (twl) stage_twiddles(F, raw, F.CB);
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int r = idx / F.CB, cc = idx - r * F.CB;
        double2 v = make_double2(0.0f, 0.0f);
        if (r < F.rows && u0 + cc < F.SP) v = F.S[(size_t)r * F.SP + u0 + cc];
        buf[cc * F.P + bitrev(r, F.logP)] = v;
    }
    __syncthreads();
    SP_FFT(fft_dit, F.CB, -1.0f);
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
    SP_FFT(fft_dif, F.CB, 1.0f);
    for (int idx = threadIdx.x; idx < F.rows * F.CB; idx += blockDim.x) {
        const int r = idx / F.CB, cc = idx - r * F.CB;
        if (u0 + cc < F.SP) F.S[(size_t)r * F.SP + u0 + cc] = buf[cc * F.P + bitrev(r, F.logP)];
    }
}

__global__ __launch_bounds__(512) void k_cols(FFTPlan F, double mu, double rho, const int* __restrict__ run,
                                              const int* __restrict__ halt) {
    if (halt && *halt) return;
    if (run && !*run) return;
    extern __shared__ double2 buf[];
    cols_body(F, mu, rho, buf, blockIdx.x);
}

// With xp, z is also written to R's padded float64 copies (xp row-major with
// row pitch pitchX, xTp transposed with pitch pitchXT, both PAD-offset), as
// R's prep would write them.
__device__ __forceinline__ void rows_inv_body(const FFTPlan& F, float* __restrict__ z,
                                              const float* __restrict__ dotv,
                                              double* __restrict__ partials, double2* raw, int bx,
                                              double* __restrict__ xp = nullptr,
                                              double* __restrict__ xTp = nullptr, int pitchX = 0,
                                              int pitchXT = 0) {
    const LdsBuf buf{raw, fft_lds_shift(F.P, 1)};
    double* red = reinterpret_cast<double*>(raw);   // reused after the transform is read
    const int r0 = 2 * bx, r1 = r0 + 1;
    const bool has1 = r1 < F.rows;
    const bool twl = tw_in_lds(F.P, 1);
    if (twl) stage_twiddles(F, raw, 1);
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
    SP_FFT(fft_dit, 1, 1.0f);
    const double scale = 1.0 / ((double)F.P * (double)F.P);
    double dot = 0.0;
    for (int j = threadIdx.x; j < F.cols; j += blockDim.x) {
        const double2 v = buf[j];
        const float a = (float)(v.x * scale);
        z[(size_t)r0 * F.cols + j] = a;
        if (dotv) dot += (double)a * (double)dotv[(size_t)r0 * F.cols + j];
        if (xp) {
            xp[(size_t)r0 * pitchX + PAD + j] = (double)a;
            xTp[(size_t)j * pitchXT + PAD + r0] = (double)a;
        }
        if (has1) {
            const float bv = (float)(v.y * scale);
            z[(size_t)r1 * F.cols + j] = bv;
            if (dotv) dot += (double)bv * (double)dotv[(size_t)r1 * F.cols + j];
            if (xp) {
                xp[(size_t)r1 * pitchX + PAD + j] = (double)bv;
                xTp[(size_t)j * pitchXT + PAD + r1] = (double)bv;
            }
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
                                                  const int* __restrict__ halt,
                                                  double* __restrict__ xp, double* __restrict__ xTp,
                                                  int pitchX, int pitchXT) {
    if (halt && *halt) return;
    if (run && !*run) return;
    extern __shared__ double2 buf[];
    rows_inv_body(F, z, dotv, partials, buf, blockIdx.x, xp, xTp, pitchX, pitchXT);
}

// Batched: z = M g per slice.
__global__ __launch_bounds__(512) void kb_rows_fwd(const SliceDev* __restrict__ sl, ItemTable t) {
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

__global__ __launch_bounds__(512) void kb_cols(const SliceDev* __restrict__ sl, ItemTable t, double mu,
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
        rows_inv_body(F, gmem(S.z), nullptr, nullptr, buf, lin);
    });
}

void launch_precond_b(hipStream_t st, const SliceDev* sl, ItemTable rows, ItemTable cols,
                      size_t lds_rows, size_t lds_cols, double mu, double rho) {
    hipLaunchKernelGGL(kb_rows_fwd, dim3(rows.grid), dim3(512), lds_rows, st, sl, rows);
    hipLaunchKernelGGL(kb_cols, dim3(cols.grid), dim3(512), lds_cols, st, sl, cols, mu, rho);
    hipLaunchKernelGGL(kb_rows_inv, dim3(rows.grid), dim3(256), lds_rows, st, sl, rows);
}

int precond_dot_blocks(const FFTPlan& F) { return (F.rows + 1) / 2; }

size_t fft_lds_bytes(int P, int ncol) {
    return (fft_data_len(P, ncol) + (tw_in_lds(P, ncol) ? P / 2 : 0)) * sizeof(double2);
}

void launch_precond(hipStream_t st, const FFTPlan& F, double mu, double rho, const float* g,
                    float* z, const float* dotv, double* partials, const int* halt, const int* run,
                    const GeomDev* G, double* xp, double* xTp) {
    const int nrow = (F.rows + 1) / 2;
    const size_t row_lds = fft_lds_bytes(F.P, 1);
    hipLaunchKernelGGL(k_rows_fwd, dim3(nrow), dim3(512), row_lds, st, F, g, run, halt);
    const int ncb = (F.SP + F.CB - 1) / F.CB;
    hipLaunchKernelGGL(k_cols, dim3(ncb), dim3(512), fft_lds_bytes(F.P, F.CB), st, F, mu, rho, run,
                       halt);
    hipLaunchKernelGGL(k_rows_inv, dim3(nrow), dim3(256), row_lds, st, F, z, run, dotv, partials, halt,
                       G ? xp : nullptr, G ? xTp : nullptr, G ? G->pitchX : 0, G ? G->pitchXT : 0);
}

}  // namespace sp
