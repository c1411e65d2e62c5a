// R and R^T as stored sparse matrices (Section 2: R is the m x n matrix of
// eq. 2.1 whose entry (ray, pixel) is the length of the ray inside the pixel;
// eq. 2.2 solves with R and R^T).  Layout: sliced ELLPACK with slices of 64
// rows, one per lane of a wave -- R by rays (row a * nB + k, columns pixels),
// R^T by pixels (row i * cols + j, columns rays).  Slice s holds width_s
// entries per row, stored entry-major ([e][lane]) from offset sp[s] (so
// width_s = (sp[s + 1] - sp[s]) / 64), with the row's length in len[row];
// entries past a row's length are padding and are never read.  Neighbouring
// rows of a slice are neighbouring rays of one angle (or pixels of one image
// row), so a wave's 64 loads of an entry are contiguous and its gathers of
// the vector land on neighbouring pixels (or bins).  Column indices are int32
// and weights float32: a product streams 8 bytes per stored entry.
//
// Both matrices are built on the device from one weight function
// (stored_weight), R ray by ray and R^T pixel by pixel, so they are exact
// transposes of each other.  Two passes: count the nonzeros of each row, size
// the slices (the longest row of each) and scan them into offsets, then fill.
#include "sp_internal.h"
#include "sp_reduce.h"
#include "sp_stored.h"

namespace sp {

// nat: the angle table in natural order (entry a is angle a).
__global__ __launch_bounds__(256) void k_count_rays(GeomDev G, const AngleDev* __restrict__ nat,
                                                    int32_t* __restrict__ cnt) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= G.nA * G.nB) return;
    int c = 0;
    ray_nonzeros(G, nat[r / G.nB], r % G.nB, [&](int, double) { ++c; });
    cnt[r] = c;
}

__global__ __launch_bounds__(256) void k_fill_rays(GeomDev G, const AngleDev* __restrict__ nat,
                                                   const int64_t* __restrict__ sp,
                                                   const int32_t* __restrict__ len,
                                                   int32_t* __restrict__ col, float* __restrict__ val) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= G.nA * G.nB) return;
    const int L = len[r];
    int64_t p = sp[r >> 6] + (r & 63);
    int e = 0;
    ray_nonzeros(G, nat[r / G.nB], r % G.nB, [&](int q, double w) {
        if (e < L) {
            col[p] = q;
            val[p] = (float)w;
        }
        ++e;
        p += 64;
    });
}

__global__ __launch_bounds__(256) void k_count_pixels(GeomDev G, const AngleDev* __restrict__ nat,
                                                      int32_t* __restrict__ cnt) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= G.rows * G.cols) return;
    int c = 0;
    pixel_nonzeros(G, nat, q / G.cols, q % G.cols, [&](int, double) { ++c; });
    cnt[q] = c;
}

__global__ __launch_bounds__(256) void k_fill_pixels(GeomDev G, const AngleDev* __restrict__ nat,
                                                     const int64_t* __restrict__ sp,
                                                     const int32_t* __restrict__ len,
                                                     int32_t* __restrict__ col, float* __restrict__ val) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= G.rows * G.cols) return;
    const int L = len[q];
    int64_t p = sp[q >> 6] + (q & 63);
    int e = 0;
    pixel_nonzeros(G, nat, q / G.cols, q % G.cols, [&](int r, double w) {
        if (e < L) {
            col[p] = r;
            val[p] = (float)w;
        }
        ++e;
        p += 64;
    });
}

// Entries of slice s: 64 times its longest row (rows past nrows count 0).
__global__ __launch_bounds__(256) void k_slice_sizes(const int32_t* __restrict__ len, int64_t nrows,
                                                     int64_t nslices, int32_t* __restrict__ size) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= nslices) return;
    int w = 0;
    for (int l = 0; l < 64; ++l) {
        const int64_t r = s * 64 + l;
        if (r < nrows) w = imax(w, len[r]);
    }
    size[s] = 64 * w;
}

// ---- exclusive scan of the row counts into int64 row offsets ------------------
// Blocks of SCAN_BLOCK counts; sums[b] = total of block b; then one workgroup
// scans the block totals in order; then each block adds its offset.
constexpr int SCAN_PER_THREAD = 4;
constexpr int SCAN_BLOCK = 256 * SCAN_PER_THREAD;

// Inclusive scan over the workgroup of one int64 per thread (Kogge-Stone in LDS).
__device__ __forceinline__ int64_t block_inclusive_scan(int64_t v, int64_t* lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int64_t add = threadIdx.x >= (unsigned)off ? lds[threadIdx.x - off] : 0;
        __syncthreads();
        v += add;
        lds[threadIdx.x] = v;
        __syncthreads();
    }
    return v;
}

__global__ __launch_bounds__(256) void k_scan_local(const int32_t* __restrict__ cnt, int64_t n,
                                                    int64_t* __restrict__ rp,
                                                    int64_t* __restrict__ sums) {
    __shared__ int64_t lds[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int64_t v[SCAN_PER_THREAD];
    int64_t run = 0;
    for (int u = 0; u < SCAN_PER_THREAD; ++u) {
        run += base + u < n ? cnt[base + u] : 0;
        v[u] = run;
    }
    const int64_t incl = block_inclusive_scan(run, lds);
    const int64_t before = incl - run;
    for (int u = 0; u < SCAN_PER_THREAD; ++u)
        if (base + u < n) rp[base + u + 1] = before + v[u];
    if (threadIdx.x == 255) sums[blockIdx.x] = incl;
}

__global__ __launch_bounds__(256) void k_scan_sums(int64_t* __restrict__ sums, int nb) {
    __shared__ int64_t lds[256];
    int64_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const int64_t v = b < nb ? sums[b] : 0;
        const int64_t incl = block_inclusive_scan(v, lds);
        if (b < nb) sums[b] = carry + incl - v;   // exclusive: offset of block b
        carry += lds[255];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_scan_add(int64_t n, int64_t* __restrict__ rp,
                                                  const int64_t* __restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    const int64_t off = sums[blockIdx.x];
    for (int u = 0; u < SCAN_PER_THREAD; ++u)
        if (base + u < n) rp[base + u + 1] += off;
    if (blockIdx.x == 0 && threadIdx.x == 0) rp[0] = 0;
}

int scan_blocks(int64_t n) { return (int)((n + SCAN_BLOCK - 1) / SCAN_BLOCK); }

void launch_scan(hipStream_t st, const int32_t* cnt, int64_t n, int64_t* rp, int64_t* sums) {
    const int nb = scan_blocks(n);
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(256), 0, st, cnt, n, rp, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, st, sums, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(256), 0, st, n, rp, sums);
}

void launch_stored_count(hipStream_t st, const GeomDev& G, const AngleDev* nat, bool pixels,
                         int32_t* cnt) {
    const int64_t n = pixels ? (int64_t)G.rows * G.cols : (int64_t)G.nA * G.nB;
    const int nb = (int)((n + 255) / 256);
    if (pixels) hipLaunchKernelGGL(k_count_pixels, dim3(nb), dim3(256), 0, st, G, nat, cnt);
    else hipLaunchKernelGGL(k_count_rays, dim3(nb), dim3(256), 0, st, G, nat, cnt);
}

void launch_slice_sizes(hipStream_t st, const int32_t* len, int64_t nrows, int32_t* size) {
    const int64_t ns = (nrows + 63) / 64;
    hipLaunchKernelGGL(k_slice_sizes, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, len, nrows, ns,
                       size);
}

void launch_stored_fill(hipStream_t st, const GeomDev& G, const AngleDev* nat, bool pixels,
                        const int64_t* sp, const int32_t* len, int32_t* col, float* val) {
    const int64_t n = pixels ? (int64_t)G.rows * G.cols : (int64_t)G.nA * G.nB;
    const int nb = (int)((n + 255) / 256);
    if (pixels) hipLaunchKernelGGL(k_fill_pixels, dim3(nb), dim3(256), 0, st, G, nat, sp, len, col, val);
    else hipLaunchKernelGGL(k_fill_rays, dim3(nb), dim3(256), 0, st, G, nat, sp, len, col, val);
}

// ---- y = A x for a stored matrix ------------------------------------------------
// One workgroup per slice; its four waves take the four contiguous quarters of
// the slice's entry range, lane l summing row 64 s + l over its quarter in
// order with U entries' loads in flight; the quarters' sums are then added in
// wave order through LDS.  The matrix streams through once, so its loads are
// nontemporal and leave the caches to the gathered vector.
template <int U>
__global__ __launch_bounds__(256) void k_sell_spmv(int64_t nrows, const int64_t* __restrict__ sp,
                                                   const int32_t* __restrict__ len,
                                                   const int32_t* __restrict__ col,
                                                   const float* __restrict__ val,
                                                   const float* __restrict__ x,
                                                   float* __restrict__ y) {
    __shared__ double part[4][64];
    const int64_t s = blockIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row = s * 64 + lane;
    const int L = row < nrows ? len[row] : 0;
    const int64_t base = sp[s];
    const int W = (int)((sp[s + 1] - base) >> 6);
    const int e0 = W * w / 4, e1 = imin(W * (w + 1) / 4, L);
    const int32_t* cp = col + base + lane;
    const float* vp = val + base + lane;
    double acc = 0.0;
    int e = e0;
    for (; e + U <= e1; e += U) {
        int32_t c[U];
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = __builtin_nontemporal_load(cp + (int64_t)(e + u) * 64);
            v[u] = __builtin_nontemporal_load(vp + (int64_t)(e + u) * 64);
        }
        float xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) acc = fma((double)v[u], (double)xv[u], acc);
    }
    for (; e < e1; ++e)
        acc = fma((double)__builtin_nontemporal_load(vp + (int64_t)e * 64),
                  (double)x[__builtin_nontemporal_load(cp + (int64_t)e * 64)], acc);
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0 && row < nrows) y[row] = (float)(((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
}

void launch_sell_spmv(hipStream_t st, int64_t nrows, const int64_t* sp, const int32_t* len,
                      const int32_t* col, const float* val, const float* x, float* y) {
    const int64_t ns = (nrows + 63) / 64;
    hipLaunchKernelGGL(k_sell_spmv<8>, dim3((unsigned)ns), dim3(256), 0, st, nrows, sp, len, col, val, x, y);
}

}  // namespace sp
