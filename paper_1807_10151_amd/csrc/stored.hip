// R and R^T as stored sparse matrices (Section 2: R is the m x n matrix of
// eq. 2.1 whose entry (ray, pixel) is the length of the ray inside the pixel;
// eq. 2.2 solves with R and R^T).  Layout: sliced ELLPACK with slices of 64
// rows, one per lane of a wave -- R by rays (row a * nB + k, columns pixels),
// R^T by pixels (row i * cols + j, columns rays).  Slice s holds width_s
// entries per row, stored entry-major ([e][lane]) from offset sp[s] (so
// width_s = (sp[s + 1] - sp[s]) / 128 words: each group of four entries of
// the 64 lanes is 256 column indices followed by their 256 weights), with the
// row's length in len[row]; entries past a row's length are padding.  Neighbouring
// rows of a slice are neighbouring rays of one angle (or pixels of one image
// row), so a wave's loads of a group are one contiguous 2 KiB run and its
// gathers of the vector land on neighbouring pixels (or bins).  Column
// indices are int32 and weights float32: a product streams 8 bytes per
// stored entry.
//
// Both matrices are built on the device from one weight function
// (stored_weight), R ray by ray and R^T pixel by pixel, so they are exact
// transposes of each other.  Two passes: count the nonzeros of each row, size
// the slices (the longest row of each) and scan them into offsets, then fill.
#include "sp_internal.h"
#include "sp_reduce.h"
#include "sp_stored.h"

namespace sp {

// Rows are grouped in segments (one angle's rays for R, one image row's
// pixels for R^T) of lseg rows; each segment starts a new slice, so a slice
// never mixes angles or image rows.  Row r = seg * lseg + k sits in slice
// seg * spseg + k / 64, lane k % 64.  A slice holds 64 lanes x width entries,
// width a multiple of 4; lane l's entry e is at offset
// sp[slice] + (e / 4) * 256 + 4 l + e % 4, so each lane reads its entries four
// at a time with 16-byte loads.
// nat: the angle table in natural order (entry a is angle a).
__global__ __launch_bounds__(256) void k_count_rays(GeomDev G, const AngleDev* __restrict__ nat,
                                                    int32_t* __restrict__ cnt) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= G.nA * G.nB) return;
    int c = 0;
    ray_nonzeros(G, nat[r / G.nB], r % G.nB, [&](int, double) { ++c; });
    cnt[r] = c;
}

// Rays of near-horizontal angles (|sin| > |cos|, walked column by column)
// store the transposed pixel index j * rows + i: their products gather from a
// transposed copy of the image, where the pixels of neighbouring rays are
// neighbours.
__global__ __launch_bounds__(256) void k_fill_rays(GeomDev G, SellShape S, const AngleDev* __restrict__ nat,
                                                   const int64_t* __restrict__ sp,
                                                   const int32_t* __restrict__ len,
                                                   int32_t* __restrict__ ent) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= G.nA * G.nB) return;
    const int L = len[r];
    const AngleDev A = nat[r / G.nB];
    const bool tr = (A.flags & ANG_HORIZ) != 0;
    const int64_t p0 = sp[sell_slice(S, r)];
    const int lane = sell_lane(S, r);
    int e = 0;
    ray_nonzeros(G, A, r % G.nB, [&](int q, double w) {
        if (e < L) {
            const int64_t p = p0 + sell_offset(lane, e);
            ent[p] = tr ? (q % G.cols) * G.rows + q / G.cols : q;
            ent[p + SELL_VAL] = __float_as_int((float)w);
        }
        ++e;
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

__global__ __launch_bounds__(256) void k_fill_pixels(GeomDev G, SellShape S, const AngleDev* __restrict__ nat,
                                                     const int64_t* __restrict__ sp,
                                                     const int32_t* __restrict__ len,
                                                     int32_t* __restrict__ ent) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= G.rows * G.cols) return;
    const int L = len[q];
    const int64_t p0 = sp[sell_slice(S, q)];
    const int lane = sell_lane(S, q);
    int e = 0;
    pixel_nonzeros(G, nat, q / G.cols, q % G.cols, [&](int r, double w) {
        if (e < L) {
            const int64_t p = p0 + sell_offset(lane, e);
            ent[p] = r;
            ent[p + SELL_VAL] = __float_as_int((float)w);
        }
        ++e;
    });
}

// Words of slice s: 128 times its longest row rounded up to a multiple of 4.
__global__ __launch_bounds__(256) void k_slice_sizes(const int32_t* __restrict__ len, SellShape S,
                                                     int32_t* __restrict__ size) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= S.nseg * S.spseg) return;
    const int64_t seg = s / S.spseg, k0 = (s % S.spseg) * 64;
    int w = 0;
    for (int l = 0; l < 64 && k0 + l < S.lseg; ++l) w = imax(w, len[seg * S.lseg + k0 + l]);
    size[s] = 128 * ((w + 3) & ~3);
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

void launch_slice_sizes(hipStream_t st, const int32_t* len, const SellShape& S, int32_t* size) {
    const int64_t ns = S.nseg * S.spseg;
    hipLaunchKernelGGL(k_slice_sizes, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, len, S, size);
}

void launch_stored_fill(hipStream_t st, const GeomDev& G, const SellShape& S, const AngleDev* nat,
                        bool pixels, const int64_t* sp, const int32_t* len, int32_t* ent) {
    const int64_t n = pixels ? (int64_t)G.rows * G.cols : (int64_t)G.nA * G.nB;
    const int nb = (int)((n + 255) / 256);
    if (pixels) hipLaunchKernelGGL(k_fill_pixels, dim3(nb), dim3(256), 0, st, G, S, nat, sp, len, ent);
    else hipLaunchKernelGGL(k_fill_rays, dim3(nb), dim3(256), 0, st, G, S, nat, sp, len, ent);
}

// ---- y = A x for a stored matrix ------------------------------------------------
// One workgroup per slice; its four waves take the four contiguous quarters of
// the slice's groups of four entries (each group read as one 16-byte load of
// column indices and one of weights per lane), lane l summing its row over its quarter
// in order with U groups' loads in flight; the quarters' sums are then added
// in wave order through LDS.  Entries past a row's length (padding, column 0,
// weight 0) add nothing: their gathered value is masked to 0.  The matrix
// streams through once, so its loads are nontemporal and leave the caches to
// the gathered vector.  segT (nullable): 1 for segments whose column indices
// refer to xT, the transposed vector.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int U>
__global__ __launch_bounds__(256) void k_sell_spmv(SellShape S, const int64_t* __restrict__ sp,
                                                   const int32_t* __restrict__ len,
                                                   const int32_t* __restrict__ ent,
                                                   const float* __restrict__ x,
                                                   const float* __restrict__ xT,
                                                   const uint8_t* __restrict__ segT,
                                                   float* __restrict__ y) {
    __shared__ double part[4][64];
    const int64_t s = blockIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t seg = s / S.spseg, k = (s % S.spseg) * 64 + lane;
    const bool valid = k < S.lseg;
    const int64_t row = seg * S.lseg + k;
    const int L = valid ? len[row] : 0;
    const float* __restrict__ xs = (segT && segT[seg]) ? xT : x;
    const int64_t base = sp[s];
    const int NG = (int)((sp[s + 1] - base) >> 9);
    const int g0 = NG * w / 4, g1 = imin(NG * (w + 1) / 4, (L + 3) >> 2);
    const i32x4* cp = reinterpret_cast<const i32x4*>(ent + base) + lane;
    const f32x4* vp = reinterpret_cast<const f32x4*>(ent + base + SELL_VAL) + lane;
    double acc = 0.0;
    int g = g0;
    for (; g + U <= g1; g += U) {
        i32x4 c[U];
        f32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = __builtin_nontemporal_load(cp + (int64_t)(g + u) * 128);
            v[u] = __builtin_nontemporal_load(vp + (int64_t)(g + u) * 128);
        }
        float xv[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) xv[u][q] = xs[c[u][q]];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc = fma((double)v[u][q], 4 * (g + u) + q < L ? (double)xv[u][q] : 0.0, acc);
    }
    for (; g < g1; ++g) {
        const i32x4 c = __builtin_nontemporal_load(cp + (int64_t)g * 128);
        const f32x4 v = __builtin_nontemporal_load(vp + (int64_t)g * 128);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float xq = xs[c[q]];
            acc = fma((double)v[q], 4 * g + q < L ? (double)xq : 0.0, acc);
        }
    }
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0 && valid) y[row] = (float)(((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
}

void launch_sell_spmv(hipStream_t st, const SellShape& S, const int64_t* sp, const int32_t* len,
                      const int32_t* ent, const float* x, const float* xT, const uint8_t* segT, float* y) {
    const int64_t ns = S.nseg * S.spseg;
    hipLaunchKernelGGL(k_sell_spmv<4>, dim3((unsigned)ns), dim3(256), 0, st, S, sp, len, ent, x, xT, segT, y);
}

// xT[j * rows + i] = x[i * cols + j], through 64 x 64 LDS tiles.
__global__ __launch_bounds__(256) void k_transpose(int rows, int cols, const float* __restrict__ x,
                                                   float* __restrict__ xT) {
    __shared__ float t[64][65];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4)
        if (i0 + r < rows && j0 + tx < cols) t[r][tx] = x[(size_t)(i0 + r) * cols + j0 + tx];
    __syncthreads();
    for (int r = ty; r < 64; r += 4)
        if (j0 + r < cols && i0 + tx < rows) xT[(size_t)(j0 + r) * rows + i0 + tx] = t[tx][r];
}

void launch_transpose(hipStream_t st, int rows, int cols, const float* x, float* xT) {
    hipLaunchKernelGGL(k_transpose, dim3((cols + 63) / 64, (rows + 63) / 64), dim3(256), 0, st, rows, cols, x,
                       xT);
}

}  // namespace sp
