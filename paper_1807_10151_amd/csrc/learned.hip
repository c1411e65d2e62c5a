// Learned SPD preconditioner M = C^T diag(softplus(d)) C (used in Algorithm 2,
// step 2, in place of the Fourier preconditioner of Section 3.2).
//
// C is a stack of L linear 3x3 cross-correlations without bias with zero
// "same" padding: 1 -> 16 channels, then 16 -> 16.  C^T applies, in reverse
// layer order, each layer's adjoint: the correlation with the spatially
// flipped kernel and swapped channel roles.  d has one entry per channel.
//
// Layout: activations are channels-last float32 [B][H][W][16]; images are
// [B][H][W].  Parameters theta (float32) = W_1 [16][1][3][3], W_2..W_L
// [16][16][3][3], d [16]; tap t = 3 ky + kx reads the input at offset
// (ky - 1, kx - 1).
//
// The 16 -> 16 layers run as implicit GEMM on MFMA: a wave computes tiles of
// 16 consecutive pixels of one image row for all 16 output channels with
// v_mfma_f32_16x16x4f32 (A = 16 pixels x 4 input channels of one tap,
// B = 4 input channels x 16 output channels), 9 taps x 4 channel groups =
// 36 MFMAs per tile.  MFMA cg takes input channel 4 kq + cg from lane group
// kq, so each lane reads its 4 channels of a pixel as one 16-byte load; a wave
// keeps the weights in registers over TPW tiles (4 for large grids, 1 for
// small ones, which need the waves more) with independent
// accumulators.  The 16 -> 16 weight gradients are MFMA products over the
// pixels of a tile; the 1 <-> 16 layers, the first layer's weight gradient,
// the loss and Adam are plain VALU kernels.
#include "sp_internal.h"
#include "sp_reduce.h"

namespace sp {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int LF = 16;   // channels

__device__ __forceinline__ bool in_img(int h, int w, int H, int W) {
    return h >= 0 && h < H && w >= 0 && w < W;
}

// ---- 16 -> 16 correlation on MFMA --------------------------------------------
// out[b,h,w,j] = sum_{t, ci} in[b, h+dy_t, w+dx_t, ci] * K[j][ci][t], with
// K = W (TRANS = false) or K[j][ci][t] = W[ci][j][8 - t] (TRANS: the adjoint).
// If scale != nullptr, out2 = scale[j] * out as well.
template <bool TRANS, int TPW>
__global__ __launch_bounds__(256) void k_lp_conv_mid(int B, int H, int W,
                                                     const float* __restrict__ in,
                                                     float* __restrict__ out,
                                                     const float* __restrict__ Wl,
                                                     const float* __restrict__ scale,
                                                     float* __restrict__ out2,
                                                     const int* __restrict__ halt,
                                                     const int* __restrict__ run) {
    if (halt && *halt) return;
    if (run && !*run) return;
    const int lane = threadIdx.x & 63;
    const int wtiles = (W + 15) >> 4;
    const long ntiles = (long)B * H * wtiles;
    const long tile0 = ((long)blockIdx.x * 4 + (threadIdx.x >> 6)) * TPW;
    if (tile0 >= ntiles) return;                    // whole wave; no barriers below
    const int i = lane & 15;     // A row (pixel) / B column (out channel)
    const int kq = lane >> 4;    // A column / B row within a group of 4 input channels
    float wr[36];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
#pragma unroll
        for (int cg = 0; cg < 4; ++cg) {
            const int ci = 4 * kq + cg;   // MFMA cg: lane kq supplies input channel 4 kq + cg
            wr[t * 4 + cg] = TRANS ? Wl[(ci * LF + i) * 9 + (8 - t)] : Wl[(i * LF + ci) * 9 + t];
        }
    }
    // TPW consecutive tiles per wave (weights loaded once, independent
    // accumulators); tile j = (b, h, w0) of tile0 + j
    int tb[TPW], th[TPW], tw0[TPW];
    bool tv[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        const long tile = tile0 + j;
        tv[j] = tile < ntiles;
        const long tt = tv[j] ? tile : tile0;
        tw0[j] = (int)(tt % wtiles) * 16;
        const long bh = tt / wtiles;
        th[j] = (int)(bh % H);
        tb[j] = (int)(bh / H);
    }
    f4v acc[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j) acc[j] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        f4v a[TPW];
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            const int hh = th[j] + t / 3 - 1;
            const int ww = tw0[j] + i + t % 3 - 1;
            const bool ok = tv[j] && in_img(hh, ww, H, W);
            // channels 4 kq .. 4 kq + 3 of the pixel: one 16-byte load
            const f4v* p = reinterpret_cast<const f4v*>(
                in + (((size_t)tb[j] * H + (ok ? hh : 0)) * W + (ok ? ww : 0)) * LF + 4 * kq);
            a[j] = ok ? *p : f4v{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int cg = 0; cg < 4; ++cg) {
#pragma unroll
            for (int j = 0; j < TPW; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j][cg], wr[t * 4 + cg], acc[j], 0, 0, 0);
        }
    }
    // lane holds D[4*(lane>>4) + r][lane & 15]: pixel w0 + 4*kq + r, channel i
    const float sc = scale ? scale[i] : 0.0f;
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        if (!tv[j]) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int px = tw0[j] + 4 * kq + r;
            if (px < W) {
                const size_t o = (((size_t)tb[j] * H + th[j]) * W + px) * LF + i;
                if (out) out[o] = acc[j][r];
                if (out2) out2[o] = acc[j][r] * sc;
            }
        }
    }
}

// ---- 1 -> 16 (first layer) and its adjoint 16 -> 1 ------------------------------
// out[b,h,w,co] = sum_t W1[co][t] * in[src(b), h+dy, w+dx]; src(b) = idx[b] if idx.
__global__ __launch_bounds__(256) void k_lp_conv_in(int B, int H, int W, const float* __restrict__ in,
                                                    const int32_t* __restrict__ idx, int nsrc,
                                                    float* __restrict__ out,
                                                    const float* __restrict__ W1,
                                                    const int* __restrict__ halt,
                                                    const int* __restrict__ run) {
    if (halt && *halt) return;
    if (run && !*run) return;
    __shared__ float w[LF * 9];
    for (int q = threadIdx.x; q < LF * 9; q += 256) w[q] = W1[q];
    __syncthreads();
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= (long)B * H * W) return;
    const int x = (int)(p % W);
    const long bh = p / W;
    const int y = (int)(bh % H);
    const int b = (int)(bh / H);
    const int src = idx ? min(max(idx[b], 0), nsrc - 1) : b;
    float v[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
        v[t] = in_img(yy, xx, H, W) ? in[((size_t)src * H + yy) * W + xx] : 0.0f;
    }
    float* o = out + (size_t)p * LF;
#pragma unroll
    for (int co = 0; co < LF; ++co) {
        float s = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) s = fmaf(w[co * 9 + t], v[t], s);
        o[co] = s;
    }
}

// out[b,h,w] = sum_co sum_t W1[co][t] * in[b, h-dy, w-dx, co]   (adjoint of k_lp_conv_in)
__global__ __launch_bounds__(256) void k_lp_conv_out(int B, int H, int W, const float* __restrict__ in,
                                                     float* __restrict__ out,
                                                     const float* __restrict__ W1,
                                                     const int* __restrict__ halt,
                                                     const int* __restrict__ run) {
    if (halt && *halt) return;
    if (run && !*run) return;
    __shared__ float w[LF * 9];
    for (int q = threadIdx.x; q < LF * 9; q += 256) w[q] = W1[q];
    __syncthreads();
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= (long)B * H * W) return;
    const int x = (int)(p % W);
    const long bh = p / W;
    const int y = (int)(bh % H);
    const int b = (int)(bh / H);
    float s = 0.0f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y - (t / 3 - 1), xx = x - (t % 3 - 1);
        if (!in_img(yy, xx, H, W)) continue;
        const float4* q = reinterpret_cast<const float4*>(in + (((size_t)b * H + yy) * W + xx) * LF);
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
            const float4 u = q[c4];
            s = fmaf(w[(4 * c4 + 0) * 9 + t], u.x, s);
            s = fmaf(w[(4 * c4 + 1) * 9 + t], u.y, s);
            s = fmaf(w[(4 * c4 + 2) * 9 + t], u.z, s);
            s = fmaf(w[(4 * c4 + 3) * 9 + t], u.w, s);
        }
    }
    out[p] = s;
}

// out = scale[c] * in, channels-last
__global__ __launch_bounds__(256) void k_lp_scale(long n16, const float* __restrict__ in,
                                                  const float* __restrict__ scale,
                                                  float* __restrict__ out) {
    const long q = (long)blockIdx.x * 256 + threadIdx.x;
    if (q < n16) out[q] = in[q] * scale[q & (LF - 1)];
}

// softplus(d) and sigmoid(d) into sc[0..15], sg[0..15]
__global__ void k_lp_softplus(const float* __restrict__ d, float* __restrict__ sp_out,
                              float* __restrict__ sg_out) {
    const int c = threadIdx.x;
    if (c < LF) {
        const double x = d[c];
        sp_out[c] = (float)(x > 20.0 ? x : log1p(exp(x)));
        if (sg_out) sg_out[c] = (float)(1.0 / (1.0 + exp(-x)));
    }
}

// ---- loss ---------------------------------------------------------------------
// One workgroup per sample b: nv = ||v||^2, lb = ||z - v||^2 / nv,
// e0 = (2 / B) (z - v) / nv; loss partial lb / B.
// Per sample b: loss over the pixels at least `margin` from every edge,
// e0 = d loss / dz (zero on the margin).
__global__ __launch_bounds__(256) void k_lp_loss(int B, int H, int W, int margin,
                                                 const float* __restrict__ z,
                                                 const float* __restrict__ v,
                                                 const int32_t* __restrict__ idx, int nsrc,
                                                 float* __restrict__ e0,
                                                 double* __restrict__ lpart) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const int HW = H * W;
    const float* vb = v + (size_t)(idx ? min(max(idx[b], 0), nsrc - 1) : b) * HW;
    const float* zb = z + (size_t)b * HW;
    auto inside = [&](int q) {
        const int y = q / W, x = q - (q / W) * W;
        return y >= margin && y < H - margin && x >= margin && x < W - margin;
    };
    double nv = 0.0;
    for (int q = threadIdx.x; q < HW; q += 256)
        if (inside(q)) nv += (double)vb[q] * (double)vb[q];
    nv = block_sum(nv, red);
    const double sc = nv > 0.0 ? 2.0 / ((double)B * nv) : 0.0;
    double r2 = 0.0;
    for (int q = threadIdx.x; q < HW; q += 256) {
        const double r = inside(q) ? (double)zb[q] - (double)vb[q] : 0.0;
        r2 += r * r;
        e0[(size_t)b * HW + q] = (float)(sc * r);
    }
    r2 = block_sum(r2, red);
    if (threadIdx.x == 0) lpart[b] = nv > 0.0 ? r2 / nv / (double)B : 0.0;
}

// ---- weight gradients ----------------------------------------------------------
// partial[blk][o][i][t] = sum over the block's pixels p of G[p][o] * X[p + t][i]
// (X zero outside the image).  G: [B][H][W][16]; X: [B][H][W][FI].  A block
// covers LP_WG_TILES consecutive 16 x 16 pixel tiles of one tile row of one
// image, each staged in LDS in turn (one: more blocks in flight outweigh the
// smaller reduction that larger blocks leave).
constexpr int LP_WG_TILES = 1;

struct WgTile {
    int b, y0, x0, ntile;   // image, tile row origin, first tile's column origin, tiles in the block
};

__device__ __forceinline__ WgTile wg_tile(int blk, int H, int W) {
    const int tx = (W + 15) / 16, ty = (H + 15) / 16;
    const int gx = (tx + LP_WG_TILES - 1) / LP_WG_TILES;
    const int b = blk / (gx * ty);
    const int rem = blk - b * gx * ty;
    const int g = rem % gx;
    WgTile T;
    T.b = b;
    T.y0 = (rem / gx) * 16;
    T.x0 = g * LP_WG_TILES * 16;
    T.ntile = min(LP_WG_TILES, tx - g * LP_WG_TILES);
    return T;
}

// Stages tile j of the block: gs = G over the tile, xs = X over the tile and
// a one-pixel halo (FI channels).
template <int FI, int NT>
__device__ __forceinline__ void wg_stage(const WgTile& T, int j, int H, int W, const float* __restrict__ G,
                                         const float* __restrict__ X, float* gs, float* xs) {
    const int x0 = T.x0 + 16 * j;
    for (int q = threadIdx.x; q < 256 * LF; q += NT) {
        const int p = q / LF, c = q - p * LF;
        const int yy = T.y0 + p / 16, xx = x0 + p % 16;
        gs[q] = in_img(yy, xx, H, W) ? G[(((size_t)T.b * H + yy) * W + xx) * LF + c] : 0.0f;
    }
    for (int q = threadIdx.x; q < 18 * 18 * FI; q += NT) {
        const int p = q / FI, c = q - p * FI;
        const int yy = T.y0 - 1 + p / 18, xx = x0 - 1 + p % 18;
        xs[q] = in_img(yy, xx, H, W) ? X[(((size_t)T.b * H + yy) * W + xx) * FI + c] : 0.0f;
    }
}

// First layer (FI = 1): 16 x 9 outputs, one thread each, on the VALU.
__global__ __launch_bounds__(256) void k_lp_wgrad1(int B, int H, int W, const float* __restrict__ G,
                                                   const float* __restrict__ X,
                                                   float* __restrict__ partial) {
    __shared__ float gs[256 * LF];
    __shared__ float xs[18 * 18];
    const WgTile T = wg_tile(blockIdx.x, H, W);
    const int o = threadIdx.x / 9, t = threadIdx.x % 9;
    float acc = 0.0f;
    for (int j = 0; j < T.ntile; ++j) {
        if (j) __syncthreads();             // the previous tile's reads are done
        wg_stage<1, 256>(T, j, H, W, G, X, gs, xs);
        __syncthreads();
        if (threadIdx.x < LF * 9) {
            for (int p = 0; p < 256; ++p) {
                const int py = p / 16, px = p % 16;
                acc = fmaf(gs[p * LF + o], xs[(py + t / 3) * 18 + px + t % 3], acc);
            }
        }
    }
    if (threadIdx.x < LF * 9) partial[(size_t)blockIdx.x * (LF * 9) + threadIdx.x] = acc;
}

// The 16 -> 16 weight gradient on MFMA: per tap t, dW_t[o][ci] = sum_p
// G[p][o] X[p + t][ci] is a [16 x 256] x [256 x 16] product over a tile's
// pixels.  Nine waves per block, one per tap, each 64 v_mfma_f32_16x16x4f32
// per tile (A = G of 4 pixels, B = X of the same 4 pixels shifted by the tap)
// over the LDS-staged tiles; no cross-wave sum, so the partial of a block is
// written once per output.
constexpr int LP_WG_THREADS = 64 * 9;

__global__ __launch_bounds__(LP_WG_THREADS) void k_lp_wgrad_mfma(int B, int H, int W,
                                                               const float* __restrict__ G,
                                                               const float* __restrict__ X,
                                                               float* __restrict__ partial) {
    __shared__ float gs[256 * LF];
    __shared__ float xs[18 * 18 * LF];
    const WgTile T = wg_tile(blockIdx.x, H, W);
    const int t = threadIdx.x >> 6;          // tap of this wave
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, kq = lane >> 4;
    const int dy = t / 3, dx = t % 3;
    f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int j = 0; j < T.ntile; ++j) {
        if (j) __syncthreads();             // the previous tile's reads are done
        wg_stage<LF, LP_WG_THREADS>(T, j, H, W, G, X, gs, xs);
        __syncthreads();
#pragma unroll 4
        for (int p0 = 0; p0 < 256; p0 += 4) {
            const int p = p0 + kq;           // this lane's K slot: pixel p of the tile
            const int py = p >> 4, px = p & 15;
            const float a = gs[p * LF + i];                              // A[o = i][k] = G[p][o]
            const float bv = xs[((py + dy) * 18 + px + dx) * LF + i];     // B[k][ci = i] = X[p + t][ci]
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc, 0, 0, 0);
        }
    }
    // lane holds D[4 kq + r][i] = dW_t[o = 4 kq + r][ci = i]
    float* dst = partial + (size_t)blockIdx.x * (LF * LF * 9);
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[((4 * kq + r) * LF + i) * 9 + t] = acc[r];
}

// Two-level fixed-order float64 sum over blocks: tmp[chunk][q] sums the
// partials of 64 consecutive blocks, then out[q] (+)= sum over chunks.
constexpr int LP_CHUNK = 64;

__global__ __launch_bounds__(256) void k_lp_reduce1(int nblk, int nout, const float* __restrict__ pa,
                                                    double* __restrict__ tmp) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= nout) return;
    const int k0 = blockIdx.y * LP_CHUNK, k1 = min(nblk, k0 + LP_CHUNK);
    double s = 0.0;
    for (int k = k0; k < k1; ++k) s += (double)pa[(size_t)k * nout + q];
    tmp[(size_t)blockIdx.y * nout + q] = s;
}

__global__ __launch_bounds__(256) void k_lp_reduce2(int nchunk, int nout, const double* __restrict__ tmp,
                                                    int accumulate, float* __restrict__ out) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= nout) return;
    double s = 0.0;
    for (int k = 0; k < nchunk; ++k) s += tmp[(size_t)k * nout + q];
    out[q] = (float)(accumulate ? (double)out[q] + s : s);
}

// gd partials: part[blk][c] = sum over the block's pixels of E[p][c] * A[p][c]
__global__ __launch_bounds__(256) void k_lp_gd_part(long npix, const float* __restrict__ E,
                                                    const float* __restrict__ A,
                                                    double* __restrict__ part) {
    __shared__ double red[256];
    const int c = threadIdx.x & (LF - 1);
    const int lane_pix = threadIdx.x >> 4;   // 16 pixels per pass
    double s = 0.0;
    for (long p = (long)blockIdx.x * 16 + lane_pix; p < npix; p += (long)gridDim.x * 16)
        s += (double)E[p * LF + c] * (double)A[p * LF + c];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < LF) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += red[k * LF + threadIdx.x];
        part[(size_t)blockIdx.x * LF + threadIdx.x] = t;
    }
}

// 16 groups of threads per channel sum strided blocks, then the groups are
// added in order.
__global__ __launch_bounds__(256) void k_lp_gd_final(int nblk, const double* __restrict__ part,
                                                     const float* __restrict__ sg,
                                                     float* __restrict__ gd) {
    __shared__ double red[256];
    const int c = threadIdx.x & (LF - 1), grp = threadIdx.x >> 4;
    double s = 0.0;
    for (int k = grp; k < nblk; k += 16) s += part[(size_t)k * LF + c];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < LF) {
        double t = 0.0;
        for (int g = 0; g < 16; ++g) t += red[g * LF + threadIdx.x];
        gd[threadIdx.x] = (float)(t * (double)sg[threadIdx.x]);
    }
}

__global__ __launch_bounds__(256) void k_lp_adam(int n, float* __restrict__ theta,
                                                 float* __restrict__ m, float* __restrict__ v,
                                                 const float* __restrict__ g, double lr, double b1,
                                                 double b2, double eps, double c1, double c2) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const double gq = g[q];
    const double mq = b1 * (double)m[q] + (1.0 - b1) * gq;
    const double vq = b2 * (double)v[q] + (1.0 - b2) * gq * gq;
    m[q] = (float)mq;
    v[q] = (float)vq;
    theta[q] = (float)((double)theta[q] - lr * (mq / c1) / (sqrt(vq / c2) + eps));
}

// ---- launchers ------------------------------------------------------------------
static inline unsigned nblk(long n, int per) { return (unsigned)((n + per - 1) / per); }

void lp_conv_mid(hipStream_t st, bool trans, int B, int H, int W, const float* in, float* out,
                 const float* Wl, const float* scale, float* out2, const int* halt, const int* run) {
    const long tiles = (long)B * H * ((W + 15) / 16);
    // four tiles per wave once the grid has enough of them to fill the GPU
    if (tiles >= 16384) {
        const unsigned g = nblk(tiles, 16);
        if (trans)
            hipLaunchKernelGGL((k_lp_conv_mid<true, 4>), dim3(g), dim3(256), 0, st, B, H, W, in, out, Wl, scale, out2, halt, run);
        else
            hipLaunchKernelGGL((k_lp_conv_mid<false, 4>), dim3(g), dim3(256), 0, st, B, H, W, in, out, Wl, scale, out2, halt, run);
    } else {
        const unsigned g = nblk(tiles, 4);
        if (trans)
            hipLaunchKernelGGL((k_lp_conv_mid<true, 1>), dim3(g), dim3(256), 0, st, B, H, W, in, out, Wl, scale, out2, halt, run);
        else
            hipLaunchKernelGGL((k_lp_conv_mid<false, 1>), dim3(g), dim3(256), 0, st, B, H, W, in, out, Wl, scale, out2, halt, run);
    }
}

void lp_conv_in(hipStream_t st, int B, int H, int W, const float* in, const int32_t* idx, int nsrc,
                float* out, const float* W1, const int* halt, const int* run) {
    hipLaunchKernelGGL(k_lp_conv_in, dim3(nblk((long)B * H * W, 256)), dim3(256), 0, st, B, H, W, in,
                       idx, nsrc, out, W1, halt, run);
}

__global__ __launch_bounds__(256) void k_lp_gather(int B, int HW, const float* __restrict__ src,
                                                   const int32_t* __restrict__ idx, int nsrc,
                                                   float* __restrict__ dst) {
    const long q = (long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long)B * HW) return;
    const int b = (int)(q / HW);
    const int s = min(max(idx[b], 0), nsrc - 1);
    dst[q] = src[(size_t)s * HW + (q - (long)b * HW)];
}

void lp_gather(hipStream_t st, int B, int HW, const float* src, const int32_t* idx, int nsrc, float* dst) {
    hipLaunchKernelGGL(k_lp_gather, dim3(nblk((long)B * HW, 256)), dim3(256), 0, st, B, HW, src, idx,
                       nsrc, dst);
}

void lp_conv_out(hipStream_t st, int B, int H, int W, const float* in, float* out, const float* W1,
                 const int* halt, const int* run) {
    hipLaunchKernelGGL(k_lp_conv_out, dim3(nblk((long)B * H * W, 256)), dim3(256), 0, st, B, H, W,
                       in, out, W1, halt, run);
}

void lp_scale(hipStream_t st, long npix, const float* in, const float* scale, float* out) {
    hipLaunchKernelGGL(k_lp_scale, dim3(nblk(npix * LF, 256)), dim3(256), 0, st, npix * LF, in, scale, out);
}

void lp_softplus(hipStream_t st, const float* d, float* sp_out, float* sg_out) {
    hipLaunchKernelGGL(k_lp_softplus, dim3(1), dim3(64), 0, st, d, sp_out, sg_out);
}

void lp_loss(hipStream_t st, int B, int H, int W, int margin, const float* z, const float* v,
             const int32_t* idx, int nsrc, float* e0, double* lpart) {
    hipLaunchKernelGGL(k_lp_loss, dim3(B), dim3(256), 0, st, B, H, W, margin, z, v, idx, nsrc, e0,
                       lpart);
}

int lp_wgrad_blocks(int B, int H, int W) {
    return B * ((H + 15) / 16) * (((W + 15) / 16 + LP_WG_TILES - 1) / LP_WG_TILES);
}

void lp_wgrad(hipStream_t st, int fi, int B, int H, int W, const float* G, const float* X, float* partial) {
    const unsigned g = (unsigned)lp_wgrad_blocks(B, H, W);
    if (fi == LF)
        hipLaunchKernelGGL(k_lp_wgrad_mfma, dim3(g), dim3(LP_WG_THREADS), 0, st, B, H, W, G, X, partial);
    else
        hipLaunchKernelGGL(k_lp_wgrad1, dim3(g), dim3(256), 0, st, B, H, W, G, X, partial);
}

int lp_reduce_chunks(int nb) { return (nb + LP_CHUNK - 1) / LP_CHUNK; }

void lp_reduce(hipStream_t st, int nb, int nout, const float* pa, bool accumulate, float* out,
               double* tmp) {
    const int nch = lp_reduce_chunks(nb);
    hipLaunchKernelGGL(k_lp_reduce1, dim3(nblk(nout, 256), nch), dim3(256), 0, st, nb, nout, pa, tmp);
    hipLaunchKernelGGL(k_lp_reduce2, dim3(nblk(nout, 256)), dim3(256), 0, st, nch, nout, tmp,
                       accumulate ? 1 : 0, out);
}

int lp_gd_blocks() { return 2048; }

void lp_gd(hipStream_t st, long npix, const float* E, const float* A, double* part, const float* sg,
           float* gd) {
    hipLaunchKernelGGL(k_lp_gd_part, dim3(lp_gd_blocks()), dim3(256), 0, st, npix, E, A, part);
    hipLaunchKernelGGL(k_lp_gd_final, dim3(1), dim3(256), 0, st, lp_gd_blocks(), part, sg, gd);
}

void lp_adam(hipStream_t st, int n, float* theta, float* m, float* v, const float* g, double lr,
             double b1, double b2, double eps, int step) {
    const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    hipLaunchKernelGGL(k_lp_adam, dim3(nblk(n, 256)), dim3(256), 0, st, n, theta, m, v, g, lr, b1, b2,
                       eps, c1, c2);
}

}  // namespace sp
