// Matrix-free parallel-beam projector R (ray-driven gather) and its exact
// transpose R^T (pixel-driven gather, no atomics).
//
// R[(a,k),(i,j)] is the length of ray (a,k) inside pixel (i,j) (the projection
// matrix of Section 2, rays as in Section 4.1).  Both operators evaluate the
// weight with the same float64 instruction sequence (projection t of the pixel
// centre, offset d = s_k - t, chord_w), so R^T uses bit-identical weights and is
// the exact adjoint up to summation order.  Data are float32; offsets, weights
// and sums are float64 (FP64 FMA issues at the non-packed FP32 rate on CDNA4,
// and float32 angles alone would move a ray by ~1e-5 pixel at radius 256).
//
// Canonical projection of pixel centre (xj, yi) on the normal of angle a:
//   |c| >= |s| ("vertical" angles):   t = fma(xj, c, yi * s)
//   |s| >  |c| ("horizontal" angles): t = fma(yi, s, xj * c)
// The product outside the fma is the one a forward walk shares between the
// candidates of one step.
//
// Forward walk.  For a vertical angle a ray crosses every image row; at row i
// its nonzero pixels lie within hw columns of the crossing point, which moves
// by `slope` columns per row.  A lane owns one ray; the 64 lanes of a wave hold
// consecutive rays of one angle and walk the union of their row ranges
// together, so each step gathers consecutive addresses of one row.  Candidate
// columns outside the image are clamped into a zero pad and contribute 0.
// Horizontal angles walk columns of a zero-padded transposed copy.
//
// Backward gather.  A lane owns one pixel and loops over the angles, which are
// sorted into four classes (vertical/horizontal x oblique/axis-parallel) so
// the inner loop has no branch; at each angle the pixel's nonzero bins are the
// NB bins after floor(kf - hb), read from a zero-padded sinogram.
#include "sp_internal.h"
#include "sp_reduce.h"

namespace sp {

// 32 x 32 tile (bx, by): padded copy and padded transposed copy.
__device__ __forceinline__ void prep_body(const GeomDev& G, const float* __restrict__ x,
                                          float* __restrict__ xp, float* __restrict__ xTp, int bx,
                                          int by) {
    __shared__ float tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int j = bx * 32 + tx;
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int i = by * 32 + ty + r;
        float v = 0.0f;
        if (i < G.rows && j < G.cols) {
            v = x[(size_t)i * G.cols + j];
            xp[(size_t)i * G.pitchX + PAD + j] = v;
        }
        tile[ty + r][tx] = v;
    }
    __syncthreads();
    const int ii = by * 32 + tx;
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int jj = bx * 32 + ty + r;
        if (ii < G.rows && jj < G.cols) xTp[(size_t)jj * G.pitchXT + PAD + ii] = tile[tx][ty + r];
    }
}

__global__ __launch_bounds__(256) void k_prep(GeomDev G, const float* __restrict__ x,
                                              float* __restrict__ xp, float* __restrict__ xTp,
                                              const int* __restrict__ halt) {
    if (halt && *halt) return;
    prep_body(G, x, xp, xTp, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void kb_prep(const SliceDev* __restrict__ sl, ItemTable t, int which) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const GeomDev G = S.G;
        const int gx = (G.cols + 31) / 32;
        prep_body(G, batch_vec(S, which), gmem(S.xp), gmem(S.xTp), lin % gx, lin / gx);
    });
}

void launch_prep_b(hipStream_t st, const SliceDev* sl, ItemTable t, int which) {
    hipLaunchKernelGGL(kb_prep, dim3(t.grid), dim3(256), 0, st, sl, t, which);
}

void launch_prep(hipStream_t st, const GeomDev& G, const float* x, float* xp, float* xTp,
                 const int* halt) {
    dim3 grid((G.cols + 31) / 32, (G.rows + 31) / 32);
    hipLaunchKernelGGL(k_prep, grid, dim3(256), 0, st, G, x, xp, xTp, halt);
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Major-axis steps [lo, hi) of [0, n) where base + m * slope lies in [vlo, vhi],
// widened by one step on each side (candidate selection only).
__device__ __forceinline__ void step_range(double base, double slope, double vlo, double vhi, int n,
                                           int& lo, int& hi) {
    if (slope == 0.0) {
        const bool in = base >= vlo && base <= vhi;
        lo = 0;
        hi = in ? n : 0;
        return;
    }
    const double t0 = (vlo - base) / slope, t1 = (vhi - base) / slope;
    double tmin = fmin(t0, t1) - 1.0, tmax = fmax(t0, t1) + 2.0;
    tmin = fmin(fmax(tmin, 0.0), (double)n);
    tmax = fmin(fmax(tmax, 0.0), (double)n);
    lo = (int)floor(tmin);
    hi = (int)ceil(tmax);
    if (hi < lo) hi = lo;
}

// One ray's sum.  HORIZ = walk columns of the transposed copy.  img points at
// element PAD of row 0 of the padded copy.
template <bool HORIZ, bool AXIS, int NC>
__device__ __forceinline__ double ray_sum(const GeomDev& G, const AngleDev& A, double sk,
                                          const float* __restrict__ img, bool valid) {
    const int nmaj = HORIZ ? G.cols : G.rows;
    const int nmin = HORIZ ? G.rows : G.cols;
    const int pitch = HORIZ ? G.pitchXT : G.pitchX;
    const double fM = HORIZ ? A.c : A.s;   // factor of the shared (major) product
    const double fm = HORIZ ? A.s : A.c;   // factor of the per-candidate fma
    // fractional minor index of the ray's crossing at major step 0, minus hw
    const double start = (HORIZ ? G.yoff - (sk + G.xoff * A.c) / A.s
                                : (sk - G.yoff * A.s) / A.c + G.xoff) - (double)A.hw;
    int lo, hi;
    step_range(start, A.slope, -(double)(NC + 1), (double)(nmin + 1), nmaj, lo, hi);
    if (!valid) {
        lo = nmaj;
        hi = 0;
    }
    lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    double acc = 0.0;
    if (lo >= hi) return acc;
    // Candidate n of step m is minor index floor(nf_m) + 1 + q, clamped so that
    // the NC reads stay inside the padded row (clamped reads hit zero pads).
    // Offsets are kept relative to the start of the padded row (>= 0).
    const float* row = img - PAD;
    // minor coordinate of candidate 0 = floor(nf) + c1 (exact: small half-integers)
    const double c1 = HORIZ ? G.yoff - 1.0 : 1.0 - G.xoff;
    const double dM = HORIZ ? 1.0 : -1.0;                     // major coordinate step
    double cM = HORIZ ? (double)lo - G.xoff : G.yoff - (double)lo;
    double nf = fma((double)lo, A.slope, start);
    const int omax = nmin + 2 * PAD - NC;
    const float* rp = row + (size_t)lo * pitch;
    // one major step: gather is issued by the caller, weights and sum here
    auto step = [&](const float* v, double nfl, double cMv) {
        const double P = cMv * fM;
        const double cm0 = HORIZ ? c1 - nfl : nfl + c1;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const double cm = HORIZ ? cm0 - (double)q : cm0 + (double)q;
            const double d = sk - fma(cm, fm, P);
            acc = fma(chord_w<AXIS>(d, A.einv, A.inv, A.wmax), (double)v[q], acc);
        }
    };
    int m = lo;
    // two steps per iteration: both gathers are in flight before either step's math
    for (; m + 1 < hi; m += 2) {
        const double nfl0 = floor(nf);
        const double nfl1 = floor(nf + A.slope);
        const float* p0 = rp + min(max((int)nfl0 + 1 + PAD, 0), omax);
        const float* p1 = rp + pitch + min(max((int)nfl1 + 1 + PAD, 0), omax);
        float v0[NC], v1[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) v0[q] = p0[q];
#pragma unroll
        for (int q = 0; q < NC; ++q) v1[q] = p1[q];
        step(v0, nfl0, cM);
        step(v1, nfl1, cM + dM);
        nf += 2.0 * A.slope;
        cM += 2.0 * dM;
        rp += 2 * pitch;
    }
    if (m < hi) {
        const double nfl0 = floor(nf);
        const float* p0 = rp + min(max((int)nfl0 + 1 + PAD, 0), omax);
        float v0[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) v0[q] = p0[q];
        step(v0, nfl0, cM);
    }
    return acc;
}

template <bool HORIZ, bool AXIS>
__device__ __forceinline__ double ray_sum_nc(const GeomDev& G, const AngleDev& A, double sk,
                                             const float* __restrict__ img, bool valid) {
    return A.nc == 3 ? ray_sum<HORIZ, AXIS, 3>(G, A, sk, img, valid)
                     : ray_sum<HORIZ, AXIS, 2>(G, A, sk, img, valid);
}

// out[row*out_pitch + out_pad + k] = (R x)_{row,k}, or the residual (R x - b)
// with its float64 squared norm per workgroup in partials when b != nullptr.
// Block bx indexes the class-sorted angle table, by the 256-bin chunk.
__device__ __forceinline__ void project_body(const GeomDev& G, const AngleDev* __restrict__ ang,
                                             const float* __restrict__ xp,
                                             const float* __restrict__ xTp,
                                             const float* __restrict__ b, float* __restrict__ out,
                                             int out_pitch, int out_pad,
                                             double* __restrict__ partials, int bx, int by, int gx) {
    __shared__ double red[4];
    const AngleDev A = ang[bx];
    const int a = A.row;
    const int k = by * 256 + threadIdx.x;
    const bool valid = k < G.nB;
    const double sk = bin_pos((double)k, G);
    const bool horiz = A.flags & ANG_HORIZ, axis = A.flags & ANG_AXIS;
    double acc;
    if (!horiz) {
        acc = axis ? ray_sum_nc<false, true>(G, A, sk, xp + PAD, valid)
                   : ray_sum_nc<false, false>(G, A, sk, xp + PAD, valid);
    } else {
        acc = axis ? ray_sum_nc<true, true>(G, A, sk, xTp + PAD, valid)
                   : ray_sum_nc<true, false>(G, A, sk, xTp + PAD, valid);
    }
    double r2 = 0.0;
    if (valid) {
        float val;
        if (b) {
            val = (float)(fma(acc, G.pixel, -(double)b[(size_t)a * G.nB + k]));
            r2 = (double)val * (double)val;
        } else {
            val = (float)(acc * G.pixel);
        }
        out[(size_t)a * out_pitch + out_pad + k] = val;
    }
    if (b) {
        const double tot = block_sum(r2, red);
        if (threadIdx.x == 0) partials[by * gx + bx] = tot;
    }
}

__global__ __launch_bounds__(256) void k_project(GeomDev G, const AngleDev* __restrict__ ang,
                                                 const float* __restrict__ xp,
                                                 const float* __restrict__ xTp,
                                                 const float* __restrict__ b,
                                                 float* __restrict__ out, int out_pitch,
                                                 int out_pad, double* __restrict__ partials,
                                                 const int* __restrict__ halt) {
    if (halt && *halt) return;
    project_body(G, ang, xp, xTp, b, out, out_pitch, out_pad, partials, blockIdx.x, blockIdx.y,
                 gridDim.x);
}

// residual: rp = R xh - b with f partials; else rp = R p.
__global__ __launch_bounds__(256) void kb_project(const SliceDev* __restrict__ sl, ItemTable t,
                                                  int residual) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const GeomDev G = S.G;
        const int gx = G.nA;
        project_body(G, cmem(S.ang), gmem(S.xp), gmem(S.xTp), residual ? gmem(S.b) : nullptr,
                     gmem(S.rp) + PAD, G.pitchB, 0, residual ? gmem(S.pf) : nullptr, lin % gx,
                     lin / gx, gx);
    });
}

void launch_project_b(hipStream_t st, const SliceDev* sl, ItemTable t, bool residual) {
    hipLaunchKernelGGL(kb_project, dim3(t.grid), dim3(256), 0, st, sl, t, residual ? 1 : 0);
}

int project_blocks(const GeomDev& G) { return G.nA * ((G.nB + 255) / 256); }

void launch_project(hipStream_t st, const GeomDev& G, const AngleDev* ang, const float* xp,
                    const float* xTp, const float* b, float* out, int out_pitch, int out_pad,
                    double* partials, const int* halt) {
    dim3 grid(G.nA, (G.nB + 255) / 256);
    hipLaunchKernelGGL(k_project, grid, dim3(256), 0, st, G, ang, xp, xTp, b, out, out_pitch,
                       out_pad, partials, halt);
}

__global__ __launch_bounds__(256) void k_pad_sino(GeomDev G, const float* __restrict__ y,
                                                  float* __restrict__ yp) {
    const int a = blockIdx.x;
    for (int k = threadIdx.x; k < G.nB; k += 256)
        yp[(size_t)a * G.pitchB + PAD + k] = y[(size_t)a * G.nB + k];
}

void launch_pad_sino(hipStream_t st, const GeomDev& G, const float* y, float* yp) {
    hipLaunchKernelGGL(k_pad_sino, dim3(G.nA), dim3(256), 0, st, G, y, yp);
}

// Sum over the angles [beg, end) of one class for pixel (xj, yi).  The angle
// and its sinogram row are wave-uniform (scalar loads); lanes differ only in
// the pixel.
template <bool HORIZ, bool AXIS, int NB>
__device__ __forceinline__ double bp_class(const GeomDev& G, const AngleDev* __restrict__ ang,
                                           int beg, int end, const float* __restrict__ yp,
                                           double xj, double yi, double acc) {
    const int kmax = G.nB + 2 * PAD - NB;        // last padded start index
#pragma unroll 2
    for (int a = beg; a < end; ++a) {
        const AngleDev A = ang[a];
        const double t = HORIZ ? fma(yi, A.s, xj * A.c) : fma(xj, A.c, yi * A.s);
        const double kfl = floor(fma(t, G.inv_ds, A.kb));
        // padded index of candidate bin floor(kf) + 1, clamped into the zero pads
        const unsigned o = (unsigned)min(max((int)kfl + 1 + PAD, 0), kmax);
        const float* pr = yp + (size_t)A.row * G.pitchB;
        float v[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) v[q] = pr[o + q];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const double d = bin_pos(kfl + (double)(1 + q), G) - t;
            acc = fma(chord_w<AXIS>(d, A.einv, A.inv, A.wmax), (double)v[q], acc);
        }
    }
    return acc;
}

constexpr int BP_TILE = 8;      // 8 x 8 pixels per wave
constexpr int BP_SPLIT = 4;     // waves per workgroup, each over a quarter of the angles

__device__ __forceinline__ void split_range(int beg, int end, int w, int& b, int& e) {
    const int len = end - beg;
    b = beg + (len * w) / BP_SPLIT;
    e = beg + (len * (w + 1)) / BP_SPLIT;
}

// out[i][j] = (R^T y)_{ij} from the padded sinogram yp; with dotv != nullptr
// also the float64 partial sum of out * dotv per workgroup.  A workgroup owns
// an 8 x 8 pixel tile; its wave w sums the w-th quarter of every angle class,
// and the four partial sums are added in wave order through LDS.
template <int NB>
__device__ __forceinline__ void backproject_body(const GeomDev& G, const AngleDev* __restrict__ ang,
                                                 const float* __restrict__ yp,
                                                 float* __restrict__ out,
                                                 const float* __restrict__ dotv,
                                                 double* __restrict__ partials, int bx, int by,
                                                 int gx) {
    __shared__ double part[BP_SPLIT][64];
    __shared__ double red[4];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = by * BP_TILE + (lane >> 3);
    const int j = bx * BP_TILE + (lane & 7);
    const double xj = (double)j - G.xoff;
    const double yi = G.yoff - (double)i;
    double acc = 0.0;
    int b, e;
    split_range(G.cls[0], G.cls[1], w, b, e);
    acc = bp_class<false, false, NB>(G, ang, b, e, yp, xj, yi, acc);
    split_range(G.cls[1], G.cls[2], w, b, e);
    acc = bp_class<true, false, NB>(G, ang, b, e, yp, xj, yi, acc);
    split_range(G.cls[2], G.cls[3], w, b, e);
    acc = bp_class<false, true, NB>(G, ang, b, e, yp, xj, yi, acc);
    split_range(G.cls[3], G.cls[4], w, b, e);
    acc = bp_class<true, true, NB>(G, ang, b, e, yp, xj, yi, acc);
    part[w][lane] = acc;
    __syncthreads();
    double v = 0.0;
    if (w == 0) {
        const double tot = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        const float val = (float)(tot * G.pixel);
        const bool valid = i < G.rows && j < G.cols;
        if (valid) {
            out[(size_t)i * G.cols + j] = val;
            if (dotv) v = (double)val * (double)dotv[(size_t)i * G.cols + j];
        }
    }
    if (dotv) {
        const double tot = block_sum(v, red);
        if (threadIdx.x == 0) partials[by * gx + bx] = tot;
    }
}

template <int NB>
__global__ __launch_bounds__(256) void k_backproject(GeomDev G, const AngleDev* __restrict__ ang,
                                                     const float* __restrict__ yp,
                                                     float* __restrict__ out,
                                                     const float* __restrict__ dotv,
                                                     double* __restrict__ partials,
                                                     const int* __restrict__ halt) {
    if (halt && *halt) return;
    backproject_body<NB>(G, ang, yp, out, dotv, partials, blockIdx.x, blockIdx.y, gridDim.x);
}

// normal: h = R^T rp with the partials of h^T p; else g = R^T rp.  NB is the
// largest candidate count of the batch (extra candidates weigh exactly 0).
template <int NB>
__global__ __launch_bounds__(256) void kb_backproject(const SliceDev* __restrict__ sl, ItemTable t,
                                                      int normal) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const GeomDev G = S.G;
        const int gx = (G.cols + BP_TILE - 1) / BP_TILE;
        backproject_body<NB>(G, cmem(S.ang), gmem(S.rp), gmem(normal ? S.h : S.g),
                             normal ? gmem(S.p) : nullptr, normal ? gmem(S.pph) : nullptr,
                             lin % gx, lin / gx, gx);
    });
}

void launch_backproject_b(hipStream_t st, const SliceDev* sl, ItemTable t, int nbmax, bool normal) {
    const int nm = normal ? 1 : 0;
    switch (nbmax) {
    case 1: hipLaunchKernelGGL(kb_backproject<1>, dim3(t.grid), dim3(256), 0, st, sl, t, nm); break;
    case 2: hipLaunchKernelGGL(kb_backproject<2>, dim3(t.grid), dim3(256), 0, st, sl, t, nm); break;
    case 3: hipLaunchKernelGGL(kb_backproject<3>, dim3(t.grid), dim3(256), 0, st, sl, t, nm); break;
    default: hipLaunchKernelGGL(kb_backproject<4>, dim3(t.grid), dim3(256), 0, st, sl, t, nm); break;
    }
}

int backproject_blocks(const GeomDev& G) {
    return ((G.cols + BP_TILE - 1) / BP_TILE) * ((G.rows + BP_TILE - 1) / BP_TILE);
}

void launch_backproject(hipStream_t st, const GeomDev& G, const AngleDev* ang, const float* yp,
                        float* out, const float* dotv, double* partials, const int* halt) {
    dim3 grid((G.cols + BP_TILE - 1) / BP_TILE, (G.rows + BP_TILE - 1) / BP_TILE);
    switch (G.nbmax) {
    case 1: hipLaunchKernelGGL(k_backproject<1>, grid, dim3(256), 0, st, G, ang, yp, out, dotv, partials, halt); break;
    case 2: hipLaunchKernelGGL(k_backproject<2>, grid, dim3(256), 0, st, G, ang, yp, out, dotv, partials, halt); break;
    case 3: hipLaunchKernelGGL(k_backproject<3>, grid, dim3(256), 0, st, G, ang, yp, out, dotv, partials, halt); break;
    default: hipLaunchKernelGGL(k_backproject<4>, grid, dim3(256), 0, st, G, ang, yp, out, dotv, partials, halt); break;
    }
}

}  // namespace sp
