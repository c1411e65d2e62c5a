// Matrix-free parallel-beam projector R (ray-driven gather) and its exact
// transpose R^T (pixel-driven gather, no atomics).
//
// R[(a,k),(i,j)] is the length of ray (a,k) inside pixel (i,j) (the projection
// matrix of Section 2, rays as in Section 4.1).  R^T evaluates each weight as
// the chord length of a line through a square (offset d = s_k - t of the bin
// from the projection t of the pixel centre, the clamped trapezoid u of
// chord_u, times the angle's wmax).  R walks each ray band by band and splits
// a band's path length at the pixel boundary it crosses (ray_split): the same
// lengths in exact arithmetic, equal to rounding in float64, so R^T is the
// adjoint of R to float64 rounding (axis-parallel angles use the trapezoid in
// both, bit for bit, with its half weight for a ray on a pixel edge).  Data
// are float32; coordinates, weights and sums are float64 (FP64 FMA issues at
// the non-packed FP32 rate on CDNA4, and float32 angles alone would move a ray
// by ~1e-5 pixel at radius 256).
//
// Gathers stay inside one zero-padded row (of the image copy, its transpose or
// the sinogram).  R^T reads through buffer loads whose descriptor spans the
// row, so an index past either end reads 0 in hardware; R clamps its index
// into the row's pads.  A legitimate candidate always lies inside the row (its
// pads included), which the host index checker verifies for every geometry it
// is given.
//
// Forward walk.  For a vertical angle a ray crosses every image row; within
// row i it meets at most two pixels, as its crossing point moves by `slope`
// (|slope| <= 1) columns per row.  A lane owns one ray and the 64 lanes of a
// wave walk the union of their (nonempty) row ranges together, so each step
// gathers neighbouring addresses of one row.  R's wave table (WaveDev) gives
// each wave its rays: 16 consecutive bins of four neighbouring angles (rays
// whose image extents differ little, so few lane-steps fall outside a lane's
// own ray), the last nB % 16 bins of consecutive angles of one class packed
// into full waves, or 64 bins of one axis-parallel angle; a workgroup's four
// waves are four consecutive table entries (the four 16-bin parts of one
// 64-bin chunk of the same angles), and the workgroups run in a
// host-computed order (project_order).  Horizontal angles walk columns of a zero-padded
// transposed copy.
//
// Backward gather.  A lane owns PX (2 or 4) pixels of one row, 8 columns
// apart, and loops over the angles, which are sorted into four classes
// (vertical/horizontal x oblique/axis-parallel) so the inner loop has no
// branch; at each angle a pixel's nonzero bins are the NB bins from padded
// index trunc(kf), read from a zero-padded sinogram (float32, or float64 for
// the solvers' residual) whose rows carry the angle's wmax.
#include "sp_internal.h"
#include "sp_reduce.h"
#include "sp_scalar.h"
#include "sp_walk.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace sp {

// 32 x 32 tile (bx, by): padded copy and padded transposed copy of a float32
// image or of a float64 iterate.
template <class T>
__device__ __forceinline__ void prep_body(const GeomDev& G, const T* __restrict__ x,
                                          double* __restrict__ xp, double* __restrict__ xTp, int bx,
                                          int by) {
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int j = bx * 32 + tx;
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int i = by * 32 + ty + r;
        T v = 0;
        if (i < G.rows && j < G.cols) {
            v = x[(size_t)i * G.cols + j];
            xp[(size_t)i * G.pitchX + PAD + j] = (double)v;
        }
        tile[ty + r][tx] = v;
    }
    __syncthreads();
    const int ii = by * 32 + tx;
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int jj = bx * 32 + ty + r;
        if (ii < G.rows && jj < G.cols)
            xTp[(size_t)jj * G.pitchXT + PAD + ii] = (double)tile[tx][ty + r];
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_prep(GeomDev G, const T* __restrict__ x,
                                              double* __restrict__ xp, double* __restrict__ xTp,
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
        if (which == BV_Z) prep_body(G, (const float*)gmem(S.z), gmem(S.xp), gmem(S.xTp), lin % gx, lin / gx);
        else prep_body(G, (const double*)batch_vec(S, which), gmem(S.xp), gmem(S.xTp), lin % gx, lin / gx);
    });
}

void launch_prep_b(hipStream_t st, const SliceDev* sl, ItemTable t, int which) {
    hipLaunchKernelGGL(kb_prep, dim3(t.grid), dim3(256), 0, st, sl, t, which);
}

void launch_prep(hipStream_t st, const GeomDev& G, const float* x, double* xp, double* xTp,
                 const int* halt) {
    dim3 grid((G.cols + 31) / 32, (G.rows + 31) / 32);
    hipLaunchKernelGGL(k_prep<float>, grid, dim3(256), 0, st, G, x, xp, xTp, halt);
}

void launch_prep(hipStream_t st, const GeomDev& G, const double* x, double* xp, double* xTp,
                 const int* halt) {
    dim3 grid((G.cols + 31) / 32, (G.rows + 31) / 32);
    hipLaunchKernelGGL(k_prep<double>, grid, dim3(256), 0, st, G, x, xp, xTp, halt);
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

// ---- range-checked row gathers ---------------------------------------------
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
// Descriptor word 3 of a raw gfx9 buffer (32-bit data format, no swizzle).
constexpr int BUF_WORD3 = 0x00020000;

// Buffer resource over `bytes` bytes from `row` (wave-uniform).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* row, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(row), (short)0, bytes, BUF_WORD3);
}

// The N elements e, e + 1, ... of a row; every element past either end of the
// row reads 0 (e is taken as unsigned, so a negative index is past the end).
template <class T, int N>
__device__ __forceinline__ void row_load(__amdgpu_buffer_rsrc_t r, unsigned e, T (&v)[N]) {
    const unsigned off = e * (unsigned)sizeof(T);
    if constexpr (sizeof(T) == 8 && N == 2) {
        const d2v t = __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
        v[0] = t.x;
        v[1] = t.y;
    } else if constexpr (sizeof(T) == 4 && N == 2) {
        const f2v t = __builtin_bit_cast(f2v, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
        v[0] = t.x;
        v[1] = t.y;
    } else if constexpr (sizeof(T) == 4 && N == 4) {
        const f4v t = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    } else {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            if constexpr (sizeof(T) == 8)
                v[q] = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(r, off + 8u * q, 0, 0));
            else
                v[q] = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(r, off + 4u * q, 0, 0));
        }
    }
}

// The forward walks gather with plain global loads from a row, the index
// clamped to the row's last full window: a clamped index lands in the row's
// zero pads, and every true candidate of such a step lies outside the image.
// (Buffer loads, whose descriptor is rebuilt per row on the scalar unit,
// measured 3-4% slower here; the backprojector, one row per angle, gains.)
struct RowRef {
    const char* p;
    int bytes;
};
__device__ __forceinline__ RowRef row_ref(const void* row, int bytes) {
    return RowRef{reinterpret_cast<const char*>(row), bytes};
}
template <class T, int N>
__device__ __forceinline__ void row_load(RowRef r, unsigned e, T (&v)[N]) {
    const unsigned emax = (unsigned)(r.bytes / (int)sizeof(T) - N);
    e = min(e, emax);
    const T* q = reinterpret_cast<const T*>(r.p) + e;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = q[i];
}
// ---- forward walk ----------------------------------------------------------
// The wave's common step range from the lanes' own ranges: lanes without a
// ray, or whose ray misses the image, take no part.  Then part `part` of it.
__device__ __forceinline__ bool wave_steps_dev(int l, int h, bool valid, int nmaj, int part,
                                               int nparts, int& lo, int& hi) {
    if (!valid || l >= h) {
        l = nmaj;
        h = 0;
    }
    lo = __builtin_amdgcn_readfirstlane(wave_min(l));
    hi = __builtin_amdgcn_readfirstlane(wave_max(h));
    part_range(lo, hi, part, nparts);
    return lo < hi;
}

// One axis-parallel ray's sum, or part `part` of nparts of it, with the
// trapezoid per candidate (its half weight for a ray on a pixel edge).
// HORIZ = walk columns of the transposed copy.  img points at element PAD of
// row 0 of the padded copy.  Candidate q of step m is minor index
// floor(nf_m) + 1 + q; nf carries the + 1 + PAD of the padded index, so the
// first candidate's padded index is trunc(nf) where nf >= 0 (a negative nf
// reads past the row's start, i.e. 0, as does any index past its end; every
// true candidate of such a step lies outside the image).  The minor coordinate
// of candidate q is taken from the index read -- (o + q - PAD) - xoff for
// columns, yoff - (o + q - PAD) for rows, exact small half-integers.
// Axis-parallel rays cross the whole image, so their waves are among the
// longest of the launch: U steps per iteration keep U gathers in flight, as a
// wave's walk is otherwise bound by the latency of its chain of gathers.
template <bool HORIZ>
__device__ __forceinline__ double ray_sum_axis(const GeomDev& G, const AngleDev& A, double sk,
                                               const double* __restrict__ img, bool valid,
                                               int part, int nparts) {
    constexpr int NC = 2, U = 4;
    const int nmaj = HORIZ ? G.cols : G.rows;
    const int pitch = HORIZ ? G.pitchXT : G.pitchX;
    int l, h, lo, hi;
    ray_steps<HORIZ>(G, A, sk, l, h);
    double acc = 0.0;
    if (!wave_steps_dev(l, h, valid, nmaj, part, nparts, lo, hi)) return acc;
    const double start = walk_start<HORIZ>(G, A, sk);
    const double fm = HORIZ ? A.s : A.c;   // factor of the per-candidate fma
    const double c2 = HORIZ ? G.yoff + (double)PAD : -(double)PAD - G.xoff;
    const double fM = HORIZ ? A.c : A.s;   // factor of the shared (major) product
    const double dM = HORIZ ? 1.0 : -1.0;  // major coordinate step
    double cM = HORIZ ? (double)lo - G.xoff : G.yoff - (double)lo;
    double nf = fma((double)lo, A.slope, start + (double)(1 + PAD));
    const int rowbytes = pitch * 8;
    const char* rowp = reinterpret_cast<const char*>(img - PAD) + (size_t)lo * rowbytes;
    auto step = [&](const double (&v)[NC], int o, double cMv) {
        const double P = cMv * fM;
        const double cm0 = HORIZ ? c2 - (double)o : (double)o + c2;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const double cm = HORIZ ? cm0 - (double)q : cm0 + (double)q;
            const double d = sk - fma(cm, fm, P);
            acc = fma(chord_u<true>(d, A.einv, A.inv), v[q], acc);
        }
    };
    int m = lo;
    for (; m + U <= hi; m += U) {
        int o[U];
        double v[U][NC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            o[u] = (int)nf;
            row_load<double, NC>(row_ref(rowp + u * rowbytes, rowbytes), (unsigned)o[u], v[u]);
            nf += A.slope;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            step(v[u], o[u], cM);
            cM += dM;
        }
        rowp += U * rowbytes;
    }
    for (; m < hi; ++m) {
        const int o = (int)nf;
        double v[NC];
        row_load<double, NC>(row_ref(rowp, rowbytes), (unsigned)o, v);
        step(v, o, cM);
        nf += A.slope;
        cM += dM;
        rowp += rowbytes;
    }
    return acc;
}

// One oblique ray's sum of u-weighted values, or part `part` of it, by
// splitting each major step's band at the pixel boundary.  With |slope| <= 1
// the ray crosses a band (an image row for vertical angles, a column of the
// transposed copy for horizontal ones) over a minor-axis interval of length
// |slope| starting at lp = b0 + m * slope (padded minor coordinate, pixel q
// spanning [q, q + 1)), so it meets at most pixels floor(lp) and
// floor(lp) + 1.  The share of the band's path length (wmax, applied by the
// caller) in the first is f = clamp((floor(lp) + 1 - lp) / |slope|, 0, 1) =
// clamp((1 - fract(lp)) / |slope|, 0, 1) and the rest falls in the second:
// the exact chord lengths of the pixel model, the same values chord_u * wmax
// gives up to rounding.  lp advances by slope per step (its rounding error
// stays ~1e-11 pixel over the longest walk).  A truncated index below the row
// or past it reads 0, where the pixels contribute 0.  The longest waves set
// the launch's length and their walk is bound by the latency of its chain of
// gathers, so U steps' gathers are issued before their math.
template <bool HORIZ>
__device__ __forceinline__ double ray_split(const GeomDev& G, const AngleDev& A, double sk,
                                            const double* __restrict__ img, bool valid, int part,
                                            int nparts) {
    const int nmaj = HORIZ ? G.cols : G.rows;
    const int pitch = HORIZ ? G.pitchXT : G.pitchX;
    int l, h, lo, hi;
    ray_steps<HORIZ>(G, A, sk, l, h);
    double acc = 0.0;
    if (!wave_steps_dev(l, h, valid, nmaj, part, nparts, lo, hi)) return acc;
    constexpr int U = 2;   // steps per iteration: their gathers are in flight together
    const double sig = A.slope;
    const double isg = 1.0 / fabs(sig);
    double lp = fma((double)lo, sig, split_b0<HORIZ>(G, A, sk));
    const int rowbytes = pitch * 8;
    const char* rowp = reinterpret_cast<const char*>(img - PAD) + (size_t)lo * rowbytes;
    auto step = [&](const double (&v)[2], double lpv) {
        const double f = fmin(fmax(fma(__builtin_amdgcn_fract(lpv), -isg, isg), 0.0), 1.0);
        acc += fma(f, v[0] - v[1], v[1]);
    };
    int m = lo;
    for (; m + U <= hi; m += U) {
        double lpu[U], v[U][2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            lpu[u] = lp;
            row_load<double, 2>(row_ref(rowp + u * rowbytes, rowbytes), (unsigned)(int)lp, v[u]);
            lp += sig;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) step(v[u], lpu[u]);
        rowp += U * rowbytes;
    }
    for (; m < hi; ++m) {
        double v[2];
        row_load<double, 2>(row_ref(rowp, rowbytes), (unsigned)(int)lp, v);
        step(v, lp);
        lp += sig;
        rowp += rowbytes;
    }
    return acc;
}

// Stores ray (row a, bin k): v = (R x)_{a,k}, or the residual r = R x - b when
// b != nullptr, with the float64 sum of r^2 over the workgroup in
// partials[pidx].  The value goes, rounded to float32, to out[a*out_pitch + k];
// the padded sinograms that feed R^T get it times the angle's wmax (see
// bp_class), rounded to float32 in outp[a*pitchB + PAD + k] and unrounded in
// the float64 outpd (each nullable).  With dq (and no b), the workgroup's sum
// of v dq[a*nB + k] goes to partials[pidx] instead; wout (nullable) receives v
// unrounded at a*nB + k.
__device__ __forceinline__ void project_store(const GeomDev& G, int a, double wmax, int k,
                                              bool valid, double acc,
                                              const float* __restrict__ b, float* __restrict__ out,
                                              int out_pitch, float* __restrict__ outp,
                                              double* __restrict__ outpd,
                                              double* __restrict__ partials, int pidx,
                                              const double* __restrict__ dq,
                                              double* __restrict__ wout) {
    __shared__ double red[4];
    double r2 = 0.0;
    if (valid) {
        double v;
        const size_t i = (size_t)a * G.nB + k;
        if (b) {
            v = fma(acc, G.pixel, -(double)b[i]);
            r2 = v * v;
        } else {
            v = acc * G.pixel;
            if (dq) r2 = v * dq[i];
        }
        if (out) out[(size_t)a * out_pitch + k] = (float)v;
        if (wout) wout[i] = v;
        const double vs = v * wmax;
        if (outp) outp[(size_t)a * G.pitchB + PAD + k] = (float)vs;
        if (outpd) outpd[(size_t)a * G.pitchB + PAD + k] = vs;
    }
    if (b || dq) {
        const double tot = block_sum(r2, red);
        if (threadIdx.x == 0) partials[pidx] = tot;
    }
}

// Rays of ray workgroup wg: its wave w runs entry 4 wg + w of the wave table
// (lane l one ray of it, see WaveDev).  With seg == nullptr each ray is summed
// whole and stored by project_store (partials index wg).  Otherwise
// (G.parts > 1) only part `part` of each ray is summed and its float64 value
// goes to seg[(part*nA + ai)*nB + k] (ai: class-sorted table index); the
// combine step adds the parts in order.  Splitting the rays keeps the image
// rows that the resident waves read close together and makes the work items
// shorter and more even.
__device__ __forceinline__ void project_body(const GeomDev& G, const AngleDev* __restrict__ ang,
                                             const WaveDev* __restrict__ waves,
                                             const double* __restrict__ xp,
                                             const double* __restrict__ xTp,
                                             const float* __restrict__ b, float* __restrict__ out,
                                             int out_pitch, float* __restrict__ outp,
                                             double* __restrict__ outpd,
                                             double* __restrict__ partials,
                                             double* __restrict__ seg, int wg, int part,
                                             const double* __restrict__ dq = nullptr,
                                             double* __restrict__ wout = nullptr) {
    const int wi = 4 * wg + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool wvalid = wi < G.nwaves;
    const WaveDev W = waves[wvalid ? wi : 0];
    int ai, k;
    bool valid = wvalid && wave_ray(W, threadIdx.x & 63, G.nB, ai, k);
    if (!valid) {   // no ray: a valid angle of the wave's class, summing nothing
        ai = W.a0;
        k = 0;
    }
    const AngleDev A = ang[ai];
    const int flags = ang[W.a0].flags;   // the wave's class (wave-uniform)
    const double sk = bin_pos((double)k, G);
    const int np = seg ? G.parts : 1;
    double acc;
    if (!(flags & ANG_HORIZ)) {
        acc = (flags & ANG_AXIS) ? ray_sum_axis<false>(G, A, sk, xp + PAD, valid, part, np)
                                 : ray_split<false>(G, A, sk, xp + PAD, valid, part, np);
    } else {
        acc = (flags & ANG_AXIS) ? ray_sum_axis<true>(G, A, sk, xTp + PAD, valid, part, np)
                                 : ray_split<true>(G, A, sk, xTp + PAD, valid, part, np);
    }
    acc *= A.wmax;   // the ray sums u-weighted values (see chord_u)
    if (seg) {
        if (valid) seg[((size_t)part * G.nA + ai) * G.nB + k] = acc;
        return;
    }
    project_store(G, A.row, A.wmax, k, valid, acc, b, out, out_pitch, outp, outpd, partials, wg, dq,
                  wout);
}

// Sum of the parts of the rays of combine block (bx, by): angle bx of the
// class-sorted table, 256-bin chunk by; then the store (partials index
// by * gx + bx).
__device__ __forceinline__ void project_comb_body(const GeomDev& G, const AngleDev* __restrict__ ang,
                                                  const double* __restrict__ seg,
                                                  const float* __restrict__ b,
                                                  float* __restrict__ out, int out_pitch,
                                                  float* __restrict__ outp,
                                                  double* __restrict__ outpd,
                                                  double* __restrict__ partials, int bx, int by,
                                                  int gx, const double* __restrict__ dq = nullptr,
                                                  double* __restrict__ wout = nullptr) {
    const int a = ang[bx].row;
    const double wmax = ang[bx].wmax;
    const int k = by * 256 + threadIdx.x;
    const bool valid = k < G.nB;
    double acc = 0.0;
    if (valid) {
        const double* v = seg + (size_t)bx * G.nB + k;
        const size_t stride = (size_t)G.nA * G.nB;
        for (int j = 0; j < G.parts; ++j) acc += v[j * stride];
    }
    project_store(G, a, wmax, k, valid, acc, b, out, out_pitch, outp, outpd, partials,
                  by * gx + bx, dq, wout);
}

__global__ __launch_bounds__(256, 8) void k_project(GeomDev G, const AngleDev* __restrict__ ang,
                                                 const WaveDev* __restrict__ waves,
                                                 const double* __restrict__ xp,
                                                 const double* __restrict__ xTp,
                                                 const float* __restrict__ b,
                                                 float* __restrict__ out, int out_pitch,
                                                 float* __restrict__ outp,
                                                 double* __restrict__ outpd,
                                                 double* __restrict__ partials,
                                                 const int* __restrict__ ord,
                                                 const int* __restrict__ halt,
                                                 const double* __restrict__ dq,
                                                 double* __restrict__ wout) {
    if (halt && *halt) return;
    project_body(G, ang, waves, xp, xTp, b, out, out_pitch, outp, outpd, partials, nullptr,
                 ord[blockIdx.x], 0, dq, wout);
}

// grid (ray workgroups, parts): blockIdx.y is the part, so the parts run in order.
__global__ __launch_bounds__(256, 8) void k_project_part(GeomDev G, const AngleDev* __restrict__ ang,
                                                      const WaveDev* __restrict__ waves,
                                                      const double* __restrict__ xp,
                                                      const double* __restrict__ xTp,
                                                      double* __restrict__ seg,
                                                      const int* __restrict__ ord,
                                                      const int* __restrict__ halt) {
    if (halt && *halt) return;
    project_body(G, ang, waves, xp, xTp, nullptr, nullptr, 0, nullptr, nullptr, nullptr, seg,
                 ord[blockIdx.x], blockIdx.y);
}

__global__ __launch_bounds__(256) void k_project_comb(GeomDev G, const AngleDev* __restrict__ ang,
                                                      const double* __restrict__ seg,
                                                      const float* __restrict__ b,
                                                      float* __restrict__ out, int out_pitch,
                                                      float* __restrict__ outp,
                                                      double* __restrict__ outpd,
                                                      double* __restrict__ partials,
                                                      const int* __restrict__ halt,
                                                      const double* __restrict__ dq,
                                                      double* __restrict__ wout) {
    if (halt && *halt) return;
    project_comb_body(G, ang, seg, b, out, out_pitch, outp, outpd, partials, blockIdx.x,
                      blockIdx.y, gridDim.x, dq, wout);
}

// residual: rpd = R xh - b (float64) with f partials; else w = R z (float64)
// with the partials of w^T q, both into pf.  Item lin = part * G.nwg + i runs
// ray workgroup S.pord[i].
__global__ __launch_bounds__(256, 8) void kb_project(const SliceDev* __restrict__ sl, ItemTable t,
                                                  int residual) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const GeomDev G = S.G;
        if (G.parts > 1) {
            project_body(G, cmem(S.ang), cmem(S.pwave), gmem(S.xp), gmem(S.xTp), nullptr, nullptr,
                         0, nullptr, nullptr, nullptr, gmem(S.seg), cmem(S.pord)[lin % G.nwg],
                         lin / G.nwg);
        } else if (residual) {
            project_body(G, cmem(S.ang), cmem(S.pwave), gmem(S.xp), gmem(S.xTp), gmem(S.b), nullptr,
                         0, nullptr, gmem(S.rpd), gmem(S.pf), nullptr, cmem(S.pord)[lin], 0);
        } else {
            project_body(G, cmem(S.ang), cmem(S.pwave), gmem(S.xp), gmem(S.xTp), nullptr, nullptr,
                         0, nullptr, nullptr, gmem(S.pf), nullptr, cmem(S.pord)[lin], 0, gmem(S.q),
                         gmem(S.w));
        }
    });
}

// The combine step of the slices with G.parts > 1; virtual block by * nA + bx.
__global__ __launch_bounds__(256) void kb_project_comb(const SliceDev* __restrict__ sl, ItemTable t,
                                                       int residual) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const GeomDev G = S.G;
        const int gx = G.nA;
        if (residual)
            project_comb_body(G, cmem(S.ang), gmem(S.seg), gmem(S.b), nullptr, 0, nullptr,
                              gmem(S.rpd), gmem(S.pf), lin % gx, lin / gx, gx);
        else
            project_comb_body(G, cmem(S.ang), gmem(S.seg), nullptr, nullptr, 0, nullptr, nullptr,
                              gmem(S.pf), lin % gx, lin / gx, gx, gmem(S.q), gmem(S.w));
    });
}

void launch_project_b(hipStream_t st, const SliceDev* sl, ItemTable t, ItemTable tc,
                      bool residual) {
    hipLaunchKernelGGL(kb_project, dim3(t.grid), dim3(256), 0, st, sl, t, residual ? 1 : 0);
    if (tc.n > 0)
        hipLaunchKernelGGL(kb_project_comb, dim3(tc.grid), dim3(256), 0, st, sl, tc,
                           residual ? 1 : 0);
}

void launch_project(hipStream_t st, const GeomDev& G, const AngleDev* ang, const WaveDev* waves,
                    const double* xp, const double* xTp, const float* b, float* out, int out_pitch,
                    float* outp, double* outpd, double* partials, double* seg, const int* ord,
                    const int* halt, const double* dq, double* wout) {
    if (G.parts > 1) {
        hipLaunchKernelGGL(k_project_part, dim3(G.nwg, G.parts), dim3(256), 0, st, G, ang, waves, xp,
                           xTp, seg, ord, halt);
        hipLaunchKernelGGL(k_project_comb, dim3(G.nA, (G.nB + 255) / 256), dim3(256), 0, st, G,
                           ang, (const double*)seg, b, out, out_pitch, outp, outpd, partials, halt,
                           dq, wout);
        return;
    }
    hipLaunchKernelGGL(k_project, dim3(G.nwg), dim3(256), 0, st, G, ang, waves, xp, xTp, b, out,
                       out_pitch, outp, outpd, partials, ord, halt, dq, wout);
}

// Padded copy of a caller's sinogram for R^T, each row times its angle's wmax
// (the scaling bp_class expects), pads written as zeros; one workgroup per
// entry of the angle table.
__global__ __launch_bounds__(256) void k_pad_sino(GeomDev G, const AngleDev* __restrict__ ang,
                                                  const float* __restrict__ y,
                                                  float* __restrict__ yp) {
    const int a = ang[blockIdx.x].row;
    const double wmax = ang[blockIdx.x].wmax;
    float* row = yp + (size_t)a * G.pitchB;
    for (int k = threadIdx.x; k < G.pitchB; k += 256) {
        const int kk = k - PAD;
        row[k] = kk >= 0 && kk < G.nB ? (float)((double)y[(size_t)a * G.nB + kk] * wmax) : 0.0f;
    }
}

void launch_pad_sino(hipStream_t st, const GeomDev& G, const AngleDev* ang, const float* y,
                     float* yp) {
    hipLaunchKernelGGL(k_pad_sino, dim3(G.nA), dim3(256), 0, st, G, ang, y, yp);
}

// ---- backward gather ----------------------------------------------------------
// Sum over the angles [beg, end) of one class for pixel row yi and the PX
// pixels xj[u] of this lane.  The angle and its sinogram row are wave-uniform
// (scalar loads); lanes differ only in the pixel.  The padded sinogram rows
// arrive multiplied by their angle's wmax (project_store, k_pad_sino), so each
// candidate adds u * y' with the u of chord_u: the same weights as the
// projector's wmax * u.
//
// Candidate window: the NB bins from padded index trunc(kf), kf = t / ds + kb
// with t = xj c + yi s (A.kb carries the - s0 / ds, the half-width hb of the
// nonzero band plus a margin, and the + 1 + PAD of the padded index; see
// bp_kf).  For oblique angles kf = fma(xj, c / ds, yi s / ds + kb), the
// second term shared by the lane's pixels, and the first candidate's offset
// s_k - t is dc - ds fract(kf) with dc = ds (1 - hb) (the same value as
// s_k - t up to the rounding of kf, ~1e-13 pixel); the next ones follow by
// + ds.  For axis-parallel angles the offset must be
// exact -- a ray on a pixel edge takes half the pixel -- so s_k is formed from
// the bin index as in bin_pos and t is exact.  A window index below the row
// or past it reads 0 (pads and out-of-row reads), so such candidates add 0.
template <bool AXIS, int NB, class TY, int PX>
__device__ __forceinline__ void bp_class(const GeomDev& G, const AngleDev* __restrict__ ang,
                                         int beg, int end, const TY* __restrict__ yp,
                                         const double* xj, double yi, double* acc) {
    const int rowbytes = G.pitchB * (int)sizeof(TY);
    // 1/ds held in a vector register, so the index FMA's one scalar operand
    // can be the angle's kb (an FMA reads at most one scalar register)
    double ids = G.inv_ds;
    asm volatile("" : "+v"(ids));
    double ds = G.ds;   // likewise for the offset FMA, whose addend is the angle's dc
    asm volatile("" : "+v"(ds));
#pragma unroll 2
    for (int a = beg; a < end; ++a) {
        const AngleDev A = ang[a];
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(yp + (size_t)A.row * G.pitchB, rowbytes);
        const double ys = AXIS ? yi * A.s : 0.0;
        const double kc = AXIS ? 0.0 : bp_kc(yi, A);
        TY v[PX][NB];
        double d0[PX], tt[PX];
        int oo[PX];
#pragma unroll
        for (int u = 0; u < PX; ++u) {
            double kf;
            if (AXIS) {
                tt[u] = fma(xj[u], A.c, ys);
                kf = bp_kf(tt[u], ids, A.kb);
            } else {
                kf = bp_kf_oblique(xj[u], kc, A);
            }
            const int o = (int)kf;
            row_load<TY, NB>(rs, (unsigned)o, v[u]);
            if (AXIS) oo[u] = o;
            else d0[u] = fma(__builtin_amdgcn_fract(kf), -ds, A.dc);
        }
#pragma unroll
        for (int u = 0; u < PX; ++u) {
            double d = AXIS ? 0.0 : d0[u];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                if (AXIS) d = bin_pos((double)(oo[u] - PAD + q), G) - tt[u];
                acc[u] = fma(chord_u<AXIS>(d, A.einv, A.inv), (double)v[u][q], acc[u]);
                if (!AXIS) d += ds;
            }
        }
    }
}

__device__ __forceinline__ void split_range(int beg, int end, int w, int& b, int& e) {
    const int len = end - beg;
    b = beg + (len * w) / BP_SPLIT;
    e = beg + (len * (w + 1)) / BP_SPLIT;
}

// out[i][j] = (R^T y)_{ij} from the padded sinogram yp; with dotv != nullptr
// also the float64 partial sum of out * dotv per 8 x 16 sub-tile.  A
// workgroup owns an 8 x 8PX pixel tile (PX pixels, 8 columns apart, per lane);
// its wave w sums the w-th quarter of every angle class, and the four partial
// sums are added in wave order through LDS.
template <int NB, class TY, int PX>
__device__ __forceinline__ void backproject_body(const GeomDev& G, const AngleDev* __restrict__ ang,
                                                 const TY* __restrict__ yp,
                                                 float* __restrict__ out,
                                                 const double* __restrict__ dotv,
                                                 double* __restrict__ partials, int bx, int by) {
    constexpr int NS = PX / 2;   // 8 x 16 sub-tiles per tile
    __shared__ double part[BP_SPLIT][PX][64];
    __shared__ double red[4 * NS];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = by * BP_TILE + (lane >> 3);
    const int j0 = bx * 8 * PX + (lane & 7);
    const double yi = G.yoff - (double)i;
    double acc[PX], xj[PX];
#pragma unroll
    for (int u = 0; u < PX; ++u) {
        acc[u] = 0.0;
        xj[u] = (double)(j0 + 8 * u) - G.xoff;
    }
    int b, e;
    split_range(G.cls[0], G.cls[2], w, b, e);   // oblique angles of both orientations
    bp_class<false, NB, TY, PX>(G, ang, b, e, yp, xj, yi, acc);
    split_range(G.cls[2], G.cls[4], w, b, e);   // axis-parallel angles
    bp_class<true, NB, TY, PX>(G, ang, b, e, yp, xj, yi, acc);
#pragma unroll
    for (int u = 0; u < PX; ++u) part[w][u][lane] = acc[u];
    __syncthreads();
    double v[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) v[q] = 0.0;
    if (w == 0) {
#pragma unroll
        for (int u = 0; u < PX; ++u) {
            const int j = j0 + 8 * u;
            const double tot =
                ((part[0][u][lane] + part[1][u][lane]) + part[2][u][lane]) + part[3][u][lane];
            const float val = (float)(tot * G.pixel);
            if (i < G.rows && j < G.cols) {
                out[(size_t)i * G.cols + j] = val;
                if (dotv) v[u / 2] += (double)val * dotv[(size_t)i * G.cols + j];
            }
        }
    }
    if (dotv) {
        // partial of 8 x 16 sub-tile (by, NS bx + q) at by * gx16 + NS bx + q
        block_sum_n<NS>(v, red);
        const int gx16 = (G.cols + BP_TW - 1) / BP_TW;
        if (threadIdx.x == 0) {
#pragma unroll
            for (int q = 0; q < NS; ++q)
                if (NS * bx + q < gx16) partials[by * gx16 + NS * bx + q] = v[q];
        }
    }
}

template <int NB, class TY, int PX>
__global__ __launch_bounds__(256) void k_backproject(GeomDev G, const AngleDev* __restrict__ ang,
                                                     const TY* __restrict__ yp,
                                                     float* __restrict__ out,
                                                     const double* __restrict__ dotv,
                                                     double* __restrict__ partials,
                                                     ScalarRide ride,
                                                     const int* __restrict__ halt) {
    if (halt && *halt) return;
    int bx, by;
    bp_tile_of(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x, gridDim.y, bx, by);
    backproject_body<NB, TY, PX>(G, ang, yp, out, dotv, partials, bx, by);
    if (ride.sc && blockIdx.x == 0 && blockIdx.y == 0) {
        if (ride.ps) scalar_body(OP_SNORM, ride.sc, ride.tr, ride.ps, ride.ns, nullptr, 0);
        if (ride.pf) scalar_body(OP_F, ride.sc, ride.tr, ride.pf, ride.nf, nullptr, 0);
    }
}

// g = R^T rpd from the float64 residual.  NB is the largest candidate count of
// the batch (extra candidates weigh exactly 0).
template <int NB, int PX>
__global__ __launch_bounds__(256) void kb_backproject(const SliceDev* __restrict__ sl, ItemTable t) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const GeomDev G = S.G;
        int bx, by;
        bp_tile_of(lin, (G.cols + 8 * PX - 1) / (8 * PX), (G.rows + BP_TILE - 1) / BP_TILE, bx, by);
        backproject_body<NB, double, PX>(G, cmem(S.ang), gmem(S.rpd), gmem(S.g), nullptr, nullptr, bx, by);
    });
}

template <int PX>
void launch_bp_b_px(hipStream_t st, const SliceDev* sl, ItemTable t, int nbmax) {
    switch (nbmax) {
    case 1: hipLaunchKernelGGL((kb_backproject<1, PX>), dim3(t.grid), dim3(256), 0, st, sl, t); break;
    case 2: hipLaunchKernelGGL((kb_backproject<2, PX>), dim3(t.grid), dim3(256), 0, st, sl, t); break;
    case 3: hipLaunchKernelGGL((kb_backproject<3, PX>), dim3(t.grid), dim3(256), 0, st, sl, t); break;
    default: hipLaunchKernelGGL((kb_backproject<4, PX>), dim3(t.grid), dim3(256), 0, st, sl, t); break;
    }
}

void launch_backproject_b(hipStream_t st, const SliceDev* sl, ItemTable t, int nbmax, int px) {
    if (px == 4) launch_bp_b_px<4>(st, sl, t, nbmax);
    else launch_bp_b_px<2>(st, sl, t, nbmax);
}

template <class TY, int PX>
void launch_bp_px(hipStream_t st, const GeomDev& G, const AngleDev* ang, const TY* yp, float* out,
                  const double* dotv, double* partials, const int* halt, const ScalarRide& ride) {
    dim3 grid((G.cols + 8 * PX - 1) / (8 * PX), (G.rows + BP_TILE - 1) / BP_TILE);
    switch (G.nbmax) {
    case 1: hipLaunchKernelGGL((k_backproject<1, TY, PX>), grid, dim3(256), 0, st, G, ang, yp, out, dotv, partials, ride, halt); break;
    case 2: hipLaunchKernelGGL((k_backproject<2, TY, PX>), grid, dim3(256), 0, st, G, ang, yp, out, dotv, partials, ride, halt); break;
    case 3: hipLaunchKernelGGL((k_backproject<3, TY, PX>), grid, dim3(256), 0, st, G, ang, yp, out, dotv, partials, ride, halt); break;
    default: hipLaunchKernelGGL((k_backproject<4, TY, PX>), grid, dim3(256), 0, st, G, ang, yp, out, dotv, partials, ride, halt); break;
    }
}

void launch_backproject(hipStream_t st, const GeomDev& G, const AngleDev* ang, const float* yp,
                        float* out, const double* dotv, double* partials, const int* halt,
                        const ScalarRide& ride) {
    if (G.bp_px == 4) launch_bp_px<float, 4>(st, G, ang, yp, out, dotv, partials, halt, ride);
    else launch_bp_px<float, 2>(st, G, ang, yp, out, dotv, partials, halt, ride);
}

void launch_backproject(hipStream_t st, const GeomDev& G, const AngleDev* ang, const double* yp,
                        float* out, const double* dotv, double* partials, const int* halt,
                        const ScalarRide& ride) {
    if (G.bp_px == 4) launch_bp_px<double, 4>(st, G, ang, yp, out, dotv, partials, halt, ride);
    else launch_bp_px<double, 2>(st, G, ang, yp, out, dotv, partials, halt, ride);
}

}  // namespace sp
