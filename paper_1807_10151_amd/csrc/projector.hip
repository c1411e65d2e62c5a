// Matrix-free parallel-beam projector R (ray-driven gather) and its exact
// transpose R^T (pixel-driven gather, no atomics).
//
// R[(a,k),(i,j)] is the length of ray (a,k) inside pixel (i,j) (the projection
// matrix of Section 2, rays as in Section 4.1).  R^T evaluates each weight as
// the chord length of a line through a square (projection t of the pixel
// centre, offset d = s_k - t, the clamped trapezoid u of chord_u, times the
// angle's wmax).  R walks each ray band by band and splits a band's path
// length at the pixel boundary it crosses (ray_split): the same lengths in
// exact arithmetic, equal to rounding in float64, so R^T is the adjoint of R
// to float64 rounding (axis-parallel angles use the trapezoid in both, bit for
// bit).  Data are float32; coordinates, weights and sums are float64 (FP64
// FMA issues at the non-packed FP32 rate on CDNA4, and float32 angles alone
// would move a ray by ~1e-5 pixel at radius 256).
//
// Canonical projection of pixel centre (xj, yi) on the normal of angle a:
//   |c| >= |s| ("vertical" angles):   t = fma(xj, c, yi * s)
//   |s| >  |c| ("horizontal" angles): t = fma(yi, s, xj * c)
// The product outside the fma is the one the axis-parallel forward walk
// shares between the candidates of one step.
//
// Forward walk.  For a vertical angle a ray crosses every image row; within
// row i it meets at most two pixels, as its crossing point moves by `slope`
// (|slope| <= 1) columns per row.  A lane owns one ray; the 64 lanes of a wave hold
// consecutive rays of one angle and walk the union of their row ranges
// together, so each step gathers consecutive addresses of one row.  A
// workgroup's four waves take four consecutive angles and the same 64-bin
// chunk, and the workgroups run in a host-computed order (project_order).  Candidate
// columns outside the image are clamped into a zero pad and contribute 0.
// Horizontal angles walk columns of a zero-padded transposed copy.
//
// Backward gather.  A lane owns PX (2 or 4) pixels of one row, 8 columns
// apart, and loops over the angles, which are sorted into four classes
// (vertical/horizontal x oblique/axis-parallel) so the inner loop has no
// branch; at each angle a
// pixel's nonzero bins are the NB bins after floor(kf - hb), read from a
// zero-padded sinogram (float32, or float64 for the solvers' residual) whose
// rows carry the angle's wmax.
#include "sp_internal.h"
#include "sp_reduce.h"
#include "sp_scalar.h"

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
        prep_body(G, batch_vec(S, which), gmem(S.xp), gmem(S.xTp), lin % gx, lin / gx);
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

// base + o for a wave-uniform base and a 32-bit element index: the byte offset
// is formed in 32 bits so the load can use the scalar-base addressing form.
template <class T>
__device__ __forceinline__ const T* at(const T* base, unsigned o) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + o * (unsigned)sizeof(T));
}

// One ray's sum, or part `part` of nparts of it.  HORIZ = walk columns of the
// transposed copy.  img points at element PAD of row 0 of the padded copy.  A
// part covers the steps [lo + len*part/nparts, lo + len*(part+1)/nparts) of
// the wave's common step range [lo, lo + len).
template <bool HORIZ, bool AXIS, int NC>
__device__ __forceinline__ double ray_sum(const GeomDev& G, const AngleDev& A, double sk,
                                          const double* __restrict__ img, bool valid, int part,
                                          int nparts) {
    const int nmaj = HORIZ ? G.cols : G.rows;
    const int nmin = HORIZ ? G.rows : G.cols;
    const int pitch = HORIZ ? G.pitchXT : G.pitchX;
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
    if (nparts > 1 && hi > lo) {
        const int len = hi - lo;
        const int l0 = lo + len * part / nparts;
        hi = lo + len * (part + 1) / nparts;
        lo = l0;
    }
    double acc = 0.0;
    if (lo >= hi) return acc;
    // Candidate q of step m is minor index floor(nf_m) + 1 + q.  nf carries the
    // + 1 + PAD of the padded index, so the first candidate's padded index is
    // trunc(nf) where nf >= 0.  A negative value (read as unsigned) or one past
    // the row is clamped to omax: every read of that step then hits zero pads
    // and, as all true candidates lie outside the image, the step contributes
    // exactly 0.  The minor coordinate of candidate q is taken from the index
    // actually read -- (o + q - PAD) - xoff for columns, yoff - (o + q - PAD)
    // for rows, exact small half-integers -- which is the candidate's own
    // coordinate whenever the read is not clamped.
    const double* row = img - PAD;
    const double c2 = HORIZ ? G.yoff + (double)PAD : -(double)PAD - G.xoff;
    const double fM = HORIZ ? A.c : A.s;   // factor of the shared (major) product
    const double dM = HORIZ ? 1.0 : -1.0;  // major coordinate step
    double cM = HORIZ ? (double)lo - G.xoff : G.yoff - (double)lo;
    double nf = fma((double)lo, A.slope, start + (double)(1 + PAD));
    const unsigned omax = (unsigned)(nmin + 2 * PAD - NC);
    const double* rp = row + (size_t)lo * pitch;
    // one major step: gather is issued by the caller, weights and sum here
    auto step = [&](const double* v, unsigned o, double cMv) {
        const double P = cMv * fM;
        const double cm0 = HORIZ ? c2 - (double)o : (double)o + c2;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const double cm = HORIZ ? cm0 - (double)q : cm0 + (double)q;
            const double d = sk - fma(cm, fm, P);
            acc = fma(chord_u<AXIS>(d, A.einv, A.inv), v[q], acc);
        }
    };
    int m = lo;
    // two steps per iteration: both gathers are in flight before either step's math
    for (; m + 1 < hi; m += 2) {
        const unsigned o0 = min((unsigned)(int)nf, omax);
        const unsigned o1 = min((unsigned)(int)(nf + A.slope), omax);
        const double* p0 = at(rp, o0);
        const double* p1 = at(rp + pitch, o1);
        double v0[NC], v1[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) v0[q] = p0[q];
#pragma unroll
        for (int q = 0; q < NC; ++q) v1[q] = p1[q];
        step(v0, o0, cM);
        step(v1, o1, cM + dM);
        nf += 2.0 * A.slope;
        cM += 2.0 * dM;
        rp += 2 * pitch;
    }
    if (m < hi) {
        const unsigned o0 = min((unsigned)(int)nf, omax);
        const double* p0 = at(rp, o0);
        double v0[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) v0[q] = p0[q];
        step(v0, o0, cM);
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
// caller) in the first is f = clamp((floor(lp) + 1 - lp) / |slope|, 0, 1) and
// the rest falls in the second: the exact chord lengths of the pixel model,
// the same values chord_u * wmax gives up to rounding, with fewer operations
// per step than evaluating the trapezoid per candidate.  Indices and the
// step range are handled as in ray_sum: a truncated index below the row or
// past it is clamped into the zero pads, where the pixels contribute 0.
template <bool HORIZ>
__device__ __forceinline__ double ray_split(const GeomDev& G, const AngleDev& A, double sk,
                                            const double* __restrict__ img, bool valid, int part,
                                            int nparts) {
    const int nmaj = HORIZ ? G.cols : G.rows;
    const int nmin = HORIZ ? G.rows : G.cols;
    const int pitch = HORIZ ? G.pitchXT : G.pitchX;
    const double start = (HORIZ ? G.yoff - (sk + G.xoff * A.c) / A.s
                                : (sk - G.yoff * A.s) / A.c + G.xoff) - (double)A.hw;
    int lo, hi;
    step_range(start, A.slope, -(double)(A.nc + 1), (double)(nmin + 1), nmaj, lo, hi);
    if (!valid) {
        lo = nmaj;
        hi = 0;
    }
    lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    if (nparts > 1 && hi > lo) {
        const int len = hi - lo;
        const int l0 = lo + len * part / nparts;
        hi = lo + len * (part + 1) / nparts;
        lo = l0;
    }
    double acc = 0.0;
    if (lo >= hi) return acc;
    const double sig = A.slope;
    const double isg = 1.0 / fabs(sig);
    // minor coordinate where the ray enters band 0 on its lower side, padded
    const double b0 = (HORIZ ? G.yoff + 0.5 - (sk + (G.xoff + 0.5) * A.c) / A.s
                             : (sk - (G.yoff + 0.5) * A.s) / A.c + G.xoff + 0.5) +
                      fmin(sig, 0.0) + (double)PAD;
    const unsigned omax = (unsigned)(nmin + 2 * PAD - 2);
    const double* rp = img - PAD + (size_t)lo * pitch;
    auto step = [&](const double* v, int fl, double lpv) {
        const double f = fmin(fmax(fma(lpv - (double)fl, -isg, isg), 0.0), 1.0);
        acc += fma(f, v[0] - v[1], v[1]);
    };
    double dm = (double)lo;
    int m = lo;
    for (; m + 1 < hi; m += 2) {
        const double lp0 = fma(dm, sig, b0), lp1 = lp0 + sig;
        const int f0 = (int)lp0, f1 = (int)lp1;
        const double* p0 = at(rp, min((unsigned)f0, omax));
        const double* p1 = at(rp + pitch, min((unsigned)f1, omax));
        const double v0[2] = {p0[0], p0[1]};
        const double v1[2] = {p1[0], p1[1]};
        step(v0, f0, lp0);
        step(v1, f1, lp1);
        dm += 2.0;
        rp += 2 * pitch;
    }
    if (m < hi) {
        const double lp0 = fma(dm, sig, b0);
        const int f0 = (int)lp0;
        const double* p0 = at(rp, min((unsigned)f0, omax));
        const double v0[2] = {p0[0], p0[1]};
        step(v0, f0, lp0);
    }
    return acc;
}

// Axis-parallel angles keep the per-candidate trapezoid (with its half weight
// for a ray on a pixel edge); oblique ones split each band.
template <bool HORIZ, bool AXIS>
__device__ __forceinline__ double ray_sum_nc(const GeomDev& G, const AngleDev& A, double sk,
                                             const double* __restrict__ img, bool valid,
                                             int part, int nparts) {
    if (AXIS) return ray_sum<HORIZ, true, 2>(G, A, sk, img, valid, part, nparts);
    return ray_split<HORIZ>(G, A, sk, img, valid, part, nparts);
}

// Stores ray (row a, bin k): (R x)_{a,k}, or the residual r = R x - b when
// b != nullptr, with the float64 sum of r^2 over the workgroup in
// partials[pidx].  The value goes, rounded to float32, to out[a*out_pitch + k];
// the padded sinograms that feed R^T get it times the angle's wmax (see
// bp_class), rounded to float32 in outp[a*pitchB + PAD + k] and unrounded in
// the float64 outpd (each nullable).
__device__ __forceinline__ void project_store(const GeomDev& G, int a, double wmax, int k,
                                              bool valid, double acc,
                                              const float* __restrict__ b, float* __restrict__ out,
                                              int out_pitch, float* __restrict__ outp,
                                              double* __restrict__ outpd,
                                              double* __restrict__ partials, int pidx) {
    __shared__ double red[4];
    double r2 = 0.0;
    if (valid) {
        double v;
        if (b) {
            v = fma(acc, G.pixel, -(double)b[(size_t)a * G.nB + k]);
            r2 = v * v;
        } else {
            v = acc * G.pixel;
        }
        if (out) out[(size_t)a * out_pitch + k] = (float)v;
        const double vs = v * wmax;
        if (outp) outp[(size_t)a * G.pitchB + PAD + k] = (float)vs;
        if (outpd) outpd[(size_t)a * G.pitchB + PAD + k] = vs;
    }
    if (b) {
        const double tot = block_sum(r2, red);
        if (threadIdx.x == 0) partials[pidx] = tot;
    }
}

// Ray workgroups.  Wave w of virtual block blk = q * nag + ag takes angle
// 4 ag + w of the class-sorted table and the 64 bins of chunk q, so the four
// waves of a workgroup hold rays of nearly the same length.  Workgroup i of a
// launch runs virtual block ord[i] (project_order: longest first, snaked over
// the compute units).

// Rays of virtual block blk.  With seg == nullptr each ray is
// summed whole and stored by project_store (partials index blk).  Otherwise
// (G.parts > 1) only part `part` of each ray is summed and its float64 value
// goes to seg[(part*nA + ai)*nB + k]; the combine step adds the parts in
// order.  Splitting the rays keeps the image rows that the resident waves
// read close together and makes the work items shorter and more even.
__device__ __forceinline__ void project_body(const GeomDev& G, const AngleDev* __restrict__ ang,
                                             const double* __restrict__ xp,
                                             const double* __restrict__ xTp,
                                             const float* __restrict__ b, float* __restrict__ out,
                                             int out_pitch, float* __restrict__ outp,
                                             double* __restrict__ outpd,
                                             double* __restrict__ partials,
                                             double* __restrict__ seg, int blk, int part) {
    const int nag = (G.nA + 3) >> 2;
    const int ag = blk % nag, q = blk / nag;
    const int ai = 4 * ag + (threadIdx.x >> 6);   // one angle per wave
    const int k = q * 64 + (threadIdx.x & 63);
    const bool valid = ai < G.nA && k < G.nB;
    const AngleDev A = ang[ai < G.nA ? ai : G.nA - 1];
    const double sk = bin_pos((double)k, G);
    const bool horiz = A.flags & ANG_HORIZ, axis = A.flags & ANG_AXIS;
    const int np = seg ? G.parts : 1;
    double acc;
    if (!horiz) {
        acc = axis ? ray_sum_nc<false, true>(G, A, sk, xp + PAD, valid, part, np)
                   : ray_sum_nc<false, false>(G, A, sk, xp + PAD, valid, part, np);
    } else {
        acc = axis ? ray_sum_nc<true, true>(G, A, sk, xTp + PAD, valid, part, np)
                   : ray_sum_nc<true, false>(G, A, sk, xTp + PAD, valid, part, np);
    }
    acc *= A.wmax;   // the ray sums u-weighted values (see chord_u)
    if (seg) {
        if (valid) seg[((size_t)part * G.nA + ai) * G.nB + k] = acc;
        return;
    }
    project_store(G, A.row, A.wmax, k, valid, acc, b, out, out_pitch, outp, outpd, partials, blk);
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
                                                  int gx) {
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
                  by * gx + bx);
}

__global__ __launch_bounds__(256) void k_project(GeomDev G, const AngleDev* __restrict__ ang,
                                                 const double* __restrict__ xp,
                                                 const double* __restrict__ xTp,
                                                 const float* __restrict__ b,
                                                 float* __restrict__ out, int out_pitch,
                                                 float* __restrict__ outp,
                                                 double* __restrict__ outpd,
                                                 double* __restrict__ partials,
                                                 const int* __restrict__ ord,
                                                 const int* __restrict__ halt) {
    if (halt && *halt) return;
    project_body(G, ang, xp, xTp, b, out, out_pitch, outp, outpd, partials, nullptr,
                 ord[blockIdx.x], 0);
}

// grid (ray blocks, parts): blockIdx.y is the part, so the parts run in order.
__global__ __launch_bounds__(256) void k_project_part(GeomDev G, const AngleDev* __restrict__ ang,
                                                      const double* __restrict__ xp,
                                                      const double* __restrict__ xTp,
                                                      double* __restrict__ seg,
                                                      const int* __restrict__ ord,
                                                      const int* __restrict__ halt) {
    if (halt && *halt) return;
    project_body(G, ang, xp, xTp, nullptr, nullptr, 0, nullptr, nullptr, nullptr, seg,
                 ord[blockIdx.x], blockIdx.y);
}

__global__ __launch_bounds__(256) void k_project_comb(GeomDev G, const AngleDev* __restrict__ ang,
                                                      const double* __restrict__ seg,
                                                      const float* __restrict__ b,
                                                      float* __restrict__ out, int out_pitch,
                                                      float* __restrict__ outp,
                                                      double* __restrict__ outpd,
                                                      double* __restrict__ partials,
                                                      const int* __restrict__ halt) {
    if (halt && *halt) return;
    project_comb_body(G, ang, seg, b, out, out_pitch, outp, outpd, partials, blockIdx.x,
                      blockIdx.y, gridDim.x);
}

// residual: rpd = R xh - b (float64) with f partials; else rp = R p.  Item
// lin = part * project_ray_blocks(G) + i runs virtual block S.pord[i].
__global__ __launch_bounds__(256) void kb_project(const SliceDev* __restrict__ sl, ItemTable t,
                                                  int residual) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const GeomDev G = S.G;
        if (G.parts > 1) {
            const int nblk = project_ray_blocks(G);
            project_body(G, cmem(S.ang), gmem(S.xp), gmem(S.xTp), nullptr, nullptr, 0, nullptr,
                         nullptr, nullptr, gmem(S.seg), cmem(S.pord)[lin % nblk], lin / nblk);
        } else if (residual) {
            project_body(G, cmem(S.ang), gmem(S.xp), gmem(S.xTp), gmem(S.b), nullptr, 0, nullptr,
                         gmem(S.rpd), gmem(S.pf), nullptr, cmem(S.pord)[lin], 0);
        } else {
            project_body(G, cmem(S.ang), gmem(S.xp), gmem(S.xTp), nullptr, nullptr, 0, gmem(S.rp),
                         nullptr, nullptr, nullptr, cmem(S.pord)[lin], 0);
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
            project_comb_body(G, cmem(S.ang), gmem(S.seg), nullptr, nullptr, 0, gmem(S.rp), nullptr,
                              nullptr, lin % gx, lin / gx, gx);
    });
}

void launch_project_b(hipStream_t st, const SliceDev* sl, ItemTable t, ItemTable tc,
                      bool residual) {
    hipLaunchKernelGGL(kb_project, dim3(t.grid), dim3(256), 0, st, sl, t, residual ? 1 : 0);
    if (tc.n > 0)
        hipLaunchKernelGGL(kb_project_comb, dim3(tc.grid), dim3(256), 0, st, sl, tc,
                           residual ? 1 : 0);
}

int project_comb_blocks(const GeomDev& G) { return G.nA * ((G.nB + 255) / 256); }

int project_blocks(const GeomDev& G) {
    return G.parts > 1 ? project_comb_blocks(G) : project_ray_blocks(G);
}

int project_parts(int rows, int cols, int n_angles, int n_bins, int resident_waves) {
    // Large images: 8 parts keep the resident waves on a band of the float64
    // copies (measured: 2048^2 x 2048 angles 9.3 -> 5.8 ms).
    if ((long)rows * cols >= (1L << 21)) return 8;
    // Otherwise split only a grid that would leave wave slots empty.
    const long waves = (long)n_angles * ((n_bins + 63) / 64);
    if (waves >= resident_waves) return 1;
    const long p = (resident_waves + waves - 1) / waves;
    return p > 4 ? 4 : (int)p;
}

// Step count of one wave of R: the union of its lanes' step ranges, found as
// the kernel finds it (a lane's range is monotone in the bin index, so the
// two end lanes of the chunk bound it).
static long wave_steps(const GeomDev& G, const AngleDev& A, int k0, int k1) {
    const bool horiz = A.flags & ANG_HORIZ;
    const int nmaj = horiz ? G.cols : G.rows, nmin = horiz ? G.rows : G.cols;
    int lo = nmaj, hi = 0;
    for (int k : {k0, k1}) {
        const double sk = std::fma((double)k, G.ds, G.s0);
        const double start = (horiz ? G.yoff - (sk + G.xoff * A.c) / A.s
                                    : (sk - G.yoff * A.s) / A.c + G.xoff) - (double)A.hw;
        const double vlo = -(double)(A.nc + 1), vhi = (double)(nmin + 1);
        int l, h;
        if (A.slope == 0.0) {
            l = 0;
            h = nmaj;   // an axis-parallel chunk may straddle the image: count it whole
        } else {
            const double t0 = (vlo - start) / A.slope, t1 = (vhi - start) / A.slope;
            const double tmin = std::min(std::max(std::min(t0, t1) - 1.0, 0.0), (double)nmaj);
            const double tmax = std::min(std::max(std::max(t0, t1) + 2.0, 0.0), (double)nmaj);
            l = (int)std::floor(tmin);
            h = std::max(l, (int)std::ceil(tmax));
        }
        lo = std::min(lo, l);
        hi = std::max(hi, h);
    }
    return hi > lo ? (long)(hi - lo) : 0;   // the split walk costs the same per step
}

std::vector<int32_t> project_order(const GeomDev& G, const std::vector<AngleDev>& tab,
                                   int n_cu) {
    const int nag = (G.nA + 3) / 4, nq = (G.nB + 63) / 64, nblk = nag * nq;
    std::vector<long> cost((size_t)nblk, 0);
    for (int q = 0; q < nq; ++q) {
        const int k0 = q * 64, k1 = std::min(G.nB, k0 + 64) - 1;
        for (int ai = 0; ai < G.nA; ++ai)
            cost[(size_t)q * nag + ai / 4] += 16 + wave_steps(G, tab[(size_t)ai], k0, k1);
    }
    std::vector<int32_t> ord((size_t)nblk);
    for (int b = 0; b < nblk; ++b) ord[(size_t)b] = b;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int32_t x, int32_t y) { return cost[(size_t)x] > cost[(size_t)y]; });
    const int band = std::max(1, n_cu);
    for (int b0 = band, i = 1; b0 < nblk; b0 += band, ++i)
        if (i & 1) std::reverse(ord.begin() + b0, ord.begin() + std::min(nblk, b0 + band));
    return ord;
}

void launch_project(hipStream_t st, const GeomDev& G, const AngleDev* ang, const double* xp,
                    const double* xTp, const float* b, float* out, int out_pitch, float* outp,
                    double* outpd, double* partials, double* seg, const int* ord,
                    const int* halt) {
    const int nblk = project_ray_blocks(G);
    if (G.parts > 1) {
        hipLaunchKernelGGL(k_project_part, dim3(nblk, G.parts), dim3(256), 0, st, G, ang, xp, xTp,
                           seg, ord, halt);
        hipLaunchKernelGGL(k_project_comb, dim3(G.nA, (G.nB + 255) / 256), dim3(256), 0, st, G,
                           ang, (const double*)seg, b, out, out_pitch, outp, outpd, partials, halt);
        return;
    }
    hipLaunchKernelGGL(k_project, dim3(nblk), dim3(256), 0, st, G, ang, xp, xTp, b, out, out_pitch,
                       outp, outpd, partials, ord, halt);
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

// Sum over the angles [beg, end) of one class for pixel (xj, yi).  The angle
// and its sinogram row are wave-uniform (scalar loads); lanes differ only in
// the pixel.  sk[PAD + k] = s_k = bin_pos(k) for the padded bin range (the
// float64 values the projector computes per ray), read from LDS (LSK) or from
// global memory, so a candidate's offset d is one subtraction.  The padded
// sinogram rows arrive multiplied by their angle's wmax (project_store,
// k_pad_sino), so each candidate adds u * y' with the u of chord_u: the same
// weights as the projector's wmax * u.
//
// Candidate window: bins floor(kf) + 1 .. floor(kf) + NB, kf = t / ds + kb
// (A.kb also carries the + 1 + PAD of the padded index).  Truncation equals
// floor for kf >= 0; a negative kf truncates to a value that, read as
// unsigned, is either 0 or huge, and the clamp to kmax then points at zero
// pads -- in both cases every true candidate lies outside the detector.  A
// candidate that reads a pad gets a weight evaluated at the pad's position and
// multiplies 0.
// Each lane sums PX pixels of one row, (xj[0], yi) ... (xj[PX-1], yi): the
// angle's uniform work (constants, yi s) is shared, the per-pixel sequence is
// the one above.
template <bool HORIZ, bool AXIS, int NB, bool LSK, class TY, int PX>
__device__ __forceinline__ void bp_class(const GeomDev& G, const AngleDev* __restrict__ ang,
                                         int beg, int end, const TY* __restrict__ yp,
                                         const double* __restrict__ skg, const double* sks,
                                         const double* xj, double yi, double* acc) {
    const unsigned kmax = (unsigned)(G.nB + 2 * PAD - NB);   // last padded start index
    // 1/ds held in a vector register, so the index FMA's one scalar operand
    // can be the angle's kb (an FMA reads at most one scalar register)
    double ids = G.inv_ds;
    asm volatile("" : "+v"(ids));
#pragma unroll 2
    for (int a = beg; a < end; ++a) {
        const AngleDev A = ang[a];
        const TY* row = yp + (size_t)A.row * G.pitchB;
        double t[PX];
        const double ys = yi * A.s;
#pragma unroll
        for (int u = 0; u < PX; ++u) t[u] = HORIZ ? fma(yi, A.s, xj[u] * A.c) : fma(xj[u], A.c, ys);
        TY v[PX][NB];
        double sk[PX][NB];
#pragma unroll
        for (int u = 0; u < PX; ++u) {
            const unsigned o = min((unsigned)(int)fma(t[u], ids, A.kb), kmax);
            const TY* pv = at(row, o);
            const double* ps = LSK ? sks + o : skg + o;
#pragma unroll
            for (int q = 0; q < NB; ++q) v[u][q] = pv[q];
#pragma unroll
            for (int q = 0; q < NB; ++q) sk[u][q] = ps[q];
        }
#pragma unroll
        for (int u = 0; u < PX; ++u)   // the sinogram rows carry wmax: y' = wmax y
#pragma unroll
            for (int q = 0; q < NB; ++q)
                acc[u] = fma(chord_u<AXIS>(sk[u][q] - t[u], A.einv, A.inv), (double)v[u][q], acc[u]);
    }
}

// A workgroup owns a tile of 8 rows x 8 PX columns, PX pixels per lane 8
// columns apart (PX = 2 or 4, chosen per launch).  Partial dot products are
// kept per 8 x 16 sub-tile whatever PX is, so the result does not depend on it.
constexpr int BP_TILE = 8;
constexpr int BP_TW = 16;       // sub-tile width of the partials
constexpr int BP_SPLIT = 4;     // waves per workgroup, each over a quarter of the angles
// The bin-position table goes to LDS when it takes at most this many bytes.
constexpr size_t BP_LDS_SK_MAX = 24 * 1024;

__device__ __forceinline__ void split_range(int beg, int end, int w, int& b, int& e) {
    const int len = end - beg;
    b = beg + (len * w) / BP_SPLIT;
    e = beg + (len * (w + 1)) / BP_SPLIT;
}

// out[i][j] = (R^T y)_{ij} from the padded sinogram yp; with dotv != nullptr
// also the float64 partial sum of out * dotv per workgroup.  A workgroup owns
// an 8 x 8PX pixel tile (PX pixels, 8 columns apart, per lane); its wave w
// sums the w-th quarter of every angle class,
// and the four partial sums are added in wave order through LDS.  With LSK the
// workgroup first writes the bin-position table into the dynamic LDS `sks`.
template <int NB, bool LSK, class TY, int PX>
__device__ __forceinline__ void backproject_body(const GeomDev& G, const AngleDev* __restrict__ ang,
                                                 const TY* __restrict__ yp,
                                                 const double* __restrict__ skg, double* sks,
                                                 float* __restrict__ out,
                                                 const double* __restrict__ dotv,
                                                 double* __restrict__ partials, int bx, int by) {
    constexpr int NS = PX / 2;   // 8 x 16 sub-tiles per tile
    __shared__ double part[BP_SPLIT][PX][64];
    __shared__ double red[4 * NS];
    if (LSK) {
        for (int k = threadIdx.x; k < G.nB + 2 * PAD; k += 256) sks[k] = bin_pos((double)(k - PAD), G);
        __syncthreads();
    }
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
    split_range(G.cls[0], G.cls[1], w, b, e);
    bp_class<false, false, NB, LSK, TY, PX>(G, ang, b, e, yp, skg, sks, xj, yi, acc);
    split_range(G.cls[1], G.cls[2], w, b, e);
    bp_class<true, false, NB, LSK, TY, PX>(G, ang, b, e, yp, skg, sks, xj, yi, acc);
    split_range(G.cls[2], G.cls[3], w, b, e);
    bp_class<false, true, NB, LSK, TY, PX>(G, ang, b, e, yp, skg, sks, xj, yi, acc);
    split_range(G.cls[3], G.cls[4], w, b, e);
    bp_class<true, true, NB, LSK, TY, PX>(G, ang, b, e, yp, skg, sks, xj, yi, acc);
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

template <int NB, bool LSK, class TY, int PX>
__global__ __launch_bounds__(256) void k_backproject(GeomDev G, const AngleDev* __restrict__ ang,
                                                     const TY* __restrict__ yp,
                                                     const double* __restrict__ skg,
                                                     float* __restrict__ out,
                                                     const double* __restrict__ dotv,
                                                     double* __restrict__ partials,
                                                     ScalarRide ride,
                                                     const int* __restrict__ halt) {
    if (halt && *halt) return;
    extern __shared__ double sks[];
    backproject_body<NB, LSK, TY, PX>(G, ang, yp, skg, sks, out, dotv, partials, blockIdx.x,
                                      blockIdx.y);
    if (ride.sc && blockIdx.x == 0 && blockIdx.y == 0) {
        if (ride.ps) scalar_body(OP_SNORM, ride.sc, ride.tr, ride.ps, ride.ns, nullptr, 0);
        if (ride.pf) scalar_body(OP_F, ride.sc, ride.tr, ride.pf, ride.nf, nullptr, 0);
    }
}

// TY = float: h = R^T rp (rp = R p) with the partials of h^T p; TY = double:
// g = R^T rpd from the float64 residual.  NB is the largest candidate count of
// the batch (extra candidates weigh exactly 0).
template <int NB, bool LSK, class TY, int PX>
__global__ __launch_bounds__(256) void kb_backproject(const SliceDev* __restrict__ sl, ItemTable t) {
    constexpr bool normal = sizeof(TY) == sizeof(float);
    extern __shared__ double sks[];
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const GeomDev G = S.G;
        const int gx = (G.cols + 8 * PX - 1) / (8 * PX);
        const TY* yp;
        if constexpr (normal) yp = gmem(S.rp);
        else yp = gmem(S.rpd);
        backproject_body<NB, LSK, TY, PX>(G, cmem(S.ang), yp, gmem(S.skp), sks,
                                      gmem(normal ? S.h : S.g), normal ? gmem(S.p) : nullptr,
                                      normal ? gmem(S.pph) : nullptr, lin % gx, lin / gx);
    });
}

size_t bp_lds_bytes(int nbins) {
    const size_t b = ((size_t)nbins + 2 * PAD) * sizeof(double);
    return b <= BP_LDS_SK_MAX ? b : 0;
}

template <bool LSK, class TY, int PX>
void launch_bp_b_px(hipStream_t st, const SliceDev* sl, ItemTable t, int nbmax, size_t lds) {
    switch (nbmax) {
    case 1: hipLaunchKernelGGL((kb_backproject<1, LSK, TY, PX>), dim3(t.grid), dim3(256), lds, st, sl, t); break;
    case 2: hipLaunchKernelGGL((kb_backproject<2, LSK, TY, PX>), dim3(t.grid), dim3(256), lds, st, sl, t); break;
    case 3: hipLaunchKernelGGL((kb_backproject<3, LSK, TY, PX>), dim3(t.grid), dim3(256), lds, st, sl, t); break;
    default: hipLaunchKernelGGL((kb_backproject<4, LSK, TY, PX>), dim3(t.grid), dim3(256), lds, st, sl, t); break;
    }
}

template <bool LSK, class TY>
void launch_bp_b(hipStream_t st, const SliceDev* sl, ItemTable t, int nbmax, size_t lds, int px) {
    if (px == 4) launch_bp_b_px<LSK, TY, 4>(st, sl, t, nbmax, lds);
    else launch_bp_b_px<LSK, TY, 2>(st, sl, t, nbmax, lds);
}

void launch_backproject_b(hipStream_t st, const SliceDev* sl, ItemTable t, int nbmax, int max_bins,
                          bool normal, int px) {
    const size_t lds = bp_lds_bytes(max_bins);
    if (normal) {
        if (lds) launch_bp_b<true, float>(st, sl, t, nbmax, lds, px);
        else launch_bp_b<false, float>(st, sl, t, nbmax, 0, px);
    } else {
        if (lds) launch_bp_b<true, double>(st, sl, t, nbmax, lds, px);
        else launch_bp_b<false, double>(st, sl, t, nbmax, 0, px);
    }
}

int backproject_blocks(const GeomDev& G) {
    return ((G.cols + BP_TW - 1) / BP_TW) * ((G.rows + BP_TILE - 1) / BP_TILE);
}

int backproject_tiles(const GeomDev& G, int px) {
    return ((G.cols + 8 * px - 1) / (8 * px)) * ((G.rows + BP_TILE - 1) / BP_TILE);
}

int backproject_px(int rows, int cols, int resident_waves) {
    // four pixels per lane amortise more of each angle's work but need ~100
    // VGPRs (4 waves per SIMD): take them when the 4-pixel grid still gives
    // every SIMD four waves
    GeomDev G{};
    G.rows = rows;
    G.cols = cols;
    return (long)backproject_tiles(G, 4) * BP_SPLIT >= resident_waves / 2 ? 4 : 2;
}

template <bool LSK, class TY, int PX>
void launch_bp_px(hipStream_t st, const GeomDev& G, const AngleDev* ang, const TY* yp,
                  const double* skp, float* out, const double* dotv, double* partials,
                  const int* halt, size_t lds, const ScalarRide& ride) {
    dim3 grid((G.cols + 8 * PX - 1) / (8 * PX), (G.rows + BP_TILE - 1) / BP_TILE);
    switch (G.nbmax) {
    case 1: hipLaunchKernelGGL((k_backproject<1, LSK, TY, PX>), grid, dim3(256), lds, st, G, ang, yp, skp, out, dotv, partials, ride, halt); break;
    case 2: hipLaunchKernelGGL((k_backproject<2, LSK, TY, PX>), grid, dim3(256), lds, st, G, ang, yp, skp, out, dotv, partials, ride, halt); break;
    case 3: hipLaunchKernelGGL((k_backproject<3, LSK, TY, PX>), grid, dim3(256), lds, st, G, ang, yp, skp, out, dotv, partials, ride, halt); break;
    default: hipLaunchKernelGGL((k_backproject<4, LSK, TY, PX>), grid, dim3(256), lds, st, G, ang, yp, skp, out, dotv, partials, ride, halt); break;
    }
}

template <bool LSK, class TY>
void launch_bp(hipStream_t st, const GeomDev& G, const AngleDev* ang, const TY* yp,
               const double* skp, float* out, const double* dotv, double* partials, const int* halt,
               size_t lds, const ScalarRide& ride) {
    if (G.bp_px == 4) launch_bp_px<LSK, TY, 4>(st, G, ang, yp, skp, out, dotv, partials, halt, lds, ride);
    else launch_bp_px<LSK, TY, 2>(st, G, ang, yp, skp, out, dotv, partials, halt, lds, ride);
}

void launch_backproject(hipStream_t st, const GeomDev& G, const AngleDev* ang, const float* yp,
                        const double* skp, float* out, const double* dotv, double* partials,
                        const int* halt, const ScalarRide& ride) {
    const size_t lds = bp_lds_bytes(G.nB);
    if (lds) launch_bp<true, float>(st, G, ang, yp, skp, out, dotv, partials, halt, lds, ride);
    else launch_bp<false, float>(st, G, ang, yp, skp, out, dotv, partials, halt, 0, ride);
}

void launch_backproject(hipStream_t st, const GeomDev& G, const AngleDev* ang, const double* yp,
                        const double* skp, float* out, const double* dotv, double* partials,
                        const int* halt, const ScalarRide& ride) {
    const size_t lds = bp_lds_bytes(G.nB);
    if (lds) launch_bp<true, double>(st, G, ang, yp, skp, out, dotv, partials, halt, lds, ride);
    else launch_bp<false, double>(st, G, ang, yp, skp, out, dotv, partials, halt, 0, ride);
}

}  // namespace sp
