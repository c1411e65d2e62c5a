// The nonzeros of R (Section 2, eq. 2.1) one row at a time, for building R
// and R^T as stored matrices: the visiting order of a ray's pixels and of a
// pixel's rays, and the weight of each.  __host__ __device__, so the host
// index checker replays exactly what the build kernels do.
#pragma once

#include <cmath>

#include "sp_internal.h"

namespace sp {

__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }
__host__ __device__ inline int imin(int a, int b) { return a < b ? a : b; }

// Length (in the geometry's unit) of ray k of angle A inside pixel (i, j):
// wmax * u with the trapezoid u of chord_u on the offset s_k - t of the
// pixel centre's projection t (formed as the forward walk forms it).
__host__ __device__ inline double stored_weight(const GeomDev& G, const AngleDev& A, int i, int j,
                                                double sk) {
    const double xj = (double)j - G.xoff, yi = G.yoff - (double)i;
    const double t = (A.flags & ANG_HORIZ) ? fma(yi, A.s, xj * A.c) : fma(xj, A.c, yi * A.s);
    const double d = sk - t;
    const double u = (A.flags & ANG_AXIS) ? chord_u<true>(d, A.einv, A.inv)
                                          : chord_u<false>(d, A.einv, A.inv);
    return A.wmax * u * G.pixel;
}

__host__ __device__ inline double half_band(const AngleDev& A) { return 0.5 * (fabs(A.c) + fabs(A.s)); }

// Visits the nonzeros of ray k of angle A on one major line m (image row m
// when |cos| >= |sin|, else column m): the minor indices of the band
// |s_k - t| < e in increasing order.
template <class F>
__host__ __device__ inline void ray_line_nonzeros(const GeomDev& G, const AngleDev& A, double sk, int m,
                                                  F&& emit) {
    const double e = half_band(A);
    if (!(A.flags & ANG_HORIZ)) {
        const double hw = e / fabs(A.c);
        const double yi = G.yoff - (double)m;
        const double xs = (sk - yi * A.s) / A.c + G.xoff;   // column coordinate of the crossing
        const int lo = imax((int)floor(xs - hw) - 1, 0);
        const int hi = imin((int)ceil(xs + hw) + 1, G.cols - 1);
        for (int j = lo; j <= hi; ++j) {
            const double w = stored_weight(G, A, m, j, sk);
            if (w > 0.0) emit(m * G.cols + j, w);
        }
    } else {
        const double hw = e / fabs(A.s);
        const double xj = (double)m - G.xoff;
        const double ys = G.yoff - (sk - xj * A.c) / A.s;   // row coordinate of the crossing
        const int lo = imax((int)floor(ys - hw) - 1, 0);
        const int hi = imin((int)ceil(ys + hw) + 1, G.rows - 1);
        for (int i = lo; i <= hi; ++i) {
            const double w = stored_weight(G, A, i, m, sk);
            if (w > 0.0) emit(i * G.cols + m, w);
        }
    }
}

// Major lines of angle A: image rows when |cos| >= |sin|, else columns.
__host__ __device__ inline int ray_lines(const GeomDev& G, const AngleDev& A) {
    return (A.flags & ANG_HORIZ) ? G.cols : G.rows;
}

// Visits the nonzeros of ray (a, k) in a fixed order: major lines in
// increasing order, and on each the band's minor indices in increasing order.
template <class F>
__host__ __device__ inline void ray_nonzeros(const GeomDev& G, const AngleDev& A, int k, F&& emit) {
    const double sk = bin_pos((double)k, G);
    const int nl = ray_lines(G, A);
    for (int m = 0; m < nl; ++m) ray_line_nonzeros(G, A, sk, m, emit);
}

// ART's ray phases of angle A (Section 3.4): rays of one angle whose bin
// indices differ by q or more touch disjoint pixels when q ds > 2 e (e =
// half the width of a pixel's footprint on the detector), so one phase of an
// angle is the rays k = ph, ph + q, ...; q = floor(2 e / ds + 1e-9) + 1 (the
// 1e-9 keeps a ratio that rounds just below an integer from giving a zero
// margin).
__host__ __device__ inline int art_phases(const GeomDev& G, const AngleDev& A) {
    return (int)floor(2.0 * half_band(A) / G.ds + 1e-9) + 1;
}

// Visits the nonzeros of pixel (i, j): angles in increasing order, and for
// each the bins of |s_k - t| < e in increasing order (ray index a * nB + k).
template <class F>
__host__ __device__ inline void pixel_nonzeros(const GeomDev& G, const AngleDev* nat,
                                               int i, int j, F&& emit) {
    const double xj = (double)j - G.xoff, yi = G.yoff - (double)i;
    for (int a = 0; a < G.nA; ++a) {
        const AngleDev A = nat[a];
        const double t = (A.flags & ANG_HORIZ) ? fma(yi, A.s, xj * A.c) : fma(xj, A.c, yi * A.s);
        const double e = half_band(A);
        const int lo = imax((int)floor((t - e - G.s0) * G.inv_ds) - 1, 0);
        const int hi = imin((int)ceil((t + e - G.s0) * G.inv_ds) + 1, G.nB - 1);
        for (int k = lo; k <= hi; ++k) {
            const double w = stored_weight(G, A, i, j, bin_pos((double)k, G));
            if (w > 0.0) emit(a * G.nB + k, w);
        }
    }
}

// Sliced-ELL placement (64-row slices, segments start new slices, entries
// in groups of four per lane, a group's column indices and weights side by
// side): the slice and lane of row r, and the word offset of the column index
// of a lane's entry e from its slice's start (its weight is SELL_VAL words
// further).  A slice of width w (a multiple of 4) spans 128 w words.
constexpr int SELL_VAL = 256;
__host__ __device__ inline int64_t sell_slice(const SellShape& S, int64_t r) {
    return (r / S.lseg) * S.spseg + (r % S.lseg) / 64;
}
__host__ __device__ inline int sell_lane(const SellShape& S, int64_t r) { return (int)((r % S.lseg) & 63); }
__host__ __device__ inline int64_t sell_offset(int lane, int e) {
    return (int64_t)(e >> 2) * 512 + 4 * lane + (e & 3);
}

}  // namespace sp
