// Index arithmetic of the projector pair, shared by the kernels and the host
// index checker (all __host__ __device__): the ray a lane of R owns, the
// major-step range and the padded minor coordinate of its walk, and the first
// candidate bin of a pixel in R^T.  Coordinates are in pixel units with the
// image centred at the origin (pixel centre x_j = j - xoff, y_i = yoff - i).
#pragma once

#include "sp_internal.h"

namespace sp {

// Ray of lane `lane` of wave W: index ai of the class-sorted angle table and
// bin k; false for a lane past the end of its class, its tail stream or the
// bins.
__host__ __device__ inline bool wave_ray(const WaveDev& W, int lane, int nB, int& ai, int& k) {
    if (W.tail == WAVE_BLOCK) {
        ai = W.a0 + lane / WAVE_BINS;
        k = W.k0 + lane % WAVE_BINS;
        return ai < W.aend && k < nB;
    }
    if (W.tail == WAVE_ROW) {
        ai = W.a0;
        k = W.k0 + lane;
        return k < nB;
    }
    const int r = nB % WAVE_BINS;
    const int e = W.k0 + lane;
    ai = W.a0 + e / r;
    k = nB - r + e % r;
    return ai < W.aend;
}

// Fractional minor index where ray (A, sk) crosses the centre line of major
// step 0 (row 0 for vertical angles, column 0 for horizontal ones), minus the
// half-width hw of its nonzero band: the axis walk's candidate reference.
template <bool HORIZ>
__host__ __device__ inline double walk_start(const GeomDev& G, const AngleDev& A, double sk) {
    return (HORIZ ? G.yoff - (sk + G.xoff * A.c) / A.s : (sk - G.yoff * A.s) / A.c + G.xoff) -
           (double)A.hw;
}

// Padded minor coordinate (pixel q spans [q, q + 1) after the PAD offset)
// where an oblique ray enters major band 0 on its lower side: band m is then
// met over [b0 + m slope, b0 + m slope + |slope|].
template <bool HORIZ>
__host__ __device__ inline double split_b0(const GeomDev& G, const AngleDev& A, double sk) {
    return (HORIZ ? G.yoff + 0.5 - (sk + (G.xoff + 0.5) * A.c) / A.s
                  : (sk - (G.yoff + 0.5) * A.s) / A.c + G.xoff + 0.5) +
           fmin(A.slope, 0.0) + (double)PAD;
}

// Major-axis steps [lo, hi) of [0, n) where base + m * slope lies in [vlo, vhi],
// widened by one step on each side (a superset of the steps where the ray
// meets the image).
__host__ __device__ inline void step_range(double base, double slope, double vlo, double vhi,
                                           int n, int& lo, int& hi) {
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

// One lane's step range of its ray (before the wave's union is taken).
template <bool HORIZ>
__host__ __device__ inline void ray_steps(const GeomDev& G, const AngleDev& A, double sk, int& lo,
                                          int& hi) {
    const int nmaj = HORIZ ? G.cols : G.rows;
    const int nmin = HORIZ ? G.rows : G.cols;
    step_range(walk_start<HORIZ>(G, A, sk), A.slope, -(double)(A.nc + 1), (double)(nmin + 1), nmaj,
               lo, hi);
}

// Steps [lo, hi) of part `part` of nparts of a wave's common range [lo, hi).
__host__ __device__ inline void part_range(int& lo, int& hi, int part, int nparts) {
    if (nparts > 1 && hi > lo) {
        const int len = hi - lo;
        const int l0 = lo + len * part / nparts;
        hi = lo + len * (part + 1) / nparts;
        lo = l0;
    }
}

// R^T: window index kf = t / ds + kb of a pixel whose centre (xj, yi)
// projects to t = xj c + yi s on the angle's normal.  The pixel's candidate
// bins are the NB bins from padded index trunc(kf) (bin trunc(kf) - PAD).
// Axis-parallel angles form t exactly and divide; oblique ones fold 1/ds into
// the angle's constants (kc = yi s / ds + kb is shared by a lane's pixels),
// and their first candidate's offset s_k - t is dc - ds fract(kf).
__host__ __device__ inline double bp_kf(double t, double inv_ds, double kb) {
    return fma(t, inv_ds, kb);
}
__host__ __device__ inline double bp_kc(double yi, const AngleDev& A) { return fma(yi, A.sids, A.kb); }
__host__ __device__ inline double bp_kf_oblique(double xj, double kc, const AngleDev& A) {
    return fma(xj, A.cids, kc);
}

// Tile (bx, by) of R^T's gx x gy tile grid that launch-order workgroup `id`
// takes.  Workgroups go to the 8 XCDs round-robin in launch order (id mod 8);
// when the grid splits into 4 x 2 equal regions, XCD q takes region
// (q mod 4, q / 4), row by row: a compact image region projects onto a narrow
// band of each sinogram row, so each XCD's L2 holds fewer windows.  Otherwise
// row-major.  The tiles' sums do not depend on the order.
__host__ __device__ inline void bp_tile_of(int id, int gx, int gy, int& bx, int& by) {
    if ((gx & 3) == 0 && (gy & 1) == 0) {
        const int q = id & 7, jj = id >> 3, rw = gx >> 2, rh = gy >> 1;
        bx = (q & 3) * rw + jj % rw;
        by = (q >> 2) * rh + jj / rw;
    } else {
        bx = id % gx;
        by = id / gx;
    }
}

}  // namespace sp
