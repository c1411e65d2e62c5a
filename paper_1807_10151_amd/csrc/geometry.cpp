// Host side of the geometry: the class-sorted angle table (Section 4.1's
// equally spaced angles, cos/sin snapped at multiples of pi/4), the bin
// positions, R's wave table and dispatch order, and the launch shapes of R and
// R^T.  Plain C++ with no runtime calls, so that the index checker can build it
// on the host alone.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "../../include/suppcg.h"
#include "sp_internal.h"
#include "sp_walk.h"

namespace sp {

void angle_cos_sin(const sp_geometry& g, int a, double& co, double& si) {
    const double dth = g.dtheta > 0.0 ? g.dtheta : M_PI / g.n_angles;
    const double th = g.theta0 + a * dth;
    const double q = th / (M_PI / 4.0);
    const double m = std::nearbyint(q);
    if (std::fabs(q - m) < 1e-12) {
        static const double h = std::sqrt(0.5);
        static const double tc[8] = {1.0, h, 0.0, -h, -1.0, -h, 0.0, h};
        static const double ts[8] = {0.0, h, 1.0, h, 0.0, -h, -1.0, -h};
        long long mi = (long long)m % 8;
        if (mi < 0) mi += 8;
        co = tc[mi];
        si = ts[mi];
    } else {
        co = std::cos(th);
        si = std::sin(th);
    }
}

AngleDev angle_entry(const sp_geometry& g, int a, double ds, double s0, double margin) {
    double co, si;
    angle_cos_sin(g, a, co, si);
    AngleDev A{};
    A.c = co;
    A.s = si;
    const double ac = std::fabs(co), as = std::fabs(si);
    const bool axis = ac == 0.0 || as == 0.0;
    const bool horiz = as > ac;
    const double e = 0.5 * (ac + as);
    const double inv = axis ? 0.0 : 1.0 / std::min(ac, as);
    A.inv = inv;
    A.einv = e * inv;
    A.wmax = 1.0 / std::max(ac, as);
    A.slope = horiz ? co / si : si / co;
    const double hw = e / std::max(ac, as) + margin;
    A.hw = (float)hw;
    A.nc = (int)std::ceil(2.0 * hw);
    const double hb = (e + margin) / ds;
    A.nb = (int)std::ceil(2.0 * hb);
    A.kb = -s0 / ds - hb + 1.0 + PAD;
    A.dc = ds * (1.0 - hb);
    A.cids = co / ds;
    A.sids = si / ds;
    A.row = a;
    A.flags = (axis ? ANG_AXIS : 0) | (horiz ? ANG_HORIZ : 0);
    return A;
}

int angle_class(const AngleDev& A) {
    const bool axis = A.flags & ANG_AXIS, horiz = A.flags & ANG_HORIZ;
    return (axis ? 2 : 0) + (horiz ? 1 : 0);
}

namespace {
int geom_fail(char* err, size_t n, const char* fmt, ...) {
    if (err && n) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(err, n, fmt, ap);
        va_end(ap);
    }
    return SP_ERR_ARG;
}
}  // namespace

int project_wave_count(const GeomDev& G) { return project_waves(G, nullptr); }

int project_waves(const GeomDev& G, WaveDev* out) {
    // Oblique classes: waves of WAVE_ANGLES angles by WAVE_BINS bins, a
    // workgroup's four waves the four 16-bin sub-chunks of one 64-bin chunk
    // for the same four neighbouring angles (rays that cross nearly the same
    // pixels), chunk by chunk; then the classes' packed tails (the last
    // nB % WAVE_BINS bins).  Axis-parallel classes: waves of 64 bins of one
    // angle.  The dispatch order sorts workgroups by cost and keeps this
    // order among equal costs, so workgroups that run side by side on the GPU
    // read neighbouring parts of the image.
    const int r = G.nB % WAVE_BINS, full = G.nB / WAVE_BINS;
    int w = 0;
    auto put = [&](const WaveDev& W) {
        if (out) out[w] = W;
        ++w;
    };
    for (int c = 0; c < full; c += 4)
        for (int q = 0; q < 2; ++q) {
            const int a0 = G.cls[q], a1 = G.cls[q + 1];
            for (int g0 = a0; g0 < a1; g0 += WAVE_ANGLES)
                for (int j = c; j < std::min(full, c + 4); ++j) put(WaveDev{g0, WAVE_BINS * j, a1, WAVE_BLOCK});
        }
    for (int q = 0; q < 2; ++q) {
        const int a0 = G.cls[q], a1 = G.cls[q + 1];
        if (r == 0) continue;
        const int stream = (a1 - a0) * r;
        for (int e = 0; e < stream; e += 64) put(WaveDev{a0, e, a1, WAVE_TAIL});
    }
    for (int q = 2; q < 4; ++q)
        for (int a = G.cls[q]; a < G.cls[q + 1]; ++a)
            for (int k0 = 0; k0 < G.nB; k0 += 64) put(WaveDev{a, k0, a + 1, WAVE_ROW});
    return w;
}

int project_parts(int rows, int cols, int nwaves, int resident_waves) {
    // Large images: 8 parts keep the resident waves on a band of the float64
    // copies (measured: 2048^2 x 2048 angles 9.3 -> 5.8 ms).
    if ((long)rows * cols >= (1L << 21)) return 8;
    // Otherwise split only a grid that would leave a tenth of the wave slots
    // or more empty (a split costs a combine pass and a second walk set-up;
    // 512^2 x 720, 8,159 waves on 8,192 slots: one part 0.095 ms, two 0.12).
    if (10L * nwaves >= 9L * resident_waves) return 1;
    const long p = (resident_waves + nwaves - 1) / nwaves;
    return p > 4 ? 4 : (int)p;
}

int backproject_tiles(const GeomDev& G, int px) {
    return ((G.cols + 8 * px - 1) / (8 * px)) * ((G.rows + BP_TILE - 1) / BP_TILE);
}


int backproject_px(int rows, int cols, int resident_waves) {
    // four pixels per lane amortise more of each angle's work but need more
    // VGPRs: take them when the 4-pixel grid still gives every SIMD four waves
    GeomDev G{};
    G.rows = rows;
    G.cols = cols;
    return (long)backproject_tiles(G, 4) * BP_SPLIT >= resident_waves / 2 ? 4 : 2;
}

int project_comb_blocks(const GeomDev& G) { return G.nA * ((G.nB + 255) / 256); }

int project_blocks(const GeomDev& G) {
    return G.parts > 1 ? project_comb_blocks(G) : G.nwg;
}

int build_geometry_into(const sp_geometry* g, int n_cu, GeomDev& G, AngleDev* tab, char* err,
                        size_t errlen) {
    G = GeomDev{};
    G.rows = g->rows;
    G.cols = g->cols;
    G.nA = g->n_angles;
    G.nB = g->n_bins;
    G.xoff = (g->cols - 1) / 2.0;
    G.yoff = (g->rows - 1) / 2.0;
    const double ds = g->bin_spacing / g->pixel;
    const double s0 = (-(g->n_bins - 1) / 2.0 * g->bin_spacing + g->bin_offset) / g->pixel;
    G.ds = ds;
    G.s0 = s0;
    G.inv_ds = 1.0 / ds;
    G.pixel = g->pixel;
    G.pitchX = g->cols + 2 * PAD;
    G.pitchXT = g->rows + 2 * PAD;
    G.pitchB = g->n_bins + 2 * PAD;
    const double margin = 1e-3 + 4e-7 * (double)(g->rows + g->cols + g->n_bins);
    G.nbmax = 1;
    for (int q = 0; q <= 4; ++q) G.cls[q] = 0;
    for (int a = 0; a < g->n_angles; ++a) {
        const AngleDev A = angle_entry(*g, a, ds, s0, margin);
        if (A.nc < 2 || A.nc > 3 || A.nb < 1 || A.nb > 4)
            return geom_fail(err, errlen, "unsupported geometry at angle %d (nc=%d nb=%d)", a, A.nc, A.nb);
        G.nbmax = std::max(G.nbmax, A.nb);
        G.cls[angle_class(A) + 1] += 1;
    }
    for (int q = 1; q <= 4; ++q) G.cls[q] += G.cls[q - 1];
    // stable counting sort by class, no allocation
    int pos = 0;
    for (int q = 0; q < 4; ++q)
        for (int a = 0; a < g->n_angles; ++a) {
            const AngleDev A = angle_entry(*g, a, ds, s0, margin);
            if (angle_class(A) == q) tab[pos++] = A;
        }
    G.nwaves = project_wave_count(G);
    G.nwg = (G.nwaves + 3) / 4;
    G.parts = project_parts(g->rows, g->cols, G.nwaves, n_cu * 32);
    G.bp_px = backproject_px(g->rows, g->cols, n_cu * 32);
    return SP_OK;
}

void bin_sk_fill(const GeomDev& G, double* t) {
    for (int k = -PAD; k < G.nB + PAD; ++k) t[k + PAD] = std::fma((double)k, G.ds, G.s0);
}

namespace {
// A lane's step range as the kernel forms it; false when it is empty (the lane
// then takes no part in its wave's union).
bool lane_steps(const GeomDev& G, const AngleDev& A, int k, int& lo, int& hi) {
    const double sk = std::fma((double)k, G.ds, G.s0);
    if (A.flags & ANG_HORIZ) ray_steps<true>(G, A, sk, lo, hi);
    else ray_steps<false>(G, A, sk, lo, hi);
    return hi > lo;
}
}  // namespace

long wave_steps(const GeomDev& G, const AngleDev* tab, const WaveDev& W) {
    int lo = 1 << 30, hi = -1;
    auto add = [&](int lane) {
        int ai, k, l, h;
        if (!wave_ray(W, lane, G.nB, ai, k)) return false;
        if (!lane_steps(G, tab[ai], k, l, h)) return false;
        lo = std::min(lo, l);
        hi = std::max(hi, h);
        return true;
    };
    if (W.tail != WAVE_ROW) {
        for (int l = 0; l < 64; ++l) add(l);
    } else {
        // the rays of one angle that meet the image are consecutive bins, and a
        // ray's range moves monotonically with its bin: the first and last
        // lanes with a nonempty range bound the union
        const int last = std::min(63, G.nB - 1 - W.k0);
        int l = 0;
        while (l <= last && !add(l)) ++l;
        int m = last;
        while (m > l && !add(m)) --m;
    }
    return hi > lo ? (long)(hi - lo) : 0;
}

std::vector<int32_t> project_order(const GeomDev& G, const AngleDev* tab, const WaveDev* waves,
                                   int n_cu) {
    const int nwg = G.nwg;
    std::vector<long> cost((size_t)nwg, 0);
    for (int w = 0; w < G.nwaves; ++w) cost[(size_t)(w / 4)] += 16 + wave_steps(G, tab, waves[w]);
    std::vector<int32_t> ord((size_t)nwg);
    for (int b = 0; b < nwg; ++b) ord[(size_t)b] = b;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int32_t x, int32_t y) { return cost[(size_t)x] > cost[(size_t)y]; });
    const int band = std::max(1, n_cu);
    for (int b0 = band, i = 1; b0 < nwg; b0 += band, ++i)
        if (i & 1) std::reverse(ord.begin() + b0, ord.begin() + std::min(nwg, b0 + band));
    return ord;
}

}  // namespace sp
