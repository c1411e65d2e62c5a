// Host check of the projector pair's index arithmetic, built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host only.  For each geometry read from
// stdin it builds the library's own tables (geometry.cpp) and replays, with the
// same __host__ __device__ helpers the kernels call (sp_walk.h), every index
// the kernels form:
//
//   R (forward walk): the wave table covers every ray exactly once, every wave
//   holds one angle class; the wave's common step range contains every band in
//   which each of its rays meets the image (found here by clipping the line
//   against each band, independently of the kernels' step-range formula); in
//   those bands the gathered pair of minor indices lies inside the padded row
//   and holds every pixel the ray crosses.
//
//   R^T (backward gather): for every pixel of every tile -- including the
//   pixels of partial tiles past the image edge, which the kernel evaluates
//   and does not store -- and every angle, the candidate window; for pixels
//   of the image it lies inside the padded sinogram row and holds every bin
//   whose ray crosses the pixel (|s_k - t| below the trapezoid's half-width,
//   or at most half a pixel for axis-parallel angles), and a window that holds
//   such a bin lies wholly inside the padded sinogram row.  Windows that leave
//   the row (pixels past the image, or outside the detector's field of view)
//   are counted: the kernels' range-checked loads read 0 there.
//
// Input lines: rows cols n_angles n_bins pixel theta0 dtheta bin_spacing
// bin_offset ray_stride pixel_stride (strides > 1 sample rays / pixels).
// Prints one summary line per geometry; exits 1 at the first violation.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/suppcg.h"
#include "../../paper_1807_10151_amd/csrc/sp_internal.h"
#include "../../paper_1807_10151_amd/csrc/sp_walk.h"

using namespace sp;

static int g_fail = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            std::fprintf(stderr, "VIOLATION: " __VA_ARGS__); \
            std::fprintf(stderr, "\n");                   \
            g_fail = 1;                                   \
            return false;                                 \
        }                                                 \
    } while (0)

// Bands [m_in, m_out] in which the line x c + y s = sk meets the image (closed
// pixel squares), by clipping against each band; -1 if none.
template <bool HORIZ>
static void bands_met(const GeomDev& G, const AngleDev& A, double sk, int& m_in, int& m_out) {
    const int nmaj = HORIZ ? G.cols : G.rows;
    const double half = HORIZ ? G.yoff + 0.5 : G.xoff + 0.5;   // minor half-extent
    m_in = m_out = -1;
    for (int m = 0; m < nmaj; ++m) {
        // major coordinate of band m: a row's y, a column's x
        const double c0 = HORIZ ? (double)m - G.xoff - 0.5 : G.yoff - (double)m - 0.5;
        const double c1 = c0 + 1.0;
        // minor coordinate of the line at both band edges
        double u0, u1;
        if (HORIZ) {   // y = (sk - x c) / s
            u0 = (sk - c0 * A.c) / A.s;
            u1 = (sk - c1 * A.c) / A.s;
        } else {       // x = (sk - y s) / c
            u0 = (sk - c0 * A.s) / A.c;
            u1 = (sk - c1 * A.s) / A.c;
        }
        const double lo = std::fmin(u0, u1), hi = std::fmax(u0, u1);
        if (hi >= -half && lo <= half) {
            if (m_in < 0) m_in = m;
            m_out = m;
        }
    }
}

template <bool HORIZ>
static bool check_ray(const GeomDev& G, const AngleDev& A, int k, int wlo, int whi, long& reads) {
    const int nmin = HORIZ ? G.rows : G.cols;
    const int pitch = HORIZ ? G.pitchXT : G.pitchX;
    const double sk = bin_pos((double)k, G);
    int m_in, m_out;
    bands_met<HORIZ>(G, A, sk, m_in, m_out);
    if (m_in < 0) return true;
    CHECK(wlo <= m_in && m_out < whi, "ray k=%d row %d: bands [%d, %d] outside the wave's range [%d, %d)",
          k, A.row, m_in, m_out, wlo, whi);
    if (A.flags & ANG_AXIS) return true;   // trapezoid walk: candidates checked by R^T's window test
    // the split walk's gathered pair, lp advanced as the kernel advances it
    const double sig = A.slope, asig = std::fabs(sig);
    double lp = std::fma((double)wlo, sig, split_b0<HORIZ>(G, A, sk));
    for (int m = wlo; m < whi; ++m, lp += sig) {
        if (m < m_in || m > m_out) continue;
        const int f = (int)lp;   // the kernel's truncation
        CHECK(lp >= 0.0 && f + 1 < pitch,
              "ray k=%d row %d band %d: pair (%d, %d) leaves the padded row of %d", k, A.row, m, f,
              f + 1, pitch);
        // pixels the band's interval [lp, lp + |slope|] overlaps (padded indices)
        const int p0 = (int)std::floor(lp), p1 = (int)std::ceil(lp + asig) - 1;
        for (int q = std::max(p0, PAD); q <= std::min(p1, PAD + nmin - 1); ++q)
            CHECK(q == f || q == f + 1, "ray k=%d row %d band %d: pixel %d not in the pair (%d, %d)",
                  k, A.row, m, q, f, f + 1);
        ++reads;
    }
    return true;
}

static bool check_forward(const GeomDev& G, const std::vector<AngleDev>& tab, int stride,
                          long& rays, long& reads) {
    std::vector<WaveDev> waves((size_t)G.nwaves);
    project_waves(G, waves.data());
    CHECK(G.nwg == (G.nwaves + 3) / 4, "nwg %d for %d waves", G.nwg, G.nwaves);
    std::vector<unsigned char> seen((size_t)G.nA * G.nB, 0);
    for (int w = 0; w < G.nwaves; ++w) {
        const WaveDev& W = waves[(size_t)w];
        CHECK(W.a0 >= 0 && W.a0 < G.nA && W.aend <= G.nA, "wave %d: angles [%d, %d)", w, W.a0, W.aend);
        const int cls = angle_class(tab[(size_t)W.a0]);
        int lo = 1 << 30, hi = -1;
        for (int l = 0; l < 64; ++l) {
            int ai, k;
            if (!wave_ray(W, l, G.nB, ai, k)) continue;
            CHECK(ai >= 0 && ai < G.nA && k >= 0 && k < G.nB, "wave %d lane %d: ray (%d, %d)", w, l, ai, k);
            CHECK(angle_class(tab[(size_t)ai]) == cls, "wave %d lane %d: angle of another class", w, l);
            unsigned char& s = seen[(size_t)ai * G.nB + k];
            CHECK(!s, "ray (%d, %d) in two waves", ai, k);
            s = 1;
            int a, b;
            const double sk = bin_pos((double)k, G);
            if (tab[(size_t)ai].flags & ANG_HORIZ) ray_steps<true>(G, tab[(size_t)ai], sk, a, b);
            else ray_steps<false>(G, tab[(size_t)ai], sk, a, b);
            if (a < b) {   // the kernel's union skips empty lanes
                lo = std::min(lo, a);
                hi = std::max(hi, b);
            }
        }
        const int nmaj = (tab[(size_t)W.a0].flags & ANG_HORIZ) ? G.cols : G.rows;
        if (hi <= lo) continue;
        CHECK(lo >= 0 && hi <= nmaj, "wave %d: step range [%d, %d) of %d", w, lo, hi, nmaj);
        CHECK(wave_steps(G, tab.data(), W) == (long)(hi - lo), "wave %d: host step count differs", w);
        for (int l = 0; l < 64; ++l) {
            int ai, k;
            if (!wave_ray(W, l, G.nB, ai, k)) continue;
            if (((long)ai * G.nB + k) % stride) continue;
            const AngleDev& A = tab[(size_t)ai];
            const bool ok = (A.flags & ANG_HORIZ) ? check_ray<true>(G, A, k, lo, hi, reads)
                                                  : check_ray<false>(G, A, k, lo, hi, reads);
            if (!ok) return false;
            ++rays;
        }
    }
    for (size_t r = 0; r < seen.size(); ++r)
        CHECK(seen[r], "ray (%zu, %zu) in no wave", r / G.nB, r % G.nB);
    return true;
}

static bool check_backward(const GeomDev& G, const std::vector<AngleDev>& tab, int stride,
                           long& pixels, long& out_of_row) {
    const int NB = G.nbmax;
    for (int px : {2, 4}) {
        const int gx = (G.cols + 8 * px - 1) / (8 * px), gy = (G.rows + BP_TILE - 1) / BP_TILE;
        for (int by = 0; by < gy; ++by)
            for (int bx = 0; bx < gx; ++bx)
                for (int lane = 0; lane < 64; ++lane)
                    for (int u = 0; u < px; ++u) {
                        const int i = by * BP_TILE + (lane >> 3);
                        const int j = bx * 8 * px + (lane & 7) + 8 * u;
                        const bool inside = i < G.rows && j < G.cols;
                        if (inside && ((long)i * G.cols + j) % stride) continue;
                        const double yi = G.yoff - (double)i, xj = (double)j - G.xoff;
                        for (int a = 0; a < G.nA; ++a) {
                            const AngleDev& A = tab[(size_t)a];
                            const bool axis = A.flags & ANG_AXIS;
                            const double t = std::fma(xj, A.c, yi * A.s);
                            const double kf = axis ? bp_kf(t, G.inv_ds, A.kb)
                                                   : bp_kf_oblique(xj, bp_kc(yi, A), A);
                            CHECK(std::fabs(kf) < 2.0e9, "pixel (%d, %d) angle %d: window index %g", i, j, a, kf);
                            const int o = (int)kf;
                            const bool in_row = o >= 0 && o + NB <= G.pitchB;
                            if (!in_row) ++out_of_row;
                            if (!inside) continue;
                            // bins whose ray crosses the pixel: all inside the window, and
                            // then the window lies wholly inside the row (so how a load that
                            // straddles a row end is range-checked never matters)
                            const double e = axis ? 0.5 : 0.5 * (std::fabs(A.c) + std::fabs(A.s));
                            const int k0 = (int)std::ceil((t - e - G.s0) / G.ds) - 1;
                            for (int k = std::max(0, k0); k <= std::min(G.nB - 1, k0 + 4 + (int)(2 * e / G.ds)); ++k) {
                                const double d = std::fabs(bin_pos((double)k, G) - t);
                                const bool hit = axis ? d <= 0.5 : d < e;
                                if (!hit) continue;
                                CHECK(k + PAD >= o && k + PAD < o + NB,
                                      "pixel (%d, %d) angle %d: bin %d outside the window [%d, %d)", i,
                                      j, a, k, o - PAD, o - PAD + NB);
                                CHECK(in_row, "pixel (%d, %d) angle %d: window [%d, %d) with bin %d leaves the row of %d",
                                      i, j, a, o, o + NB, k, G.pitchB);
                            }
                        }
                        ++pixels;
                    }
    }
    return true;
}

// R^T's tile order (bp_tile_of): in every gx x gy grid each launch-order
// workgroup takes a tile inside the grid and every tile is taken exactly once.
static bool check_tile_order(int& grids) {
    std::vector<std::pair<int, int>> shapes;
    for (int gx = 1; gx <= 72; ++gx)
        for (int gy = 1; gy <= 160; ++gy) shapes.push_back({gx, gy});
    for (auto s : {std::make_pair(64, 256), std::make_pair(128, 256), std::make_pair(64, 512),
                   std::make_pair(32, 128), std::make_pair(16, 64)})
        shapes.push_back(s);
    for (auto [gx, gy] : shapes) {
        std::vector<char> seen((size_t)gx * gy, 0);
        for (int id = 0; id < gx * gy; ++id) {
            int bx = -1, by = -1;
            bp_tile_of(id, gx, gy, bx, by);
            if (bx < 0 || bx >= gx || by < 0 || by >= gy || seen[(size_t)by * gx + bx]++) {
                std::printf("tile order %dx%d: workgroup %d -> (%d, %d) out of the grid or taken twice\n", gx, gy,
                            id, bx, by);
                return false;
            }
        }
        ++grids;
    }
    return true;
}

int main() {
    char line[512];
    int count = 0;
    int grids = 0;
    if (!check_tile_order(grids)) return 1;
    std::printf("tile order: ok (%d grids)\n", grids);
    while (std::fgets(line, sizeof line, stdin)) {
        sp_geometry g{};
        int rs = 1, ps = 1;
        if (std::sscanf(line, "%d %d %d %d %lf %lf %lf %lf %lf %d %d", &g.rows, &g.cols, &g.n_angles,
                        &g.n_bins, &g.pixel, &g.theta0, &g.dtheta, &g.bin_spacing, &g.bin_offset, &rs,
                        &ps) != 11)
            continue;
        GeomDev G{};
        std::vector<AngleDev> tab((size_t)g.n_angles);
        char err[256] = {0};
        if (build_geometry_into(&g, 256, G, tab.data(), err, sizeof err) != SP_OK) {
            std::printf("%dx%d %dx%d: rejected (%s)\n", g.rows, g.cols, g.n_angles, g.n_bins, err);
            continue;
        }
        long rays = 0, reads = 0, pixels = 0, oor = 0;
        if (!check_forward(G, tab, rs, rays, reads) || !check_backward(G, tab, ps, pixels, oor)) {
            std::printf("%dx%d %dx%d: FAILED\n", g.rows, g.cols, g.n_angles, g.n_bins);
            return 1;
        }
        std::printf("%dx%d %dx%d: ok (waves %d, rays %ld, band reads %ld, pixels %ld, "
                    "windows leaving the row %ld)\n",
                    g.rows, g.cols, g.n_angles, g.n_bins, G.nwaves, rays, reads, pixels, oor);
        ++count;
    }
    std::printf("checked %d geometries\n", count);
    return g_fail;
}
