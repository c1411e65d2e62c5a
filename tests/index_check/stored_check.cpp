// Host replay of the stored-matrix build (the row enumeration of sp_stored.h
// that the build kernels run), built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host only.  For each geometry read from
// stdin it enumerates every row of R (by ray) and of R^T (by pixel) twice, as
// the count and the fill kernels do, and checks that
//   * both passes of a row visit the same entries (the fill stays inside the
//     row's slot of the counted offsets),
//   * every column index lies in [0, n) for R and [0, m) for R^T and every
//     stored weight is positive and finite,
//   * R^T is exactly the transpose of R (same entries, bit-identical weights),
//   * the sliced-ELL placement (slice sizes from the longest row, offsets from
//     their scan, entry offsets of sell_offset) puts every entry of every row
//     inside its slice and no two entries at the same place.
// With --dump PATH the entries of R for the last geometry are written to PATH
// as records (int32 ray, int32 pixel, float64 weight) in R's row order.
//
// Input lines: rows cols n_angles n_bins pixel theta0 dtheta bin_spacing bin_offset
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/suppcg.h"
#include "../../paper_1807_10151_amd/csrc/sp_internal.h"
#include "../../paper_1807_10151_amd/csrc/sp_stored.h"

using namespace sp;

struct Entry {
    int32_t row, col;
    double w;
};

int main(int argc, char** argv) {
    const char* dump = nullptr;
    if (argc == 3 && std::strcmp(argv[1], "--dump") == 0) dump = argv[2];
    char line[512];
    int count = 0;
    std::vector<Entry> last;
    while (std::fgets(line, sizeof line, stdin)) {
        sp_geometry g{};
        if (std::sscanf(line, "%d %d %d %d %lf %lf %lf %lf %lf", &g.rows, &g.cols, &g.n_angles, &g.n_bins,
                        &g.pixel, &g.theta0, &g.dtheta, &g.bin_spacing, &g.bin_offset) != 9)
            continue;
        GeomDev G{};
        std::vector<AngleDev> tab((size_t)g.n_angles);
        char err[256] = {0};
        if (build_geometry_into(&g, 256, G, tab.data(), err, sizeof err) != SP_OK) {
            std::printf("%dx%d %dx%d: rejected (%s)\n", g.rows, g.cols, g.n_angles, g.n_bins, err);
            continue;
        }
        std::vector<AngleDev> nat((size_t)G.nA);
        for (const AngleDev& A : tab) nat[(size_t)A.row] = A;
        const int n = G.rows * G.cols, m = G.nA * G.nB;
        std::vector<Entry> r_ent, t_ent;
        for (int r = 0; r < m; ++r) {
            int cnt = 0;
            ray_nonzeros(G, nat[(size_t)(r / G.nB)], r % G.nB, [&](int, double) { ++cnt; });
            int fill = 0;
            ray_nonzeros(G, nat[(size_t)(r / G.nB)], r % G.nB, [&](int q, double w) {
                if (q < 0 || q >= n || !(w > 0.0) || !std::isfinite(w)) {
                    std::fprintf(stderr, "VIOLATION: ray %d pixel %d weight %g\n", r, q, w);
                    std::exit(1);
                }
                r_ent.push_back({r, q, w});
                ++fill;
            });
            if (fill != cnt) {
                std::fprintf(stderr, "VIOLATION: ray %d counted %d filled %d\n", r, cnt, fill);
                return 1;
            }
        }
        for (int q = 0; q < n; ++q) {
            int cnt = 0;
            pixel_nonzeros(G, nat.data(), q / G.cols, q % G.cols, [&](int, double) { ++cnt; });
            int fill = 0;
            int prev = -1;
            pixel_nonzeros(G, nat.data(), q / G.cols, q % G.cols, [&](int r, double w) {
                if (r < 0 || r >= m || r <= prev || !(w > 0.0) || !std::isfinite(w)) {
                    std::fprintf(stderr, "VIOLATION: pixel %d ray %d (after %d) weight %g\n", q, r, prev, w);
                    std::exit(1);
                }
                prev = r;
                t_ent.push_back({q, r, w});
                ++fill;
            });
            if (fill != cnt) {
                std::fprintf(stderr, "VIOLATION: pixel %d counted %d filled %d\n", q, cnt, fill);
                return 1;
            }
        }
        // sliced-ELL placement of both sides
        for (int sd = 0; sd < 2; ++sd) {
            const SellShape S = sd == 0 ? SellShape{G.nA, G.nB, (G.nB + 63) / 64}
                                        : SellShape{G.rows, G.cols, (G.cols + 63) / 64};
            const int64_t rows = sd == 0 ? m : n, ns = S.nseg * S.spseg;
            std::vector<int32_t> len((size_t)rows, 0);
            for (const Entry& en : sd == 0 ? r_ent : t_ent) ++len[(size_t)en.row];
            std::vector<int64_t> sp((size_t)ns + 1, 0);
            for (int64_t sl = 0; sl < ns; ++sl) {
                const int64_t seg = sl / S.spseg, k0 = (sl % S.spseg) * 64;
                int w = 0;
                for (int l = 0; l < 64 && k0 + l < S.lseg; ++l) w = imax(w, len[(size_t)(seg * S.lseg + k0 + l)]);
                sp[(size_t)sl + 1] = sp[(size_t)sl] + 128 * ((w + 3) & ~3);
            }
            std::vector<unsigned char> used((size_t)sp[(size_t)ns], 0);
            for (int64_t r = 0; r < rows; ++r) {
                const int64_t sl = sell_slice(S, r);
                const int lane = sell_lane(S, r);
                if (sl < 0 || sl >= ns || lane < 0 || lane > 63 || (r % S.lseg) / 64 != sl % S.spseg) {
                    std::fprintf(stderr, "VIOLATION: side %d row %lld slice %lld lane %d\n", sd, (long long)r,
                                 (long long)sl, lane);
                    return 1;
                }
                for (int e = 0; e < len[(size_t)r]; ++e) {
                    const int64_t p = sp[(size_t)sl] + sell_offset(lane, e);
                    const int64_t pv = p + SELL_VAL;
                    if (p < sp[(size_t)sl] || pv >= sp[(size_t)sl + 1] || used[(size_t)p] || used[(size_t)pv]) {
                        std::fprintf(stderr, "VIOLATION: side %d row %lld entry %d at %lld\n", sd, (long long)r,
                                     e, (long long)p);
                        return 1;
                    }
                    used[(size_t)p] = used[(size_t)pv] = 1;
                }
            }
        }
        // R^T = R transposed: sort R's entries by (pixel, ray)
        std::vector<Entry> rt = r_ent;
        std::sort(rt.begin(), rt.end(), [](const Entry& a, const Entry& b) {
            return a.col != b.col ? a.col < b.col : a.row < b.row;
        });
        if (rt.size() != t_ent.size()) {
            std::fprintf(stderr, "VIOLATION: R has %zu nonzeros, R^T %zu\n", rt.size(), t_ent.size());
            return 1;
        }
        for (size_t e = 0; e < rt.size(); ++e)
            if (rt[e].col != t_ent[e].row || rt[e].row != t_ent[e].col || rt[e].w != t_ent[e].w) {
                std::fprintf(stderr, "VIOLATION: entry %zu: R (%d, %d, %.17g) R^T (%d, %d, %.17g)\n", e,
                             rt[e].row, rt[e].col, rt[e].w, t_ent[e].col, t_ent[e].row, t_ent[e].w);
                return 1;
            }
        std::printf("%dx%d %dx%d: ok (nnz %zu)\n", g.rows, g.cols, g.n_angles, g.n_bins, r_ent.size());
        last.swap(r_ent);
        ++count;
    }
    if (dump) {
        FILE* f = std::fopen(dump, "wb");
        if (!f) return 2;
        for (const Entry& e : last) {
            std::fwrite(&e.row, 4, 1, f);
            std::fwrite(&e.col, 4, 1, f);
            std::fwrite(&e.w, 8, 1, f);
        }
        std::fclose(f);
    }
    std::printf("checked %d geometries\n", count);
    return 0;
}
