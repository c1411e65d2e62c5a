// Kaiser-Bessel blob of BlobART (Section 3.4, blob basis): its line integral
// p(d) as a table with cubic Hermite interpolation, shared by the kernels and
// the host check of the table (all of it __host__ __device__ or host-only).
//
// The blob is b(r) = w^m I_m(alpha w) / I_m(alpha), w = sqrt(1 - (r/a)^2), of
// order m = 2.  Its integral along a line at distance d is
//   p(d) = cproj w^(5/2) I_(5/2)(alpha w),  cproj = a sqrt(2 pi / alpha) / I_2(alpha),
// with w = sqrt(1 - (d/a)^2), and, from d/dz [z^nu I_nu(z)] = z^nu I_(nu-1)(z),
//   p'(d) = -cproj alpha (d / a^2) w^(3/2) I_(3/2)(alpha w).
// The table holds (p(d_k), h p'(d_k)) at d_k = k h, h = a / N, k = 0 .. N, from
// the power series of I_nu (all terms positive: no cancellation); p is even,
// so a lookup takes |d|.  Near d = a, p vanishes like (1 - d/a)^(5/2), so the
// interpolation's error there is far below the weights that matter.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace sp {

constexpr int BLOB_TAB_N = 2048;

// I_nu(z) by its power series (host).
inline double blob_bessel_i(double nu, double z) {
    double term = std::pow(0.5 * z, nu) / std::tgamma(nu + 1.0), sum = term;
    for (int k = 1; k < 400; ++k) {
        term *= (0.25 * z * z) / ((double)k * (k + nu));
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

// Fills out[k] = (p(k h), h p'(k h)), k = 0 .. n, h = a / n (host).
inline void blob_table_fill(double a, double alpha, double cproj, int n, double2* out) {
    const double h = a / n;
    for (int k = 0; k <= n; ++k) {
        const double d = k * h, q = d / a, t = 1.0 - q * q;
        double p = 0.0, dp = 0.0;
        if (t > 0.0) {
            const double w = std::sqrt(t), z = alpha * w;
            p = cproj * w * w * std::sqrt(w) * blob_bessel_i(2.5, z);
            dp = -cproj * alpha * (d / (a * a)) * w * std::sqrt(w) * blob_bessel_i(1.5, z);
        }
        out[k] = make_double2(p, h * dp);
    }
}

// p(d) from the table (n intervals of width 1 / inv_h); 0 at and beyond the
// radius.
__host__ __device__ inline double blob_interp(const double2* tab, int n, double inv_h, double d) {
    const double q = fabs(d) * inv_h;
    if (!(q < (double)n)) return 0.0;
    const int k = (int)q;
    const double t = q - (double)k;
    const double2 e0 = tab[k], e1 = tab[k + 1];
    const double t2 = t * t, t3 = t2 * t;
    const double h00 = 2.0 * t3 - 3.0 * t2 + 1.0, h10 = t3 - 2.0 * t2 + t;
    const double h01 = 3.0 * t2 - 2.0 * t3, h11 = t3 - t2;
    return fma(h00, e0.x, fma(h10, e0.y, fma(h01, e1.x, h11 * e1.y)));
}

}  // namespace sp
