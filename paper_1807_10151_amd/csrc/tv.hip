// Total-variation superiorization (Section 3.1, Algorithm 1) on the GPU.
//
// One S_TV inner step is four launches:
//   k_tv_grad    t_bar (minus the TV gradient where defined, 0 elsewhere) and
//                per-workgroup partials of ||t_bar||^2 (one pixel per thread
//                for an S_TV call's first step, tv_px for later ones, whose
//                t_bar the single-slice solver forms in k_tv_apply_grad);
//   k_tv_trials  TV(y) and TV(y + lam_j t_bar) for the next J trial step
//                lengths lam_j = gamma a^(l + j) / ||t_bar|| in one pass, each as
//                per-workgroup float64 partials (tv_px pixels per thread: on
//                large images fewer workgroups re-read the ||t_bar||^2
//                partials and the decision sums fewer partials);
//   k_tv_decide  one workgroup: sums the partials in a fixed order, takes the
//                first trial with TV(trial) <= TV(y) (Algorithm 1's "until"),
//                advances l by the trials used, records the step; if none of the
//                J is accepted it evaluates further batches itself;
//   k_tv_apply   y <- y + lam t_bar (and ||s_k||^2 partials on the last step).
// The single-slice solver fuses two pairs: between inner steps the update and
// the next t_bar are one launch (k_tv_apply_grad), and the last update also
// writes R's padded copies of x_{k+1/2} (k_tv_apply_prep; the batched solver
// runs the same body).  k_tv_apply_grad repeats the arithmetic of the two
// launches it replaces, so results are bitwise those of the batched solver,
// which keeps them separate.
// Trial TVs are evaluated in float64 directly on y + lam t_bar (the trial image
// is never rounded to float32), so the acceptance test sees the step itself.
#include "sp_internal.h"
#include "sp_reduce.h"

namespace sp {

constexpr int TVJ = 4;   // trials evaluated per pass (the first is accepted in most loop bodies)
// Pixels per thread of the trials and of t_bar after an S_TV call's first
// inner step: 4 from 2^18 pixels up (at least one workgroup per compute unit),
// else 1.
__host__ __device__ __forceinline__ int tv_px(size_t n) { return n >= ((size_t)1 << 18) ? 4 : 1; }

// t_bar at pixel p = (i, j) of a rows x cols float64 image whose value at q
// is y(q), evaluated in float64 and rounded to float32 (reading: the partial
// derivative is undefined when a square-root term it enters is zero).
template <class Y>
__device__ __forceinline__ float tv_neg_grad_at(Y&& y, int rows, int cols, int i, int j, size_t p) {
    const double v = y(p);
    double gsum = 0.0;
    bool bad = false;
    if (i < rows - 1 && j < cols - 1) {          // T_{i,j}
        const double dv = v - y(p + cols), dh = v - y(p + 1);
        if (dv == 0.0 && dh == 0.0) bad = true;
        else gsum += (dv + dh) / sqrt(dv * dv + dh * dh);
    }
    if (i >= 1 && j < cols - 1) {                // T_{i-1,j}
        const double u = y(p - cols);
        const double dv = u - v, dh = u - y(p - cols + 1);
        if (dv == 0.0 && dh == 0.0) bad = true;
        else gsum -= dv / sqrt(dv * dv + dh * dh);
    }
    if (i < rows - 1 && j >= 1) {                // T_{i,j-1}
        const double u = y(p - 1);
        const double dv = u - y(p - 1 + cols), dh = u - v;
        if (dv == 0.0 && dh == 0.0) bad = true;
        else gsum -= dh / sqrt(dv * dv + dh * dh);
    }
    return bad ? 0.0f : (float)(-gsum);
}
__device__ __forceinline__ float tv_neg_grad(const double* __restrict__ y, int rows, int cols,
                                             int i, int j, size_t p) {
    return tv_neg_grad_at([&](size_t q) { return y[q]; }, rows, cols, i, j, p);
}

__device__ __forceinline__ void tv_grad_body(int rows, int cols, const double* __restrict__ y,
                                             float* __restrict__ tb, double* __restrict__ partials,
                                             int bx, int gpx) {
    __shared__ double red[4];
    const size_t n = (size_t)rows * cols;
    double sq = 0.0;
    for (int r = 0; r < gpx; ++r) {
        const size_t p = ((size_t)bx * gpx + r) * 256 + threadIdx.x;
        if (p < n) {
            const int i = (int)(p / cols), j = (int)(p - (size_t)i * cols);
            const float t = tv_neg_grad(y, rows, cols, i, j, p);
            tb[p] = t;
            sq += (double)t * (double)t;
        }
    }
    const double tot = block_sum(sq, red);
    if (partials && threadIdx.x == 0) partials[bx] = tot;
}

__global__ __launch_bounds__(256) void k_tv_grad(int rows, int cols, const double* __restrict__ y,
                                                 float* __restrict__ tb,
                                                 double* __restrict__ partials, int gpx,
                                                 const int* __restrict__ halt) {
    if (halt && *halt) return;
    tv_grad_body(rows, cols, y, tb, partials, blockIdx.x, gpx);
}

int tv_blocks(int rows, int cols) { return (int)(((size_t)rows * cols + 255) / 256); }
int tv_grad_blocks(int rows, int cols) {
    const size_t n = (size_t)rows * cols;
    return (int)((n + 256 * tv_px(n) - 1) / (256 * tv_px(n)));
}
int tv_tpx_blocks(int rows, int cols) {
    const size_t n = (size_t)rows * cols;
    return (int)((n + 256 * tv_px(n) - 1) / (256 * tv_px(n)));
}

void launch_tv_grad(hipStream_t st, int rows, int cols, const double* y, float* tb, double* partials,
                    const int* halt, bool later) {
    const int gpx = later ? tv_px((size_t)rows * cols) : 1;
    hipLaunchKernelGGL(k_tv_grad, dim3(later ? tv_grad_blocks(rows, cols) : tv_blocks(rows, cols)), dim3(256),
                       0, st, rows, cols, y, tb, partials, gpx, halt);
}

// TV terms of pixel p for the base image (q = 0) and nq trial steps lam[0..nq).
template <int NQ>
__device__ __forceinline__ void tv_terms(const double* __restrict__ y, const float* __restrict__ tb,
                                         int cols, size_t p, const double* lam, int nq,
                                         double* acc) {
    const double dv = y[p] - y[p + cols];
    const double dh = y[p] - y[p + 1];
    const double ev = (double)tb[p] - (double)tb[p + cols];
    const double eh = (double)tb[p] - (double)tb[p + 1];
    acc[0] += sqrt(dv * dv + dh * dh);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (q < nq) {
            const double a = fma(lam[q], ev, dv);
            const double b = fma(lam[q], eh, dh);
            acc[q + 1] += sqrt(a * a + b * b);
        }
    }
}

__device__ __forceinline__ double trial_lambda(const Scalars* sc, int trial, double tn) {
    // trial = 0-based index from the current l: step gamma * a^(l + trial)
    return tn > 0.0 ? sc->gamma * pow(sc->a, (double)(sc->ell + trial)) / tn : 0.0;
}

__device__ __forceinline__ void tv_trials_body(int rows, int cols, const double* __restrict__ y,
                                               const float* __restrict__ tb,
                                               const double* __restrict__ gpart, int ngpart,
                                               const Scalars* __restrict__ sc,
                                               double* __restrict__ tpart, int bx) {
    __shared__ double red[4];
    __shared__ double lam[TVJ];
    const double tn = sqrt(reduce_partials(gpart, ngpart, red));
    if (threadIdx.x < TVJ) lam[threadIdx.x] = trial_lambda(sc, threadIdx.x, tn);
    __syncthreads();
    double lam_r[TVJ];
#pragma unroll
    for (int q = 0; q < TVJ; ++q) lam_r[q] = lam[q];
    double acc[TVJ + 1];
#pragma unroll
    for (int q = 0; q <= TVJ; ++q) acc[q] = 0.0;
    const size_t n = (size_t)rows * cols;
    const int px = tv_px(n);
    for (int r = 0; r < px; ++r) {
        const size_t p = ((size_t)bx * px + r) * 256 + threadIdx.x;
        if (p < n) {
            const int i = (int)(p / cols), j = (int)(p - (size_t)i * cols);
            if (i < rows - 1 && j < cols - 1) tv_terms<TVJ>(y, tb, cols, p, lam_r, TVJ, acc);
        }
    }
    __shared__ double redn[4 * (TVJ + 1)];
    block_sum_n<TVJ + 1>(acc, redn);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q <= TVJ; ++q) tpart[(size_t)bx * (TVJ + 1) + q] = acc[q];
    }
}

__global__ __launch_bounds__(256) void k_tv_trials(int rows, int cols, const double* __restrict__ y,
                                                   const float* __restrict__ tb,
                                                   const double* __restrict__ gpart, int ngpart,
                                                   const Scalars* __restrict__ sc,
                                                   double* __restrict__ tpart,
                                                   const int* __restrict__ halt) {
    if (halt && *halt) return;
    tv_trials_body(rows, cols, y, tb, gpart, ngpart, sc, tpart, blockIdx.x);
}

void launch_tv_trials(hipStream_t st, int rows, int cols, const double* y, const float* tb,
                      const double* gpart, int ngpart, Scalars* sc, int J, double* tpart,
                      const int* halt) {
    (void)J;
    hipLaunchKernelGGL(k_tv_trials, dim3(tv_tpx_blocks(rows, cols)), dim3(256), 0, st, rows, cols, y, tb,
                       gpart, ngpart, sc, tpart, halt);
}

// One workgroup evaluates TV(y) and TV(y + lam_q t_bar), q < nq, over the whole
// image (the rare path of k_tv_decide).  out[0] = TV(y), out[1 + q] = trials.
__device__ void tv_trials_wg(const double* __restrict__ y, const float* __restrict__ tb, int rows,
                             int cols, const double* lam, int nq, double* out, double* red) {
    double acc[TVJ + 1];
#pragma unroll
    for (int q = 0; q <= TVJ; ++q) acc[q] = 0.0;
    const size_t n = (size_t)rows * cols;
    for (size_t p = threadIdx.x; p < n; p += 256) {
        const int i = (int)(p / cols), j = (int)(p - (size_t)i * cols);
        if (i < rows - 1 && j < cols - 1) tv_terms<TVJ>(y, tb, cols, p, lam, nq, acc);
    }
    __shared__ double redn[4 * (TVJ + 1)];
    (void)red;
    block_sum_n<TVJ + 1>(acc, redn);
    if (threadIdx.x == 0) {
        for (int q = 0; q <= TVJ; ++q) out[q] = acc[q];
    }
    __syncthreads();
}

__device__ __forceinline__ void tv_decide_body(int rows, int cols, const double* __restrict__ y,
                                               const float* __restrict__ tb,
                                               const double* __restrict__ gpart, int ngpart,
                                               const double* __restrict__ tpart, int ntpart,
                                               Scalars* __restrict__ sc, const TraceDev& tr,
                                               int32_t* __restrict__ trials_out) {
    __shared__ double red[4];
    __shared__ double tv[TVJ + 1];
    __shared__ double lam[TVJ];
    __shared__ int chosen_s;
    __shared__ double tvc_s;
    const double tn = sqrt(reduce_partials(gpart, ngpart, red));
    {
        // per q, thread t adds entries t, t+256, ... in order (the q's interleaved)
        double v[TVJ + 1];
#pragma unroll
        for (int q = 0; q <= TVJ; ++q) v[q] = 0.0;
        for (int bidx = threadIdx.x; bidx < ntpart; bidx += 256) {
            const double* row = tpart + (size_t)bidx * (TVJ + 1);
#pragma unroll
            for (int q = 0; q <= TVJ; ++q) v[q] += row[q];
        }
        __shared__ double redn[4 * (TVJ + 1)];
        block_sum_n<TVJ + 1>(v, redn);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int q = 0; q <= TVJ; ++q) tv[q] = v[q];
        }
    }
    __syncthreads();
    const int max_trials = sc->max_trials;
    if (threadIdx.x == 0) {
        chosen_s = -1;
        tvc_s = tv[0];
        if (sc->replay) {
            const int want = tr.replay[(size_t)sc->iter * sc->K + sc->inner];
            if (want >= 1 && want <= max_trials) {
                chosen_s = want;
                tvc_s = want <= TVJ ? tv[want] : -1.0;   // -1: evaluate below
            }
        } else {
            const int first = max_trials < TVJ ? max_trials : TVJ;
            for (int q = 0; q < first; ++q) {
                if (tv[q + 1] <= tv[0]) {
                    chosen_s = q + 1;
                    tvc_s = tv[q + 1];
                    break;
                }
            }
        }
    }
    __syncthreads();
    // Rare path: more trials than the first batch, evaluated by this workgroup.
    if (!sc->replay && chosen_s < 0 && max_trials > TVJ) {
        __shared__ double out[TVJ + 1];
        for (int start = TVJ; start < max_trials && chosen_s < 0; start += TVJ) {
            const int nq = min(TVJ, max_trials - start);
            if (threadIdx.x < TVJ)
                lam[threadIdx.x] = (int)threadIdx.x < nq ? trial_lambda(sc, start + threadIdx.x, tn) : 0.0;
            __syncthreads();
            tv_trials_wg(y, tb, rows, cols, lam, nq, out, red);
            if (threadIdx.x == 0) {
                for (int q = 0; q < nq; ++q) {
                    if (out[q + 1] <= out[0]) {
                        chosen_s = start + q + 1;
                        tvc_s = out[q + 1];
                        break;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (sc->replay && chosen_s > TVJ) {
        __shared__ double out[TVJ + 1];
        if (threadIdx.x == 0) lam[0] = trial_lambda(sc, chosen_s - 1, tn);
        __syncthreads();
        tv_trials_wg(y, tb, rows, cols, lam, 1, out, red);
        if (threadIdx.x == 0) tvc_s = out[1];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int chosen = chosen_s;
        const int ell0 = sc->ell;
        const int slot = sc->inner;
        int used;
        if (chosen > 0) {
            sc->lam = trial_lambda(sc, chosen - 1, tn);
            sc->ell = ell0 + chosen;
            sc->tv_new = tvc_s;
            used = chosen;
        } else {
            sc->lam = 0.0;
            sc->ell = ell0 + max_trials;
            sc->tv_new = tv[0];
            sc->exhausted = 1;
            used = max_trials + 1;
        }
        if (trials_out) trials_out[slot] = used;
        if (tr.trials && sc->iter < tr.cap) tr.trials[(size_t)sc->iter * sc->K + slot] = used;
        if (slot == sc->K - 1 && sc->iter < tr.cap) {
            if (tr.ell) tr.ell[sc->iter] = sc->ell;
            if (tr.tv_half) tr.tv_half[sc->iter] = sc->tv_new;
        }
        sc->inner = slot + 1;
    }
}

__global__ __launch_bounds__(256) void k_tv_decide(int rows, int cols, const double* __restrict__ y,
                                                   const float* __restrict__ tb,
                                                   const double* __restrict__ gpart, int ngpart,
                                                   const double* __restrict__ tpart, int ntpart,
                                                   Scalars* __restrict__ sc, TraceDev tr,
                                                   int32_t* __restrict__ trials_out,
                                                   const int* __restrict__ halt) {
    if (halt && *halt) return;
    tv_decide_body(rows, cols, y, tb, gpart, ngpart, tpart, ntpart, sc, tr, trials_out);
}

void launch_tv_decide(hipStream_t st, int rows, int cols, const double* y, const float* tb,
                      const double* gpart, int ngpart, const double* tpart, int ntpart, int J,
                      Scalars* sc, TraceDev tr, int32_t* trials_out, const int* halt) {
    (void)J;
    hipLaunchKernelGGL(k_tv_decide, dim3(1), dim3(256), 0, st, rows, cols, y, tb, gpart, ngpart,
                       tpart, ntpart, sc, tr, trials_out, halt);
}

__device__ __forceinline__ void tv_apply_body(int n, const double* __restrict__ src,
                                              double* __restrict__ dst, const float* __restrict__ tb,
                                              const Scalars* __restrict__ sc,
                                              const double* __restrict__ xk,
                                              double* __restrict__ partials, int bx) {
    __shared__ double red[4];
    const double lam = sc->lam;
    const int p = bx * 256 + threadIdx.x;
    double s2 = 0.0;
    if (p < n) {
        const double v = fma(lam, (double)tb[p], src[p]);
        dst[p] = v;
        if (xk) {
            const double s = v - xk[p];
            s2 = s * s;
        }
    }
    if (xk) {
        const double tot = block_sum(s2, red);
        if (threadIdx.x == 0) partials[bx] = tot;
    }
}

__global__ __launch_bounds__(256) void k_tv_apply(int n, const double* __restrict__ src,
                                                  double* __restrict__ dst,
                                                  const float* __restrict__ tb,
                                                  const Scalars* __restrict__ sc,
                                                  const double* __restrict__ xk,
                                                  double* __restrict__ partials,
                                                  const int* __restrict__ halt) {
    if (halt && *halt) return;
    tv_apply_body(n, src, dst, tb, sc, xk, partials, blockIdx.x);
}

void launch_tv_apply(hipStream_t st, int n, const double* src, double* dst, const float* tb,
                     const Scalars* sc, const double* xk, double* partials, const int* halt) {
    hipLaunchKernelGGL(k_tv_apply, dim3((n + 255) / 256), dim3(256), 0, st, n, src, dst, tb, sc, xk,
                       partials, halt);
}

// S_TV's last update written also to R's padded copies: for the 32 x 32 tile
// (bx, by), dst = src + lam t_bar (tb != nullptr; as k_tv_apply) or dst = src
// (tb == nullptr: the K = 0 copy), the padded copy xp and the padded
// transposed copy xTp of dst (as R's prep), and with xk the tile's sum of
// (dst - xk)^2 in partials[by * tiles_x + bx].  dst may alias src.
__device__ __forceinline__ void tv_apply_prep_body(const GeomDev& G, const double* src, double* dst,
                                                   const float* __restrict__ tb,
                                                   const Scalars* __restrict__ sc,
                                                   const double* __restrict__ xk,
                                                   double* __restrict__ partials,
                                                   double* __restrict__ xp, double* __restrict__ xTp,
                                                   int bx, int by) {
    __shared__ double tile[32][33];
    __shared__ double red[4];
    const double lam = tb ? sc->lam : 0.0;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int j = bx * 32 + tx;
    double s2 = 0.0;
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int i = by * 32 + ty + r;
        double v = 0.0;
        if (i < G.rows && j < G.cols) {
            const size_t p = (size_t)i * G.cols + j;
            v = tb ? fma(lam, (double)tb[p], src[p]) : src[p];
            dst[p] = v;
            xp[(size_t)i * G.pitchX + PAD + j] = v;
            if (xk) {
                const double d = v - xk[p];
                s2 += d * d;
            }
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
    if (xk) {
        const double tot = block_sum(s2, red);
        if (threadIdx.x == 0) partials[by * ((G.cols + 31) / 32) + bx] = tot;
    }
}

__global__ __launch_bounds__(256) void k_tv_apply_prep(GeomDev G, const double* src, double* dst,
                                                       const float* __restrict__ tb,
                                                       const Scalars* __restrict__ sc,
                                                       const double* __restrict__ xk,
                                                       double* __restrict__ partials,
                                                       double* __restrict__ xp,
                                                       double* __restrict__ xTp,
                                                       const int* __restrict__ halt) {
    if (halt && *halt) return;
    tv_apply_prep_body(G, src, dst, tb, sc, xk, partials, xp, xTp, blockIdx.x, blockIdx.y);
}

int tv_prep_tiles(int rows, int cols) { return ((cols + 31) / 32) * ((rows + 31) / 32); }

void launch_tv_apply_prep(hipStream_t st, const GeomDev& G, const double* src, double* dst,
                          const float* tb, const Scalars* sc, const double* xk, double* partials,
                          double* xp, double* xTp, const int* halt) {
    dim3 grid((G.cols + 31) / 32, (G.rows + 31) / 32);
    hipLaunchKernelGGL(k_tv_apply_prep, grid, dim3(256), 0, st, G, src, dst, tb, sc, xk, partials, xp,
                       xTp, halt);
}

// One S_TV inner step's update followed by the next step's gradient, in one
// launch: dst = src + lam tb_in (as k_tv_apply) and tb_out = t_bar(dst) with
// the partials of ||tb_out||^2 (as k_tv_grad).  A thread forms dst at its
// pixel and at the neighbours its t_bar reads, with the same fma, so the
// values are those of the two launches bit for bit; dst and src (and tb_in
// and tb_out) must not overlap.
__global__ __launch_bounds__(256) void k_tv_apply_grad(int rows, int cols, const double* __restrict__ src,
                                                       double* __restrict__ dst,
                                                       const float* __restrict__ tb_in,
                                                       float* __restrict__ tb_out,
                                                       const Scalars* __restrict__ sc,
                                                       double* __restrict__ partials,
                                                       const int* __restrict__ halt) {
    if (halt && *halt) return;
    __shared__ double red[4];
    const double lam = sc->lam;
    const size_t n = (size_t)rows * cols;
    auto y = [&](size_t q) { return fma(lam, (double)tb_in[q], src[q]); };
    double sq = 0.0;
    const int px = tv_px(n);
    for (int r = 0; r < px; ++r) {   // the pixels and partial layout of a later k_tv_grad
        const size_t p = ((size_t)blockIdx.x * px + r) * 256 + threadIdx.x;
        if (p < n) {
            dst[p] = y(p);
            const int i = (int)(p / cols), j = (int)(p - (size_t)i * cols);
            const float t = tv_neg_grad_at(y, rows, cols, i, j, p);
            tb_out[p] = t;
            sq += (double)t * (double)t;
        }
    }
    const double tot = block_sum(sq, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

void launch_tv_apply_grad(hipStream_t st, int rows, int cols, const double* src, double* dst,
                          const float* tb_in, float* tb_out, const Scalars* sc, double* partials,
                          const int* halt) {
    hipLaunchKernelGGL(k_tv_apply_grad, dim3(tv_grad_blocks(rows, cols)), dim3(256), 0, st, rows, cols, src, dst,
                       tb_in, tb_out, sc, partials, halt);
}

__global__ __launch_bounds__(256) void k_tv_value(int rows, int cols, const double* __restrict__ y,
                                                  double* __restrict__ partials,
                                                  const int* __restrict__ halt) {
    if (halt && *halt) return;
    __shared__ double red[4];
    const size_t n = (size_t)rows * cols;
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    double acc = 0.0;
    if (p < n) {
        const int i = (int)(p / cols), j = (int)(p - (size_t)i * cols);
        if (i < rows - 1 && j < cols - 1) {
            const double dv = y[p] - y[p + cols];
            const double dh = y[p] - y[p + 1];
            acc = sqrt(dv * dv + dh * dh);
        }
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

void launch_tv_value(hipStream_t st, int rows, int cols, const double* y, double* partials,
                     const int* halt) {
    hipLaunchKernelGGL(k_tv_value, dim3(tv_blocks(rows, cols)), dim3(256), 0, st, rows, cols, y,
                       partials, halt);
}

// ---- batched S_TV inner step: src selects x (first inner step) or x_half ----
__global__ __launch_bounds__(256) void kb_tv_grad(const SliceDev* __restrict__ sl, ItemTable t, int src) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        tv_grad_body(S.G.rows, S.G.cols, batch_vec(S, src), gmem(S.tb), gmem(S.ptg), lin,
                     src == BV_X ? 1 : tv_px((size_t)S.n));   // the first inner step reads x
    });
}

__global__ __launch_bounds__(256) void kb_tv_trials(const SliceDev* __restrict__ sl, ItemTable t, int src) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        tv_trials_body(S.G.rows, S.G.cols, batch_vec(S, src), gmem(S.tb), gmem(S.ptg), src == BV_X ? S.ntv : S.ntg,
                       gmem(S.sc), gmem(S.ptt), lin);
    });
}

__global__ __launch_bounds__(256) void kb_tv_decide(const SliceDev* __restrict__ sl, ItemTable t, int src) {
    for_items(t, [&](int s, int) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const TraceDev tr = S.tr;
        tv_decide_body(S.G.rows, S.G.cols, batch_vec(S, src), gmem(S.tb), gmem(S.ptg), src == BV_X ? S.ntv : S.ntg,
                       gmem(S.ptt), S.ntt, gmem(S.sc), tr, nullptr);
    });
}

__global__ __launch_bounds__(256) void kb_tv_apply(const SliceDev* __restrict__ sl, ItemTable t, int src,
                                                   int snorm) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        tv_apply_body(S.n, batch_vec(S, src), gmem(S.xh), gmem(S.tb), gmem(S.sc),
                      snorm ? gmem(S.x) : nullptr, gmem(S.pts), lin);
    });
}

// BS_PREP items: the last update (tb: t_bar; else the K = 0 copy of x) with
// R's padded copies, and with snorm the ||x_{k+1/2} - x_k||^2 tile partials.
__global__ __launch_bounds__(256) void kb_tv_apply_prep(const SliceDev* __restrict__ sl, ItemTable t,
                                                        int src, int copy, int snorm) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const GeomDev G = S.G;
        const int gx = (G.cols + 31) / 32;
        tv_apply_prep_body(G, batch_vec(S, src), gmem(S.xh), copy ? nullptr : gmem(S.tb), gmem(S.sc),
                           snorm ? gmem(S.x) : nullptr, gmem(S.pts), gmem(S.xp), gmem(S.xTp), lin % gx,
                           lin / gx);
    });
}

void launch_tv_apply_prep_b(hipStream_t st, const SliceDev* sl, ItemTable t, int src, bool copy,
                            bool snorm) {
    hipLaunchKernelGGL(kb_tv_apply_prep, dim3(t.grid), dim3(256), 0, st, sl, t, src, copy ? 1 : 0,
                       snorm ? 1 : 0);
}

void launch_tv_grad_b(hipStream_t st, const SliceDev* sl, ItemTable t, int src) {
    hipLaunchKernelGGL(kb_tv_grad, dim3(t.grid), dim3(256), 0, st, sl, t, src);
}
void launch_tv_trials_b(hipStream_t st, const SliceDev* sl, ItemTable t, int src) {
    hipLaunchKernelGGL(kb_tv_trials, dim3(t.grid), dim3(256), 0, st, sl, t, src);
}
void launch_tv_decide_b(hipStream_t st, const SliceDev* sl, ItemTable t, int src) {
    hipLaunchKernelGGL(kb_tv_decide, dim3(t.grid), dim3(256), 0, st, sl, t, src);
}
void launch_tv_apply_b(hipStream_t st, const SliceDev* sl, ItemTable t, int src, bool snorm) {
    hipLaunchKernelGGL(kb_tv_apply, dim3(t.grid), dim3(256), 0, st, sl, t, src, snorm ? 1 : 0);
}

}  // namespace sp
