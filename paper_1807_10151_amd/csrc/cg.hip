// Conjugate-gradient vector updates and the float64 scalar recurrence of
// Algorithm 2 (U_PCG):  beta = z^T h / p^T h,  p <- -z + beta p,
// alpha = -g^T p / p^T h,  x <- x + alpha p.
//
// h = A p = R^T R p enters Algorithm 2 only through the two dot products
// z^T h = (R z)^T (R p) and p^T h = ||R p||^2, so the solvers never form it:
// they keep q = R p (nA x nB rays, float64) by the direction's own recurrence
// q <- -R z + beta q, which costs one projection of z per loop body in place
// of a projection and a backprojection of p.
//
// The iterate x, x_{k+1/2}, the direction p and q are float64 vectors; g and z
// are float32.  Dot products are float64 partial sums per workgroup (fixed
// order); a single
// workgroup (k_scalar) sums them and updates the device-resident scalars, so a
// loop body needs no host synchronisation and can be captured in a graph.
#include "sp_internal.h"
#include "sp_reduce.h"
#include "sp_scalar.h"
#include "../../include/suppcg.h"

namespace sp {

int vec_blocks(int n) {
    const int b = (n + 255) / 256;
    return b < 2048 ? b : 2048;
}

__device__ __forceinline__ int vec_blocks_dev(int n) {
    const int b = (n + 255) / 256;
    return b < 2048 ? b : 2048;
}

__global__ __launch_bounds__(256) void k_dot(int n, const float* __restrict__ a,
                                             const float* __restrict__ b,
                                             double* __restrict__ partials,
                                             const int* __restrict__ halt) {
    if (halt && *halt) return;
    __shared__ double red[4];
    double acc = 0.0;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < n; p += gridDim.x * 256)
        acc += (double)a[p] * (double)b[p];
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

void launch_dot(hipStream_t st, int n, const float* a, const float* b, double* partials,
                const int* halt) {
    hipLaunchKernelGGL(k_dot, dim3(vec_blocks(n)), dim3(256), 0, st, n, a, b, partials, halt);
}

// Virtual block bx of vec_blocks(max(n, m)):
//   bx < vec_blocks(n): p <- -z + beta p over its grid-stride share of the n
//     pixels, with the partial of g^T p (new p) in pgp[bx];
//   bx < vec_blocks(m): q <- -w + beta q over its share of the m rays
//     (w = R z, q = R p), with the partial of q^T q in pqq[bx].
// The first direction (no previous p) is p = -z, q = -w.
__device__ __forceinline__ void update_pq_body(int n, int m, const float* __restrict__ z,
                                               double* __restrict__ p, const float* __restrict__ g,
                                               const double* __restrict__ w,
                                               double* __restrict__ q, double beta, bool first,
                                               double* __restrict__ pgp, double* __restrict__ pqq,
                                               int bx) {
    __shared__ double red[4];
    const int gp = vec_blocks_dev(n), gq = vec_blocks_dev(m);
    if (bx < gp) {
        double acc = 0.0;
        for (int i = bx * 256 + threadIdx.x; i < n; i += gp * 256) {
            const double v = first ? -(double)z[i] : fma(beta, p[i], -(double)z[i]);
            p[i] = v;
            acc += (double)g[i] * v;
        }
        const double tot = block_sum(acc, red);
        if (threadIdx.x == 0) pgp[bx] = tot;
    }
    if (bx < gq) {
        double acc = 0.0;
        for (int i = bx * 256 + threadIdx.x; i < m; i += gq * 256) {
            const double v = first ? -w[i] : fma(beta, q[i], -w[i]);
            q[i] = v;
            acc += v * v;
        }
        const double tot = block_sum(acc, red);
        if (threadIdx.x == 0) pqq[bx] = tot;
    }
}

int pq_blocks(int n, int m) { return vec_blocks(n > m ? n : m); }

// The beta step folded into the update: every workgroup sums the (R z)^T q
// partials (pdot) in the same fixed order, so all use the beta that workgroup
// 0 commits to the scalars (and trace).  A non-finite beta halts without an
// update, as the separate scalar step would.
__global__ __launch_bounds__(256) void k_update_pq_beta(int n, int m, const float* __restrict__ z,
                                                        double* __restrict__ p,
                                                        const float* __restrict__ g,
                                                        const double* __restrict__ w,
                                                        double* __restrict__ q,
                                                        Scalars* __restrict__ sc, TraceDev tr,
                                                        const double* __restrict__ pdot, int ndot,
                                                        double* __restrict__ pgp,
                                                        double* __restrict__ pqq) {
    if (sc->halt) return;
    __shared__ double red[4];
    const double A = reduce_partials(pdot, ndot, red);
    const double beta = beta_from(sc, A);
    const bool first = sc->first != 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) scalar_commit(OP_BETA, sc, tr, A, 0.0);
    if (!finite(beta)) return;
    update_pq_body(n, m, z, p, g, w, q, beta, first, pgp, pqq, blockIdx.x);
}

void launch_update_pq_beta(hipStream_t st, int n, int m, const float* z, double* p, const float* g,
                           const double* w, double* q, Scalars* sc, TraceDev tr, const double* pdot,
                           int ndot, double* pgp, double* pqq) {
    hipLaunchKernelGGL(k_update_pq_beta, dim3(pq_blocks(n, m)), dim3(256), 0, st, n, m, z, p, g, w, q,
                       sc, tr, pdot, ndot, pgp, pqq);
}

// x <- xh + alpha p
__device__ __forceinline__ void update_x_body(int n, const double* __restrict__ xh,
                                              const double* __restrict__ p, double* __restrict__ x,
                                              double alpha, int bx, int gx) {
    for (int q = bx * 256 + threadIdx.x; q < n; q += gx * 256)
        x[q] = fma(alpha, p[q], xh[q]);
}

// The alpha step (op OP_ALPHA or OP_ALPHA0) folded into the update: every
// workgroup sums the p^T h (= q^T q) and g^T p partials in the same order and takes the
// same halt decision (breakdown, non-finite) that workgroup 0 commits; on a
// halt no workgroup updates x.  (Workgroups that start after workgroup 0 has
// committed a halt return at the entry check; they would not have updated x
// either.)
__global__ __launch_bounds__(256) void k_update_x_alpha(int n, const double* __restrict__ xh,
                                                        const double* __restrict__ p,
                                                        double* __restrict__ x,
                                                        Scalars* __restrict__ sc, TraceDev tr,
                                                        const double* __restrict__ pph, int nph,
                                                        const double* __restrict__ pgp, int ngp,
                                                        int op) {
    if (sc->halt) return;
    __shared__ double red[4];
    const double pth = reduce_partials(pph, nph, red);
    const double gp = reduce_partials(pgp, ngp, red);
    double alpha;
    const int code = alpha_from(pth, gp, alpha);
    if (blockIdx.x == 0 && threadIdx.x == 0) scalar_commit(op, sc, tr, pth, gp);
    if (code) return;
    update_x_body(n, xh, p, x, alpha, blockIdx.x, gridDim.x);
}

void launch_update_x_alpha(hipStream_t st, int n, const double* xh, const double* p, double* x,
                           Scalars* sc, TraceDev tr, const double* pph, int nph, const double* pgp,
                           int ngp, int op) {
    hipLaunchKernelGGL(k_update_x_alpha, dim3(vec_blocks(n)), dim3(256), 0, st, n, xh, p, x, sc,
                       tr, pph, nph, pgp, ngp, op);
}

template <class T>
__global__ __launch_bounds__(256) void k_copy(int n, const T* __restrict__ src, T* __restrict__ dst,
                                              const int* __restrict__ halt) {
    if (halt && *halt) return;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < n; q += gridDim.x * 256) dst[q] = src[q];
}

void launch_copy(hipStream_t st, int n, const float* src, float* dst, const int* halt) {
    hipLaunchKernelGGL(k_copy<float>, dim3(vec_blocks(n)), dim3(256), 0, st, n, src, dst, halt);
}

void launch_copy(hipStream_t st, int n, const double* src, double* dst, const int* halt) {
    hipLaunchKernelGGL(k_copy<double>, dim3(vec_blocks(n)), dim3(256), 0, st, n, src, dst, halt);
}

__global__ __launch_bounds__(256) void k_widen(int n, const float* __restrict__ src,
                                               double* __restrict__ dst) {
    for (int q = blockIdx.x * 256 + threadIdx.x; q < n; q += gridDim.x * 256)
        dst[q] = src ? (double)src[q] : 0.0;
}

void launch_widen(hipStream_t st, int n, const float* src, double* dst) {
    hipLaunchKernelGGL(k_widen, dim3(vec_blocks(n)), dim3(256), 0, st, n, src, dst);
}

__global__ __launch_bounds__(256) void k_narrow(int n, const double* __restrict__ src,
                                                float* __restrict__ dst) {
    for (int q = blockIdx.x * 256 + threadIdx.x; q < n; q += gridDim.x * 256) dst[q] = (float)src[q];
}

void launch_narrow(hipStream_t st, int n, const double* src, float* dst) {
    hipLaunchKernelGGL(k_narrow, dim3(vec_blocks(n)), dim3(256), 0, st, n, src, dst);
}

// dst[iter][:] = src for the loop body index iter held in the scalars, while
// iter < count.
__global__ __launch_bounds__(256) void k_snap(int n, const float* __restrict__ src,
                                              float* __restrict__ dst, int count,
                                              const Scalars* __restrict__ sc) {
    if (sc->halt) return;
    const int it = sc->iter;
    if (it < 0 || it >= count) return;
    float* d = dst + (size_t)it * n;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < n; q += gridDim.x * 256) d[q] = src[q];
}

void launch_snap(hipStream_t st, int n, const float* src, float* dst, int count, const Scalars* sc) {
    hipLaunchKernelGGL(k_snap, dim3(vec_blocks(n)), dim3(256), 0, st, n, src, dst, count, sc);
}

// End of a solve that does not return to the host in between: x_k = x_{k-1/2}
// when the run stopped on a breakdown after the initial step (the step could
// not be formed), and k to device memory (nullable).
__global__ __launch_bounds__(256) void k_finish(int n, const double* __restrict__ xh,
                                                double* __restrict__ x,
                                                const Scalars* __restrict__ sc,
                                                int32_t* __restrict__ k_out) {
    if (sc->halt == SP_BREAKDOWN_CONVERGED && sc->k > 1)
        for (int q = blockIdx.x * 256 + threadIdx.x; q < n; q += gridDim.x * 256) x[q] = xh[q];
    if (k_out && blockIdx.x == 0 && threadIdx.x == 0) *k_out = sc->k;
}

void launch_finish(hipStream_t st, int n, const double* xh, double* x, const Scalars* sc,
                   int32_t* k_out) {
    hipLaunchKernelGGL(k_finish, dim3(vec_blocks(n)), dim3(256), 0, st, n, xh, x, sc, k_out);
}

__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ partials, int np,
                                                double* __restrict__ out) {
    __shared__ double red[4];
    const double tot = reduce_partials(partials, np, red);
    if (threadIdx.x == 0) *out = tot;
}

void launch_reduce(hipStream_t st, const double* partials, int np, double* out) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, partials, np, out);
}

__global__ __launch_bounds__(256) void k_scalar(int op, Scalars* __restrict__ sc, TraceDev tr,
                                                const double* __restrict__ pa, int na,
                                                const double* __restrict__ pb, int nb) {
    if (sc->halt) return;
    scalar_body(op, sc, tr, pa, na, pb, nb);
}

void launch_scalar(hipStream_t st, int op, Scalars* sc, TraceDev tr, const double* pa, int na,
                   const double* pb, int nb) {
    hipLaunchKernelGGL(k_scalar, dim3(1), dim3(256), 0, st, op, sc, tr, pa, na, pb, nb);
}

// ---- batched forms (one item table entry per virtual block of each slice) ----
__global__ __launch_bounds__(256) void kb_init(const SliceDev* __restrict__ sl, ItemTable t) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        const int gx = vec_blocks_dev(S.n);
        for (int q = lin * 256 + threadIdx.x; q < S.n; q += gx * 256) {
            const double v = S.x0 ? (double)gmem(S.x0)[q] : 0.0;
            gmem(S.xh)[q] = v;
            gmem(S.x)[q] = v;
        }
    });
}

// The p and q updates with the beta that OP_BETA committed.
__global__ __launch_bounds__(256) void kb_update_pq(const SliceDev* __restrict__ sl, ItemTable t) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        const Scalars* sc = gmem(S.sc);
        if (sc->halt) return;
        update_pq_body(S.n, S.m, gmem(S.z), gmem(S.p), gmem(S.g), gmem(S.w), gmem(S.q), sc->beta,
                       sc->first != 0, gmem(S.pgp), gmem(S.pqq), lin);
    });
}

__global__ __launch_bounds__(256) void kb_update_x(const SliceDev* __restrict__ sl, ItemTable t) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        update_x_body(S.n, gmem(S.xh), gmem(S.p), gmem(S.x), gmem(S.sc)->alpha, lin,
                      vec_blocks_dev(S.n));
    });
}

// M = I: z = g.
__global__ __launch_bounds__(256) void kb_copy_gz(const SliceDev* __restrict__ sl, ItemTable t) {
    for_items(t, [&](int s, int lin) {
        const SliceDev& S = sl[s];
        if (gmem(S.sc)->halt) return;
        const int gx = vec_blocks_dev(S.n);
        const float* g = gmem(S.g);
        float* z = gmem(S.z);
        for (int q = lin * 256 + threadIdx.x; q < S.n; q += gx * 256) z[q] = g[q];
    });
}

__global__ __launch_bounds__(256) void kb_scalar(const SliceDev* __restrict__ sl, ItemTable t, int op) {
    for_items(t, [&](int s, int) {
        const SliceDev& S = sl[s];
        Scalars* sc = gmem(S.sc);
        if (sc->halt) return;
        const TraceDev tr = S.tr;
        switch (op) {
        case OP_F0:
        case OP_F: scalar_body(op, sc, tr, gmem(S.pf), S.nf, nullptr, 0); break;
        case OP_BETA: scalar_body(op, sc, tr, gmem(S.pf), S.nf, nullptr, 0); break;
        case OP_ALPHA0:
        case OP_ALPHA: scalar_body(op, sc, tr, gmem(S.pqq), S.nqq, gmem(S.pgp), S.ngp); break;
        case OP_SNORM: scalar_body(op, sc, tr, gmem(S.pts), S.nsn, nullptr, 0); break;
        case OP_EPS: scalar_body(op, sc, tr, nullptr, 0, nullptr, 0); break;
        default: break;
        }
    });
}

void launch_init_b(hipStream_t st, const SliceDev* sl, ItemTable t) {
    hipLaunchKernelGGL(kb_init, dim3(t.grid), dim3(256), 0, st, sl, t);
}
void launch_update_pq_b(hipStream_t st, const SliceDev* sl, ItemTable t) {
    hipLaunchKernelGGL(kb_update_pq, dim3(t.grid), dim3(256), 0, st, sl, t);
}
void launch_update_x_b(hipStream_t st, const SliceDev* sl, ItemTable t) {
    hipLaunchKernelGGL(kb_update_x, dim3(t.grid), dim3(256), 0, st, sl, t);
}
void launch_copy_gz_b(hipStream_t st, const SliceDev* sl, ItemTable t) {
    hipLaunchKernelGGL(kb_copy_gz, dim3(t.grid), dim3(256), 0, st, sl, t);
}
void launch_scalar_b(hipStream_t st, const SliceDev* sl, ItemTable t, int op) {
    hipLaunchKernelGGL(kb_scalar, dim3(t.grid), dim3(256), 0, st, sl, t, op);
}

}  // namespace sp
