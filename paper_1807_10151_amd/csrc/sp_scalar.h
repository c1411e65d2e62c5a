// The float64 scalar steps of the solvers (f, beta, alpha, the S_TV step norm
// and the learned-preconditioner check), evaluated by one workgroup from the
// per-workgroup partial sums.  Shared by the single-workgroup scalar kernel,
// the kernels that fold a scalar step into their own launch, and the batched
// forms, so every path computes the same values.
#pragma once

#include "sp_internal.h"
#include "sp_reduce.h"
#include "../../include/suppcg.h"

namespace sp {

__device__ __forceinline__ bool finite(double v) { return v == v && v - v == 0.0; }

// Algorithm 2: beta = z^T h / p^T h from the sum A of z^T h (0 on the first
// direction, which has no previous p).
__device__ __forceinline__ double beta_from(const Scalars* __restrict__ sc, double A) {
    return sc->first ? 0.0 : A / sc->pth;
}

// Algorithm 2: alpha = -g^T p / p^T h.  Returns the halt code the step sets:
// breakdown when p^T h = 0, non-finite values; 0 to go on (x is then
// updated).  Algorithm 3's termination test is not taken here: it belongs to
// the top of the next loop body (OP_EPS), after x_{k+1} has been formed.
__device__ __forceinline__ int alpha_from(double pth, double gp, double& alpha) {
    int code = 0;
    alpha = 0.0;
    if (pth == 0.0) {
        code = SP_BREAKDOWN_CONVERGED;
    } else {
        alpha = -gp / pth;
        if (!finite(alpha) || !finite(pth)) code = SP_ERR_NONFINITE;
    }
    return code;
}

// Thread 0's part of scalar step `op` with the reduced sums A and B.
__device__ __forceinline__ void scalar_commit(int op, Scalars* __restrict__ sc, const TraceDev& tr,
                                              double A, double B) {
    const int it = sc->iter;
    const bool rec = it < tr.cap;
    switch (op) {
    case OP_F0:
        sc->f = A;
        sc->f0 = A;
        if (!finite(A)) sc->halt = SP_ERR_NONFINITE;
        break;
    case OP_F:
        sc->f = A;
        if (rec && tr.f_half) tr.f_half[it] = A;
        if (!finite(A)) sc->halt = SP_ERR_NONFINITE;
        break;
    case OP_BETA: {
        const double beta = beta_from(sc, A);
        sc->beta = beta;
        if (!sc->first && rec && tr.beta) tr.beta[it] = beta;
        if (!finite(beta)) sc->halt = SP_ERR_NONFINITE;
        break;
    }
    case OP_ALPHA0:
    case OP_ALPHA: {
        double alpha;
        const int code = alpha_from(A, B, alpha);
        sc->alpha = alpha;
        sc->pth = A;
        if (op == OP_ALPHA0) {
            sc->alpha0 = alpha;
            sc->k = 1;
            sc->first = 0;
        } else {
            if (rec && tr.alpha) tr.alpha[it] = alpha;
            sc->iter = it + 1;
            sc->k = sc->k + 1;
        }
        sc->inner = 0;
        if (code) sc->halt = code;
        break;
    }
    case OP_SNORM:
        if (rec && tr.s_norm) tr.s_norm[it] = sqrt(A);
        break;
    case OP_NEXT:
        sc->iter = it + 1;
        sc->k = sc->k + 1;
        sc->inner = 0;
        break;
    case OP_EPS:   // Algorithm 3, step 10: stop when f(x_{k-1/2}) <= eps
        if (sc->eps > 0.0 && !(sc->f > sc->eps)) sc->halt = SP_CONVERGED;
        break;
    case OP_LCHECK:
        if (sc->gate_learned && !(A > 0.0 && finite(A))) {
            sc->gate_learned = 0;
            sc->gate_ramp = 1;
            sc->fallbacks += 1;
        }
        break;
    default:
        break;
    }
}

// Scalar step `op` by the whole workgroup: A = sum(pa), B = sum(pb) in fixed
// order (nullptr: 0), then thread 0 commits.
__device__ __forceinline__ void scalar_body(int op, Scalars* __restrict__ sc, const TraceDev& tr,
                                            const double* __restrict__ pa, int na,
                                            const double* __restrict__ pb, int nb) {
    __shared__ double red[4];
    const double A = pa ? reduce_partials(pa, na, red) : 0.0;
    const double B = pb ? reduce_partials(pb, nb, red) : 0.0;
    if (threadIdx.x == 0) scalar_commit(op, sc, tr, A, B);
}

}  // namespace sp
