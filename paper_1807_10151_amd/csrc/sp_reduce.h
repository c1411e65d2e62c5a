// Deterministic float64 reductions for 256-thread workgroups (4 wave64s), and
// block_sum_w for workgroups of other sizes.
#pragma once

#include <hip/hip_runtime.h>

namespace sp {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup; the result is valid in every thread.  `lds` must
// hold 4 doubles.  Fixed reduction order: lanes by xor-butterfly, then waves
// 0..3 in order.
__device__ __forceinline__ double block_sum(double v, double* lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    return ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// Sum over a workgroup of NW waves (64 NW threads); the result is valid in
// every thread.  `lds` must hold NW doubles.  Fixed order: lanes by
// xor-butterfly, then waves 0..NW-1 in order.
template <int NW>
__device__ __forceinline__ double block_sum_w(double v, double* lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = lds[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) s += lds[i];
    return s;
}

// N independent block sums with one pair of barriers: v[i] becomes exactly
// block_sum(v[i]) (same lane butterfly, same wave order) in every thread.
// `lds` must hold 4 * N doubles.
template <int N>
__device__ __forceinline__ void block_sum_n(double* v, double* lds) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) lds[w * N + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = ((lds[i] + lds[N + i]) + lds[2 * N + i]) + lds[3 * N + i];
}

// Sums `np` partials in a fixed order with one workgroup: thread t adds
// entries t, t+256, ... in that order; then block_sum.  Every thread gets the
// result.  Eight loads are issued before their adds so that one memory
// latency covers them (the order of the additions is unchanged).
__device__ __forceinline__ double reduce_partials(const double* p, int np, double* lds) {
    double v = 0.0;
    int q = threadIdx.x;
    for (; q + 7 * 256 < np; q += 8 * 256) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = p[q + u * 256];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += a[u];
    }
    for (; q < np; q += 256) v += p[q];
    return block_sum(v, lds);
}

}  // namespace sp
