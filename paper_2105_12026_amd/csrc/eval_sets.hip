// f(S_j) for many CSR-packed sets at once (Sec. 4.1: optimisers score a whole
// family S_multi = {S_1..S_l} per step; Alg. 1 gives f per set as a running
// minimum per ground point, a sum, and a division by |V|).
//
// A workgroup owns kSetsPerBlock sets and streams every ground point v once:
// each thread keeps, per owned set, the float64 running sum of
//     ||v||^2 - min(||v||^2, min_{s in S_j} d(v, s))
// (the e0 = 0 term of S_j u {e0} is the ||v||^2 start value), so
//     f(S_j) = |V|^-1 sum_v that term  = L({e0}) - L(S_j u {e0}).
// Distances are float32 direct differences; the per-point term and every sum
// are float64; the block sum runs in a fixed tree order.
#include <math.h>

#include "ebc_internal.h"

namespace ebc {

constexpr int kSetsPerBlock = 4;

__global__ void __launch_bounds__(kBlock)
k_eval_sets(const float* __restrict__ x, int64_t n, int32_t d, const double* __restrict__ n64,
            const int64_t* __restrict__ off, const int32_t* __restrict__ idx, int64_t l,
            double* __restrict__ f_out, DevState* st) {
    __shared__ double red[kSetsPerBlock][kBlock];
    __shared__ int s_bad[kSetsPerBlock];
    const int64_t j0 = int64_t(blockIdx.x) * kSetsPerBlock;
    if (threadIdx.x < kSetsPerBlock) {
        const int64_t j = j0 + threadIdx.x;
        int bad = 0;
        if (j < l) {
            const int64_t a = off[j], z = off[j + 1];
            if (a < 0 || z < a || z > off[l]) bad = 1;
            else
                for (int64_t q = a; q < z; ++q)
                    if (idx[q] < 0 || int64_t(idx[q]) >= n) { bad = 1; break; }
        }
        s_bad[threadIdx.x] = bad;
        if (bad) atomicCAS(&st->error, 0, kDevErrIndex);
    }
    __syncthreads();
    int64_t beg[kSetsPerBlock], end[kSetsPerBlock];
#pragma unroll
    for (int s = 0; s < kSetsPerBlock; ++s) {
        const int64_t j = j0 + s;
        const bool ok = j < l && !s_bad[s];
        beg[s] = ok ? off[j] : 0;
        end[s] = ok ? off[j + 1] : 0;
    }
    double acc[kSetsPerBlock];
#pragma unroll
    for (int s = 0; s < kSetsPerBlock; ++s) acc[s] = 0.0;
    for (int64_t v = threadIdx.x; v < n; v += kBlock) {
        const float* xv = x + v * d;
        const double nv = n64[v];
#pragma unroll
        for (int s = 0; s < kSetsPerBlock; ++s) {
            float dmin = INFINITY;
            for (int64_t q = beg[s]; q < end[s]; ++q) {
                const float* xs = x + int64_t(idx[q]) * d;
                float t = 0.0f;
                for (int k = 0; k < d; ++k) {
                    const float u = xv[k] - xs[k];
                    t = fmaf(u, u, t);
                }
                dmin = fminf(dmin, t);
            }
            const double m = fmin(nv, double(dmin));
            acc[s] += nv - m;
        }
    }
#pragma unroll
    for (int s = 0; s < kSetsPerBlock; ++s) red[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int s = 0; s < kSetsPerBlock; ++s) red[s][threadIdx.x] += red[s][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < kSetsPerBlock) {
        const int64_t j = j0 + threadIdx.x;
        if (j < l) f_out[j] = s_bad[threadIdx.x] ? NAN : red[threadIdx.x][0] / double(n);
    }
}

hipError_t launch_eval_sets(const ebc_dataset* ds, const int64_t* offsets, const int32_t* idx, int64_t l,
                            double* f_out, hipStream_t s) {
    const int64_t nb = (l + kSetsPerBlock - 1) / kSetsPerBlock;
    hipLaunchKernelGGL(k_eval_sets, dim3(unsigned(nb)), dim3(kBlock), 0, s, ds->x, ds->n, ds->d, ds->b.n64,
                       offsets, idx, l, f_out, ds->b.state);
    return hipGetLastError();
}

}  // namespace ebc
