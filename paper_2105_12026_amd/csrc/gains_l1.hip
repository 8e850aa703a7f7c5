// Marginal gains under the L1 (Manhattan) dissimilarity d(v,c) = sum_k |v_k - c_k|.
//
// Sec. 4 defines the k-medoids loss and f for any dissimilarity; the paper's
// experiments use the squared Euclidean distance, whose dot-product form runs
// on the matrix cores. The L1 distance has no such form: every (candidate,
// point, dimension) triple costs one subtraction and one absolute-value add
// on the vector ALUs, so this kernel is bound by plain FP32 issue, not by the
// matrix units or HBM.
//
//     G[c] = sum_v max(0, m_v - d(v, c))          (|V| * Delta(c|S), Sec. 3)
//
// Work decomposition: a workgroup (256 threads) owns 64 candidates and one
// chunk of the ground set, and walks the chunk in tiles of 128 points. Both
// the candidates' and the points' values are staged through LDS 32
// dimensions at a time (row-major, 36-float stride), the next stage's values
// loaded into registers while the current one is consumed. Thread (tc, tv)
// holds a 4 x 8 register tile: candidates tc + 16 i and points tv + 16 j,
// so that a wave's 16-byte LDS reads of one row index fall on distinct bank
// groups. Distances are float32 sums in dimension order; the clamped terms
// are added in float64 per thread, and the 16 threads of each candidate are
// added in a fixed order. Reads the caller's float32 rows directly.
#include "ebc_internal.h"

namespace ebc {

namespace {

constexpr int kL1Cand = 64;    // candidates per workgroup
constexpr int kL1VTile = 128;  // ground points per tile
constexpr int kL1K = 32;       // dimensions per LDS stage
constexpr int kL1S = kL1K + 4; // LDS row stride (floats)

// 4 consecutive values of row r from column k (zeros past d or for r < 0)
__device__ __forceinline__ float4 l1_row4(const float* __restrict__ x, int64_t r, int d, int k, bool vec) {
    float4 v = {0.0f, 0.0f, 0.0f, 0.0f};
    if (r < 0) return v;
    const float* __restrict__ xr = x + r * d;
    if (vec && k + 3 < d) return *reinterpret_cast<const float4*>(xr + k);
    if (k < d) v.x = xr[k];
    if (k + 1 < d) v.y = xr[k + 1];
    if (k + 2 < d) v.z = xr[k + 2];
    if (k + 3 < d) v.w = xr[k + 3];
    return v;
}

struct L1Args {
    const float* x;
    const float* hm;  // m_v / 2 in float32 (0 for padding rows)
    const int32_t* cand;
    int64_t n, n_cand, n_pad, chunk, part_stride;
    int32_t d, v_splits;
    double* part;
    int* err;
};

__global__ void __launch_bounds__(256) k_gains_l1(L1Args a) {
    __shared__ float4 lc4[kL1Cand * kL1S / 4];
    __shared__ float4 lp4[kL1VTile * kL1S / 4];
    __shared__ float lm[kL1VTile];
    __shared__ double red[16][kL1Cand];
    const float* lc = reinterpret_cast<const float*>(lc4);
    const float* lp = reinterpret_cast<const float*>(lp4);

    const int tid = threadIdx.x;
    const int tc = tid & 15, tv = tid >> 4;
    const int split = int(blockIdx.x % unsigned(a.v_splits));
    const int64_t ctile = int64_t(blockIdx.x / unsigned(a.v_splits));
    const int d = a.d;
    const bool vec = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(a.x) & 15) == 0;

    // staging assignment: candidate rows (64 rows x 8 float4) and point rows
    // (128 rows x 8 float4): thread t loads float4 column (t & 7) of rows t/8 + 32 q
    const int sk = (tid & 7) * 4;
    const int sr = tid >> 3;
    int64_t crow[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int64_t p = ctile * kL1Cand + sr + 32 * q;
        int64_t r = -1;
        if (p < a.n_cand) {
            r = a.cand ? int64_t(a.cand[p]) : p;
            if (r < 0 || r >= a.n_pad) {
                atomicCAS(a.err, 0, kDevErrIndex);
                r = -1;
            }
            if (r >= a.n) r = -1;  // padding rows: zero row, their gain is never read
        }
        crow[q] = r;
    }

    const int64_t v_begin = int64_t(split) * a.chunk;
    int64_t v_end = v_begin + a.chunk;
    if (v_end > a.n_pad) v_end = a.n_pad;

    double csum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t v0 = v_begin; v0 < v_end; v0 += kL1VTile) {
        float acc[4][8];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[i][j] = 0.0f;
        int64_t prow[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t v = v0 + sr + 32 * q;
            prow[q] = (v < v_end && v < a.n) ? v : -1;
        }
        // first stage of this tile into registers
        float4 pc[2], pp[4];
#pragma unroll
        for (int q = 0; q < 2; ++q) pc[q] = l1_row4(a.x, crow[q], d, sk, vec);
#pragma unroll
        for (int q = 0; q < 4; ++q) pp[q] = l1_row4(a.x, prow[q], d, sk, vec);
        __syncthreads();  // the previous tile's m_v reads are done
        if (tid < kL1VTile) {
            const int64_t v = v0 + tid;
            lm[tid] = (v < v_end) ? 2.0f * a.hm[v] : 0.0f;  // m_v (exact: twice m_v / 2)
        }
        for (int k0 = 0; k0 < d; k0 += kL1K) {
            __syncthreads();  // previous stage consumed
#pragma unroll
            for (int q = 0; q < 2; ++q) lc4[((sr + 32 * q) * kL1S + sk) / 4] = pc[q];
#pragma unroll
            for (int q = 0; q < 4; ++q) lp4[((sr + 32 * q) * kL1S + sk) / 4] = pp[q];
            __syncthreads();
            if (k0 + kL1K < d) {  // next stage in flight during this one
#pragma unroll
                for (int q = 0; q < 2; ++q) pc[q] = l1_row4(a.x, crow[q], d, k0 + kL1K + sk, vec);
#pragma unroll
                for (int q = 0; q < 4; ++q) pp[q] = l1_row4(a.x, prow[q], d, k0 + kL1K + sk, vec);
            }
            const int kn = (d - k0) < kL1K ? (d - k0) : kL1K;
            // columns past d hold 0 in both operands (|0 - 0| = 0), so whole
            // groups of 4 are summed
            for (int k = 0; k < kn; k += 4) {
                float4 c[4], p[8];
#pragma unroll
                for (int i = 0; i < 4; ++i) c[i] = *reinterpret_cast<const float4*>(lc + (tc + 16 * i) * kL1S + k);
#pragma unroll
                for (int j = 0; j < 8; ++j) p[j] = *reinterpret_cast<const float4*>(lp + (tv + 16 * j) * kL1S + k);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        acc[i][j] += fabsf(c[i].x - p[j].x);
                        acc[i][j] += fabsf(c[i].y - p[j].y);
                        acc[i][j] += fabsf(c[i].z - p[j].z);
                        acc[i][j] += fabsf(c[i].w - p[j].w);
                    }
            }
        }
        // clamp and accumulate: max(0, m_v - d(v, c)) (padding points have m_v = 0)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float mv = lm[tv + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i) csum[i] += double(fmaxf(mv - acc[i][j], 0.0f));
        }
    }
    // the 16 point-threads of each candidate, added in tv order
#pragma unroll
    for (int i = 0; i < 4; ++i) red[tv][tc + 16 * i] = csum[i];
    __syncthreads();
    if (tid < kL1Cand) {
        double g = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) g += red[q][tid];
        const int64_t p = ctile * kL1Cand + tid;
        if (p < a.n_cand) a.part[int64_t(split) * a.part_stride + p] = g;
    }
}

}  // namespace

hipError_t launch_gains_l1(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    L1Args a;
    a.x = ds->x;
    a.hm = ds->b.hm;
    a.cand = cand;
    a.n = ds->n;
    a.n_cand = n_cand;
    a.n_pad = ds->n_pad;
    a.chunk = gains_chunk(ds);
    a.part_stride = ds->n_pad;
    a.d = ds->d;
    a.v_splits = ds->v_splits;
    a.part = ds->b.part;
    a.err = &ds->b.state->error;
    const int64_t tiles = (n_cand + kL1Cand - 1) / kL1Cand;
    hipLaunchKernelGGL(k_gains_l1, dim3(unsigned(tiles * ds->v_splits)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ebc
