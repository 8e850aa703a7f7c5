// Marginal gains of many candidates at once, float32 on the MFMA units.
//
// For the current running minima m_v (the per-point terms of L(S u {e0}),
// Sec. 4.1, Eq. loss_decomposed) the gain of candidate c is
//     G[c] = sum_v max(0, m_v - d(v, c))               (|V| * Delta(c|S), Sec. 3)
// With d(v,c) = ||v||^2 + ||c||^2 - 2 v.c and all terms halved (exact in
// binary floating point):
//     G[c] / 2 = sum_v med3( v.c + ha_v - hn_c, 0, hm_v )
// where hn = ||.||^2/2, hm_v = m_v/2, ha_v = hm_v - hn_v, and med3 clamps the
// per-point term to [0, m_v/2] (the clamp at m_v is the clamp d >= 0).
//
// The paper's kernel (Alg. 2) gives every (set, point) cell of the work
// matrix W its own thread and writes W to global memory before a W*1 sum.
// Here the dot products v.c are a dense contraction on the matrix cores
// (v_mfma_f32_32x32x2_f32), the clamp and the sum over v are fused into the
// accumulator epilogue, and no distance or work matrix is ever written.
//
// Work decomposition: a workgroup (4 waves) owns 128 candidates (32 per
// wave, their rows held in registers for the whole kernel) and one chunk of
// the ground set; it streams that chunk through LDS in tiles of 64 points.
// MFMA tile: rows = 32 candidates, columns = 32 ground points, K = the
// dimension, split in two halves so that every lane reads contiguous K.
// Rows are padded to KP (a multiple of 8); when the last 4 values of a row
// are padding (TRIM: d <= KP - 4), the last two K steps pair values KH - 4,
// KH - 3 (lane half 0) with KH - 2, KH - 1 (lane half 1) instead of running
// two more steps whose half-1 values are all zeros: KH - 2 matrix
// instructions per column block instead of KH (50 instead of 52 at d = 100).
#include "ebc_internal.h"

namespace ebc {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// The prefetched tile lives in one wide vector value (not an array) so that
// it stays in registers across the loop.
template <int PER>
using PreVec = float __attribute__((ext_vector_type(4 * PER)));

template <int PER, int NV4>
__device__ __forceinline__ PreVec<PER> load_rows(const float4* __restrict__ src, int tid) {
    PreVec<PER> pre;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = tid + i * 256;
        const float4 t = src[e < NV4 ? e : NV4 - 1];  // clamped: stays inside the tile
        pre[4 * i + 0] = t.x;
        pre[4 * i + 1] = t.y;
        pre[4 * i + 2] = t.z;
        pre[4 * i + 3] = t.w;
    }
    return pre;
}

template <int KP, bool TRIM>
__device__ __forceinline__ void gains_f32_body(const GainsArgs& ga, int64_t bid) {
    const float* __restrict__ xq = static_cast<const float*>(ga.xq);
    const float* __restrict__ hn = ga.hn;
    const float* __restrict__ ha = ga.ha;
    const float* __restrict__ hm = ga.hm;
    const int32_t* __restrict__ cand = ga.cand;
    const int64_t n_cand = ga.n_cand, n_pad = ga.n_pad, chunk = ga.chunk, part_stride = ga.part_stride;
    const int32_t v_splits = ga.v_splits;
    double* __restrict__ part = ga.part;
    int* __restrict__ err = ga.err;
    constexpr int KH = KP / 2;        // K values per lane half
    constexpr int S = KP + 4;         // LDS row stride in floats (S/4 odd: conflict-free b128)
    constexpr int VT = kGainsVTile;   // ground points per LDS stage
    constexpr int NV4 = VT * KP / 4;  // float4 per stage
    constexpr int PER = (NV4 + 255) / 256;
    static_assert(KP % 8 == 0, "row length must be a multiple of 8");

    __shared__ float4 lds_x4[VT * S / 4];
    __shared__ float lds_ha[VT];
    __shared__ float lds_hm[VT];
    float* lds_x = reinterpret_cast<float*>(lds_x4);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 31;  // MFMA column within a 32-block
    const int half = lane >> 5;

    // (candidate tile, ground chunk) of this workgroup. Consecutive ids go to
    // the 8 XCDs in turn; with 8 G chunks, XCD x takes chunks x, x + 8, ...
    // one after the other (every candidate tile of chunk x first), so its L2
    // holds one chunk's rows at a time. 8 chunks: chunk = id % 8.
    int split;
    int64_t ctile;
    if (v_splits % 8 == 0) {
        const int64_t ntiles = (n_cand + kGainsCandTile - 1) / kGainsCandTile;
        const int64_t r = bid / 8;
        split = int(bid % 8) + 8 * int(r / ntiles);
        ctile = r % ntiles;
    } else {
        split = int(bid % v_splits);
        ctile = bid / v_splits;
    }

    // ---- candidate rows of this wave, in registers (MFMA A operand) ----
    const int64_t cpos = ctile * kGainsCandTile + wave * 32 + col;  // position in the candidate list
    // Candidate rows outside [0, n_pad) (a bad caller list) compute as zero
    // rows and raise EBC_E_INDEX.
    int64_t crow = -1;
    if (cpos < n_cand) crow = cand ? int64_t(cand[cpos]) : cpos;
    if (crow >= n_pad || crow < -1 || (cpos < n_cand && crow < 0)) {
        atomicCAS(err, 0, kDevErrIndex);
        crow = -1;
    }
    constexpr int QF = TRIM ? KH / 4 - 1 : KH / 4;  // groups of 4 K steps on contiguous halves
    float a[KH];
    if (crow >= 0) {
        const float4* src = reinterpret_cast<const float4*>(xq + crow * KP + half * KH);
#pragma unroll
        for (int q = 0; q < QF; ++q) {
            const float4 t = src[q];
            a[4 * q + 0] = t.x;
            a[4 * q + 1] = t.y;
            a[4 * q + 2] = t.z;
            a[4 * q + 3] = t.w;
        }
        if constexpr (TRIM) {  // half 0: values KH-4, KH-3; half 1: KH-2, KH-1
            const float2 t = *reinterpret_cast<const float2*>(xq + crow * KP + (half ? KH - 2 : KH - 4));
            a[KH - 4] = t.x;
            a[KH - 3] = t.y;
            a[KH - 2] = 0.0f;
            a[KH - 1] = 0.0f;
        }
    } else {
#pragma unroll
        for (int j = 0; j < KH; ++j) a[j] = 0.0f;
    }
    // -hn of the 16 candidate rows this lane holds in the MFMA result.
    float nhn[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t p = ctile * kGainsCandTile + wave * 32 + 8 * (r / 4) + 4 * half + (r % 4);
        float v = 0.0f;
        if (p < n_cand) {
            const int64_t row = cand ? int64_t(cand[p]) : p;
            if (row >= 0 && row < n_pad) v = hn[row];
        }
        nhn[r] = -v;
    }
    float acc_sum[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc_sum[r] = 0.0f;
    // the previous column block, its clamp-and-sum still to do (none yet:
    // -inf clamps to +0, which leaves the sums as they are)
    floatx16 accP;
    float hmP = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) accP[r] = -INFINITY;

    // ---- stream the ground-set chunk ----
    const int64_t v_begin = int64_t(split) * chunk;
    int64_t v_end = v_begin + chunk;
    if (v_end > n_pad) v_end = n_pad;

    // Next tile's rows are fetched into registers while the current tile's
    // MFMAs run, then written to LDS between two barriers.
    PreVec<PER> pre;
    float pre_ha = 0.0f, pre_hm = 0.0f;
    if (v_begin < v_end) {
        pre = load_rows<PER, NV4>(reinterpret_cast<const float4*>(xq + v_begin * KP), tid);
        if (tid < VT) {
            pre_ha = ha[v_begin + tid];
            pre_hm = hm[v_begin + tid];
        }
    }
    for (int64_t v0 = v_begin; v0 < v_end; v0 += VT) {
        __syncthreads();  // previous tile fully consumed
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + i * 256;
            if (e < NV4) {
                const int row = e / (KP / 4);
                const int q = e % (KP / 4);
                lds_x4[(row * S) / 4 + q] = make_float4(pre[4 * i], pre[4 * i + 1], pre[4 * i + 2], pre[4 * i + 3]);
            }
        }
        if (tid < VT) {
            lds_ha[tid] = pre_ha;
            lds_hm[tid] = pre_hm;
        }
        __syncthreads();
        if (v0 + VT < v_end) {  // in flight during the MFMAs
            pre = load_rows<PER, NV4>(reinterpret_cast<const float4*>(xq + (v0 + VT) * KP), tid);
            if (tid < VT) {
                pre_ha = ha[v0 + VT + tid];
                pre_hm = hm[v0 + VT + tid];
            }
        }

#pragma unroll
        for (int cb = 0; cb < VT / 32; ++cb) {
            const int vrow = cb * 32 + col;
            const float hav = lds_ha[vrow];
            const float hmv = lds_hm[vrow];
            floatx16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = nhn[r] + hav;
            const float4* b4 = reinterpret_cast<const float4*>(lds_x + vrow * S + half * KH);
            // The previous block's clamp-and-sum is issued in slices between
            // groups of this block's MFMAs (it does not depend on them, and
            // the sums keep their block order); the next group's operand read
            // is issued before each group.
            constexpr int SL = QF > 0 ? (16 + QF - 1) / QF : 16;  // terms per group
            float4 bv = b4[0];
#pragma unroll
            for (int q = 0; q < QF; ++q) {
                const float4 bn = q + 1 < QF ? b4[q + 1] : bv;
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[4 * q + 0], bv.x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[4 * q + 1], bv.y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[4 * q + 2], bv.z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[4 * q + 3], bv.w, acc, 0, 0, 0);
#pragma unroll
                for (int r = q * SL; r < (q + 1) * SL && r < 16; ++r)
                    acc_sum[r] += __builtin_amdgcn_fmed3f(accP[r], 0.0f, hmP);
                __builtin_amdgcn_sched_barrier(0);
                bv = bn;
            }
            if constexpr (TRIM) {
                const float2 bt = *reinterpret_cast<const float2*>(lds_x + vrow * S + (half ? KH - 2 : KH - 4));
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[KH - 4], bt.x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[KH - 3], bt.y, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = QF * SL; r < 16; ++r) acc_sum[r] += __builtin_amdgcn_fmed3f(accP[r], 0.0f, hmP);  // QF = 0
            accP = acc;
            hmP = hmv;
        }
    }
    // the last block's clamp-and-sum
#pragma unroll
    for (int r = 0; r < 16; ++r) acc_sum[r] += __builtin_amdgcn_fmed3f(accP[r], 0.0f, hmP);

    // ---- sum over the 32 columns (ground points) of each half, in float64 ----
    // Lane (half*32 + r), r < 16, keeps the total of candidate row
    // 8*(r/4) + 4*half + r%4.
    double mine = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        double v = double(acc_sum[r]);
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (col == r) mine = v;
    }
    if (col < 16) {
        const int r = col;
        const int64_t p = ctile * kGainsCandTile + wave * 32 + 8 * (r / 4) + 4 * half + (r % 4);
        if (p < n_cand) part[int64_t(split) * part_stride + p] = 2.0 * mine;
    }
}

template <int KP, bool TRIM>
__global__ void __launch_bounds__(256) k_gains_f32(GainsArgs ga) {
    gains_f32_body<KP, TRIM>(ga, blockIdx.x);
}

// Batched: workgroups wg_pre[j] .. wg_pre[j+1] serve descriptor slot_inst[j]
// (all candidates, in the same geometry as a solo launch).
template <int KP, bool TRIM>
__global__ void __launch_bounds__(256)
kb_gains_f32(const InstDesc* __restrict__ descs, const int32_t* __restrict__ slot_inst,
             const int64_t* __restrict__ wg_pre, int32_t slots, int32_t t) {
    const int j = find_slot(wg_pre, slots, blockIdx.x);
    const InstDesc c = descs[slot_inst[j]];
    if (c.t0 + t >= c.k) return;
    gains_f32_body<KP, TRIM>(gains_args(c, nullptr, c.n_pad), int64_t(blockIdx.x) - wg_pre[j]);
}

template <int KP>
static void launch_kp(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    const int64_t tiles = (n_cand + kGainsCandTile - 1) / kGainsCandTile;
    InstDesc c;
    fill_desc(ds, 0, nullptr, nullptr, nullptr, &c);
    if (ds->d <= KP - 4)  // the rows' last 4 padded slots are empty
        hipLaunchKernelGGL((k_gains_f32<KP, true>), dim3(unsigned(tiles * ds->v_splits)), dim3(256), 0, s,
                           gains_args(c, cand, n_cand));
    else
        hipLaunchKernelGGL((k_gains_f32<KP, false>), dim3(unsigned(tiles * ds->v_splits)), dim3(256), 0, s,
                           gains_args(c, cand, n_cand));
}

#define EBC_F32_KPS(X) \
    X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64) X(72) X(80) X(88) X(96) X(104) X(112) X(120) X(128)

hipError_t launch_gains_f32(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    switch (ds->k_pad) {
#define EBC_KP(K) \
    case K: launch_kp<K>(ds, cand, n_cand, s); break;
        EBC_F32_KPS(EBC_KP)
#undef EBC_KP
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// trim: every instance of the bucket has d <= k_pad - 4 (the bucket key says so)
hipError_t launch_gains_f32_batched(int32_t k_pad, bool trim, const InstDesc* descs, const int32_t* slot_inst,
                                    const int64_t* wg_pre, int32_t slots, int64_t total_wgs, int32_t t,
                                    hipStream_t s) {
    switch (k_pad) {
#define EBC_KP(K)                                                                                             \
    case K:                                                                                                   \
        if (trim)                                                                                             \
            hipLaunchKernelGGL((kb_gains_f32<K, true>), dim3(unsigned(total_wgs)), dim3(256), 0, s, descs,    \
                               slot_inst, wg_pre, slots, t);                                                  \
        else                                                                                                  \
            hipLaunchKernelGGL((kb_gains_f32<K, false>), dim3(unsigned(total_wgs)), dim3(256), 0, s, descs,   \
                               slot_inst, wg_pre, slots, t);                                                  \
        break;
        EBC_F32_KPS(EBC_KP)
#undef EBC_KP
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ebc
