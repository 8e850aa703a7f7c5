// Marginal gains for long rows: padded row length above 128 values (the
// paper's case study summarises N = 1000 series of d = 3524 samples, Sec. 6).
//
// Same quantity and halving as the short-row kernels (Sec. 3 discrete
// derivative, Sec. 4.1 per-point decomposition):
//     G[c]/2 = sum_v med3( x_v . x_c + ha_v - hn_c, 0, hm_v )
// with the dataset's distance-dtype rows, their norms and (FP8) per-row E8M0
// scales. A whole row no longer fits in registers, so each wave walks the
// dimension: row pieces are loaded straight from global memory (the next
// batch while the current one is multiplied) and fed to the dtype's 32x32
// matrix instruction. MFMA tile: rows = 32 candidates, columns = 32 ground
// points; lane half h takes half h of every piece, for both operands.
//
// Work decomposition: a workgroup owns 128/KS candidates and one chunk of
// the ground set, walked in tiles of 64 points. KS = 1: each wave owns 32
// candidates of its own. KS = 4 (small ground sets, where candidate blocks
// alone leave most of the chip idle): the four waves share one block of 32
// candidates, each multiplies a quarter of the dimension, and the four
// partial dot products of a tile are added through LDS in wave order before
// the clamp. The clamp sums and the float64 column sums run in a fixed
// order, so results do not depend on the schedule.
#include "ebc_internal.h"
#include "wide_row.h"

namespace ebc {

namespace {

template <int DT, int KS>
__device__ __forceinline__ void gains_wide_body(const GainsArgs& ga, int32_t k_pad, int64_t bid) {
    using R = WideRow<DT>;
    using Piece = typename R::Piece;
    constexpr int B = R::kBatch;
    constexpr int CT = 32 * 4 / KS;             // candidates per workgroup
    constexpr int NR = KS > 1 ? 8 : 16;         // candidate rows whose clamps this lane sums
    constexpr bool kFp8 = DT == EBC_DT_FP8_E4M3;
    static_assert(KS == 1 || KS == 4, "K split of 1 or 4 waves");
    // KS = 4: partial dot products [wave][cb][r][lane], then column sums [wave][half][8]
    __shared__ float red[KS > 1 ? 4 * 2 * 16 * 64 : 1];
    __shared__ double tot[KS > 1 ? 4 * 2 * 8 : 1];

    const void* xq = ga.xq;
    const float* __restrict__ hn = ga.hn;
    const float* __restrict__ ha = ga.ha;
    const float* __restrict__ hm = ga.hm;
    const int* __restrict__ scale = ga.scale;
    const int32_t* __restrict__ cand = ga.cand;
    const int64_t n_cand = ga.n_cand, n_pad = ga.n_pad;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 31;
    const int half = lane >> 5;
    const int split = int(bid % ga.v_splits);
    const int64_t ctile = bid / ga.v_splits;
    const int64_t cbase = ctile * CT + (KS > 1 ? 0 : wave * 32);  // this wave's candidate block
    const int r0 = KS > 1 ? 8 * (wave & 1) : 0;                    // first of its NR rows

    // candidate row of this lane (A operand row `col`); rows outside
    // [0, n_pad) in a caller's list compute as zero rows and raise EBC_E_INDEX
    const int64_t cpos = cbase + col;
    int64_t crow = -1;
    if (cpos < n_cand) crow = cand ? int64_t(cand[cpos]) : cpos;
    if (crow >= n_pad || crow < -1 || (cpos < n_cand && crow < 0)) {
        atomicCAS(ga.err, 0, kDevErrIndex);
        crow = -1;
    }
    const bool alive = crow >= 0;
    const int64_t arow = alive ? crow : 0;
    const int sa = kFp8 ? (alive ? scale[crow] : 127) : 127;
    // -hn of the candidate rows this lane sums (result rows 8*(r/4) + 4*half + r%4)
    float nhn[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int r = r0 + i;
        const int64_t p = cbase + 8 * (r / 4) + 4 * half + (r % 4);
        float v = 0.0f;
        if (p < n_cand) {
            const int64_t row = cand ? int64_t(cand[p]) : p;
            if (row >= 0 && row < n_pad) v = hn[row];
        }
        nhn[i] = -v;
    }
    float acc_sum[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) acc_sum[i] = 0.0f;

    const int np = R::pieces(k_pad);
    const int kq = KS > 1 ? wave : 0;
    const int p0 = KS > 1 ? np * kq / 4 : 0;
    const int p1 = KS > 1 ? np * (kq + 1) / 4 : np;

    const int64_t v_begin = int64_t(split) * ga.chunk;
    int64_t v_end = v_begin + ga.chunk;
    if (v_end > n_pad) v_end = n_pad;

    for (int64_t v0 = v_begin; v0 < v_end; v0 += 64) {
        int64_t prow[2];
        int sb[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            prow[cb] = v0 + cb * 32 + col;
            sb[cb] = kFp8 ? scale[prow[cb]] : 127;
        }
        floatx16 acc[2];
        float hmv[2] = {0.0f, 0.0f};
        if constexpr (KS == 1) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const float hav = ha[prow[cb]];
                hmv[cb] = hm[prow[cb]];
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[cb][r] = nhn[r % NR] + hav;
            }
        } else {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[cb][r] = 0.0f;
        }
        // this wave's pieces [p0, p1), batches of B, the next batch in flight
        Piece a[B], b[2][B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const bool in = p0 + i < p1;
            a[i] = (in && alive) ? R::load(xq, arow, k_pad, p0 + i, half) : Piece{};
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) b[cb][i] = in ? R::load(xq, prow[cb], k_pad, p0 + i, half) : Piece{};
        }
        for (int p = p0; p < p1; p += B) {
            const bool more = p + B < p1;
            Piece an[B], bn[2][B];
            if (more) {
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    const bool in = p + B + i < p1;
                    an[i] = (in && alive) ? R::load(xq, arow, k_pad, p + B + i, half) : Piece{};
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        bn[cb][i] = in ? R::load(xq, prow[cb], k_pad, p + B + i, half) : Piece{};
                }
            }
#pragma unroll
            for (int i = 0; i < B; ++i)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) acc[cb] = R::mma(a[i], b[cb][i], acc[cb], sa, sb[cb]);
            if (more) {
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    a[i] = an[i];
                    b[0][i] = bn[0][i];
                    b[1][i] = bn[1][i];
                }
            }
        }
        if constexpr (KS == 1) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc_sum[r % NR] += __builtin_amdgcn_fmed3f(acc[cb][r], 0.0f, hmv[cb]);
        } else {
            // the four quarters of this tile's dot products, added in wave order
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) red[((wave * 2 + cb) * 16 + r) * 64 + lane] = acc[cb][r];
            __syncthreads();
            const int cbe = wave >> 1;  // the 32-point block whose clamps this wave takes
            const int64_t v = v0 + cbe * 32 + col;
            const float hav = ha[v], hmw = hm[v];
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const int r = r0 + i;
                float t = nhn[i] + hav;
#pragma unroll
                for (int w = 0; w < 4; ++w) t += red[((w * 2 + cbe) * 16 + r) * 64 + lane];
                acc_sum[i] += __builtin_amdgcn_fmed3f(t, 0.0f, hmw);
            }
            __syncthreads();  // red is rewritten by the next tile
        }
    }

    // ---- float64 sums over the 32 columns (ground points) of each half ----
    double mine = 0.0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        double v = double(acc_sum[i]);
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (col == i) mine = v;
    }
    double* __restrict__ part = ga.part + int64_t(split) * ga.part_stride;
    if constexpr (KS == 1) {
        if (col < 16) {
            const int r = col;
            const int64_t p = cbase + 8 * (r / 4) + 4 * half + (r % 4);
            if (p < n_cand) part[p] = 2.0 * mine;
        }
    } else {
        // waves w and w+2 hold the same rows for the two 32-point blocks
        if (col < 8) tot[(wave * 2 + half) * 8 + col] = mine;
        __syncthreads();
        if (wave < 2 && col < 8) {
            const double g = tot[(wave * 2 + half) * 8 + col] + tot[((wave + 2) * 2 + half) * 8 + col];
            const int r = r0 + col;
            const int64_t p = cbase + 8 * (r / 4) + 4 * half + (r % 4);
            if (p < n_cand) part[p] = 2.0 * g;
        }
    }
}

template <int DT, int KS>
__global__ void __launch_bounds__(256) k_gains_wide(GainsArgs ga, int32_t k_pad) {
    gains_wide_body<DT, KS>(ga, k_pad, blockIdx.x);
}

// Batched: workgroups wg_pre[j] .. wg_pre[j+1] serve descriptor slot_inst[j]
// (all candidates, in the same geometry as a solo launch).
template <int DT, int KS>
__global__ void __launch_bounds__(256)
kb_gains_wide(const InstDesc* __restrict__ descs, const int32_t* __restrict__ slot_inst,
              const int64_t* __restrict__ wg_pre, int32_t slots, int32_t t) {
    const int j = find_slot(wg_pre, slots, blockIdx.x);
    const InstDesc c = descs[slot_inst[j]];
    if (c.t0 + t >= c.k) return;
    gains_wide_body<DT, KS>(gains_args(c, nullptr, c.n_pad), c.k_pad, int64_t(blockIdx.x) - wg_pre[j]);
}

template <int DT, int KS>
void launch_w(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    const int64_t ct = 32 * 4 / KS;
    const int64_t tiles = (n_cand + ct - 1) / ct;
    InstDesc c;
    fill_desc(ds, 0, nullptr, nullptr, nullptr, &c);
    hipLaunchKernelGGL((k_gains_wide<DT, KS>), dim3(unsigned(tiles * ds->v_splits)), dim3(256), 0, s,
                       gains_args(c, cand, n_cand), ds->k_pad);
}

template <int DT>
void launch_w_ks(int32_t ks, const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    if (ks == 4)
        launch_w<DT, 4>(ds, cand, n_cand, s);
    else
        launch_w<DT, 1>(ds, cand, n_cand, s);
}

template <int DT>
void launch_wb(int32_t ks, const InstDesc* descs, const int32_t* slot_inst, const int64_t* wg_pre, int32_t slots,
               int64_t total_wgs, int32_t t, hipStream_t s) {
    const dim3 g = dim3(unsigned(total_wgs)), b = dim3(256);
    if (ks == 4)
        hipLaunchKernelGGL((kb_gains_wide<DT, 4>), g, b, 0, s, descs, slot_inst, wg_pre, slots, t);
    else
        hipLaunchKernelGGL((kb_gains_wide<DT, 1>), g, b, 0, s, descs, slot_inst, wg_pre, slots, t);
}

}  // namespace

hipError_t launch_gains_wide(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    const int32_t ks = wide_ksplit(ds->n_pad);
    switch (ds->dt) {
        case EBC_DT_F32: launch_w_ks<EBC_DT_F32>(ks, ds, cand, n_cand, s); break;
        case EBC_DT_F16: launch_w_ks<EBC_DT_F16>(ks, ds, cand, n_cand, s); break;
        case EBC_DT_BF16: launch_w_ks<EBC_DT_BF16>(ks, ds, cand, n_cand, s); break;
        case EBC_DT_FP8_E4M3: launch_w_ks<EBC_DT_FP8_E4M3>(ks, ds, cand, n_cand, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gains_wide_batched(int32_t dt, int32_t ksplit, const InstDesc* descs, const int32_t* slot_inst,
                                     const int64_t* wg_pre, int32_t slots, int64_t total_wgs, int32_t t,
                                     hipStream_t s) {
    switch (dt) {
        case EBC_DT_F32: launch_wb<EBC_DT_F32>(ksplit, descs, slot_inst, wg_pre, slots, total_wgs, t, s); break;
        case EBC_DT_F16: launch_wb<EBC_DT_F16>(ksplit, descs, slot_inst, wg_pre, slots, total_wgs, t, s); break;
        case EBC_DT_BF16: launch_wb<EBC_DT_BF16>(ksplit, descs, slot_inst, wg_pre, slots, total_wgs, t, s); break;
        case EBC_DT_FP8_E4M3:
            launch_wb<EBC_DT_FP8_E4M3>(ksplit, descs, slot_inst, wg_pre, slots, total_wgs, t, s);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ebc
