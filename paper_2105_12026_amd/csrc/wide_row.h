// Row pieces of the long-row kernels (padded row length above 128 values):
// the part of a candidate or ground-point row that one lane half feeds to
// the matrix instruction(s) of one K step, loaded straight from global
// memory, and the matching 32x32 matrix step. Both operands use the same
// split of every piece between the lane halves, so each K step covers the
// piece's values exactly once.
#pragma once

#include "ebc_internal.h"
#include "lp_mfma.h"

namespace ebc {

template <int DT>
struct WideRow;

// Tiled rows (64-row tiles, 16-byte units unit-major): unit u of row r at
// 16-byte index ((r/64)*RU + u)*64 + r%64, so the 32 rows of an operand
// block read one unit as 512 contiguous bytes.
__device__ __forceinline__ uint4 tiled_unit(const void* xq, int64_t row, int ru, int u) {
    return static_cast<const uint4*>(xq)[((row >> 6) * ru + u) * 64 + (row & 63)];
}

// float32 long rows, tiled (k_pad/4 units a row): piece p = values
// 8p .. 8p+7, half h holds unit 2p+h = 8p+4h .. 8p+4h+3 (four 32x32x2 steps).
template <>
struct WideRow<EBC_DT_F32> {
    struct Piece {
        float4 v;
    };
    static constexpr int kBatch = 4;  // pieces per load batch
    __device__ static int pieces(int k_pad) { return k_pad / 8; }
    __device__ static Piece load(const void* xq, int64_t row, int k_pad, int p, int half) {
        return {static_cast<const float4*>(xq)[((row >> 6) * (k_pad / 4) + 2 * p + half) * 64 + (row & 63)]};
    }
    // the caller's unpadded rows [n, d]: values past d read as 0
    __device__ static Piece load_x(const float* x, int64_t row, int d, int p, int half) {
        const int k = 8 * p + 4 * half;
        const float* r = x + row * d;
        if ((d & 3) == 0) return {k < d ? *reinterpret_cast<const float4*>(r + k) : make_float4(0.0f, 0.0f, 0.0f, 0.0f)};
        return {make_float4(k < d ? r[k] : 0.0f, k + 1 < d ? r[k + 1] : 0.0f, k + 2 < d ? r[k + 2] : 0.0f,
                            k + 3 < d ? r[k + 3] : 0.0f)};
    }
    __device__ static floatx16 mma(const Piece& a, const Piece& b, floatx16 c, int, int) {
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v.x, b.v.x, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v.y, b.v.y, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v.z, b.v.z, c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a.v.w, b.v.w, c, 0, 0, 0);
    }
};

// BF16 / FP16: piece p = units 2p, 2p+1; half h holds unit 2p+h (one
// 32x32x16 step).
template <int DT>
struct WideHalf {
    struct Piece {
        uint4 v;
    };
    static constexpr int kBatch = 4;
    __device__ static int pieces(int k_pad) { return k_pad / 16; }
    __device__ static Piece load(const void* xq, int64_t row, int k_pad, int p, int half) {
        return {tiled_unit(xq, row, k_pad / 8, 2 * p + half)};
    }
    __device__ static floatx16 mma(const Piece& a, const Piece& b, floatx16 c, int, int) {
        return mfma_main<DT>(&a.v, &b.v, c, 0, 0);
    }
};
template <>
struct WideRow<EBC_DT_BF16> : WideHalf<EBC_DT_BF16> {};
template <>
struct WideRow<EBC_DT_F16> : WideHalf<EBC_DT_F16> {};

// FP8-e4m3: piece p = units 4p .. 4p+3; half h holds units 4p+2h, 4p+2h+1
// (one scaled 32x32x64 step with the row and column E8M0 scales).
template <>
struct WideRow<EBC_DT_FP8_E4M3> {
    struct Piece {
        uint4 v[2];
    };
    static constexpr int kBatch = 2;
    __device__ static int pieces(int k_pad) { return k_pad / 64; }
    __device__ static Piece load(const void* xq, int64_t row, int k_pad, int p, int half) {
        const int ru = k_pad / 16;
        return {{tiled_unit(xq, row, ru, 4 * p + 2 * half), tiled_unit(xq, row, ru, 4 * p + 2 * half + 1)}};
    }
    __device__ static floatx16 mma(const Piece& a, const Piece& b, floatx16 c, int sa, int sb) {
        return mfma_main<EBC_DT_FP8_E4M3>(a.v, b.v, c, sa, sb);
    }
};

}  // namespace ebc
