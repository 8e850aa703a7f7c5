// Reduced-precision matrix-core helpers shared by the marginal-gains and the
// multi-set kernels: operand traits per distance dtype and one 32x32 MFMA
// step on 16-byte operand units (BF16/FP16: 8 values; FP8-e4m3: 32 values in
// two units, with the E8M0 scales of the lane's row and column).
#pragma once

#include "ebc_internal.h"

namespace ebc {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;

template <int DT>
struct Lp;
template <>
struct Lp<EBC_DT_BF16> {
    static constexpr int kElem = 2, kChunkK = 16, kU4 = 1;  // uint4 per lane-half per chunk
};
template <>
struct Lp<EBC_DT_F16> {
    static constexpr int kElem = 2, kChunkK = 16, kU4 = 1;
};
template <>
struct Lp<EBC_DT_FP8_E4M3> {
    static constexpr int kElem = 1, kChunkK = 64, kU4 = 2;
};

// Clamp-and-sum of one 32x32 result tile for this lane. Each term is
// clamp(s (acc - lo), 0, 1) with s = 2^-e a power of two and 2^e >= m_v / 2
// for every point: one v_fma_f32 with the clamp bit, fed the per-column
// shift sh = -lo s. Scaling by a power of two is exact, so each term is
// s (acc - lo) rounded once, i.e. the scaled term max(0, m_v/2 - d^/2); the
// upper bound 1 stands for the scaled m_v/2 and only binds when rounding
// makes a computed distance negative. A value at or below the lane's lower
// bound lo adds exactly 0, so a tile whose every value, in every lane, lies
// at or below its lane's bound (the largest of the lane's 16 values, a ballot
// over the wave) adds only zeros and is skipped: the same sums, bit for bit,
// so whether a tile is skipped never changes a result. Otherwise the 16
// terms are issued back to back into 16 registers (the empty asm statement
// keeps them all live, so the compiler cannot reuse one temporary and make
// every add wait for the term just before it), then the 16 adds; the
// per-lane sum order is the same in every tile variant.
__device__ __forceinline__ void clamp_sum16(const floatx16& acc, float lo, float s, float sh, float (&sum)[16]) {
    float m = fmaxf(fmaxf(acc[0], acc[1]), acc[2]);
#pragma unroll
    for (int r = 3; r < 15; r += 2) m = fmaxf(fmaxf(m, acc[r]), acc[r + 1]);
    m = fmaxf(m, acc[15]);
    if (__builtin_amdgcn_ballot_w64(m > lo) == 0) return;
    float t[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) t[r] = __builtin_amdgcn_fmed3f(fmaf(acc[r], s, sh), 0.0f, 1.0f);
    asm volatile(""
                 : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]), "+v"(t[6]), "+v"(t[7]),
                   "+v"(t[8]), "+v"(t[9]), "+v"(t[10]), "+v"(t[11]), "+v"(t[12]), "+v"(t[13]), "+v"(t[14]),
                   "+v"(t[15]));
#pragma unroll
    for (int r = 0; r < 16; ++r) sum[r] += t[r];
}

// s_waitcnt with only the vector-memory counter constrained (<= N).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Workgroup barrier for the LDS ring without the release/acquire fences of
// __syncthreads (those would also wait for the copies still in flight into
// the other stages). The caller has already waited for its own copies of the
// stage about to be read; here the wave's LDS reads are drained, and the
// empty asm statements keep the compiler from moving memory accesses across.
__device__ __forceinline__ void ring_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xF | (0x3 << 14) | (0x7 << 4));  // lgkmcnt(0), vmcnt/expcnt untouched
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <int DT>
__device__ __forceinline__ floatx16 mfma_main(const uint4* a, const uint4* b, floatx16 c, int sa, int sb);

template <>
__device__ __forceinline__ floatx16 mfma_main<EBC_DT_BF16>(const uint4* a, const uint4* b, floatx16 c, int,
                                                           int) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[0]), __builtin_bit_cast(bf16x8, b[0]),
                                                  c, 0, 0, 0);
}
template <>
__device__ __forceinline__ floatx16 mfma_main<EBC_DT_F16>(const uint4* a, const uint4* b, floatx16 c, int, int) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a[0]), __builtin_bit_cast(halfx8, b[0]),
                                                 c, 0, 0, 0);
}
template <>
__device__ __forceinline__ floatx16 mfma_main<EBC_DT_FP8_E4M3>(const uint4* a, const uint4* b, floatx16 c, int sa,
                                                               int sb) {
    const intx8 av = {int(a[0].x), int(a[0].y), int(a[0].z), int(a[0].w), int(a[1].x), int(a[1].y), int(a[1].z),
                      int(a[1].w)};
    const intx8 bv = {int(b[0].x), int(b[0].y), int(b[0].z), int(b[0].w), int(b[1].x), int(b[1].y), int(b[1].z),
                      int(b[1].w)};
    // format 0 = e4m3 for both operands; E8M0 scales of the lane's row / column
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, sa, 0, sb);
}

}  // namespace ebc
