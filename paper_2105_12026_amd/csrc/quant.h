// Device helpers for the reduced-precision copies of V (round-to-nearest-even
// conversions) and the float32 terms the gains kernels read for a ground
// point (its half running minimum and the affine term of the distance
// expansion).
#pragma once

#include <math.h>

#include "ebc_internal.h"

namespace ebc {

__device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// OCP FP8 e4m3 (bias 7, no infinities, max finite 448), round to nearest
// even, saturating. |x| is expected <= 448 after the per-row scale.
__device__ inline uint8_t f32_to_e4m3_rne(float x) {
    const uint8_t sign = x < 0.0f ? 0x80 : 0x00;
    const float a = fabsf(x);
    if (!(a == a)) return 0x7f;
    if (a >= 448.0f) return sign | 0x7e;
    if (a < 0.015625f) {  // below the smallest normal 2^-6: steps of 2^-9
        const float q = rintf(a * 512.0f);  // 0..8; 8 encodes 2^-6 (exponent field 1)
        return sign | uint8_t(q);
    }
    int e;
    (void)frexpf(a, &e);
    int E = e - 1;  // a in [2^E, 2^(E+1))
    float q = rintf(ldexpf(a, 3 - E));  // 8..16
    if (q >= 16.0f) {
        q = 8.0f;
        E += 1;
    }
    if (E > 8 || (E == 8 && q > 14.0f)) return sign | 0x7e;
    return sign | uint8_t(((E + 7) << 3) | (int(q) - 8));
}

__device__ inline float e4m3_to_f32(uint8_t b) {
    const int e = (b >> 3) & 15, m = b & 7;
    const float v = e == 0 ? ldexpf(float(m), -9) : ldexpf(float(8 + m), e - 10);
    return (b & 0x80) ? -v : v;
}

// Refresh the float32 terms of ground point v after its running minimum
// changed to mv: hm = mv/2 and ha = mv/2 - hn.
__device__ inline void set_point_terms(const Buffers& b, int64_t v, double mv) {
    const float ha = float(0.5 * mv - double(b.hn[v]));
    const float hm = float(0.5 * mv);
    b.ha[v] = ha;
    b.hm[v] = hm;
    if (b.inv) {  // grouped order: the slot-order copies follow
        const int32_t s = b.inv[v];
        b.hap[s] = ha;
        b.hmp[s] = hm;
    }
}

}  // namespace ebc
