// Residency and precompute for one ground set V (Sec. 4.1: L({e0}) is
// computed once and reused by every evaluation; Sec. 4.2: V is copied to the
// device once). Also the workspace layout and the greedy-state resets.
#include <math.h>

#include "ebc_internal.h"
#include "quant.h"

namespace ebc {

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int64_t pad_rows(int64_t n) { return (n + kRowAlign - 1) / kRowAlign * kRowAlign; }

int32_t k_pad_for(int32_t d, ebc_dtype dt) {
    // Row length of the distance-dtype copy, padded with zeros to the K of
    // the matrix instruction (each half of a row is whole 16-byte vectors):
    // float32 32x32x2 -> 8, bf16/f16 32x32x16 -> 16, e4m3 32x32x64 -> 64.
    const int g = dt == EBC_DT_F32 ? 8 : (dt == EBC_DT_FP8_E4M3 ? 64 : 16);
    return (d + g - 1) / g * g;
}

int elem_bytes(ebc_dtype dt) { return dt == EBC_DT_F32 ? 4 : (dt == EBC_DT_FP8_E4M3 ? 1 : 2); }

int64_t gains_chunk(const ebc_dataset* ds) {
    // ground-set chunk per workgroup: a multiple of the kernel's LDS tile
    // (float32: 64 rows; reduced precision: 256, the same for every variant)
    // (long rows: 64 for every dtype)
    const int64_t g = (ds->dt == EBC_DT_F32 || wide_rows(ds->k_pad)) ? kGainsVTile : 256;
    const int64_t c = (ds->n_pad + ds->v_splits - 1) / ds->v_splits;
    return (c + g - 1) / g * g;
}

int64_t gains_cand_tile(const ebc_dataset* ds) {
    if (wide_rows(ds->k_pad)) return 32 * 4 / wide_ksplit(ds->n_pad);
    if (ds->dt == EBC_DT_F32) return kGainsCandTile;
    // variant 1: 4 waves x 32 rows x 4 blocks; 3: 8 waves x 32 x pp_blocks; else 4 x 32 x 2
    if (ds->variant == 3) {
        const int kc = ds->k_pad / (ds->dt == EBC_DT_FP8_E4M3 ? 64 : 16);
        return 8 * 32 * pp_blocks(ds->dt, kc);
    }
    return ds->variant == 1 ? 512 : 256;
}

int32_t gains_bucket(const ebc_dataset* ds) {
    // last digit: the tile variant (reduced precision), for long rows the K
    // split, for float32 whether the rows' last 4 padded slots are empty (the
    // kernel then shortens its last K step)
    if (wide_rows(ds->k_pad)) return int32_t(ds->dt) * 100000 + ds->k_pad * 10 + wide_ksplit(ds->n_pad);
    const int32_t last = ds->dt == EBC_DT_F32 ? (ds->d <= ds->k_pad - 4 ? 1 : 0) : ds->variant;
    return int32_t(ds->dt) * 100000 + ds->k_pad * 10 + last;
}

void fill_desc(const ebc_dataset* ds, int32_t k, int32_t* sel, double* f, double* gain, InstDesc* out) {
    InstDesc& c = *out;
    c.b = ds->b;
    c.x = ds->x;
    c.n = ds->n;
    c.n_pad = ds->n_pad;
    c.d = ds->d;
    c.k_pad = ds->k_pad;
    c.v_splits = ds->v_splits;
    c.nb = int32_t(ds->n_pad / kBlock);
    c.k = k;
    c.t0 = 0;
    c.dt = int32_t(ds->dt);
    c.variant = ds->variant;
    c.metric = ds->metric;
    c.pad_m = 0;
    c.chunk = gains_chunk(ds);
    c.sel = sel;
    c.f = f;
    c.gain = gain;
}

hipError_t launch_gains_batched(int32_t bucket, const InstDesc* descs, const int32_t* slot_inst,
                                const int64_t* wg_pre, int32_t slots, int64_t total_wgs, int32_t t, hipStream_t s) {
    const int32_t dt = bucket / 100000, k_pad = (bucket % 100000) / 10, variant = bucket % 10;
    if (wide_rows(k_pad))
        return launch_gains_wide_batched(dt, variant, descs, slot_inst, wg_pre, slots, total_wgs, t, s);
    if (dt == EBC_DT_F32)
        return launch_gains_f32_batched(k_pad, variant == 1, descs, slot_inst, wg_pre, slots, total_wgs, t, s);
    const int32_t kc = k_pad / (dt == EBC_DT_FP8_E4M3 ? 64 : 16);
    return launch_gains_lp_batched(dt, kc, variant, descs, slot_inst, wg_pre, slots, total_wgs, t, s);
}

int32_t v_splits_for(int64_t n_pad, int32_t k_pad, ebc_dtype dt) {
    if (wide_rows(k_pad)) {
        // long rows: enough (candidate block, chunk) workgroups for about
        // eight waves per compute unit, chunks of at least 64 points
        const int64_t tiles = n_pad / (32 * 4 / wide_ksplit(n_pad));
        int64_t v = (2048 + tiles - 1) / tiles;
        if (v > 16) v = 16;
        if (v > n_pad / 64) v = n_pad / 64;
        return int32_t(v < 1 ? 1 : v);
    }
    // The ground set is cut into one chunk per XCD (8 on MI355X) once there
    // are enough candidate tiles; a workgroup then owns (candidate tile,
    // chunk) and consecutive workgroup ids, which the dispatcher deals round
    // robin over the XCDs, land on different chunks. Float32 with fewer than
    // 1024 candidate tiles: two chunks per XCD, so that the launch still runs
    // about 24 rounds of resident workgroups and its last, partial round is a
    // small part of it (100000 x 100: 1-1.6% faster; 24 and 32 chunks were
    // slower, reduced precision measured no faster with 16).
    int64_t tiles = n_pad / kGainsCandTile;
    if (tiles >= 64) return (dt == EBC_DT_F32 && tiles < 1024) ? 16 : 8;
    if (tiles >= 16) return 4;
    return 1;
}

Layout layout(int64_t n, int32_t d, ebc_dtype dt) {
    Layout L{};
    const int64_t np = pad_rows(n);
    const int32_t kp = k_pad_for(d, dt);
    const int64_t nb = np / kBlock + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.off_xq = take(size_t(np) * kp * elem_bytes(dt));
    L.off_scale = dt == EBC_DT_FP8_E4M3 ? take(size_t(np) * sizeof(int)) : 0;
    L.off_mu = wide_rows(kp) ? take(size_t(kp) * sizeof(double)) : 0;
    L.off_n64 = take(size_t(np) * sizeof(double));
    L.off_m0 = take(size_t(np) * sizeof(double));
    L.off_m64 = take(size_t(np) * sizeof(double));
    L.off_hn = take(size_t(np) * sizeof(float));
    L.off_ha = take(size_t(np) * sizeof(float));
    L.off_hm = take(size_t(np) * sizeof(float));
    L.off_sel = take(size_t(np));
    L.off_part = take(size_t(v_splits_for(np, kp, dt)) * np * sizeof(double));
    L.off_gsum = take(size_t(np) * sizeof(double));
    L.off_bmax = take(size_t(nb) * sizeof(double));
    L.off_barg = take(size_t(nb) * sizeof(int32_t));
    L.off_bcnt = take(size_t(nb) * sizeof(int32_t));
    L.off_wstage = take(size_t(np) * sizeof(WindowEntry));
    L.off_wfinal = take(size_t(kWindowMax) * sizeof(WindowEntry));
    L.off_rpart = take(size_t(wide_rows(kp) ? 4 * nb : nb) * kWindowMax * sizeof(double));
    L.off_fpart = take(size_t(nb) * sizeof(double));
    L.off_state = take(sizeof(DevState));
    if (grouped(kp, dt)) {
        L.off_perm = take(size_t(np) * sizeof(int32_t));
        L.off_inv = take(size_t(np) * sizeof(int32_t));
        L.off_xqp = take(size_t(np) * kp * elem_bytes(dt));
        L.off_hnp = take(size_t(np) * sizeof(float));
        L.off_hap = take(size_t(np) * sizeof(float));
        L.off_hmp = take(size_t(np) * sizeof(float));
        L.off_scp = dt == EBC_DT_FP8_E4M3 ? take(size_t(np) * sizeof(int)) : 0;
        L.off_gbucket = take(size_t(np) * sizeof(int32_t));
        L.off_gcount = take(size_t(np / kBlock) * group_count(n) * sizeof(int32_t));
    }
    L.total = o;
    return L;
}

// Column means of V in float64 for long rows, in a fixed order: a block
// takes 64 columns, thread (column, phase) sums rows phase, phase + 16, ...,
// and the 16 phase sums are added in phase order.
__global__ void __launch_bounds__(1024) k_colmean(const float* __restrict__ x, int64_t n, int32_t d, int32_t kp,
                                                  double* __restrict__ mu) {
    __shared__ double part[16][64];
    const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + c;
    double s = 0.0;
    if (k < d)
        for (int64_t r = ph; r < n; r += 16) s += double(x[r * d + k]);
    part[ph][c] = s;
    __syncthreads();
    if (ph == 0 && k < kp) {
        double t = 0.0;
        for (int i = 0; i < 16; ++i) t += part[i][c];
        mu[k] = k < d ? t / double(n) : 0.0;
    }
}

// One thread per padded row: float64 norm, finiteness check, the padded
// float32 copy (columns d.. hold 0; long rows: centred at the column means,
// which leaves every distance unchanged and shrinks the dot products whose
// cancellation limits the float32 gains), and the initial state
// m_v = ||v||^2 (S = {}). Per-block norm sums go to fpart for L({e0}).
__global__ void __launch_bounds__(kBlock) k_prep(const float* __restrict__ x, int64_t n, int32_t d,
                                                 int32_t kp, Buffers b) {
    __shared__ double red[kBlock];
    __shared__ double rmax[kBlock];
    const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double nv = 0.0;
    bool bad = false;
    if (r < n) {
        const float* xr = x + r * d;
        float* q = b.xq + r * kp;
        double nc = 0.0;  // norm of the stored (centred) copy
        auto one = [&](float v, int k) -> float {
            bad |= !isfinite(v);
            nv += double(v) * double(v);
            const float c = b.mu ? float(double(v) - b.mu[k]) : v;
            nc += double(c) * double(c);
            return c;
        };
        if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
            // 16-byte pieces (same values and summation order as below)
            const float4* __restrict__ x4 = reinterpret_cast<const float4*>(xr);
            float4* q4 = reinterpret_cast<float4*>(q);
            for (int k4 = 0; k4 < d / 4; ++k4) {
                const float4 v = x4[k4];
                float4 c;
                c.x = one(v.x, 4 * k4);
                c.y = one(v.y, 4 * k4 + 1);
                c.z = one(v.z, 4 * k4 + 2);
                c.w = one(v.w, 4 * k4 + 3);
                q4[k4] = c;
            }
        } else {
            for (int k = 0; k < d; ++k) q[k] = one(xr[k], k);
        }
        for (int k = d; k < kp; ++k) q[k] = 0.0f;
        const float hn = float(0.5 * nc);
        b.n64[r] = nv;
        b.m0[r] = nv;
        b.m64[r] = nv;
        b.hn[r] = hn;
        b.ha[r] = float(0.5 * nv - double(hn));
        b.hm[r] = float(0.5 * nv);
        b.selected[r] = 0;
    } else {
        float* q = b.xq + r * kp;
        for (int k = 0; k < kp; ++k) q[k] = 0.0f;
        b.n64[r] = 0.0;
        b.m0[r] = 0.0;
        b.m64[r] = 0.0;
        b.hn[r] = 0.0f;
        b.ha[r] = 0.0f;
        b.hm[r] = 0.0f;
        b.selected[r] = 1;  // padding is never a candidate
    }
    if (bad) atomicCAS(&b.state->error, 0, kDevErrNonFinite);
    red[threadIdx.x] = nv;
    rmax[threadIdx.x] = nv;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        b.fpart[blockIdx.x] = red[0];
        b.bmax[blockIdx.x] = rmax[0];
    }
}

// L1 datasets: one thread per padded row. The L1 kernels read the caller's
// float32 rows directly, so no distance-dtype copy is written; the float64
// d(v, 0) = sum_k |v_k| gives the initial state m_v and L({e0}), and the
// finiteness check is the same as for the squared distance.
__global__ void __launch_bounds__(kBlock) k_prep_l1(const float* __restrict__ x, int64_t n, int32_t d, Buffers b) {
    __shared__ double red[kBlock];
    __shared__ double rmax[kBlock];
    const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double nv = 0.0;
    if (r < n) {
        const float* xr = x + r * d;
        bool bad = false;
        for (int k = 0; k < d; ++k) {
            const float v = xr[k];
            bad |= !isfinite(v);
            nv += fabs(double(v));
        }
        if (bad) atomicCAS(&b.state->error, 0, kDevErrNonFinite);
        b.n64[r] = nv;
        b.m0[r] = nv;
        b.m64[r] = nv;
        b.hn[r] = 0.0f;
        b.selected[r] = 0;
        set_point_terms(b, r, nv);
    } else {
        b.n64[r] = 0.0;
        b.m0[r] = 0.0;
        b.m64[r] = 0.0;
        b.hn[r] = 0.0f;
        b.ha[r] = 0.0f;
        b.hm[r] = 0.0f;
        b.selected[r] = 1;  // padding is never a candidate
    }
    red[threadIdx.x] = nv;
    rmax[threadIdx.x] = nv;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        b.fpart[blockIdx.x] = red[0];
        b.bmax[blockIdx.x] = rmax[0];
    }
}

// Reduced-precision copy: one thread per padded row. Exact float64 norm and
// initial state as in k_prep, then the row (long rows: centred at the column
// means) cast with round-to-nearest-even
// (FP8: after a power-of-two row scale) into the tiled layout, and the
// float32 norm of the cast row. FP16 values beyond its range raise
// EBC_E_RANGE.
__global__ void __launch_bounds__(kBlock) k_prep_lp(const float* __restrict__ x, int64_t n, int32_t d,
                                                    int32_t kp, int dt, Buffers b) {
    __shared__ double red[kBlock];
    __shared__ double rmax[kBlock];
    const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double nv = 0.0;
    if (r < n) {
        const float* xr = x + r * d;
        // value cast at column k (long rows: centred at the column mean)
        auto cv = [&](int k) -> float { return b.mu ? float(double(xr[k]) - b.mu[k]) : xr[k]; };
        bool bad = false, range = false;
        float amax = 0.0f;
        for (int k = 0; k < d; ++k) {
            const float v = xr[k];
            bad |= !isfinite(v);
            nv += double(v) * double(v);
            amax = fmaxf(amax, fabsf(cv(k)));
        }
        double nq = 0.0;  // norm of the cast row
        const int eb = dt == EBC_DT_FP8_E4M3 ? 1 : 2;
        const int ru = kp * eb / 16;
        uint8_t* base = reinterpret_cast<uint8_t*>(b.xq);
        if (dt == EBC_DT_FP8_E4M3) {
            int se = 0;  // scale exponent: ceil(log2(amax / 448))
            if (amax > 0.0f) {
                int e;
                const float m = frexpf(amax / 448.0f, &e);
                se = (m == 0.5f) ? e - 1 : e;
                se = se < -126 ? -126 : (se > 126 ? 126 : se);
            }
            b.scale[r] = 127 + se;
            for (int k = 0; k < kp; ++k) {
                uint8_t c = 0;
                if (k < d) {
                    c = f32_to_e4m3_rne(ldexpf(cv(k), -se));
                    const double xv = ldexp(double(e4m3_to_f32(c)), se);
                    nq += xv * xv;
                }
                base[tiled_offset(r, k, ru)] = c;
            }
        } else {
            for (int k = 0; k < kp; ++k) {
                uint16_t c = 0;
                if (k < d) {
                    float back;
                    if (dt == EBC_DT_BF16) {
                        c = f32_to_bf16_rne(cv(k));
                        back = bf16_to_f32(c);
                    } else {
                        range |= fabsf(cv(k)) > 65504.0f;
                        const _Float16 h = _Float16(cv(k));
                        c = __builtin_bit_cast(uint16_t, h);
                        back = float(h);
                    }
                    nq += double(back) * double(back);
                }
                *reinterpret_cast<uint16_t*>(base + tiled_offset(r, 2 * k, ru)) = c;
            }
        }
        if (bad) atomicCAS(&b.state->error, 0, kDevErrNonFinite);
        if (range) atomicCAS(&b.state->error, 0, int(EBC_E_RANGE));
        b.hn[r] = float(0.5 * nq);
        b.n64[r] = nv;
        b.m0[r] = nv;
        b.m64[r] = nv;
        b.selected[r] = 0;
        Buffers own = b;  // the grouped order does not exist yet: k_group_copy fills the slot-order terms
        own.inv = nullptr;
        set_point_terms(own, r, nv);
    } else {
        const int eb = dt == EBC_DT_FP8_E4M3 ? 1 : 2;
        const int ru = kp * eb / 16;
        uint8_t* base = reinterpret_cast<uint8_t*>(b.xq);
        for (int k = 0; k < kp * eb; ++k) base[tiled_offset(r, k, ru)] = 0;
        if (b.scale) b.scale[r] = 127;
        b.n64[r] = 0.0;
        b.m0[r] = 0.0;
        b.m64[r] = 0.0;
        b.hn[r] = 0.0f;
        b.ha[r] = 0.0f;
        b.hm[r] = 0.0f;
        b.selected[r] = 1;
    }
    red[threadIdx.x] = nv;
    rmax[threadIdx.x] = nv;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        b.fpart[blockIdx.x] = red[0];
        b.bmax[blockIdx.x] = rmax[0];
    }
}

// ---- grouped order of the reduced-precision gains ----
// The ground set is sorted by nearest pivot (pivot j = row j * (n / G) of V,
// G = group_count(n) pivots; squared Euclidean distance in float32 on the
// caller's rows, ties to the lowest pivot), stably (equal pivots keep row
// order), so the order is a deterministic function of V. The gains kernel
// then walks candidates and points in this slot order; a pair's distance and
// a candidate's gain do not depend on the order, only which 32 x 32 tiles
// group them (and so the float32 summation order of each gain) does.
constexpr int kPivChunk = 32;  // pivots staged in LDS at a time

template <int KP>
__global__ void __launch_bounds__(kBlock) k_group_assign(const float* __restrict__ x, int64_t n, int32_t d,
                                                         int32_t groups, Buffers b) {
    __shared__ float piv[kPivChunk][KP];
    const int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const bool live = v < n;
    float xv[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) xv[k] = (live && k < d) ? x[v * d + k] : 0.0f;
    const int64_t stride = n / groups;
    float best = INFINITY;
    int arg = 0;
    for (int j0 = 0; j0 < groups; j0 += kPivChunk) {
        const int jn = (groups - j0) < kPivChunk ? (groups - j0) : kPivChunk;
        __syncthreads();
        for (int e = threadIdx.x; e < kPivChunk * KP; e += kBlock) {
            const int j = e / KP, k = e % KP;
            piv[j][k] = (j < jn && k < d) ? x[int64_t(j0 + j) * stride * d + k] : 0.0f;
        }
        __syncthreads();
        for (int j = 0; j < jn; ++j) {
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const float t = xv[k] - piv[j][k];
                s = fmaf(t, t, s);
            }
            if (s < best) {
                best = s;
                arg = j0 + j;
            }
        }
    }
    b.gbucket[v] = live ? arg : -1;
}

// Per block of 256 rows: how many rows of the block fall in each bucket.
__global__ void __launch_bounds__(kBlock) k_group_count(int32_t groups, Buffers b) {
    __shared__ int hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int g = b.gbucket[int64_t(blockIdx.x) * kBlock + threadIdx.x];
    if (g >= 0) atomicAdd(&hist[g], 1);
    __syncthreads();
    if (int(threadIdx.x) < groups) b.gcount[int64_t(blockIdx.x) * groups + threadIdx.x] = hist[threadIdx.x];
}

// One workgroup: bucket totals, their exclusive prefix (bucket-major slot
// ranges), then each (block, bucket) count replaced by its first slot.
__global__ void __launch_bounds__(kBlock) k_group_scan(int32_t nblocks, int32_t groups, Buffers b) {
    __shared__ int tot[256];
    const int g = threadIdx.x;
    int t = 0;
    if (g < groups)
        for (int blk = 0; blk < nblocks; ++blk) t += b.gcount[int64_t(blk) * groups + g];
    tot[g] = t;
    __syncthreads();
    if (g == 0) {
        int run = 0;
        for (int q = 0; q < 256; ++q) {
            const int c = tot[q];
            tot[q] = run;
            run += c;
        }
    }
    __syncthreads();
    if (g < groups) {
        int run = tot[g];
        for (int blk = 0; blk < nblocks; ++blk) {
            const int64_t i = int64_t(blk) * groups + g;
            const int c = b.gcount[i];
            b.gcount[i] = run;
            run += c;
        }
    }
}

// Slots: a row's slot is its (block, bucket) offset plus the number of
// earlier rows of the block in the same bucket (stable). Padding rows keep
// their own index.
__global__ void __launch_bounds__(kBlock) k_group_place(int64_t n, int32_t groups, Buffers b) {
    __shared__ int lb[kBlock];
    const int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const int g = b.gbucket[v];
    lb[threadIdx.x] = g;
    __syncthreads();
    if (v >= n) {
        b.perm[v] = int32_t(v);
        b.inv[v] = int32_t(v);
        return;
    }
    int rank = 0;
    for (int t = 0; t < int(threadIdx.x); ++t) rank += lb[t] == g ? 1 : 0;
    const int32_t slot = b.gcount[int64_t(blockIdx.x) * groups + g] + rank;
    b.perm[slot] = int32_t(v);
    b.inv[v] = slot;
}

// Slot-order copies: row perm[s] of the tiled distance-dtype copy (all of
// its 16-byte units) and its per-row terms go to slot s.
__global__ void __launch_bounds__(kBlock) k_group_copy(int32_t row_units, int32_t fp8, Buffers b) {
    const int64_t s = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t r = b.perm[s];
    const uint4* __restrict__ src = reinterpret_cast<const uint4*>(b.xq);
    uint4* __restrict__ dst = reinterpret_cast<uint4*>(b.xqp);
    for (int u = 0; u < row_units; ++u)
        dst[(s / 64 * row_units + u) * 64 + s % 64] = src[(r / 64 * row_units + u) * 64 + r % 64];
    b.hnp[s] = b.hn[r];
    b.hap[s] = b.ha[r];
    b.hmp[s] = b.hm[r];
    if (fp8) b.scp[s] = b.scale[r];
}

// Long rows: one workgroup of 16 waves per 64-row tile. Lane = row of the
// tile (the tiled stores of a wave cover whole 1 KB runs), wave = one of 16
// column slices (multiples of 16 columns); the per-slice float64 sums and
// maxima are combined through LDS in slice order. Pass 1: norm, finiteness
// and the largest centred magnitude (FP8 row scale); pass 2: the stored copy
// (centred at the column means, tiled in 16-byte units like the cast rows
// of every dtype, float32 included) and its norm.
// Per-block norm sums follow in k_norm_blocks. Same values as the one-thread-
// per-row kernels up to the order of the float64 norm sums.
constexpr int kPrepSlices = 16;

__device__ __forceinline__ float4 row4(const float* __restrict__ xr, int k, int d, bool vec) {
    if (vec && k < d) return *reinterpret_cast<const float4*>(xr + k);
    float4 v;
    v.x = k < d ? xr[k] : 0.0f;
    v.y = k + 1 < d ? xr[k + 1] : 0.0f;
    v.z = k + 2 < d ? xr[k + 2] : 0.0f;
    v.w = k + 3 < d ? xr[k + 3] : 0.0f;
    return v;
}

template <int DT>
__global__ void __launch_bounds__(1024) k_prep_wide(const float* __restrict__ x, int64_t n, int32_t d, int32_t kp,
                                                    Buffers b) {
    __shared__ double pn[kPrepSlices][64];
    __shared__ float pa[kPrepSlices][64];
    __shared__ int pf[kPrepSlices][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r = int64_t(blockIdx.x) * 64 + lane;
    const bool live = r < n;
    const int sw = ((kp + kPrepSlices - 1) / kPrepSlices + 15) / 16 * 16;  // columns per slice
    const int k0 = w * sw;
    const int k1 = (k0 + sw) < kp ? (k0 + sw) : kp;
    const float* __restrict__ xr = x + (live ? r : 0) * d;
    const double* __restrict__ mu = b.mu;
    const bool vec = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    auto cv = [&](float v, int k) -> float { return k < d ? float(double(v) - mu[k]) : 0.0f; };

    // pass 1: float64 norm, finiteness, largest centred magnitude
    double nv = 0.0;
    float amax = 0.0f;
    int bad = 0;
    if (live) {
        for (int k = k0; k < k1 && k < d; k += 4) {
            const float4 v4 = row4(xr, k, d, vec);
            const float v[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (k + i >= d) break;
                bad |= !isfinite(v[i]);
                nv += double(v[i]) * double(v[i]);
                if (DT == EBC_DT_FP8_E4M3) amax = fmaxf(amax, fabsf(cv(v[i], k + i)));
            }
        }
    }
    pn[w][lane] = nv;
    pa[w][lane] = amax;
    pf[w][lane] = bad;
    __syncthreads();
    double nvt = 0.0;
    float amt = 0.0f;
    int badt = 0;
#pragma unroll
    for (int q = 0; q < kPrepSlices; ++q) {
        nvt += pn[q][lane];
        amt = fmaxf(amt, pa[q][lane]);
        badt |= pf[q][lane];
    }
    __syncthreads();  // pn and pf are rewritten below

    // pass 2: the stored copy and its norm
    int se = 0;  // FP8 scale exponent: ceil(log2(amax / 448))
    if (DT == EBC_DT_FP8_E4M3 && amt > 0.0f) {
        int e;
        const float m = frexpf(amt / 448.0f, &e);
        se = (m == 0.5f) ? e - 1 : e;
        se = se < -126 ? -126 : (se > 126 ? 126 : se);
    }
    double nq = 0.0;
    int range = 0;
    if (DT == EBC_DT_F32) {
        // tiled like the cast rows: unit k/4 of row r (kp/4 units a row)
        float4* __restrict__ q4 = reinterpret_cast<float4*>(b.xq);
        const int64_t row_at = (r >> 6) * (kp / 4) * 64 + (r & 63);
        for (int k = k0; k < k1; k += 4) {
            float4 c = {0.0f, 0.0f, 0.0f, 0.0f};
            if (live) {
                const float4 v = row4(xr, k, d, vec);
                c.x = cv(v.x, k);
                c.y = cv(v.y, k + 1);
                c.z = cv(v.z, k + 2);
                c.w = cv(v.w, k + 3);
                nq += double(c.x) * double(c.x);
                nq += double(c.y) * double(c.y);
                nq += double(c.z) * double(c.z);
                nq += double(c.w) * double(c.w);
            }
            q4[row_at + int64_t(k / 4) * 64] = c;
        }
    } else {
        constexpr int eb = DT == EBC_DT_FP8_E4M3 ? 1 : 2;
        constexpr int per_unit = 16 / eb;  // columns per 16-byte unit
        const int ru = kp * eb / 16;
        uint8_t* base = reinterpret_cast<uint8_t*>(b.xq);
        for (int k = k0; k < k1; k += per_unit) {
            uint32_t wv[4] = {0u, 0u, 0u, 0u};
            if (live) {
#pragma unroll
                for (int j = 0; j < per_unit; j += 4) {
                    const float4 v4 = row4(xr, k + j, d, vec);
                    const float v[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int kk = k + j + i;
                        if (kk >= d) continue;
                        const float c = cv(v[i], kk);
                        uint32_t code;
                        double back;
                        if (DT == EBC_DT_FP8_E4M3) {
                            const uint8_t e8 = f32_to_e4m3_rne(ldexpf(c, -se));
                            back = ldexp(double(e4m3_to_f32(e8)), se);
                            code = e8;
                        } else if (DT == EBC_DT_BF16) {
                            const uint16_t h = f32_to_bf16_rne(c);
                            back = double(bf16_to_f32(h));
                            code = h;
                        } else {
                            range |= fabsf(c) > 65504.0f;
                            const _Float16 h = _Float16(c);
                            back = double(float(h));
                            code = __builtin_bit_cast(uint16_t, h);
                        }
                        nq += back * back;
                        const int bit = (j + i) * eb * 8;  // bit offset of column kk in the unit
                        wv[bit / 32] |= code << (bit % 32);
                    }
                }
            }
            *reinterpret_cast<uint4*>(base + tiled_offset(r, k * eb, ru)) = make_uint4(wv[0], wv[1], wv[2], wv[3]);
        }
    }
    pn[w][lane] = nq;
    pf[w][lane] = range;
    __syncthreads();
    if (w != 0) return;
    double nqt = 0.0;
    int ranget = 0;
#pragma unroll
    for (int q = 0; q < kPrepSlices; ++q) {
        nqt += pn[q][lane];
        ranget |= pf[q][lane];
    }
    if (live) {
        if (badt) atomicCAS(&b.state->error, 0, kDevErrNonFinite);
        if (ranget) atomicCAS(&b.state->error, 0, int(EBC_E_RANGE));
        if (DT == EBC_DT_FP8_E4M3) b.scale[r] = 127 + se;
        b.hn[r] = float(0.5 * nqt);
        b.n64[r] = nvt;
        b.m0[r] = nvt;
        b.m64[r] = nvt;
        b.selected[r] = 0;
        set_point_terms(b, r, nvt);
    } else {
        if (DT == EBC_DT_FP8_E4M3) b.scale[r] = 127;
        b.n64[r] = 0.0;
        b.m0[r] = 0.0;
        b.m64[r] = 0.0;
        b.hn[r] = 0.0f;
        b.ha[r] = 0.0f;
        b.hm[r] = 0.0f;
        b.selected[r] = 1;  // padding is never a candidate
    }
}

// Per-block sum and maximum of the float64 norms (the epilogue of k_prep).
__global__ void __launch_bounds__(kBlock) k_norm_blocks(Buffers b) {
    __shared__ double red[kBlock];
    __shared__ double rmax[kBlock];
    const double nv = b.n64[int64_t(blockIdx.x) * kBlock + threadIdx.x];
    red[threadIdx.x] = nv;
    rmax[threadIdx.x] = nv;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        b.fpart[blockIdx.x] = red[0];
        b.bmax[blockIdx.x] = rmax[0];
    }
}

// Raise DevState::gexp so that 2^gexp >= mmax / 2 (0 <= gexp <= 126, so the
// scale 2^-gexp stays a normal float). Atomic: blocks of k_load_m race.
__device__ inline void raise_gexp(DevState* st, double mmax) {
    int e = 0;
    if (mmax > 0.0) (void)frexp(0.5 * mmax, &e);  // 0.5 mmax < 2^e
    if (!(mmax <= 1.0e300)) e = 126;             // non-finite (reported elsewhere) or huge
    e = e < 0 ? 0 : (e > 126 ? 126 : e);
    atomicMax(&st->gexp, e);
}

// One block: L({e0}) = |V|^-1 sum of the per-block norm sums (fixed order),
// and the largest norm.
__global__ void __launch_bounds__(kBlock) k_l0(int64_t n, int32_t nblocks, Buffers b) {
    __shared__ double red[kBlock];
    __shared__ double rmax[kBlock];
    double s = 0.0, mx = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += kBlock) {
        s += b.fpart[i];
        mx = fmax(mx, b.bmax[i]);
    }
    red[threadIdx.x] = s;
    rmax[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        b.state->l0 = red[0] / double(n);
        b.state->nmax = rmax[0];
        raise_gexp(b.state, rmax[0]);
    }
}

__global__ void k_state_init(DevState* st) {
    if (threadIdx.x == 0) {
        st->error = 0;
        st->window_count = 0;
        st->window_max = 0;
        st->window_overflow = 0;
        st->cstar = -1;
        st->pad0 = 0;
        st->gstar = 0.0;
        st->l0 = 0.0;
        st->tau = 0.0;
        st->tau_abs = 0.0;
        st->nmax = 0.0;
        st->gexp = 0;
        st->pad1 = 0;
    }
}

hipError_t launch_prep(const ebc_dataset* ds, hipStream_t s) {
    const int nb = int(ds->n_pad / kBlock);
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, ds->b.state);
    if (ds->metric == 1) {
        hipLaunchKernelGGL(k_prep_l1, dim3(nb), dim3(kBlock), 0, s, ds->x, ds->n, ds->d, ds->b);
        hipLaunchKernelGGL(k_l0, dim3(1), dim3(kBlock), 0, s, ds->n, nb, ds->b);
        return hipGetLastError();
    }
    if (ds->b.mu)
        hipLaunchKernelGGL(k_colmean, dim3(unsigned((ds->k_pad + 63) / 64)), dim3(1024), 0, s, ds->x, ds->n, ds->d,
                           ds->k_pad, ds->b.mu);
    if (wide_rows(ds->k_pad)) {
        const dim3 g = dim3(unsigned(ds->n_pad / 64)), blk = dim3(64 * kPrepSlices);
        switch (ds->dt) {
            case EBC_DT_F32:
                hipLaunchKernelGGL(k_prep_wide<EBC_DT_F32>, g, blk, 0, s, ds->x, ds->n, ds->d, ds->k_pad, ds->b);
                break;
            case EBC_DT_BF16:
                hipLaunchKernelGGL(k_prep_wide<EBC_DT_BF16>, g, blk, 0, s, ds->x, ds->n, ds->d, ds->k_pad, ds->b);
                break;
            case EBC_DT_F16:
                hipLaunchKernelGGL(k_prep_wide<EBC_DT_F16>, g, blk, 0, s, ds->x, ds->n, ds->d, ds->k_pad, ds->b);
                break;
            default:
                hipLaunchKernelGGL(k_prep_wide<EBC_DT_FP8_E4M3>, g, blk, 0, s, ds->x, ds->n, ds->d, ds->k_pad,
                                   ds->b);
                break;
        }
        hipLaunchKernelGGL(k_norm_blocks, dim3(nb), dim3(kBlock), 0, s, ds->b);
    } else if (ds->dt == EBC_DT_F32)
        hipLaunchKernelGGL(k_prep, dim3(nb), dim3(kBlock), 0, s, ds->x, ds->n, ds->d, ds->k_pad, ds->b);
    else
        hipLaunchKernelGGL(k_prep_lp, dim3(nb), dim3(kBlock), 0, s, ds->x, ds->n, ds->d, ds->k_pad, int(ds->dt),
                           ds->b);
    if (ds->b.perm) {
        const int32_t groups = group_count(ds->n);
        const int kp8 = (ds->d + 7) / 8 * 8;  // float32 row length held in registers
        switch (kp8) {
#define EBC_GA(K)                                                                                             \
    case K:                                                                                                   \
        hipLaunchKernelGGL(k_group_assign<K>, dim3(nb), dim3(kBlock), 0, s, ds->x, ds->n, ds->d, groups, ds->b); \
        break;
            EBC_GA(8) EBC_GA(16) EBC_GA(24) EBC_GA(32) EBC_GA(40) EBC_GA(48) EBC_GA(56) EBC_GA(64)
            EBC_GA(72) EBC_GA(80) EBC_GA(88) EBC_GA(96) EBC_GA(104) EBC_GA(112) EBC_GA(120) EBC_GA(128)
#undef EBC_GA
            default: return hipErrorInvalidValue;
        }
        hipLaunchKernelGGL(k_group_count, dim3(nb), dim3(kBlock), 0, s, groups, ds->b);
        hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(kBlock), 0, s, nb, groups, ds->b);
        hipLaunchKernelGGL(k_group_place, dim3(nb), dim3(kBlock), 0, s, ds->n, groups, ds->b);
        const int32_t row_units = ds->k_pad * elem_bytes(ds->dt) / 16;
        hipLaunchKernelGGL(k_group_copy, dim3(nb), dim3(kBlock), 0, s, row_units,
                           int32_t(ds->dt == EBC_DT_FP8_E4M3), ds->b);
    }
    hipLaunchKernelGGL(k_l0, dim3(1), dim3(kBlock), 0, s, ds->n, nb, ds->b);
    return hipGetLastError();
}

// Greedy restart: m_v = d(v, e0), nothing selected, window counters cleared.
__device__ void reset_body(const InstDesc& c, int64_t blk) {
    const Buffers& b = c.b;
    const int64_t r = blk * kBlock + threadIdx.x;
    if (r < c.n) {
        const double nv = b.m0[r];
        b.m64[r] = nv;
        set_point_terms(b, r, nv);
        b.selected[r] = 0;
    }
    if (r == 0) {
        b.state->window_count = 0;
        b.state->window_max = 0;
        b.state->window_overflow = 0;
        b.state->cstar = -1;
        b.state->gstar = 0.0;
        b.state->tau = window_tau(ebc_dtype(c.dt));
        b.state->tau_abs = window_tau_abs(ebc_dtype(c.dt));
    }
}

__global__ void __launch_bounds__(kBlock) k_reset(InstDesc c) { reset_body(c, blockIdx.x); }

__global__ void __launch_bounds__(kBlock)
kb_reset(const InstDesc* __restrict__ descs, const int64_t* __restrict__ row_pre, int32_t count) {
    const int i = find_slot(row_pre, count, blockIdx.x);
    const InstDesc c = descs[i];
    if (c.t0 == 0) reset_body(c, int64_t(blockIdx.x) - row_pre[i]);
}

hipError_t launch_reset_state(const ebc_dataset* ds, hipStream_t s) {
    InstDesc c;
    fill_desc(ds, 0, nullptr, nullptr, nullptr, &c);
    hipLaunchKernelGGL(k_reset, dim3(c.nb), dim3(kBlock), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_reset_batched(const InstDesc* descs, const int64_t* row_pre, int32_t count, int64_t total_rows,
                                hipStream_t s) {
    hipLaunchKernelGGL(kb_reset, dim3(unsigned(total_rows)), dim3(kBlock), 0, s, descs, row_pre, count);
    return hipGetLastError();
}

// The auxiliary vector e0 (Sec. 4: any fixed vector, the zero vector being
// the paper's example): d(v, e0) in float64 by direct differences (e0 null:
// ||v||^2), with per-block sums and maxima for L({e0}); a non-finite e0
// raises EBC_E_NONFINITE.
__global__ void __launch_bounds__(kBlock) k_set_e0(const float* __restrict__ x, int64_t n, int32_t d,
                                                   const float* __restrict__ e0, int32_t metric, Buffers b) {
    __shared__ float ce[EBC_MAX_DIM];
    __shared__ double red[kBlock];
    __shared__ double rmax[kBlock];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    if (e0)
        for (int k = threadIdx.x; k < d; k += kBlock) {
            ce[k] = e0[k];
            if (!isfinite(ce[k])) bad = 1;
        }
    __syncthreads();
    const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double mv = 0.0;
    if (r < n) {
        if (e0) {
            const float* xr = x + r * d;
            for (int k = 0; k < d; ++k) {
                const double t = double(xr[k]) - double(ce[k]);
                mv += metric == 1 ? fabs(t) : t * t;  // d(v, e0): L1 or squared Euclidean
            }
        } else {
            mv = b.n64[r];
        }
        b.m0[r] = mv;
    }
    if (threadIdx.x == 0 && blockIdx.x == 0 && bad) atomicCAS(&b.state->error, 0, kDevErrNonFinite);
    red[threadIdx.x] = mv;
    rmax[threadIdx.x] = mv;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        b.fpart[blockIdx.x] = red[0];
        b.bmax[blockIdx.x] = rmax[0];
    }
}

hipError_t launch_set_e0(const ebc_dataset* ds, const float* e0, hipStream_t s) {
    const int nb = int(ds->n_pad / kBlock);
    hipLaunchKernelGGL(k_set_e0, dim3(nb), dim3(kBlock), 0, s, ds->x, ds->n, ds->d, e0, ds->metric, ds->b);
    hipLaunchKernelGGL(k_l0, dim3(1), dim3(kBlock), 0, s, ds->n, nb, ds->b);
    return launch_reset_state(ds, s);
}

// Replace the running minima by a caller-supplied m (float64, [n]), and
// raise the gains scale exponent to cover the largest of them.
__global__ void __launch_bounds__(kBlock) k_load_m(int64_t n, const double* __restrict__ m, Buffers b) {
    __shared__ double rmax[kBlock];
    const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double mv = 0.0;
    if (r < n) {
        mv = m[r];
        b.m64[r] = mv;
        set_point_terms(b, r, mv);
    }
    rmax[threadIdx.x] = mv;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) raise_gexp(b.state, rmax[0]);
}

hipError_t launch_load_m(const ebc_dataset* ds, const double* m, hipStream_t s) {
    hipLaunchKernelGGL(k_load_m, dim3(ds->n_pad / kBlock), dim3(kBlock), 0, s, ds->n, m, ds->b);
    return hipGetLastError();
}

}  // namespace ebc
