// f(S_j) for many CSR-packed sets at once (Sec. 4.1: optimisers score a whole
// family S_multi = {S_1..S_l} per step; Alg. 1 gives f per set as a running
// minimum per ground point, a sum, and a division by |V|; Alg. 2 assigns the
// (set, point) cells of that computation to GPU threads).
//
// With e0 = 0 in every set, d(v,e0) = ||v||^2 = n_v and d(v,s) = n_v + n_s -
// 2 v.s, the per-point term of f is
//     n_v - min(n_v, min_{s in S} d(v,s)) = 2 max(0, max_{s in S} (v.s - n_s/2)),
// so f(S) = (2/|V|) sum_v max(0, max_{s in S} (v.s - n_s/2)): a dense
// contraction of set members against ground points (float32 on the matrix
// cores, v_mfma_f32_32x32x2_f32), a maximum over each set's members, a clamp
// at 0 and a sum over v. No (set, point) work matrix is ever written.
//
// Work decomposition. Each set's members are laid out in units of 4 rows
// (ceil(|S_j|/4) units, padding rows contribute -inf); units of consecutive
// sets follow each other, 8 units form a 32-row member block (in the MFMA
// result a unit is the 4 rows one lane half holds), and a group is every set
// whose first unit lies in one window of 64 units. A work item is (group,
// ground-set split); a workgroup (4 waves) walks the group's member blocks
// through a double-buffered LDS stage (the next block's rows are gathered
// into registers while the current one is multiplied) while each wave holds
// 64 ground points in registers, and keeps a running maximum per (set,
// point) across the set's units (also across blocks, so sets of any size
// work). At each set's last unit the two lane halves are joined, clamped at
// 0 and added to the lane's float accumulator of that set; float64 sums over
// the lanes and waves, and a final pass over the splits, run in a fixed
// order, so the result does not depend on the schedule.
#include <math.h>

#include "ebc_internal.h"
#include "lp_mfma.h"
#include "wide_row.h"

namespace ebc {

namespace {

constexpr int kUnitRows = 4;    // rows per unit
constexpr int kBlockUnits = 8;  // units per 32-row member block
constexpr int kWindow = 64;     // units per group window (float32 kernel)
// units per group window of the reduced-precision kernel: its resident
// member rows and per-set column sums stay within about 64 KB of LDS
constexpr int lp_window(int dt, int kc) { return 2 * kc * (dt == EBC_DT_FP8_E4M3 ? 2 : 1) <= 8 ? 64 : 32; }
constexpr int kVSub = 256;      // ground points per workgroup pass (4 waves x 64)
constexpr int kMaxSplits = 16;

// Scratch of one call: unit prefix U[l+1], non-empty prefix E[l+1], set
// status (0 ok, 1 bad), counts (n_groups[0]: group windows; [1], [2], [3]:
// window width, window count and rows per unit of the register kernels), per-split partial sums
// [splits][l], first set of each register-kernel window [l+2].
struct EsScratch {
    int64_t* U;
    int32_t* E;
    int32_t* bad;
    int64_t* n_groups;
    double* part;
    int32_t* win_j0;  // [l + 2]: first set of each window of the register kernel
};

// One thread per set: validate the offsets and indices, count the units.
__global__ void __launch_bounds__(256) k_es_units(const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
                                                   int64_t l, int64_t n, EsScratch sc, DevState* st) {
    const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (j >= l) return;
    const int64_t a = off[j], z = off[j + 1];
    int bad = 0;
    if (a < 0 || z < a || z > off[l]) bad = 1;
    else
        for (int64_t q = a; q < z; ++q)
            if (idx[q] < 0 || int64_t(idx[q]) >= n) {
                bad = 1;
                break;
            }
    if (bad) atomicCAS(&st->error, 0, kDevErrIndex);
    sc.bad[j] = bad;
    sc.U[j + 1] = bad ? 0 : (z - a + kUnitRows - 1) / kUnitRows;  // counts, scanned next
    sc.E[j + 1] = (!bad && z > a) ? 1 : 0;
}

// Single workgroup: inclusive scans of the unit and non-empty counts (in
// place, U[0] = E[0] = 0), and the number of group windows. Also, for the
// kernels that keep member rows in registers: when no set has more than
// kRegMaxSet units, their window width G = kRegUnits + 1 - (the largest
// set's units) and window count (sets whose first unit lies in [w G, (w+1) G)
// go to wave window w, which then spans at most kRegUnits units); else 0
// windows (those kernels stand aside). n_groups[3] holds the rows per unit of
// the windows: 4, or 2 when reg2 is set (a float32 call on the dataset's own
// rows) and every non-empty set has kReg2MinRows .. 32 members. Then the
// counts are rescanned as 2-row units and a window holds 32 of them: sets of
// 10 members fill 10 rows instead of 12, and windows hold more whole sets.
constexpr int kRegUnits = 16;  // units per wave window of the register kernel (two 32-row blocks)
constexpr int kRegMaxSet = 8;  // largest set (units) it takes: then G >= 9 and there are at most l windows
constexpr int kReg2Units = 32;    // 2-row units per window (the same two 32-row blocks)
constexpr int kReg2MaxSet = 16;   // largest set in 2-row units (32 members)
constexpr int kReg2MinRows = 3;   // smallest set: 2 units, so set ends are at least 2 units apart

__global__ void __launch_bounds__(1024) k_es_scan(int64_t l, int32_t window, EsScratch sc,
                                                   const int64_t* __restrict__ off, int32_t reg2) {
    __shared__ int64_t su[1024];
    __shared__ int32_t se[1024];
    __shared__ int64_t carry_u;
    __shared__ int32_t carry_e;
    __shared__ int64_t umax[1024];
    __shared__ int64_t umin[1024];
    const int t = threadIdx.x;
    if (t == 0) {
        carry_u = 0;
        carry_e = 0;
        sc.U[0] = 0;
        sc.E[0] = 0;
    }
    // 2-row units: only if every non-empty valid set has 3 .. 32 members
    bool two = false;
    if (reg2) {
        int64_t lo = INT64_MAX, hi = 0;
        for (int64_t j = t; j < l; j += 1024) {
            if (sc.bad[j]) continue;
            const int64_t z = off[j + 1] - off[j];
            if (z == 0) continue;
            if (z < lo) lo = z;
            if (z > hi) hi = z;
        }
        umin[t] = lo;
        umax[t] = hi;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if (t < w) {
                if (umax[t + w] > umax[t]) umax[t] = umax[t + w];
                if (umin[t + w] < umin[t]) umin[t] = umin[t + w];
            }
            __syncthreads();
        }
        two = umax[0] >= kReg2MinRows && umax[0] <= 2 * kReg2MaxSet && umin[0] >= kReg2MinRows;
        if (two)  // the same thread reads these counts in the scan below
            for (int64_t j = t; j < l; j += 1024)
                sc.U[j + 1] = sc.bad[j] ? 0 : (off[j + 1] - off[j] + 1) / 2;
        __syncthreads();
    }
    const int64_t cap = two ? kReg2Units : kRegUnits;
    const int64_t max_set = two ? kReg2MaxSet : kRegMaxSet;
    int64_t my_max = 0;
    __syncthreads();
    for (int64_t base = 0; base < l; base += 1024) {
        const int64_t j = base + t;
        su[t] = j < l ? sc.U[j + 1] : 0;
        se[t] = j < l ? sc.E[j + 1] : 0;
        if (su[t] > my_max) my_max = su[t];
        __syncthreads();
        for (int w = 1; w < 1024; w <<= 1) {
            const int64_t u = t >= w ? su[t - w] : 0;
            const int32_t e = t >= w ? se[t - w] : 0;
            __syncthreads();
            su[t] += u;
            se[t] += e;
            __syncthreads();
        }
        if (j < l) {
            sc.U[j + 1] = carry_u + su[t];
            sc.E[j + 1] = carry_e + se[t];
        }
        __syncthreads();
        if (t == 1023) {
            carry_u += su[1023];
            carry_e += se[1023];
        }
        __syncthreads();
    }
    umax[t] = my_max;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w && umax[t + w] > umax[t]) umax[t] = umax[t + w];
        __syncthreads();
    }
    const int64_t mx = umax[0];
    const int64_t G = cap + 1 - mx;
    const bool fits = mx >= 1 && mx <= max_set;
    const int64_t n_win = fits ? (carry_u + G - 1) / G : 0;
    if (t == 0) {
        sc.n_groups[0] = (carry_u + window - 1) / window;
        sc.n_groups[1] = fits ? G : 0;
        sc.n_groups[2] = n_win;
        sc.n_groups[3] = two ? 2 : kUnitRows;
    }
    // first set of every window: window w starts at the first set whose first
    // unit is at or after w G (set j owns the windows w with U[j-1] < w G <= U[j]);
    // windows past the last set's start, and the end marker n_win, get l
    if (fits)
        for (int64_t j = t; j <= l; j += 1024) {
            const int64_t w_lo = j == 0 ? 0 : sc.U[j - 1] / G + 1;
            const int64_t w_hi = j == l ? n_win : sc.U[j] / G;
            for (int64_t w = w_lo; w <= w_hi && w <= n_win; ++w) sc.win_j0[w] = int32_t(j);
        }
}

// first j in [lo, hi) with U[j] >= key (hi if none)
__device__ __forceinline__ int64_t lower_bound_u(const int64_t* __restrict__ U, int64_t lo, int64_t hi,
                                                 int64_t key) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (U[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// the set that owns unit u: last j in [lo, hi) with U[j] <= u
__device__ __forceinline__ int64_t owner_of(const int64_t* __restrict__ U, int64_t lo, int64_t hi, int64_t u) {
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (U[mid] <= u)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Row and unit bookkeeping of one 32-row member block.
struct BlockInfo {
    int32_t row_mem[32];             // member row of V, -1 for padding
    float row_c[32];                 // -n_s/2, or -inf for padding
    int32_t row_sc[32];              // E8M0 row scale (FP8 rows; 127 otherwise)
    int32_t unit_flags[kBlockUnits];  // bit0 first unit of its set, bit1 last, bit2 valid
    int32_t unit_local[kBlockUnits];  // the set's index within the group
};

// Set table of the current group: U, E and offsets of sets j0 .. j1, cached
// in LDS when the group has at most kTab sets (else read from global memory).
constexpr int kTab = 128;

struct SetTable {
    const int64_t* U;
    const int32_t* E;
    const int64_t* off;
    int64_t base;  // global index of entry 0
};

// Threads 0..31 fill the rows, threads 32..39 the units of block blk.
// Norms: n64 (float64 ||s||^2 of the float32 rows) when hn is null, else hn
// (float32 ||s^||^2 / 2 of the cast rows); sc: FP8 row scales or null.
__device__ __forceinline__ void block_info(int tid, int64_t blk, int64_t u0, int64_t u1, int64_t j0, int64_t j1,
                                           const SetTable& tb, const int32_t* __restrict__ idx,
                                           const double* __restrict__ n64, const float* __restrict__ hn,
                                           const int* __restrict__ sc, BlockInfo& bi) {
    if (tid < 32) {
        const int64_t u = u0 + blk * kBlockUnits + tid / kUnitRows;
        int32_t mem = -1;
        if (u < u1) {
            const int64_t j = owner_of(tb.U, j0 - tb.base, j1 - tb.base, u);
            const int64_t q = (u - tb.U[j]) * kUnitRows + tid % kUnitRows;
            if (tb.off[j] + q < tb.off[j + 1]) mem = idx[tb.off[j] + q];
        }
        bi.row_mem[tid] = mem;
        bi.row_c[tid] = mem < 0 ? -INFINITY : (hn ? -hn[mem] : -float(0.5 * n64[mem]));
        bi.row_sc[tid] = (mem >= 0 && sc) ? sc[mem] : 127;
    } else if (tid < 32 + kBlockUnits) {
        const int uu = tid - 32;
        const int64_t u = u0 + blk * kBlockUnits + uu;
        int flags = 0, loc = 0;
        if (u < u1) {
            const int64_t j = owner_of(tb.U, j0 - tb.base, j1 - tb.base, u);
            flags = 4 | (u == tb.U[j] ? 1 : 0) | (u == tb.U[j + 1] - 1 ? 2 : 0);
            loc = tb.E[j] - tb.E[j0 - tb.base];
        }
        bi.unit_flags[uu] = flags;
        bi.unit_local[uu] = loc;
    }
}

// Units of 4 rows of one member block against this wave's 64 points: unit
// uu is held by lane half uu%2 in result registers 4*(uu/2) .. +3. Running
// maximum per (set, point) in cur (per 32-point block); at a set's last unit
// the two lane halves are joined, shifted by the point's wsh (below), clamped
// at 0, and each column's value is added to the lane's own float accumulator
// of that set (lacc[wave][set][col]; the final pass sums them in float64 in
// a fixed order).
//
// wsh: with a general auxiliary vector e0 (and, for the cast rows, norms
// that are not those of the exact rows) the per-point term is
//     n_v - min(n_v, d(v,s)) = 2 max(0, v.s - ||s||^2/2 + (n_v - ||v||^2)/2)
// with n_v = d(v, e0); the last part is the per-point shift wsh (0 for the
// float32 rows when e0 = 0).
template <int WIN>
__device__ __forceinline__ void es_units(const floatx16 (&acc)[2], const int32_t* unit_flags, const int32_t* unit_local,
                                         const float (&wsh)[2], float (&cur)[2], int half, int col,
                                         float (&lacc)[WIN][32]) {
    // the block's unit bookkeeping (the same for every lane) read up front
    int fl[kBlockUnits], lo[kBlockUnits];
#pragma unroll
    for (int uu = 0; uu < kBlockUnits; ++uu) {
        fl[uu] = unit_flags[uu];
        lo[uu] = unit_local[uu];
    }
    // each lane's maximum over the 4 rows of each register group: in group g,
    // half 0 holds unit 2g and half 1 unit 2g+1; the other half's lanes see -inf
    float mg[2][kBlockUnits];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int g = 0; g < kBlockUnits / 2; ++g) {
            const float m = fmaxf(fmaxf(acc[cb][4 * g + 0], acc[cb][4 * g + 1]),
                                  fmaxf(acc[cb][4 * g + 2], acc[cb][4 * g + 3]));
            mg[cb][2 * g] = half == 0 ? m : -INFINITY;
            mg[cb][2 * g + 1] = half == 1 ? m : -INFINITY;
        }
#pragma unroll
    for (int uu = 0; uu < kBlockUnits; ++uu) {
        const int flags = __builtin_amdgcn_readfirstlane(fl[uu]);
        if (!(flags & 4)) continue;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) cur[cb] = fmaxf((flags & 1) ? -INFINITY : cur[cb], mg[cb][uu]);
        if (__builtin_expect((flags & 2) != 0, 0)) {  // a set's last unit (about one in three)
            float sv = 0.0f;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) sv += fmaxf(fmaxf(cur[cb], __shfl_xor(cur[cb], 32, 64)) + wsh[cb], 0.0f);
            if (half == 0) lacc[__builtin_amdgcn_readfirstlane(lo[uu])][col] += sv;
        }
    }
}

// Per non-empty set of the group: float64 sum of the per-lane accumulators
// over the waves and columns (fixed order), one write per set and split.
template <int WIN>
__device__ __forceinline__ void es_finish(int tid, int64_t j0, int64_t j1, int split, int64_t l, const EsScratch& sc,
                                          const float (&lacc)[4][WIN][32]) {
    for (int64_t j = j0 + tid; j < j1; j += 256) {
        if (sc.E[j + 1] == sc.E[j]) continue;
        const int loc = int(sc.E[j] - sc.E[j0]);
        double t = 0.0;
        for (int w = 0; w < 4; ++w)
            for (int c = 0; c < 32; ++c) t += double(lacc[w][loc][c]);
        sc.part[int64_t(split) * l + j] = t;
    }
}

template <int KP, bool TRIM>
__global__ void __launch_bounds__(256)
k_es_main(const float* __restrict__ x, int64_t n, int32_t d, const double* __restrict__ n64,
          const double* __restrict__ m0, const int64_t* __restrict__ off, const int32_t* __restrict__ idx, int64_t l, int32_t splits,
          EsScratch sc, int32_t after_regs) {
    // after k_es_regs32: that kernel took the call if every set fits its windows
    if (after_regs && sc.n_groups[2] > 0) return;
    constexpr int KH = KP / 2;  // K values per lane half
    constexpr int S = KP + 4;   // LDS row stride (S/4 odd: conflict-free 16-byte reads)
    constexpr int PF = KP / 8;  // member-row values each thread gathers per block
    static_assert(KP % 8 == 0, "row length must be a multiple of 8");
    // TRIM (d <= KP - 4): the last 4 K values of lane half 1 are padding, so
    // the last K group pairs values KH-4, KH-3 (half 0) with KH-2, KH-1
    // (half 1) in 2 MFMAs instead of 4
    constexpr int QF = TRIM ? KH / 4 - 1 : KH / 4;
    __shared__ float4 lds_m4[2][32 * S / 4];
    __shared__ BlockInfo info[3];
    __shared__ int64_t t_u[kTab + 1], t_off[kTab + 1];
    __shared__ int32_t t_e[kTab + 1];
    __shared__ float lacc[4][kWindow][32];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 31;
    const int half = lane >> 5;
    const int grow = tid >> 3;  // gather: row and first column of this thread
    const int gk = tid & 7;
    const int64_t n_items = *sc.n_groups * splits;
    const int64_t vchunk = ((n + splits - 1) / splits + kVSub - 1) / kVSub * kVSub;

    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t g = item / splits;
        const int split = int(item % splits);
        // sets whose first unit lies in window g (empty sets own no unit)
        const int64_t j0 = lower_bound_u(sc.U, 0, l, g * kWindow);
        const int64_t j1 = lower_bound_u(sc.U, j0, l, (g + 1) * kWindow);
        const int64_t u0 = sc.U[j0], u1 = sc.U[j1];
        const int64_t v_begin = int64_t(split) * vchunk;
        int64_t v_end = v_begin + vchunk;
        if (v_end > n) v_end = n;
        const bool cached = j1 - j0 <= kTab;
        if (cached)
            for (int64_t i = tid; i <= j1 - j0; i += 256) {
                t_u[i] = sc.U[j0 + i];
                t_e[i] = sc.E[j0 + i];
                t_off[i] = off[j0 + i];
            }
        for (int i = tid; i < 4 * kWindow * 32; i += 256) (&lacc[0][0][0])[i] = 0.0f;
        __syncthreads();
        const SetTable tb = cached ? SetTable{t_u, t_e, t_off, j0} : SetTable{sc.U, sc.E, off, 0};
        if (u1 > u0 && v_end > v_begin) {
            const int64_t nblk = (u1 - u0 + kBlockUnits - 1) / kBlockUnits;
            for (int64_t vs = v_begin; vs < v_end; vs += kVSub) {
                // this wave's 64 ground points (B operand), K split in lane halves
                float b[2][KH];
                float wsh[2];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const int64_t v = vs + wave * 64 + cb * 32 + col;
                    const bool ok = v < v_end;
                    wsh[cb] = ok ? float(0.5 * (m0[v] - n64[v])) : 0.0f;
                    if (d % 4 == 0) {
                        // rows 16-byte aligned: 4 values per load; a 4-group is
                        // either wholly inside the row or wholly padding
#pragma unroll
                        for (int s4 = 0; s4 < QF; ++s4) {
                            const int k = half * KH + 4 * s4;
                            float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                            if (ok && k < d) q = *reinterpret_cast<const float4*>(x + v * d + k);
                            b[cb][4 * s4 + 0] = q.x;
                            b[cb][4 * s4 + 1] = q.y;
                            b[cb][4 * s4 + 2] = q.z;
                            b[cb][4 * s4 + 3] = q.w;
                        }
                    } else {
#pragma unroll
                        for (int s = 0; s < 4 * QF; ++s) {
                            const int k = half * KH + s;
                            b[cb][s] = (ok && k < d) ? x[v * d + k] : 0.0f;
                        }
                    }
                    if constexpr (TRIM) {
                        const int k = half ? KH - 2 : KH - 4;
                        b[cb][KH - 4] = (ok && k < d) ? x[v * d + k] : 0.0f;
                        b[cb][KH - 3] = (ok && k + 1 < d) ? x[v * d + k + 1] : 0.0f;
                        b[cb][KH - 2] = 0.0f;
                        b[cb][KH - 1] = 0.0f;
                    }
                }
                float cur[2] = {-INFINITY, -INFINITY};
                // prologue: bookkeeping of blocks 0 and 1, rows of block 0
                block_info(tid, 0, u0, u1, j0, j1, tb, idx, n64, nullptr, nullptr, info[0]);
                if (nblk > 1) block_info(tid, 1, u0, u1, j0, j1, tb, idx, n64, nullptr, nullptr, info[1]);
                __syncthreads();
                {
                    const int32_t mem = info[0].row_mem[grow];
                    float* dst = reinterpret_cast<float*>(lds_m4[0]) + grow * S;
#pragma unroll
                    for (int i = 0; i < PF; ++i) {
                        const int k = gk + 8 * i;
                        dst[k] = (mem >= 0 && k < d) ? x[int64_t(mem) * d + k] : 0.0f;
                    }
                }
                __syncthreads();
                for (int64_t blk = 0; blk < nblk; ++blk) {
                    const int rb = int(blk & 1);
                    const BlockInfo& bi = info[blk % 3];
                    // rows of block blk+1 into registers (their stores follow the MFMAs)
                    float pf[PF];
                    const bool more = blk + 1 < nblk;
                    if (more) {
                        const int32_t mem = info[(blk + 1) % 3].row_mem[grow];
#pragma unroll
                        for (int i = 0; i < PF; ++i) {
                            const int k = gk + 8 * i;
                            pf[i] = (mem >= 0 && k < d) ? x[int64_t(mem) * d + k] : 0.0f;
                        }
                    }
                    // bookkeeping of block blk+2 (its slot was last read in block blk-1)
                    if (blk + 2 < nblk)
                        block_info(tid, blk + 2, u0, u1, j0, j1, tb, idx, n64, nullptr, nullptr, info[(blk + 2) % 3]);
                    // member rows x this wave's points
                    floatx16 acc[2];
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                        for (int r = 0; r < 16; ++r) acc[cb][r] = bi.row_c[8 * (r / 4) + 4 * half + (r % 4)];
                    const float* arow = reinterpret_cast<const float*>(lds_m4[rb]) + col * S + half * KH;
#pragma unroll
                    for (int s4 = 0; s4 < QF; ++s4) {
                        const float4 a4 = *reinterpret_cast<const float4*>(arow + 4 * s4);
                        const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int cb = 0; cb < 2; ++cb)
                                acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], b[cb][4 * s4 + i], acc[cb], 0,
                                                                               0, 0);
                    }
                    if constexpr (TRIM) {
                        const float2 a2 = *reinterpret_cast<const float2*>(reinterpret_cast<const float*>(lds_m4[rb]) +
                                                                           col * S + (half ? KH - 2 : KH - 4));
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb) {
                            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a2.x, b[cb][KH - 4], acc[cb], 0, 0, 0);
                            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a2.y, b[cb][KH - 3], acc[cb], 0, 0, 0);
                        }
                    }
                    es_units<kWindow>(acc, bi.unit_flags, bi.unit_local, wsh, cur, half, col, lacc[wave]);
                    if (more) {
                        float* dst = reinterpret_cast<float*>(lds_m4[rb ^ 1]) + grow * S;
#pragma unroll
                        for (int i = 0; i < PF; ++i) dst[gk + 8 * i] = pf[i];
                    }
                    __syncthreads();
                }
            }
        }
        __syncthreads();
        es_finish<kWindow>(tid, j0, j1, split, l, sc, lacc);
        __syncthreads();
    }
}

// The same evaluation with the dot products in the dataset's reduced
// precision (the paper's FP16 GPU variant, Sec. 5): member and ground-point
// rows come from the cast copy (64-row tiles of 16-byte units, unit-major),
// the norms are those of the cast rows, the matrix instruction is the
// dtype's 32x32 one (FP8 with the rows' E8M0 scales); maxima, clamps and
// sums as above.
template <int DT, int KC, int W>
__global__ void __launch_bounds__(256)
k_es_lp(const uint4* __restrict__ xq, const float* __restrict__ hn, const int* __restrict__ scale, int64_t n,
        const double* __restrict__ n64, const double* __restrict__ m0, const int64_t* __restrict__ off,
        const int32_t* __restrict__ idx, int64_t l, int32_t splits, EsScratch sc) {
    using T = Lp<DT>;
    constexpr int HU = KC * T::kU4;  // 16-byte units per lane half-row
    constexpr int RU = 2 * HU;       // units per row
    constexpr int PFU = (32 * RU + 255) / 256;
    constexpr bool kFp8 = DT == EBC_DT_FP8_E4M3;
    constexpr int RB = W / kBlockUnits;  // member blocks a resident group can hold
    // resident groups (at most W units): all member rows and bookkeeping in LDS
    __shared__ uint4 res_rows[RB][RU * 32];  // [block][unit][row]
    __shared__ int32_t res_mem[RB * 32];
    __shared__ float res_c[RB * 32];
    __shared__ int32_t res_sc[RB * 32];
    __shared__ int32_t res_flags[W], res_local[W];
    __shared__ float lacc[4][W][32];  // per wave, set and column: float sums over points
    // larger groups (a set longer than the window): stream blocks as in the float32 kernel
    __shared__ uint4 lds_m[2][RU * 32];
    __shared__ BlockInfo info[3];
    __shared__ int64_t t_u[kTab + 1], t_off[kTab + 1];
    __shared__ int32_t t_e[kTab + 1];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 31;
    const int half = lane >> 5;
    if (sc.n_groups[2] > 0) return;  // every set fits the register kernel, which takes the call
    const int64_t n_items = *sc.n_groups * splits;
    const int64_t vchunk = ((n + splits - 1) / splits + kVSub - 1) / kVSub * kVSub;
    const int* sc_rows = kFp8 ? scale : nullptr;

    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t g = item / splits;
        const int split = int(item % splits);
        const int64_t j0 = lower_bound_u(sc.U, 0, l, g * W);
        const int64_t j1 = lower_bound_u(sc.U, j0, l, (g + 1) * W);
        const int64_t u0 = sc.U[j0], u1 = sc.U[j1];
        const int64_t v_begin = int64_t(split) * vchunk;
        int64_t v_end = v_begin + vchunk;
        if (v_end > n) v_end = n;
        const bool cached = j1 - j0 <= kTab;
        if (cached)
            for (int64_t i = tid; i <= j1 - j0; i += 256) {
                t_u[i] = sc.U[j0 + i];
                t_e[i] = sc.E[j0 + i];
                t_off[i] = off[j0 + i];
            }
        for (int i = tid; i < 4 * W * 32; i += 256) (&lacc[0][0][0])[i] = 0.0f;
        __syncthreads();
        const SetTable tb = cached ? SetTable{t_u, t_e, t_off, j0} : SetTable{sc.U, sc.E, off, 0};
        const int64_t nunits = u1 - u0;
        const bool resident = nunits <= W;
        if (nunits > 0 && v_end > v_begin && resident) {
            const int nblk = int((nunits + kBlockUnits - 1) / kBlockUnits);
            // bookkeeping of every row and unit of the group, once per item
            for (int r = tid; r < nblk * 32; r += 256) {
                const int64_t u = u0 + r / kUnitRows;
                int32_t mem = -1;
                if (u < u1) {
                    const int64_t jj = owner_of(tb.U, j0 - tb.base, j1 - tb.base, u);
                    const int64_t q = (u - tb.U[jj]) * kUnitRows + r % kUnitRows;
                    if (tb.off[jj] + q < tb.off[jj + 1]) mem = idx[tb.off[jj] + q];
                }
                res_mem[r] = mem;
                res_c[r] = mem < 0 ? -INFINITY : -hn[mem];
                res_sc[r] = (mem >= 0 && kFp8) ? scale[mem] : 127;
            }
            for (int uu = tid; uu < nblk * kBlockUnits; uu += 256) {
                const int64_t u = u0 + uu;
                int flags = 0, loc = 0;
                if (u < u1) {
                    const int64_t jj = owner_of(tb.U, j0 - tb.base, j1 - tb.base, u);
                    flags = 4 | (u == tb.U[jj] ? 1 : 0) | (u == tb.U[jj + 1] - 1 ? 2 : 0);
                    loc = tb.E[jj] - tb.E[j0 - tb.base];
                }
                res_flags[uu] = flags;
                res_local[uu] = loc;
            }
            __syncthreads();
            // member rows of the group into LDS
            for (int e = tid; e < nblk * 32 * RU; e += 256) {
                const int blk = e / (32 * RU), rem = e % (32 * RU), u = rem / 32, r = rem % 32;
                const int32_t mem = res_mem[blk * 32 + r];
                res_rows[blk][u * 32 + r] =
                    mem >= 0 ? xq[(int64_t(mem) / 64 * RU + u) * 64 + mem % 64] : make_uint4(0, 0, 0, 0);
            }
            __syncthreads();
            // every pass over 64 points per wave reads the resident rows only: no barriers
            for (int64_t vs = v_begin; vs < v_end; vs += kVSub) {
                uint4 b[2][HU];
                int sb[2];
                float wsh[2];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const int64_t v = vs + wave * 64 + cb * 32 + col;
                    const bool ok = v < v_end;
                    wsh[cb] = ok ? float(0.5 * m0[v] - double(hn[v])) : 0.0f;
                    const uint4* src = xq + (v / 64) * (RU * 64) + (v % 64);
#pragma unroll
                    for (int u = 0; u < HU; ++u) b[cb][u] = ok ? src[(half * HU + u) * 64] : make_uint4(0, 0, 0, 0);
                    sb[cb] = (kFp8 && ok) ? scale[v] : 127;
                }
                float cur[2] = {-INFINITY, -INFINITY};
                for (int blk = 0; blk < nblk; ++blk) {
                    uint4 a[HU];
#pragma unroll
                    for (int u = 0; u < HU; ++u) a[u] = res_rows[blk][(half * HU + u) * 32 + col];
                    const int sa = res_sc[blk * 32 + col];
                    floatx16 acc[2];
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                        for (int r = 0; r < 16; ++r) acc[cb][r] = res_c[blk * 32 + 8 * (r / 4) + 4 * half + (r % 4)];
#pragma unroll
                    for (int q = 0; q < KC; ++q)
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb)
                            acc[cb] = mfma_main<DT>(&a[q * T::kU4], &b[cb][q * T::kU4], acc[cb], sa, sb[cb]);
                    es_units<W>(acc, res_flags + blk * kBlockUnits, res_local + blk * kBlockUnits, wsh, cur, half,
                                col, lacc[wave]);
                }
            }
        } else if (nunits > 0 && v_end > v_begin) {
            const int64_t nblk = (nunits + kBlockUnits - 1) / kBlockUnits;
            for (int64_t vs = v_begin; vs < v_end; vs += kVSub) {
                uint4 b[2][HU];
                int sb[2];
                float wsh[2];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const int64_t v = vs + wave * 64 + cb * 32 + col;
                    const bool ok = v < v_end;
                    wsh[cb] = ok ? float(0.5 * m0[v] - double(hn[v])) : 0.0f;
                    const uint4* src = xq + (v / 64) * (RU * 64) + (v % 64);
#pragma unroll
                    for (int u = 0; u < HU; ++u) b[cb][u] = ok ? src[(half * HU + u) * 64] : make_uint4(0, 0, 0, 0);
                    sb[cb] = (kFp8 && ok) ? scale[v] : 127;
                }
                float cur[2] = {-INFINITY, -INFINITY};
                block_info(tid, 0, u0, u1, j0, j1, tb, idx, n64, hn, sc_rows, info[0]);
                if (nblk > 1) block_info(tid, 1, u0, u1, j0, j1, tb, idx, n64, hn, sc_rows, info[1]);
                __syncthreads();
#pragma unroll
                for (int i = 0; i < PFU; ++i) {
                    const int e = tid + 256 * i;
                    if (e < 32 * RU) {
                        const int r = e % 32, u = e / 32;
                        const int32_t mem = info[0].row_mem[r];
                        lds_m[0][u * 32 + r] =
                            mem >= 0 ? xq[(int64_t(mem) / 64 * RU + u) * 64 + mem % 64] : make_uint4(0, 0, 0, 0);
                    }
                }
                __syncthreads();
                for (int64_t blk = 0; blk < nblk; ++blk) {
                    const int rb = int(blk & 1);
                    const BlockInfo& bi = info[blk % 3];
                    uint4 pf[PFU];
                    const bool more = blk + 1 < nblk;
                    if (more) {
#pragma unroll
                        for (int i = 0; i < PFU; ++i) {
                            const int e = tid + 256 * i;
                            pf[i] = make_uint4(0, 0, 0, 0);
                            if (e < 32 * RU) {
                                const int32_t mem = info[(blk + 1) % 3].row_mem[e % 32];
                                if (mem >= 0) pf[i] = xq[(int64_t(mem) / 64 * RU + e / 32) * 64 + mem % 64];
                            }
                        }
                    }
                    if (blk + 2 < nblk)
                        block_info(tid, blk + 2, u0, u1, j0, j1, tb, idx, n64, hn, sc_rows, info[(blk + 2) % 3]);
                    uint4 a[HU];
#pragma unroll
                    for (int u = 0; u < HU; ++u) a[u] = lds_m[rb][(half * HU + u) * 32 + col];
                    const int sa = bi.row_sc[col];
                    floatx16 acc[2];
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                        for (int r = 0; r < 16; ++r) acc[cb][r] = bi.row_c[8 * (r / 4) + 4 * half + (r % 4)];
#pragma unroll
                    for (int q = 0; q < KC; ++q)
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb)
                            acc[cb] = mfma_main<DT>(&a[q * T::kU4], &b[cb][q * T::kU4], acc[cb], sa, sb[cb]);
                    es_units<W>(acc, bi.unit_flags, bi.unit_local, wsh, cur, half, col, lacc[wave]);
                    if (more) {
#pragma unroll
                        for (int i = 0; i < PFU; ++i) {
                            const int e = tid + 256 * i;
                            if (e < 32 * RU) lds_m[rb ^ 1][(e / 32) * 32 + e % 32] = pf[i];
                        }
                    }
                    __syncthreads();
                }
            }
        }
        __syncthreads();
        es_finish<W>(tid, j0, j1, split, l, sc, lacc);
        __syncthreads();
    }
}

// ---- shared parts of the register kernels (k_es_regs, k_es_regs32) ----

// One wave's window: its sets [j0, j1) and units [ua, ub), the member row of
// each of its 64 rows in rmem_w (lane r: row r, unit ua + r/UR; -1 padding)
// and the wave-uniform mask of the units that end a set (bit u: unit ua + u;
// UR rows per unit, NU units per window).
struct RegWindow {
    int64_t j0, j1, ua, ub;
    uint32_t m_last;
};

template <int UR = kUnitRows, int NU = kRegUnits>
__device__ __forceinline__ RegWindow reg_window(const EsScratch& sc, int64_t w, int64_t n_win, int lane,
                                                const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
                                                int32_t* rmem_w) {
    static_assert(UR * NU == 64 && NU <= 32, "a window is 64 rows; one mask bit per unit");
    RegWindow r{0, 0, 0, 0, 0u};
    if (w < n_win) {
        r.j0 = sc.win_j0[w];
        r.j1 = sc.win_j0[w + 1];
    }
    r.ua = sc.U[r.j0];
    r.ub = sc.U[r.j1];
    {
        const int64_t u = r.ua + lane / UR;
        int32_t mem = -1;
        if (u < r.ub) {
            const int64_t j = owner_of(sc.U, r.j0, r.j1, u);
            const int64_t q = (u - sc.U[j]) * UR + lane % UR;
            if (off[j] + q < off[j + 1]) mem = idx[off[j] + q];
        }
        rmem_w[lane] = mem;
    }
    {
        const int64_t u = r.ua + lane;
        bool last = false;
        if (lane < NU && u < r.ub) {
            const int64_t j = owner_of(sc.U, r.j0, r.j1, u);
            last = u == sc.U[j + 1] - 1;
        }
        r.m_last = __builtin_amdgcn_readfirstlane(uint32_t(__builtin_amdgcn_ballot_w64(last)));
    }
    return r;
}

// rs[u] = -inf at a set's first unit (the unit after a last one), else 0
__device__ __forceinline__ void reg_restarts(uint32_t m_last, float (&rs)[kRegUnits]) {
#pragma unroll
    for (int u = 0; u < kRegUnits; ++u) rs[u] = (u > 0 && ((m_last >> (u - 1)) & 1u)) ? -INFINITY : 0.0f;
}

// Close one tile: pair the unit maxima of its two column blocks (x0: block
// 0, x1: block 1; upper half of x0 <-> lower half of x1, so lane (col, h)
// gets the 8 + 8 unit maxima of ground point 32h + col), then the running
// maximum over the window's units, restarting at each set's first unit, and
// at a set's last unit u the lane adds max(0, running max + wsh) to acc_u[u].
// Units past the window's last set are padding rows at -inf, so they never
// reach a last unit.
__device__ __forceinline__ void reg_close(const float (&x0)[8], const float (&x1)[8], const float (&rs)[kRegUnits],
                                          uint32_t m_last, float wsh, float (&acc_u)[kRegUnits]) {
    float um[kRegUnits];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int gq = 0; gq < kBlockUnits / 2; ++gq) {
            const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x0[mb * 4 + gq]),
                                                            __float_as_uint(x1[mb * 4 + gq]), false, false);
            um[mb * kBlockUnits + 2 * gq] = __uint_as_float(r[0]);
            um[mb * kBlockUnits + 2 * gq + 1] = __uint_as_float(r[1]);
        }
    float cur = -INFINITY;
    // the set ends as an opaque scalar per tile: the compiler tests its bits
    // with scalar instructions instead of keeping per-unit lane masks
    uint32_t ml = m_last;
    asm volatile("" : "+s"(ml));
#pragma unroll
    for (int u = 0; u < kRegUnits; ++u) {
        cur = fmaxf(cur + rs[u], um[u]);
        if ((ml >> u) & 1u) {
            // a scalar branch, not selects over every unit (the empty volatile
            // statement keeps the compiler from speculating it)
            asm volatile("");
            acc_u[u] += fmaxf(cur + wsh, 0.0f);
        }
    }
}

// The same for a window of 32 two-row units (x0, x1: the 8 + 8 two-row
// maxima per lane of column block 0 / 1, index mb 8 + 2 g + e for rows
// 8 g + 4 h + 2 e, +1 of member block mb, i.e. unit 4 g + 2 h + e of that
// block). Every set spans at least two units, so two set ends are at least
// two units apart and set ends of units u share accumulator u / 2 with no
// other set. The restarts come from the scalar mask (-inf or 0 added in a
// scalar register), not from a register array.
__device__ __forceinline__ void reg_close2(const float (&x0)[16], const float (&x1)[16], uint32_t m_last, float wsh,
                                           float (&acc_s)[kReg2Units / 2]) {
    float um[kReg2Units];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int k = mb * 8 + 2 * g + e;
                const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x0[k]), __float_as_uint(x1[k]), false,
                                                                false);
                um[mb * 16 + 4 * g + e] = __uint_as_float(r[0]);
                um[mb * 16 + 4 * g + 2 + e] = __uint_as_float(r[1]);
            }
    float cur = -INFINITY;
    uint32_t ml = m_last;
    asm volatile("" : "+s"(ml));
#pragma unroll
    for (int u = 0; u < kReg2Units; ++u) {
        const float rs = (u > 0 && ((ml >> (u - 1)) & 1u)) ? -INFINITY : 0.0f;
        cur = fmaxf(cur + rs, um[u]);
        if ((ml >> u) & 1u) {
            asm volatile("");
            acc_s[u >> 1] += fmaxf(cur + wsh, 0.0f);
        }
    }
}

// Each set's accumulator (acc[u >> SH] for the set ending at unit u) summed
// over the 64 lanes in a fixed order in float64, one write per set and
// ground-set split.
template <int NU = kRegUnits, int SH = 0>
__device__ __forceinline__ void reg_write(const EsScratch& sc, const RegWindow& wv, const float (&acc_u)[NU >> SH],
                                          int lane, int split, int64_t l) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        if (!((wv.m_last >> u) & 1u)) continue;
        double v = double(acc_u[u >> SH]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) {
            const int64_t j = owner_of(sc.U, wv.j0, wv.j1, wv.ua + u);
            sc.part[int64_t(split) * l + j] = v;
        }
    }
}

// Reduced-precision multi-set evaluation with the member rows in registers
// (calls whose sets all have at most kRegMaxSet units, i.e. 32 members;
// others go to k_es_lp). The structure is that of the marginal-gains kernel: each wave
// holds its window's member rows (two 32-row blocks) as the MFMA A operand in
// registers for the whole item, and the ground set streams through a 2-stage
// LDS ring of 64-point tiles (global_load_lds copies of tile t+1 issued after
// the barrier of tile t) shared by the workgroup's 4 waves. Work item = (4 consecutive wave windows,
// ground-set split). Wave window w holds the sets whose first unit lies in
// [w G, (w+1) G) (G from k_es_scan), so no set crosses windows and a window
// spans at most kRegUnits units.
//
// Per tile and member block: the two 32-point column blocks' MFMAs (C
// operand -||s^||^2/2 per row, -inf for padding rows), each lane's maximum
// over every unit's four rows, and one lane swap between the halves
// (v_permlane32_swap) that leaves lane (col, h) with the eight unit maxima of
// ground point 32h + col. Then, for that point, the running maximum over the
// window's units under wave-uniform flags (first / last unit of a set), and
// at a set's last unit u the lane adds max(0, running max + wsh_v) to its
// register accumulator acc_u[u] (u is a compile-time index after unrolling).
// wsh_v = m_v/2 - ||v^||^2/2 folds e0 and the cast rows' norms in as in
// k_es_lp; points outside the split get -inf, so they add nothing. After the
// split, each set's accumulator is summed over the 64 lanes in a fixed order
// in float64 and written as the set's partial sum of this split.
template <int DT, int KC>
__global__ void __launch_bounds__(256)
k_es_regs(const uint4* __restrict__ xq, const float* __restrict__ hn, const int* __restrict__ scale, int64_t n,
          const double* __restrict__ m0, const int64_t* __restrict__ off, const int32_t* __restrict__ idx, int64_t l,
          int32_t splits, EsScratch sc) {
    using T = Lp<DT>;
    constexpr int HU = KC * T::kU4;  // 16-byte units per lane half-row
    constexpr int RU = 2 * HU;       // 16-byte units per row
    constexpr int VT = 64;           // ground points per tile
    constexpr bool kFp8 = DT == EBC_DT_FP8_E4M3;
    constexpr int OFF_SC = RU * VT;                          // FP8: the tile's row scales after its units
    constexpr int STAGE1 = RU * VT + (kFp8 ? VT / 4 : 0);    // uint4 per 64-point tile
    constexpr int NI = RU + (kFp8 ? 1 : 0);                  // wave copy instructions per tile
    constexpr int L = (NI + 3) / 4;                          // copy instructions per wave per tile
    // tiles per ring stage: two (one barrier per 128 points) when two
    // stages of them fit the 64 KB a workgroup may hold
    constexpr int SUBT = 4 * STAGE1 * 16 + 1024 <= 65536 ? 2 : 1;
    __shared__ uint4 ring0[SUBT * STAGE1];
    __shared__ uint4 ring1[SUBT * STAGE1];
    __shared__ int32_t rmem[4][64];  // per wave: member row of each of its 64 rows (-1: padding)

    const int64_t n_win = sc.n_groups[2];
    if (n_win == 0) return;  // some set is longer than kRegMaxSet units (k_es_lp runs), or none has units
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane & 31;
    const int half = lane >> 5;
    const int64_t n_items = (n_win + 3) / 4 * splits;
    const int64_t vchunk = ((n + splits - 1) / splits + kVSub - 1) / kVSub * kVSub;

    // every wave issues exactly L copy instructions per stage (pieces beyond NI
    // repeat one another wave also copies: same bytes to the same place)
    auto copy_stage = [&](int64_t tile, uint4* st) {
#pragma unroll
        for (int q = 0; q < L; ++q) {
            const int j = (wave + 4 * q) % NI;
            if (j < RU)
                __builtin_amdgcn_global_load_lds(xq + (tile * RU + j) * VT + lane, (lds_void*)(st + j * VT), 16, 0, 0);
            else
                __builtin_amdgcn_global_load_lds(scale + tile * VT + lane, (lds_void*)(st + OFF_SC), 4, 0, 0);
        }
    };

    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t g = item / splits;
        const int split = int(item % splits);
        const int64_t w = g * 4 + wave;
        const RegWindow wv = reg_window(sc, w, n_win, lane, off, idx, rmem[wave]);
        const uint32_t m_last = wv.m_last;
        __syncthreads();  // rmem of every wave written (and the ring of the previous item drained)
        // member rows (A operand) and the C operand -||s^||^2/2 of the rows this lane holds
        uint4 a[2][HU];
        int sa[2];
        floatx16 cinit[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int32_t mem = rmem[wave][mb * 32 + col];
            const uint4* src = xq + (int64_t(mem) / 64) * (RU * 64) + (mem % 64);
#pragma unroll
            for (int u = 0; u < HU; ++u) a[mb][u] = mem >= 0 ? src[(half * HU + u) * 64] : make_uint4(0, 0, 0, 0);
            sa[mb] = (kFp8 && mem >= 0) ? scale[mem] : 127;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int32_t mr = rmem[wave][mb * 32 + 8 * (r / 4) + 4 * half + (r % 4)];
                cinit[mb][r] = mr >= 0 ? -hn[mr] : -INFINITY;
            }
        }
        float acc_u[kRegUnits];
#pragma unroll
        for (int u = 0; u < kRegUnits; ++u) acc_u[u] = 0.0f;
        float rs[kRegUnits];
        reg_restarts(m_last, rs);

        // ground tiles of this split
        const int64_t v_begin = int64_t(split) * vchunk;
        int64_t v_end = v_begin + vchunk;
        if (v_end > n) v_end = n;
        const int64_t t_begin = v_begin / VT;
        const int64_t nt = v_end > v_begin ? (v_end - v_begin + VT - 1) / VT : 0;
        // this lane's ground point of tile t and its shift (next tile's in flight)
        auto shift_of = [&](int64_t t) -> float {
            const int64_t v = (t_begin + t) * VT + lane;
            return (t < nt && v >= v_begin && v < v_end) ? float(0.5 * m0[v] - double(hn[v])) : -INFINITY;
        };
        float wsh_nx[SUBT];  // shifts of the next stage's tiles (in flight)
#pragma unroll
        for (int q = 0; q < SUBT; ++q) wsh_nx[q] = shift_of(q);
#pragma unroll
        for (int q = 0; q < SUBT; ++q)
            if (q < nt) copy_stage(t_begin + q, ring0 + q * STAGE1);
        // Software-pipelined over column blocks: while the MFMAs of column
        // block 0 of tile t run, the lane takes the unit maxima of column
        // block 1 of tile t-1, pairs them with those of its block 0 (taken
        // while block 1's MFMAs ran) and closes tile t-1's sets; while the
        // MFMAs of block 1 of tile t run, it takes the maxima of block 0 of
        // tile t. Tile -1 is all -inf, so closing it adds +0 to every sum.
        floatx16 acc[2][2];  // [member block][column block]
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mb][1][r] = -INFINITY;
        float x0[8];  // unit maxima of column block 0 of the previous tile
#pragma unroll
        for (int i = 0; i < 8; ++i) x0[i] = -INFINITY;
        float wsh_prev = 0.0f;
        // maxima over each unit's four rows held by this lane, one column block
        auto unit_max = [&](int cb, float (&x)[8]) {
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int gq = 0; gq < kBlockUnits / 2; ++gq) {
                    const floatx16& p = acc[mb][cb];
                    x[mb * 4 + gq] = fmaxf(fmaxf(p[4 * gq], p[4 * gq + 1]), fmaxf(p[4 * gq + 2], p[4 * gq + 3]));
                }
        };
        // the MFMAs of one column block (both member blocks) from operand b
        auto mfma_block = [&](int cb, const uint4 (&b)[HU], int sb) {
            acc[0][cb] = cinit[0];
            acc[1][cb] = cinit[1];
#pragma unroll
            for (int q = 0; q < KC; ++q)
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
                    acc[mb][cb] = mfma_main<DT>(&a[mb][q * T::kU4], &b[q * T::kU4], acc[mb][cb], sa[mb], sb);
        };
        constexpr int NMF = 2 * KC;  // matrix instructions per column block
        // one 64-point tile from its place st in a stage
        auto tile = [&](const uint4* st, float wsh) {
            const int* st_sc = reinterpret_cast<const int*>(st + OFF_SC);
            uint4 b[HU];
            // column block 0 of tile t, with the maxima of block 1 of tile t-1
#pragma unroll
            for (int u = 0; u < HU; ++u) b[u] = st[(half * HU + u) * VT + col];
            float x1[8];
            unit_max(1, x1);
            mfma_block(0, b, kFp8 ? st_sc[col] : 127);
#pragma unroll
            for (int i = 0; i < NMF; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // then part of the maxima
            }
            reg_close(x0, x1, rs, m_last, wsh_prev, acc_u);
            // column block 1 of tile t, with the maxima of block 0 of tile t
#pragma unroll
            for (int u = 0; u < HU; ++u) b[u] = st[(half * HU + u) * VT + 32 + col];
            unit_max(0, x0);
            mfma_block(1, b, kFp8 ? st_sc[32 + col] : 127);
#pragma unroll
            for (int i = 0; i < NMF; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
            }
            wsh_prev = wsh;
        };
        // ring stage t: tiles SUBT t .. SUBT t + SUBT - 1
        auto stage = [&](int64_t t, const uint4* st, uint4* next) {
            wait_vmcnt<0>();  // this stage's copies (issued one stage ago) and its shift loads
            ring_barrier();   // ... of every wave; every wave is done reading the other stage
            float wsh[SUBT];
#pragma unroll
            for (int q = 0; q < SUBT; ++q) {
                wsh[q] = wsh_nx[q];
                wsh_nx[q] = shift_of(SUBT * (t + 1) + q);
            }
#pragma unroll
            for (int q = 0; q < SUBT; ++q)
                if (SUBT * (t + 1) + q < nt) copy_stage(t_begin + SUBT * (t + 1) + q, next + q * STAGE1);
#pragma unroll
            for (int q = 0; q < SUBT; ++q)
                if (q == 0 || SUBT * t + q < nt) tile(st + q * STAGE1, wsh[q]);
        };
        // stage t: ring t % 2 (distinct LDS objects)
        const int64_t nst = (nt + SUBT - 1) / SUBT;
        for (int64_t t = 0; t < nst; t += 2) {
            stage(t, ring0, ring1);
            if (t + 1 < nst) stage(t + 1, ring1, ring0);
        }
        // the last tile
        {
            float x1[8];
            unit_max(1, x1);
            reg_close(x0, x1, rs, m_last, wsh_prev, acc_u);
        }
        reg_write(sc, wv, acc_u, lane, split, l);
    }
}

// The float32 evaluation of an FP32 dataset with the member rows in
// registers: the register kernel above with v_mfma_f32_32x32x2_f32 (64
// cycles each, K = 2), taking the same calls (every set at most kRegMaxSet
// units) and the same windows, work items, epilogue and per-set sums. The
// dataset's float32 copy is row-major [n_pad, KP]; each lane copies its own
// row's 16-byte units of a 64-point tile into the LDS stage (unit-major, so
// the operand reads of a half-wave are 32 consecutive units), two stages of
// KP/4 KB each. Lane half h takes K values h KP/2 .. (h+1) KP/2 - 1 of both
// operands (one 16-byte unit feeds 4 MFMAs; when the rows' last 4 slots are
// padding, the last unit of half 0 feeds both halves in 2 MFMAs: values
// KP/2-4, -3 on half 0 and KP/2-2, -1 on half 1). A tile's epilogue costs about as
// much as 3 of its 4 KP MFMAs, so it is not overlapped with them. UR = rows
// per unit of the call's windows: 4 (16 units per window), or 2 (32 units;
// calls whose sets all have 3 .. 32 members, so a set of 10 fills 10 rows,
// not 12); the instance of the other unit size returns at once. The member
// rows' maxima and sums are the same in both, bit for bit.
template <int KP, int UR, bool TRIM>
__global__ void __launch_bounds__(256)
k_es_regs32(const uint4* __restrict__ xq, const float* __restrict__ hn, int64_t n, const double* __restrict__ m0,
            const int64_t* __restrict__ off, const int32_t* __restrict__ idx, int64_t l, int32_t splits,
            EsScratch sc) {
    // two stages of KP/4 KB within the 64 KB of LDS a workgroup can hold
    static_assert(KP % 8 == 0 && KP <= 120, "rows of 8 .. 120 floats, a multiple of 8");
    constexpr int RU = KP / 4;  // 16-byte units per row
    constexpr int HU = RU / 2;  // units per lane half
    constexpr int VT = 64;      // ground points per tile
    constexpr int STAGE = RU * VT;
    constexpr int L = (RU + 3) / 4;  // copy instructions per wave per stage
    __shared__ uint4 ring0[STAGE];
    __shared__ uint4 ring1[STAGE];
    __shared__ int32_t rmem[4][64];

    static_assert(UR == 2 || UR == 4, "units of 2 or 4 rows");
    constexpr int NU = 64 / UR;  // units per window
    constexpr int NA = 16;       // per-lane set accumulators (UR 4: one per unit; UR 2: one per unit pair)
    const int64_t n_win = sc.n_groups[2];
    // some set is longer than the window allows (k_es_main runs), none has
    // units, or the windows are in the other unit size
    if (n_win == 0 || sc.n_groups[3] != UR) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane & 31;
    const int half = lane >> 5;
    const int64_t n_items = (n_win + 3) / 4 * splits;
    const int64_t vchunk = ((n + splits - 1) / splits + kVSub - 1) / kVSub * kVSub;

    // lane i copies unit j of row tile*64 + i (the rows are row-major); every
    // wave issues exactly L copy instructions per stage (pieces beyond RU
    // repeat one another wave also copies: same bytes to the same place)
    auto copy_stage = [&](int64_t tile, uint4* st) {
#pragma unroll
        for (int q = 0; q < L; ++q) {
            const int j = (wave + 4 * q) % RU;
            __builtin_amdgcn_global_load_lds(xq + (tile * VT + lane) * RU + j, (lds_void*)(st + j * VT), 16, 0, 0);
        }
    };

    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t g = item / splits;
        const int split = int(item % splits);
        const int64_t w = g * 4 + wave;
        const RegWindow wv = reg_window<UR, NU>(sc, w, n_win, lane, off, idx, rmem[wave]);
        const uint32_t m_last = wv.m_last;
        __syncthreads();  // rmem of every wave written (and the ring of the previous item drained)
        uint4 a[2][HU];
        floatx16 cinit[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int32_t mem = rmem[wave][mb * 32 + col];
            const uint4* src = xq + int64_t(mem < 0 ? 0 : mem) * RU + half * HU;
#pragma unroll
            for (int u = 0; u < HU; ++u) a[mb][u] = mem >= 0 ? src[u] : make_uint4(0, 0, 0, 0);
            if constexpr (TRIM) {  // last step: half 0 takes values KP/2-4, -3, half 1 takes KP/2-2, -1
                const uint4 t = mem >= 0 ? src[HU - 1 - half * HU] : make_uint4(0, 0, 0, 0);
                a[mb][HU - 1] = half ? make_uint4(t.z, t.w, 0, 0) : t;
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int32_t mr = rmem[wave][mb * 32 + 8 * (r / 4) + 4 * half + (r % 4)];
                cinit[mb][r] = mr >= 0 ? -hn[mr] : -INFINITY;
            }
        }
        float acc_u[NA];
#pragma unroll
        for (int u = 0; u < NA; ++u) acc_u[u] = 0.0f;
        float rs[kRegUnits];
        if constexpr (UR == 4) reg_restarts(m_last, rs);

        const int64_t v_begin = int64_t(split) * vchunk;
        int64_t v_end = v_begin + vchunk;
        if (v_end > n) v_end = n;
        const int64_t t_begin = v_begin / VT;
        const int64_t nt = v_end > v_begin ? (v_end - v_begin + VT - 1) / VT : 0;
        auto shift_of = [&](int64_t t) -> float {
            const int64_t v = (t_begin + t) * VT + lane;
            return (t < nt && v >= v_begin && v < v_end) ? float(0.5 * m0[v] - double(hn[v])) : -INFINITY;
        };
        float wsh_next = shift_of(0);
        if (nt > 0) copy_stage(t_begin, ring0);
        auto tile = [&](int64_t t, const uint4* st, uint4* next) {
            wait_vmcnt<0>();  // this tile's copies (issued one tile ago) and its shift loads
            ring_barrier();   // ... of every wave; every wave is done reading the other stage
            const float wsh = wsh_next;
            wsh_next = shift_of(t + 1);
            if (t + 1 < nt) copy_stage(t_begin + t + 1, next);
            float xm[2][32 / UR];  // unit maxima per column block
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                floatx16 acc[2] = {cinit[0], cinit[1]};
#pragma unroll
                for (int u = 0; u < HU; ++u) {
                    if (TRIM && u == HU - 1) {
                        // the row's last 4 slots are padding: one unit (the
                        // last of half 0) feeds both halves, 2 steps instead of 4
                        const uint4 bq = st[(HU - 1) * VT + cb * 32 + col];
                        const float b0 = __uint_as_float(half ? bq.z : bq.x);
                        const float b1 = __uint_as_float(half ? bq.w : bq.y);
#pragma unroll
                        for (int mb = 0; mb < 2; ++mb) {
                            acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[mb][u].x), b0, acc[mb],
                                                                           0, 0, 0);
                            acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[mb][u].y), b1, acc[mb],
                                                                           0, 0, 0);
                        }
                        continue;
                    }
                    const uint4 bq = st[(half * HU + u) * VT + cb * 32 + col];
                    const float bv[4] = {__uint_as_float(bq.x), __uint_as_float(bq.y), __uint_as_float(bq.z),
                                         __uint_as_float(bq.w)};
#pragma unroll
                    for (int e = 0; e < 4; ++e)
#pragma unroll
                        for (int mb = 0; mb < 2; ++mb) {
                            const uint4& aq = a[mb][u];
                            const float av = e == 0 ? __uint_as_float(aq.x)
                                             : e == 1 ? __uint_as_float(aq.y)
                                             : e == 2 ? __uint_as_float(aq.z)
                                                      : __uint_as_float(aq.w);
                            acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[e], acc[mb], 0, 0, 0);
                        }
                }
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                    for (int gq = 0; gq < kBlockUnits / 2; ++gq) {
                        const floatx16& pq = acc[mb];
                        if constexpr (UR == 4) {
                            xm[cb][mb * 4 + gq] =
                                fmaxf(fmaxf(pq[4 * gq], pq[4 * gq + 1]), fmaxf(pq[4 * gq + 2], pq[4 * gq + 3]));
                        } else {
                            xm[cb][mb * 8 + 2 * gq] = fmaxf(pq[4 * gq], pq[4 * gq + 1]);
                            xm[cb][mb * 8 + 2 * gq + 1] = fmaxf(pq[4 * gq + 2], pq[4 * gq + 3]);
                        }
                    }
            }
            if constexpr (UR == 4)
                reg_close(xm[0], xm[1], rs, m_last, wsh, acc_u);
            else
                reg_close2(xm[0], xm[1], m_last, wsh, acc_u);
        };
        // stage of tile t: t % 2 (distinct LDS objects)
        for (int64_t t = 0; t < nt; t += 2) {
            tile(t, ring0, ring1);
            if (t + 1 < nt) tile(t + 1, ring1, ring0);
        }
        reg_write<NU, UR == 4 ? 0 : 1>(sc, wv, acc_u, lane, split, l);
    }
}

// Long rows (padded length above 128): the same work items, windows and
// per-set sums as above, but no row is held whole. For every member block
// each wave walks the dimension (row pieces straight from global memory,
// the next batch in flight while the current one is multiplied), and it
// computes the block's bookkeeping in its own lanes (lane r < 32: row r;
// lanes 32..39: the units), so the waves meet at a barrier only for the
// item's final sums. kCallerRows (DT = F32 over a reduced-precision
// dataset) reads the caller's float32 rows [n, d] with the float64 norms;
// otherwise the dataset's own copy (float32 or cast, tiled), its norms and
// (FP8) scales. The copy of long rows is centred at the column means mu: with
// x' = x - mu, v.s - ||s||^2/2 = x'_v.x'_s - ||x'_s||^2/2 + (||v||^2 -
// ||x'_v||^2)/2, so the per-point shift of es_units is taken against the
// centred norms.
template <int DT, bool kCallerRows>
__global__ void __launch_bounds__(256)
k_es_wide(const void* src, int32_t len, const float* __restrict__ hn, const int* __restrict__ scale, int64_t n,
          const double* __restrict__ n64, const double* __restrict__ m0, const int64_t* __restrict__ off,
          const int32_t* __restrict__ idx, int64_t l, int32_t splits, EsScratch sc) {
    using R = WideRow<DT>;
    using Piece = typename R::Piece;
    constexpr int B = R::kBatch;
    static_assert(!kCallerRows || DT == EBC_DT_F32, "the caller's rows are float32");
    constexpr bool kF32 = kCallerRows;
    constexpr bool kFp8 = DT == EBC_DT_FP8_E4M3;
    __shared__ int64_t t_u[kTab + 1], t_off[kTab + 1];
    __shared__ int32_t t_e[kTab + 1];
    __shared__ float lacc[4][kWindow][32];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 31;
    const int half = lane >> 5;
    const int64_t n_items = *sc.n_groups * splits;
    const int64_t vchunk = ((n + splits - 1) / splits + kVSub - 1) / kVSub * kVSub;
    // the caller's rows: pieces of 8 values over d (the tail reads as 0); else the padded copy
    const int np = kF32 ? (len + 7) / 8 : R::pieces(len);
    auto piece = [&](int64_t row, int p) -> Piece {
        if constexpr (kF32)
            return R::load_x(static_cast<const float*>(src), row, len, p, half);
        else
            return R::load(src, row, len, p, half);
    };

    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t g = item / splits;
        const int split = int(item % splits);
        const int64_t j0 = lower_bound_u(sc.U, 0, l, g * kWindow);
        const int64_t j1 = lower_bound_u(sc.U, j0, l, (g + 1) * kWindow);
        const int64_t u0 = sc.U[j0], u1 = sc.U[j1];
        const int64_t v_begin = int64_t(split) * vchunk;
        int64_t v_end = v_begin + vchunk;
        if (v_end > n) v_end = n;
        const bool cached = j1 - j0 <= kTab;
        if (cached)
            for (int64_t i = tid; i <= j1 - j0; i += 256) {
                t_u[i] = sc.U[j0 + i];
                t_e[i] = sc.E[j0 + i];
                t_off[i] = off[j0 + i];
            }
        for (int i = tid; i < 4 * kWindow * 32; i += 256) (&lacc[0][0][0])[i] = 0.0f;
        __syncthreads();
        const SetTable tb = cached ? SetTable{t_u, t_e, t_off, j0} : SetTable{sc.U, sc.E, off, 0};
        if (u1 > u0 && v_end > v_begin) {
            const int64_t nblk = (u1 - u0 + kBlockUnits - 1) / kBlockUnits;
            for (int64_t vs = v_begin; vs < v_end; vs += kVSub) {
                // this wave's 64 ground points (B operand); points past the
                // split compute as zero rows, whose clamped terms are 0
                int64_t prow[2];
                bool pok[2];
                int sb[2];
                float wsh[2];  // per-point shift (see es_units)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const int64_t v = vs + wave * 64 + cb * 32 + col;
                    pok[cb] = v < v_end;
                    prow[cb] = pok[cb] ? v : 0;
                    sb[cb] = (kFp8 && pok[cb]) ? scale[v] : 127;
                    wsh[cb] = !pok[cb] ? 0.0f
                                       : (kF32 ? float(0.5 * (m0[v] - n64[v])) : float(0.5 * m0[v] - double(hn[v])));
                }
                float cur[2] = {-INFINITY, -INFINITY};
                for (int64_t blk = 0; blk < nblk; ++blk) {
                    // bookkeeping of block blk in this wave's lanes
                    int32_t my_mem = -1, my_sc = 127, my_flags = 0, my_loc = 0;
                    float my_c = -INFINITY;
                    if (lane < 32) {
                        const int64_t u = u0 + blk * kBlockUnits + lane / kUnitRows;
                        if (u < u1) {
                            const int64_t j = owner_of(tb.U, j0 - tb.base, j1 - tb.base, u);
                            const int64_t q = (u - tb.U[j]) * kUnitRows + lane % kUnitRows;
                            if (tb.off[j] + q < tb.off[j + 1]) my_mem = idx[tb.off[j] + q];
                        }
                        if (my_mem >= 0) {
                            my_c = kF32 ? -float(0.5 * n64[my_mem]) : -hn[my_mem];
                            if (kFp8) my_sc = scale[my_mem];
                        }
                    } else if (lane < 32 + kBlockUnits) {
                        const int64_t u = u0 + blk * kBlockUnits + (lane - 32);
                        if (u < u1) {
                            const int64_t j = owner_of(tb.U, j0 - tb.base, j1 - tb.base, u);
                            my_flags = 4 | (u == tb.U[j] ? 1 : 0) | (u == tb.U[j + 1] - 1 ? 2 : 0);
                            my_loc = tb.E[j] - tb.E[j0 - tb.base];
                        }
                    }
                    const int32_t amem = __shfl(my_mem, col, 64);  // A operand: member row `col`
                    const bool alive = amem >= 0;
                    const int64_t arow = alive ? amem : 0;
                    const int sa = __shfl(my_sc, col, 64);
                    int32_t uflags[kBlockUnits], ulocal[kBlockUnits];
#pragma unroll
                    for (int uu = 0; uu < kBlockUnits; ++uu) {
                        uflags[uu] = __shfl(my_flags, 32 + uu, 64);
                        ulocal[uu] = __shfl(my_loc, 32 + uu, 64);
                    }
                    floatx16 acc[2];
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float c = __shfl(my_c, 8 * (r / 4) + 4 * half + (r % 4), 64);
                        acc[0][r] = c;
                        acc[1][r] = c;
                    }
                    // member rows x this wave's points over the whole dimension
                    Piece a[B], b[2][B];
#pragma unroll
                    for (int i = 0; i < B; ++i) {
                        const bool in = i < np;
                        a[i] = (in && alive) ? piece(arow, i) : Piece{};
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb) b[cb][i] = (in && pok[cb]) ? piece(prow[cb], i) : Piece{};
                    }
                    for (int p = 0; p < np; p += B) {
                        const bool more = p + B < np;
                        Piece an[B], bn[2][B];
                        if (more) {
#pragma unroll
                            for (int i = 0; i < B; ++i) {
                                const bool in = p + B + i < np;
                                an[i] = (in && alive) ? piece(arow, p + B + i) : Piece{};
#pragma unroll
                                for (int cb = 0; cb < 2; ++cb)
                                    bn[cb][i] = (in && pok[cb]) ? piece(prow[cb], p + B + i) : Piece{};
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
                    es_units<kWindow>(acc, uflags, ulocal, wsh, cur, half, col, lacc[wave]);
                }
            }
        }
        __syncthreads();
        es_finish<kWindow>(tid, j0, j1, split, l, sc, lacc);
        __syncthreads();
    }
}

// L1 dissimilarity (d(v,s) = sum_k |v_k - s_k|, no dot-product form): the
// same groups and splits, on the vector ALUs. A thread owns one ground point
// of a 256-point pass; the group's non-empty sets are taken in order, each
// set's members 16 at a time, their values staged in LDS 256 dimensions at a
// time (read by every thread at the same address); the thread reads its own
// row in 16-byte pieces where aligned. Per (set, point) the running minimum
// starts at d(v, e0) (m0); the term d(v, e0) - min is added to the thread's
// float accumulator of the set, and the accumulators are summed in float64
// in a fixed order at the end of the item (part holds f * |V| per split).
constexpr int kL1EsWin = 32;  // units per group window (non-empty sets per group <= 32)
constexpr int kL1EsMem = 16;  // members per staged chunk
constexpr int kL1EsK = 256;   // dimensions per staged chunk

__global__ void __launch_bounds__(256)
k_es_l1(const float* __restrict__ x, int64_t n, int32_t d, const double* __restrict__ m0,
        const int64_t* __restrict__ off, const int32_t* __restrict__ idx, int64_t l, int32_t splits, EsScratch sc) {
    __shared__ float lacc[kL1EsWin][256];
    __shared__ __attribute__((aligned(16))) float ms[kL1EsMem][kL1EsK];
    const int tid = threadIdx.x;
    const int64_t n_items = *sc.n_groups * splits;
    const int64_t vchunk = ((n + splits - 1) / splits + kVSub - 1) / kVSub * kVSub;
    const bool vec = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;

    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t g = item / splits;
        const int split = int(item % splits);
        const int64_t j0 = lower_bound_u(sc.U, 0, l, g * kL1EsWin);
        const int64_t j1 = lower_bound_u(sc.U, j0, l, (g + 1) * kL1EsWin);
        const int64_t v_begin = int64_t(split) * vchunk;
        int64_t v_end = v_begin + vchunk;
        if (v_end > n) v_end = n;
        for (int q = 0; q < kL1EsWin; ++q) lacc[q][tid] = 0.0f;  // each thread its own column
        for (int64_t vs = v_begin; vs < v_end; vs += 256) {
            const int64_t v = vs + tid;
            const bool live = v < v_end;
            const double m0v = live ? m0[v] : 0.0;
            const float* __restrict__ xv = x + (live ? v : 0) * d;
            for (int64_t j = j0; j < j1; ++j) {
                if (sc.E[j + 1] == sc.E[j]) continue;  // empty or invalid set (the same for every thread)
                const int loc = int(sc.E[j] - sc.E[j0]);
                const int64_t a = off[j], z = off[j + 1];
                float tmin = float(m0v);
                for (int64_t q0 = a; q0 < z; q0 += kL1EsMem) {
                    const int mc = (z - q0) < kL1EsMem ? int(z - q0) : kL1EsMem;
                    float dist[kL1EsMem];
#pragma unroll
                    for (int m = 0; m < kL1EsMem; ++m) dist[m] = 0.0f;
                    for (int k0 = 0; k0 < d; k0 += kL1EsK) {
                        const int kn = (d - k0) < kL1EsK ? (d - k0) : kL1EsK;
                        __syncthreads();
                        for (int e = tid; e < kL1EsMem * kL1EsK; e += 256) {
                            const int m = e / kL1EsK, k = e % kL1EsK;
                            ms[m][k] = (m < mc && k < kn) ? x[int64_t(idx[q0 + m]) * d + k0 + k] : 0.0f;
                        }
                        __syncthreads();
                        if (live) {
                            int k = 0;
                            if (vec)
                                for (; k + 3 < kn; k += 4) {
                                    const float4 x4 = *reinterpret_cast<const float4*>(xv + k0 + k);
#pragma unroll
                                    for (int m = 0; m < kL1EsMem; ++m) {
                                        const float4 s4 = *reinterpret_cast<const float4*>(&ms[m][k]);
                                        dist[m] += fabsf(x4.x - s4.x);
                                        dist[m] += fabsf(x4.y - s4.y);
                                        dist[m] += fabsf(x4.z - s4.z);
                                        dist[m] += fabsf(x4.w - s4.w);
                                    }
                                }
                            for (; k < kn; ++k) {
                                const float xk = xv[k0 + k];
#pragma unroll
                                for (int m = 0; m < kL1EsMem; ++m) dist[m] += fabsf(xk - ms[m][k]);
                            }
                        }
                    }
#pragma unroll
                    for (int m = 0; m < kL1EsMem; ++m)
                        if (m < mc) tmin = fminf(tmin, dist[m]);
                }
                if (live) lacc[loc][tid] += float(m0v) - tmin;
            }
        }
        __syncthreads();
        for (int64_t j = j0 + tid; j < j1; j += 256) {
            if (sc.E[j + 1] == sc.E[j]) continue;
            const int loc = int(sc.E[j] - sc.E[j0]);
            double t = 0.0;
            for (int c = 0; c < 256; ++c) t += double(lacc[loc][c]);
            sc.part[int64_t(split) * l + j] = t;
        }
        __syncthreads();
    }
}

// f_j = (scale/|V|) sum over splits (fixed order); empty sets 0; bad sets NaN.
// scale: 2 for the halved dot-product terms, 1 for the L1 terms.
__global__ void __launch_bounds__(256) k_es_final(int64_t l, int64_t n, int32_t splits, EsScratch sc, double scale,
                                                  double* __restrict__ f_out) {
    const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (j >= l) return;
    if (sc.bad[j]) {
        f_out[j] = __longlong_as_double(0x7ff8000000000000ll);  // quiet NaN
        return;
    }
    if (sc.E[j + 1] == sc.E[j]) {
        f_out[j] = 0.0;
        return;
    }
    double s = 0.0;
    for (int p = 0; p < splits; ++p) s += sc.part[int64_t(p) * l + j];
    f_out[j] = scale * s / double(n);
}

template <int KP>
void launch_es_main(dim3 g, hipStream_t s, const ebc_dataset* ds, const int64_t* off, const int32_t* idx, int64_t l,
                    int32_t splits, const EsScratch& sc) {
    // an FP32 dataset's own padded rows (up to 120 values): the register
    // kernel first (it takes calls whose sets all have at most kRegMaxSet
    // units), then k_es_main for the others; a reduced-precision dataset
    // evaluated in float32, and 128-value rows, use k_es_main alone
    bool own = false;
    if constexpr (KP <= 120) {
        own = ds->dt == EBC_DT_F32 && ds->k_pad == KP;
        if (own) {
            // the scan chose 4- or 2-row units; the other instance returns at once
            const uint4* xq = static_cast<const uint4*>(static_cast<const void*>(ds->b.xq));
            if (ds->d <= KP - 4) {  // the rows' last 4 slots are padding
                hipLaunchKernelGGL((k_es_regs32<KP, 4, true>), g, dim3(256), 0, s, xq, ds->b.hn, ds->n, ds->b.m0, off,
                                   idx, l, splits, sc);
                hipLaunchKernelGGL((k_es_regs32<KP, 2, true>), g, dim3(256), 0, s, xq, ds->b.hn, ds->n, ds->b.m0, off,
                                   idx, l, splits, sc);
            } else {
                hipLaunchKernelGGL((k_es_regs32<KP, 4, false>), g, dim3(256), 0, s, xq, ds->b.hn, ds->n, ds->b.m0, off,
                                   idx, l, splits, sc);
                hipLaunchKernelGGL((k_es_regs32<KP, 2, false>), g, dim3(256), 0, s, xq, ds->b.hn, ds->n, ds->b.m0, off,
                                   idx, l, splits, sc);
            }
        }
    }
    if (ds->d <= KP - 4)
        hipLaunchKernelGGL((k_es_main<KP, true>), g, dim3(256), 0, s, ds->x, ds->n, ds->d, ds->b.n64, ds->b.m0, off,
                           idx, l, splits, sc, int32_t(own));
    else
        hipLaunchKernelGGL((k_es_main<KP, false>), g, dim3(256), 0, s, ds->x, ds->n, ds->d, ds->b.n64, ds->b.m0, off,
                           idx, l, splits, sc, int32_t(own));
}

}  // namespace

namespace {
// ground-set splits: as many as keep every split at least one pass long
int32_t es_splits(int64_t n) {
    int64_t splits = (n + kVSub - 1) / kVSub;
    return int32_t(splits > kMaxSplits ? kMaxSplits : splits);
}
size_t a256(size_t v) { return (v + 255) & ~size_t(255); }
}  // namespace

size_t eval_sets_scratch_bytes(int64_t n, int64_t l) {
    const int32_t splits = es_splits(n);
    return a256(size_t(l + 1) * sizeof(int64_t)) + a256(size_t(l + 1) * sizeof(int32_t)) +
           a256(size_t(l) * sizeof(int32_t)) + a256(sizeof(int64_t)) + a256(size_t(splits) * size_t(l) * sizeof(double)) +
           a256(size_t(l + 2) * sizeof(int32_t));
}

hipError_t launch_eval_sets(const ebc_dataset* ds, const int64_t* offsets, const int32_t* idx, int64_t l,
                            double* f_out, bool in_dtype, void* scratch, hipStream_t s) {
    const int32_t splits = es_splits(ds->n);
    auto a8 = a256;
    char* base = static_cast<char*>(scratch);
    EsScratch sc;
    char* p = base;
    sc.U = reinterpret_cast<int64_t*>(p);
    p += a8((l + 1) * sizeof(int64_t));
    sc.E = reinterpret_cast<int32_t*>(p);
    p += a8((l + 1) * sizeof(int32_t));
    sc.bad = reinterpret_cast<int32_t*>(p);
    p += a8(l * sizeof(int32_t));
    sc.n_groups = reinterpret_cast<int64_t*>(p);
    p += a8(sizeof(int64_t));
    sc.part = reinterpret_cast<double*>(p);
    p += a8(size_t(splits) * size_t(l) * sizeof(double));
    sc.win_j0 = reinterpret_cast<int32_t*>(p);

    const unsigned nb = unsigned((l + 255) / 256);
    hipLaunchKernelGGL(k_es_units, dim3(nb), dim3(256), 0, s, offsets, idx, l, ds->n, sc, ds->b.state);
    if (ds->metric == 1) {
        // L1: float32 rows of the caller on the vector ALUs, whatever in_dtype says
        hipLaunchKernelGGL(k_es_scan, dim3(1), dim3(1024), 0, s, l, kL1EsWin, sc, offsets, 0);
        hipLaunchKernelGGL(k_es_l1, dim3(2048), dim3(256), 0, s, ds->x, ds->n, ds->d, ds->b.m0, offsets, idx, l,
                           splits, sc);
        hipLaunchKernelGGL(k_es_final, dim3(nb), dim3(256), 0, s, l, ds->n, splits, sc, 1.0, f_out);
        return hipGetLastError();
    }
    const bool lowp = in_dtype && ds->dt != EBC_DT_F32;
    const int lp_kc = ds->k_pad / (ds->dt == EBC_DT_FP8_E4M3 ? 64 : 16);
    // long rows (float32 rows padded to 8, or the cast rows): the long-row kernel
    const bool wide = wide_rows(lowp ? ds->k_pad : (ds->d + 7) / 8 * 8);
    // 2-row units are open to the float32 register kernel only (the dataset's
    // own rows, up to 120 values): the same condition under which
    // launch_es_main launches it
    const int kp32 = (ds->d + 7) / 8 * 8;
    const int32_t reg2 = (!lowp && !wide && ds->dt == EBC_DT_F32 && ds->k_pad == kp32 && kp32 <= 120) ? 1 : 0;
    hipLaunchKernelGGL(k_es_scan, dim3(1), dim3(1024), 0, s, l,
                       (lowp && !wide) ? lp_window(ds->dt, lp_kc) : kWindow, sc, offsets, reg2);
    // persistent grid over (group, split) items; the item count is read on the device
    const dim3 g = dim3(2048);
    if (wide) {
        const ebc_dtype dt = lowp ? ds->dt : EBC_DT_F32;
        // float32 over a float32 dataset: its tiled, centred float32 copy
        const bool own = lowp || ds->dt == EBC_DT_F32;
        const void* src = own ? static_cast<const void*>(ds->b.xq) : static_cast<const void*>(ds->x);
        const int32_t len = own ? ds->k_pad : ds->d;
        switch (dt) {
#define EBC_ESW(DTV, CALLER)                                                                                \
    hipLaunchKernelGGL((k_es_wide<DTV, CALLER>), g, dim3(256), 0, s, src, len, ds->b.hn, ds->b.scale, ds->n,  \
                       ds->b.n64, ds->b.m0, offsets, idx, l, splits, sc)
            case EBC_DT_F32:
                if (own)
                    EBC_ESW(EBC_DT_F32, false);
                else
                    EBC_ESW(EBC_DT_F32, true);
                break;
            case EBC_DT_F16: EBC_ESW(EBC_DT_F16, false); break;
            case EBC_DT_BF16: EBC_ESW(EBC_DT_BF16, false); break;
            case EBC_DT_FP8_E4M3: EBC_ESW(EBC_DT_FP8_E4M3, false); break;
#undef EBC_ESW
            default: return hipErrorInvalidValue;
        }
    } else if (lowp) {
        const int kc = ds->k_pad / (ds->dt == EBC_DT_FP8_E4M3 ? 64 : 16);
        const uint4* xq = static_cast<const uint4*>(static_cast<const void*>(ds->b.xq));
#define EBC_ESL(DTV, K)                                                                                         \
    case K:                                                                                                     \
        hipLaunchKernelGGL((k_es_regs<DTV, K>), g, dim3(256), 0, s, xq, ds->b.hn, ds->b.scale, ds->n, ds->b.m0,   \
                           offsets, idx, l, splits, sc);                                                        \
        hipLaunchKernelGGL((k_es_lp<DTV, K, lp_window(DTV, K)>), g, dim3(256), 0, s, xq, ds->b.hn, ds->b.scale,   \
                           ds->n, ds->b.n64, ds->b.m0, offsets, idx, l, splits, sc);                     \
        break;
        bool ok = true;
        switch (ds->dt) {
            case EBC_DT_BF16:
                switch (kc) {
                    EBC_ESL(EBC_DT_BF16, 1) EBC_ESL(EBC_DT_BF16, 2) EBC_ESL(EBC_DT_BF16, 3) EBC_ESL(EBC_DT_BF16, 4)
                    EBC_ESL(EBC_DT_BF16, 5) EBC_ESL(EBC_DT_BF16, 6) EBC_ESL(EBC_DT_BF16, 7) EBC_ESL(EBC_DT_BF16, 8)
                    default: ok = false;
                }
                break;
            case EBC_DT_F16:
                switch (kc) {
                    EBC_ESL(EBC_DT_F16, 1) EBC_ESL(EBC_DT_F16, 2) EBC_ESL(EBC_DT_F16, 3) EBC_ESL(EBC_DT_F16, 4)
                    EBC_ESL(EBC_DT_F16, 5) EBC_ESL(EBC_DT_F16, 6) EBC_ESL(EBC_DT_F16, 7) EBC_ESL(EBC_DT_F16, 8)
                    default: ok = false;
                }
                break;
            case EBC_DT_FP8_E4M3:
                switch (kc) {
                    EBC_ESL(EBC_DT_FP8_E4M3, 1) EBC_ESL(EBC_DT_FP8_E4M3, 2)
                    default: ok = false;
                }
                break;
            default: ok = false;
        }
#undef EBC_ESL
        if (!ok) return hipErrorInvalidValue;
    } else {
        const int kp = (ds->d + 7) / 8 * 8;
        switch (kp) {
#define EBC_ES(K) \
    case K: launch_es_main<K>(g, s, ds, offsets, idx, l, splits, sc); break;
            EBC_ES(8) EBC_ES(16) EBC_ES(24) EBC_ES(32) EBC_ES(40) EBC_ES(48) EBC_ES(56) EBC_ES(64)
            EBC_ES(72) EBC_ES(80) EBC_ES(88) EBC_ES(96) EBC_ES(104) EBC_ES(112) EBC_ES(120) EBC_ES(128)
#undef EBC_ES
            default: return hipErrorInvalidValue;
        }
    }
    hipLaunchKernelGGL(k_es_final, dim3(nb), dim3(256), 0, s, l, ds->n, splits, sc, 2.0, f_out);
    return hipGetLastError();
}

}  // namespace ebc
