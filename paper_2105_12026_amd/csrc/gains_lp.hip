// Marginal gains with the distances in reduced precision (BF16, FP16 or
// FP8-e4m3 with a power-of-two scale per row) on the MFMA units, float32
// accumulation, float64 cross-lane and cross-chunk sums.
//
// Same quantity as the float32 kernel (G[c] = sum_v max(0, m_v - d(v,c)),
// Sec. 3 discrete derivative, Sec. 4.1 per-point decomposition), halved:
//     G[c]/2 = sum_v max(0, x^_v . x^_c + ha_v - hn_c)
// where x^ are the quantised rows, hn = ||x^||^2/2 in float32, hm_v = m_v/2,
// ha_v = hm_v - hn_v (the term is hm_v - d^(v,c)/2). The accumulator starts
// from the constant tile -hn_c (the MFMA's C operand, the same for every
// ground point), so with lo = -ha_v the term is max(0, acc - lo). The
// epilogue scales it by s = 2^-e (2^e >= hm_v for every point, so the term
// lies in [0, 1]) and takes it with one v_fma_f32 carrying the clamp bit,
//     t = clamp(acc * s + ha_v * s, 0, 1),
// then one add per (candidate, point) pair; the power-of-two scale is exact
// and is undone in float64 when the sums are stored. The clamp at 1 stands
// for the cap at hm_v, which only a computed distance below zero (rounding,
// near-duplicate points) can reach. A term with acc <= lo is exactly 0, so a
// 32 x 32 tile whose every value lies at or below its column's bound adds
// nothing, and the wave skips its epilogue after one test (bitwise the same
// sums).
//
// Grouped order: the ground set is sorted by nearest pivot at residency, and
// candidates (when all points are scored) and points are walked in that
// order, so a tile pairs 32 nearby candidates with 32 nearby points; once a
// point's minimum m_v is below its distance to other regions, whole tiles
// clamp and are skipped (about 80-95% of them on the 200000 x 64 mixture).
// The matrix work is the same for every tile.
//
// Layout in HBM: the quantised rows are stored in tiles of 64 rows,
// "unit-major" inside a tile (16-byte unit u of all 64 rows, then unit u+1).
// One wave instruction (global_load_lds_dwordx4) copies a contiguous
// kilobyte of a tile straight into LDS with no register staging, and the
// MFMA operand reads from LDS are 32 consecutive 16-byte units per half-wave
// (no bank conflicts). A workgroup (4 waves, 32*CB candidates per wave held
// in registers) streams one chunk of the ground set through an LDS ring,
// one barrier per stage: two stages (the copy of stage t+1 issued right
// after the barrier of stage t, while stage t is multiplied) of 64 points,
// up to 256 in the interleaved variant; the ping-pong variant keeps three. MFMA tile: rows = candidates, columns = ground
// points; each lane reads contiguous K from its half of a row (the order of
// K inside a dot product is free as long as both operands use the same one).
#include "ebc_internal.h"
#include "lp_mfma.h"

namespace ebc {


// Geometry of one kernel instance. A ring stage holds VT ground points: VT/64
// consecutive 64-row HBM tiles (contiguous in memory, copied as they lie).
template <int DT, int KC, int CB, int VTS = 64>
struct LpGeom {
    using T = Lp<DT>;
    static constexpr int RB = KC * T::kChunkK * T::kElem;  // bytes per quantised row
    static constexpr int RU = RB / 16;                     // 16-byte units per row
    static constexpr int HU = RU / 2;                      // units per lane half-row
    static constexpr int HT = 64;                          // rows per tile in HBM
    static constexpr int VT = VTS;                         // ground points per ring stage
    static_assert(VT == 64 || VT == 128 || VT == 256, "stages of 64, 128 or 256 points");
    static constexpr int NU = RU * (VT / 64);              // 1 KB unit pieces per stage
    static constexpr bool kFp8 = DT == EBC_DT_FP8_E4M3;
    // per-point pieces (ha, FP8 scales): one 16-byte-per-lane copy per 256
    // points, else one 4-byte-per-lane copy per 64 points
    static constexpr int PB = VT % 256 == 0 ? 16 : 4;       // bytes per lane of a per-point piece
    static constexpr int PP = VT * 4 / (64 * PB);           // pieces per per-point array
    // LDS stage: [VT/64 tiles][RU units][64 rows][ha: VT floats][scale: VT ints]
    static constexpr int OFF_HA = NU * 64;
    static constexpr int OFF_SC = OFF_HA + VT / 4;
    static constexpr int STAGE = OFF_SC + (kFp8 ? VT / 4 : 0);  // uint4 per stage
    static constexpr int NI = NU + PP * (kFp8 ? 2 : 1);        // wave copy instructions per stage
    static constexpr int L = (NI + 3) / 4;                      // copy instructions per wave per stage
    static constexpr int CAND_TILE = 4 * 32 * CB;
};

// Wave-wide copy of one piece of ground-set stage `tile` into LDS stage `st`.
// Piece j: j < NU unit piece j (a kilobyte of one 64-row tile); then the ha
// pieces; then (FP8) the row-scale pieces.
template <class G>
__device__ __forceinline__ void copy_piece(int j, int64_t tile, int lane, const uint4* __restrict__ xqt,
                                           const float* __restrict__ ha, const int* __restrict__ sc, uint4* st) {
    if (j < G::NU) {
        __builtin_amdgcn_global_load_lds(xqt + (tile * G::NU + j) * 64 + lane, (lds_void*)(st + j * 64), 16, 0, 0);
        return;
    }
    int k = j - G::NU;
    const bool scale = k >= G::PP;
    if (scale) k -= G::PP;
    const void* src = scale ? static_cast<const void*>(sc + tile * G::VT) : static_cast<const void*>(ha + tile * G::VT);
    uint4* dst = st + (scale ? G::OFF_SC : G::OFF_HA);
    if (G::PB == 16)
        __builtin_amdgcn_global_load_lds(static_cast<const uint4*>(src) + k * 64 + lane, (lds_void*)(dst + k * 64), 16,
                                         0, 0);
    else
        __builtin_amdgcn_global_load_lds(static_cast<const float*>(src) + k * 64 + lane, (lds_void*)(dst + k * 16), 4,
                                         0, 0);
}

// Every wave issues exactly L copy instructions per stage (some repeat a
// piece another wave also copies: same bytes to the same place), so the
// vector-memory counter is the same on every wave.
template <class G>
__device__ __forceinline__ void copy_stage(int wave, int lane, int64_t tile, const uint4* __restrict__ xqt,
                                           const float* __restrict__ ha, const int* __restrict__ sc, uint4* st) {
#pragma unroll
    for (int l = 0; l < G::L; ++l) copy_piece<G>((wave + 4 * l) % G::NI, tile, lane, xqt, ha, sc, st);
}

// One ground-set tile: wait for its copy, start the copy of the next tile
// into the other stage `next2`, then the MFMAs and the fused clamp-and-sum
// epilogue against the wave's candidate blocks.
template <class G, int DT, int KC, int CB>
__device__ __forceinline__ void lp_tile(int64_t t, int64_t nt, int64_t t_begin, int wave, int lane, int col, int half,
                                        const uint4* __restrict__ xqt, const float* __restrict__ ha,
                                        const int* __restrict__ sc, const uint4* st,
                                        uint4* next2, const uint4 (&a)[CB][G::HU], const floatx16 (&cinit)[CB],
                                        const int (&sa)[CB], float (&acc_sum)[CB][16], float s) {
    using T = Lp<DT>;
    constexpr int HU = G::HU, VT = G::VT;
    // this wave's copies of tile t are done ...
    wait_vmcnt<0>();
    // ... and every wave's, and every wave finished reading tile t-1, whose
    // stage the next copy overwrites
    ring_barrier();
    if (t + 1 < nt) copy_stage<G>(wave, lane, t_begin + t + 1, xqt, ha, sc, next2);
    const float* st_ha = reinterpret_cast<const float*>(st + G::OFF_HA);
    const int* st_sc = reinterpret_cast<const int*>(st + G::OFF_SC);
#pragma unroll
    for (int colb = 0; colb < VT / 32; ++colb) {
        const int vrow = colb * 32 + col;
        uint4 b[HU];
#pragma unroll
        for (int u = 0; u < HU; ++u) b[u] = st[(half * HU + u) * VT + vrow];
        const float hav = st_ha[vrow];
        const float lo = -hav, sh = hav * s;
        const int sb = G::kFp8 ? st_sc[vrow] : 127;
        // CB independent accumulator chains, each starting from -hn_c
        floatx16 acc[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[cb] = cinit[cb];
#pragma unroll
        for (int q = 0; q < KC; ++q)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                acc[cb] = mfma_main<DT>(&a[cb][q * T::kU4], &b[q * T::kU4], acc[cb], sa[cb], sb);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) clamp_sum16(acc[cb], lo, s, sh, acc_sum[cb]);
    }
}

// Software-pipelined variant of lp_tile: the MFMAs of each column block are
// issued before the epilogue of the previous block (kept in `prev`, also
// across tiles), and sched_group_barrier asks the scheduler to interleave one
// MFMA with a slice of that epilogue, so each wave keeps the matrix unit
// busy while its VALU clamps and sums the previous block.
template <class G, int DT, int KC, int CB>
__device__ __forceinline__ void lp_tile_pipe(int64_t t, int64_t nt, int64_t t_begin, int wave, int lane, int col,
                                             int half, const uint4* __restrict__ xqt, const float* __restrict__ ha,
                                             const int* __restrict__ sc,
                                             const uint4* st, uint4* next2, const uint4 (&a)[CB][G::HU],
                                             const floatx16 (&cinit)[CB], const int (&sa)[CB],
                                             float (&acc_sum)[CB][16],
                                             floatx16 (&prev)[CB], float& prev_lo, float& prev_sh, bool& pending, float s) {
    using T = Lp<DT>;
    constexpr int HU = G::HU, VT = G::VT;
    constexpr int NMF = KC * CB;            // matrix instructions per column block
    constexpr int NVA = 2 * 16 * CB;        // epilogue VALU instructions per column block
    constexpr int PER = (NVA + NMF - 1) / NMF;
    wait_vmcnt<0>();
    ring_barrier();
    if (t + 1 < nt) copy_stage<G>(wave, lane, t_begin + t + 1, xqt, ha, sc, next2);
    const float* st_ha = reinterpret_cast<const float*>(st + G::OFF_HA);
    const int* st_sc = reinterpret_cast<const int*>(st + G::OFF_SC);
#pragma unroll
    for (int colb = 0; colb < VT / 32; ++colb) {
        const int vrow = colb * 32 + col;
        uint4 b[HU];
#pragma unroll
        for (int u = 0; u < HU; ++u) b[u] = st[(half * HU + u) * VT + vrow];
        const float hav = st_ha[vrow];
        const float lo = -hav, sh = hav * s;
        const int sb = G::kFp8 ? st_sc[vrow] : 127;
        floatx16 acc[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[cb] = cinit[cb];
#pragma unroll
        for (int q = 0; q < KC; ++q)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                acc[cb] = mfma_main<DT>(&a[cb][q * T::kU4], &b[q * T::kU4], acc[cb], sa[cb], sb);
        if (pending) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) clamp_sum16(prev[cb], prev_lo, s, prev_sh, acc_sum[cb]);
        }
#pragma unroll
        for (int i = 0; i < NMF; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, PER, 0);  // then a slice of VALU
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) prev[cb] = acc[cb];
        prev_lo = lo;
        prev_sh = sh;
        pending = true;
    }
}

// Candidate rows of one wave (A operand, 32*CB rows), their E8M0 scales and
// the constant accumulator tiles -hn_c, in registers.
template <class G, int DT, int CB>
__device__ __forceinline__ void load_candidates(const GainsArgs& ga, int64_t wbase, int col, int half,
                                                uint4 (&a)[CB][G::HU], floatx16 (&cinit)[CB], int (&sa)[CB]) {
    constexpr int HU = G::HU, RU = G::RU, HT = G::HT;
    const uint4* __restrict__ xqt = static_cast<const uint4*>(ga.xq);
    const int32_t* __restrict__ cand = ga.cand;
    const int64_t n_cand = ga.n_cand, n_pad = ga.n_pad;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int64_t cpos = wbase + cb * 32 + col;
        int64_t crow = -1;  // slot of the candidate's row (its row without the grouped order)
        if (cpos < n_cand) crow = cand ? int64_t(cand[cpos]) : cpos;
        if (crow >= n_pad || (cpos < n_cand && crow < 0)) {
            atomicCAS(ga.err, 0, kDevErrIndex);
            crow = -1;
        }
        if (crow >= 0 && cand && ga.inv) crow = ga.inv[crow];
        if (crow >= 0) {
            const uint4* src = xqt + (crow / HT) * (RU * HT) + (crow % HT);
#pragma unroll
            for (int u = 0; u < HU; ++u) a[cb][u] = src[(half * HU + u) * HT];
            sa[cb] = G::kFp8 ? ga.scale[crow] : 127;
        } else {
#pragma unroll
            for (int u = 0; u < HU; ++u) a[cb][u] = make_uint4(0, 0, 0, 0);
            sa[cb] = 127;
        }
        // the lane holds result rows 8*(r/4) + 4*half + r%4 of this block
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t p = wbase + cb * 32 + 8 * (r / 4) + 4 * half + (r % 4);
            float v = 0.0f;
            if (p < n_cand) {
                int64_t row = cand ? int64_t(cand[p]) : p;
                if (row >= 0 && row < n_pad) {
                    if (cand && ga.inv) row = ga.inv[row];
                    v = ga.hn[row];
                }
            }
            cinit[cb][r] = -v;
        }
    }
}

// float64 sums over the 32 columns of each half, scaled back by 2^ge; one
// lane per row writes.
// In the grouped order (all candidates, no list) a slot's sum goes to its row.
template <int CB>
__device__ __forceinline__ void store_partials(const GainsArgs& ga, int64_t wbase, int split, int col, int half,
                                               const float (&acc_sum)[CB][16], int ge) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        double mine = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double v = double(acc_sum[cb][r]);
#pragma unroll
            for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (col == r) mine = v;
        }
        if (col < 16) {
            const int r = col;
            const int64_t p = wbase + cb * 32 + 8 * (r / 4) + 4 * half + (r % 4);
            if (p < ga.n_cand) {
                const int64_t at = (ga.perm && !ga.cand) ? int64_t(ga.perm[p]) : p;
                ga.part[int64_t(split) * ga.part_stride + at] = ldexp(2.0 * mine, ge);  // exact: a power of two
            }
        }
    }
}

template <int DT, int KC, int CB, bool PIPE>
__device__ __forceinline__ void gains_lp_body(const GainsArgs& ga, int64_t bid) {
    const uint4* __restrict__ xqt = static_cast<const uint4*>(ga.xq);
    const float* __restrict__ ha = ga.ha;
    const int* __restrict__ sc = ga.scale;
    const int ge = *ga.gexp;                // 2^ge >= m_v / 2 for every point
    const float s = ldexpf(1.0f, -ge);      // the epilogue's power-of-two scale
    const int64_t n_pad = ga.n_pad, chunk = ga.chunk;
    const int32_t v_splits = ga.v_splits;
    using G = LpGeom<DT, KC, CB>;
    using T = Lp<DT>;
    constexpr int HU = G::HU, VT = G::VT;
    static_assert(HU == KC * T::kU4, "lane half-row must hold KC chunks");

    __shared__ uint4 lds0[G::STAGE];
    __shared__ uint4 lds1[G::STAGE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 31;
    const int half = lane >> 5;
    const int split = int(bid % v_splits);
    const int64_t ctile = bid / v_splits;
    const int64_t wbase = ctile * G::CAND_TILE + int64_t(wave) * (32 * CB);

    // ---- candidate rows (A operand) and -hn of the result rows, in registers ----
    uint4 a[CB][HU];
    floatx16 cinit[CB];
    int sa[CB];
    load_candidates<G, DT, CB>(ga, wbase, col, half, a, cinit, sa);
    float acc_sum[CB][16];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc_sum[cb][r] = 0.0f;

    // ---- stream the ground-set chunk through the LDS ring ----
    const int64_t v_begin = int64_t(split) * chunk;
    int64_t v_end = v_begin + chunk;
    if (v_end > n_pad) v_end = n_pad;
    const int64_t t_begin = v_begin / VT;
    const int64_t nt = v_end > v_begin ? (v_end - v_begin) / VT : 0;

    if (nt > 0) copy_stage<G>(wave, lane, t_begin, xqt, ha, sc, lds0);
    // two stages are two distinct LDS objects and the loop is unrolled by
    // two, so the compiler can see that the copy in flight never targets the
    // stage being read and does not wait for it
    if (PIPE) {
        floatx16 prev[CB];
        float prev_lo = 0.0f, prev_sh = 0.0f;
        bool pending = false;
        for (int64_t t = 0; t < nt; t += 2) {
            lp_tile_pipe<G, DT, KC, CB>(t, nt, t_begin, wave, lane, col, half, xqt, ha, sc, lds0, lds1, a,
                                        cinit, sa, acc_sum, prev, prev_lo, prev_sh, pending, s);
            if (t + 1 < nt)
                lp_tile_pipe<G, DT, KC, CB>(t + 1, nt, t_begin, wave, lane, col, half, xqt, ha, sc, lds1, lds0,
                                            a, cinit, sa, acc_sum, prev, prev_lo, prev_sh, pending, s);
        }
        if (pending) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) clamp_sum16(prev[cb], prev_lo, s, prev_sh, acc_sum[cb]);
        }
    } else {
        for (int64_t t = 0; t < nt; t += 2) {
            lp_tile<G, DT, KC, CB>(t, nt, t_begin, wave, lane, col, half, xqt, ha, sc, lds0, lds1, a, cinit, sa,
                                   acc_sum, s);
            if (t + 1 < nt)
                lp_tile<G, DT, KC, CB>(t + 1, nt, t_begin, wave, lane, col, half, xqt, ha, sc, lds1, lds0, a,
                                       cinit, sa, acc_sum, s);
        }
    }

    store_partials<CB>(ga, wbase, split, col, half, acc_sum, ge);
}

// ---------------------------------------------------------------------------
// Ping-pong variant: 8 waves, two per SIMD. At d = 64 in BF16 the epilogue
// (one clamped fma and one add per pair, 4 cycles per wave instruction) costs as
// many cycles as the matrix instructions, and a single wave cannot keep
// both busy because its epilogue depends on its own MFMA results. Here the
// two waves of a SIMD belong to two groups that run half a period apart:
// while one group issues the matrix instructions of tile t, the other clamps
// and sums its tile t-1, and a workgroup barrier swaps the roles. Both groups
// read the same LDS tiles (so one tile copy now feeds 256 or more
// candidates), only the leading group issues the copies, and each group
// prefetches the next tile's operands into registers during its epilogue
// phase. Per-lane sums run in the same order as in the other variants, so
// the gains are bitwise identical.
// ---------------------------------------------------------------------------
template <class G>
struct TileRegs {
    static constexpr int NCB = G::VT / 32;
    uint4 b[NCB][G::HU];
    float ha[NCB];  // raw, so that no instruction waits for this read before the next phase
    int sb[NCB];
};

template <class G>
__device__ __forceinline__ void read_tile(const uint4* st, int col, int half, TileRegs<G>& r) {
    const float* st_ha = reinterpret_cast<const float*>(st + G::OFF_HA);
    const int* st_sc = reinterpret_cast<const int*>(st + G::OFF_SC);
#pragma unroll
    for (int colb = 0; colb < TileRegs<G>::NCB; ++colb) {
        const int vrow = colb * 32 + col;
#pragma unroll
        for (int u = 0; u < G::HU; ++u) r.b[colb][u] = st[(half * G::HU + u) * G::VT + vrow];
        r.ha[colb] = st_ha[vrow];
        r.sb[colb] = G::kFp8 ? st_sc[vrow] : 127;
    }
}

template <class G, int DT, int KC, int CB>
__device__ __forceinline__ void mfma_tile(const TileRegs<G>& r, const uint4 (&a)[CB][G::HU],
                                          const floatx16 (&cinit)[CB], const int (&sa)[CB],
                                          floatx16 (&acc)[TileRegs<G>::NCB][CB]) {
    using T = Lp<DT>;
#pragma unroll
    for (int colb = 0; colb < TileRegs<G>::NCB; ++colb) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[colb][cb] = cinit[cb];
#pragma unroll
        for (int q = 0; q < KC; ++q)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                acc[colb][cb] =
                    mfma_main<DT>(&a[cb][q * T::kU4], &r.b[colb][q * T::kU4], acc[colb][cb], sa[cb], r.sb[colb]);
    }
}

template <int NCB, int CB>
__device__ __forceinline__ void epilogue_tile(const floatx16 (&acc)[NCB][CB], const float (&lo)[NCB],
                                              const float (&sh)[NCB], float s, float (&acc_sum)[CB][16]) {
#pragma unroll
    for (int colb = 0; colb < NCB; ++colb) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) clamp_sum16(acc[colb][cb], lo[colb], s, sh[colb], acc_sum[cb]);
    }
}

// Phase boundary: no instruction is scheduled across it, LDS reads drained,
// workgroup barrier.
__device__ __forceinline__ void phase_barrier() {
    __builtin_amdgcn_sched_barrier(0);
    ring_barrier();
    __builtin_amdgcn_sched_barrier(0);
}

// Leading group, tile t: phase 2t (copies of tile t+2, matrix work of tile
// t), phase 2t+1 (operands of tile t+1, epilogue of tile t).
template <class G, int DT, int KC, int CB>
__device__ __forceinline__ void pp_lead(int64_t t, int64_t nt, int64_t t_begin, int wave, int lane, int col, int half,
                                        const uint4* __restrict__ xqt, const float* __restrict__ ha,
                                        const int* __restrict__ sc, const uint4* nxt,
                                        uint4* nx2, TileRegs<G>& r, const uint4 (&a)[CB][G::HU],
                                        const floatx16 (&cinit)[CB], const int (&sa)[CB], float (&acc_sum)[CB][16],
                                        float s) {
    constexpr int NCB = TileRegs<G>::NCB;
    if (t + 2 < nt) copy_stage<G>(wave, lane, t_begin + t + 2, xqt, ha, sc, nx2);
    floatx16 acc[NCB][CB];
    // the whole matrix phase at raised priority (lowered after the barrier
    // that ends it), so each MFMA issues as soon as the matrix pipe takes it
    // even while the other wave has VALU work
    __builtin_amdgcn_s_setprio(1);
    mfma_tile<G, DT, KC, CB>(r, a, cinit, sa, acc);
    float lo[NCB], sh[NCB];
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        lo[c] = -r.ha[c];
        sh[c] = r.ha[c] * s;
    }
    // this wave's copies of tile t+1 have landed (those of t+2 may still fly)
    if (t + 1 < nt) {
        if (t + 2 < nt)
            wait_vmcnt<G::L>();
        else
            wait_vmcnt<0>();
    }
    phase_barrier();
    __builtin_amdgcn_s_setprio(0);
    if (t + 1 < nt) read_tile<G>(nxt, col, half, r);
    epilogue_tile<NCB, CB>(acc, lo, sh, s, acc_sum);
    phase_barrier();
}

// Following group, tile t: phase 2t+1 (matrix work of tile t), phase 2t+2
// (operands of tile t+1, epilogue of tile t; no barrier after the last).
template <class G, int DT, int KC, int CB>
__device__ __forceinline__ void pp_follow(int64_t t, int64_t nt, int col, int half, const uint4* nxt, TileRegs<G>& r,
                                          const uint4 (&a)[CB][G::HU], const floatx16 (&cinit)[CB],
                                          const int (&sa)[CB], float (&acc_sum)[CB][16], float s) {
    constexpr int NCB = TileRegs<G>::NCB;
    floatx16 acc[NCB][CB];
    // the whole matrix phase at raised priority (lowered after the barrier
    // that ends it), so each MFMA issues as soon as the matrix pipe takes it
    // even while the other wave has VALU work
    __builtin_amdgcn_s_setprio(1);
    mfma_tile<G, DT, KC, CB>(r, a, cinit, sa, acc);
    float lo[NCB], sh[NCB];
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        lo[c] = -r.ha[c];
        sh[c] = r.ha[c] * s;
    }
    phase_barrier();
    __builtin_amdgcn_s_setprio(0);
    if (t + 1 < nt) read_tile<G>(nxt, col, half, r);
    epilogue_tile<NCB, CB>(acc, lo, sh, s, acc_sum);
    if (t + 1 < nt) phase_barrier();
}

template <int DT, int KC, int CB>
__device__ __forceinline__ void gains_lp_pp_body(const GainsArgs& ga, int64_t bid) {
    const uint4* __restrict__ xqt = static_cast<const uint4*>(ga.xq);
    const float* __restrict__ ha = ga.ha;
    const int* __restrict__ sc = ga.scale;
    const int ge = *ga.gexp;                // 2^ge >= m_v / 2 for every point
    const float s = ldexpf(1.0f, -ge);      // the epilogue's power-of-two scale
    using G = LpGeom<DT, KC, CB>;
    using T = Lp<DT>;
    constexpr int HU = G::HU, VT = G::VT;
    static_assert(HU == KC * T::kU4, "lane half-row must hold KC chunks");

    __shared__ uint4 lds0[G::STAGE];
    __shared__ uint4 lds1[G::STAGE];
    __shared__ uint4 lds2[G::STAGE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // 0..7, uniform per wave
    const int grp = wave >> 2;                                   // waves w and w+4 share a SIMD
    const int col = lane & 31;
    const int half = lane >> 5;
    const int split = int(bid % ga.v_splits);
    const int64_t ctile = bid / ga.v_splits;
    const int64_t wbase = ctile * (2 * G::CAND_TILE) + int64_t(wave) * (32 * CB);

    uint4 a[CB][HU];
    floatx16 cinit[CB];
    int sa[CB];
    load_candidates<G, DT, CB>(ga, wbase, col, half, a, cinit, sa);
    float acc_sum[CB][16];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc_sum[cb][r] = 0.0f;

    const int64_t v_begin = int64_t(split) * ga.chunk;
    int64_t v_end = v_begin + ga.chunk;
    if (v_end > ga.n_pad) v_end = ga.n_pad;
    const int64_t t_begin = v_begin / VT;
    const int64_t nt = v_end > v_begin ? (v_end - v_begin) / VT : 0;

    TileRegs<G> r;
    if (grp == 0) {
        // leading group: issues every copy; barriers B0 + 2 per tile
        const int w4 = wave & 3;
        if (nt > 0) copy_stage<G>(w4, lane, t_begin, xqt, ha, sc, lds0);
        if (nt > 1) copy_stage<G>(w4, lane, t_begin + 1, xqt, ha, sc, lds1);
        if (nt > 1)
            wait_vmcnt<G::L>();
        else
            wait_vmcnt<0>();
        phase_barrier();  // B0: tile 0 in LDS
        if (nt > 0) read_tile<G>(lds0, col, half, r);
        for (int64_t t = 0; t < nt; t += 3) {
            pp_lead<G, DT, KC, CB>(t, nt, t_begin, w4, lane, col, half, xqt, ha, sc, lds1, lds2, r, a, cinit, sa,
                                   acc_sum, s);
            if (t + 1 < nt)
                pp_lead<G, DT, KC, CB>(t + 1, nt, t_begin, w4, lane, col, half, xqt, ha, sc, lds2, lds0, r, a,
                                       cinit, sa, acc_sum, s);
            if (t + 2 < nt)
                pp_lead<G, DT, KC, CB>(t + 2, nt, t_begin, w4, lane, col, half, xqt, ha, sc, lds0, lds1, r, a,
                                       cinit, sa, acc_sum, s);
        }
    } else {
        // following group, one phase behind: barriers B0 + 1 + 2 per tile - 1
        phase_barrier();  // B0
        if (nt > 0) {
            read_tile<G>(lds0, col, half, r);
            phase_barrier();  // end of phase 0 (the leading group's first matrix phase)
            for (int64_t t = 0; t < nt; t += 3) {
                pp_follow<G, DT, KC, CB>(t, nt, col, half, lds1, r, a, cinit, sa, acc_sum, s);
                if (t + 1 < nt)
                    pp_follow<G, DT, KC, CB>(t + 1, nt, col, half, lds2, r, a, cinit, sa, acc_sum, s);
                if (t + 2 < nt)
                    pp_follow<G, DT, KC, CB>(t + 2, nt, col, half, lds0, r, a, cinit, sa, acc_sum, s);
            }
        }
    }
    store_partials<CB>(ga, wbase, split, col, half, acc_sum, ge);
}

// ---------------------------------------------------------------------------
// Interleaved variant (4): one wave keeps its matrix unit and its vector ALU
// busy together. A column block's matrix instructions are issued alternately
// with the bound test of the previous block's tiles (max over the 16 values
// of each lane, one compare and a wave-wide ballot: all in one basic block,
// so the scheduler can put the test between the MFMAs, where it runs while
// they execute); the clamp-and-sum then runs only for a previous tile with a
// value above its bound. A ring stage holds wide_stage(DT, KC) points (one
// barrier per stage), and the ring has two stages: the copy of stage t+1 is
// issued right after the barrier of stage t (three stages, with the copy of
// t+2 in flight, measured 1-2% slower); both column blocks' operands of each
// 64-point tile of the stage are read from LDS together. The previous block's values carry
// over tile and stage boundaries, and the very first test sees -inf (no tile
// to sum). Per-lane sums are added in column-block order with the same
// arithmetic as clamp_sum16, so gains are bitwise those of the other
// variants.
// ---------------------------------------------------------------------------
template <int CB>
__device__ __forceinline__ void sp_test(const floatx16 (&acc)[CB], float lo, uint64_t (&hit)[CB]) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        float m = fmaxf(fmaxf(acc[cb][0], acc[cb][1]), acc[cb][2]);
#pragma unroll
        for (int r = 3; r < 15; r += 2) m = fmaxf(fmaxf(m, acc[cb][r]), acc[cb][r + 1]);
        m = fmaxf(m, acc[cb][15]);
        hit[cb] = __builtin_amdgcn_ballot_w64(m > lo);
    }
}

template <int CB>
__device__ __forceinline__ void sp_sum(const floatx16 (&acc)[CB], float s, float sh, const uint64_t (&hit)[CB],
                                       float (&acc_sum)[CB][16]) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        if (hit[cb] == 0) continue;
        float t[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) t[r] = __builtin_amdgcn_fmed3f(fmaf(acc[cb][r], s, sh), 0.0f, 1.0f);
        asm volatile(""
                     : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]), "+v"(t[6]),
                       "+v"(t[7]), "+v"(t[8]), "+v"(t[9]), "+v"(t[10]), "+v"(t[11]), "+v"(t[12]), "+v"(t[13]),
                       "+v"(t[14]), "+v"(t[15]));
#pragma unroll
        for (int r = 0; r < 16; ++r) acc_sum[cb][r] += t[r];
    }
}

// One column block: MFMAs into acc, interleaved with the test of pacc (the
// previous block, bound plo, shift psh), then the previous block's clamp-and-sum
// where the test found values above the bound.
template <class G, int DT, int KC, int CB>
__device__ __forceinline__ void sp_colb(const uint4 (&b)[G::HU], int sb, const uint4 (&a)[CB][G::HU],
                                        const floatx16 (&cinit)[CB], const int (&sa)[CB], floatx16 (&acc)[CB],
                                        const floatx16 (&pacc)[CB], float plo, float psh, float s,
                                        float (&acc_sum)[CB][16]) {
    using T = Lp<DT>;
    constexpr int NMF = KC * CB;     // matrix instructions of the block
    constexpr int NVA = 12 * CB;     // test instructions of the previous block
    constexpr int PER = (NVA + NMF - 1) / NMF;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[cb] = cinit[cb];
#pragma unroll
    for (int q = 0; q < KC; ++q)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[cb] = mfma_main<DT>(&a[cb][q * T::kU4], &b[q * T::kU4], acc[cb], sa[cb], sb);
    uint64_t hit[CB];
    sp_test<CB>(pacc, plo, hit);
#pragma unroll
    for (int i = 0; i < NMF; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, PER, 0);  // then part of the test
    }
    uint64_t any = 0;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) any |= hit[cb];
    if (any) sp_sum<CB>(pacc, s, psh, hit, acc_sum);
}

// One ring stage (VT/64 sub-tiles of two column blocks each) of the
// interleaved variant.
template <class G, int DT, int KC, int CB>
__device__ __forceinline__ void sp_tile(int64_t t, int64_t nt, int64_t t_begin, int wave, int lane, int col, int half,
                                        const uint4* __restrict__ xqt, const float* __restrict__ ha,
                                        const int* __restrict__ sc, const uint4* st,
                                        uint4* next2, const uint4 (&a)[CB][G::HU], const floatx16 (&cinit)[CB],
                                        const int (&sa)[CB], float (&acc_sum)[CB][16], floatx16 (&accA)[CB],
                                        floatx16 (&accB)[CB], float& loB, float& shB, float s) {
    constexpr int HU = G::HU, RU = G::RU;
    wait_vmcnt<0>();  // this stage's copies, issued one stage ago
    ring_barrier();   // ... of every wave; every wave is done reading the other stage
    if (t + 1 < nt) copy_stage<G>(wave, lane, t_begin + t + 1, xqt, ha, sc, next2);
    const float* st_ha = reinterpret_cast<const float*>(st + G::OFF_HA);
    const int* st_sc = reinterpret_cast<const int*>(st + G::OFF_SC);
#pragma unroll
    for (int p = 0; p < G::VT / 64; ++p) {
        const uint4* sub = st + p * RU * 64;  // 64-row tile p of the stage
        uint4 b0[HU], b1[HU];
#pragma unroll
        for (int u = 0; u < HU; ++u) b0[u] = sub[(half * HU + u) * 64 + col];
#pragma unroll
        for (int u = 0; u < HU; ++u) b1[u] = sub[(half * HU + u) * 64 + 32 + col];
        const float ha0 = st_ha[p * 64 + col], ha1 = st_ha[p * 64 + 32 + col];
        const int sb0 = G::kFp8 ? st_sc[p * 64 + col] : 127, sb1 = G::kFp8 ? st_sc[p * 64 + 32 + col] : 127;
        const float lo0 = -ha0, sh0 = ha0 * s;
        // column block 0 (into accA) with the previous block (accB)
        sp_colb<G, DT, KC, CB>(b0, sb0, a, cinit, sa, accA, accB, loB, shB, s, acc_sum);
        // column block 1 (into accB) with block 0 (accA)
        sp_colb<G, DT, KC, CB>(b1, sb1, a, cinit, sa, accB, accA, lo0, sh0, s, acc_sum);
        loB = -ha1;
        shB = ha1 * s;
    }
}

template <int DT, int KC, int CB, int VTS>
__device__ __forceinline__ void gains_lp_sp_body(const GainsArgs& ga, int64_t bid) {
    const uint4* __restrict__ xqt = static_cast<const uint4*>(ga.xq);
    const float* __restrict__ ha = ga.ha;
    const int* __restrict__ sc = ga.scale;
    const int ge = *ga.gexp;                // 2^ge >= m_v / 2 for every point
    const float s = ldexpf(1.0f, -ge);      // the epilogue's power-of-two scale
    using G = LpGeom<DT, KC, CB, VTS>;
    using T = Lp<DT>;
    constexpr int HU = G::HU, VT = G::VT;
    static_assert(HU == KC * T::kU4, "lane half-row must hold KC chunks");

    __shared__ uint4 lds0[G::STAGE];
    __shared__ uint4 lds1[G::STAGE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave: scalar copy branches
    const int col = lane & 31;
    const int half = lane >> 5;
    const int split = int(bid % ga.v_splits);
    const int64_t ctile = bid / ga.v_splits;
    const int64_t wbase = ctile * G::CAND_TILE + int64_t(wave) * (32 * CB);

    uint4 a[CB][HU];
    floatx16 cinit[CB];
    int sa[CB];
    load_candidates<G, DT, CB>(ga, wbase, col, half, a, cinit, sa);
    float acc_sum[CB][16];
    floatx16 accA[CB], accB[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc_sum[cb][r] = 0.0f;
            accB[cb][r] = -INFINITY;  // no previous block yet: its test finds nothing
        }
    float loB = 0.0f, shB = 0.0f;

    const int64_t v_begin = int64_t(split) * ga.chunk;
    int64_t v_end = v_begin + ga.chunk;
    if (v_end > ga.n_pad) v_end = ga.n_pad;
    const int64_t t_begin = v_begin / VT;
    const int64_t nt = v_end > v_begin ? (v_end - v_begin) / VT : 0;

    if (nt > 0) copy_stage<G>(wave, lane, t_begin, xqt, ha, sc, lds0);
    for (int64_t t = 0; t < nt; t += 2) {
        sp_tile<G, DT, KC, CB>(t, nt, t_begin, wave, lane, col, half, xqt, ha, sc, lds0, lds1, a, cinit, sa,
                               acc_sum, accA, accB, loB, shB, s);
        if (t + 1 < nt)
            sp_tile<G, DT, KC, CB>(t + 1, nt, t_begin, wave, lane, col, half, xqt, ha, sc, lds1, lds0, a, cinit,
                                   sa, acc_sum, accA, accB, loB, shB, s);
    }
    // the last column block
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) clamp_sum16(accB[cb], loB, s, shB, acc_sum[cb]);
    store_partials<CB>(ga, wbase, split, col, half, acc_sum, ge);
}

template <int DT, int KC, int CB, int VTS>
__global__ void __launch_bounds__(256) k_gains_lp_sp(GainsArgs ga) {
    gains_lp_sp_body<DT, KC, CB, VTS>(ga, blockIdx.x);
}

template <int DT, int KC, int CB, int VTS>
__global__ void __launch_bounds__(256)
kb_gains_lp_sp(const InstDesc* __restrict__ descs, const int32_t* __restrict__ slot_inst,
               const int64_t* __restrict__ wg_pre, int32_t slots, int32_t t) {
    const int j = find_slot(wg_pre, slots, blockIdx.x);
    const InstDesc c = descs[slot_inst[j]];
    if (c.t0 + t >= c.k) return;
    gains_lp_sp_body<DT, KC, CB, VTS>(gains_args(c, nullptr, c.n_pad), int64_t(blockIdx.x) - wg_pre[j]);
}

// Ring-stage width of the interleaved variant by row length (16-byte units
// per row, measured): 256 points for BF16/FP16 rows of 4 units, 128 for FP8
// rows of 4 units and for rows of 8 units, else 64. Wider stages mean fewer
// barriers and copy waits per matrix instruction; rows of 2 units measured
// slower with them, and longer rows have no LDS left for them at two
// workgroups per CU.
constexpr int wide_stage(int DT, int KC) {
    return (DT == EBC_DT_FP8_E4M3 ? 4 * KC : 2 * KC) == 4   ? (DT == EBC_DT_FP8_E4M3 ? 128 : 256)
           : (DT == EBC_DT_FP8_E4M3 ? 4 * KC : 2 * KC) == 8 ? 128
                                                            : 64;
}

template <int DT, int KC, int CB>
__global__ void __launch_bounds__(512) k_gains_lp_pp(GainsArgs ga) {
    gains_lp_pp_body<DT, KC, CB>(ga, blockIdx.x);
}

template <int DT, int KC, int CB>
__global__ void __launch_bounds__(512)
kb_gains_lp_pp(const InstDesc* __restrict__ descs, const int32_t* __restrict__ slot_inst,
               const int64_t* __restrict__ wg_pre, int32_t slots, int32_t t) {
    const int j = find_slot(wg_pre, slots, blockIdx.x);
    const InstDesc c = descs[slot_inst[j]];
    if (c.t0 + t >= c.k) return;
    gains_lp_pp_body<DT, KC, CB>(gains_args(c, nullptr, c.n_pad), int64_t(blockIdx.x) - wg_pre[j]);
}

template <int DT, int KC, int CB, bool PIPE>
__global__ void __launch_bounds__(256) k_gains_lp(GainsArgs ga) {
    gains_lp_body<DT, KC, CB, PIPE>(ga, blockIdx.x);
}

// Batched: workgroups wg_pre[j] .. wg_pre[j+1] serve descriptor slot_inst[j]
// (all candidates, in the same geometry as a solo launch).
template <int DT, int KC, int CB, bool PIPE>
__global__ void __launch_bounds__(256)
kb_gains_lp(const InstDesc* __restrict__ descs, const int32_t* __restrict__ slot_inst,
            const int64_t* __restrict__ wg_pre, int32_t slots, int32_t t) {
    const int j = find_slot(wg_pre, slots, blockIdx.x);
    const InstDesc c = descs[slot_inst[j]];
    if (c.t0 + t >= c.k) return;
    gains_lp_body<DT, KC, CB, PIPE>(gains_args(c, nullptr, c.n_pad), int64_t(blockIdx.x) - wg_pre[j]);
}

template <int DT, int KC, int CB, bool PIPE>
static void launch_lp_v(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    using G = LpGeom<DT, KC, CB>;
    const int64_t tiles = (n_cand + G::CAND_TILE - 1) / G::CAND_TILE;
    InstDesc c;
    fill_desc(ds, 0, nullptr, nullptr, nullptr, &c);
    hipLaunchKernelGGL((k_gains_lp<DT, KC, CB, PIPE>), dim3(unsigned(tiles * ds->v_splits)), dim3(256), 0, s,
                       gains_args(c, cand, n_cand));
}

template <int DT, int KC, int CB, int VTS>
static void launch_lp_sp(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    using G = LpGeom<DT, KC, CB, VTS>;
    const int64_t tiles = (n_cand + G::CAND_TILE - 1) / G::CAND_TILE;
    InstDesc c;
    fill_desc(ds, 0, nullptr, nullptr, nullptr, &c);
    hipLaunchKernelGGL((k_gains_lp_sp<DT, KC, CB, VTS>), dim3(unsigned(tiles * ds->v_splits)), dim3(256), 0, s,
                       gains_args(c, cand, n_cand));
}

template <int DT, int KC, int CB>
static void launch_lp_pp(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    using G = LpGeom<DT, KC, CB>;
    const int64_t tiles = (n_cand + 2 * G::CAND_TILE - 1) / (2 * G::CAND_TILE);
    InstDesc c;
    fill_desc(ds, 0, nullptr, nullptr, nullptr, &c);
    hipLaunchKernelGGL((k_gains_lp_pp<DT, KC, CB>), dim3(unsigned(tiles * ds->v_splits)), dim3(512), 0, s,
                       gains_args(c, cand, n_cand));
}

// Variants: 4 waves with (32-row candidate blocks per wave, software-pipelined
// epilogue) 0 = (2, no), 1 = (4, no), 2 = (2, yes); 3 = ping-pong, 8 waves
// with pp_blocks(DT, KC) blocks each; 4 = interleaved test, 4 waves x 2 blocks,
// ring stages of wide_stage(DT, KC) points.
template <int DT, int KC>
static void launch_lp(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    switch (ds->variant) {
        case 1: launch_lp_v<DT, KC, 4, false>(ds, cand, n_cand, s); break;
        case 2: launch_lp_v<DT, KC, 2, true>(ds, cand, n_cand, s); break;
        case 3: launch_lp_pp<DT, KC, pp_blocks(DT, KC)>(ds, cand, n_cand, s); break;
        case 4: launch_lp_sp<DT, KC, 2, wide_stage(DT, KC)>(ds, cand, n_cand, s); break;
        default: launch_lp_v<DT, KC, 2, false>(ds, cand, n_cand, s); break;
    }
}

hipError_t launch_gains_lp(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    const int kc = ds->k_pad / (ds->dt == EBC_DT_FP8_E4M3 ? 64 : 16);
    switch (ds->dt) {
        case EBC_DT_BF16:
            switch (kc) {
                case 1: launch_lp<EBC_DT_BF16, 1>(ds, cand, n_cand, s); break;
                case 2: launch_lp<EBC_DT_BF16, 2>(ds, cand, n_cand, s); break;
                case 3: launch_lp<EBC_DT_BF16, 3>(ds, cand, n_cand, s); break;
                case 4: launch_lp<EBC_DT_BF16, 4>(ds, cand, n_cand, s); break;
                case 5: launch_lp<EBC_DT_BF16, 5>(ds, cand, n_cand, s); break;
                case 6: launch_lp<EBC_DT_BF16, 6>(ds, cand, n_cand, s); break;
                case 7: launch_lp<EBC_DT_BF16, 7>(ds, cand, n_cand, s); break;
                case 8: launch_lp<EBC_DT_BF16, 8>(ds, cand, n_cand, s); break;
                default: return hipErrorInvalidValue;
            }
            break;
        case EBC_DT_F16:
            switch (kc) {
                case 1: launch_lp<EBC_DT_F16, 1>(ds, cand, n_cand, s); break;
                case 2: launch_lp<EBC_DT_F16, 2>(ds, cand, n_cand, s); break;
                case 3: launch_lp<EBC_DT_F16, 3>(ds, cand, n_cand, s); break;
                case 4: launch_lp<EBC_DT_F16, 4>(ds, cand, n_cand, s); break;
                case 5: launch_lp<EBC_DT_F16, 5>(ds, cand, n_cand, s); break;
                case 6: launch_lp<EBC_DT_F16, 6>(ds, cand, n_cand, s); break;
                case 7: launch_lp<EBC_DT_F16, 7>(ds, cand, n_cand, s); break;
                case 8: launch_lp<EBC_DT_F16, 8>(ds, cand, n_cand, s); break;
                default: return hipErrorInvalidValue;
            }
            break;
        case EBC_DT_FP8_E4M3:
            switch (kc) {
                case 1: launch_lp<EBC_DT_FP8_E4M3, 1>(ds, cand, n_cand, s); break;
                case 2: launch_lp<EBC_DT_FP8_E4M3, 2>(ds, cand, n_cand, s); break;
                default: return hipErrorInvalidValue;
            }
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int DT, int KC>
static void launch_lp_b(int32_t variant, const InstDesc* descs, const int32_t* slot_inst, const int64_t* wg_pre,
                        int32_t slots, int64_t total_wgs, int32_t t, hipStream_t s) {
    const dim3 g = dim3(unsigned(total_wgs)), b = dim3(256);
    switch (variant) {
        case 1: hipLaunchKernelGGL((kb_gains_lp<DT, KC, 4, false>), g, b, 0, s, descs, slot_inst, wg_pre, slots, t); break;
        case 2: hipLaunchKernelGGL((kb_gains_lp<DT, KC, 2, true>), g, b, 0, s, descs, slot_inst, wg_pre, slots, t); break;
        case 3:
            hipLaunchKernelGGL((kb_gains_lp_pp<DT, KC, pp_blocks(DT, KC)>), g, dim3(512), 0, s, descs, slot_inst, wg_pre,
                               slots, t);
            break;
        case 4:
            hipLaunchKernelGGL((kb_gains_lp_sp<DT, KC, 2, wide_stage(DT, KC)>), g, b, 0, s, descs, slot_inst, wg_pre,
                               slots, t);
            break;
        default: hipLaunchKernelGGL((kb_gains_lp<DT, KC, 2, false>), g, b, 0, s, descs, slot_inst, wg_pre, slots, t); break;
    }
}

hipError_t launch_gains_lp_batched(int32_t dt, int32_t kc, int32_t variant, const InstDesc* descs,
                                   const int32_t* slot_inst, const int64_t* wg_pre, int32_t slots, int64_t total_wgs,
                                   int32_t t, hipStream_t s) {
#define EBC_LPB(DTV, K) \
    case K: launch_lp_b<DTV, K>(variant, descs, slot_inst, wg_pre, slots, total_wgs, t, s); break;
    switch (dt) {
        case EBC_DT_BF16:
            switch (kc) {
                EBC_LPB(EBC_DT_BF16, 1) EBC_LPB(EBC_DT_BF16, 2) EBC_LPB(EBC_DT_BF16, 3) EBC_LPB(EBC_DT_BF16, 4)
                EBC_LPB(EBC_DT_BF16, 5) EBC_LPB(EBC_DT_BF16, 6) EBC_LPB(EBC_DT_BF16, 7) EBC_LPB(EBC_DT_BF16, 8)
                default: return hipErrorInvalidValue;
            }
            break;
        case EBC_DT_F16:
            switch (kc) {
                EBC_LPB(EBC_DT_F16, 1) EBC_LPB(EBC_DT_F16, 2) EBC_LPB(EBC_DT_F16, 3) EBC_LPB(EBC_DT_F16, 4)
                EBC_LPB(EBC_DT_F16, 5) EBC_LPB(EBC_DT_F16, 6) EBC_LPB(EBC_DT_F16, 7) EBC_LPB(EBC_DT_F16, 8)
                default: return hipErrorInvalidValue;
            }
            break;
        case EBC_DT_FP8_E4M3:
            switch (kc) {
                EBC_LPB(EBC_DT_FP8_E4M3, 1) EBC_LPB(EBC_DT_FP8_E4M3, 2)
                default: return hipErrorInvalidValue;
            }
            break;
        default: return hipErrorInvalidValue;
    }
#undef EBC_LPB
    return hipGetLastError();
}

}  // namespace ebc
