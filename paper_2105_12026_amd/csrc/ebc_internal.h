// Internal declarations shared by the host side of libebc.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ebc.h"

namespace ebc {

constexpr int kWindowCap = 1024;   // candidates that may enter the re-score window list
constexpr int kWindowMax = 256;    // candidates actually re-scored in float64 per step
constexpr int kRowAlign = 256;     // rows of every per-point array are padded to this (= kBlock)
constexpr int kBlock = 256;        // threads of the per-point kernels
constexpr int kGainsCandTile = 128;  // candidates per gains workgroup (4 waves x 32)
constexpr int kGainsVTile = 64;      // ground points per LDS stage of the gains kernel
// Rows longer than this (padded length) take the long-row kernels, which
// loop over the dimension instead of holding whole rows in registers.
constexpr int kNarrowMaxK = 128;
__host__ __device__ inline bool wide_rows(int32_t k_pad) { return k_pad > kNarrowMaxK; }
// Long-row gains: waves of a workgroup that split one candidate block's dot
// products over K (1: four candidate blocks, no split; 4: one block, K in
// quarters). Small ground sets split K to give the chip enough workgroups.
inline int32_t wide_ksplit(int64_t n_pad) { return n_pad >= 16384 ? 1 : 4; }

// Error codes the device writes into DevState::error (first one wins).
constexpr int kDevErrIndex = EBC_E_INDEX;
constexpr int kDevErrNonFinite = EBC_E_NONFINITE;

// Small per-dataset device state of the greedy loop.
struct DevState {
    int error;           // first device-detected ebc_status, 0 if none
    int window_count;    // candidates in wfinal this step
    int window_max;      // largest window seen in this greedy run
    int window_overflow; // steps whose window list overflowed kWindowCap
    int cstar;           // index picked by the last step
    int pad0;
    double gstar;        // float64 gain of the last pick (unnormalised sum)
    double l0;           // L({e0}) = |V|^-1 sum ||v||^2
    double tau;          // relative window half-width for the gains dtype
    double tau_abs;      // absolute window half-width, in units of nmax
    double nmax;         // max_v ||v||^2
    int32_t gexp;        // 2^gexp >= m_v / 2 for every point and every m loaded since the dataset's
                         // creation (raised, never lowered): the reduced-precision gains scale
                         // their clamped terms by 2^-gexp into [0, 1]
    int32_t pad1;
};

struct WindowEntry {
    double g;
    int idx;
    int pad;
};

// Pointers into the caller's workspace (see layout()).
struct Buffers {
    float* xq;          // distance-dtype copy of x, columns d.. are 0: float32 rows up to 128 row-major
                        // [n_pad, k_pad]; longer float32 rows and reduced precision: 64-row tiles,
                        // 16-byte units unit-major inside a tile
    int* scale;         // [n_pad] E8M0 row scales (FP8 only, else null)
    double* n64;        // [n_pad] ||v||^2 in float64 (0 for pad rows)
    double* m0;         // [n_pad] d(v, e0) in float64, the minima of S = {} (= n64 for e0 = 0)
    double* mu;         // [k_pad] column means; long rows only (the distance-dtype copy then
                        // holds x - mu, and hn is the norm of that centred copy), else null
    double* m64;        // [n_pad] running minima m_v (float64 master copy)
    float* hn;          // [n_pad] ||v||^2 / 2 rounded to float32
    float* ha;          // [n_pad] (m_v - ||v||^2) / 2 in float32
    float* hm;          // [n_pad] m_v / 2 in float32 (0 for pad rows)
    uint8_t* selected;  // [n_pad] 1 if picked by greedy
    double* part;       // [v_splits, n_pad] per-chunk gain sums
    double* gsum;       // [n_pad] gain sums (unnormalised) of the current step
    double* bmax;       // [nb] per-block maxima of gsum
    int32_t* barg;      // [nb] lowest index attaining bmax in its block
    int32_t* bcnt;      // [nb] window entries found in each block
    WindowEntry* wstage;// [n_pad] window entries, block b's at [b*kBlock ..)
    WindowEntry* wfinal;// [kWindowMax] candidates re-scored in float64 this step
    double* rpart;      // [nb, kWindowMax] float64 re-score partial sums ([4 nb, ...] for long rows)
    double* fpart;      // [nb] partial sums of m_v or norms
    DevState* state;
    // Grouped order of the reduced-precision gains (rows up to 128 values):
    // the ground set sorted by nearest pivot, so that a 32 x 32 tile pairs
    // nearby candidates with nearby points and most tiles clamp to their
    // lower bound as a whole (the gains kernel then skips their epilogue).
    // Null for every other dataset.
    int32_t* perm;      // [n_pad] slot -> row (identity on padding rows)
    int32_t* inv;       // [n_pad] row -> slot
    void* xqp;          // the distance-dtype copy in slot order (same tiled layout as xq)
    float* hnp;         // [n_pad] hn in slot order
    float* hap;         // [n_pad] ha in slot order (kept in step with ha)
    float* hmp;         // [n_pad] hm in slot order (kept in step with hm)
    int* scp;           // [n_pad] FP8 row scales in slot order (FP8 only)
    int32_t* gbucket;   // [n_pad] nearest pivot of each row (set-up only)
    int32_t* gcount;    // [nb, groups] per-block bucket counts, then slot offsets (set-up only)
};

// Everything a kernel of one greedy step needs about one dataset. Solo
// launches pass it by value; batched launches read it from a device table
// and map their blocks onto the instances, so both run the same code on the
// same per-instance geometry (bitwise-identical results).
struct InstDesc {
    Buffers b;
    const float* x;
    int64_t n, n_pad;
    int32_t d, k_pad, v_splits, nb;  // nb = n_pad / kBlock
    int32_t k;                       // greedy steps of this instance
    int32_t t0;                      // steps already done: a batched tick t runs step t0 + t
    int32_t dt, variant;
    int32_t metric;                  // dissimilarity: 0 squared Euclidean, 1 L1
    int32_t pad_m;
    int64_t chunk;                   // ground-set chunk of the gains kernel
    int32_t* sel;
    double* f;
    double* gain;
};

// Arguments of one gains-kernel launch for one instance.
struct GainsArgs {
    const void* xq;
    const float* hn;
    const float* ha;
    const float* hm;
    const int* scale;
    const int32_t* cand;
    const int32_t* perm;  // grouped order: slot -> row (null: slot = row)
    const int32_t* inv;   // grouped order: row -> slot
    int64_t n_cand, n_pad;
    int32_t v_splits, pad0;
    int64_t chunk;
    double* part;
    int64_t part_stride;
    int* err;
    const int32_t* gexp;  // DevState::gexp of the instance
};

// Block -> instance map of a batched launch: instance i owns blocks
// [pre[i], pre[i+1]) (pre[0] = 0); `inst` maps slot i to a descriptor.
__device__ inline int find_slot(const int64_t* __restrict__ pre, int count, int64_t blk) {
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= blk)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

struct Layout {
    size_t off_xq, off_scale, off_mu, off_n64, off_m0, off_m64, off_hn, off_ha, off_hm, off_sel, off_part, off_gsum, off_bmax,
        off_barg, off_bcnt, off_wstage, off_wfinal, off_rpart, off_fpart, off_state, off_perm, off_inv, off_xqp,
        off_hnp, off_hap, off_hmp, off_scp, off_gbucket, off_gcount, total;
};

// Datasets whose reduced-precision gains run in grouped order (see Buffers::perm).
__host__ __device__ inline bool grouped(int32_t k_pad, ebc_dtype dt) { return dt != EBC_DT_F32 && !wide_rows(k_pad); }
// Number of pivots (buckets) of the grouped order: one per 256 points, 1 .. 256.
__host__ __device__ inline int32_t group_count(int64_t n) {
    const int64_t g = n / 256;
    return int32_t(g < 1 ? 1 : (g > 256 ? 256 : g));
}

int64_t pad_rows(int64_t n);
int32_t k_pad_for(int32_t d, ebc_dtype dt);
int32_t v_splits_for(int64_t n_pad, int32_t k_pad, ebc_dtype dt);
Layout layout(int64_t n, int32_t d, ebc_dtype dt);

}  // namespace ebc

namespace ebc {
struct Profiler;
}

struct ebc_dataset {
    const float* x;
    int64_t n;
    int64_t n_pad;
    int32_t d;
    int32_t k_pad;
    int32_t v_splits;
    ebc_dtype dt;
    int32_t metric;  // dissimilarity: 0 squared Euclidean, 1 L1 (EBC_FLAG_L1)
    ebc::Buffers b;
    double l0_host;
    ebc_greedy_stats stats;
    ebc::Profiler* prof;  // non-null while profiling is on
    int32_t variant;      // tile variant of the gains kernel (0 = default)
    // captured greedy run (graph mode): replayed while the key matches
    int32_t graph_on;
    hipStream_t cap_stream;  // private stream used only to record the graph
    hipGraphExec_t gexec;
    int32_t g_k, g_variant;
    const void *g_sel, *g_f, *g_gain;
};

namespace ebc {

// Device table block of a batched launch set: descriptors and block maps for
// up to `slots` instances, contiguous, filled on the host in pinned memory
// (double-buffered, each buffer guarded by an event) and copied in one
// transfer per use.
struct TableLayout {
    size_t desc, row_pre, slot_inst, wg_pre, total;
};
inline TableLayout table_layout(int32_t slots) {
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    TableLayout L{};
    size_t o = 0;
    L.desc = o;
    o = al(o + size_t(slots) * sizeof(InstDesc));
    L.row_pre = o;
    o = al(o + size_t(slots + 1) * sizeof(int64_t));
    L.slot_inst = o;
    o = al(o + size_t(slots) * sizeof(int32_t));
    L.wg_pre = o;
    o = al(o + size_t(2 * slots) * sizeof(int64_t));
    L.total = o;
    return L;
}

struct PinnedTables {
    char* host[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    int next = 0;
    size_t bytes = 0;
    hipError_t init(size_t b) {
        bytes = b;
        for (int i = 0; i < 2; ++i) {
            hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&host[i]), b, hipHostMallocDefault);
            if (e != hipSuccess) return e;
            if ((e = hipEventCreateWithFlags(&done[i], hipEventDisableTiming)) != hipSuccess) return e;
        }
        return hipSuccess;
    }
    // a staging buffer whose previous copy has finished
    char* acquire(hipError_t* e) {
        *e = hipEventSynchronize(done[next]);
        return host[next];
    }
    // copy the acquired buffer to `dev` on `s` and rotate
    hipError_t submit(void* dev, size_t n, hipStream_t s) {
        hipError_t e = hipMemcpyAsync(dev, host[next], n, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventRecord(done[next], s);
        next ^= 1;
        return e;
    }
    ~PinnedTables() {
        for (int i = 0; i < 2; ++i) {
            if (done[i]) {
                (void)hipEventSynchronize(done[i]);
                (void)hipEventDestroy(done[i]);
            }
            if (host[i]) (void)hipHostFree(host[i]);
        }
    }
};

// Host helpers shared by the solo and batched paths.
int64_t gains_chunk(const ebc_dataset* ds);
int64_t gains_cand_tile(const ebc_dataset* ds);
int32_t gains_bucket(const ebc_dataset* ds);  // datasets with equal keys share a batched gains launch
void fill_desc(const ebc_dataset* ds, int32_t k, int32_t* sel, double* f, double* gain, InstDesc* out);

// Gains-kernel arguments of one instance (candidates: a list, or all rows).
__host__ __device__ inline GainsArgs gains_args(const InstDesc& d, const int32_t* cand, int64_t n_cand) {
    GainsArgs a;
    const bool g = d.b.perm != nullptr;  // grouped order: the slot-order copies
    a.xq = g ? d.b.xqp : d.b.xq;
    a.hn = g ? d.b.hnp : d.b.hn;
    a.ha = g ? d.b.hap : d.b.ha;
    a.hm = g ? d.b.hmp : d.b.hm;
    a.scale = g ? d.b.scp : d.b.scale;
    a.perm = d.b.perm;
    a.inv = d.b.inv;
    a.cand = cand;
    a.n_cand = n_cand;
    a.n_pad = d.n_pad;
    a.v_splits = d.v_splits;
    a.pad0 = 0;
    a.chunk = d.chunk;
    a.part = d.b.part;
    a.part_stride = d.n_pad;
    a.err = &d.b.state->error;
    a.gexp = &d.b.state->gexp;
    return a;
}

// Batched launches over a device table of descriptors (see ebc_batch).
hipError_t launch_gains_f32_batched(int32_t k_pad, bool trim, const InstDesc* descs, const int32_t* slot_inst,
                                    const int64_t* wg_pre, int32_t slots, int64_t total_wgs, int32_t t,
                                    hipStream_t s);
hipError_t launch_gains_lp_batched(int32_t dt, int32_t kc, int32_t variant, const InstDesc* descs,
                                   const int32_t* slot_inst, const int64_t* wg_pre, int32_t slots, int64_t total_wgs,
                                   int32_t t, hipStream_t s);
hipError_t launch_gains_wide_batched(int32_t dt, int32_t ksplit, const InstDesc* descs, const int32_t* slot_inst,
                                     const int64_t* wg_pre, int32_t slots, int64_t total_wgs, int32_t t,
                                     hipStream_t s);
hipError_t launch_gains_batched(int32_t bucket, const InstDesc* descs, const int32_t* slot_inst,
                                const int64_t* wg_pre, int32_t slots, int64_t total_wgs, int32_t t, hipStream_t s);
// 32-row candidate blocks per wave in the ping-pong gains variant (3):
// two where the registers allow, one for long rows.
constexpr int pp_blocks(int dt, int kc) {
    return dt == EBC_DT_FP8_E4M3 ? (kc <= 1 ? 2 : 1) : (kc <= 6 ? 2 : 1);
}
// Tile variant recorded by the autotuner for this dataset's key, or -1.
int32_t tuned_variant(const ebc_dataset* ds);
// long_rows: some instance has rows longer than kNarrowMaxK (their re-score
// and update run in the long-row kernels)
hipError_t launch_step_batched(const InstDesc* descs, const int64_t* row_pre, int32_t count, int64_t total_rows,
                               int32_t t, bool long_rows, hipStream_t s);
hipError_t launch_reset_batched(const InstDesc* descs, const int64_t* row_pre, int32_t count, int64_t total_rows,
                                hipStream_t s);

// Launchers (each defined next to its kernels). All return hipGetLastError().
hipError_t launch_prep(const ebc_dataset* ds, hipStream_t s);
hipError_t launch_reset_state(const ebc_dataset* ds, hipStream_t s);
hipError_t launch_set_e0(const ebc_dataset* ds, const float* e0, hipStream_t s);
hipError_t launch_load_m(const ebc_dataset* ds, const double* m, hipStream_t s);
hipError_t launch_gains_f32(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s);
hipError_t launch_gains_lp(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s);
hipError_t launch_gains_wide(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s);
hipError_t launch_gains_l1(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s);
hipError_t launch_gains(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s);
int elem_bytes(ebc_dtype dt);

// Byte offset of byte `byte` of row r in a tiled reduced-precision array whose
// rows are `row_units` 16-byte units long (64-row tiles, unit-major).
__host__ __device__ inline int64_t tiled_offset(int64_t r, int byte, int row_units) {
    return ((r / 64 * row_units + byte / 16) * 64 + r % 64) * 16 + byte % 16;
}
// Half-widths of the float64 re-score window per distance dtype: a candidate
// whose gain sum is within tau * |best| + tau_abs * max_v ||v||^2 of the best
// is re-scored in float64. The absolute part keeps every candidate of a
// zero-gain step (all points already covered) inside the window.
__host__ __device__ inline double window_tau(ebc_dtype dt) {
    switch (dt) {
        case EBC_DT_F32: return 1e-4;
        case EBC_DT_F16: return 2e-3;
        case EBC_DT_BF16: return 1e-2;
        case EBC_DT_FP8_E4M3: return 4e-2;
    }
    return 1e-2;
}
__host__ __device__ inline double window_tau_abs(ebc_dtype dt) { return dt == EBC_DT_F32 ? 1e-4 : 1e-2; }
hipError_t launch_gains_out(const ebc_dataset* ds, int64_t n_cand, double* out, hipStream_t s);
hipError_t launch_greedy_step(const ebc_dataset* ds, int32_t t, int32_t* sel_out, double* f_out,
                              double* gain_out, hipStream_t s, hipEvent_t ev_gains_done);
// device scratch of one multi-set evaluation of l sets over n ground points
size_t eval_sets_scratch_bytes(int64_t n, int64_t l);
// `scratch`: at least eval_sets_scratch_bytes(ds->n, l) bytes, 256-byte aligned
hipError_t launch_eval_sets(const ebc_dataset* ds, const int64_t* offsets, const int32_t* idx,
                            int64_t l, double* f_out, bool in_dtype, void* scratch, hipStream_t s);

}  // namespace ebc
