// Internal declarations shared by the host side of libebc.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ebc.h"

namespace ebc {

constexpr int kWindowCap = 1024;   // candidates that may enter the re-score window list
constexpr int kWindowMax = 64;     // candidates actually re-scored in float64 per step
constexpr int kRowAlign = 256;     // rows of every per-point array are padded to this (= kBlock)
constexpr int kBlock = 256;        // threads of the per-point kernels
constexpr int kGainsCandTile = 128;  // candidates per gains workgroup (4 waves x 32)
constexpr int kGainsVTile = 64;      // ground points per LDS stage of the gains kernel

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
};

struct WindowEntry {
    double g;
    int idx;
    int pad;
};

// Pointers into the caller's workspace (see layout()).
struct Buffers {
    float* xq;          // distance-dtype copy of x, columns d.. are 0: float32 row-major [n_pad, k_pad];
                        // reduced precision: 64-row tiles, 16-byte units unit-major inside a tile
    uint16_t* aug_c;    // [n_pad, 16] bf16 affine chunk, candidate role, row-major (reduced precision only)
    uint16_t* aug_v;    // [n_pad, 16] bf16 affine chunk, ground-point role, tiled like xq (reduced precision only)
    int* scale;         // [n_pad] E8M0 row scales (FP8 only, else null)
    double* n64;        // [n_pad] ||v||^2 in float64 (0 for pad rows)
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
    double* rpart;      // [nb, kWindowMax] float64 re-score partial sums
    double* fpart;      // [nb] partial sums of m_v or norms
    DevState* state;
};

struct Layout {
    size_t off_xq, off_aug_c, off_aug_v, off_scale, off_n64, off_m64, off_hn, off_ha, off_hm, off_sel, off_part, off_gsum, off_bmax,
        off_barg, off_bcnt, off_wstage, off_wfinal, off_rpart, off_fpart, off_state, total;
};

int64_t pad_rows(int64_t n);
int32_t k_pad_for(int32_t d, ebc_dtype dt);
int32_t v_splits_for(int64_t n_pad);
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

// Launchers (each defined next to its kernels). All return hipGetLastError().
hipError_t launch_prep(const ebc_dataset* ds, hipStream_t s);
hipError_t launch_reset_state(const ebc_dataset* ds, hipStream_t s);
hipError_t launch_load_m(const ebc_dataset* ds, const double* m, hipStream_t s);
hipError_t launch_gains_f32(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s);
hipError_t launch_gains_lp(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s);
hipError_t launch_gains(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s);
int elem_bytes(ebc_dtype dt);

// Byte offset of byte `byte` of row r in a tiled reduced-precision array whose
// rows are `row_units` 16-byte units long (64-row tiles, unit-major).
__host__ __device__ inline int64_t tiled_offset(int64_t r, int byte, int row_units) {
    return ((r / 64 * row_units + byte / 16) * 64 + r % 64) * 16 + byte % 16;
}
double window_tau(ebc_dtype dt);
double window_tau_abs(ebc_dtype dt);
hipError_t launch_gains_out(const ebc_dataset* ds, int64_t n_cand, double* out, hipStream_t s);
hipError_t launch_greedy_step(const ebc_dataset* ds, int32_t t, int32_t* sel_out, double* f_out,
                              double* gain_out, hipStream_t s, hipEvent_t ev_gains_done);
hipError_t launch_eval_sets(const ebc_dataset* ds, const int64_t* offsets, const int32_t* idx,
                            int64_t l, double* f_out, hipStream_t s);

}  // namespace ebc
