// C ABI of libebc.so (declared in include/ebc.h): host-side validation,
// workspace carving and kernel sequencing. No entry point blocks except
// ebc_sync_status, and no C++ exception leaves this file.
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "ebc_internal.h"

using namespace ebc;

namespace ebc {
// Host-side event triples (step start, gains done, step end) of timed steps.
struct Profiler {
    std::vector<hipEvent_t> ev;  // 3 per step, reused across reads
    int used = 0;                // triples recorded since the last read
    double gains_ms = 0.0, select_ms = 0.0;
    int32_t launches = 0, steps = 0;
    ~Profiler() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    hipError_t next(hipEvent_t* out3) {
        while (int(ev.size()) < 3 * (used + 1)) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            ev.push_back(e);
        }
        for (int i = 0; i < 3; ++i) out3[i] = ev[3 * used + i];
        ++used;
        return hipSuccess;
    }
    hipError_t collect() {
        for (int i = 0; i < used; ++i) {
            hipError_t r = hipEventSynchronize(ev[3 * i + 2]);
            if (r != hipSuccess) return r;
            float a = 0.f, b = 0.f;
            if ((r = hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1])) != hipSuccess) return r;
            if ((r = hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2])) != hipSuccess) return r;
            gains_ms += a;
            select_ms += b;
            ++launches;
            ++steps;
        }
        used = 0;
        return hipSuccess;
    }
};
}  // namespace ebc

namespace {

void drop_graph(ebc_dataset* ds);

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

ebc_status from_hip(hipError_t e) { return e == hipSuccess ? EBC_OK : EBC_E_DEVICE; }

// sets per multi-set evaluation call (set indices fit the kernels' int32 unit counts)
constexpr int64_t kMaxSets = (int64_t(1) << 31) - 1;

bool valid_dtype(ebc_dtype dt) {
    return dt == EBC_DT_F32 || dt == EBC_DT_F16 || dt == EBC_DT_BF16 || dt == EBC_DT_FP8_E4M3;
}

}  // namespace

extern "C" {

const char* ebc_status_string(ebc_status st) {
    switch (st) {
        case EBC_OK: return "ok";
        case EBC_E_INVALID_ARG: return "invalid argument";
        case EBC_E_INDEX: return "set index out of range or offsets not non-decreasing";
        case EBC_E_NONFINITE: return "non-finite value in the input points";
        case EBC_E_RANGE: return "value out of range of the distance dtype";
        case EBC_E_NOMEM: return "out of memory (host allocation, no room in the arena, or beyond a fixed scratch)";
        case EBC_E_DEVICE: return "HIP runtime error";
        case EBC_E_UNSUPPORTED: return "unsupported by this build";
    }
    return "unknown status";
}

size_t ebc_dataset_bytes(int64_t n, int32_t d, ebc_dtype dt) {
    if (n < 1 || n >= (int64_t(1) << 31) - kRowAlign || d < 1 || d > EBC_MAX_DIM || !valid_dtype(dt)) return 0;
    return layout(n, d, dt).total;
}

ebc_status ebc_dataset_create(const float* x, int64_t n, int32_t d, ebc_dtype dt, uint32_t flags,
                              void* workspace, size_t workspace_bytes, void* stream, ebc_dataset** out) {
    if (!out) return EBC_E_INVALID_ARG;
    *out = nullptr;
    if (!x || !workspace || (flags & ~uint32_t(EBC_FLAG_L1)) != 0) return EBC_E_INVALID_ARG;
    if (!valid_dtype(dt)) return EBC_E_INVALID_ARG;
    if (n < 1 || n >= (int64_t(1) << 31) - kRowAlign || d < 1) return EBC_E_INVALID_ARG;
    if (d > EBC_MAX_DIM) return EBC_E_UNSUPPORTED;
    if ((flags & EBC_FLAG_L1) && dt != EBC_DT_F32) return EBC_E_UNSUPPORTED;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return EBC_E_INVALID_ARG;
    const Layout L = layout(n, d, dt);
    if (workspace_bytes < L.total) return EBC_E_INVALID_ARG;

    ebc_dataset* ds = new (std::nothrow) ebc_dataset;
    if (!ds) return EBC_E_NOMEM;
    memset(ds, 0, sizeof(*ds));
    ds->x = x;
    ds->n = n;
    ds->n_pad = pad_rows(n);
    ds->d = d;
    ds->k_pad = k_pad_for(d, dt);
    ds->dt = dt;
    ds->v_splits = v_splits_for(ds->n_pad, ds->k_pad, dt);
    ds->metric = (flags & EBC_FLAG_L1) ? 1 : 0;
    // reduced precision: the interleaved-test tile variant (bitwise the same
    // gains as every other variant, the fastest on the measured shapes)
    ds->variant = dt == EBC_DT_F32 ? 0 : 4;
    char* w = static_cast<char*>(workspace);
    Buffers& b = ds->b;
    b.xq = reinterpret_cast<float*>(w + L.off_xq);
    b.scale = dt == EBC_DT_FP8_E4M3 ? reinterpret_cast<int*>(w + L.off_scale) : nullptr;
    b.mu = wide_rows(ds->k_pad) ? reinterpret_cast<double*>(w + L.off_mu) : nullptr;
    b.n64 = reinterpret_cast<double*>(w + L.off_n64);
    b.m0 = reinterpret_cast<double*>(w + L.off_m0);
    b.m64 = reinterpret_cast<double*>(w + L.off_m64);
    b.hn = reinterpret_cast<float*>(w + L.off_hn);
    b.ha = reinterpret_cast<float*>(w + L.off_ha);
    b.hm = reinterpret_cast<float*>(w + L.off_hm);
    b.selected = reinterpret_cast<uint8_t*>(w + L.off_sel);
    b.part = reinterpret_cast<double*>(w + L.off_part);
    b.gsum = reinterpret_cast<double*>(w + L.off_gsum);
    b.bmax = reinterpret_cast<double*>(w + L.off_bmax);
    b.barg = reinterpret_cast<int32_t*>(w + L.off_barg);
    b.bcnt = reinterpret_cast<int32_t*>(w + L.off_bcnt);
    b.wstage = reinterpret_cast<WindowEntry*>(w + L.off_wstage);
    b.wfinal = reinterpret_cast<WindowEntry*>(w + L.off_wfinal);
    b.rpart = reinterpret_cast<double*>(w + L.off_rpart);
    b.fpart = reinterpret_cast<double*>(w + L.off_fpart);
    b.state = reinterpret_cast<DevState*>(w + L.off_state);
    if (grouped(ds->k_pad, dt)) {
        b.perm = reinterpret_cast<int32_t*>(w + L.off_perm);
        b.inv = reinterpret_cast<int32_t*>(w + L.off_inv);
        b.xqp = w + L.off_xqp;
        b.hnp = reinterpret_cast<float*>(w + L.off_hnp);
        b.hap = reinterpret_cast<float*>(w + L.off_hap);
        b.hmp = reinterpret_cast<float*>(w + L.off_hmp);
        b.scp = dt == EBC_DT_FP8_E4M3 ? reinterpret_cast<int*>(w + L.off_scp) : nullptr;
        b.gbucket = reinterpret_cast<int32_t*>(w + L.off_gbucket);
        b.gcount = reinterpret_cast<int32_t*>(w + L.off_gcount);
    }

    const hipError_t e = launch_prep(ds, as_stream(stream));
    if (e != hipSuccess) {
        delete ds;
        return EBC_E_DEVICE;
    }
    *out = ds;
    return EBC_OK;
}

ebc_status ebc_dataset_destroy(ebc_dataset* ds) {
    if (!ds) return EBC_E_INVALID_ARG;
    drop_graph(ds);
    if (ds->cap_stream) (void)hipStreamDestroy(ds->cap_stream);
    delete ds->prof;
    delete ds;
    return EBC_OK;
}

ebc_status ebc_dataset_set_e0(ebc_dataset* ds, const float* e0, void* stream) {
    if (!ds) return EBC_E_INVALID_ARG;
    return from_hip(launch_set_e0(ds, e0, as_stream(stream)));
}

ebc_status ebc_set_gains_variant(ebc_dataset* ds, int32_t variant) {
    if (!ds || variant < 0 || variant >= ebc_gains_variant_count(ds->dt)) return EBC_E_INVALID_ARG;
    ds->variant = variant;
    return EBC_OK;
}

int32_t ebc_gains_variant_count(ebc_dtype dt) { return dt == EBC_DT_F32 ? 1 : 5; }

ebc_status ebc_profile_enable(ebc_dataset* ds, int32_t on) {
    if (!ds) return EBC_E_INVALID_ARG;
    if (on && !ds->prof) {
        ds->prof = new (std::nothrow) Profiler;
        if (!ds->prof) return EBC_E_NOMEM;
    } else if (!on && ds->prof) {
        delete ds->prof;
        ds->prof = nullptr;
    }
    return EBC_OK;
}

ebc_status ebc_profile_read(ebc_dataset* ds, ebc_profile* out, int32_t reset) {
    if (!ds || !out) return EBC_E_INVALID_ARG;
    if (!ds->prof) return EBC_E_INVALID_ARG;
    if (ds->prof->collect() != hipSuccess) return EBC_E_DEVICE;
    out->gains_ms = ds->prof->gains_ms;
    out->select_ms = ds->prof->select_ms;
    out->gains_launches = ds->prof->launches;
    out->steps = ds->prof->steps;
    if (reset) {
        ds->prof->gains_ms = ds->prof->select_ms = 0.0;
        ds->prof->launches = ds->prof->steps = 0;
    }
    return EBC_OK;
}

ebc_status ebc_dataset_get_info(ebc_dataset* ds, ebc_dataset_info* info) {
    if (!ds || !info) return EBC_E_INVALID_ARG;
    info->n = ds->n;
    info->n_pad = ds->n_pad;
    info->d = ds->d;
    info->k_pad = ds->k_pad;
    info->v_splits = ds->v_splits;
    info->cand_tile = int32_t(gains_cand_tile(ds));
    info->window_cap = kWindowMax;
    info->dtype = int32_t(ds->dt);
    info->flags = ds->metric == 1 ? EBC_FLAG_L1 : 0u;
    info->reserved = 0;
    info->l0 = ds->l0_host;
    return EBC_OK;
}

size_t ebc_eval_sets_bytes(int64_t n, int64_t l) {
    if (n < 1 || n >= (int64_t(1) << 31) - kRowAlign || l < 0 || l > kMaxSets) return 0;
    return eval_sets_scratch_bytes(n, l);
}

static ebc_status eval_sets_impl(ebc_dataset* ds, const int64_t* offsets, const int32_t* idx, int64_t l,
                                 double* f_out, bool in_dtype, void* scratch, size_t scratch_bytes, void* stream) {
    if (!ds || l < 0 || l > kMaxSets) return EBC_E_INVALID_ARG;
    if (l == 0) return EBC_OK;
    if (!offsets || !f_out || !idx || !scratch) return EBC_E_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(scratch) % 256 != 0) return EBC_E_INVALID_ARG;
    if (scratch_bytes < eval_sets_scratch_bytes(ds->n, l)) return EBC_E_INVALID_ARG;
    return from_hip(launch_eval_sets(ds, offsets, idx, l, f_out, in_dtype, scratch, as_stream(stream)));
}

ebc_status ebc_eval_sets(ebc_dataset* ds, const int64_t* offsets, const int32_t* idx, int64_t l, double* f_out,
                         void* scratch, size_t scratch_bytes, void* stream) {
    return eval_sets_impl(ds, offsets, idx, l, f_out, false, scratch, scratch_bytes, stream);
}

ebc_status ebc_eval_sets_in_dtype(ebc_dataset* ds, const int64_t* offsets, const int32_t* idx, int64_t l,
                                  double* f_out, void* scratch, size_t scratch_bytes, void* stream) {
    return eval_sets_impl(ds, offsets, idx, l, f_out, true, scratch, scratch_bytes, stream);
}

ebc_status ebc_marginal_gains(ebc_dataset* ds, const double* m, const int32_t* cand, int64_t n_cand,
                              double* gains_out, void* stream) {
    if (!ds || n_cand < 0) return EBC_E_INVALID_ARG;
    if (!cand && n_cand != ds->n) return EBC_E_INVALID_ARG;
    if (n_cand == 0) return EBC_OK;
    if (!gains_out) return EBC_E_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    hipError_t e = hipSuccess;
    if (m) e = launch_load_m(ds, m, s);
    // The per-chunk sums hold at most n_pad candidates per pass.
    for (int64_t p0 = 0; p0 < n_cand && e == hipSuccess; p0 += ds->n_pad) {
        const int64_t cnt = (n_cand - p0) < ds->n_pad ? (n_cand - p0) : ds->n_pad;
        const int32_t* c = cand ? cand + p0 : nullptr;
        e = launch_gains(ds, c, cnt, s);
        if (e == hipSuccess) e = launch_gains_out(ds, cnt, gains_out + p0, s);
    }
    return from_hip(e);
}

namespace {

void drop_graph(ebc_dataset* ds) {
    if (ds->gexec) (void)hipGraphExecDestroy(ds->gexec);
    ds->gexec = nullptr;
}

// Record reset + k greedy steps into a graph on the dataset's private stream
// (recording executes nothing), instantiate it, and keep it for replays with
// the same k, outputs and gains variant.
hipError_t capture_greedy(ebc_dataset* ds, int32_t k, int32_t* sel_out, double* f_out, double* gain_out) {
    drop_graph(ds);
    hipError_t e = hipSuccess;
    if (!ds->cap_stream && (e = hipStreamCreateWithFlags(&ds->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return e;
    if ((e = hipStreamBeginCapture(ds->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
    hipError_t le = launch_reset_state(ds, ds->cap_stream);
    for (int32_t t = 0; t < k && le == hipSuccess; ++t)
        le = launch_greedy_step(ds, t, sel_out, f_out, gain_out, ds->cap_stream, nullptr);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(ds->cap_stream, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&ds->gexec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        ds->gexec = nullptr;
        return e;
    }
    ds->g_k = k;
    ds->g_variant = ds->variant;
    ds->g_sel = sel_out;
    ds->g_f = f_out;
    ds->g_gain = gain_out;
    return hipSuccess;
}

}  // namespace

ebc_status ebc_set_greedy_graph(ebc_dataset* ds, int32_t on) {
    if (!ds) return EBC_E_INVALID_ARG;
    ds->graph_on = on ? 1 : 0;
    if (!on) drop_graph(ds);
    return EBC_OK;
}

ebc_status ebc_greedy(ebc_dataset* ds, int32_t k, int32_t* sel_out, double* f_out, double* gain_out,
                      void* stream) {
    if (!ds || k < 0 || int64_t(k) > ds->n) return EBC_E_INVALID_ARG;
    if (k == 0) return EBC_OK;
    if (!sel_out || !f_out) return EBC_E_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    ds->stats.steps = k;
    if (ds->graph_on && !ds->prof) {
        hipError_t e = hipSuccess;
        if (!(ds->gexec && ds->g_k == k && ds->g_variant == ds->variant && ds->g_sel == sel_out &&
              ds->g_f == f_out && ds->g_gain == gain_out))
            e = capture_greedy(ds, k, sel_out, f_out, gain_out);
        if (e == hipSuccess) e = hipGraphLaunch(ds->gexec, s);
        return from_hip(e);
    }
    hipError_t e = launch_reset_state(ds, s);
    for (int32_t t = 0; t < k && e == hipSuccess; ++t) {
        hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
        if (ds->prof && (e = ds->prof->next(ev)) != hipSuccess) break;
        if (ev[0] && (e = hipEventRecord(ev[0], s)) != hipSuccess) break;
        e = launch_greedy_step(ds, t, sel_out, f_out, gain_out, s, ev[1]);
        if (e == hipSuccess && ev[2]) e = hipEventRecord(ev[2], s);
    }
    ds->stats.steps = k;
    return from_hip(e);
}

ebc_status ebc_sync_status(ebc_dataset* ds, void* stream, ebc_greedy_stats* stats) {
    if (!ds) return EBC_E_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    if (hipStreamSynchronize(s) != hipSuccess) return EBC_E_DEVICE;
    DevState st;
    if (hipMemcpy(&st, ds->b.state, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return EBC_E_DEVICE;
    ds->l0_host = st.l0;
    ds->stats.window_max = st.window_max;
    ds->stats.window_overflow = st.window_overflow;
    if (stats) *stats = ds->stats;
    if (st.error != 0) {
        const int zero = 0;
        if (hipMemcpy(&ds->b.state->error, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
            return EBC_E_DEVICE;
        return ebc_status(st.error);
    }
    return EBC_OK;
}

}  // extern "C"
