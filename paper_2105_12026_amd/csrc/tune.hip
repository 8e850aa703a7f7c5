// Autotuner for the tile variant of the marginal-gains kernel.
//
// Every variant computes bitwise-identical gains (same per-candidate sum
// order), so the choice only affects speed. The tuner times each variant
// with HIP events on the dataset itself (all-candidate gains at the current
// state, which does not modify the state), keeps the fastest, and records it
// in a process-wide table keyed by (distance dtype, padded row length, size
// bucket floor(log2(n_pad))). The table can be loaded from and saved to a
// text file ("dtype k_pad size_bucket variant" per line).
#include <math.h>
#include <stdio.h>

#include <map>
#include <mutex>
#include <tuple>

#include "ebc_internal.h"

using namespace ebc;

namespace {

using TuneKey = std::tuple<int32_t, int32_t, int32_t>;
std::mutex g_mu;
std::map<TuneKey, int32_t> g_table;

TuneKey key_of(const ebc_dataset* ds) {
    int32_t bucket = 0;
    for (int64_t v = ds->n_pad; v > 1; v >>= 1) ++bucket;
    return TuneKey(int32_t(ds->dt), ds->k_pad, bucket);
}

hipError_t time_variant(ebc_dataset* ds, int32_t reps, hipStream_t s, float* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_gains(ds, nullptr, ds->n_pad, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int32_t r = 0; r < reps && e == hipSuccess; ++r) e = launch_gains(ds, nullptr, ds->n_pad, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}

}  // namespace

namespace ebc {

// Tuned variant for this dataset's key, or -1 when the table has none (no timing).
int32_t tuned_variant(const ebc_dataset* ds) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_table.find(key_of(ds));
    if (it == g_table.end() || it->second >= ebc_gains_variant_count(ds->dt)) return -1;
    return it->second;
}

}  // namespace ebc

extern "C" {

ebc_status ebc_autotune(ebc_dataset* ds, int32_t reps, int32_t force, void* stream, int32_t* variant_out,
                        float* times_ms_out) {
    if (!ds || reps < 1) return EBC_E_INVALID_ARG;
    const TuneKey key = key_of(ds);
    if (!force) {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_table.find(key);
        if (it != g_table.end() && it->second < ebc_gains_variant_count(ds->dt)) {
            ds->variant = it->second;
            if (variant_out) *variant_out = it->second;
            return EBC_OK;
        }
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int32_t nv = ebc_gains_variant_count(ds->dt);
    const int32_t keep = ds->variant;
    int32_t best = 0;
    float best_ms = INFINITY;
    for (int32_t v = 0; v < nv; ++v) {
        ds->variant = v;
        float ms = 0.0f;
        if (time_variant(ds, reps, s, &ms) != hipSuccess) {
            ds->variant = keep;
            return EBC_E_DEVICE;
        }
        if (times_ms_out) times_ms_out[v] = ms / float(reps);
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    ds->variant = best;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_table[key] = best;
    }
    if (variant_out) *variant_out = best;
    return EBC_OK;
}

ebc_status ebc_tune_cache_load(const char* path) {
    if (!path) return EBC_E_INVALID_ARG;
    FILE* f = fopen(path, "r");
    if (!f) return EBC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    int dt, kp, b, v;
    while (fscanf(f, "%d %d %d %d", &dt, &kp, &b, &v) == 4) g_table[TuneKey(dt, kp, b)] = v;
    fclose(f);
    return EBC_OK;
}

ebc_status ebc_tune_cache_save(const char* path) {
    if (!path) return EBC_E_INVALID_ARG;
    FILE* f = fopen(path, "w");
    if (!f) return EBC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    for (const auto& kv : g_table)
        fprintf(f, "%d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second);
    fclose(f);
    return EBC_OK;
}

int32_t ebc_tune_cache_size(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    return int32_t(g_table.size());
}

}  // extern "C"
