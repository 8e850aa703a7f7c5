// Many independent greedy instances (different n, d, k and distance dtype)
// advanced together: per step tick one marginal-gains launch per kernel
// bucket (same dtype, row padding and tile variant) plus the seven step
// launches, each covering every instance through a block -> instance map.
// Each instance runs exactly the arithmetic of its solo ebc_greedy (same
// kernels bodies, same per-instance geometry), so results are bitwise equal
// to solo runs and do not depend on the batch composition.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "ebc_internal.h"

using namespace ebc;

namespace {

struct Bucket {
    int32_t key;
    int32_t slot_begin, slots;  // slots [slot_begin, slot_begin + slots) of slot_inst
    int32_t pre_off;            // its prefix array starts at wg_pre[pre_off] (slots + 1 entries)
    int64_t total_wgs;
};

}  // namespace

struct ebc_batch {
    int32_t count;
    std::vector<ebc_dataset*> ds;
    TableLayout tl;
    char* d_tables;
    InstDesc* d_desc;
    int64_t* d_row_pre;
    int32_t* d_slot_inst;
    int64_t* d_wg_pre;
    int64_t total_rows;
    bool long_rows;  // some instance has rows longer than kNarrowMaxK
    std::vector<Bucket> buckets;
    std::vector<int64_t> h_row_pre, h_wg_pre;
    std::vector<int32_t> h_slot_inst;
    PinnedTables staging;
    // graph mode
    int32_t graph_on;
    hipStream_t cap_stream;
    hipGraphExec_t gexec;
    int32_t g_ticks;
};

namespace {

hipError_t enqueue_ticks(ebc_batch* bt, int32_t ticks, hipStream_t s) {
    hipError_t e = launch_reset_batched(bt->d_desc, bt->d_row_pre, bt->count, bt->total_rows, s);
    for (int32_t t = 0; t < ticks && e == hipSuccess; ++t) {
        for (const Bucket& b : bt->buckets) {
            e = launch_gains_batched(b.key, bt->d_desc, bt->d_slot_inst + b.slot_begin, bt->d_wg_pre + b.pre_off,
                                     b.slots, b.total_wgs, t, s);
            if (e != hipSuccess) return e;
        }
        e = launch_step_batched(bt->d_desc, bt->d_row_pre, bt->count, bt->total_rows, t, bt->long_rows, s);
    }
    return e;
}

void drop_batch_graph(ebc_batch* bt) {
    if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
    bt->gexec = nullptr;
}

}  // namespace

extern "C" {

size_t ebc_batch_bytes(int32_t count) {
    if (count < 1) return 0;
    return table_layout(count).total;
}

ebc_status ebc_batch_create(ebc_dataset* const* ds, int32_t count, void* workspace, size_t workspace_bytes,
                            void* stream, ebc_batch** out) {
    if (!out) return EBC_E_INVALID_ARG;
    *out = nullptr;
    if (!ds || count < 1 || !workspace) return EBC_E_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return EBC_E_INVALID_ARG;
    const TableLayout L = table_layout(count);
    if (workspace_bytes < L.total) return EBC_E_INVALID_ARG;
    for (int32_t i = 0; i < count; ++i)
        if (!ds[i]) return EBC_E_INVALID_ARG;
    for (int32_t i = 0; i < count; ++i)
        if (ds[i]->metric != 0) return EBC_E_UNSUPPORTED;  // batched gains are the squared-distance kernels

    ebc_batch* bt = new (std::nothrow) ebc_batch();
    if (!bt) return EBC_E_NOMEM;
    bt->count = count;
    bt->ds.assign(ds, ds + count);
    char* w = static_cast<char*>(workspace);
    bt->tl = L;
    bt->d_tables = w;
    bt->d_desc = reinterpret_cast<InstDesc*>(w + L.desc);
    bt->d_row_pre = reinterpret_cast<int64_t*>(w + L.row_pre);
    bt->d_slot_inst = reinterpret_cast<int32_t*>(w + L.slot_inst);
    bt->d_wg_pre = reinterpret_cast<int64_t*>(w + L.wg_pre);

    // row-block prefix over all instances
    bt->h_row_pre.resize(count + 1);
    bt->h_row_pre[0] = 0;
    for (int32_t i = 0; i < count; ++i) bt->h_row_pre[i + 1] = bt->h_row_pre[i] + ds[i]->n_pad / kBlock;
    bt->total_rows = bt->h_row_pre[count];
    bt->long_rows = false;
    for (int32_t i = 0; i < count; ++i) bt->long_rows |= wide_rows(ds[i]->k_pad);

    // gains buckets: instances grouped by kernel, in first-seen order
    std::vector<int32_t> keys;
    for (int32_t i = 0; i < count; ++i) {
        const int32_t key = gains_bucket(ds[i]);
        if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
    }
    bt->h_slot_inst.clear();
    bt->h_wg_pre.clear();
    for (int32_t key : keys) {
        Bucket b{};
        b.key = key;
        b.slot_begin = int32_t(bt->h_slot_inst.size());
        b.pre_off = int32_t(bt->h_wg_pre.size());
        int64_t acc = 0;
        bt->h_wg_pre.push_back(0);
        for (int32_t i = 0; i < count; ++i) {
            if (gains_bucket(ds[i]) != key) continue;
            const int64_t tile = gains_cand_tile(ds[i]);
            acc += (ds[i]->n_pad + tile - 1) / tile * ds[i]->v_splits;
            bt->h_slot_inst.push_back(i);
            bt->h_wg_pre.push_back(acc);
        }
        b.slots = int32_t(bt->h_slot_inst.size()) - b.slot_begin;
        b.total_wgs = acc;
        bt->buckets.push_back(b);
    }
    if (bt->staging.init(L.total) != hipSuccess) {
        delete bt;
        return EBC_E_DEVICE;
    }
    *out = bt;
    return EBC_OK;
}

ebc_status ebc_batch_destroy(ebc_batch* bt) {
    if (!bt) return EBC_E_INVALID_ARG;
    drop_batch_graph(bt);
    if (bt->cap_stream) (void)hipStreamDestroy(bt->cap_stream);
    delete bt;
    return EBC_OK;
}

ebc_status ebc_batch_set_graph(ebc_batch* bt, int32_t on) {
    if (!bt) return EBC_E_INVALID_ARG;
    bt->graph_on = on ? 1 : 0;
    if (!on) drop_batch_graph(bt);
    return EBC_OK;
}

ebc_status ebc_greedy_batched(ebc_batch* bt, const int32_t* k, int32_t* const* sel_out, double* const* f_out,
                              double* const* gain_out, void* stream) {
    if (!bt || !k || !sel_out || !f_out) return EBC_E_INVALID_ARG;
    int32_t ticks = 0;
    for (int32_t i = 0; i < bt->count; ++i) {
        if (k[i] < 0 || int64_t(k[i]) > bt->ds[i]->n) return EBC_E_INVALID_ARG;
        if (k[i] > 0 && (!sel_out[i] || !f_out[i])) return EBC_E_INVALID_ARG;
        ticks = std::max(ticks, k[i]);
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // descriptors and block maps, staged in pinned memory, one copy
    hipError_t e = hipSuccess;
    char* h = bt->staging.acquire(&e);
    if (e != hipSuccess) return EBC_E_DEVICE;
    InstDesc* hd = reinterpret_cast<InstDesc*>(h + bt->tl.desc);
    for (int32_t i = 0; i < bt->count; ++i) {
        fill_desc(bt->ds[i], k[i], sel_out[i], f_out[i], gain_out ? gain_out[i] : nullptr, &hd[i]);
        bt->ds[i]->stats.steps = k[i];
    }
    memcpy(h + bt->tl.row_pre, bt->h_row_pre.data(), bt->h_row_pre.size() * sizeof(int64_t));
    memcpy(h + bt->tl.slot_inst, bt->h_slot_inst.data(), bt->h_slot_inst.size() * sizeof(int32_t));
    memcpy(h + bt->tl.wg_pre, bt->h_wg_pre.data(), bt->h_wg_pre.size() * sizeof(int64_t));
    if (bt->staging.submit(bt->d_tables, bt->tl.total, s) != hipSuccess) return EBC_E_DEVICE;
    if (ticks == 0) return EBC_OK;
    if (bt->graph_on) {
        if (!(bt->gexec && bt->g_ticks == ticks)) {
            drop_batch_graph(bt);
            if (!bt->cap_stream && (e = hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking)) != hipSuccess)
                return EBC_E_DEVICE;
            if ((e = hipStreamBeginCapture(bt->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess)
                return EBC_E_DEVICE;
            hipError_t le = enqueue_ticks(bt, ticks, bt->cap_stream);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(bt->cap_stream, &g);
            if (le != hipSuccess) e = le;
            if (e == hipSuccess) e = hipGraphInstantiate(&bt->gexec, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                bt->gexec = nullptr;
                return EBC_E_DEVICE;
            }
            bt->g_ticks = ticks;
        }
        return hipGraphLaunch(bt->gexec, s) == hipSuccess ? EBC_OK : EBC_E_DEVICE;
    }
    return enqueue_ticks(bt, ticks, s) == hipSuccess ? EBC_OK : EBC_E_DEVICE;
}

ebc_status ebc_batch_info(ebc_batch* bt, int32_t* buckets, int64_t* gains_workgroups_per_tick,
                          int64_t* row_blocks_per_tick) {
    if (!bt) return EBC_E_INVALID_ARG;
    if (buckets) *buckets = int32_t(bt->buckets.size());
    if (gains_workgroups_per_tick) {
        int64_t w = 0;
        for (const Bucket& b : bt->buckets) w += b.total_wgs;
        *gains_workgroups_per_tick = w;
    }
    if (row_blocks_per_tick) *row_blocks_per_tick = bt->total_rows;
    return EBC_OK;
}

}  // extern "C"
