// Serving core: summarisation requests (a ground set and a greedy bound k)
// are admitted into one device arena by their exact footprint, stay resident
// (points, distance-dtype copy, running minima) while active, and advance
// together by one greedy step per scheduler tick (continuous batching at
// step granularity): requests that arrive while others run join at the next
// tick as slots and arena space free up, and each finished request is copied
// out and its space released at the tick it completes. One tick issues one
// gains launch per kernel bucket and seven step launches for all active
// requests; each request computes exactly what a solo ebc_greedy computes.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "ebc_internal.h"

using namespace ebc;

// ---------------------------------------------------------------------------
// First-fit arena allocator (host bookkeeping only; offsets into a device
// block the caller owns). Free blocks are kept sorted and coalesced.
// ---------------------------------------------------------------------------
struct ebc_arena {
    size_t capacity;
    std::map<size_t, size_t> free_;   // offset -> size
    std::map<size_t, size_t> used_;   // offset -> size
    size_t free_bytes() const {
        size_t s = 0;
        for (const auto& kv : free_) s += kv.second;
        return s;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t o = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[o + bytes] = rest;
                used_[o] = bytes;
                *off = o;
                return true;
            }
        }
        return false;
    }
    bool release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        size_t o = off, sz = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(o);
        if (nx != free_.end() && o + sz == nx->first) {
            sz += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == o) {
                pv->second += sz;
                return true;
            }
        }
        free_[o] = sz;
        return true;
    }
};

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

enum ReqState { kQueued = 0, kActive = 1, kDone = 2, kFailed = 3 };

struct Request {
    int64_t id;
    int64_t n;
    int32_t d, k;
    ebc_dtype dt;
    std::vector<float> xh;
    int state = kQueued;
    int32_t t = 0;  // steps done
    size_t off = 0, bytes = 0;
    float* xd = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int32_t* sel_d = nullptr;
    double* f_d = nullptr;
    double* gain_d = nullptr;
    ebc_dataset* ds = nullptr;
    std::vector<int32_t> sel_h;
    std::vector<double> f_h, gain_h;
    double t_arrive = 0, t_admit = 0, t_done = 0;
    int error = 0;
};

// Device footprint of one request inside the arena: its points, the dataset
// workspace and the outputs.
size_t request_bytes(int64_t n, int32_t d, int32_t k, ebc_dtype dt, size_t* ws_bytes) {
    *ws_bytes = ebc_dataset_bytes(n, d, dt);
    if (*ws_bytes == 0) return 0;
    return a256(size_t(n) * d * sizeof(float)) + a256(*ws_bytes) + a256(size_t(k) * sizeof(int32_t)) +
           2 * a256(size_t(k) * sizeof(double));
}

}  // namespace

struct ebc_server {
    char* base;
    size_t bytes;
    int32_t max_slots;
    hipStream_t stream;
    ebc_arena arena;
    // batched-tick tables, reserved at the start of the arena for max_slots
    TableLayout tl;
    InstDesc* d_desc;
    int64_t* d_row_pre;
    int32_t* d_slot;
    int64_t* d_wg_pre;
    PinnedTables staging;
    std::vector<int64_t> h_row_pre, h_wg_pre;
    std::vector<int32_t> h_slot;
    struct Bucket {
        int32_t key, slot_begin, slots, pre_off;
        int64_t total_wgs;
    };
    std::vector<Bucket> buckets;
    int64_t total_rows = 0;
    bool dirty = true;
    std::deque<Request*> queue;
    std::vector<Request*> active;
    std::map<int64_t, Request*> all;
    int64_t next_id = 1;
    int64_t ticks = 0, completed = 0, admitted = 0;
    double busy_s = 0;
    ~ebc_server() {
        for (auto& kv : all) {
            if (kv.second->ds) ebc_dataset_destroy(kv.second->ds);
            delete kv.second;
        }
    }
};

namespace {

ebc_status admit(ebc_server* sv, Request* r) {
    size_t ws_bytes = 0;
    const size_t need = request_bytes(r->n, r->d, r->k, r->dt, &ws_bytes);
    size_t off = 0;
    if (!sv->arena.alloc(need, &off)) return EBC_E_NOMEM;
    r->off = off;
    r->bytes = need;
    char* p = sv->base + off;
    r->xd = reinterpret_cast<float*>(p);
    p += a256(size_t(r->n) * r->d * sizeof(float));
    r->ws = p;
    r->ws_bytes = ws_bytes;
    p += a256(ws_bytes);
    r->sel_d = reinterpret_cast<int32_t*>(p);
    p += a256(size_t(r->k) * sizeof(int32_t));
    r->f_d = reinterpret_cast<double*>(p);
    p += a256(size_t(r->k) * sizeof(double));
    r->gain_d = reinterpret_cast<double*>(p);
    hipError_t e = hipMemcpyAsync(r->xd, r->xh.data(), r->xh.size() * sizeof(float), hipMemcpyHostToDevice,
                                  sv->stream);
    ebc_status st = e == hipSuccess ? EBC_OK : EBC_E_DEVICE;
    if (st == EBC_OK) st = ebc_dataset_create(r->xd, r->n, r->d, r->dt, 0, r->ws, ws_bytes, sv->stream, &r->ds);
    if (st == EBC_OK) st = launch_reset_state(r->ds, sv->stream) == hipSuccess ? EBC_OK : EBC_E_DEVICE;
    if (st != EBC_OK) {
        if (r->ds) ebc_dataset_destroy(r->ds);
        r->ds = nullptr;
        sv->arena.release(off);
        return st;
    }
    // gains tile variant from the autotuner's table (results do not depend on it)
    const int32_t v = tuned_variant(r->ds);
    if (v >= 0) r->ds->variant = v;
    r->state = kActive;
    r->t = 0;
    r->t_admit = now_s();
    return EBC_OK;
}

void rebuild_tables(ebc_server* sv) {
    const int32_t count = int32_t(sv->active.size());
    sv->h_row_pre.assign(count + 1, 0);
    for (int32_t i = 0; i < count; ++i) sv->h_row_pre[i + 1] = sv->h_row_pre[i] + sv->active[i]->ds->n_pad / kBlock;
    sv->total_rows = sv->h_row_pre[count];
    std::vector<int32_t> keys;
    for (Request* r : sv->active) {
        const int32_t key = gains_bucket(r->ds);
        if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
    }
    sv->buckets.clear();
    sv->h_slot.clear();
    sv->h_wg_pre.clear();
    for (int32_t key : keys) {
        ebc_server::Bucket b{};
        b.key = key;
        b.slot_begin = int32_t(sv->h_slot.size());
        b.pre_off = int32_t(sv->h_wg_pre.size());
        int64_t acc = 0;
        sv->h_wg_pre.push_back(0);
        for (int32_t i = 0; i < count; ++i) {
            const ebc_dataset* ds = sv->active[i]->ds;
            if (gains_bucket(ds) != key) continue;
            const int64_t tile = gains_cand_tile(ds);
            acc += (ds->n_pad + tile - 1) / tile * ds->v_splits;
            sv->h_slot.push_back(i);
            sv->h_wg_pre.push_back(acc);
        }
        b.slots = int32_t(sv->h_slot.size()) - b.slot_begin;
        b.total_wgs = acc;
        sv->buckets.push_back(b);
    }
}

}  // namespace

extern "C" {

// ---- arena allocator (host bookkeeping; exported for tests and drivers) ----
ebc_status ebc_arena_create(size_t capacity, ebc_arena** out) {
    if (!out || capacity == 0) return EBC_E_INVALID_ARG;
    ebc_arena* a = new (std::nothrow) ebc_arena();
    if (!a) return EBC_E_NOMEM;
    a->capacity = capacity & ~size_t(255);
    if (a->capacity) a->free_[0] = a->capacity;
    *out = a;
    return EBC_OK;
}
ebc_status ebc_arena_alloc(ebc_arena* a, size_t bytes, size_t* offset) {
    if (!a || !offset) return EBC_E_INVALID_ARG;
    return a->alloc(bytes, offset) ? EBC_OK : EBC_E_NOMEM;
}
ebc_status ebc_arena_free(ebc_arena* a, size_t offset) {
    if (!a) return EBC_E_INVALID_ARG;
    return a->release(offset) ? EBC_OK : EBC_E_INVALID_ARG;
}
size_t ebc_arena_free_bytes(const ebc_arena* a) { return a ? a->free_bytes() : 0; }
size_t ebc_arena_largest_free(const ebc_arena* a) {
    size_t m = 0;
    if (a)
        for (const auto& kv : a->free_) m = std::max(m, kv.second);
    return m;
}
ebc_status ebc_arena_destroy(ebc_arena* a) {
    if (!a) return EBC_E_INVALID_ARG;
    delete a;
    return EBC_OK;
}

size_t ebc_request_bytes(int64_t n, int32_t d, int32_t k, ebc_dtype dt) {
    size_t ws = 0;
    if (k < 1 || int64_t(k) > n) return 0;
    return request_bytes(n, d, k, dt, &ws);
}

// ---- server ----
ebc_status ebc_server_create(void* arena, size_t arena_bytes, int32_t max_slots, void* stream, ebc_server** out) {
    if (!out) return EBC_E_INVALID_ARG;
    *out = nullptr;
    if (!arena || max_slots < 1 || reinterpret_cast<uintptr_t>(arena) % 256 != 0) return EBC_E_INVALID_ARG;
    const TableLayout tl = table_layout(max_slots);
    const size_t tb = tl.total;
    if (arena_bytes < tb + 256) return EBC_E_INVALID_ARG;
    ebc_server* sv = new (std::nothrow) ebc_server();
    if (!sv) return EBC_E_NOMEM;
    sv->base = static_cast<char*>(arena);
    sv->bytes = arena_bytes;
    sv->max_slots = max_slots;
    sv->stream = reinterpret_cast<hipStream_t>(stream);
    sv->tl = tl;
    sv->d_desc = reinterpret_cast<InstDesc*>(sv->base + tl.desc);
    sv->d_row_pre = reinterpret_cast<int64_t*>(sv->base + tl.row_pre);
    sv->d_slot = reinterpret_cast<int32_t*>(sv->base + tl.slot_inst);
    sv->d_wg_pre = reinterpret_cast<int64_t*>(sv->base + tl.wg_pre);
    if (sv->staging.init(tb) != hipSuccess) {
        delete sv;
        return EBC_E_DEVICE;
    }
    // the allocator manages the rest: offsets are relative to sv->base
    sv->arena.capacity = arena_bytes & ~size_t(255);
    sv->arena.free_[tb] = sv->arena.capacity - tb;
    *out = sv;
    return EBC_OK;
}

ebc_status ebc_server_destroy(ebc_server* sv) {
    if (!sv) return EBC_E_INVALID_ARG;
    (void)hipStreamSynchronize(sv->stream);
    delete sv;
    return EBC_OK;
}

ebc_status ebc_server_submit(ebc_server* sv, const float* x_host, int64_t n, int32_t d, int32_t k, ebc_dtype dt,
                             double t_arrival, int64_t* req_id) {
    if (!sv || !x_host || !req_id || k < 1 || int64_t(k) > n) return EBC_E_INVALID_ARG;
    size_t ws = 0;
    const size_t need = request_bytes(n, d, k, dt, &ws);
    if (need == 0) return d > EBC_MAX_DIM ? EBC_E_UNSUPPORTED : EBC_E_INVALID_ARG;
    if (need > sv->arena.capacity) return EBC_E_NOMEM;  // can never fit
    Request* r = new (std::nothrow) Request();
    if (!r) return EBC_E_NOMEM;
    r->id = sv->next_id++;
    r->n = n;
    r->d = d;
    r->k = k;
    r->dt = dt;
    r->xh.assign(x_host, x_host + size_t(n) * d);
    r->t_arrive = t_arrival >= 0 ? t_arrival : now_s();
    sv->queue.push_back(r);
    sv->all[r->id] = r;
    *req_id = r->id;
    return EBC_OK;
}

// One scheduler tick: admit queued requests (FIFO) while a slot and arena
// space are free, advance every active request by one greedy step in one
// batched launch set, then copy out and release the requests that reached k.
ebc_status ebc_server_step(ebc_server* sv, int32_t* completed) {
    if (!sv) return EBC_E_INVALID_ARG;
    if (completed) *completed = 0;
    const double t_begin = now_s();
    while (!sv->queue.empty() && int32_t(sv->active.size()) < sv->max_slots) {
        Request* r = sv->queue.front();
        const ebc_status st = admit(sv, r);
        if (st == EBC_E_NOMEM) break;  // head of the queue waits for space
        sv->queue.pop_front();
        if (st != EBC_OK) {
            r->state = kFailed;
            r->error = st;
            r->t_done = now_s();
            std::vector<float>().swap(r->xh);
            continue;
        }
        sv->active.push_back(r);
        ++sv->admitted;
        sv->dirty = true;
    }
    if (sv->active.empty()) return EBC_OK;
    hipError_t e = hipSuccess;
    const int32_t count = int32_t(sv->active.size());
    if (sv->dirty) {
        rebuild_tables(sv);
        sv->dirty = false;
    }
    // descriptors (with each request's step) and block maps: one pinned copy
    char* h = sv->staging.acquire(&e);
    if (e != hipSuccess) return EBC_E_DEVICE;
    InstDesc* hd = reinterpret_cast<InstDesc*>(h + sv->tl.desc);
    for (int32_t i = 0; i < count; ++i) {
        Request* r = sv->active[i];
        fill_desc(r->ds, r->k, r->sel_d, r->f_d, r->gain_d, &hd[i]);
        hd[i].t0 = r->t;
    }
    memcpy(h + sv->tl.row_pre, sv->h_row_pre.data(), sv->h_row_pre.size() * sizeof(int64_t));
    memcpy(h + sv->tl.slot_inst, sv->h_slot.data(), sv->h_slot.size() * sizeof(int32_t));
    memcpy(h + sv->tl.wg_pre, sv->h_wg_pre.data(), sv->h_wg_pre.size() * sizeof(int64_t));
    e = sv->staging.submit(sv->base, sv->tl.total, sv->stream);
    for (const auto& b : sv->buckets) {
        if (e != hipSuccess) break;
        e = launch_gains_batched(b.key, sv->d_desc, sv->d_slot + b.slot_begin, sv->d_wg_pre + b.pre_off, b.slots,
                                 b.total_wgs, 0, sv->stream);
    }
    bool long_rows = false;
    for (const Request* r : sv->active) long_rows |= wide_rows(r->ds->k_pad);
    if (e == hipSuccess)
        e = launch_step_batched(sv->d_desc, sv->d_row_pre, count, sv->total_rows, 0, long_rows, sv->stream);
    if (e != hipSuccess) return EBC_E_DEVICE;
    ++sv->ticks;
    // finished requests: copy out at the end of this tick
    std::vector<Request*> finished, still;
    for (Request* r : sv->active) {
        ++r->t;
        (r->t >= r->k ? finished : still).push_back(r);
    }
    if (!finished.empty()) {
        for (Request* r : finished) {
            r->sel_h.resize(r->k);
            r->f_h.resize(r->k);
            r->gain_h.resize(r->k);
            e = hipMemcpyAsync(r->sel_h.data(), r->sel_d, r->k * sizeof(int32_t), hipMemcpyDeviceToHost, sv->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->f_h.data(), r->f_d, r->k * sizeof(double), hipMemcpyDeviceToHost, sv->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->gain_h.data(), r->gain_d, r->k * sizeof(double), hipMemcpyDeviceToHost,
                                   sv->stream);
            if (e != hipSuccess) return EBC_E_DEVICE;
        }
        if (hipStreamSynchronize(sv->stream) != hipSuccess) return EBC_E_DEVICE;
        const double t_now = now_s();
        for (Request* r : finished) {
            ebc_greedy_stats st;
            r->error = ebc_sync_status(r->ds, sv->stream, &st);
            r->state = r->error ? kFailed : kDone;
            r->t_done = t_now;
            ebc_dataset_destroy(r->ds);
            r->ds = nullptr;
            sv->arena.release(r->off);
            std::vector<float>().swap(r->xh);  // its upload finished long ago (stream synchronised)
            ++sv->completed;
        }
        sv->active.swap(still);
        sv->dirty = true;
        if (completed) *completed = int32_t(finished.size());
    }
    sv->busy_s += now_s() - t_begin;
    return EBC_OK;
}

// state: 0 queued, 1 active, 2 done, 3 failed. Outputs (k entries each) are
// filled when done; NULL pointers are skipped. Times are seconds on the
// server's steady clock (ebc_server_now); latency = done - arrival.
ebc_status ebc_server_poll(ebc_server* sv, int64_t req_id, int32_t* state, int32_t* sel_host, double* f_host,
                           double* gain_host, double* t_arrive, double* t_admit, double* t_done) {
    if (!sv || !state) return EBC_E_INVALID_ARG;
    auto it = sv->all.find(req_id);
    if (it == sv->all.end()) return EBC_E_INVALID_ARG;
    Request* r = it->second;
    *state = r->state;
    if (r->state == kDone) {
        if (sel_host) memcpy(sel_host, r->sel_h.data(), r->k * sizeof(int32_t));
        if (f_host) memcpy(f_host, r->f_h.data(), r->k * sizeof(double));
        if (gain_host) memcpy(gain_host, r->gain_h.data(), r->k * sizeof(double));
    }
    if (t_arrive) *t_arrive = r->t_arrive;
    if (t_admit) *t_admit = r->t_admit;
    if (t_done) *t_done = r->t_done;
    return r->state == kFailed ? ebc_status(r->error) : EBC_OK;
}

ebc_status ebc_server_stats(ebc_server* sv, int32_t* queued, int32_t* active, int64_t* completed,
                            int64_t* ticks, size_t* free_bytes) {
    if (!sv) return EBC_E_INVALID_ARG;
    if (queued) *queued = int32_t(sv->queue.size());
    if (active) *active = int32_t(sv->active.size());
    if (completed) *completed = sv->completed;
    if (ticks) *ticks = sv->ticks;
    if (free_bytes) *free_bytes = sv->arena.free_bytes();
    return EBC_OK;
}

double ebc_server_now(void) { return now_s(); }

}  // extern "C"
