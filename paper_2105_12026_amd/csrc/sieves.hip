// Three Sieves: a streaming optimiser for f (the paper cites it in Sec. 2 and
// runs it beside greedy in the Sec. 6 case study). One summary S, a stream of
// points of V, and a threshold v that walks down the grid of guesses
// (1+eps)^i in [m, k m] (m = max_e f({e})) after T consecutive rejections;
// a point joins while |S| < k and Delta(e|S) >= (v/2 - f(S)) / (k - |S|).
//
// The stream is consumed in stretches. One marginal-gains launch scores the
// next `batch` points against the current S (the same matrix-core kernels as
// greedy, with a candidate list). The host then walks the stretch in order,
// applying the rule. A point whose gain is within twice the dtype's
// re-score half-width (relative to m) of its bound is re-scored in float64
// by direct differences, and the decision uses that value; points clearly
// above or below need no re-score. The first such point of a stretch takes
// the later points of the stretch that may need it into the same re-score
// list (the window re-score of a greedy step). At an acceptance the summary
// grows (m_v update and f(S) in float64) and the next stretch starts right
// after the accepted point, because every later gain changed. Rejections do
// not change S, so the gains of a stretch stay valid until its first
// acceptance.
//
// Sieve Streaming (named with greedy in Sec. 2 and Sec. 4.1 as an optimiser
// that scores many sets per step) keeps one summary per guess v and offers
// every point to each of them under the same rule. Each summary has its own
// running minima m^v (float64, on the device); scoring or growing summary v
// loads m^v into the dataset state first. Each summary has its own stretch
// of gains, re-scored only after that summary changes. The best summary
// (first in grid order among equal f) is returned.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ebc_internal.h"

using namespace ebc;

namespace {

// Guesses (1+eps)^i, m <= (1+eps)^i <= k m, largest first.
std::vector<double> sieve_grid(double m, int32_t k, double eps) {
    std::vector<double> g;
    if (!(m > 0.0)) return g;
    const double base = log1p(eps);
    const int64_t lo = int64_t(ceil(log(m) / base));
    const int64_t hi = int64_t(floor(log(double(k) * m) / base));
    for (int64_t i = hi; i >= lo; --i) g.push_back(pow(1.0 + eps, double(i)));
    return g;
}

hipError_t read_state(const ebc_dataset* ds, DevState* st, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(st, ds->b.state, sizeof(DevState), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

// Device room for a float64 re-score list: indices and gain sums.
constexpr size_t kListBytes = size_t(kWindowMax) * (sizeof(int32_t) + sizeof(double));

// float64 gains in f units of points items[0..W), 1 <= W <= kWindowMax
// (stream-synchronous); `list` is kListBytes of device scratch.
hipError_t gain64_list(const ebc_dataset* ds, const int32_t* items, int32_t W, char* list, double* out,
                       hipStream_t s) {
    int32_t* d_items = reinterpret_cast<int32_t*>(list);
    double* d_out = reinterpret_cast<double*>(list + size_t(kWindowMax) * sizeof(int32_t));
    hipError_t e = hipMemcpyAsync(d_items, items, size_t(W) * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_gain64_many(ds, d_items, W, d_out, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, size_t(W) * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (int32_t j = 0; j < W; ++j) out[j] /= double(ds->n);
    return e;
}

// The float64 gains a stretch needs, computed in lists. When point p of the
// stretch falls inside its band, p and the later points of the stretch whose
// gains lie in [lo, hi) (every bound the rule can still reach, widened by the
// band) are re-scored together; their values hold until the summary changes,
// which ends the stretch. A list holds at most twice the points examined
// since the summary last changed (at least 8, at most kWindowMax), so short
// gaps between acceptances re-score little that goes unused.
struct Gain64Cache {
    std::vector<double> g64;
    std::vector<char> have;
    std::vector<int32_t> items;
    std::vector<int64_t> at;
    std::vector<double> out;
    explicit Gain64Cache(size_t n) : g64(n), have(n, 0) {}
    void clear() { std::fill(have.begin(), have.end(), 0); }
    hipError_t get(const ebc_dataset* ds, const double* gain, const int32_t* stream_items, int64_t p, int64_t len,
                   double lo, double hi, int64_t since, char* list, hipStream_t s, double* g) {
        if (!have[size_t(p)]) {
            const int64_t cap = std::min<int64_t>(kWindowMax, std::max<int64_t>(8, 2 * since));
            items.clear();
            at.clear();
            for (int64_t q = p; q < len && int64_t(at.size()) < cap; ++q)
                if (!have[size_t(q)] && (q == p || (gain[q] >= lo && gain[q] < hi))) {
                    items.push_back(stream_items[q]);
                    at.push_back(q);
                }
            out.resize(at.size());
            const hipError_t e = gain64_list(ds, items.data(), int32_t(at.size()), list, out.data(), s);
            if (e != hipSuccess) return e;
            for (size_t j = 0; j < at.size(); ++j) {
                g64[size_t(at[j])] = out[j];
                have[size_t(at[j])] = 1;
            }
        }
        *g = g64[size_t(p)];
        return hipSuccess;
    }
};

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

// Batch size a call uses: 0 selects 1024, and a stretch never exceeds n_pad.
int32_t effective_batch(int64_t n_pad, int32_t batch) {
    if (batch == 0) batch = 1024;
    if (batch > n_pad) batch = int32_t(n_pad);
    return batch;
}

bool valid_n(int64_t n) { return n >= 1 && n < (int64_t(1) << 31) - kRowAlign; }

// Most guesses (1+eps)^i in [m, k m] for any m > 0: floor(log k / log(1+eps)) + 1,
// plus one for rounding in the logarithms that place the grid ends.
int64_t max_guesses(int32_t k, double eps) { return int64_t(floor(log(double(k)) / log1p(eps))) + 2; }

// Device scratch of Three Sieves: stream indices, one stretch of gains, one re-score list.
size_t three_sieves_scratch(int64_t n_order, int32_t batch) {
    return al256(size_t(n_order) * sizeof(int32_t)) + al256(size_t(batch) * sizeof(double)) + kListBytes;
}

// Per summary of Sieve Streaming: m^v [n_pad] f64, gains of its stretch [batch]
// f64, f [k] f64, members [k] i32.
size_t sieve_summary_bytes(int64_t n_pad, int32_t k, int32_t batch) {
    return al256(size_t(n_pad) * sizeof(double)) + al256(size_t(batch) * sizeof(double)) +
           al256(size_t(k) * sizeof(double)) + al256(size_t(k) * sizeof(int32_t));
}

size_t sieve_streaming_scratch(int64_t n_pad, int32_t k, double eps, int64_t n_order, int32_t batch) {
    return al256(size_t(n_order) * sizeof(int32_t)) +
           size_t(max_guesses(k, eps)) * sieve_summary_bytes(n_pad, k, batch) + kListBytes;
}

// The stream's indices on the host (validated) and on the device, at the
// start of the caller's scratch; *d_extra is the scratch after them.
ebc_status prepare_stream(const ebc_dataset* ds, const int32_t* order, int64_t n_order, char* scratch, hipStream_t s,
                          std::vector<int32_t>& h_order, int32_t** d_order, char** d_extra) {
    h_order.assign(static_cast<size_t>(n_order), 0);
    if (order && n_order > 0) {
        if (hipMemcpyAsync(h_order.data(), order, size_t(n_order) * sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return EBC_E_DEVICE;
        for (int32_t v : h_order)
            if (v < 0 || int64_t(v) >= ds->n) return EBC_E_INDEX;
    } else {
        for (int64_t i = 0; i < n_order; ++i) h_order[size_t(i)] = int32_t(i);
    }
    *d_order = reinterpret_cast<int32_t*>(scratch);
    *d_extra = scratch + al256(size_t(n_order) * sizeof(int32_t));
    if (n_order > 0 && hipMemcpyAsync(*d_order, h_order.data(), size_t(n_order) * sizeof(int32_t),
                                      hipMemcpyHostToDevice, s) != hipSuccess)
        return EBC_E_DEVICE;
    return EBC_OK;
}

// Host checks shared by both optimisers' scratch arguments.
bool scratch_ok(const void* scratch, size_t have, size_t need) {
    return scratch && reinterpret_cast<uintptr_t>(scratch) % 256 == 0 && have >= need;
}

// S = {} in the dataset state; m = max_e f({e}) unless given (> 0): one
// greedy step (the float64 re-scored best singleton), then S = {} again.
ebc_status start_stream(ebc_dataset* ds, double* m_max, int32_t* sel_tmp, double* f_tmp, hipStream_t s,
                        DevState* st) {
    if (launch_reset_state(ds, s) != hipSuccess) return EBC_E_DEVICE;
    if (!(*m_max > 0.0)) {
        if (launch_greedy_step(ds, 0, sel_tmp, f_tmp, nullptr, s, nullptr) != hipSuccess ||
            read_state(ds, st, s) != hipSuccess)
            return EBC_E_DEVICE;
        *m_max = st->gstar / double(ds->n);
        if (launch_reset_state(ds, s) != hipSuccess) return EBC_E_DEVICE;
    }
    return read_state(ds, st, s) == hipSuccess ? EBC_OK : EBC_E_DEVICE;
}

}  // namespace

extern "C" {

size_t ebc_three_sieves_bytes(int64_t n, int64_t n_order, int32_t batch) {
    if (!valid_n(n) || n_order < 0 || batch < 0) return 0;
    return three_sieves_scratch(n_order, effective_batch(pad_rows(n), batch));
}

ebc_status ebc_three_sieves(ebc_dataset* ds, int32_t k, double eps, int64_t T, double m_max, const int32_t* order,
                            int64_t n_order, int32_t batch, int32_t* sel_out, double* f_out, int32_t* count_out,
                            int64_t* examined_out, void* scratch, size_t scratch_bytes, void* stream) {
    if (!ds || !count_out || k < 1 || int64_t(k) > ds->n || !(eps > 0.0) || T < 1 || batch < 0) return EBC_E_INVALID_ARG;
    if (!sel_out || !f_out || n_order < 0 || (!order && n_order > ds->n)) return EBC_E_INVALID_ARG;
    *count_out = 0;
    if (examined_out) *examined_out = 0;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    batch = effective_batch(ds->n_pad, batch);
    if (!scratch_ok(scratch, scratch_bytes, three_sieves_scratch(n_order, batch))) return EBC_E_INVALID_ARG;

    std::vector<int32_t> h_order;
    int32_t* d_order = nullptr;
    char* d_extra = nullptr;
    const size_t gain_bytes = al256(size_t(batch) * sizeof(double));
    ebc_status pst = prepare_stream(ds, order, n_order, static_cast<char*>(scratch), s, h_order, &d_order, &d_extra);
    if (pst != EBC_OK) return pst;
    double* d_gain = reinterpret_cast<double*>(d_extra);
    char* d_list = d_extra + gain_bytes;
    DevState st;
    if ((pst = start_stream(ds, &m_max, sel_out, f_out, s, &st)) != EBC_OK) return pst;
    if (st.error != 0) return EBC_OK;  // reported by ebc_sync_status
    const std::vector<double> grid = sieve_grid(m_max, k, eps);
    if (grid.empty()) return EBC_OK;
    // Every gain is at most m (submodularity: Delta(e|S) <= f({e}) <= m), and
    // the dtype's gains are within window_tau * (largest gain) of float64, so
    // a point whose gain is more than 2 window_tau m away from its bound is
    // decided without a float64 re-score: every decision is the float64 one.
    const double tol = 2.0 * window_tau(ds->dt) * m_max;

    std::vector<double> h_gain(static_cast<size_t>(batch));
    Gain64Cache c64(static_cast<size_t>(batch));
    size_t j = 0;
    int64_t t = 0, pos = 0, examined = 0, last = 0;
    int32_t nsel = 0;
    double fS = 0.0;
    // stretch length: twice the last gap between acceptances (at least 64),
    // doubled after every stretch without one, at most `batch`; only the
    // amount of discarded work depends on it, never a decision
    int64_t stretch = std::min<int64_t>(batch, 256);
    while (pos < n_order && nsel < k) {
        const int64_t cnt = std::min<int64_t>(stretch, n_order - pos);
        if (launch_gains(ds, d_order + pos, cnt, s) != hipSuccess || launch_gains_out(ds, cnt, d_gain, s) != hipSuccess ||
            hipMemcpyAsync(h_gain.data(), d_gain, size_t(cnt) * sizeof(double), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return EBC_E_DEVICE;
        c64.clear();
        int64_t next = pos + cnt;
        for (int64_t i = 0; i < cnt && nsel < k; ++i) {
            ++examined;
            const int32_t item = h_order[size_t(pos + i)];
            const double v = grid[j];
            const double bound = (0.5 * v - fS) / double(k - nsel);
            const double g = h_gain[size_t(i)];
            bool take = g >= bound + tol;  // clearly above: the float64 gain is too
            if (!take && g >= bound - tol) {
                // until the next acceptance the bound can only fall, to that of the last guess
                const double lowest = (0.5 * grid.back() - fS) / double(k - nsel);
                double g64 = 0.0;
                if (c64.get(ds, h_gain.data(), h_order.data() + pos, i, cnt, lowest - tol, bound + tol,
                            pos + i + 1 - last, d_list, s, &g64) != hipSuccess)
                    return EBC_E_DEVICE;
                take = g64 >= bound;
            }
            if (take) {
                if (launch_accept_one(ds, item, nsel, sel_out, f_out, nullptr, s) != hipSuccess ||
                    hipMemcpyAsync(&fS, f_out + nsel, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    return EBC_E_DEVICE;
                ++nsel;
                t = 0;
                next = pos + i + 1;  // later gains are stale: rescore from the next point
                stretch = std::min<int64_t>(batch, std::max<int64_t>(64, 2 * (next - last)));
                last = next;
                break;
            }
            if (++t >= T && j + 1 < grid.size()) {
                ++j;
                t = 0;
            }
        }
        if (next == pos + cnt) stretch = std::min<int64_t>(batch, 2 * stretch);
        pos = next;
    }
    *count_out = nsel;
    if (examined_out) *examined_out = examined;
    ds->stats.steps = nsel;
    return EBC_OK;
}

size_t ebc_sieve_streaming_bytes(int64_t n, int32_t k, double eps, int64_t n_order, int32_t batch) {
    if (!valid_n(n) || k < 1 || int64_t(k) > n || !(eps > 0.0) || n_order < 0 || batch < 0) return 0;
    return sieve_streaming_scratch(pad_rows(n), k, eps, n_order, effective_batch(pad_rows(n), batch));
}

ebc_status ebc_sieve_streaming(ebc_dataset* ds, int32_t k, double eps, double m_max, const int32_t* order,
                               int64_t n_order, int32_t batch, int32_t* sel_out, double* f_out, int32_t* count_out,
                               double* v_out, int64_t* examined_out, void* scratch, size_t scratch_bytes,
                               void* stream) {
    if (!ds || !count_out || k < 1 || int64_t(k) > ds->n || !(eps > 0.0) || batch < 0) return EBC_E_INVALID_ARG;
    if (!sel_out || !f_out || n_order < 0 || (!order && n_order > ds->n)) return EBC_E_INVALID_ARG;
    *count_out = 0;
    if (v_out) *v_out = 0.0;
    if (examined_out) *examined_out = 0;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    batch = effective_batch(ds->n_pad, batch);
    if (!scratch_ok(scratch, scratch_bytes, sieve_streaming_scratch(ds->n_pad, k, eps, n_order, batch)))
        return EBC_E_INVALID_ARG;

    // the grid needs m before the per-summary buffers are laid out
    DevState st;
    ebc_status pst = start_stream(ds, &m_max, sel_out, f_out, s, &st);
    if (pst != EBC_OK) return pst;
    if (st.error != 0) return EBC_OK;  // reported by ebc_sync_status
    const std::vector<double> grid = sieve_grid(m_max, k, eps);
    const int64_t J = int64_t(grid.size());
    if (J == 0) return EBC_OK;
    if (J > max_guesses(k, eps)) return EBC_E_INVALID_ARG;  // not reached: the grid spans a factor k

    auto al = al256;
    const size_t m_bytes = al(size_t(ds->n_pad) * sizeof(double)), g_bytes = al(size_t(batch) * sizeof(double));
    const size_t f_bytes = al(size_t(k) * sizeof(double));
    const size_t per = sieve_summary_bytes(ds->n_pad, k, batch);
    std::vector<int32_t> h_order;
    int32_t* d_order = nullptr;
    char* d_extra = nullptr;
    pst = prepare_stream(ds, order, n_order, static_cast<char*>(scratch), s, h_order, &d_order, &d_extra);
    if (pst != EBC_OK) return pst;
    auto m_of = [&](int64_t j) { return reinterpret_cast<double*>(d_extra + j * per); };
    auto g_of = [&](int64_t j) { return reinterpret_cast<double*>(d_extra + j * per + m_bytes); };
    auto f_of = [&](int64_t j) { return reinterpret_cast<double*>(d_extra + j * per + m_bytes + g_bytes); };
    auto s_of = [&](int64_t j) { return reinterpret_cast<int32_t*>(d_extra + j * per + m_bytes + g_bytes + f_bytes); };
    char* d_list = d_extra + size_t(J) * per;
    const size_t n_bytes = size_t(ds->n) * sizeof(double);
    for (int64_t j = 0; j < J; ++j)  // every summary starts at S = {}: m^v = the current minima
        if (hipMemcpyAsync(m_of(j), ds->b.m64, n_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return EBC_E_DEVICE;

    const double tol = 2.0 * window_tau(ds->dt) * m_max;  // as in ebc_three_sieves
    std::vector<std::vector<double>> h_gain(size_t(J), std::vector<double>(static_cast<size_t>(batch)));
    std::vector<Gain64Cache> c64(size_t(J), Gain64Cache(static_cast<size_t>(batch)));
    std::vector<int64_t> base(size_t(J), 0), len(size_t(J), 0), stretch(size_t(J), std::min<int64_t>(batch, 256));
    std::vector<int64_t> last(size_t(J), 0);
    std::vector<int32_t> cnt(size_t(J), 0);
    std::vector<double> fS(size_t(J), 0.0);
    int64_t loaded = -1, full = 0, examined = 0;
    auto load = [&](int64_t j) -> hipError_t {  // summary j's minima into the dataset state
        if (loaded == j) return hipSuccess;
        loaded = j;
        return launch_load_m(ds, m_of(j), s);
    };
    for (int64_t i = 0; i < n_order && full < J; ++i) {
        ++examined;
        const int32_t item = h_order[size_t(i)];
        for (int64_t j = 0; j < J; ++j) {
            if (cnt[size_t(j)] == k) continue;
            if (!(i >= base[size_t(j)] && i < base[size_t(j)] + len[size_t(j)])) {
                // gains of summary j for the next stretch of the stream
                if (len[size_t(j)] > 0 && i == base[size_t(j)] + len[size_t(j)])
                    stretch[size_t(j)] = std::min<int64_t>(batch, 2 * stretch[size_t(j)]);
                const int64_t L = std::min<int64_t>(stretch[size_t(j)], n_order - i);
                if (load(j) != hipSuccess || launch_gains(ds, d_order + i, L, s) != hipSuccess ||
                    launch_gains_out(ds, L, g_of(j), s) != hipSuccess ||
                    hipMemcpyAsync(h_gain[size_t(j)].data(), g_of(j), size_t(L) * sizeof(double),
                                   hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    return EBC_E_DEVICE;
                base[size_t(j)] = i;
                len[size_t(j)] = L;
                c64[size_t(j)].clear();
            }
            const double bound = (0.5 * grid[size_t(j)] - fS[size_t(j)]) / double(k - cnt[size_t(j)]);
            const double g = h_gain[size_t(j)][size_t(i - base[size_t(j)])];
            bool take = g >= bound + tol;
            if (!take && g >= bound - tol) {
                // summary j's bound holds until it changes
                const int64_t b0 = base[size_t(j)];
                double g64 = 0.0;
                if ((!c64[size_t(j)].have[size_t(i - b0)] && load(j) != hipSuccess) ||
                    c64[size_t(j)].get(ds, h_gain[size_t(j)].data(), h_order.data() + b0, i - b0, len[size_t(j)],
                                       bound - tol, bound + tol, i + 1 - last[size_t(j)], d_list, s,
                                       &g64) != hipSuccess)
                    return EBC_E_DEVICE;
                take = g64 >= bound;
            }
            if (!take) continue;
            const int32_t t = cnt[size_t(j)];
            if (load(j) != hipSuccess || launch_accept_one(ds, item, t, s_of(j), f_of(j), nullptr, s) != hipSuccess ||
                hipMemcpyAsync(m_of(j), ds->b.m64, n_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                hipMemcpyAsync(&fS[size_t(j)], f_of(j) + t, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return EBC_E_DEVICE;
            if (++cnt[size_t(j)] == k) ++full;
            len[size_t(j)] = 0;  // its later gains are stale
            stretch[size_t(j)] = std::min<int64_t>(batch, std::max<int64_t>(64, 2 * (i + 1 - last[size_t(j)])));
            last[size_t(j)] = i + 1;
        }
    }
    int64_t best = 0;
    for (int64_t j = 1; j < J; ++j)
        if (fS[size_t(j)] > fS[size_t(best)]) best = j;
    const int32_t nb = cnt[size_t(best)];
    if ((nb > 0 && (hipMemcpyAsync(sel_out, s_of(best), size_t(nb) * sizeof(int32_t), hipMemcpyDeviceToDevice, s) !=
                        hipSuccess ||
                    hipMemcpyAsync(f_out, f_of(best), size_t(nb) * sizeof(double), hipMemcpyDeviceToDevice, s) !=
                        hipSuccess)) ||
        load(best) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return EBC_E_DEVICE;
    *count_out = nb;
    if (v_out) *v_out = grid[size_t(best)];
    if (examined_out) *examined_out = examined;
    ds->stats.steps = nb;
    return EBC_OK;
}

}  // extern "C"
