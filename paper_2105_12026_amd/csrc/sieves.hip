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
// above or below need no re-score. At an acceptance the summary
// grows (m_v update and f(S) in float64) and the next stretch starts right
// after the accepted point, because every later gain changed. Rejections do
// not change S, so the gains of a stretch stay valid until its first
// acceptance.
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

// float64 gain of one point in f units (stream-synchronous)
hipError_t gain64(const ebc_dataset* ds, int32_t item, hipStream_t s, double* g) {
    hipError_t e = launch_gain64_one(ds, item, s);
    DevState st;
    if (e == hipSuccess) e = read_state(ds, &st, s);
    *g = st.gstar / double(ds->n);
    return e;
}

}  // namespace

extern "C" {

ebc_status ebc_three_sieves(ebc_dataset* ds, int32_t k, double eps, int64_t T, double m_max, const int32_t* order,
                            int64_t n_order, int32_t batch, int32_t* sel_out, double* f_out, int32_t* count_out,
                            int64_t* examined_out, void* stream) {
    if (!ds || !count_out || k < 1 || int64_t(k) > ds->n || !(eps > 0.0) || T < 1 || batch < 0) return EBC_E_INVALID_ARG;
    if (!sel_out || !f_out || n_order < 0 || (!order && n_order > ds->n)) return EBC_E_INVALID_ARG;
    *count_out = 0;
    if (examined_out) *examined_out = 0;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = ds->n;
    if (batch == 0) batch = 1024;
    if (batch > ds->n_pad) batch = int32_t(ds->n_pad);

    // the stream's indices, on the host (validated) and on the device
    std::vector<int32_t> h_order(static_cast<size_t>(n_order));
    if (order && n_order > 0) {
        if (hipMemcpyAsync(h_order.data(), order, size_t(n_order) * sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return EBC_E_DEVICE;
        for (int32_t v : h_order)
            if (v < 0 || int64_t(v) >= n) return EBC_E_INDEX;
    } else {
        for (int64_t i = 0; i < n_order; ++i) h_order[size_t(i)] = int32_t(i);
    }
    char* scratch = nullptr;
    const size_t ord_bytes = (size_t(n_order) * sizeof(int32_t) + 255) & ~size_t(255);
    if (hipMallocAsync(reinterpret_cast<void**>(&scratch), ord_bytes + size_t(batch) * sizeof(double), s) != hipSuccess)
        return EBC_E_DEVICE;
    int32_t* d_order = reinterpret_cast<int32_t*>(scratch);
    double* d_gain = reinterpret_cast<double*>(scratch + ord_bytes);
    auto done = [&](ebc_status st) {
        (void)hipFreeAsync(scratch, s);
        return st;
    };
    if (n_order > 0 && hipMemcpyAsync(d_order, h_order.data(), size_t(n_order) * sizeof(int32_t),
                                      hipMemcpyHostToDevice, s) != hipSuccess)
        return done(EBC_E_DEVICE);

    // S = {}; m = max_e f({e}) unless given: one greedy step (float64 re-scored
    // best singleton), then S = {} again
    if (launch_reset_state(ds, s) != hipSuccess) return done(EBC_E_DEVICE);
    DevState st;
    if (!(m_max > 0.0)) {
        if (launch_greedy_step(ds, 0, sel_out, f_out, nullptr, s, nullptr) != hipSuccess ||
            read_state(ds, &st, s) != hipSuccess)
            return done(EBC_E_DEVICE);
        m_max = st.gstar / double(n);
        if (launch_reset_state(ds, s) != hipSuccess) return done(EBC_E_DEVICE);
    }
    if (read_state(ds, &st, s) != hipSuccess) return done(EBC_E_DEVICE);
    if (st.error != 0) return done(EBC_OK);  // reported by ebc_sync_status
    const std::vector<double> grid = sieve_grid(m_max, k, eps);
    if (grid.empty()) return done(EBC_OK);
    // Every gain is at most m (submodularity: Delta(e|S) <= f({e}) <= m), and
    // the dtype's gains are within window_tau * (largest gain) of float64, so
    // a point whose gain is more than 2 window_tau m away from its bound is
    // decided without a float64 re-score: every decision is the float64 one.
    const double tol = 2.0 * window_tau(ds->dt) * m_max;

    std::vector<double> h_gain(static_cast<size_t>(batch));
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
            return done(EBC_E_DEVICE);
        int64_t next = pos + cnt;
        for (int64_t i = 0; i < cnt && nsel < k; ++i) {
            ++examined;
            const int32_t item = h_order[size_t(pos + i)];
            const double v = grid[j];
            const double bound = (0.5 * v - fS) / double(k - nsel);
            const double g = h_gain[size_t(i)];
            bool take = g >= bound + tol;  // clearly above: the float64 gain is too
            if (!take && g >= bound - tol) {
                double g64 = 0.0;
                if (gain64(ds, item, s, &g64) != hipSuccess) return done(EBC_E_DEVICE);
                take = g64 >= bound;
            }
            if (take) {
                if (launch_accept_one(ds, item, nsel, sel_out, f_out, nullptr, s) != hipSuccess ||
                    hipMemcpyAsync(&fS, f_out + nsel, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    return done(EBC_E_DEVICE);
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
    return done(EBC_OK);
}

}  // extern "C"
