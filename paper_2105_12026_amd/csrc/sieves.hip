// Streaming optimisers for f: Three Sieves (the paper cites it in Sec. 2 and
// runs it beside greedy in the Sec. 6 case study) and Sieve Streaming (named
// with greedy in Sec. 2 and Sec. 4.1 as an optimiser that scores many sets
// per step).
//
// Both walk a stream of points of V. Three Sieves keeps one summary S and a
// threshold v that walks down the grid of guesses (1+eps)^i in [m, k m]
// (m = max_e f({e})) after T consecutive rejections; Sieve Streaming keeps
// one summary per guess. A point e joins summary S (guess v) while |S| < k
// and
//     Delta(e|S) >= (v/2 - f(S)) / (k - |S|),
//     Delta(e|S) = |V|^-1 sum_v max(0, m_v - d(v, e))      (Sec. 3, Sec. 4.1)
// with m_v the running minima of S u {e0}.
//
// What a decision needs of the arriving point e is the distance vector
// d(., e) over the ground set, and that vector does not depend on any
// summary. So the stream is processed in stretches of points: one launch
// computes the float64 distances of a stretch's points to every ground point
// (direct differences, the same definition as the float64 re-score and the
// oracle), and one launch with a workgroup per summary walks the stretch in
// stream order, each workgroup clamping and summing its own minima against
// each distance row, deciding, and on acceptance lowering its minima and
// recomputing f(S) -- all in float64 on the device, so every decision is a
// float64 one in every distance dtype, and no host round trip happens
// between the first launch and the result. Distance rows are prefetched into
// registers several points ahead (they do not depend on the decisions), so
// the sequential walk waits only on its own reductions.
#include <math.h>

#include <algorithm>
#include <vector>

#include "ebc_internal.h"

using namespace ebc;

namespace {

constexpr int kST = 256;             // threads of the stream kernels
constexpr int kDI = 32;              // stream points per distance tile
constexpr int kDV = 64;              // ground points per distance tile
constexpr int kDK = 16;              // dimensions per LDS stage of the distance tile
constexpr int kRegMax = 16;          // ground points per thread kept in registers (n_pad <= 4096)
constexpr size_t kStretchBytes = size_t(256) << 20;  // distance rows of one default stretch, at most

// One summary's state, in the caller's scratch.
struct Summary {
    int32_t cnt;      // members so far
    int32_t t;        // consecutive rejections (Three Sieves)
    int32_t gi;       // index of the current guess (Three Sieves)
    int32_t pad;
    int64_t full_at;  // stream position of the k-th acceptance, -1 before
    double fS;        // f of the summary
};

struct Result {
    int32_t count;     // members of the returned summary
    int32_t best;      // its index (0 for Three Sieves)
    int64_t examined;  // points taken from the stream
};

__device__ __forceinline__ int64_t stream_row(const int32_t* __restrict__ order, int64_t p) {
    return order ? int64_t(order[p]) : p;
}

// float64 sum over the 64 lanes; lane 0's value has a fixed association
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Distances of stream points pos + [0, cnt) to every ground point, float64
// direct differences in dimension order, into D [cnt][n_pad] (columns >= n
// are not written). A workgroup computes a 32 x 64 tile, both sides staged
// through LDS 16 dimensions at a time (the next stage's values loaded into
// registers while the current one is used); thread (ti, tv) owns stream
// points ti + 16a and ground points tv + 16b. Nothing runs once every
// summary is full.
template <int METRIC>
__global__ void __launch_bounds__(kST) k_stream_dist(const float* __restrict__ x, int64_t n, int32_t d,
                                                     const int32_t* __restrict__ order, int64_t pos, int32_t cnt,
                                                     int64_t n_pad, double* __restrict__ D,
                                                     const Summary* __restrict__ sm, int32_t ns, int32_t k) {
    __shared__ int open;
    __shared__ double A[2][kDK][kDI];
    __shared__ double B[2][kDK][kDV];
    const int tid = threadIdx.x;
    if (tid == 0) open = 0;
    __syncthreads();
    for (int j = tid; j < ns; j += kST)
        if (sm[j].cnt < k) open = 1;
    __syncthreads();
    if (!open) return;

    const int tv = tid & 15, ti = tid >> 4;
    const int64_t v0 = int64_t(blockIdx.x) * kDV;
    const int i0 = int(blockIdx.y) * kDI;
    // loaders: stream row ar, dimensions ak, ak+1; ground row br, dimensions bk .. bk+3
    const int ar = tid >> 3, ak = 2 * (tid & 7);
    const int br = tid >> 2, bk = 4 * (tid & 3);
    const float* __restrict__ arow = (i0 + ar < cnt) ? x + stream_row(order, pos + i0 + ar) * d : nullptr;
    const float* __restrict__ brow = (v0 + br < n) ? x + (v0 + br) * d : nullptr;
    float ra[2], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int kk = k0 + ak + q;
            ra[q] = (arow && kk < d) ? arow[kk] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = k0 + bk + q;
            rb[q] = (brow && kk < d) ? brow[kk] : 0.0f;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) A[buf][ak + q][ar] = double(ra[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) B[buf][bk + q][br] = double(rb[q]);
    };

    double acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    const int nk = (d + kDK - 1) / kDK;
    load(0);
    store(0);
    __syncthreads();
    for (int c = 0; c < nk; ++c) {
        const int buf = c & 1;
        if (c + 1 < nk) load((c + 1) * kDK);
#pragma unroll
        for (int kk = 0; kk < kDK; ++kk) {
            double a[2], b[4];
#pragma unroll
            for (int q = 0; q < 2; ++q) a[q] = A[buf][kk][ti + 16 * q];
#pragma unroll
            for (int q = 0; q < 4; ++q) b[q] = B[buf][kk][tv + 16 * q];
#pragma unroll
            for (int qa = 0; qa < 2; ++qa)
#pragma unroll
                for (int qb = 0; qb < 4; ++qb) {
                    const double df = a[qa] - b[qb];
                    if (METRIC == 1)
                        acc[qa][qb] += fabs(df);
                    else
                        acc[qa][qb] = fma(df, df, acc[qa][qb]);
                }
        }
        // the other stage was last read before the previous barrier
        if (c + 1 < nk) store(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int qa = 0; qa < 2; ++qa) {
        const int i = i0 + ti + 16 * qa;
        if (i >= cnt) continue;
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) {
            const int64_t v = v0 + tv + 16 * qb;
            if (v < n) D[int64_t(i) * n_pad + v] = acc[qa][qb];
        }
    }
}

// Arguments of the decision walk over one stretch.
struct WalkArgs {
    const double* D;       // [cnt][n_pad] distances of the stretch
    int64_t n, n_pad;
    int32_t cnt;           // points in the stretch
    int32_t k;
    int64_t pos;           // stream position of the stretch's first point
    const int32_t* order;  // stream indices (null: 0, 1, ...)
    const double* grid;    // guesses, largest first
    int32_t J;             // guesses
    int32_t pad;
    int64_t T;             // Three Sieves: rejections before the next guess; 0: Sieve Streaming
    const DevState* dst;   // L({e0}) of the dataset
    Summary* sm;           // [summaries]
    double* M;             // [summaries][n_pad] running minima
    int32_t* sel;          // [summaries][k] members
    double* fv;            // [summaries][k] f after each acceptance
};

// The rule for one point, given its float64 gain sum over V (uniform across
// the workgroup). Returns true when the point joins.
__device__ __forceinline__ bool decide(const WalkArgs& w, int j, const Summary& s, double gsum) {
    const double g = gsum / double(w.n);
    const double v = w.T > 0 ? w.grid[s.gi] : w.grid[j];
    const double bound = (0.5 * v - s.fS) / double(w.k - s.cnt);
    return g >= bound;
}

// Bookkeeping after a decision; returns true once the summary is full.
__device__ __forceinline__ bool record(const WalkArgs& w, int j, Summary& s, bool take, int i, double msum) {
    if (take) {
        const double fS = w.dst->l0 - msum / double(w.n);
        if (threadIdx.x == 0) {
            w.sel[int64_t(j) * w.k + s.cnt] = int32_t(stream_row(w.order, w.pos + i));
            w.fv[int64_t(j) * w.k + s.cnt] = fS;
        }
        s.fS = fS;
        s.cnt += 1;
        s.t = 0;
        if (s.cnt == w.k) {
            s.full_at = w.pos + i;
            return true;
        }
    } else if (w.T > 0) {
        if (++s.t >= w.T && s.gi + 1 < w.J) {
            s.gi += 1;
            s.t = 0;
        }
    }
    return false;
}

// Workgroup-uniform float64 sum of one value per thread: lane 0 of each wave
// writes its wave's sum, then every thread adds the four in wave order.
__device__ __forceinline__ double block_sum(double v, double* slot) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((slot[0] + slot[1]) + slot[2]) + slot[3];
}

// Decision walk, one workgroup per summary, thread t owning ground points
// t + 256 r (r < R) with their minima in registers; rows of the next P
// points in flight.
template <int R, int P>
__global__ void __launch_bounds__(kST) k_stream_walk(WalkArgs w) {
    const int j = blockIdx.x;
    Summary s = w.sm[j];
    if (s.cnt >= w.k) return;
    __shared__ double red[2][4];
    __shared__ double fred[4];
    const int tid = threadIdx.x;
    double* __restrict__ m = w.M + int64_t(j) * w.n_pad;
    double mr[R];
    bool ok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t v = tid + int64_t(kST) * r;
        ok[r] = v < w.n;
        mr[r] = ok[r] ? m[v] : 0.0;
    }
    double row[P][R];
    auto load_row = [&](int i, double (&dst)[R]) {
        const double* __restrict__ src = w.D + int64_t(i) * w.n_pad + tid;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r] = ok[r] ? src[kST * r] : 0.0;
    };
#pragma unroll
    for (int q = 0; q < P; ++q)
        if (q < w.cnt) load_row(q, row[q]);
    bool changed = false, stop = false;
    for (int i0 = 0; i0 < w.cnt && !stop; i0 += P) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int i = i0 + q;
            if (stop || i >= w.cnt) break;
            double p = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) p += fmax(0.0, mr[r] - row[q][r]);
            const double g = block_sum(p, red[i & 1]);
            const bool take = decide(w, j, s, g);
            double msum = 0.0;
            if (take) {
                double qs = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    mr[r] = fmin(mr[r], row[q][r]);
                    qs += mr[r];
                }
                msum = block_sum(qs, fred);
                changed = true;
            }
            stop = record(w, j, s, take, i, msum);
            if (!stop && i + P < w.cnt) load_row(i + P, row[q]);
        }
    }
    if (changed) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (ok[r]) m[tid + int64_t(kST) * r] = mr[r];
    }
    if (tid == 0) w.sm[j] = s;
}

// The same walk for ground sets above 256 * kRegMax points: minima in the
// scratch, rows read as they are used (same per-thread summation order).
__global__ void __launch_bounds__(kST) k_stream_walk_big(WalkArgs w) {
    const int j = blockIdx.x;
    Summary s = w.sm[j];
    if (s.cnt >= w.k) return;
    __shared__ double red[2][4];
    __shared__ double fred[4];
    const int tid = threadIdx.x;
    double* __restrict__ m = w.M + int64_t(j) * w.n_pad;
    for (int i = 0; i < w.cnt; ++i) {
        const double* __restrict__ row = w.D + int64_t(i) * w.n_pad;
        double p = 0.0;
        for (int64_t v = tid; v < w.n; v += kST) p += fmax(0.0, m[v] - row[v]);
        const double g = block_sum(p, red[i & 1]);
        const bool take = decide(w, j, s, g);
        double msum = 0.0;
        if (take) {
            double qs = 0.0;
            for (int64_t v = tid; v < w.n; v += kST) {
                const double mv = fmin(m[v], row[v]);
                m[v] = mv;
                qs += mv;
            }
            msum = block_sum(qs, fred);
        }
        if (record(w, j, s, take, i, msum)) break;
    }
    if (tid == 0) w.sm[j] = s;
}

// Every summary starts at S = {}: minima m0 = d(., e0), empty state.
__global__ void __launch_bounds__(kST) k_stream_init(const double* __restrict__ m0, int64_t n_pad, int32_t ns,
                                                     double* __restrict__ M, Summary* __restrict__ sm) {
    const int64_t r = int64_t(blockIdx.x) * kST + threadIdx.x;
    if (r < int64_t(ns) * n_pad) M[r] = m0[r % n_pad];
    if (r < ns) {
        Summary s;
        s.cnt = 0;
        s.t = 0;
        s.gi = 0;
        s.pad = 0;
        s.full_at = -1;
        s.fS = 0.0;
        sm[r] = s;
    }
}

// The returned summary (Sieve Streaming: the first in grid order with the
// largest f), the points examined (the stream stops once every summary is
// full), and its members and f values copied to the caller's outputs.
__global__ void __launch_bounds__(kST) k_stream_finish(const Summary* __restrict__ sm, int32_t ns, int32_t k,
                                                       int64_t n_order, const int32_t* __restrict__ sel,
                                                       const double* __restrict__ fv, int32_t* __restrict__ sel_out,
                                                       double* __restrict__ f_out, Result* __restrict__ res) {
    __shared__ int best_s, count_s;
    if (threadIdx.x == 0) {
        int best = 0;
        bool all_full = true;
        int64_t last = -1;
        for (int j = 0; j < ns; ++j) {
            if (sm[j].fS > sm[best].fS) best = j;
            if (sm[j].cnt < k)
                all_full = false;
            else if (sm[j].full_at > last)
                last = sm[j].full_at;
        }
        res->count = sm[best].cnt;
        res->best = best;
        res->examined = all_full ? last + 1 : n_order;
        best_s = best;
        count_s = sm[best].cnt;
    }
    __syncthreads();
    if (sel == sel_out) return;  // a single summary writes the outputs directly
    for (int t = threadIdx.x; t < count_s; t += kST) {
        sel_out[t] = sel[int64_t(best_s) * k + t];
        f_out[t] = fv[int64_t(best_s) * k + t];
    }
}

// The returned summary's minima into `out` (then loaded as the dataset state).
__global__ void __launch_bounds__(kST) k_stream_take_m(const double* __restrict__ M, int64_t n_pad,
                                                       const Result* __restrict__ res, double* __restrict__ out) {
    const int64_t r = int64_t(blockIdx.x) * kST + threadIdx.x;
    if (r < n_pad) out[r] = M[int64_t(res->best) * n_pad + r];
}

// The returned summary's members marked selected in the dataset state.
__global__ void __launch_bounds__(kST) k_stream_mark(const int32_t* __restrict__ sel, const Result* __restrict__ res,
                                                     uint8_t* __restrict__ selected) {
    for (int t = threadIdx.x; t < res->count; t += kST) selected[sel[t]] = 1;
}

// ---- host side ----

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

// Most guesses (1+eps)^i in [m, k m] for any m > 0: floor(log k / log(1+eps)) + 1,
// plus one for rounding in the logarithms that place the grid ends.
int64_t max_guesses(int32_t k, double eps) { return int64_t(floor(log(double(k)) / log1p(eps))) + 2; }

bool valid_n(int64_t n) { return n >= 1 && n < (int64_t(1) << 31) - kRowAlign; }

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

// Stream points per stretch: `batch`, or by default as many as keep the
// stretch's distance rows within kStretchBytes (32 .. 1024); never more than
// the stream.
int32_t stretch_len(int64_t n_pad, int64_t n_order, int32_t batch) {
    int64_t b = batch;
    if (b == 0) b = std::min<int64_t>(1024, std::max<int64_t>(32, int64_t(kStretchBytes / (8 * size_t(n_pad)))));
    return int32_t(std::max<int64_t>(1, std::min<int64_t>(b, n_order)));
}

// Scratch of one call with `ns` summaries (1 for Three Sieves) and J guesses.
struct StreamLayout {
    size_t d, m, sel, fv, sm, grid, res, total;
};

StreamLayout stream_layout(int64_t n_pad, int32_t k, int64_t ns, int64_t J, int32_t stretch) {
    StreamLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += al256(bytes);
        return at;
    };
    // the distance rows; also the returned minima at the end (n_pad <= stretch rows)
    L.d = take(size_t(std::max<int64_t>(stretch, 1)) * size_t(n_pad) * sizeof(double));
    L.m = take(size_t(ns) * size_t(n_pad) * sizeof(double));
    L.sel = take(ns > 1 ? size_t(ns) * size_t(k) * sizeof(int32_t) : 0);
    L.fv = take(ns > 1 ? size_t(ns) * size_t(k) * sizeof(double) : 0);
    L.sm = take(size_t(ns) * sizeof(Summary));
    L.grid = take(size_t(J) * sizeof(double));
    L.res = take(sizeof(Result));
    L.total = o;
    return L;
}

hipError_t read_state(const ebc_dataset* ds, DevState* st, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(st, ds->b.state, sizeof(DevState), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

// The caller's stream indices, checked on the host before any work.
ebc_status check_order(const ebc_dataset* ds, const int32_t* order, int64_t n_order, hipStream_t s) {
    if (!order || n_order == 0) return EBC_OK;
    std::vector<int32_t> h(static_cast<size_t>(n_order));
    if (hipMemcpyAsync(h.data(), order, size_t(n_order) * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return EBC_E_DEVICE;
    for (int32_t v : h)
        if (v < 0 || int64_t(v) >= ds->n) return EBC_E_INDEX;
    return EBC_OK;
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

template <int R, int P>
void launch_walk(int32_t ns, const WalkArgs& w, hipStream_t s) {
    hipLaunchKernelGGL((k_stream_walk<R, P>), dim3(unsigned(ns)), dim3(kST), 0, s, w);
}

// Both optimisers: T > 0 runs Three Sieves (one summary, the guess walking
// down after T rejections), T = 0 Sieve Streaming (one summary per guess).
ebc_status run_stream(ebc_dataset* ds, int32_t k, double eps, int64_t T, double m_max, const int32_t* order,
                      int64_t n_order, int32_t batch, int32_t* sel_out, double* f_out, int32_t* count_out,
                      double* v_out, int64_t* examined_out, void* scratch, size_t scratch_bytes, hipStream_t s) {
    if (!scratch || reinterpret_cast<uintptr_t>(scratch) % 256 != 0) return EBC_E_INVALID_ARG;
    const int32_t stretch = stretch_len(ds->n_pad, n_order, batch);
    const int64_t ns_max = T > 0 ? 1 : max_guesses(k, eps);
    if (scratch_bytes < stream_layout(ds->n_pad, k, ns_max, max_guesses(k, eps), stretch).total)
        return EBC_E_INVALID_ARG;
    ebc_status st_ = check_order(ds, order, n_order, s);
    if (st_ != EBC_OK) return st_;
    DevState st;
    if ((st_ = start_stream(ds, &m_max, sel_out, f_out, s, &st)) != EBC_OK) return st_;
    if (st.error != 0) return EBC_OK;  // reported by ebc_sync_status
    const std::vector<double> grid = sieve_grid(m_max, k, eps);
    const int64_t J = int64_t(grid.size());
    if (J == 0) return EBC_OK;
    if (J > max_guesses(k, eps)) return EBC_E_INVALID_ARG;  // not reached: the grid spans a factor k
    const int32_t ns = T > 0 ? 1 : int32_t(J);

    const StreamLayout L = stream_layout(ds->n_pad, k, ns, J, stretch);
    char* base = static_cast<char*>(scratch);
    double* D = reinterpret_cast<double*>(base + L.d);
    double* M = reinterpret_cast<double*>(base + L.m);
    int32_t* sel = ns > 1 ? reinterpret_cast<int32_t*>(base + L.sel) : sel_out;
    double* fv = ns > 1 ? reinterpret_cast<double*>(base + L.fv) : f_out;
    Summary* sm = reinterpret_cast<Summary*>(base + L.sm);
    double* d_grid = reinterpret_cast<double*>(base + L.grid);
    Result* d_res = reinterpret_cast<Result*>(base + L.res);

    if (hipMemcpyAsync(d_grid, grid.data(), size_t(J) * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return EBC_E_DEVICE;
    const int64_t init_n = std::max<int64_t>(int64_t(ns) * ds->n_pad, ns);
    hipLaunchKernelGGL(k_stream_init, dim3(unsigned((init_n + kST - 1) / kST)), dim3(kST), 0, s, ds->b.m0, ds->n_pad,
                       ns, M, sm);

    WalkArgs w;
    w.D = D;
    w.n = ds->n;
    w.n_pad = ds->n_pad;
    w.k = k;
    w.order = order;
    w.grid = d_grid;
    w.J = int32_t(J);
    w.pad = 0;
    w.T = T;
    w.dst = ds->b.state;
    w.sm = sm;
    w.M = M;
    w.sel = sel;
    w.fv = fv;
    const int64_t rpt = ds->n_pad / kST;  // ground points per thread of the walk
    for (int64_t pos = 0; pos < n_order; pos += stretch) {
        const int32_t cnt = int32_t(std::min<int64_t>(stretch, n_order - pos));
        const dim3 g(unsigned(ds->n_pad / kDV), unsigned((cnt + kDI - 1) / kDI));
        if (ds->metric == 1)
            hipLaunchKernelGGL(k_stream_dist<1>, g, dim3(kST), 0, s, ds->x, ds->n, ds->d, order, pos, cnt, ds->n_pad,
                               D, sm, ns, k);
        else
            hipLaunchKernelGGL(k_stream_dist<0>, g, dim3(kST), 0, s, ds->x, ds->n, ds->d, order, pos, cnt, ds->n_pad,
                               D, sm, ns, k);
        w.cnt = cnt;
        w.pos = pos;
        if (rpt <= 1)
            launch_walk<1, 8>(ns, w, s);
        else if (rpt <= 2)
            launch_walk<2, 8>(ns, w, s);
        else if (rpt <= 4)
            launch_walk<4, 8>(ns, w, s);
        else if (rpt <= 8)
            launch_walk<8, 4>(ns, w, s);
        else if (rpt <= kRegMax)
            launch_walk<kRegMax, 2>(ns, w, s);
        else
            hipLaunchKernelGGL(k_stream_walk_big, dim3(unsigned(ns)), dim3(kST), 0, s, w);
        if (hipGetLastError() != hipSuccess) return EBC_E_DEVICE;
    }
    hipLaunchKernelGGL(k_stream_finish, dim3(1), dim3(kST), 0, s, sm, ns, k, n_order, sel, fv, sel_out, f_out, d_res);
    // the dataset state afterwards: the returned summary's minima and members
    hipLaunchKernelGGL(k_stream_take_m, dim3(unsigned(ds->n_pad / kST)), dim3(kST), 0, s, M, ds->n_pad, d_res, D);
    if (launch_load_m(ds, D, s) != hipSuccess) return EBC_E_DEVICE;
    hipLaunchKernelGGL(k_stream_mark, dim3(1), dim3(kST), 0, s, sel_out, d_res, ds->b.selected);
    Result res;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&res, d_res, sizeof(Result), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return EBC_E_DEVICE;
    *count_out = res.count;
    if (v_out) *v_out = T > 0 ? 0.0 : grid[size_t(res.best)];
    if (examined_out) *examined_out = res.examined;
    ds->stats.steps = res.count;
    return EBC_OK;
}

}  // namespace

extern "C" {

size_t ebc_three_sieves_bytes(int64_t n, int32_t k, double eps, int64_t n_order, int32_t batch) {
    if (!valid_n(n) || k < 1 || int64_t(k) > n || !(eps > 0.0) || n_order < 0 || batch < 0) return 0;
    const int64_t np = pad_rows(n);
    return stream_layout(np, k, 1, max_guesses(k, eps), stretch_len(np, n_order, batch)).total;
}

ebc_status ebc_three_sieves(ebc_dataset* ds, int32_t k, double eps, int64_t T, double m_max, const int32_t* order,
                            int64_t n_order, int32_t batch, int32_t* sel_out, double* f_out, int32_t* count_out,
                            int64_t* examined_out, void* scratch, size_t scratch_bytes, void* stream) {
    if (!ds || !count_out || k < 1 || int64_t(k) > ds->n || !(eps > 0.0) || T < 1 || batch < 0) return EBC_E_INVALID_ARG;
    if (!sel_out || !f_out || n_order < 0 || (!order && n_order > ds->n)) return EBC_E_INVALID_ARG;
    *count_out = 0;
    if (examined_out) *examined_out = 0;
    return run_stream(ds, k, eps, T, m_max, order, n_order, batch, sel_out, f_out, count_out, nullptr, examined_out,
                      scratch, scratch_bytes, reinterpret_cast<hipStream_t>(stream));
}

size_t ebc_sieve_streaming_bytes(int64_t n, int32_t k, double eps, int64_t n_order, int32_t batch) {
    if (!valid_n(n) || k < 1 || int64_t(k) > n || !(eps > 0.0) || n_order < 0 || batch < 0) return 0;
    const int64_t np = pad_rows(n);
    const int64_t J = max_guesses(k, eps);
    return stream_layout(np, k, J, J, stretch_len(np, n_order, batch)).total;
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
    return run_stream(ds, k, eps, 0, m_max, order, n_order, batch, sel_out, f_out, count_out, v_out, examined_out,
                      scratch, scratch_bytes, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
