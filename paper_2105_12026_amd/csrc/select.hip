// One greedy step after the gains kernel (Sec. 3 and Sec. 4.1: greedy picks
// the not-yet-selected point of largest marginal gain). Each stage is a
// device function of (instance descriptor, step, block); the solo kernels
// run it on one instance, the batched kernels map their blocks onto many.
//   k_gsum     sum the per-chunk gain sums, mask selected points, block maxima
//   k_wcount   every candidate within tau*|best| of the best enters the window
//   k_wselect  choose at most kWindowMax window candidates, deterministically
//   k_rescore  float64 direct-difference gains of the window candidates
//   k_pick     best float64 gain, ties to the lowest index; record the pick
//   k_update   m_v <- min(m_v, d(v, c*)) in float64, per-block sums of m_v
//   k_fsum     f(S_t) = L({e0}) - |V|^-1 sum_v m_v  (Alg. 1: sum, then / |V|)
// No step reads anything back to the host; all sums run in a fixed order.
#include <math.h>

#include "ebc_internal.h"
#include "quant.h"

namespace ebc {

__device__ inline bool better(double ga, int ia, double gb, int ib) {
    return ga > gb || (ga == gb && ia < ib);
}

// Threshold of the re-score window from the global best float32 gain.
__device__ double window_threshold(double gmax, const DevState* st) {
    return gmax - (st->tau * fabs(gmax) + st->tau_abs * st->nmax);
}

// Block-wide maximum of bmax[0..nb) (every block computes the same value).
__device__ double block_gmax(const double* bmax, int nb, double* red) {
    double m = -INFINITY;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, bmax[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// ---- gsum: per-chunk sums -> gsum, selected masked, block maxima ----
__device__ void gsum_body(const InstDesc& c, int64_t blk) {
    __shared__ double sg[kBlock];
    __shared__ int si[kBlock];
    const Buffers& b = c.b;
    const int64_t i = blk * kBlock + threadIdx.x;
    double g = 0.0;
    for (int s = 0; s < c.v_splits; ++s) g += b.part[int64_t(s) * c.n_pad + i];
    if (b.selected[i]) g = -INFINITY;
    b.gsum[i] = g;
    sg[threadIdx.x] = g;
    si[threadIdx.x] = int(i);
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w && better(sg[threadIdx.x + w], si[threadIdx.x + w], sg[threadIdx.x], si[threadIdx.x])) {
            sg[threadIdx.x] = sg[threadIdx.x + w];
            si[threadIdx.x] = si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        b.bmax[blk] = sg[0];
        b.barg[blk] = si[0];
    }
}

// ---- wcount: candidates within the window, compacted per block in index order ----
__device__ void wcount_body(const InstDesc& c, int64_t blk) {
    __shared__ double red[kBlock];
    __shared__ int scan[kBlock];
    const Buffers& b = c.b;
    const double gmax = block_gmax(b.bmax, c.nb, red);
    const double thr = window_threshold(gmax, b.state);
    const int64_t i = blk * kBlock + threadIdx.x;
    const double g = b.gsum[i];
    const int q = (g >= thr && g > -INFINITY) ? 1 : 0;
    // inclusive scan of q across the block (Hillis-Steele), index order kept
    scan[threadIdx.x] = q;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const int add = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += add;
        __syncthreads();
    }
    if (q) {
        WindowEntry e;
        e.g = g;
        e.idx = int(i);
        e.pad = 0;
        b.wstage[blk * kBlock + scan[threadIdx.x] - 1] = e;
    }
    if (threadIdx.x == kBlock - 1) b.bcnt[blk] = scan[kBlock - 1];
}

// ---- wselect (one block of 1024 threads per instance) ----
// Gather the window entries in index order, then keep at most kWindowMax:
//   total <= kWindowMax          all of them;
//   total <= kWindowCap          the kWindowMax best by (gain desc, index asc);
//   otherwise (counted overflow) the best one plus the lowest-index others.
constexpr int kSelThreads = 1024;
__device__ void wselect_body(const InstDesc& c) {
    __shared__ WindowEntry list[kWindowCap];
    __shared__ int scan[kSelThreads];
    __shared__ double red[kSelThreads];
    const Buffers& b = c.b;
    const int nb = c.nb;
    const int tid = threadIdx.x;
    int total = 0;
    for (int base = 0; base < nb; base += kSelThreads) {
        const int blk = base + tid;
        const int cnt = blk < nb ? b.bcnt[blk] : 0;
        scan[tid] = cnt;
        __syncthreads();
        for (int off = 1; off < kSelThreads; off <<= 1) {
            const int add = tid >= off ? scan[tid - off] : 0;
            __syncthreads();
            scan[tid] += add;
            __syncthreads();
        }
        const int excl = total + scan[tid] - cnt;
        for (int i = 0; i < cnt; ++i) {
            const int pos = excl + i;
            if (pos < kWindowCap) list[pos] = b.wstage[int64_t(blk) * kBlock + i];
        }
        total += scan[kSelThreads - 1];
        __syncthreads();
    }
    const int nl = total < kWindowCap ? total : kWindowCap;
    if (total <= kWindowMax) {
        if (tid < total) b.wfinal[tid] = list[tid];
    } else if (total <= kWindowCap) {
        for (int i = tid; i < nl; i += kSelThreads) {
            int rank = 0;
            for (int j = 0; j < nl; ++j)
                rank += better(list[j].g, list[j].idx, list[i].g, list[i].idx) ? 1 : 0;
            if (rank < kWindowMax) b.wfinal[rank] = list[i];
        }
    } else {
        // overflow: the global best float32 candidate first ...
        const double gmax = block_gmax(b.bmax, nb, red);
        if (tid == 0) {
            int first = -1;
            for (int i = 0; i < nb && first < 0; ++i)
                if (b.bmax[i] == gmax) first = b.barg[i];
            WindowEntry e;
            e.g = gmax;
            e.idx = first;
            e.pad = 0;
            b.wfinal[0] = e;
            int w = 1;
            for (int i = 0; i < nl && w < kWindowMax; ++i)
                if (list[i].idx != first) b.wfinal[w++] = list[i];
        }
    }
    if (tid == 0) {
        const int W = total < kWindowMax ? total : kWindowMax;
        b.state->window_count = W;
        if (total > b.state->window_max) b.state->window_max = total;
        if (total > kWindowCap) b.state->window_overflow += 1;
    }
}

// ---- rescore: float64 direct-difference gains of the window candidates ----
// One thread per ground point, from the caller's float32 points; candidates
// in groups of 8 staged in LDS as float64, up to 128 dimensions at a time
// (longer rows take several passes, summed in dimension order); each thread
// reads its own row in 16-byte pieces when rows are 16-byte aligned, four
// pieces in flight (the other lanes' pieces of the same cache lines follow
// in the next iterations); per-block sums in a fixed order.
constexpr int kRescoreGroup = 8;
constexpr int kRescoreChunk = 128;

// One dimension's term for the NJ staged candidates (stride kRescoreChunk):
// squared difference (METRIC 0) or absolute difference (METRIC 1).
template <int METRIC, int NJ>
__device__ __forceinline__ void dim_terms(double xk, const double* __restrict__ cxk, double (&acc)[NJ]) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const double t = xk - cxk[j * kRescoreChunk];
        if (METRIC == 1)
            acc[j] += fabs(t);
        else
            acc[j] = fma(t, t, acc[j]);
    }
}

// acc[j] += sum over k < kn, in k order, of the terms between row piece xv
// (float32, global) and the staged candidates cx[j][0..kn).
template <int METRIC, int NJ>
__device__ __forceinline__ void row_terms(const float* __restrict__ xv, bool vec, int kn,
                                          const double* __restrict__ cx, double (&acc)[NJ]) {
    int k = 0;
    if (vec) {
        const float4* __restrict__ x4 = reinterpret_cast<const float4*>(xv);
        for (; k + 16 <= kn; k += 16) {
            float4 q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = x4[k / 4 + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                dim_terms<METRIC, NJ>(double(q[u].x), cx + k + 4 * u, acc);
                dim_terms<METRIC, NJ>(double(q[u].y), cx + k + 4 * u + 1, acc);
                dim_terms<METRIC, NJ>(double(q[u].z), cx + k + 4 * u + 2, acc);
                dim_terms<METRIC, NJ>(double(q[u].w), cx + k + 4 * u + 3, acc);
            }
        }
        for (; k + 4 <= kn; k += 4) {
            const float4 q = x4[k / 4];
            dim_terms<METRIC, NJ>(double(q.x), cx + k, acc);
            dim_terms<METRIC, NJ>(double(q.y), cx + k + 1, acc);
            dim_terms<METRIC, NJ>(double(q.z), cx + k + 2, acc);
            dim_terms<METRIC, NJ>(double(q.w), cx + k + 3, acc);
        }
    }
    for (; k < kn; ++k) dim_terms<METRIC, NJ>(double(xv[k]), cx + k, acc);
}

// METRIC 0: squared Euclidean (the paper's d); 1: L1, sum of |x_vk - x_ck|.
template <int METRIC>
__device__ void rescore_impl(const InstDesc& c, int64_t blk, double* __restrict__ cx, double (*red)[kBlock]) {
    const Buffers& b = c.b;
    const float* __restrict__ x = c.x;
    const int d = c.d;
    const int W = b.state->window_count;
    const int64_t v = blk * kBlock + threadIdx.x;
    const bool live = v < c.n;
    const double mv = live ? b.m64[v] : 0.0;
    const float* __restrict__ xv = x + (live ? v : 0) * d;
    const bool vec = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    for (int g0 = 0; g0 < W; g0 += kRescoreGroup) {
        const int gn = (W - g0) < kRescoreGroup ? (W - g0) : kRescoreGroup;
        double acc[kRescoreGroup];
#pragma unroll
        for (int j = 0; j < kRescoreGroup; ++j) acc[j] = 0.0;
        for (int k0 = 0; k0 < d; k0 += kRescoreChunk) {
            const int kn = (d - k0) < kRescoreChunk ? (d - k0) : kRescoreChunk;
            __syncthreads();
            for (int e = threadIdx.x; e < kRescoreGroup * kn; e += kBlock) {
                const int j = e / kn, k = e % kn;
                // rows past the group's end repeat its first candidate (their sums are not used)
                cx[j * kRescoreChunk + k] = double(x[int64_t(b.wfinal[g0 + (j < gn ? j : 0)].idx) * d + k0 + k]);
            }
            __syncthreads();
            if (live) row_terms<METRIC, kRescoreGroup>(xv + k0, vec, kn, cx, acc);
        }
#pragma unroll
        for (int j = 0; j < kRescoreGroup; ++j) red[j][threadIdx.x] = live ? fmax(0.0, mv - acc[j]) : 0.0;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
#pragma unroll
                for (int j = 0; j < kRescoreGroup; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x < gn) b.rpart[blk * kWindowMax + g0 + threadIdx.x] = red[threadIdx.x][0];
    }
}

__device__ void rescore_body(const InstDesc& c, int64_t blk) {
    __shared__ double cx[kRescoreGroup * kRescoreChunk];
    __shared__ double red[kRescoreGroup][kBlock];
    if (c.metric == 1)
        rescore_impl<1>(c, blk, cx, red);
    else
        rescore_impl<0>(c, blk, cx, red);
}

__device__ __forceinline__ int rescore_rows(const InstDesc& c, int W);

// ---- pick (one block per instance) ----
// float64 gain of each window candidate = sum of the per-block sums: up to
// kPickColumnRows of them, thread j adds candidate j's in block order;
// otherwise, candidate by candidate, thread i takes blocks i, i+256, ...,
// then a fixed tree. Best gain wins, ties to the lowest index. Records the
// pick. A step with no valid candidate (only possible with non-finite input)
// records -1 and flags it.
constexpr int kPickColumnRows = 64;

__device__ void pick_body(const InstDesc& c, int32_t t) {
    __shared__ double red[kBlock];
    __shared__ double sg[kWindowMax];
    __shared__ int si[kWindowMax];
    const Buffers& b = c.b;
    const int W = b.state->window_count;
    const int nbv = rescore_rows(c, W);
    if (nbv <= kPickColumnRows) {
        for (int j = threadIdx.x; j < kWindowMax; j += kBlock) {
            double s = 0.0;
            if (j < W)
                for (int blk = 0; blk < nbv; ++blk) s += b.rpart[int64_t(blk) * kWindowMax + j];
            sg[j] = j < W ? s : -INFINITY;
            si[j] = j < W ? b.wfinal[j].idx : 0x7fffffff;
        }
    }
    for (int j = 0; j < kWindowMax && nbv > kPickColumnRows; ++j) {
        double s = 0.0;
        if (j < W)
            for (int blk = threadIdx.x; blk < nbv; blk += kBlock) s += b.rpart[int64_t(blk) * kWindowMax + j];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            sg[j] = j < W ? red[0] : -INFINITY;
            si[j] = j < W ? b.wfinal[j].idx : 0x7fffffff;
        }
        __syncthreads();
        if (j + 1 >= W) break;
    }
    if (nbv > kPickColumnRows) {
        for (int j = W + threadIdx.x; j < kWindowMax; j += kBlock) {
            sg[j] = -INFINITY;
            si[j] = 0x7fffffff;
        }
    }
    __syncthreads();
    const int j = threadIdx.x;
    for (int w = kWindowMax / 2; w > 0; w >>= 1) {
        if (j < w && better(sg[j + w], si[j + w], sg[j], si[j])) {
            sg[j] = sg[j + w];
            si[j] = si[j + w];
        }
        __syncthreads();
    }
    if (W > 0 && sg[0] == 0.0) {
        // The best float64 gain of the window is 0: every point is covered, so
        // every unselected point has gain 0 and the pick is the lowest
        // unselected index (also when more zero-gain candidates than the
        // window holds were ranked by their reduced-precision gains).
        __shared__ int lowest[kBlock];
        int lo = 0x7fffffff;
        for (int64_t i = threadIdx.x; i < c.n; i += kBlock)
            if (!b.selected[i]) {
                lo = int(i);
                break;
            }
        lowest[j] = lo;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (j < w && lowest[j + w] < lowest[j]) lowest[j] = lowest[j + w];
            __syncthreads();
        }
        if (j == 0 && lowest[0] != 0x7fffffff) si[0] = lowest[0];
        __syncthreads();
    }
    if (j == 0) {
        const int cs = si[0];
        if (W > 0 && cs >= 0 && int64_t(cs) < c.n) {
            b.state->cstar = cs;
            b.state->gstar = sg[0];
            b.selected[cs] = 1;
            c.sel[t] = cs;
            if (c.gain) c.gain[t] = sg[0] / double(c.n);
        } else {
            b.state->cstar = -1;
            atomicCAS(&b.state->error, 0, kDevErrNonFinite);
            c.sel[t] = -1;
            if (c.gain) c.gain[t] = NAN;
        }
    }
}

// ---- update: m_v <- min(m_v, d(v, c*)) in float64, per-block sums of m_v ----
__device__ void update_body(const InstDesc& c, int64_t blk) {
    static_assert(kNarrowMaxK <= kRescoreChunk, "short rows fit one staged piece");
    __shared__ double cx[kRescoreChunk];
    __shared__ double red[kBlock];
    const Buffers& b = c.b;
    const float* __restrict__ x = c.x;
    const int d = c.d;
    const int cs = b.state->cstar;
    if (cs >= 0)
        for (int k = threadIdx.x; k < d; k += kBlock) cx[k] = double(x[int64_t(cs) * d + k]);
    __syncthreads();
    const int64_t v = blk * kBlock + threadIdx.x;
    double mv = 0.0;
    if (v < c.n && cs < 0) {
        mv = b.m64[v];
    } else if (v < c.n) {
        const bool vec = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
        double acc[1] = {0.0};
        row_terms<0, 1>(x + v * d, vec, d, cx, acc);
        mv = b.m64[v];
        if (acc[0] < mv) {
            mv = acc[0];
            b.m64[v] = mv;
            set_point_terms(b, v, mv);
        }
    }
    red[threadIdx.x] = mv;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) b.fpart[blk] = red[0];
}

// ---- L1 update (any row length): m_v <- min(m_v, sum_k |x_vk - x_c*k|) in
// float64, the new member's values staged in LDS 128 at a time; per-block
// sums of m_v as in update_body ----
__device__ void update_l1_body(const InstDesc& c, int64_t blk) {
    __shared__ float cx[kRescoreChunk];
    __shared__ double red[kBlock];
    const Buffers& b = c.b;
    const float* __restrict__ x = c.x;
    const int d = c.d;
    const int cs = b.state->cstar;
    const int64_t v = blk * kBlock + threadIdx.x;
    const bool live = v < c.n;
    const float* xv = x + (live ? v : 0) * d;
    double acc = 0.0;
    for (int k0 = 0; k0 < d && cs >= 0; k0 += kRescoreChunk) {
        const int kn = (d - k0) < kRescoreChunk ? (d - k0) : kRescoreChunk;
        __syncthreads();
        for (int k = threadIdx.x; k < kn; k += kBlock) cx[k] = x[int64_t(cs) * d + k0 + k];
        __syncthreads();
        if (live)
            for (int k = 0; k < kn; ++k) acc += fabs(double(xv[k0 + k]) - double(cx[k]));
    }
    double mv = 0.0;
    if (live) {
        mv = b.m64[v];
        if (cs >= 0 && acc < mv) {
            mv = acc;
            b.m64[v] = mv;
            set_point_terms(b, v, mv);
        }
    }
    red[threadIdx.x] = mv;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) b.fpart[blk] = red[0];
}

// ---- long rows (padded length above 128): re-score and update ----
// One thread per ground point, as for short rows, reading its own row in
// 16-byte pieces when the rows are 16-byte aligned (the other lanes' pieces of the
// same cache lines follow in the next iterations); the candidates' values
// are staged in LDS 512 dimensions at a time. Every per-thread float64 sum
// runs in dimension order, as for short rows.
constexpr int kLongChunk = 512;

template <int NJ>
__device__ __forceinline__ void long_sums(const InstDesc& c, int64_t v, bool live, const int64_t (&cand)[kRescoreGroup],
                                          int nc, float (&cx)[kRescoreGroup][kLongChunk], double (&acc)[NJ]) {
    const float* __restrict__ x = c.x;
    const int d = c.d;
    const float* __restrict__ xv = x + (live ? v : 0) * d;
    const bool vec = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
#pragma unroll
    for (int q = 0; q < NJ; ++q) acc[q] = 0.0;
    for (int k0 = 0; k0 < d; k0 += kLongChunk) {
        const int kn = (d - k0) < kLongChunk ? (d - k0) : kLongChunk;
        __syncthreads();  // the previous piece of cx is no longer read
        for (int e = threadIdx.x; e < nc * kLongChunk; e += kBlock) {
            const int q = e / kLongChunk, k = e % kLongChunk;
            cx[q][k] = k < kn ? x[cand[q] * d + k0 + k] : 0.0f;
        }
        __syncthreads();
        if (!live) continue;
        if (vec) {
            const float4* __restrict__ x4 = reinterpret_cast<const float4*>(xv + k0);
#pragma unroll 4
            for (int k4 = 0; k4 < kn / 4; ++k4) {
                const float4 a = x4[k4];
                const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double xk = double(av[i]);
#pragma unroll
                    for (int q = 0; q < NJ; ++q) {
                        const double t = xk - double(cx[q][4 * k4 + i]);
                        acc[q] = fma(t, t, acc[q]);
                    }
                }
            }
        } else {
            for (int k = 0; k < kn; ++k) {
                const double xk = double(xv[k0 + k]);
#pragma unroll
                for (int q = 0; q < NJ; ++q) {
                    const double t = xk - double(cx[q][k]);
                    acc[q] = fma(t, t, acc[q]);
                }
            }
        }
    }
}

__host__ __device__ inline int split_window(const InstDesc& c);
__device__ __forceinline__ int long_quarter(int d);
__device__ void rescore_split_sum(const InstDesc& c, int64_t blk, double (*red)[kBlock]);

// One-pass re-score of long rows (windows above the two-pass size). A
// workgroup takes 64 ground points (sub-block s of row block blk) and group
// g of the window, blockIdx.y = 4 g + s; the window is cut into at most 32
// groups of 1, 2, 4 or 8 candidates (the smallest size that fits), so
// small windows still spread over the chip. Wave w sums
// dimension quarter w; the candidates' values are staged in LDS as
// float64, 128 dimensions of every quarter at a time. The four partial sums
// are added in quarter order and the clamped terms of the 64 points summed in
// a fixed tree into rpart row 4 blk + s.
constexpr int kLongQChunk = 128;

template <int NJ>
__device__ __forceinline__ void quarter_chunk(const float* __restrict__ xv, bool vec, int k0, int kn,
                                              const double (&cq)[kRescoreGroup][kLongQChunk],
                                              double (&acc)[kRescoreGroup]) {
    constexpr int kUnroll = NJ <= 2 ? 8 : 2;  // 16-byte loads in flight per lane
    if (vec) {
        const float4* __restrict__ x4 = reinterpret_cast<const float4*>(xv + k0);
#pragma unroll kUnroll
        for (int k4 = 0; k4 < kn / 4; ++k4) {
            const float4 a = x4[k4];
            const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double xk = double(av[i]);
#pragma unroll
                for (int q = 0; q < NJ; ++q) {
                    const double t = xk - cq[q][4 * k4 + i];
                    acc[q] = fma(t, t, acc[q]);
                }
            }
        }
    } else {
        for (int k = 0; k < kn; ++k) {
            const double xk = double(xv[k0 + k]);
#pragma unroll
            for (int q = 0; q < NJ; ++q) {
                const double t = xk - cq[q][k];
                acc[q] = fma(t, t, acc[q]);
            }
        }
    }
}

__device__ void rescore_long_body(const InstDesc& c, int64_t blk, int y) {
    __shared__ double cq[4][kRescoreGroup][kLongQChunk];
    __shared__ double red[4][kRescoreGroup][64];
    __shared__ int64_t scand[kRescoreGroup];
    const Buffers& b = c.b;
    const int W = b.state->window_count;
    if (W <= split_window(c)) {
        // small windows: pass 2 of the two-pass re-score, on the blocks of y = 0
        // (same for the whole block), in the LDS of cq
        if (y == 0) rescore_split_sum(c, blk, reinterpret_cast<double (*)[kBlock]>(&cq[0][0][0]));
        return;
    }
    const int gsz = W <= 32 ? 1 : (W <= 64 ? 2 : (W <= 128 ? 4 : kRescoreGroup));
    const int g0 = (y / 4) * gsz, sub = y % 4;
    if (g0 >= W) return;  // the same for the whole block
    const int gn = (W - g0) < gsz ? (W - g0) : gsz;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t v = blk * kBlock + sub * 64 + lane;
    const bool live = v < c.n;
    const float* __restrict__ x = c.x;
    const int d = c.d;
    const int Q = long_quarter(d);
    const int qb = w * Q;
    const int qe = (qb + Q) < d ? (qb + Q) : d;
    const float* __restrict__ xv = x + (live ? v : 0) * d;
    const bool vec = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    if (threadIdx.x < kRescoreGroup) scand[threadIdx.x] = threadIdx.x < gn ? int64_t(b.wfinal[g0 + threadIdx.x].idx) : 0;
    double acc[kRescoreGroup];
#pragma unroll
    for (int q = 0; q < kRescoreGroup; ++q) acc[q] = 0.0;
    for (int t0 = 0; t0 < Q; t0 += kLongQChunk) {
        __syncthreads();  // scand is written; the previous piece of cq is no longer read
        for (int e = threadIdx.x; e < 4 * gn * kLongQChunk; e += kBlock) {
            const int qq = e / (gn * kLongQChunk);
            const int q = (e / kLongQChunk) % gn, k = e % kLongQChunk;
            const int kk = qq * Q + t0 + k;
            const int ke = (qq * Q + Q) < d ? (qq * Q + Q) : d;
            cq[qq][q][k] = kk < ke ? double(x[scand[q] * d + kk]) : 0.0;
        }
        __syncthreads();
        const int rest = qe - (qb + t0);
        const int kn = rest < kLongQChunk ? rest : kLongQChunk;
        if (!live || kn <= 0) continue;
        if (gn == 1)
            quarter_chunk<1>(xv, vec, qb + t0, kn, cq[w], acc);
        else if (gn == 2)
            quarter_chunk<2>(xv, vec, qb + t0, kn, cq[w], acc);
        else if (gn <= 4)
            quarter_chunk<4>(xv, vec, qb + t0, kn, cq[w], acc);
        else
            quarter_chunk<kRescoreGroup>(xv, vec, qb + t0, kn, cq[w], acc);
    }
#pragma unroll
    for (int q = 0; q < kRescoreGroup; ++q) red[w][q][lane] = acc[q];
    __syncthreads();
    const double mv = live ? b.m64[v] : 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = w + 4 * h;
        double val = 0.0;
        if (live && q < gn) {
            const double dist = ((red[0][q][lane] + red[1][q][lane]) + red[2][q][lane]) + red[3][q][lane];
            val = fmax(0.0, mv - dist);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) val += __shfl_xor(val, off, 64);
        if (lane == 0 && q < gn) b.rpart[(4 * blk + sub) * kWindowMax + g0 + q] = val;
    }
}

__device__ void update_long_body(const InstDesc& c, int64_t blk) {
    __shared__ float cx[kRescoreGroup][kLongChunk];
    __shared__ double red[kBlock];
    const Buffers& b = c.b;
    const int cs = b.state->cstar;
    const int64_t v = blk * kBlock + threadIdx.x;
    double dist[1] = {0.0};
    if (cs >= 0) {
        int64_t cand[kRescoreGroup];
#pragma unroll
        for (int q = 0; q < kRescoreGroup; ++q) cand[q] = cs;
        long_sums<1>(c, v, v < c.n, cand, 1, cx, dist);
    }
    double mv = 0.0;
    if (v < c.n) {
        mv = b.m64[v];
        if (cs >= 0 && dist[0] < mv) {
            mv = dist[0];
            b.m64[v] = mv;
            set_point_terms(b, v, mv);
        }
    }
    red[threadIdx.x] = mv;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) b.fpart[blk] = red[0];
}

// Long rows with at least 4 ground-set chunks (small ground sets): the
// float64 squared distance of every point to one row in two passes, so the
// update and small re-score windows use more workgroups. Pass 1
// (blockIdx.y = slice q of the dimension, 16-byte reads as above) writes
// each point's partial sum to the per-chunk gains buffer, free at that point
// of a step, at part[q * n_pad + v]. Pass 2 adds the slices in order. The
// update takes one slice per chunk (up to 16); small re-score windows share
// the chunks among their candidates.
// Long rows take the long-row re-score and update kernels under the squared
// distance; L1 datasets take the generic ones (any row length) at every d.
__host__ __device__ inline bool long_path(const InstDesc& c) { return wide_rows(c.k_pad) && c.metric == 0; }
__host__ __device__ inline bool long_split(const InstDesc& c) { return long_path(c) && c.v_splits >= 4; }
__host__ __device__ inline int update_slices(const InstDesc& c) { return c.v_splits < 16 ? c.v_splits : 16; }
__device__ __forceinline__ int long_slice(int d, int S) { return ((d + S - 1) / S + 3) / 4 * 4; }
__device__ __forceinline__ int long_quarter(int d) { return long_slice(d, 4); }

__device__ void dist_slice_body(const InstDesc& c, int64_t blk, int q, int S, int64_t row) {
    if (row < 0 || q >= S) return;
    const float* __restrict__ x = c.x;
    const int d = c.d;
    const int Q = long_slice(d, S);
    const int k0 = q * Q;
    const int k1 = (k0 + Q) < d ? (k0 + Q) : d;
    const int64_t v = blk * kBlock + threadIdx.x;
    if (v >= c.n) return;
    const float* __restrict__ xv = x + v * d;
    const float* __restrict__ xc = x + row * d;
    double acc = 0.0;
    if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
        const float4* __restrict__ a4 = reinterpret_cast<const float4*>(xv);
        const float4* __restrict__ c4 = reinterpret_cast<const float4*>(xc);
#pragma unroll 4
        for (int k4 = k0 / 4; k4 < k1 / 4; ++k4) {
            const float4 a = a4[k4], b = c4[k4];
            const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double t = double(av[i]) - double(bv[i]);
                acc = fma(t, t, acc);
            }
        }
    } else {
        for (int k = k0; k < k1; ++k) {
            const double t = double(xv[k]) - double(xc[k]);
            acc = fma(t, t, acc);
        }
    }
    c.b.part[int64_t(q) * c.n_pad + v] = acc;
}

__device__ __forceinline__ double slices_sum(const InstDesc& c, int64_t v, int S) {
    const double* __restrict__ p = c.b.part;
    double s = p[v];
    for (int q = 1; q < S; ++q) s += p[int64_t(q) * c.n_pad + v];
    return s;
}

// m_v update from the slice sums (pass 2), per-block sums of m_v
__device__ void update_split_body(const InstDesc& c, int64_t blk) {
    __shared__ double red[kBlock];
    const Buffers& b = c.b;
    const int cs = b.state->cstar;
    const int64_t v = blk * kBlock + threadIdx.x;
    double mv = 0.0;
    if (v < c.n) {
        mv = b.m64[v];
        if (cs >= 0) {
            const double dist = slices_sum(c, v, update_slices(c));
            if (dist < mv) {
                mv = dist;
                b.m64[v] = mv;
                set_point_terms(b, v, mv);
            }
        }
    }
    red[threadIdx.x] = mv;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) b.fpart[blk] = red[0];
}

// Small re-score windows of long rows (at most v_splits/4, and 4,
// candidates): the same two passes per candidate, each candidate's distances
// over S = min(16, v_splits / W) slices; pass 1 over (candidate, slice) on
// blockIdx.y writing part[(S j + q) * n_pad + v].
__host__ __device__ inline int split_window(const InstDesc& c) {
    return long_split(c) ? (c.v_splits / 4 < 4 ? c.v_splits / 4 : 4) : 0;
}
__device__ __forceinline__ int window_slices(const InstDesc& c, int W) {
    const int s = c.v_splits / W;
    return s < 16 ? s : 16;
}

// rpart rows a re-score of W candidates fills: one per 64-point sub-block
// for the one-pass long-row re-score, one per row block otherwise
__device__ __forceinline__ int rescore_rows(const InstDesc& c, int W) {
    return (long_path(c) && W > split_window(c)) ? 4 * c.nb : c.nb;
}

__device__ void dist_window_body(const InstDesc& c, int64_t blk, int y) {
    const int W = c.b.state->window_count;
    if (W > split_window(c)) return;  // the one-pass re-score takes it
    if (W == 0) return;
    const int S = window_slices(c, W);
    const int j = y / S, q = y % S;
    if (j >= W) return;
    // slice q of candidate j into the slot block S j + q
    InstDesc cj = c;
    cj.b.part = c.b.part + int64_t(S * j) * c.n_pad;
    dist_slice_body(cj, blk, q, S, int64_t(c.b.wfinal[j].idx));
}

__device__ void rescore_split_sum(const InstDesc& c, int64_t blk, double (*red)[kBlock]) {
    const int W = c.b.state->window_count;
    if (W > split_window(c) || W == 0) return;  // the same for the whole block
    const int64_t v = blk * kBlock + threadIdx.x;
    const double mv = v < c.n ? c.b.m64[v] : 0.0;
    const int S = window_slices(c, W);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double val = 0.0;
        if (j < W && v < c.n) {
            InstDesc cj = c;
            cj.b.part = c.b.part + int64_t(S * j) * c.n_pad;
            val = fmax(0.0, mv - slices_sum(cj, v, S));
        }
        red[j][threadIdx.x] = val;
    }
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int j = 0; j < 4; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < W) c.b.rpart[blk * kWindowMax + threadIdx.x] = red[threadIdx.x][0];
}

__device__ void rescore_split_body(const InstDesc& c, int64_t blk) {
    __shared__ double red[4][kBlock];
    rescore_split_sum(c, blk, red);
}

// ---- fsum (one block per instance): f(S_t) = L({e0}) - |V|^-1 sum m_v ----
__device__ void fsum_body(const InstDesc& c, int32_t t) {
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int i = threadIdx.x; i < c.nb; i += kBlock) s += c.b.fpart[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) c.f[t] = c.b.state->l0 - red[0] / double(c.n);
}

// ---- solo kernels ----
__global__ void __launch_bounds__(kBlock) k_gsum(InstDesc c) { gsum_body(c, blockIdx.x); }
__global__ void __launch_bounds__(kBlock) k_wcount(InstDesc c) { wcount_body(c, blockIdx.x); }
__global__ void __launch_bounds__(kSelThreads) k_wselect(InstDesc c) { wselect_body(c); }
__global__ void __launch_bounds__(kBlock) k_rescore(InstDesc c) { rescore_body(c, blockIdx.x); }
__global__ void __launch_bounds__(kBlock) k_pick(InstDesc c, int32_t t) { pick_body(c, t); }
__global__ void __launch_bounds__(kBlock) k_update(InstDesc c) { update_body(c, blockIdx.x); }
__global__ void __launch_bounds__(kBlock) k_update_l1(InstDesc c) { update_l1_body(c, blockIdx.x); }
__global__ void __launch_bounds__(kBlock) k_rescore_long(InstDesc c) { rescore_long_body(c, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(kBlock) k_update_long(InstDesc c) { update_long_body(c, blockIdx.x); }
__global__ void __launch_bounds__(kBlock) k_dist_slices(InstDesc c) {
    dist_slice_body(c, blockIdx.x, blockIdx.y, update_slices(c), int64_t(c.b.state->cstar));
}
__global__ void __launch_bounds__(kBlock) k_update_split(InstDesc c) { update_split_body(c, blockIdx.x); }
__global__ void __launch_bounds__(kBlock) k_dist_window(InstDesc c) { dist_window_body(c, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(kBlock) k_rescore_split(InstDesc c) { rescore_split_body(c, blockIdx.x); }
__global__ void __launch_bounds__(kBlock) k_fsum(InstDesc c, int32_t t) { fsum_body(c, t); }

// ---- batched kernels: blocks of row_pre[i] .. row_pre[i+1] belong to instance i;
// tick t runs step t0 + t of each instance; instances whose k is reached skip ----
#define EBC_ROW_KERNEL(NAME, BODY)                                                                     \
    __global__ void __launch_bounds__(kBlock)                                                          \
        NAME(const InstDesc* __restrict__ descs, const int64_t* __restrict__ row_pre, int32_t count,   \
             int32_t t) {                                                                              \
        const int i = find_slot(row_pre, count, blockIdx.x);                                           \
        const InstDesc c = descs[i];                                                                   \
        if (c.t0 + t >= c.k) return;                                                                   \
        BODY(c, int64_t(blockIdx.x) - row_pre[i]);                                                     \
    }
EBC_ROW_KERNEL(kb_gsum, gsum_body)
EBC_ROW_KERNEL(kb_wcount, wcount_body)
// mixed batches: each re-score / update body runs only for its own row length
__device__ __forceinline__ void rescore_short(const InstDesc& c, int64_t blk) {
    if (!wide_rows(c.k_pad)) rescore_body(c, blk);
}
__device__ __forceinline__ void update_short(const InstDesc& c, int64_t blk) {
    if (!wide_rows(c.k_pad)) update_body(c, blk);
}
__device__ __forceinline__ void rescore_long(const InstDesc& c, int64_t blk) {
    if (wide_rows(c.k_pad)) rescore_long_body(c, blk, blockIdx.y);
}
__device__ __forceinline__ void update_long(const InstDesc& c, int64_t blk) {
    if (!wide_rows(c.k_pad)) return;
    if (long_split(c))
        update_split_body(c, blk);
    else
        update_long_body(c, blk);
}
__device__ __forceinline__ void dist_slices(const InstDesc& c, int64_t blk) {
    if (long_split(c)) dist_slice_body(c, blk, blockIdx.y, update_slices(c), c.b.state->cstar);
}
__device__ __forceinline__ void dist_window(const InstDesc& c, int64_t blk) {
    if (long_split(c)) dist_window_body(c, blk, blockIdx.y);
}
EBC_ROW_KERNEL(kb_rescore, rescore_short)
EBC_ROW_KERNEL(kb_update, update_short)
EBC_ROW_KERNEL(kb_rescore_long, rescore_long)
EBC_ROW_KERNEL(kb_update_long, update_long)
EBC_ROW_KERNEL(kb_dist_slices, dist_slices)
EBC_ROW_KERNEL(kb_dist_window, dist_window)
#undef EBC_ROW_KERNEL

__global__ void __launch_bounds__(kSelThreads) kb_wselect(const InstDesc* __restrict__ descs, int32_t t) {
    const InstDesc c = descs[blockIdx.x];
    if (c.t0 + t < c.k) wselect_body(c);
}
__global__ void __launch_bounds__(kBlock) kb_pick(const InstDesc* __restrict__ descs, int32_t t) {
    const InstDesc c = descs[blockIdx.x];
    if (c.t0 + t < c.k) pick_body(c, c.t0 + t);
}
__global__ void __launch_bounds__(kBlock) kb_fsum(const InstDesc* __restrict__ descs, int32_t t) {
    const InstDesc c = descs[blockIdx.x];
    if (c.t0 + t < c.k) fsum_body(c, c.t0 + t);
}

hipError_t launch_greedy_step(const ebc_dataset* ds, int32_t t, int32_t* sel_out, double* f_out,
                              double* gain_out, hipStream_t s, hipEvent_t ev_gains_done) {
    hipError_t e = launch_gains(ds, nullptr, ds->n_pad, s);
    if (e != hipSuccess) return e;
    if (ev_gains_done && (e = hipEventRecord(ev_gains_done, s)) != hipSuccess) return e;
    InstDesc c;
    fill_desc(ds, t + 1, sel_out, f_out, gain_out, &c);
    const int nb = c.nb;
    hipLaunchKernelGGL(k_gsum, dim3(nb), dim3(kBlock), 0, s, c);
    hipLaunchKernelGGL(k_wcount, dim3(nb), dim3(kBlock), 0, s, c);
    hipLaunchKernelGGL(k_wselect, dim3(1), dim3(kSelThreads), 0, s, c);
    if (c.metric == 1) {
        hipLaunchKernelGGL(k_rescore, dim3(nb), dim3(kBlock), 0, s, c);
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(kBlock), 0, s, c, t);
        hipLaunchKernelGGL(k_update_l1, dim3(nb), dim3(kBlock), 0, s, c);
    } else if (wide_rows(c.k_pad)) {
        // small windows: pass 1 over slices of the dimension here, pass 2 inside k_rescore_long
        if (long_split(c)) hipLaunchKernelGGL(k_dist_window, dim3(nb, 16), dim3(kBlock), 0, s, c);
        hipLaunchKernelGGL(k_rescore_long, dim3(nb, 4 * kWindowMax / kRescoreGroup), dim3(kBlock), 0, s, c);
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(kBlock), 0, s, c, t);
        if (long_split(c)) {
            hipLaunchKernelGGL(k_dist_slices, dim3(nb, update_slices(c)), dim3(kBlock), 0, s, c);
            hipLaunchKernelGGL(k_update_split, dim3(nb), dim3(kBlock), 0, s, c);
        } else {
            hipLaunchKernelGGL(k_update_long, dim3(nb), dim3(kBlock), 0, s, c);
        }
    } else {
        hipLaunchKernelGGL(k_rescore, dim3(nb), dim3(kBlock), 0, s, c);
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(kBlock), 0, s, c, t);
        hipLaunchKernelGGL(k_update, dim3(nb), dim3(kBlock), 0, s, c);
    }
    hipLaunchKernelGGL(k_fsum, dim3(1), dim3(kBlock), 0, s, c, t);
    return hipGetLastError();
}

hipError_t launch_step_batched(const InstDesc* descs, const int64_t* row_pre, int32_t count, int64_t total_rows,
                               int32_t t, bool long_rows, hipStream_t s) {
    const dim3 rows = dim3(unsigned(total_rows)), one = dim3(unsigned(count));
    hipLaunchKernelGGL(kb_gsum, rows, dim3(kBlock), 0, s, descs, row_pre, count, t);
    hipLaunchKernelGGL(kb_wcount, rows, dim3(kBlock), 0, s, descs, row_pre, count, t);
    hipLaunchKernelGGL(kb_wselect, one, dim3(kSelThreads), 0, s, descs, t);
    hipLaunchKernelGGL(kb_rescore, rows, dim3(kBlock), 0, s, descs, row_pre, count, t);
    if (long_rows) {
        hipLaunchKernelGGL(kb_dist_window, dim3(unsigned(total_rows), 16), dim3(kBlock), 0, s, descs, row_pre, count,
                           t);
        hipLaunchKernelGGL(kb_rescore_long, dim3(unsigned(total_rows), 4 * kWindowMax / kRescoreGroup), dim3(kBlock), 0, s,
                           descs, row_pre, count, t);
    }
    hipLaunchKernelGGL(kb_pick, one, dim3(kBlock), 0, s, descs, t);
    hipLaunchKernelGGL(kb_update, rows, dim3(kBlock), 0, s, descs, row_pre, count, t);
    if (long_rows) {
        hipLaunchKernelGGL(kb_dist_slices, dim3(unsigned(total_rows), 16), dim3(kBlock), 0, s, descs, row_pre, count,
                           t);
        hipLaunchKernelGGL(kb_update_long, rows, dim3(kBlock), 0, s, descs, row_pre, count, t);
    }
    hipLaunchKernelGGL(kb_fsum, one, dim3(kBlock), 0, s, descs, t);
    return hipGetLastError();
}

hipError_t launch_gains(const ebc_dataset* ds, const int32_t* cand, int64_t n_cand, hipStream_t s) {
    if (ds->metric == 1) return launch_gains_l1(ds, cand, n_cand, s);
    if (wide_rows(ds->k_pad)) return launch_gains_wide(ds, cand, n_cand, s);
    return ds->dt == EBC_DT_F32 ? launch_gains_f32(ds, cand, n_cand, s) : launch_gains_lp(ds, cand, n_cand, s);
}

// Marginal-gains output: sum the per-chunk sums, divide by |V|.
__global__ void __launch_bounds__(kBlock)
k_gains_out(int64_t n, int64_t n_cand, int64_t stride, int32_t v_splits, const double* part, double* out) {
    const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= n_cand) return;
    double g = 0.0;
    for (int s = 0; s < v_splits; ++s) g += part[int64_t(s) * stride + p];
    out[p] = g / double(n);
}

hipError_t launch_gains_out(const ebc_dataset* ds, int64_t n_cand, double* out, hipStream_t s) {
    const unsigned nb = unsigned((n_cand + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_gains_out, dim3(nb), dim3(kBlock), 0, s, ds->n, n_cand, ds->n_pad, ds->v_splits,
                       ds->b.part, out);
    return hipGetLastError();
}

}  // namespace ebc
