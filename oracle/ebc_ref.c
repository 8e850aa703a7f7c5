/*
 * FP64 CPU oracle for exemplar-based clustering (EBC), plain C99 + OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path. It shares no
 * source, header or helper with the HIP library.
 *
 * These are the same definitions as oracle/ebc_oracle.py, written as loops so
 * that they finish at the benchmark sizes:
 *   - the dissimilarity d: the squared Euclidean distance of the paper's
 *     experiments (Sec. 5), or, with metric = 1, the L1 (Manhattan) distance
 *     sum_k |a_k - b_k| (Sec. 4 defines L and f for any dissimilarity);
 *     direct differences in double either way;
 *   - k-medoids loss and f(S) = L({e0}) - L(S u {e0}), the auxiliary
 *     vector e0 given as a d-vector or, when NULL, the zero vector
 *     (Sec. 4, Eqs. k_medoids_loss and exemplar_based_clustering; Alg. 1);
 *   - marginal gain Delta(c|S) = |V|^-1 sum_v max(0, m_v - d(v,c)), where
 *     m_v = min(d(v,e0), min_{s in S} d(v,s)) (Sec. 3, discrete derivative);
 *   - greedy over all not-yet-selected points (Sec. 3 and Sec. 4.1), ties to
 *     the lowest index.
 * The only parallelism is over independent candidates or sets, as in the
 * paper's multi-threaded CPU variant (Sec. 5); every sum over ground points
 * runs sequentially in index order, so results do not depend on threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double sqd(const float* a, const float* b, int d)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = (double)a[k] - (double)b[k];
        s += t * t;
    }
    return s;
}

static double sqn(const float* a, int d)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += (double)a[k] * (double)a[k];
    return s;
}

/* L1 (Manhattan) distance sum_k |a_k - b_k| */
static double l1d(const float* a, const float* b, int d)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += fabs((double)a[k] - (double)b[k]);
    return s;
}

static double l1n(const float* a, int d)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += fabs((double)a[k]);
    return s;
}

/* d(a, b): metric 0 squared Euclidean, 1 L1 */
static double dis(const float* a, const float* b, int d, int metric)
{
    return metric == 1 ? l1d(a, b, d) : sqd(a, b, d);
}

/* d(v, e0): e0 NULL is the zero vector */
static double d_e0(const float* a, const float* e0, int d, int metric)
{
    if (e0) return dis(a, e0, d, metric);
    return metric == 1 ? l1n(a, d) : sqn(a, d);
}

int ebc_ref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* m[v] = min(d(v, e0), min_{s in S} d(v, s)) for all v. */
void ebc_ref_min_dist(const float* x, int64_t n, int32_t d, const int32_t* s, int64_t ns,
                      double* m, const float* e0, int metric)
{
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
        const float* xv = x + v * d;
        double t = d_e0(xv, e0, d, metric);
        for (int64_t j = 0; j < ns; ++j) {
            double dv = dis(xv, x + (int64_t)s[j] * d, d, metric);
            if (dv < t) t = dv;
        }
        m[v] = t;
    }
}

/* out[i] = |V|^-1 sum_v max(0, m[v] - d(v, cand[i])). */
void ebc_ref_gains(const float* x, int64_t n, int32_t d, const double* m, const int32_t* cand,
                   int64_t nc, double* out, int metric)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nc; ++i) {
        const float* xc = x + (int64_t)cand[i] * d;
        double acc = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            double g = m[v] - dis(x + v * d, xc, d, metric);
            if (g > 0.0) acc += g;
        }
        out[i] = acc / (double)n;
    }
}

/* f(S_j) = L({e0}) - L(S_j u {e0}) for CSR sets; set j = idx[off[j] .. off[j+1]). */
void ebc_ref_eval_sets(const float* x, int64_t n, int32_t d, const int64_t* off,
                       const int32_t* idx, int64_t l, double* out, const float* e0, int metric)
{
    double l0 = 0.0;
    for (int64_t v = 0; v < n; ++v) l0 += d_e0(x + v * d, e0, d, metric);
    l0 /= (double)n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < l; ++j) {
        double sum = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            const float* xv = x + v * d;
            double t = d_e0(xv, e0, d, metric); /* e0 is always in the set */
            for (int64_t q = off[j]; q < off[j + 1]; ++q) {
                double dv = dis(xv, x + (int64_t)idx[q] * d, d, metric);
                if (dv < t) t = dv;
            }
            sum += t;
        }
        out[j] = l0 - sum / (double)n;
    }
}

/* Paper-style CPU baseline of the multi-set evaluation (Sec. 5 times
 * single- and multi-threaded CPU runs of Alg. 1 in single precision): float32
 * direct differences vectorised over the dimension, a float32 running
 * minimum per ground point starting at ||v||^2 (e0 = 0), float64 sums over
 * the points, sets spread over `threads` OpenMP threads. A timed baseline
 * for speed comparisons only; the float64 functions above are the
 * reference of record. */
void ebc_ref_eval_sets_f32(const float* x, int64_t n, int32_t d, const int64_t* off,
                           const int32_t* idx, int64_t l, double* out, int threads)
{
    double l0 = 0.0;
    for (int64_t v = 0; v < n; ++v) l0 += sqn(x + v * d, d);
    l0 /= (double)n;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
    for (int64_t j = 0; j < l; ++j) {
        double sum = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            const float* xv = x + v * d;
            float t = 0.0f;
#pragma omp simd reduction(+ : t)
            for (int k = 0; k < d; ++k) t += xv[k] * xv[k];
            for (int64_t q = off[j]; q < off[j + 1]; ++q) {
                const float* xs = x + (int64_t)idx[q] * d;
                float dv = 0.0f;
#pragma omp simd reduction(+ : dv)
                for (int k = 0; k < d; ++k) {
                    const float u = xv[k] - xs[k];
                    dv += u * u;
                }
                if (dv < t) t = dv;
            }
            sum += (double)t;
        }
        out[j] = l0 - sum / (double)n;
    }
}

/* Paper-style CPU baseline of the marginal gains (timing only, like
 * ebc_ref_eval_sets_f32): float32 direct differences vectorised over the
 * dimension, float64 sums over the points, candidates over `threads`
 * OpenMP threads; out[i] = |V|^-1 sum_v max(0, m[v] - d(v, cand[i])). */
void ebc_ref_gains_f32(const float* x, int64_t n, int32_t d, const double* m, const int32_t* cand,
                       int64_t nc, double* out, int threads)
{
#pragma omp parallel for schedule(dynamic, 4) num_threads(threads)
    for (int64_t i = 0; i < nc; ++i) {
        const float* xc = x + (int64_t)cand[i] * d;
        double acc = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            const float* xv = x + v * d;
            float dv = 0.0f;
#pragma omp simd reduction(+ : dv)
            for (int k = 0; k < d; ++k) {
                const float u = xv[k] - xc[k];
                dv += u * u;
            }
            const double g = m[v] - (double)dv;
            if (g > 0.0) acc += g;
        }
        out[i] = acc / (double)n;
    }
}

/* Greedy to cardinality k. sel[t], f[t] = f(S_{t+1}), g[t] = gain of step t.
 * Returns 0, -1 if memory runs out, -2 if k > n. */
int ebc_ref_greedy(const float* x, int64_t n, int32_t d, int32_t k, int32_t* sel, double* f,
                   double* g, const float* e0, int metric)
{
    double* m = (double*)malloc(sizeof(double) * (size_t)n);
    double* gv = (double*)malloc(sizeof(double) * (size_t)n);
    unsigned char* chosen = (unsigned char*)calloc((size_t)n, 1);
    if (!m || !gv || !chosen) {
        free(m); free(gv); free(chosen);
        return -1;
    }
    double l0 = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        m[v] = d_e0(x + v * d, e0, d, metric);
        l0 += m[v];
    }
    l0 /= (double)n;
    for (int32_t t = 0; t < k; ++t) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t c = 0; c < n; ++c) {
            if (chosen[c]) { gv[c] = -INFINITY; continue; }
            const float* xc = x + c * d;
            double acc = 0.0;
            for (int64_t v = 0; v < n; ++v) {
                double q = m[v] - dis(x + v * d, xc, d, metric);
                if (q > 0.0) acc += q;
            }
            gv[c] = acc / (double)n;
        }
        int64_t best = -1;
        for (int64_t c = 0; c < n; ++c)
            if (!chosen[c] && (best < 0 || gv[c] > gv[best])) best = c;
        if (best < 0) { free(m); free(gv); free(chosen); return -2; }
        chosen[best] = 1;
        sel[t] = (int32_t)best;
        g[t] = gv[best];
        double sum = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            double dv = dis(x + v * d, x + best * d, d, metric);
            if (dv < m[v]) m[v] = dv;
            sum += m[v];
        }
        f[t] = l0 - sum / (double)n;
    }
    free(m); free(gv); free(chosen);
    return 0;
}

/* ---- Lazy evaluation of the same greedy (Minoux's accelerated greedy) ----
 * Same selections, f and gains as ebc_ref_greedy, computed by the same gain
 * routine on the same m (so every gain value is bitwise the one the plain
 * loop computes), but a candidate is re-evaluated only while its last gain,
 * an upper bound of its current gain by submodularity, could still beat the
 * best current gain. Stale bounds within a relative 1e-9 of the best are
 * refreshed too, so rounding in the recomputed sums cannot change the pick;
 * exact ties go to the lowest index as in the plain loop. Used to produce
 * reference runs at sizes where the plain loop takes hours. */
#define REF_BATCH 256

typedef struct {
    double key;   /* last computed gain */
    int32_t idx;
    int32_t stamp; /* step at which key was computed */
} ref_entry;

static int ref_before(const ref_entry* a, const ref_entry* b)
{
    return a->key > b->key || (a->key == b->key && a->idx < b->idx);
}

static void ref_sift_down(ref_entry* h, int64_t len, int64_t i)
{
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < len && ref_before(&h[l], &h[m])) m = l;
        if (r < len && ref_before(&h[r], &h[m])) m = r;
        if (m == i) return;
        ref_entry t = h[i]; h[i] = h[m]; h[m] = t;
        i = m;
    }
}

static void ref_sift_up(ref_entry* h, int64_t i)
{
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!ref_before(&h[i], &h[p])) return;
        ref_entry t = h[i]; h[i] = h[p]; h[p] = t;
        i = p;
    }
}

static double ref_gain_one(const float* x, int64_t n, int32_t d, const double* m, int64_t c, int metric)
{
    const float* xc = x + c * d;
    double acc = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        double q = m[v] - dis(x + v * d, xc, d, metric);
        if (q > 0.0) acc += q;
    }
    return acc / (double)n;
}

int ebc_ref_greedy_lazy(const float* x, int64_t n, int32_t d, int32_t k, int32_t* sel, double* f,
                        double* g, int64_t* evals, const float* e0, int metric)
{
    if (k > n) return -2;
    double* m = (double*)malloc(sizeof(double) * (size_t)n);
    ref_entry* h = (ref_entry*)malloc(sizeof(ref_entry) * (size_t)n);
    int64_t* stack = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* stale = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    ref_entry* batch = (ref_entry*)malloc(sizeof(ref_entry) * REF_BATCH);
    if (!m || !h || !stack || !stale || !batch) {
        free(m); free(h); free(stack); free(stale); free(batch);
        return -1;
    }
    double l0 = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        m[v] = d_e0(x + v * d, e0, d, metric);
        l0 += m[v];
    }
    l0 /= (double)n;
    /* step 0: every gain, as the plain loop computes it */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < n; ++c) {
        h[c].key = ref_gain_one(x, n, d, m, c, metric);
        h[c].idx = (int32_t)c;
        h[c].stamp = 0;
    }
    int64_t len = n, count = n;
    for (int64_t i = len / 2 - 1; i >= 0; --i) ref_sift_down(h, len, i);
    for (int32_t t = 0; t < k; ++t) {
        for (;;) {
            if (h[0].stamp != t) {
                /* stale top: take up to REF_BATCH stale entries off the top,
                   refresh them in parallel, put them back */
                int64_t nb = 0;
                while (len > 0 && h[0].stamp != t && nb < REF_BATCH) {
                    batch[nb++] = h[0];
                    h[0] = h[--len];
                    ref_sift_down(h, len, 0);
                }
#pragma omp parallel for schedule(dynamic, 1)
                for (int64_t i = 0; i < nb; ++i) {
                    batch[i].key = ref_gain_one(x, n, d, m, batch[i].idx, metric);
                    batch[i].stamp = t;
                }
                count += nb;
                for (int64_t i = 0; i < nb; ++i) {
                    h[len] = batch[i];
                    ref_sift_up(h, len);
                    ++len;
                }
                continue;
            }
            /* fresh top: every stale bound within a relative 1e-9 of it is
               refreshed first (those entries form the subtree of nodes at or
               above the threshold), then the top is the plain loop's pick */
            const double thr = h[0].key - 1e-9 * fabs(h[0].key);
            int64_t sp = 0, ns = 0;
            stack[sp++] = 0;
            while (sp > 0) {
                const int64_t i = stack[--sp];
                if (h[i].key < thr) continue;
                if (h[i].stamp != t) stale[ns++] = i;
                if (2 * i + 1 < len) stack[sp++] = 2 * i + 1;
                if (2 * i + 2 < len) stack[sp++] = 2 * i + 2;
            }
            if (ns == 0) break;
#pragma omp parallel for schedule(dynamic, 1)
            for (int64_t q = 0; q < ns; ++q) {
                h[stale[q]].key = ref_gain_one(x, n, d, m, h[stale[q]].idx, metric);
                h[stale[q]].stamp = t;
            }
            count += ns;
            for (int64_t i = len / 2 - 1; i >= 0; --i) ref_sift_down(h, len, i);
        }
        const int64_t best = h[0].idx;
        sel[t] = (int32_t)best;
        g[t] = h[0].key;
        h[0] = h[--len];
        ref_sift_down(h, len, 0);
        double sum = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            double dv = dis(x + v * d, x + best * d, d, metric);
            if (dv < m[v]) m[v] = dv;
            sum += m[v];
        }
        f[t] = l0 - sum / (double)n;
    }
    if (evals) *evals = count;
    free(m); free(h); free(stack); free(stale); free(batch);
    return 0;
}
