/*
 * ebc.h - C ABI of libebc.so: exemplar-based clustering (EBC) on one MI355X.
 *
 * The library evaluates the EBC submodular function of Honysz et al.,
 * "Providing Meaningful Data Summarizations Using Exemplar-based Clustering
 * in Industry 4.0" (arXiv 2105.12026):
 *
 *   L(S)  = |V|^-1 sum_{v in V} min_{s in S} d(v, s)        (Sec. 4, Eq. k_medoids_loss)
 *   f(S)  = L({e0}) - L(S u {e0}),  e0 = 0                   (Sec. 4, Eq. exemplar_based_clustering)
 *   d(x,y)= ||x - y||_2^2                                     (Sec. 5, experimental setup)
 *
 * over the many sets that an optimiser scores per step (Sec. 4.1: S_multi),
 * and runs the greedy optimiser (Sec. 3) on the device.
 *
 * Conventions (every entry point):
 *  - Sizes are int64_t; point indices are int32_t, so n < 2^31.
 *  - Pointers marked [device] are device (HBM) pointers; [host] are host.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call only enqueues work on `stream` and returns; results are ready
 *    when the stream has reached them. Nothing blocks except ebc_sync_status.
 *  - Host-side argument errors return at once with nothing enqueued.
 *  - Errors the device detects (bad CSR index, non-finite input) set a flag in
 *    the dataset, write NaN into the affected outputs, and are returned by the
 *    next ebc_sync_status.
 *  - No C++ exception crosses this interface.
 *  - A dataset is not thread-safe: calls on one dataset must be ordered on
 *    one stream. Distinct datasets may run concurrently on distinct streams.
 */
#ifndef EBC_H
#define EBC_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define EBC_API __attribute__((visibility("default")))
#else
#define EBC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ebc_dataset ebc_dataset; /* opaque; host struct owned by the library */
typedef struct ebc_batch ebc_batch;     /* opaque; many datasets advanced together */
typedef struct ebc_server ebc_server;   /* opaque; request loop with continuous batching */
typedef struct ebc_arena ebc_arena;     /* opaque; first-fit allocator bookkeeping */

typedef enum {
    EBC_OK = 0,
    EBC_E_INVALID_ARG = 1,  /* null pointer, size out of range, workspace too small, k > n */
    EBC_E_INDEX = 2,        /* device: CSR index outside [0, n) or offsets not non-decreasing */
    EBC_E_NONFINITE = 3,    /* device: NaN or Inf in the input points */
    EBC_E_RANGE = 4,        /* device: a value does not fit the distance dtype (FP16: |x| > 65504) */
    EBC_E_NOMEM = 5,        /* host allocation failed, or an arena block / request does not fit */
    EBC_E_DEVICE = 6,       /* a HIP runtime call failed */
    EBC_E_UNSUPPORTED = 7   /* valid request this build does not implement (e.g. d > EBC_MAX_DIM) */
} ebc_status;

/* Precision in which the candidate-point distances of the marginal gains are
 * computed (Sec. 5 compares FP32 with FP16). Inputs are cast once with
 * round-to-nearest-even; products accumulate in FP32; the norms are FP32 of
 * the cast rows; m_v, L({e0}), f, the window re-score and every cross-block
 * sum stay FP64, so greedy selections are re-scored exactly. ebc_eval_sets
 * uses FP32 dot products of the caller's rows (or, for long rows of an FP32
 * dataset, of its centred FP32 copy); ebc_eval_sets_in_dtype uses this dtype.
 *   EBC_DT_F32       float32 (v_mfma_f32_32x32x2_f32)
 *   EBC_DT_F16       IEEE half; |x| > 65504 raises EBC_E_RANGE
 *   EBC_DT_BF16      bfloat16
 *   EBC_DT_FP8_E4M3  OCP e4m3 with a power-of-two (E8M0) scale per row,
 *                    s_v = 2^ceil(log2(max_k |x_vk| / 448)), applied by the
 *                    matrix instruction's scale operands */
typedef enum {
    EBC_DT_F32 = 0,
    EBC_DT_F16 = 1,
    EBC_DT_BF16 = 2,
    EBC_DT_FP8_E4M3 = 3
} ebc_dtype;

/* Largest dimension this build accepts. Rows padded to at most 128 values
 * are held whole in registers by the distance kernels; longer rows (the
 * paper's case-study series have d = 3524, Sec. 6) take kernels that loop
 * over the dimension in chunks. */
#define EBC_MAX_DIM 4096

/* Dissimilarity flag of ebc_dataset_create. Sec. 4 defines the k-medoids
 * loss and f for any dissimilarity d; the paper's experiments (Sec. 5) and
 * this library's default use the squared Euclidean distance. EBC_FLAG_L1
 * selects the L1 (Manhattan) distance d(x,y) = sum_k |x_k - y_k| instead:
 * d(v, e0), f, the gains, greedy (including its float64 re-score and m_v
 * update), the streaming optimisers and the multi-set evaluation all use it.
 * It has no dot-product form, so its kernels run on the vector ALUs in
 * float32 (dt must be EBC_DT_F32, else EBC_E_UNSUPPORTED) with the same
 * float64 sums; L1 datasets cannot join a batch (ebc_batch_create returns
 * EBC_E_UNSUPPORTED). */
#define EBC_FLAG_L1 1u

/* Exact device workspace that ebc_dataset_create needs for (n, d, dt), in
 * bytes; 0 if the arguments are invalid. The library allocates no device
 * memory of its own, so this is the whole device footprint of a dataset
 * besides the caller's input points. */
EBC_API size_t ebc_dataset_bytes(int64_t n, int32_t d, ebc_dtype dt);

/* Make the ground set V resident and precompute what every evaluation reuses
 * (Sec. 4.2: V is copied to the device once; Sec. 4.1: L({e0}) is computed
 * once): float64 norms ||v||^2, L({e0}) = |V|^-1 sum_v ||v||^2, the greedy
 * state m_v = ||v||^2 (S = {}), and the padded distance-dtype copy of V.
 *   x         [device] float32, row-major [n, d]. Borrowed: it must stay valid
 *             and unchanged until ebc_dataset_destroy (float64 re-scoring and
 *             the m_v update read it).
 *   n, d      1 <= n < 2^31, 1 <= d <= EBC_MAX_DIM.
 *   flags     0 (squared Euclidean distance) or EBC_FLAG_L1.
 *   workspace [device] at least ebc_dataset_bytes(n, d, dt) bytes, 256-byte
 *             aligned, owned by the caller, valid until destroy.
 *   out       [host] receives the dataset handle.
 * Non-finite input is reported by ebc_sync_status as EBC_E_NONFINITE. */
EBC_API ebc_status ebc_dataset_create(const float* x, int64_t n, int32_t d, ebc_dtype dt, uint32_t flags,
                              void* workspace, size_t workspace_bytes, void* stream,
                              ebc_dataset** out);

/* Free the host struct. Does not touch the caller's workspace or x; the
 * caller must not free those before enqueued work has finished. */
EBC_API ebc_status ebc_dataset_destroy(ebc_dataset* ds);

/* Set the auxiliary vector e0 of f(S) = L({e0}) - L(S u {e0}) (Sec. 4, Eq.
 * exemplar_based_clustering: e0 is any fixed vector, the zero vector being
 * the paper's example and the default after ebc_dataset_create).
 *   e0  [device] float32 [d], read during the call's stream work only (it may
 *       be freed once that work has finished); NULL restores the origin.
 * Stream-ordered on `stream`: recomputes d(v, e0) in float64 (direct
 * differences) and L({e0}), and resets the greedy state to S = {}. Every
 * later f, gain and greedy result of this dataset uses e0. A non-finite e0
 * is reported by ebc_sync_status as EBC_E_NONFINITE.
 * Errors: EBC_E_INVALID_ARG for a null dataset; EBC_E_DEVICE if a launch
 * fails. */
EBC_API ebc_status ebc_dataset_set_e0(ebc_dataset* ds, const float* e0, void* stream);

/* Device scratch that ebc_eval_sets / ebc_eval_sets_in_dtype need for l
 * sets over a ground set of n points, in bytes: per-set unit counts,
 * validation flags, window starts and per-(set, ground-set split) float64
 * partial sums, about (20 + 8 min(16, ceil(n/256))) l bytes plus alignment. 0 if n is out
 * of range (as for ebc_dataset_bytes) or l < 0. Host-only arithmetic. */
EBC_API size_t ebc_eval_sets_bytes(int64_t n, int64_t l);

/* f(S_j) for l sets packed as CSR (Sec. 4.1, S_multi = {S_1..S_l}; Alg. 1
 * per set; Alg. 2 computes the same per-(set, point) minima).
 *   offsets [device] int64 [l+1], offsets[0] = 0, non-decreasing.
 *   idx     [device] int32 [offsets[l]]; set j = idx[offsets[j] .. offsets[j+1]).
 *           Indices are rows of V. Sets of any size; empty sets (f = 0) and
 *           repeats are allowed.
 *   f_out   [device] float64 [l].
 *   scratch [device] at least ebc_eval_sets_bytes(n, l) bytes, 256-byte
 *           aligned, owned by the caller; its contents are not needed before
 *           or after the call's stream work. The library allocates nothing.
 * Uses f(S) = (2/|V|) sum_v max(0, max_{s in S} (v.s - ||s||^2/2)) (the e0 = 0
 * term folded in): float32 dot products of the caller's float32 rows on the
 * matrix cores whatever the dataset's distance dtype (rows longer than 128
 * of a float32 dataset: its float32 copy centred at the column means, which
 * leaves f unchanged), float32 maxima, float64 sums. A bad index or offsets
 * make that set's f NaN and raise EBC_E_INDEX (deferred).
 * Errors: EBC_E_INVALID_ARG for null pointers, l < 0, a scratch that is too
 * small or not 256-byte aligned; EBC_E_DEVICE if a launch fails.
 * l = 0 is a no-op. */
EBC_API ebc_status ebc_eval_sets(ebc_dataset* ds, const int64_t* offsets, const int32_t* idx, int64_t l,
                                 double* f_out, void* scratch, size_t scratch_bytes, void* stream);

/* The same f(S_j) with the dot products in the dataset's distance dtype (the
 * paper compares FP16 with FP32 GPU evaluation, Sec. 5): the cast rows and
 * their FP32 norms, the dtype's matrix instruction (FP8 with the rows' E8M0
 * scales), FP32 maxima, FP64 sums. Same arguments, scratch and errors as
 * ebc_eval_sets; identical to it for EBC_DT_F32 datasets. */
EBC_API ebc_status ebc_eval_sets_in_dtype(ebc_dataset* ds, const int64_t* offsets, const int32_t* idx, int64_t l,
                                          double* f_out, void* scratch, size_t scratch_bytes, void* stream);

/* Size of the library's fixed device scratch (per device, held until the
 * process ends) that ebc_eval_sets_noalloc uses. */
#define EBC_FIXED_SCRATCH_BYTES ((size_t)16 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * f(S_j) as ebc_eval_sets (in_dtype = 0) or ebc_eval_sets_in_dtype
 * (in_dtype = 1), bitwise, with the per-set tables in a fixed device array of
 * EBC_FIXED_SCRATCH_BYTES owned by the library instead of a caller scratch.
 *   offsets, idx, f_out [device] as for ebc_eval_sets; the caller still owns
 *           inputs and outputs. The dataset must live on the current device.
 * The call allocates nothing (no hipMalloc, no allocating library routine);
 * the first call on a device looks up that device's copy of the array.
 * Every call on one device shares that array and it keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap on one
 * device, on different streams or threads, race and give wrong results.
 * Errors: EBC_E_INVALID_ARG for null pointers, l < 0 or in_dtype not 0/1;
 * EBC_E_NOMEM when ebc_eval_sets_bytes(n, l) > EBC_FIXED_SCRATCH_BYTES
 * (about 110000 sets over a large ground set; nothing is enqueued);
 * EBC_E_DEVICE if the array's address cannot be found or a launch fails;
 * device-detected errors as for ebc_eval_sets. l = 0 is a no-op. */
EBC_API ebc_status ebc_eval_sets_noalloc(ebc_dataset* ds, const int64_t* offsets, const int32_t* idx, int64_t l,
                                         double* f_out, int32_t in_dtype, void* stream);

/* Marginal gains Delta(c|S) = f(S u {c}) - f(S) (Sec. 3, Definition
 * "Discrete derivative") for candidates c, computed in the form
 * |V|^-1 sum_v max(0, m_v - d(v, c)) with m_v = min(||v||^2, min_{s in S} d(v,s)).
 *   m         [device] float64 [n] or NULL. Non-NULL replaces the dataset's
 *             running minima (the greedy state) by m before computing; NULL
 *             uses the current state (S = {} after create or greedy's S_k).
 *   cand      [device] int32 [n_cand] or NULL for all n points in order.
 *   gains_out [device] float64 [n_cand].
 * Distances use the dataset dtype with FP32 accumulation; sums are FP64. */
EBC_API ebc_status ebc_marginal_gains(ebc_dataset* ds, const double* m, const int32_t* cand, int64_t n_cand,
                              double* gains_out, void* stream);

/* Greedy maximisation of f under |S| <= k (Sec. 3, Eq.
 * submodular_function_optimization_cardinality_constraint; Sec. 4.1: every
 * step scores all not-yet-selected points). Starts from S = {} (resets the
 * dataset state), runs all k steps on the device with no host round trip.
 * Each step: gains of all n points -> masked argmax -> every candidate
 * within a window of the best is re-scored in float64 with direct
 * differences -> the best float64 gain wins, ties to the lowest index ->
 * m_v <- min(m_v, d(v, c*)) in float64 -> f(S_t) = L({e0}) - |V|^-1 sum m_v.
 *   k         0 <= k <= n (k = 0 is a no-op).
 *   sel_out   [device] int32 [k]: selected indices in pick order.
 *   f_out     [device] float64 [k]: f(S_1) .. f(S_k).
 *   gain_out  [device] float64 [k] or NULL: float64 gain of each pick.
 * After the call the dataset state holds S_k (usable by ebc_marginal_gains). */
EBC_API ebc_status ebc_greedy(ebc_dataset* ds, int32_t k, int32_t* sel_out, double* f_out, double* gain_out,
                      void* stream);

/* Three Sieves, a streaming optimiser for f under |S| <= k (the optimiser
 * the paper cites in Sec. 2 and runs beside greedy in its Sec. 6 case
 * study). Points arrive in `order`; one summary S; the threshold v walks
 * down the guesses (1+eps)^i in [m, k m], m = max_e f({e}), largest first,
 * after T consecutive rejections (at the smallest guess it stays); a point
 * joins while |S| < k and Delta(e|S) >= (v/2 - f(S)) / (k - |S|); the
 * stream ends early once |S| = k.
 * The stream is processed in stretches of `batch` points: one launch
 * computes the float64 distances (direct differences) of the stretch's
 * points to every point of V, and one launch walks the stretch in order on
 * the device, deciding each point on its float64 gain against the float64
 * minima of S. Decisions are therefore float64 ones whatever the dataset's
 * distance dtype (the cast copy is not used). No host round trip happens
 * between the launches; the call blocks once, at the end, for the counts.
 *   k            1 <= k <= n.
 *   eps          > 0, ratio of consecutive guesses minus 1.
 *   T            >= 1.
 *   m_max        m in f units; <= 0: computed (float64 best singleton).
 *   order        [device] int32 [n_order] indices into V (repeats allowed), or
 *                NULL for 0 .. n_order-1 (then n_order <= n).
 *   batch        stream points per stretch; 0: up to 1024, as many as keep
 *                the stretch's distances within 256 MiB (at least 32);
 *                never more than n_order.
 *   sel_out      [device] int32 [k]: accepted points in arrival order.
 *   f_out        [device] float64 [k]: f(S) after each acceptance.
 *   count_out    [host] number of accepted points.
 *   examined_out [host] or NULL: points examined before the stream ended.
 *   scratch      [device] at least ebc_three_sieves_bytes(n, k, eps, n_order,
 *                batch) bytes (one stretch's float64 distances, the float64
 *                minima, the guesses), 256-byte aligned, caller-owned;
 *                ebc_three_sieves_bytes is host-only arithmetic, 0 for
 *                arguments out of range.
 * Errors: EBC_E_INVALID_ARG (arguments, scratch too small or unaligned),
 * EBC_E_INDEX (an order entry outside [0, n), detected on the host before
 * any work), EBC_E_DEVICE. The dataset state afterwards holds the summary
 * (usable by ebc_marginal_gains). */
EBC_API size_t ebc_three_sieves_bytes(int64_t n, int32_t k, double eps, int64_t n_order, int32_t batch);
EBC_API ebc_status ebc_three_sieves(ebc_dataset* ds, int32_t k, double eps, int64_t T, double m_max,
                                    const int32_t* order, int64_t n_order, int32_t batch, int32_t* sel_out,
                                    double* f_out, int32_t* count_out, int64_t* examined_out, void* scratch,
                                    size_t scratch_bytes, void* stream);

/* Sieve Streaming, the other optimiser the paper names (Sec. 2; Sec. 4.1:
 * optimisers such as greedy or Sieve Streaming score many sets per step):
 * one summary per guess v of the same grid as ebc_three_sieves, every
 * arriving point offered to each summary under the same rule, the stream
 * ending early once every summary is full; the best summary (largest f,
 * the largest v among equal f) is returned. Each stretch's float64
 * distances are computed once and shared by every summary; the walk runs
 * one workgroup per summary, each with its own float64 minima, so the
 * decisions are float64 ones as in ebc_three_sieves. Blocking once at the
 * end, like ebc_three_sieves; arguments as there, and:
 *   sel_out, f_out  [device] the best summary's points and f after each of
 *                   its acceptances;
 *   v_out           [host] or NULL: the best summary's guess v.
 *   scratch         [device] at least ebc_sieve_streaming_bytes(n, k, eps,
 *                   n_order, batch) bytes (host-only arithmetic; 0 for
 *                   arguments out of range), 256-byte aligned, caller-owned:
 *                   one stretch's float64 distances, and per guess (at most
 *                   floor(log k / log(1+eps)) + 2 of them) its float64 minima,
 *                   members, f values and state.
 * The dataset state afterwards holds the best summary's minima. */
EBC_API size_t ebc_sieve_streaming_bytes(int64_t n, int32_t k, double eps, int64_t n_order, int32_t batch);
EBC_API ebc_status ebc_sieve_streaming(ebc_dataset* ds, int32_t k, double eps, double m_max, const int32_t* order,
                                       int64_t n_order, int32_t batch, int32_t* sel_out, double* f_out,
                                       int32_t* count_out, double* v_out, int64_t* examined_out, void* scratch,
                                       size_t scratch_bytes, void* stream);

/* Graph mode for ebc_greedy (default off): the reset and all k steps are
 * recorded once into a HIP graph (on a private stream; recording runs
 * nothing) and the graph is replayed on `stream` by every later call with
 * the same k, output pointers and gains variant; other calls re-record.
 * One graph launch replaces 8k+1 kernel launches, which is what bounds small
 * problems. Results are identical to eager mode. Ignored while profiling. */
EBC_API ebc_status ebc_set_greedy_graph(ebc_dataset* ds, int32_t on);

/* Batched greedy over many independent datasets (different n, d, k and
 * distance dtype). Per step tick the library issues one marginal-gains
 * launch per kernel bucket (same dtype, row padding and tile variant) and
 * seven step launches, each covering every instance; instances whose k is
 * reached skip the remaining ticks. Every instance computes exactly what its
 * solo ebc_greedy computes (bitwise-identical selections, f and gains),
 * independent of the batch composition.
 *
 * ebc_batch_bytes(count): device workspace of the batch tables (descriptor
 * table and block maps), 256-byte aligned, caller-owned.
 * ebc_batch_create: `ds` [host] array of `count` datasets (each keeps its
 * own workspace and state; all on the same device); copies the block maps to
 * the device and waits for `stream`. The datasets must outlive the batch and
 * not be used concurrently with it.
 * ebc_greedy_batched: k [host] int32 [count] (0 <= k[i] <= n_i); sel_out,
 * f_out [host] arrays of `count` device pointers as in ebc_greedy (entries
 * may be NULL where k[i] = 0); gain_out [host] array or NULL (entries may be
 * NULL). Resets every instance to S = {} first. Errors per instance are
 * reported by ebc_sync_status on that dataset.
 * ebc_batch_set_graph: record the reset and all ticks into one HIP graph
 * and replay it while the number of ticks (max k) is unchanged; the
 * per-instance k and output pointers live in the device table, so they may
 * change between replays. */
EBC_API size_t ebc_batch_bytes(int32_t count);
EBC_API ebc_status ebc_batch_create(ebc_dataset* const* ds, int32_t count, void* workspace,
                                    size_t workspace_bytes, void* stream, ebc_batch** out);
EBC_API ebc_status ebc_batch_destroy(ebc_batch* batch);
EBC_API ebc_status ebc_batch_set_graph(ebc_batch* batch, int32_t on);
EBC_API ebc_status ebc_greedy_batched(ebc_batch* batch, const int32_t* k, int32_t* const* sel_out,
                                      double* const* f_out, double* const* gain_out, void* stream);
/* Launch geometry of one tick: gains buckets, gains workgroups, row blocks. */
EBC_API ebc_status ebc_batch_info(ebc_batch* batch, int32_t* buckets, int64_t* gains_workgroups_per_tick,
                                  int64_t* row_blocks_per_tick);

/* ---- Serving: continuous batching at greedy-step granularity ----
 * A request is (ground set x [host float32, n x d], greedy bound k, dtype).
 * ebc_server_create: `arena` [device] block of arena_bytes (256-aligned,
 * caller-owned) that holds everything the server places on the device: the
 * batched-tick tables for max_slots requests, and per admitted request its
 * points, dataset workspace and outputs (ebc_request_bytes), sub-allocated
 * first-fit. All work is enqueued on `stream`.
 * ebc_server_submit: copies x into a host buffer (the caller's may be reused
 * at once) and queues the request; t_arrival is its arrival time on the
 * server clock (ebc_server_now), or < 0 for now. A request larger than the
 * whole arena is refused (EBC_E_NOMEM).
 * ebc_server_step: one scheduler tick: admits queued requests in arrival
 * order while a slot is free and the head request fits the arena (the head
 * waits otherwise); advances every active request by one greedy step in one
 * batched launch set (one gains launch per kernel bucket, seven step
 * launches); copies out and releases the requests that reached k, waiting
 * for `stream` only when one did. Each request computes exactly what a solo
 * ebc_greedy computes, alone or in any mix.
 * ebc_server_poll: state 0 queued, 1 active, 2 done, 3 failed; on done, the
 * k selections, f(S_1..S_k) and gains (host pointers, NULL to skip); the
 * arrival, admission and completion times (seconds, server clock).
 * The arena functions expose the server's allocator bookkeeping (no device
 * access) for drivers that plan admission and for tests. */
EBC_API size_t ebc_request_bytes(int64_t n, int32_t d, int32_t k, ebc_dtype dt);
EBC_API ebc_status ebc_server_create(void* arena, size_t arena_bytes, int32_t max_slots, void* stream,
                                     ebc_server** out);
EBC_API ebc_status ebc_server_destroy(ebc_server* server);
EBC_API ebc_status ebc_server_submit(ebc_server* server, const float* x_host, int64_t n, int32_t d, int32_t k,
                                     ebc_dtype dt, double t_arrival, int64_t* req_id);
EBC_API ebc_status ebc_server_step(ebc_server* server, int32_t* completed);
EBC_API ebc_status ebc_server_poll(ebc_server* server, int64_t req_id, int32_t* state, int32_t* sel_host,
                                   double* f_host, double* gain_host, double* t_arrive, double* t_admit,
                                   double* t_done);
EBC_API ebc_status ebc_server_stats(ebc_server* server, int32_t* queued, int32_t* active, int64_t* completed,
                                    int64_t* ticks, size_t* free_bytes);
EBC_API double ebc_server_now(void);
EBC_API ebc_status ebc_arena_create(size_t capacity, ebc_arena** out);
EBC_API ebc_status ebc_arena_alloc(ebc_arena* arena, size_t bytes, size_t* offset);
EBC_API ebc_status ebc_arena_free(ebc_arena* arena, size_t offset);
EBC_API size_t ebc_arena_free_bytes(const ebc_arena* arena);
EBC_API size_t ebc_arena_largest_free(const ebc_arena* arena);
EBC_API ebc_status ebc_arena_destroy(ebc_arena* arena);

/* Host-side counters of the last ebc_greedy on this dataset, valid after
 * ebc_sync_status: window_max = largest number of candidates re-scored in
 * one step, window_overflow = steps whose window exceeded its capacity. */
typedef struct {
    int32_t window_max;
    int32_t window_overflow;
    int32_t steps;
    int32_t reserved;
} ebc_greedy_stats;

/* Wait for `stream`, then return the first deferred device error of this
 * dataset (and clear it), or EBC_OK. Fills *stats (may be NULL). */
EBC_API ebc_status ebc_sync_status(ebc_dataset* ds, void* stream, ebc_greedy_stats* stats);

/* Static English description of a status code. */
EBC_API const char* ebc_status_string(ebc_status st);

/* Geometry the library chose for a dataset (tile shape of the gains kernel),
 * for benchmarks and tests. */
typedef struct {
    int64_t n;
    int64_t n_pad;
    int32_t d;
    int32_t k_pad;          /* padded row length of the distance-dtype copy */
    int32_t v_splits;       /* ground-set chunks a candidate tile is split into */
    int32_t cand_tile;      /* candidates per gains workgroup */
    int32_t window_cap;     /* most candidates re-scored in float64 per step */
    int32_t dtype;
    uint32_t flags;         /* the dissimilarity flag given at creation (0 or EBC_FLAG_L1) */
    int32_t reserved;
    double l0;              /* L({e0}) as of the last ebc_sync_status (follows ebc_dataset_set_e0) */
} ebc_dataset_info;

EBC_API ebc_status ebc_dataset_get_info(ebc_dataset* ds, ebc_dataset_info* info);

/* Tile shape of the marginal-gains kernel for this dataset. Every variant
 * computes the same sums in the same order per (candidate, ground chunk), so
 * results do not depend on it; an autotuner picks the fastest per dtype and
 * size. Variants 0..ebc_gains_variant_count(dt)-1; the default is 0 for
 * EBC_DT_F32 and 4 (bound test interleaved with the matrix work) for the
 * reduced-precision dtypes. Rows
 * padded past 128 values have a single long-row kernel, which every
 * variant selects. */
EBC_API ebc_status ebc_set_gains_variant(ebc_dataset* ds, int32_t variant);
EBC_API int32_t ebc_gains_variant_count(ebc_dtype dt);

/* Autotuner for the gains tile variant. Looks up the process-wide table
 * keyed by (dtype, padded row length, floor(log2(n_pad))); on a miss (or
 * with force != 0) times every variant on this dataset (reps launches each,
 * HIP events on `stream`, blocking), records the fastest and sets it. Does
 * not change the dataset's greedy state. variant_out and times_ms_out
 * ([ebc_gains_variant_count(dt)], per-launch milliseconds, only when
 * measured) may be NULL. The table persists through the text file of
 * ebc_tune_cache_load/_save (one "dtype k_pad size_bucket variant" per line). */
EBC_API ebc_status ebc_autotune(ebc_dataset* ds, int32_t reps, int32_t force, void* stream, int32_t* variant_out,
                                float* times_ms_out);
EBC_API ebc_status ebc_tune_cache_load(const char* path);
EBC_API ebc_status ebc_tune_cache_save(const char* path);
EBC_API int32_t ebc_tune_cache_size(void);

/* Per-kernel timing of ebc_greedy with HIP events recorded on the call's
 * stream around each step's marginal-gains launch and around the whole step.
 * Off by default; when on, ebc_greedy records 3 events per step (host-side
 * event objects, no device memory). ebc_profile_read waits for the last
 * recorded event and returns the totals since the last reset. */
typedef struct {
    double gains_ms;        /* summed duration of the marginal-gains kernel */
    double select_ms;       /* summed duration of the rest of each step */
    int32_t gains_launches; /* gains launches timed */
    int32_t steps;          /* greedy steps timed */
} ebc_profile;

EBC_API ebc_status ebc_profile_enable(ebc_dataset* ds, int32_t on);
EBC_API ebc_status ebc_profile_read(ebc_dataset* ds, ebc_profile* out, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* EBC_H */
