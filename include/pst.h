/*
 * pst.h -- C ABI of the MI355X MPdist-profile / snippet library.
 *
 * The library computes, on one gfx950 GPU, the snippet-finding hot path of
 * the PaSTiLa method (Goglachev 2023, "a parallel algorithm for automated
 * labelling of large time series"):
 *
 *   - MPdist profiles of a query, and of every segment, against a series
 *     (section 4.1, eqs. 9-15),
 *   - greedy minimum-area snippet selection with neighbours and frac
 *     (section 3.2, eqs. 5-8; section 4.1, eqs. 16-17),
 *   - the snippet-length criterion over candidate lengths (section 4.2, eq. 18),
 *   - multivariate series, each coordinate searched on its own (eqs. 1-2,
 *     section 3.2), and the same search in bounded device memory,
 *   - labelling of the series by its snippets and its per-element F1
 *     (section 5.2's accuracy measure),
 *   - run-time prediction and Karmarkar-Karp partitioning of candidate
 *     lengths (section 4.2; host only), and a request server.
 *
 * Conventions
 *   - Every index is 0-based (the paper is 1-based).  A snippet's index is its
 *     segment number s; the segment starts at element s*m (eq. 4).
 *   - n: series length; m: segment / snippet length; l: MPdist sub-length;
 *     w = m-l+1; nseg = floor(n/m) (the tail after the last whole segment is
 *     not a segment but is covered by the windows); Nm = n-m+1 windows.
 *   - k: order statistic of eq. 13, 1-based.  k <= 0 selects the paper's
 *     typical value ceil(0.05*2m) = (m+9)/10.  When 2w <= k the largest
 *     element of P_ABBA is taken, as eq. 13 prescribes.
 *   - Series are float64 in device memory.  Profiles are float32.
 *   - The caller owns every buffer.  *_dev arguments are device pointers on the
 *     context's device; *_host arguments are host pointers.  The library never
 *     keeps a pointer past return.
 *   - Work is issued on the stream given to pst_create.  Functions that return
 *     host results synchronise that stream before returning; the others
 *     (pst_profile_set, pst_mpdist_profile) also synchronise once, after the
 *     statistics pass, to report non-finite input.
 *   - Return value: PST_OK (0) or a negative pst_status.  A message is kept in
 *     the context (pst_last_error).  After PST_EDEVICE the context is poisoned
 *     and every later call returns PST_EDEVICE.
 *   - A context is not thread-safe; use one per host thread.
 */
#ifndef PST_H
#define PST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PST_OK = 0,
    PST_EINVAL = -1,     /* bad argument, non-finite series, workspace too small */
    PST_ENOMEM = -2,     /* does not fit the memory budget */
    PST_EDEVICE = -3,    /* HIP runtime error; context poisoned */
    PST_ENOTREADY = -4,  /* serving: result not ready yet */
    PST_ECANCELED = -5
} pst_status;

typedef struct pst_ctx pst_ctx;

/* One snippet (section 3.2): its index (the segment number, eq. 5 and the
 * definition of a snippet's index), its position in greedy order, its
 * significance frac (eq. 7), and ProfileArea (eq. 17) after it was picked. */
typedef struct {
    int32_t segment;
    int32_t greedy_rank;
    double  frac;
    double  area_after;
} pst_snippet;

/* Library version string. */
const char *pst_version(void);

/* Create a context on `device`.  `hip_stream` is a hipStream_t (for example
 * torch.cuda.current_stream().cuda_stream) or NULL for the null stream. */
int  pst_create(pst_ctx **out, int device, void *hip_stream);
void pst_destroy(pst_ctx *ctx);
const char *pst_last_error(const pst_ctx *ctx);

/* Bytes of device workspace needed by pst_profile_set, pst_mpdist_profile and
 * pst_snippets for these sizes (0 if the sizes are invalid).  The workspace is
 * caller-allocated, 256-byte aligned, and may be reused between calls. */
size_t pst_workspace_bytes(int64_t n, int32_t m, int32_t l, int32_t K);

/* Workspace for pst_select_length: the maximum over the candidate lengths.
 * l_list NULL means l = m/2 for every m. */
size_t pst_select_length_workspace_bytes(int64_t n, const int32_t *m_list, int32_t num_m,
                                         const int32_t *l_list, int32_t K);

/* eq. 14: MPdist profile of a query Q (length m) against every length-m window
 * of T.  out_dev: float32[n-m+1].  Statistics of Q's l-subsequences are taken
 * from Q itself.  Errors: PST_EINVAL if l < 2, l > m, m > n, w exceeds the
 * supported maximum (1025), the workspace is too small, or T or Q holds a
 * non-finite value. */
int pst_mpdist_profile(pst_ctx *ctx, const double *T_dev, int64_t n,
                       const double *Q_dev, int32_t m, int32_t l, int32_t k,
                       float *out_dev, void *ws_dev, size_t ws_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the eq. 14
 * query profile of pst_mpdist_profile without a workspace argument.  Its
 * scratch is a fixed 256 MiB device array of the library, one per GPU the
 * library runs on, held until the process ends; the call allocates nothing.
 * The statistics of T take 64 bytes per point (n up to about 4 million at
 * m = 256, l = 128); the persistent grid shrinks to the profile slots that
 * fit in the rest (4 MB each at that m and l), so long series run on fewer
 * compute units.  Results equal pst_mpdist_profile's.
 * Every call on one GPU uses the same array: calls that overlap on one GPU
 * (other threads, contexts or streams) race and must be serialised by the
 * caller.  The call returns once its work is done.  PST_EINVAL as
 * pst_mpdist_profile, and when n, m, l need more scratch than the array
 * holds; PST_EDEVICE if the array's address could not be looked up. */
int pst_mpdist_profile_noalloc(pst_ctx *ctx, const double *T_dev, int64_t n, const double *Q_dev, int32_t m,
                               int32_t l, int32_t k, float *out_dev);

/* eq. 15: the profile set D = (D_0 .. D_{nseg-1}), D_s = MPD(S_s, T).
 * D_dev: float32, row s at D_dev + s*ld, ld >= n-m+1.  dmax_dev (optional,
 * may be NULL): float32[1], receives max over all entries of D (the
 * denominator of eq. 18).  Errors as pst_mpdist_profile. */
int pst_profile_set(pst_ctx *ctx, const double *T_dev, int64_t n, int32_t m, int32_t l,
                    int32_t k, float *D_dev, int64_t ld, float *dmax_dev,
                    void *ws_dev, size_t ws_bytes);

/* The problem statement of section 3.2: the K most significant snippets of
 * length m.  out_host: pst_snippet[K], ordered by frac descending (eq. 8),
 * equal frac kept in greedy order.  Optional outputs (NULL to skip):
 *   profiles_dev  float32[K][n-m+1], profile of the snippet picked r-th at row r
 *   owner_dev     int32[n-m+1], greedy rank of the nearest snippet of each
 *                 window (the Neighbors sets of eq. 6, ties to the earlier pick)
 *   dmax_host     float32, max over all entries of D
 * Errors: as above, plus PST_EINVAL if K < 1 or K > nseg (the paper requires
 * 1 <= K <= n/m). */
int pst_snippets(pst_ctx *ctx, const double *T_dev, int64_t n, int32_t m, int32_t l,
                 int32_t k, int32_t K, pst_snippet *out_host, float *profiles_dev,
                 int32_t *owner_dev, float *dmax_host, void *ws_dev, size_t ws_bytes);

/* Bounded device memory (series whose profile set D does not fit): the same
 * result as pst_snippets without ever holding D whole.  Every greedy round
 * recomputes D in blocks of seg_block segments (1 <= seg_block <= n/m),
 * reduces each block to the segments' areas against the current curve (eq. 17)
 * and drops it; the picked segment's profile is recomputed alone and kept.
 * Device memory grows with seg_block * (n-m+1) + K * (n-m+1) floats instead
 * of (n/m) * (n-m+1); the profile work is K + 1 times that of pst_snippets.
 * Records, profiles_dev, owner_dev and dmax_host are bit-identical to
 * pst_snippets'.  The workspace must hold
 * pst_snippets_blocked_workspace_bytes(n, m, l, K, seg_block) bytes (0 for
 * invalid sizes); pst_snippets_blocked_max_block gives the largest seg_block
 * whose workspace fits budget_bytes (0 if none).  Errors as pst_snippets,
 * plus PST_EINVAL for seg_block outside [1, n/m]. */
size_t pst_snippets_blocked_workspace_bytes(int64_t n, int32_t m, int32_t l, int32_t K, int32_t seg_block);
int32_t pst_snippets_blocked_max_block(int64_t n, int32_t m, int32_t l, int32_t K, size_t budget_bytes);
int pst_snippets_blocked(pst_ctx *ctx, const double *T_dev, int64_t n, int32_t m, int32_t l,
                         int32_t k, int32_t K, int32_t seg_block, pst_snippet *out_host,
                         float *profiles_dev, int32_t *owner_dev, float *dmax_host,
                         void *ws_dev, size_t ws_bytes);

/* As pst_snippets_blocked, with the profile set spilled to host memory
 * instead of recomputed: it is computed once, block by block, and copied to
 * D_host (float32[n/m][n-m+1], row s = D_s, caller-owned; page-locked memory
 * from hipHostMalloc, or the copies are slow); later greedy rounds and the
 * picked rows are copied back from it.  Same workspace, same bit-identical
 * results; D_host holds the whole profile set on return. */
int pst_snippets_spilled(pst_ctx *ctx, const double *T_dev, int64_t n, int32_t m, int32_t l,
                         int32_t k, int32_t K, int32_t seg_block, float *D_host,
                         pst_snippet *out_host, float *profiles_dev, int32_t *owner_dev,
                         float *dmax_host, void *ws_dev, size_t ws_bytes);

/* eq. 18 in bounded device memory: every candidate length searched as in
 * pst_snippets_blocked (blocks of min(seg_block, n/m) segments), one length
 * after another, its criterion computed from the K kept profiles; then the
 * chosen length once more for out_host / profiles_dev / owner_dev.  Scores,
 * m_best and the outputs are bit-identical to pst_select_length's.  The
 * workspace must hold pst_select_length_blocked_workspace_bytes(...) bytes (0
 * for invalid sizes): the largest single candidate's, not the sum.  Errors as
 * pst_select_length, plus PST_EINVAL for seg_block < 1. */
size_t pst_select_length_blocked_workspace_bytes(int64_t n, const int32_t *m_list, int32_t num_m,
                                                 const int32_t *l_list, int32_t K, int32_t seg_block);
int pst_select_length_blocked(pst_ctx *ctx, const double *T_dev, int64_t n,
                              const int32_t *m_list, int32_t num_m, const int32_t *l_list,
                              int32_t K, int32_t seg_block, int32_t *m_best, double *scores_host,
                              pst_snippet *out_host, float *profiles_dev, int32_t *owner_dev,
                              void *ws_dev, size_t ws_bytes);

/* Multivariate series (eqs. 1-2): d coordinates of length n, coordinate j
 * at T_dev + j*ld (float64, ld >= n).  Section 3.2 runs the snippet search on
 * each coordinate independently; here every coordinate's profile set runs in
 * one persistent launch (one job per coordinate), then each coordinate's
 * greedy search and neighbours.  Results equal d calls of pst_snippets.
 *   out_host   pst_snippet[d][K], row j for coordinate j, ordered as in
 *              pst_snippets
 *   owner_dev  int32[d][n-m+1] (may be NULL), row j as pst_snippets' owner_dev
 *   dmax_host  float32[d] (may be NULL), max of each coordinate's D
 * The workspace must hold pst_snippets_multi_workspace_bytes(d, n, m, l, K)
 * bytes (256-byte aligned; 0 is returned for invalid sizes).  Errors as
 * pst_snippets, plus PST_EINVAL if d < 1 or d > 16 or ld < n, naming the first
 * coordinate that holds a non-finite value. */
size_t pst_snippets_multi_workspace_bytes(int32_t d, int64_t n, int32_t m, int32_t l, int32_t K);
int pst_snippets_multi(pst_ctx *ctx, const double *T_dev, int32_t d, int64_t ld, int64_t n,
                       int32_t m, int32_t l, int32_t k, int32_t K, pst_snippet *out_host,
                       int32_t *owner_dev, float *dmax_host, void *ws_dev, size_t ws_bytes);

/* eq. 18 over num_m (1..16) candidate lengths m_list (l_list NULL: l = m/2; k
 * is the default of each m).  scores_host: float64[num_m] (may be NULL).
 * m_best receives the argmax (ties to the smallest m); out_host /
 * profiles_dev / owner_dev receive the snippets of m_best as in pst_snippets.
 * K must be valid for every candidate.  By default every candidate's profiles
 * run in one persistent launch, captured with the rest of the sweep as one HIP
 * graph (replayed when the same pointers and sizes come back); see
 * pst_set_option.  The workspace must hold pst_select_length_workspace_bytes. */
int pst_select_length(pst_ctx *ctx, const double *T_dev, int64_t n,
                      const int32_t *m_list, int32_t num_m, const int32_t *l_list,
                      int32_t K, int32_t *m_best, double *scores_host,
                      pst_snippet *out_host, float *profiles_dev, int32_t *owner_dev,
                      void *ws_dev, size_t ws_bytes);

/* ---- Scheduling (section 4.2) ----
 * Run times predicted by polynomial regression on earlier runs, and the
 * Karmarkar-Karp partition that spreads candidate lengths over workers with
 * balanced predicted load.  Host-only: no device, no context.
 *
 * A model is a polynomial of total degree `degree` (1..4) in three scaled
 * sizes of a run: u = floor(n/m)/1e3 (segments), w = (m-l+1)/1e2 (window
 * width), v = (n-l+1)/1e5 (subsequences); the distance-matrix cell count is
 * proportional to u*w*v.  Monomials u^a w^b v^c in graded order: total degree
 * t = 0..degree, a from t down to 0, b from t-a down to 0.
 * pst_model_fit minimises the relative squared error sum ((p_i - ms_i)/ms_i)^2
 * plus a ridge of 1e-10 times the mean squared column norm (so that fewer
 * runs than monomials still determine it), by Householder QR.
 * Errors: PST_EINVAL for invalid sizes, a non-positive or non-finite time, a
 * degree outside 1..4; PST_ENOTREADY before the first observation / fit. */
typedef struct pst_model pst_model;
int  pst_model_create(pst_model **out, int32_t degree);
void pst_model_destroy(pst_model *model);
int  pst_model_observe(pst_model *model, int64_t n, int32_t m, int32_t l, double ms);
int  pst_model_fit(pst_model *model);
/* coef_out: up to cap coefficients in monomial order; num_out: their count */
int  pst_model_coefficients(const pst_model *model, double *coef_out, int32_t cap, int32_t *num_out);
int  pst_model_predict(const pst_model *model, int64_t n, int32_t m, int32_t l, double *ms_out);
/* k-way largest differencing of count non-negative costs into `parts`
 * (1..4096) parts: every item starts as a parts-tuple (cost, 0, .., 0); the two
 * tuples of largest spread (max - min; ties to the older tuple, items being
 * older than merges and in input order) are merged slot by slot, largest slot
 * of the first with smallest of the second, and the merged slots re-sorted
 * largest first (stable), until one tuple is left.  part_out[i]: the part of
 * item i (parts numbered by load, largest first); load_out[parts]: each part's
 * summed cost.  PST_EINVAL for a negative or non-finite cost, or when
 * count * parts exceeds 2^24 (the merge tuples hold count * parts sums). */
int  pst_partition_kk(const double *cost, int32_t count, int32_t parts, int32_t *part_out,
                      double *load_out);
/* The candidate lengths of eq. 18 (l_list NULL: l = m/2) spread over `parts`
 * workers by the model's predicted run times on a series of length n
 * (negative predictions count as 0). */
int  pst_partition_lengths(const pst_model *model, int64_t n, const int32_t *m_list,
                           const int32_t *l_list, int32_t num_m, int32_t parts,
                           int32_t *part_out, double *load_out);

/* ---- Serving ----
 * A server admits requests (one series each, with its own n, m, l, K) as
 * device memory and slots free up and keeps each result until it is
 * collected (section 4.2 runs many lengths of one series across a cluster;
 * here many series share one GPU).  Work is batched continuously: an admitted
 * request's copy-in and statistics run on a preparation stream; the profile
 * tiles of all ready requests of one workgroup shape (up to 16) run in one
 * shared persistent launch, a new batch starting on a second stream while the
 * previous one drains; each request's greedy search, neighbours and result
 * copies follow its batch.  Admission: first fit in arrival order while the
 * admitted requests' footprints (pst_request_bytes, rounded up to the
 * server's 25 % size classes) plus the profile scratch of the two batch
 * streams stay within hbm_budget_bytes, and at most max_slots (1..64)
 * requests are admitted at once.  The server owns its device memory (freed
 * blocks are cached up to a quarter of the budget; an allocation that fails
 * drops the cache and tries once more) and a worker thread.  A request whose
 * memory cannot be allocated while nothing else holds memory completes with
 * PST_ENOMEM; after a device error every admitted request completes with
 * PST_EDEVICE and the server accepts no more.  All pst_server functions are
 * thread-safe.  A request's result equals that of pst_snippets on the same
 * input (k is the default of m), whatever it is batched with. */
typedef struct pst_server pst_server;
int pst_server_create(pst_server **out, int device, size_t hbm_budget_bytes, int32_t max_slots);
void pst_server_destroy(pst_server *server);   /* drops requests not yet admitted */
const char *pst_server_last_error(const pst_server *server);
/* Device bytes one request holds while admitted, before rounding to a size
 * class: the series and its workspace without profile scratch (0 if the sizes
 * are invalid). */
size_t pst_request_bytes(int64_t n, int32_t m, int32_t l, int32_t K);
/* Host-only: the size class (bytes) the server charges for a request of
 * `bytes` (the smallest 1 MiB * 1.25^j not below it). */
int pst_pool_size_class(size_t bytes, size_t *charged);
/* Queue a request; T_host (n values) is copied before return.  PST_EINVAL for
 * invalid sizes, PST_ENOMEM if the request with the profile scratch of a
 * batch of its own width can never fit the budget, PST_EDEVICE after a device
 * error. */
int pst_submit(pst_server *server, const double *T_host, int64_t n, int32_t m, int32_t l, int32_t K,
               uint64_t *ticket);
/* As pst_submit with the series already in device memory of the server's
 * device (T_dev, n doubles, owned by the caller): the server copies it on the
 * device once the request is admitted, so T_dev must stay valid and unchanged
 * until pst_poll returns the request's status. */
int pst_submit_device(pst_server *server, const double *T_dev, int64_t n, int32_t m, int32_t l, int32_t K,
                      uint64_t *ticket);
/* PST_ENOTREADY until the request is done; then fills out_host[K] (ordered
 * as pst_snippets), the latency from submission to completion in ms, releases
 * the ticket and returns its status (PST_EINVAL for a non-finite series). */
int pst_poll(pst_server *server, uint64_t ticket, pst_snippet *out_host, int32_t K, double *latency_ms);
/* Wait until no request is queued or running: PST_OK, or PST_ENOTREADY at the timeout. */
int pst_server_drain(pst_server *server, int32_t timeout_ms);
/* Completed requests, their distance-matrix cells, running requests, bytes held. */
/* Admission order (section 4.2's run-time prediction applied to one GPU's
 * queue).  PST_POLICY_ARRIVAL (the default): first fit in arrival order.
 * PST_POLICY_SHORTEST_PREDICTED: first fit, scanning the waiting requests by
 * predicted run time, shortest first (equal predictions in arrival order).
 * The prediction comes from the server's own degree-2 model (a copy of `seed`
 * when given, which the caller keeps ownership of), extended with the device
 * time of every completed request (from its first to its last operation on
 * its stream, so overlap with other requests is included) and refitted after
 * every fourth; without a fitted model a request's cell count is its
 * prediction.  Shortest-first lowers typical latency; a long request can
 * wait behind shorter ones that keep arriving.  PST_EINVAL for an unknown
 * policy. */
enum { PST_POLICY_ARRIVAL = 0, PST_POLICY_SHORTEST_PREDICTED = 1 };
int pst_server_set_policy(pst_server *server, int32_t policy, const pst_model *seed);
int pst_server_stats(pst_server *server, uint64_t *completed, double *cells, int32_t *active,
                     size_t *bytes_in_use);
/* Profile batches launched so far. */
int pst_server_batches(pst_server *server, uint64_t *batches);
/* Host-only simulation of the admission policy (no device use), for tests:
 * request i of `bytes[i]` arrives at arrive_ms[i] (non-decreasing) and holds
 * its memory for service_ms[i] after admission; start_ms[i] receives its
 * admission time, -1 if never admitted.  PST_ENOMEM if some request exceeds
 * the budget. */
int pst_admission_simulate(size_t budget, int32_t slots, int32_t count, const size_t *bytes,
                           const double *arrive_ms, const double *service_ms, double *start_ms);
/* As pst_admission_simulate, with the waiting requests scanned by ascending
 * priority[i] (ties in arrival order) instead of arrival order; priority NULL
 * gives arrival order. */
int pst_admission_simulate_ordered(size_t budget, int32_t slots, int32_t count, const size_t *bytes,
                                   const double *arrive_ms, const double *service_ms,
                                   const double *priority, double *start_ms);

/* Labelling score (the per-element F1 of section 5.2's accuracy experiment).
 * owner_dev: int32[n-m+1], the greedy rank (0 .. K-1) of each window's nearest
 * snippet, as written by pst_snippets / pst_select_length (eq. 6).
 * truth_dev: int32[n], the true class (0 .. C-1) of each element.
 * The paper does not spell out how snippets label elements; here element t
 * takes the snippet owning window min(t, n-m), and snippet p stands for the
 * true class most of its elements have (ties to the lowest class).
 * Results (host, each optional except macro_f1_host): map_host int32[K], the
 * class of each snippet; precision_host, recall_host, f1_host double[C], per
 * true class, TP/(TP+FP), TP/(TP+FN), 2PR/(P+R), 0 where a denominator is 0;
 * *macro_f1_host, the mean F1 over the classes present in truth.
 * ws_dev: device workspace of pst_label_workspace_bytes(K, C) bytes, 256-byte
 * aligned.  Synchronises the context's stream.  PST_EINVAL for K, C out of
 * range (K <= 2^20, C <= 4096, K*C <= 2^26), m < 1, n < m, or any owner or
 * class outside its range.  pst_label_workspace_bytes returns 0 for bad K, C. */
size_t pst_label_workspace_bytes(int32_t K, int32_t C);
int pst_label_f1(pst_ctx *ctx, const int32_t *owner_dev, int64_t n, int32_t m, int32_t K,
                 const int32_t *truth_dev, int32_t C, int32_t *map_host, double *precision_host,
                 double *recall_host, double *f1_host, double *macro_f1_host, void *ws_dev, size_t ws_bytes);

/* Options of a context (value semantics in brackets, default first):
 *   PST_OPT_SWEEP_GRAPH    capture the length sweep as a HIP graph [1, 0]
 *   PST_OPT_AUTOTUNE       tune the persistent grid and tile scheduling of the
 *                          sweep's profile launch on first use of a shape
 *                          bucket [0, 1]; the choice is kept per process and,
 *                          if the environment variable PST_AUTOTUNE_CACHE names
 *                          a file, appended there and read back later (a grid
 *                          read back never exceeds the workspace's slots)
 *   PST_OPT_PROFILE_GRID   persistent workgroups of the sweep launch [0 = all
 *                          that are resident at once]
 *   PST_OPT_DYNAMIC_TILES  hand tiles out from a device counter [1, 0]
 *   PST_OPT_SWEEP_BATCHED  one launch for all candidates [1]; 0 runs the
 *                          candidates one after another (the plain path)
 * None of the above changes any result.
 *   PST_OPT_TUNE_GEOMETRY  before a batched sweep, choose each length's tile
 *                          geometry by timing every candidate (pst_tune_geometry)
 *                          [0, 1]; results stay within the profile tolerance
 *                          of the built-in geometry, not bit for bit
 *   PST_OPT_SWEEP_ONE_LAUNCH  run every length of a batched sweep in one
 *                          launch with the widest length's tile geometry [0, 1]
 *                          (0: one launch per workgroup shape among the
 *                          lengths); results within the profile tolerance
 *   PST_OPT_ANCHOR_EVERY   R > 0: besides the FP64 anchor at the first cell of
 *                          each diagonal of a sub-tile (at most w-1 FP32 steps
 *                          apart), re-anchor every diagonal with an exact FP64
 *                          dot product at rows that are multiples of R [0]
 *                          (precision study; R >= w-1 changes nothing)
 * Returns PST_EINVAL for an unknown option. */
enum {
    PST_OPT_SWEEP_GRAPH = 1,
    PST_OPT_AUTOTUNE = 2,
    PST_OPT_PROFILE_GRID = 3,
    PST_OPT_DYNAMIC_TILES = 4,
    PST_OPT_SWEEP_BATCHED = 5,
    PST_OPT_ANCHOR_EVERY = 6,
    PST_OPT_TUNE_GEOMETRY = 7,
    PST_OPT_SWEEP_ONE_LAUNCH = 8
};
int pst_set_option(pst_ctx *ctx, int option, int64_t value);

/* Tile geometry of the profile kernel (the parallel decomposition of eqs.
 * 9-13 on the GPU: workgroup size, diagonals per thread, rows per chunk,
 * selection threads, sub-tile width), per w = m-l+1, as one code: threads/256
 * << 24 | diagonals << 16 | rows << 8 | selection threads/256 << 4 |
 * sub-tile windows/992.  The choice is process-wide and applies to every
 * entry point; every workspace size already covers any candidate.  Geometries agree
 * within the profile tolerance, not bit for bit (each sub-tile anchors its
 * diagonals afresh), so change one only between calls, not while others run.
 * pst_geometry_candidates writes up to max codes the kernels can run for w and
 * returns how many there are; pst_geometry returns the code in use;
 * pst_set_geometry installs a candidate (0 restores the built-in choice;
 * PST_EINVAL for a code that is not a candidate).  pst_tune_geometry times
 * every candidate on the same segments of T (as many as give about sixteen
 * tiles per resident workgroup; best of three launches; workspace as
 * pst_workspace_bytes(n, m, l, 1)),
 * installs the fastest and returns its code and launch time; the choice is
 * remembered per (GPU architecture, w) in the process and, if
 * PST_AUTOTUNE_CACHE names a file, there ("geo arch w code ms" lines), and
 * reused without timing. */
int pst_geometry_candidates(int32_t w, int32_t *codes, int32_t max);
int32_t pst_geometry(int32_t w);
int pst_set_geometry(int32_t w, int32_t code);
int pst_tune_geometry(pst_ctx *ctx, const double *T_dev, int64_t n, int32_t m, int32_t l, int32_t *code_out,
                      float *ms_out, void *ws_dev, size_t ws_bytes);

/* Instrumentation.  With timing on, the profile kernel launched by each call
 * (eqs. 9-13, the dominant cost) is bracketed by two HIP events recorded on the
 * context's stream.  pst_last_profile_ms waits for the second event and
 * returns the kernel's duration in milliseconds; PST_ENOTREADY if no call has
 * been timed since timing was switched on. */
int pst_set_timing(pst_ctx *ctx, int on);
int pst_last_profile_ms(pst_ctx *ctx, float *ms);

#ifdef __cplusplus
}
#endif

#endif /* PST_H */
