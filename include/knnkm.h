/*
 * knnkm.h — C ABI of the MI355X (gfx950) library for KNN-graph-supported
 * k-means (C.-H. Deng and W.-L. Zhao, "Fast k-means based on KNN Graph",
 * arXiv 1705.01813).
 *
 * Problem statement (Sec. 1, Eqn. 1): n samples x_i in R^d and an integer k;
 * minimise the sum of squared distances from every sample to the centroid of
 * its cluster.  The method (Sec. 4) restricts each sample's nearest-centroid
 * search to the clusters its kappa graph neighbours belong to (Alg. 2), and
 * builds that graph by repeatedly clustering the data into small clusters of
 * about xi samples and comparing all pairs inside each one (Alg. 3).
 *
 * Conventions for every entry point
 *  - X is float32, row-major, n rows of d values with leading dimension
 *    ldx >= d (elements).  Sample ids and cluster labels are int32, so
 *    n <= 2^31-1; sizes are int64.
 *  - All pointers named X, C, G_ids, G_d2, labels*, counts, sums, best_d2,
 *    n_moved, E are DEVICE pointers on the context's device, owned by the
 *    caller, contiguous.  Pointers named *_host are host memory.
 *  - Distances are squared L2 (Eqn. 1, Eqn. 4).  Graph rows hold kappa
 *    (id, d2) entries ordered by (d2, id) ascending; d2 is the float32
 *    rounding of the pair's squared distance.
 *  - Kernel-level calls (knn_assign, centroid_update, distortion,
 *    knnkm_graph_init, knn_graph_search) are asynchronous on the context's
 *    HIP stream.  knnkm_twomeans (when its cached split plan does not match
 *    the call), knnkm_graph_refine (it reads the sizes of clusters above 128
 *    members back to the host) and knn_build (both, and the small host
 *    tables it uploads) synchronise the stream on the way.  knn_kmeans_fit
 *    synchronises the stream before returning because it writes host
 *    memory.
 *  - Every call returns a knnkm_status; nothing throws or aborts across the
 *    ABI.  Arguments are validated on the host before any launch; on a
 *    non-OK status the outputs are unspecified and knnkm_last_error() holds a
 *    message.  A HIP runtime error makes the context unusable
 *    (KNNKM_EDEVICE is sticky).
 *  - The library owns only its context workspace (device memory grown on
 *    demand, released by knnkm_destroy).
 */
#ifndef KNNKM_H
#define KNNKM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KNNKM_OK = 0,
  KNNKM_EINVAL = 1,      /* invalid argument (checked before any launch) */
  KNNKM_ENOMEM = 2,      /* workspace allocation failed */
  KNNKM_EDEVICE = 3,     /* HIP runtime error; sticky for the context */
  KNNKM_EUNSUPPORTED = 4, /* valid request outside the implemented limits */
  KNNKM_EAGAIN = 5        /* knnkm_server_wait: the job has not finished yet */
} knnkm_status;

enum { KNNKM_FP32 = 0, KNNKM_BF16_RERANK = 1 };
enum { KNNKM_INIT_TWOMEANS = 0, KNNKM_INIT_RANDOM = 1, KNNKM_INIT_LABELS = 2 };

/* Limits of this implementation (KNNKM_EUNSUPPORTED beyond them). */
#define KNNKM_MAX_D 512     /* dimensions per sample */
#define KNNKM_MAX_KAPPA 128 /* neighbours per graph row */

typedef struct {
  uint32_t struct_size; /* sizeof(knnkm_params) */
  int32_t kappa;        /* graph width kappa (Alg. 2 / Alg. 3); paper default 50 (Sec. 4.4) */
  int32_t xi;           /* cluster size of graph construction (Sec. 4.3); default 50 */
  int32_t tau;          /* graph construction rounds (Alg. 3); default 10 */
  int32_t bisect_iters; /* Lloyd 2-means steps per bisection of Alg. 1; default 2 */
  int32_t precision;    /* KNNKM_FP32 or KNNKM_BF16_RERANK (pair filter of knn_build) */
  int32_t init;         /* KNNKM_INIT_TWOMEANS (Alg. 2 start), KNNKM_INIT_RANDOM, or
                           KNNKM_INIT_LABELS (knn_kmeans_fit only: resume) */
  int32_t max_iters;    /* fit iterations T; the paper runs 30 (Sec. 5.4) */
  int32_t early_stop;   /* 1: stop after an iteration that moved no sample (Sec. 1 convergence) */
  uint64_t seed;        /* keys every random draw (graph init, bisection seeds, random init) */
} knnkm_params;

typedef struct knnkm_ctx knnkm_ctx;

/* Create a context on HIP device `device`, launching on `hip_stream`
 * (a hipStream_t, or NULL for the null stream).  device = -1 creates a dry
 * context that validates arguments and returns before any device work. */
knnkm_status knnkm_create(int device, void* hip_stream, knnkm_ctx** out);
knnkm_status knnkm_destroy(knnkm_ctx* ctx);
/* Switch the launch stream of an existing context. */
knnkm_status knnkm_set_stream(knnkm_ctx* ctx, void* hip_stream);
/* Message of the last failed call on ctx; with ctx = NULL, of the last failed
 * knnkm_create on this thread.  Owned by the library. */
const char* knnkm_last_error(const knnkm_ctx* ctx);
knnkm_status knnkm_default_params(knnkm_params* p);
/* Device bytes currently held by the context workspace. */
knnkm_status knnkm_workspace_bytes(const knnkm_ctx* ctx, int64_t* out);
/* Planning estimate (host only, no context): an upper estimate of the
 * workspace that knn_build followed by knn_kmeans_fit of one job of n rows
 * of d dimensions into k clusters with params grows a fresh context to
 * (the serving form charges its batches with the same formula).  Inputs and
 * outputs (X, graph, labels, centroids, counts) are the caller's and not
 * included.  KNNKM_EINVAL on out-of-range arguments. */
knnkm_status knnkm_workspace_estimate(int64_t n, int32_t d, int32_t k, const knnkm_params* params, int64_t* out);

/* Graph-restricted assignment, one Jacobi sweep (Alg. 2 candidate collection,
 * Lloyd form of Sec. 4.2 "GK-means^-").
 *  Q_i = {labels_in[i]} U {labels_in[G_ids[i*kappa + j]] : j < kappa}; if
 *  kappa >= k, Q_i = {0..k-1}.  labels_out[i] = the closest centroid in Q_i;
 *  the sample stays unless some candidate is strictly closer, and among equal
 *  minima the smallest id wins.  Decisions are exact up to float64 rounding
 *  (float32 evaluation, float64 re-evaluation of near ties).  When Q_i holds
 *  only the sample's own cluster it stays without a distance being
 *  evaluated, unless best_d2 is requested.
 *  C: k x d float32, row-major (leading dimension d).  G_ids: n x kappa int32
 *  with ids in [0,n).  labels_in must not alias labels_out.
 *  best_d2 (nullable): n floats, squared distance to the chosen centroid.
 *  n_moved (nullable, device int64): receives the number of i with
 *  labels_out[i] != labels_in[i] (overwritten, not accumulated).
 *  G_ids may be NULL when kappa >= k. */
knnkm_status knn_assign(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                        const float* C, int32_t k, const int32_t* G_ids, int32_t kappa,
                        const int32_t* labels_in, int32_t* labels_out, float* best_d2,
                        int64_t* n_moved);

/* Centroid update (Sec. 1: each centroid becomes the average of its
 * members; Eqn. 2 composite vectors D_r).  counts[r] = n_r; sums (nullable)
 * receives D_r as float64 k x d; C[r] (in: previous centroids, out: new) is
 * the float64 mean rounded to float32, and is left unchanged when n_r = 0.
 * Labels must lie in [0,k). */
knnkm_status centroid_update(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                             const int32_t* labels, int32_t k, float* C, int32_t* counts,
                             double* sums);

/* Average distortion, Eqn. 4: E = sum_i ||x_i - C_{labels[i]}||^2 / n,
 * evaluated in float64 with a fixed reduction order; *E (device double). */
knnkm_status distortion(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                        const float* C, int32_t k, const int32_t* labels, double* E);

/* distortion without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and bits as distortion(); its
 * partial sums live in a fixed 4 MiB device array of the library (one copy
 * per device, held until the process ends, its address resolved once per
 * device by knnkm_create) instead of the context workspace, and it calls no
 * allocating routine.  Requires n <= 134,201,344 (KNNKM_EUNSUPPORTED beyond,
 * before any launch).  Calls that overlap on one device share that array and
 * race: serialise them (one stream, or events between streams). */
knnkm_status distortion_noalloc(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                const float* C, int32_t k, const int32_t* labels, double* E);

/* Two-means tree, Alg. 1: labels in [0,k) from a level-synchronous balanced
 * bisection.  Every split seeds two centroids from two distinct members
 * (counter-based draws keyed by seed, round_tag and the node), runs
 * bisect_iters Lloyd 2-means steps, then orders the members by
 * delta = ||x-c_u||^2 - ||x-c_v||^2 (ties by id) and gives the first
 * ceil(s/2) to the left child.  Leaves are numbered left to right.
 * round_tag: 0..tau-1 for the calls inside knn_build, 0xFFFF for the fit. */
knnkm_status knnkm_twomeans(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                            int32_t k, uint64_t seed, int32_t round_tag, int32_t bisect_iters,
                            int32_t* labels);

/* Random initial KNN lists (Alg. 3 initialisation): row i holds kappa
 * distinct ids != i (Floyd's sampling on a counter-based stream keyed by
 * seed and i), with their squared distances, ordered by (d2, id).
 * Requires 1 <= kappa <= n-1. */
knnkm_status knnkm_graph_init(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                              int32_t kappa, uint64_t seed, int32_t* G_ids, float* G_d2);

/* Alg. 3 inner loops for one partition: for every cluster S_m of `labels`
 * (values in [0,k)), every pair <i,j> of S_m updates G[i] and G[j]: a pair
 * whose id is not yet in the row enters it if its (d2, id) is among the
 * kappa smallest.  Clusters of at most 32 members and of more than 1024:
 * pair distances screened on MFMA (float32, or bfloat16 with precision =
 * KNNKM_BF16_RERANK) with a rigorous error margin against the row's current
 * kappa-th distance, survivors re-evaluated exactly; 33-1024 members: every
 * pair's key from a float64 Gram on MFMA, certified or recomputed from the
 * rows.  Both precisions give identical graphs.  G_ids/G_d2 are updated in
 * place.  Synchronises the stream once (see above). */
knnkm_status knnkm_graph_refine(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                const int32_t* labels, int32_t k, int32_t precision,
                                int32_t* G_ids, float* G_d2, int32_t kappa);

/* KNN graph construction, Alg. 3: random initial lists, then tau rounds of
 * {TwoMeans into k0 = max(1, floor(n/xi)) clusters; one GK-means^- sweep
 * with the current graph; exhaustive comparison inside each cluster}.
 * Uses params->kappa, xi, tau, bisect_iters, precision, seed.
 * G_ids: n x kappa int32, G_d2: n x kappa float32 (outputs). */
knnkm_status knn_build(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                       const knnkm_params* params, int32_t* G_ids, float* G_d2);

/* GK-means^- fit (Alg. 2, Lloyd form): initial labels from Alg. 1 (or, with
 * init = KNNKM_INIT_RANDOM, k distinct rows as seeds and an exhaustive
 * assignment), C_0 = their means; then for t = 1..max_iters: knn_assign with
 * G_ids, centroid update, distortion.  trace_host (max_iters+1 doubles, host)
 * receives E_0..E_T (Eqn. 4); iters_run_host the number of sweeps done.
 * Outputs labels (n), C (k x d), counts (k) on the device.  Synchronous.
 * Resume: with init = KNNKM_INIT_LABELS the fit starts from the partition
 * held in labels (input and output; every entry in [0, k), else
 * KNNKM_EINVAL) and keeps the centroids in C of the clusters that partition
 * leaves empty; C_0 is the means of the others.  A fit of T1 sweeps followed
 * by one of T2 sweeps from its labels and C continues it: the same labels,
 * centroids and counts as one fit of T1 + T2 sweeps (its trace continues
 * from E_T1), up to the float64 summation order of the rebuilt sums. */
knnkm_status knn_kmeans_fit(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                            int32_t k, const int32_t* G_ids, const knnkm_params* params,
                            int32_t* labels, float* C, int32_t* counts, double* trace_host,
                            int32_t* iters_run_host);

/* Boost form of the fit (Alg. 2 as printed, Sec. 3.1 / Eqn. 3), in
 * data-parallel rounds.  Alg. 2 moves a sample from its cluster u to the
 * cluster v of its kappa neighbours that maximises the gain of
 * I = sum_r D_r'D_r / n_r (Eqn. 2) when that gain is positive; here that
 * gain is n_u/(n_u-1)|x - c_u|^2 - n_v/(n_v+1)|x - c_v|^2 (Eqn. 3 rewritten;
 * 0 for the first term when the move empties u), c_r the float64 mean of the
 * exact sum D_r.  A round: every sample finds its best move against the same
 * state (the smallest weighted distance n_v/(n_v+1)|x - c_v|^2 over the
 * clusters of its graph row other than u, smallest id among equal ones;
 * proposed when the own weighted distance is strictly larger); each cluster
 * keeps, among the proposals touching it, the one with the largest priority
 * (a counter-based draw of (params->seed, round, sample) in the high 32 bits,
 * the sample id in the low 32); the proposals that keep both their clusters
 * move.  No two moves of a round share a cluster, so I rises by exactly the
 * sum of their gains (the round equals the same moves made one by one).
 * Rounds stop after one with no proposal or after params->max_iters rounds
 * (at most 65535).  Initial partition as knn_kmeans_fit (params->init,
 * including KNNKM_INIT_LABELS).  Outputs labels (n), C (k x d, the float32
 * means; clusters left empty keep the initial centroid), counts (k);
 * trace_host (max_iters + 1 doubles) receives E_0..E_t (Eqn. 4);
 * rounds_run_host the rounds done.  G_ids: n x kappa, required;
 * n * kappa < 2^31 (else KNNKM_EUNSUPPORTED).  Synchronous (one host read
 * per round). */
knnkm_status knn_boost_fit(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, int32_t k,
                           const int32_t* G_ids, const knnkm_params* params, int32_t* labels, float* C,
                           int32_t* counts, double* trace_host, int32_t* rounds_run_host);

/* Approximate nearest neighbours of query rows by best-first search over a
 * KNN graph (Sec. 4.3: the graph of Alg. 3 also serves this search; the paper
 * gives no algorithm, this is the usual beam search).  Per query: a sorted
 * list of at most ef entries (d2, id), seeded with n_entry distinct entry
 * points (Floyd's sampling keyed by seed and the query index); the first
 * entry not yet expanded is expanded -- its graph neighbours not seen before
 * get their distances and are merged in, the list keeping its ef smallest --
 * until every entry is expanded or max_visits points have been looked at
 * (an expansion in progress completes).  Points are ordered by (d2, id); d2
 * is the float32 rounding of the float64 squared distance summed over the
 * dimensions in order.  Outputs (device): out_ids / out_d2, m x top_k
 * (-1 / +inf past the end of a short list).  X: n x d (leading dimension
 * ldx), G_ids: n x kappa, Q: m x d (leading dimension ldq), all device.
 * Limits: ef <= KNNKM_SEARCH_MAX_EF, max_visits <= KNNKM_SEARCH_MAX_VISITS,
 * n_entry <= KNNKM_SEARCH_MAX_ENTRY (KNNKM_EINVAL beyond).  Above 1,920
 * visits the tables of visited points live in the context's workspace
 * (64 KB for each query in flight: 512 MB with 256 compute units; KNNKM_ENOMEM
 * if it cannot grow).  Asynchronous. */
#define KNNKM_SEARCH_MAX_EF 128
#define KNNKM_SEARCH_MAX_VISITS 7680
#define KNNKM_SEARCH_MAX_ENTRY 16
knnkm_status knn_graph_search(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                              const int32_t* G_ids, int32_t kappa, const float* Q, int64_t m, int64_t ldq,
                              int32_t ef, int32_t top_k, int32_t max_visits, int32_t n_entry, uint64_t seed,
                              int32_t* out_ids, float* out_d2);

/* Batching form: m independent jobs (graph build and fit, Alg. 3 then Alg. 2)
 * in one call, every phase one launch over all jobs.
 *  X: the jobs' rows concatenated; job q owns rows [n_off_host[q],
 *     n_off_host[q+1]) (host int64 array of m+1 entries, n_off_host[0] = 0)
 *     and needs kappa + 1 <= n_q rows; k_host[q] clusters (host int32);
 *     seeds_host[q] keys its random draws (params->seed is not used).
 *  Outputs (device): G_ids / G_d2 (sum n_q) x kappa with global row ids;
 *  labels (sum n_q) job-local cluster ids; C (sum k_q) x d and counts (sum
 *  k_q), job q's clusters after those of jobs 0..q-1; trace_host (host,
 *  m x (max_iters+1)): E_0..E_T of job q at row q.  early_stop is ignored.
 *  Each job's results are bit-identical to running it alone through
 *  knn_build + knn_kmeans_fit with its seed.  init = KNNKM_INIT_LABELS is
 *  not accepted (KNNKM_EINVAL).  Synchronous. */
knnkm_status knnkm_fit_batched(knnkm_ctx* ctx, const float* X, int32_t d, int64_t ldx, int32_t m,
                               const int64_t* n_off_host, const int32_t* k_host,
                               const uint64_t* seeds_host, const knnkm_params* params, int32_t* G_ids,
                               float* G_d2, int32_t* labels, float* C, int32_t* counts,
                               double* trace_host);

/* ------------------------------------------------------------ serving form --
 * A request loop over one device.  Jobs (each a graph build plus a fit, as
 * knn_build + knn_kmeans_fit) are submitted from any host thread and return
 * at once with a ticket.  `slots` worker threads, each with its own context
 * and non-blocking HIP stream, take the queued jobs in arrival order: a free
 * worker forms a batch from the oldest queued job and every later queued job
 * of the same class (same d and the same params apart from seed), within
 * max_batch_jobs / max_batch_rows and the HBM budget, copies their rows into
 * device memory it allocates for the batch, runs them through
 * knnkm_fit_batched (one launch per phase for the whole batch), copies the
 * results to the jobs' host buffers and frees the batch's device memory.
 * Batches of different workers overlap on the device, and jobs that arrive
 * while batches run join the next batch a worker forms as soon as a slot and
 * budget free up (continuous batching at batch granularity).
 *
 * Admission: a job's footprint is its device buffers (rows, graph, labels,
 * centroids, counts) plus a workspace estimate; the sum over running batches
 * plus the workspace each worker keeps must stay within hbm_budget_bytes.
 * The oldest queued job is never overtaken by a job of another class, so a
 * large job cannot starve; when it does not fit, workers wait (idle workers
 * first release their workspace).  A job that does not fit the budget even
 * alone is rejected at submit (KNNKM_ENOMEM).
 *
 * Results: each job's labels, centroids, counts, graph and distortion trace
 * are bit-identical to running it alone through knnkm_fit_batched with m = 1
 * (and to knn_build + knn_kmeans_fit with params.seed = its seed).
 */
typedef struct knnkm_server knnkm_server;

typedef struct {
  uint32_t struct_size;     /* sizeof(knnkm_server_config) */
  int32_t device;           /* HIP device; -1: a dry server that validates and
                               schedules but runs nothing and writes no output */
  int32_t slots;            /* batches in flight at once, 1..16 */
  int32_t max_batch_jobs;   /* jobs per batch, >= 1 */
  int64_t max_batch_rows;   /* rows per batch, >= 1 (a larger job runs alone) */
  int64_t hbm_budget_bytes; /* device memory the server may hold, > 0 */
} knnkm_server_config;

typedef struct {
  uint32_t struct_size; /* sizeof(knnkm_job) */
  int32_t d;            /* dimensions, 1..KNNKM_MAX_D */
  int64_t n;            /* samples, kappa + 1 <= n < 2^31 */
  int64_t ldx;          /* row stride of X_host in elements, >= d */
  const float* X_host;  /* host rows; read until the job completes */
  int32_t k;            /* clusters, 1 <= k <= n */
  int32_t pad_;
  knnkm_params params;  /* kappa, xi, tau, bisect_iters, precision, init,
                           max_iters, seed (early_stop is not used) */
  /* host outputs, written before the job completes; may be null */
  int32_t* labels_host; /* n, cluster ids 0..k-1 */
  float* C_host;        /* k x d */
  int32_t* counts_host; /* k */
  int32_t* G_ids_host;  /* n x kappa, row ids 0..n-1 */
  double* trace_host;   /* max_iters + 1: E_0..E_T (Eqn. 4) */
} knnkm_job;

typedef struct {
  int32_t status;          /* knnkm_status of the job */
  int32_t slot;            /* worker that ran it */
  int64_t batch;           /* serial number of its batch */
  int32_t batch_jobs;      /* jobs in that batch */
  int32_t pad_;
  int64_t footprint_bytes; /* bytes charged to the budget for this job */
  double t_submit;         /* seconds on the server clock (monotonic, 0 at create) */
  double t_admit;          /* batch formed */
  double t_done;           /* outputs in host memory */
} knnkm_job_info;

typedef struct {
  int64_t submitted, completed, failed, rejected;
  int64_t batches;          /* batches run */
  int64_t queued;           /* waiting for admission now */
  int64_t running;          /* admitted, not finished */
  int64_t max_queued;       /* largest queue seen */
  int64_t max_batch_jobs_seen;
  int64_t bytes_in_use;     /* charged now (running batches + kept workspace) */
  int64_t bytes_peak;       /* largest charge seen */
  int64_t ws_overruns;      /* batches whose workspace exceeded its estimate */
} knnkm_server_stats;

/* Start the workers.  The server owns its contexts, streams and threads. */
knnkm_status knnkm_server_create(const knnkm_server_config* config, knnkm_server** out);
/* Validate and queue a job (the job struct is copied; X_host and the output
 * buffers must stay valid until knnkm_server_wait has returned for it).
 * *ticket identifies it.  Thread-safe. */
knnkm_status knnkm_server_submit(knnkm_server* srv, const knnkm_job* job, uint64_t* ticket);
/* Wait up to timeout_ms (< 0: no limit) for a job.  Returns KNNKM_EAGAIN if
 * it has not finished, else the job's own status, fills *info (may be null)
 * and forgets the ticket.  Thread-safe. */
knnkm_status knnkm_server_wait(knnkm_server* srv, uint64_t ticket, int64_t timeout_ms,
                               knnkm_job_info* info);
knnkm_status knnkm_server_stats_get(knnkm_server* srv, knnkm_server_stats* out);
/* Message of the last failed server call made by the calling thread. */
const char* knnkm_server_last_error(void);
/* Run every queued job to completion, stop the workers, free everything. */
knnkm_status knnkm_server_destroy(knnkm_server* srv);

/* Replay of the fit iterations from a HIP graph (default on).  Without
 * early stopping, knn_kmeans_fit and knnkm_fit_batched run the first two
 * sweeps eagerly and capture two sweeps (assignment, update, distortion)
 * once into a graph that is launched for the remaining pairs; results are the
 * same with graphs on or off.  A capture that fails falls back to eager
 * launches. */
knnkm_status knnkm_enable_graphs(knnkm_ctx* ctx, int32_t on);

/* Active sets in the fit sweeps (default on; graph fits with n * kappa below
 * 2^31).  A sample whose own cluster was its only candidate stays so until
 * its own label or a neighbour's label changes, so from the second sweep on
 * knn_kmeans_fit and knnkm_fit_batched evaluate only the samples that had
 * several candidates, moved, or have a neighbour that moved (found through
 * reverse lists of the graph, built once per fit) and copy the other
 * labels.  Results are the same bits with active sets on or off. */
knnkm_status knnkm_enable_active_sets(knnkm_ctx* ctx, int32_t on);

/* Subtree finishing in the two-means tree of Alg. 1 (default on).  Once a
 * node to split has at most R members, one block performs every later split
 * of its subtree (seeds, the Lloyd 2-means steps, the ordering by delta and
 * the balanced split) with the member ids held on chip, instead of one launch
 * per step per depth.  Every step keeps the same arithmetic and order, so
 * labels from knnkm_twomeans, knn_build and knn_kmeans_fit are the same bits
 * with it on or off and for every R.  on: 0 off, 1 on with R = 1,024, or R
 * itself (2..1,024).  Returns KNNKM_EINVAL for a null context or another
 * value. */
knnkm_status knnkm_enable_subtree_finish(knnkm_ctx* ctx, int32_t on);

/* Autotuner of the assignment's launch shapes (default on): the first call
 * with at least 65,536 samples for a given group shape, size bin and call
 * site (a direct knn_assign call, a graph-construction round, the fit's first
 * sweep, later fit sweeps) times every candidate shape once (samples per row
 * group and pass, samples per block, rows loaded first or lazily) on that
 * call's own data, synchronising the stream, and keeps the fastest for the
 * process.  Every shape gives the same results. */
knnkm_status knnkm_autotune(knnkm_ctx* ctx, int32_t on);
/* Early-abandoned partial distances in the assignment for wide rows
 * (256 < d <= 512, kappa <= 63).  Each sample is handled by one wavefront:
 * an upper bound of the distance to its closest candidate comes first (full
 * distances of the own centroid and of the nearest entry's cluster, or in
 * the fit's sweeps on active sets the drift bound of the own centroid), and
 * every candidate is summed 64 dimensions at a time and dropped once a
 * rigorous lower bound of its distance over those dimensions exceeds it; the
 * survivors get full float32 distances (float64 near ties).  on: 0 off, 1 on
 * (default), the sweeps of the graph build, of the fit and of knn_assign
 * (which forms it from C on each call) reading a shadow of the centroids in
 * 8-bit codes for the partial sums (a quarter of the bytes; one code step per
 * row, its largest magnitude / 127; the bound accounts for each shadow row's
 * distance to its float32 row), 2 on with the float32 centroids only, 3 on
 * with a bfloat16 shadow (half the bytes).  Decisions
 * (labels, moved counts, active-set flags) are the same in every mode;
 * calls that request best_d2 use the full-distance kernels.  Other values:
 * KNNKM_EINVAL. */
knnkm_status knnkm_enable_partial_distances(knnkm_ctx* ctx, int32_t on);

/* Fix the assignment's launch shape for this context (overrides the
 * autotuner): gs samples per row group and pass, pb samples per block (64 or
 * 128), lazy = 1 to load a sample's row only when a distance is needed (after
 * its neighbour labels are known; gs 1 or 2) or 0 to load it first (gs 1, 2
 * or 4).  gs = 0 returns to the automatic choice.  Results do not depend on
 * the shape.  KNNKM_EINVAL for any other combination. */
knnkm_status knnkm_set_assign_shape(knnkm_ctx* ctx, int32_t gs, int32_t pb, int32_t lazy);
/* The process-wide table of tuned shapes as text (one line per entry) into
 * buf (len bytes, NUL-terminated, truncated); *needed gets the full size. */
knnkm_status knnkm_autotune_table(char* buf, int64_t len, int64_t* needed);

/* Opt-in phase timing.  With on = 1, knn_build and knn_kmeans_fit record HIP
 * events on the context stream around their phases (a few microseconds of
 * overhead); with on = 2 they also record events around every assignment
 * launch of the fit, whose sweeps then run eagerly (no graph).
 * knnkm_phase_times waits for those events and writes up to `count` values
 * (milliseconds unless noted), -1 where a phase was not recorded:
 *   out[0] last knn_build, start to end
 *   out[1] last knn_kmeans_fit initialisation (partition, means, E_0, the
 *          working copy of the data in cluster order)
 *   out[2] last knn_kmeans_fit iterations (assign + update + distortion)
 *   out[3] sum of the timed assignment launches of those iterations (on = 2)
 *   out[4] iterations run (count), out[5] assignment launches timed (count)
 *   out[6] samples whose candidate distances those launches evaluated, summed
 *          (count; a sample whose neighbours all share its cluster has its
 *          own cluster as the only candidate and needs none) (on = 2)
 *   out[7] samples those launches looked at, summed (count; all of them in
 *          the first sweep, the active set after it) (on = 2) */
knnkm_status knnkm_enable_timing(knnkm_ctx* ctx, int32_t on);
knnkm_status knnkm_phase_times(knnkm_ctx* ctx, double* out, int32_t count);

/* Per-sweep record of the last knn_kmeans_fit on ctx (count >= 0 entries per
 * array, host memory, each array may be null; *n_out = the sweeps written,
 * min(count, sweeps run)).  Entry j is sweep j+1:
 *   assign_ms  duration of its assignment launches (timing level 2, else -1)
 *   listed     samples the assignment looked at (timing level 2, else -1)
 *   evaluated  samples whose candidate distances it evaluated (level 2, else -1)
 *   moved      samples whose label changed (every fit of one job)
 * Waits for the context stream. */
knnkm_status knnkm_sweep_stats(knnkm_ctx* ctx, double* assign_ms, int64_t* listed, int64_t* evaluated,
                               int64_t* moved, int32_t count, int32_t* n_out);

/* Counter-based generator used for every random draw of the method
 * (SplitMix64 output function applied to key + (ctr+1)*0x9E3779B97F4A7C15,
 * key = mix(seed ^ mix(stream))).  Writes out[c] = draw(ctr0 + c) for
 * c < count into a device uint64 buffer.  Exposed so both implementations of
 * the generator can be compared. */
knnkm_status knnkm_rng_draw(knnkm_ctx* ctx, uint64_t seed, uint64_t stream, uint64_t ctr0,
                            int64_t count, uint64_t* out);

#ifdef __cplusplus
}
#endif
#endif /* KNNKM_H */
