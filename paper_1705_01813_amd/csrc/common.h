// Shared host/device definitions of the knnkm HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/knnkm.h"

// ------------------------------------------------------------------ context --

struct knnkm_buf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct knnkm_ctx {
  int device = -1;
  bool dry = false;
  hipStream_t stream = nullptr;
  bool sticky = false;
  std::string err;
  int num_cus = 256;
  std::unordered_map<std::string, knnkm_buf> ws;  // named workspace buffers
  // cached two-means tree metadata (depends on the job sizes and leaf
  // counts only): two plans, so that a build's (k0 leaves) and a fit's (k
  // leaves) both stay; the least recently used one is replaced
  struct TMPlan* tm_plan[2] = {nullptr, nullptr};
  uint64_t tm_plan_used[2] = {0, 0};
  uint64_t tm_plan_clock = 0;
  // opt-in phase timing (HIP events on the context stream)
  int timing = 0;  // 1: phases; 2: also every assignment of the fit (sweeps run eagerly)
  std::vector<hipEvent_t> ev;  // pool
  int build_ev = -1;           // index of the build start event (end = +1)
  int fit_ev = -1;             // fit start, init end, iterations end = +0, +1, +2
  int assign_ev0 = -1, assign_n = 0;  // pairs around the assignment launches of the fit
  int fit_iters = 0;                  // sweeps of the last fit
  const int64_t* fit_evals = nullptr;  // per-sweep evaluated-sample counts of the last timed fit (device)
  const int64_t* fit_actives = nullptr;  // per-sweep listed-sample counts of the last timed fit (device)
  const int64_t* fit_moved = nullptr;    // per-sweep moved-sample counts of the last fit (device)
  // fit iterations replayed from a captured HIP graph (captured on a private
  // stream, launched on `stream`)
  bool graphs = true;
  // launch shapes of the assignment chosen by timing the candidates once
  bool autotune = true;
  bool active_sets = true;  // fit sweeps look only at samples that can change
  bool wide_pd = true;      // wide rows: early-abandoned partial distances in the assignment
  // ... reading a shadow of the centroids in the build and fit sweeps (the
  // CShadow kinds: 0 none, the float32 rows; 1 bfloat16; 2 8-bit codes)
  int pd_shadow = 2;
  int tm_finish_max = 1024;  // two-means subtrees up to this size finished by one block (0: off)
  int assign_gs = 0, assign_pb = 64, assign_lazy = 0;  // forced assignment shape (gs = 0: automatic)
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  bool capturing = false;
  hipStream_t cap_stream = nullptr;
};
// Event `i` of the context pool (created on first use); nullptr on failure.
hipEvent_t knnkm_event(knnkm_ctx* ctx, int i);
void tm_plan_free(struct TMPlan* p);

// Set the context error and return the status.
knnkm_status knnkm_fail(knnkm_ctx* ctx, knnkm_status st, const char* fmt, ...);
// Device buffer of at least `bytes` bytes, grown on demand (contents are not
// preserved across growth).  Returns nullptr and sets ENOMEM on failure.
void* knnkm_ws(knnkm_ctx* ctx, const char* name, size_t bytes);
// Release every workspace buffer (after the work queued on the context stream).
knnkm_status knnkm_ws_release(knnkm_ctx* ctx);
// Check the HIP status of the last launches; sets the sticky error.
knnkm_status knnkm_check(knnkm_ctx* ctx, const char* where);

#define KNNKM_TRY(expr)                         \
  do {                                          \
    knnkm_status _st = (expr);                  \
    if (_st != KNNKM_OK) return _st;            \
  } while (0)

#define KNNKM_HIP(ctx, expr)                                                           \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) {                                                            \
      (ctx)->sticky = true;                                                            \
      return knnkm_fail((ctx), KNNKM_EDEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
    }                                                                                  \
  } while (0)

#define KNNKM_WS(ctx, var, type, name, count)                                      \
  type* var = (type*)knnkm_ws((ctx), (name), sizeof(type) * (size_t)(count));      \
  if (!(var)) return KNNKM_ENOMEM

// ---------------------------------------------------------- random numbers --
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output c of a generator with
// state `key` is mix(key + (c+1) * GAMMA).  Keys: mix(seed ^ mix(stream)).
#define KNNKM_GAMMA 0x9E3779B97F4A7C15ull
enum { RNG_GRAPH_INIT = 1, RNG_TWOMEANS = 2, RNG_RANDOM_INIT = 3 };
#define KNNKM_ROUND_FIT 0xFFFF

__host__ __device__ inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm_stream(uint64_t purpose, uint64_t round, uint64_t index) {
  return (purpose << 56) | ((round & 0xFFFFull) << 40) | (index & ((1ull << 40) - 1));
}
__host__ __device__ inline uint64_t sm_key(uint64_t seed, uint64_t stream) {
  return sm_mix(seed ^ sm_mix(stream));
}
__host__ __device__ inline uint64_t sm_draw(uint64_t key, uint64_t ctr) {
  return sm_mix(key + (ctr + 1) * KNNKM_GAMMA);
}
// Integer in [0, m) from the high 32 bits (multiply-shift, no rejection).
__host__ __device__ inline uint32_t sm_below(uint64_t r, uint32_t m) {
  return (uint32_t)(((r >> 32) * (uint64_t)m) >> 32);
}

// --------------------------------------------------------- wave utilities --
#define WAVE 64

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ inline float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
  return v;
}
// float32 not below a non-negative double (an upper bound kept in float32):
// the next float32 up is the next bit pattern for non-negative values
__device__ inline float f32_round_up(double v) {
  float f = (float)v;
  if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);
  return f;
}
// float32 -> bfloat16 bit pattern, round to nearest even (finite values)
__device__ inline uint16_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
// float32 not above a non-negative double (0 for v <= 0)
__device__ inline float f32_round_down(double v) {
  if (v <= 0.0) return 0.f;
  float f = (float)v;
  if ((double)f > v) f = __uint_as_float(__float_as_uint(f) - 1u);
  return f;
}
__device__ inline int lane_id() { return threadIdx.x & (WAVE - 1); }
// flag r of a bit array (one bit per cluster)
__device__ inline bool bit_of(const uint32_t* __restrict__ bits, int r) { return (bits[r >> 5] >> (r & 31)) & 1u; }
__device__ inline uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

// Order-preserving map of a double to uint64 (+0 and -0 map to the same key).
__device__ inline uint64_t dkey(double v) {
  if (v == 0.0) v = 0.0;
  uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// Exclusive scan of one int per thread over a 256-thread block (all threads
// must call it); *total receives the block sum.  sh: 8 ints of LDS.
__device__ inline int32_t block_scan_excl_256(int32_t v, int32_t* sh /*[8]*/, int32_t* total) {
  // inclusive wave scan
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  int32_t base = 0, tot = 0;
  for (int j = 0; j < 4; ++j) {
    if (j < w) base += sh[j];
    tot += sh[j];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// Blocks per launch for grid-stride kernels.
inline int grid_for(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Low-precision copy of the centroid rows read by the early-abandon steps of
// the wide-row assignment; row r decodes to within eps[r] (Euclidean) of the
// float32 centroid.  kind 1: bfloat16 values (2 bytes per element); kind 2:
// 8-bit codes u standing for scale[r] * (u - 128) (1 byte per element).
struct CShadow {
  void* rows = nullptr;
  float* eps = nullptr;
  float* scale = nullptr;  // kind 2
  int kind = 0;            // 0: none
};

// 8-bit shadow of one centroid row by a whole wavefront: step s = (largest
// magnitude) / 127, codes u = 128 + clamp(rint(c / s), -127, 127) (128 for a
// zero row), and eps >= ||c - s (u - 128)|| (the products s (u - 128) are
// exact in float64).
__device__ inline void i8_shadow_row(const float* __restrict__ crow, int d, uint8_t* __restrict__ out,
                                     float* __restrict__ step, float* __restrict__ eps) {
  const int lane = threadIdx.x & 63;
  float amax = 0.f;
  for (int t = lane; t < d; t += 64) amax = fmaxf(amax, fabsf(crow[t]));
  amax = wave_max(amax);
  const float s = amax / 127.f;
  double e2 = 0.0;
  for (int t = lane; t < d; t += 64) {
    const float c = crow[t];
    const int q = s > 0.f ? (int)fminf(127.f, fmaxf(-127.f, rintf(c / s))) : 0;
    out[t] = (uint8_t)(q + 128);
    const double dq = (double)c - (double)s * (double)q;
    e2 = fma(dq, dq, e2);
  }
  e2 = wave_sum(e2);
  if (lane == 0) {
    *step = s;
    *eps = f32_round_up(sqrt(e2) * (1.0 + 0x1p-40));
  }
}

// ------------------------------------------------- internal building blocks --
// (defined in the .hip files; all enqueue on ctx->stream)

// Exclusive prefix sum of `count` int32 values (in may equal out); out[count]
// receives the total when `with_total`.
knnkm_status ks_scan_exclusive(knnkm_ctx* ctx, const int32_t* in, int32_t* out, int64_t count,
                               bool with_total);
// Stable sort of sample ids by label: offsets[k+1] and members[n] (ids of
// cluster r at members[offsets[r] .. offsets[r+1]), ascending).
knnkm_status ks_label_sort(knnkm_ctx* ctx, const int32_t* labels, int64_t n, int32_t k,
                           int32_t* counts, int32_t* offsets, int32_t* members);
// Segmented float64 sums over the CSR partition; means into C (unchanged
// where empty); Iterm[r] = ||D_r||^2 / n_r (0 where empty).
knnkm_status ks_segsum(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                       int32_t k, const int32_t* counts, const int32_t* offsets,
                       const int32_t* members, float* C, double* sums, double* Iterm,
                       float* delta = nullptr);
// Deterministic float64 sum of count values into *out (device).
knnkm_status ks_sum_f64(knnkm_ctx* ctx, const double* in, int64_t count, double* out);
// The same with the tile partials (ceil(count/8192) doubles when count >
// 65536) in a buffer the caller provides.
knnkm_status ks_sum_f64_with(knnkm_ctx* ctx, const double* in, int64_t count, double* part, double* out);
// Resolves, once per device (that device current), the device address of the
// fixed scratch array of the allocation-free calls.
knnkm_status ks_noalloc_setup(knnkm_ctx* ctx);
// Assignment kernel launcher (order: optional visiting order of samples;
// use: where the call comes from, a key of the tuned launch shapes).
enum { KS_USE_CALL = 0, KS_USE_BUILD = 1, KS_USE_FIT_FIRST = 2, KS_USE_FIT = 3 };
knnkm_status ks_assign(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                       const float* C, int32_t k, const int32_t* G_ids, int32_t kappa,
                       const int32_t* labels_in, int32_t* labels_out, float* best_d2,
                       int64_t* n_moved, const int32_t* order, bool dense,
                       const int32_t* job_of = nullptr, const int32_t* kbase = nullptr, int use = KS_USE_CALL,
                       int64_t* n_eval = nullptr, const uint8_t* act_in = nullptr, uint8_t* act_out = nullptr,
                       int64_t* n_active = nullptr, int32_t* list_count = nullptr,
                       int32_t* list_count_other = nullptr, bool zero_moved = true,
                       const int32_t* cdirty = nullptr, float* bnd_u = nullptr, float* bnd_lb = nullptr,
                       const float* cdelta = nullptr, CShadow sw = {}, const int32_t* nlab = nullptr);
// Exact keys and merge for clusters of RX_BIG_LO < s <= RX_BIG_HI members
// (tiled float64 Gram; counts/offsets/members as from ks_label_sort).  Reads
// the clusters' total size back to the host (one stream synchronisation) to
// size its key rows; *handled is false when it leaves those clusters to the
// screen path (inside a graph capture, or a launch too large); *above is
// false when no cluster has more than RX_BIG_HI members.
#define RX_BIG_LO 128
#define RX_BIG_HI 1024
knnkm_status ks_refine_big(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, int32_t kappa,
                           int32_t k, const int32_t* counts, const int32_t* offsets, const int32_t* members,
                           bool vec, int32_t* G_ids, float* G_d2, bool* handled, bool* above);
// Exact all-pairs refinement of the clusters with smin < s <= smax members
// (smax <= 128; one block per cluster, rows of the graph updated in place).
knnkm_status ks_refine_exact(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, int32_t kappa,
                             int32_t k, const int32_t* offsets, const int32_t* members, int32_t smin,
                             int32_t smax, bool vec, int32_t* G_ids, float* G_d2);
// Wide rows (256 < d <= 512, kappa <= 63): one wavefront per sample with
// early-abandoned partial distances.  list != null: the active-set sweep over
// the listed positions (list_count entries); else a full sweep in `order`
// (pb positions per block).  Same decisions and flags as the narrow kernels.
// sw: the shadow of C (ks_c_shadow) read for the early-abandon steps, or
// kind 0 (the float32 rows).
bool ks_assign_pd_ok(int32_t d, int32_t kappa);
// Workspace for the centroid shadow of the context's kind (kind 0: none) of
// K rows of d dimensions, under names starting with `tag`.
knnkm_status ks_shadow_alloc(knnkm_ctx* ctx, const char* tag, int32_t K, int32_t d, CShadow* sw);
// Shadow (kind 1 or 2) of the centroid rows of C, all or those with dirty[r]
// set, with its row bounds.
knnkm_status ks_c_shadow(knnkm_ctx* ctx, const float* C, int32_t K, int32_t d, const int32_t* dirty, CShadow sw);
knnkm_status ks_assign_pd(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, const float* C,
                          int32_t k, const int32_t* G_ids, int32_t kappa, const int32_t* labels_in,
                          int32_t* labels_out, unsigned long long* acc, unsigned long long* eacc,
                          const int32_t* order, const int32_t* job_of, const int32_t* kbase,
                          const uint8_t* act_in, uint8_t* act_out, const int32_t* list, const int32_t* list_count,
                          int64_t* n_listed, const uint32_t* cbits, int pb, float* bnd_u, float* bnd_lb,
                          const float* delta, CShadow sw = {}, const int32_t* nlab = nullptr);
knnkm_status ks_twomeans(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                         int32_t k, uint64_t seed, int32_t round_tag, int32_t iters,
                         int32_t* labels);
// TwoMeans of several independent jobs at once (job q: rows [off_q, off_q +
// n_q) in order, k_q leaves, seed seeds_dev[q] or seed1 when seeds_dev is
// null); labels are global leaf ids (job q's leaves follow job q-1's).
knnkm_status ks_twomeans_multi(knnkm_ctx* ctx, const float* X, int32_t d, int64_t ldx,
                               const std::vector<int64_t>& jn, const std::vector<int32_t>& jk,
                               const uint64_t* seeds_dev, uint64_t seed1, int32_t round_tag, int32_t iters,
                               int32_t* labels);
// Random lists; for a batch, job_of[i] / n_off / seeds give row i's job, the
// job's row range and its seed (ids stay global); null for one job.
knnkm_status ks_graph_init(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                           int32_t kappa, uint64_t seed, int32_t* G_ids, float* G_d2,
                           const int32_t* job_of = nullptr, const int64_t* n_off = nullptr,
                           const uint64_t* seeds = nullptr);
// norms: float32 squared norms of the rows, or null (computed here)
knnkm_status ks_refine(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                       const int32_t* labels, int32_t k, int32_t precision, int32_t* G_ids,
                       float* G_d2, int32_t kappa, const float* norms = nullptr);
// float32 squared norms of the rows into out[n]
knnkm_status ks_row_norms(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, float* out);
// sum_i ||x_i - C_{labels[i]}||^2 * scale into *out (C null: sum of ||x_i||^2).
knnkm_status ks_sqdist_sum(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                           const float* C, const int32_t* labels, double* out, double scale);
// Incremental update of the fit (exact fixed-point composite vectors):
// per-cluster scale exponents from each job's largest |x|; D from float64
// sums; one sweep's moves applied to D, sizes and the changed clusters'
// centroids and Eqn. 2 terms.
knnkm_status ks_row_stats(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, int m,
                          const int32_t* job_of, double* rowsq, uint32_t* jmax);
knnkm_status ks_fx_scales(knnkm_ctx* ctx, const uint32_t* jmax, int m, const int32_t* k_off, int32_t K,
                          int32_t* cs);
knnkm_status ks_fx_from_f64(knnkm_ctx* ctx, const double* sums, int32_t K, int32_t d, const int32_t* cs,
                            uint64_t* D);
knnkm_status ks_fx_update(knnkm_ctx* ctx, const float* Xp, int64_t n, int32_t d, int32_t* cur,
                          const int32_t* nxt, const int32_t* cs, uint64_t* D, int32_t K, int32_t* counts,
                          int32_t* dirty, float* C, double* Iterm, const int32_t* rev_off,
                          const int32_t* rev_src, uint8_t* act_out, int32_t* dirty_clear,
                          float* delta, int64_t* mass = nullptr, CShadow sw = {}, double* C64 = nullptr,
                          int32_t* nlab = nullptr, int32_t kappa = 0);
// Exact fixed-point D of every cluster from its members (CSR), and the
// centroids, float64 means and Eqn. 2 terms of every cluster from D.
knnkm_status ks_fx_exact_sums(knnkm_ctx* ctx, const float* X, int64_t ldx, int32_t d, int32_t K, const int32_t* off,
                              const int32_t* mem, const int32_t* cs, uint64_t* D);
knnkm_status ks_fx_finalize_all(knnkm_ctx* ctx, const uint64_t* D, int32_t K, int32_t d, const int32_t* cs,
                                const int32_t* counts, float* C, double* Iterm, double* C64);
// Boost form (boost.hip): every sample's best positive move (Eqn. 3) against
// the same state -> prop (target cluster or -1), *nprop += proposals; then
// the conflict-free selection of a round and the next labels.
// Only the listed samples (list/count as ks_act_compact writes them; list
// null: every sample) are evaluated; the others keep their proposal.
knnkm_status ks_boost_propose(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, const int32_t* G,
                              int32_t kappa, const int32_t* labels, const int32_t* counts, const double* C64,
                              int32_t* prop, const int32_t* list, const int32_t* count);
knnkm_status ks_boost_select(knnkm_ctx* ctx, int64_t n, const int32_t* labels, const int32_t* prop, int32_t K,
                             uint64_t seed, int32_t round, uint64_t* win, int32_t* next, int64_t* nprop);
// Lists the positions whose active-set flag is set (and clears the flags).
knnkm_status ks_act_compact(knnkm_ctx* ctx, int64_t n, uint8_t* act, int32_t* list, int32_t* count);
// Active-set marks of the samples moved between cur and nxt and of the rows
// listing them (reverse lists of the graph); moved labels copied into cur.
knnkm_status ks_mark_moved(knnkm_ctx* ctx, int64_t n, int32_t* cur, const int32_t* nxt, const int32_t* rev_off,
                           const int32_t* rev_src, uint8_t* act_out, const int64_t* moved, int64_t all_at,
                           int32_t kappa);
// Active-set marks (bit 0) of the samples with a dirty cluster among their
// candidates and of the samples of jobs with at most kappa clusters; every
// sample when mass is null or *mass >= all_at.
knnkm_status ks_mark_dirty(knnkm_ctx* ctx, int64_t n, const int32_t* lab, const int32_t* dirty,
                           const int32_t* rev_off, const int32_t* rev_src, uint8_t* act_out, const int64_t* mass,
                           int64_t all_at, const int32_t* job_of, const int32_t* kbase, int32_t kappa);
// Reverse lists of an n x kappa graph: rev_off (n + 1), rev_src (n * kappa).
// Reverse lists: rev_src holds graph entries (row * kappa + position; needs
// n * kappa < 2^31).
knnkm_status ks_reverse_graph(knnkm_ctx* ctx, const int32_t* G, int64_t n, int32_t kappa, int32_t* rev_off,
                              int32_t* rev_src);
// Labels of the graph entries: nlab[e] = lab[G[e]] (-1 past [0, n)).
knnkm_status ks_entry_labels(knnkm_ctx* ctx, const int32_t* G, int64_t n, int32_t kappa, const int32_t* lab,
                             int32_t* nlab);
knnkm_status ks_fill_i64(knnkm_ctx* ctx, int64_t* p, int64_t count, int64_t v);
knnkm_status ks_fill_i32(knnkm_ctx* ctx, int32_t* p, int64_t count, int32_t v);
