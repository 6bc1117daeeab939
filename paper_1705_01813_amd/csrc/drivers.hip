// Host drivers: the GK-means^- fit (Alg. 2, Lloyd form) and the KNN graph
// construction (Alg. 3), for one job or a batch of independent jobs.
//
// A batch is a ragged concatenation: job q owns rows [n_off[q], n_off[q+1])
// of X (graph ids stay global) and clusters [k_off[q], k_off[q+1]) of C.
// Every phase is one launch over all jobs: neighbours and candidate clusters
// never leave a job, so the per-sample and per-cluster kernels need no job
// awareness; only the TwoMeans tree shapes, the random lists, the exhaustive
// case kappa >= k_q and the per-job distortion read the job tables.  One job
// runs through the same code (a batch of one), so a job gives bit-identical
// results alone and inside a batch.  Every step runs in this library's
// kernels on the context stream; the host only sequences launches.
#include <algorithm>

#include "rowgroup.h"

// Job of every row (binary search in n_off).
__global__ void k_job_of(const int64_t* __restrict__ n_off, int m, int64_t n, int32_t* __restrict__ job) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = m;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (n_off[mid] <= i) lo = mid; else hi = mid;
    }
    job[i] = lo;
  }
}

// k_q distinct rows of every job by Floyd's algorithm (one thread per job;
// bitmap membership over the job's rows).  ids are global row ids.  Job q owns
// the bitmap words [r0/32 + q, r0/32 + q + ceil(n_q/32)) with its rows'
// bits counted from r0: the slices of different jobs never share a word
// (floor(a) + ceil(b) <= floor(a + b) + 1), so the thread of a job is the
// only one that reads or writes its words.  The bitmap holds
// ceil(n/32) + m words.
__global__ void k_random_init_ids(const int64_t* __restrict__ n_off, const int32_t* __restrict__ k_off, int m,
                                  const uint64_t* __restrict__ seeds, uint32_t* __restrict__ bitmap,
                                  int32_t* __restrict__ ids) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const int64_t r0 = n_off[q], nq = n_off[q + 1] - r0;
  const int32_t k0 = k_off[q], kq = k_off[q + 1] - k0;
  uint32_t* bits = bitmap + (r0 >> 5) + q;
  const uint64_t key = sm_key(seeds[q], sm_stream(RNG_RANDOM_INIT, 0, 0));
  const int64_t base = nq - kq;
  for (int64_t j = base; j < nq; ++j) {
    const int64_t t = sm_below(sm_draw(key, (uint64_t)(j - base)), (uint32_t)(j + 1));
    const bool seen = (bits[t >> 5] >> (t & 31)) & 1u;
    const int64_t v = seen ? j : t;
    bits[v >> 5] |= 1u << (v & 31);
    ids[k0 + (j - base)] = (int32_t)(r0 + v);
  }
}

__global__ void k_gather_rows(const float* __restrict__ X, int d, int64_t ldx,
                              const int32_t* __restrict__ ids, int32_t k, float* __restrict__ C) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)k * d;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / d, t = e % d;
    C[e] = X[(int64_t)ids[r] * ldx + t];
  }
}

// Working copy of the data in the cluster order of a partition: row p of the
// copy is row perm[p] of X (contiguous, leading dimension d).
__global__ void k_permute_rows(const float* __restrict__ X, int d, int64_t ldx, const int32_t* __restrict__ perm,
                               int64_t n, int vec, float* __restrict__ Xp) {
  if (vec) {
    const int q4 = d >> 2;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * q4;
         e += (int64_t)gridDim.x * blockDim.x) {
      const int64_t p = e / q4, t = (e - p * q4) * 4;
      *reinterpret_cast<float4*>(Xp + p * d + t) = *reinterpret_cast<const float4*>(X + (int64_t)perm[p] * ldx + t);
    }
  } else {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * d;
         e += (int64_t)gridDim.x * blockDim.x) {
      const int64_t p = e / d, t = e - p * d;
      Xp[e] = X[(int64_t)perm[p] * ldx + t];
    }
  }
}
__global__ void k_perm_inverse(const int32_t* __restrict__ perm, int64_t n, int32_t* __restrict__ inv) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
    inv[perm[p]] = (int32_t)p;
}
// Graph rows in the copy's numbering: Gp[p] = inv(G[perm[p]]).
__global__ void k_permute_graph(const int32_t* __restrict__ G, int kappa, const int32_t* __restrict__ perm,
                                const int32_t* __restrict__ inv, int64_t n, int32_t* __restrict__ Gp) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * kappa;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / kappa, q = e - p * kappa;
    Gp[e] = inv[G[(int64_t)perm[p] * kappa + q]];
  }
}
__global__ void k_gather_i32(const int32_t* __restrict__ src, const int32_t* __restrict__ perm, int64_t n,
                             int32_t* __restrict__ dst) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
    dst[p] = src[perm[p]];
}
__global__ void k_scatter_i32(const int32_t* __restrict__ src, const int32_t* __restrict__ perm, int64_t n,
                              int32_t* __restrict__ dst) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
    dst[perm[p]] = src[p];
}

// Per-iteration bookkeeping inside a captured fit: the moved count and the
// distortions of iteration *it go to their slots, then *it advances.
__global__ void k_fit_book(int64_t* __restrict__ mv_slot, int64_t* __restrict__ moved,
                           const double* __restrict__ tr_slot, double* __restrict__ trace, int m,
                           int32_t* __restrict__ it) {
  const int t = *it;
  for (int q = threadIdx.x; q < m; q += blockDim.x) trace[(int64_t)t * m + q] = tr_slot[q];
  if (threadIdx.x == 0) {
    moved[t] = *mv_slot;
    *mv_slot = 0;  // the next sweep accumulates from zero
  }
  __syncthreads();
  if (threadIdx.x == 0) *it = t + 1;
}

// Sum of vals[off[q] .. off[q+1]) for every range q, one block per range:
// thread t adds the elements t, t + 1024, ... of the range in index order,
// then the block reduces in a fixed tree, so the result depends on the range
// only (a job's sums are the same alone and in a batch).
__device__ inline double block_range_sum(const double* __restrict__ vals, int64_t a, int64_t b) {
  __shared__ double sh[16];
  double s = 0.0;
  int64_t i = a + threadIdx.x;
  for (; i + 7 * 1024 < b; i += 8 * 1024) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = vals[i + u * 1024];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; i < b; i += 1024) s += vals[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < 16; ++w) t += sh[w];
  return t;  // valid in thread 0
}

__global__ __launch_bounds__(1024) void k_range_sum(const double* __restrict__ vals, const int64_t* __restrict__ off,
                                                    double* __restrict__ out) {
  const int q = blockIdx.x;
  const double s = block_range_sum(vals, off[q], off[q + 1]);
  if (threadIdx.x == 0) out[q] = s;
}

// E of every job = (sum ||x||^2 - sum of the Eqn. 2 terms) / n_q (Eqn. 4
// through the Eqn. 2 identity).  The terms of job q are summed in S_q slices
// of its cluster range (S_q = TR_SLICES from TR_BIG clusters on, else 1; it
// depends on the job's own size, so a job's value is the same alone and in
// a batch): block (s, q) sums slice s as in k_range_sum, then k_range_trace
// adds the slices in order.
constexpr int TR_SLICES = 64;
constexpr int64_t TR_BIG = 65536;
__device__ inline int tr_slices(int64_t len) { return len >= TR_BIG ? TR_SLICES : 1; }
__global__ __launch_bounds__(1024) void k_range_part(const double* __restrict__ Iterm,
                                                     const int64_t* __restrict__ k_off, double* __restrict__ part) {
  const int q = blockIdx.y, sl = blockIdx.x;
  const int64_t a = k_off[q], len = k_off[q + 1] - a;
  const int S = tr_slices(len);
  if (sl >= S) return;  // block-uniform
  const double s = block_range_sum(Iterm, a + len * sl / S, a + len * (sl + 1) / S);
  if (threadIdx.x == 0) part[(int64_t)q * TR_SLICES + sl] = s;
}
__global__ void k_range_trace(const double* __restrict__ part, const int64_t* __restrict__ k_off,
                              const double* __restrict__ sxx, const int64_t* __restrict__ n_off, int m,
                              double* __restrict__ dst) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < m; q += gridDim.x * blockDim.x) {
    const int S = tr_slices(k_off[q + 1] - k_off[q]);
    double s = 0.0;
    for (int sl = 0; sl < S; ++sl) s += part[(int64_t)q * TR_SLICES + sl];
    dst[q] = (sxx[q] - s) / (double)(n_off[q + 1] - n_off[q]);
  }
}

// The distortion of every job into dst (m values); kmax: the largest job's
// cluster count (host), part: m * TR_SLICES doubles of workspace.
static knnkm_status launch_trace(knnkm_ctx* ctx, const double* Iterm, const int64_t* k_off, const double* sxx,
                                 const int64_t* n_off, int m, int64_t kmax, double* part, double* dst) {
  const dim3 grid(kmax >= TR_BIG ? TR_SLICES : 1, m);
  k_range_part<<<grid, 1024, 0, ctx->stream>>>(Iterm, k_off, part);
  k_range_trace<<<grid_for(m, 256, 1024), 256, 0, ctx->stream>>>(part, k_off, sxx, n_off, m, dst);
  return knnkm_check(ctx, "distortion trace");
}

__global__ void k_local_labels(const int32_t* __restrict__ glab, const int32_t* __restrict__ job,
                               const int32_t* __restrict__ k_off, int64_t n, int32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = glab[i] - k_off[job[i]];
}

static knnkm_status check_params(knnkm_ctx* ctx, const knnkm_params* p, const char* who) {
  if (!p) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: params is null", who);
  if (p->struct_size != sizeof(knnkm_params))
    return knnkm_fail(ctx, KNNKM_EINVAL, "%s: params.struct_size %u != %zu", who, p->struct_size,
                      sizeof(knnkm_params));
  if (p->xi < 2) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: xi must be >= 2", who);
  if (p->tau < 0) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: tau must be >= 0", who);
  if (p->bisect_iters < 0) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: bisect_iters must be >= 0", who);
  if (p->max_iters < 0) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: max_iters must be >= 0", who);
  if (p->precision != KNNKM_FP32 && p->precision != KNNKM_BF16_RERANK)
    return knnkm_fail(ctx, KNNKM_EINVAL, "%s: unknown precision %d", who, p->precision);
  if (p->init != KNNKM_INIT_TWOMEANS && p->init != KNNKM_INIT_RANDOM && p->init != KNNKM_INIT_LABELS)
    return knnkm_fail(ctx, KNNKM_EINVAL, "%s: unknown init %d", who, p->init);
  return KNNKM_OK;
}

static knnkm_status check_data(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                               const char* who) {
  if (!X) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: X is null", who);
  if (n < 2 || n > INT32_MAX) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: need 2 <= n < 2^31", who);
  if (d < 1 || ldx < d) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: need d >= 1 and ldx >= d", who);
  if (d > KNNKM_MAX_D) return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "%s: d=%d > %d", who, d, KNNKM_MAX_D);
  return KNNKM_OK;
}

// Host and device copies of the job tables of one call.
struct Jobs {
  int m = 1;
  std::vector<int64_t> n_host, n_off_host;   // n_q, row offsets (m+1)
  std::vector<uint64_t> seed_host;
  int64_t n = 0;
  // device
  const int64_t* n_off = nullptr;
  const uint64_t* seeds = nullptr;
  const int32_t* job_of = nullptr;  // null for one job
};

static knnkm_status upload_jobs(knnkm_ctx* ctx, Jobs& J, const char* tag) {
  char name[40];
  snprintf(name, sizeof(name), "%s_noff", tag);
  KNNKM_WS(ctx, noff, int64_t, name, J.m + 1);
  snprintf(name, sizeof(name), "%s_seeds", tag);
  KNNKM_WS(ctx, seeds, uint64_t, name, J.m);
  KNNKM_HIP(ctx, hipMemcpyAsync(noff, J.n_off_host.data(), sizeof(int64_t) * (J.m + 1), hipMemcpyHostToDevice,
                                ctx->stream));
  KNNKM_HIP(ctx, hipMemcpyAsync(seeds, J.seed_host.data(), sizeof(uint64_t) * J.m, hipMemcpyHostToDevice,
                                ctx->stream));
  J.n_off = noff;
  J.seeds = seeds;
  J.job_of = nullptr;
  if (J.m > 1) {
    snprintf(name, sizeof(name), "%s_jobof", tag);
    KNNKM_WS(ctx, job, int32_t, name, J.n);
    k_job_of<<<grid_for(J.n, 256, 8192), 256, 0, ctx->stream>>>(noff, J.m, J.n, job);
    KNNKM_TRY(knnkm_check(ctx, "job table"));
    J.job_of = job;
  }
  // the host copies must stay valid until the copies ran
  KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return KNNKM_OK;
}

// Cluster offsets (int32 and int64 on the device) for per-job cluster counts.
static knnkm_status upload_koff(knnkm_ctx* ctx, const std::vector<int32_t>& kq, const char* tag,
                                int32_t** k32, int64_t** k64, int32_t* total) {
  std::vector<int32_t> a(kq.size() + 1, 0);
  std::vector<int64_t> b(kq.size() + 1, 0);
  for (size_t q = 0; q < kq.size(); ++q) {
    a[q + 1] = a[q] + kq[q];
    b[q + 1] = b[q] + kq[q];
  }
  char name[40];
  snprintf(name, sizeof(name), "%s_k32", tag);
  KNNKM_WS(ctx, d32, int32_t, name, a.size());
  snprintf(name, sizeof(name), "%s_k64", tag);
  KNNKM_WS(ctx, d64, int64_t, name, b.size());
  KNNKM_HIP(ctx, hipMemcpyAsync(d32, a.data(), sizeof(int32_t) * a.size(), hipMemcpyHostToDevice, ctx->stream));
  KNNKM_HIP(ctx, hipMemcpyAsync(d64, b.data(), sizeof(int64_t) * b.size(), hipMemcpyHostToDevice, ctx->stream));
  KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *k32 = d32;
  *k64 = d64;
  *total = a.back();
  return KNNKM_OK;
}

// Alg. 3 for every job of J.
static knnkm_status build_impl(knnkm_ctx* ctx, const float* X, int32_t d, int64_t ldx, Jobs& J,
                               const knnkm_params* p, int32_t* G_ids, float* G_d2) {
  const int kappa = p->kappa;
  const int64_t n = J.n;
  auto mark = [&](int e) {
    if (ctx->timing) {
      hipEvent_t h = knnkm_event(ctx, e);
      if (h) (void)hipEventRecord(h, ctx->stream);
    }
  };
  if (ctx->timing) ctx->build_ev = 0;
  mark(0);
  KNNKM_TRY(ks_graph_init(ctx, X, n, d, ldx, kappa, J.seed_host[0], G_ids, G_d2, J.job_of, J.n_off, J.seeds));
  if (p->tau > 0) {
    // k0 = max(1, floor(n_q / xi)) clusters per job (Sec. 4.3)
    std::vector<int32_t> k0(J.m);
    bool all_dense = true;
    for (int q = 0; q < J.m; ++q) {
      k0[q] = (int32_t)std::max<int64_t>(1, J.n_host[q] / p->xi);
      all_dense = all_dense && kappa >= k0[q];
    }
    int32_t *k0_32, K0;
    int64_t* k0_64;
    KNNKM_TRY(upload_koff(ctx, k0, "kb", &k0_32, &k0_64, &K0));
    KNNKM_WS(ctx, lab, int32_t, "kb_labels", n);
    KNNKM_WS(ctx, lab2, int32_t, "kb_labels2", n);
    KNNKM_WS(ctx, counts, int32_t, "kb_counts", K0);
    KNNKM_WS(ctx, off, int32_t, "kb_offsets", (int64_t)K0 + 1);
    KNNKM_WS(ctx, mem, int32_t, "kb_members", n);
    KNNKM_WS(ctx, C, float, "kb_centroids", (int64_t)K0 * d);
    KNNKM_WS(ctx, nrm, float, "kb_norms", n);
    // wide rows: the centroid shadow the assignment's early-abandon steps read
    CShadow sw;
    if (ctx->wide_pd && ks_assign_pd_ok(d, kappa) && !all_dense)
      KNNKM_TRY(ks_shadow_alloc(ctx, "kb", K0, d, &sw));
    KNNKM_TRY(ks_row_norms(ctx, X, n, d, ldx, nrm));
    for (int t = 0; t < p->tau; ++t) {
      KNNKM_TRY(ks_twomeans_multi(ctx, X, d, ldx, J.n_host, k0, J.m > 1 ? J.seeds : nullptr, J.seed_host[0], t,
                                  p->bisect_iters, lab));
      KNNKM_TRY(ks_label_sort(ctx, lab, n, K0, counts, off, mem));
      KNNKM_TRY(ks_segsum(ctx, X, n, d, ldx, K0, counts, off, mem, C, nullptr, nullptr));
      KNNKM_TRY(ks_c_shadow(ctx, C, K0, d, nullptr, sw));
      KNNKM_TRY(ks_assign(ctx, X, n, d, ldx, C, K0, G_ids, kappa, lab, lab2, nullptr, nullptr, mem,
                          J.m == 1 && all_dense, J.job_of, k0_32, KS_USE_BUILD, nullptr, nullptr, nullptr, nullptr,
                          nullptr, nullptr, true, nullptr, nullptr, nullptr, nullptr, sw));
      KNNKM_TRY(ks_refine(ctx, X, n, d, ldx, lab2, K0, p->precision, G_ids, G_d2, kappa, nrm));
    }
  }
  mark(1);
  return KNNKM_OK;
}

// The initial partition of a fit (Alg. 2 starts from Alg. 1; or k distinct
// rows as seeds and an exhaustive assignment to them; or the caller's
// labels), and the centroids that clusters left empty keep: zero after
// Alg. 1, the seed rows after the random start, the caller's with labels.
static knnkm_status init_partition(knnkm_ctx* ctx, const float* X, int32_t d, int64_t ldx, Jobs& J,
                                   const std::vector<int32_t>& kq, const knnkm_params* p, int32_t K,
                                   const int32_t* k32, int32_t* labels, float* C) {
  const int64_t n = J.n;
  const int m = J.m;
  if (p->init == KNNKM_INIT_RANDOM) {
    const int64_t bm_words = (n + 31) / 32 + m;
    KNNKM_WS(ctx, bitmap, uint32_t, "fit_bitmap", bm_words);
    KNNKM_WS(ctx, ids, int32_t, "fit_init_ids", K);
    KNNKM_TRY(ks_fill_i32(ctx, (int32_t*)bitmap, bm_words, 0));
    k_random_init_ids<<<(m + 63) / 64, 64, 0, ctx->stream>>>(J.n_off, k32, m, J.seeds, bitmap, ids);
    k_gather_rows<<<grid_for((int64_t)K * d, 256, 4096), 256, 0, ctx->stream>>>(X, d, ldx, ids, K, C);
    KNNKM_TRY(knnkm_check(ctx, "random init"));
    // exhaustive assignment to the seeds of the sample's own job
    KNNKM_TRY(ks_assign(ctx, X, n, d, ldx, C, K, nullptr, K, nullptr, labels, nullptr, nullptr, nullptr, true,
                        J.job_of, k32));
  } else if (p->init == KNNKM_INIT_TWOMEANS) {
    KNNKM_TRY(ks_twomeans_multi(ctx, X, d, ldx, J.n_host, kq, m > 1 ? J.seeds : nullptr, J.seed_host[0],
                                KNNKM_ROUND_FIT, p->bisect_iters, labels));
    KNNKM_TRY(ks_fill_i32(ctx, (int32_t*)C, (int64_t)K * d, 0));
  }
  return KNNKM_OK;
}

// Alg. 2 (Lloyd form) for every job of J.  labels are global cluster ids;
// trace_dev receives E_t of job q at [t * m + q]; *iters_run the sweeps done.
static knnkm_status fit_impl(knnkm_ctx* ctx, const float* X, int32_t d, int64_t ldx, Jobs& J,
                             const std::vector<int32_t>& kq, const int32_t* G_ids, const knnkm_params* p,
                             int32_t* labels, float* C, int32_t* counts, double* trace_dev, int* iters_run) {
  const int kappa = p->kappa;
  const int T = p->max_iters;
  const int64_t n = J.n;
  const int m = J.m;
  int32_t *k32, K;
  int64_t* k64;
  KNNKM_TRY(upload_koff(ctx, kq, "fit", &k32, &k64, &K));
  int64_t kmax = 0;
  for (int32_t v : kq) kmax = std::max<int64_t>(kmax, v);
  KNNKM_WS(ctx, trpart, double, "fit_trace_part", (int64_t)m * TR_SLICES);
  bool all_dense = true;
  for (int q = 0; q < m; ++q) all_dense = all_dense && kappa >= kq[q];
  KNNKM_WS(ctx, lab2, int32_t, "fit_labels2", n);
  KNNKM_WS(ctx, off, int32_t, "fit_offsets", (int64_t)K + 1);
  KNNKM_WS(ctx, mem, int32_t, "fit_members", n);
  KNNKM_WS(ctx, Iterm, double, "fit_iterm", K);
  KNNKM_WS(ctx, rowsq, double, "fit_rowsq", n);
  KNNKM_WS(ctx, sxx, double, "fit_sxx", m);
  KNNKM_WS(ctx, moved, int64_t, "fit_moved", (int64_t)T + 1);
  KNNKM_TRY(ks_fill_i64(ctx, moved, (int64_t)T + 1, 0));
  // phase events: 2 fit start, 3 initialisation done, 4 iterations done,
  // 6+2j / 7+2j around the assignment of iteration j+1
  auto mark = [&](int e) {
    if (ctx->timing) {
      hipEvent_t h = knnkm_event(ctx, e);
      if (h) (void)hipEventRecord(h, ctx->stream);
    }
  };
  if (ctx->timing) {
    ctx->fit_ev = 2;
    ctx->assign_ev0 = 6;
    ctx->assign_n = 0;
  }
  mark(2);

  KNNKM_TRY(init_partition(ctx, X, d, ldx, J, kq, p, K, k32, labels, C));
  KNNKM_WS(ctx, jmax, uint32_t, "fit_jmax", m);
  KNNKM_TRY(ks_row_stats(ctx, X, n, d, ldx, m, J.job_of, rowsq, jmax));
  k_range_sum<<<m, 1024, 0, ctx->stream>>>(rowsq, J.n_off, sxx);
  KNNKM_TRY(ks_label_sort(ctx, labels, n, K, counts, off, mem));
  KNNKM_WS(ctx, sums0, double, "fit_sums0", (int64_t)K * d);
  KNNKM_TRY(ks_segsum(ctx, X, n, d, ldx, K, counts, off, mem, C, sums0, Iterm));
  KNNKM_TRY(launch_trace(ctx, Iterm, k64, sxx, J.n_off, m, kmax, trpart, trace_dev));
  KNNKM_TRY(knnkm_check(ctx, "fit initialisation"));
  // the sweeps update the composite vectors D_r incrementally (exact
  // fixed point, one scale exponent per job)
  KNNKM_WS(ctx, cs, int32_t, "fit_scale", K);
  KNNKM_WS(ctx, Dfx, uint64_t, "fit_dfx", (int64_t)K * d * 2);
  // clusters whose members changed in a sweep's update, one array per label
  // buffer (the output buffer of that sweep), read by the next sweep
  KNNKM_WS(ctx, dirty, int32_t, "fit_dirty", K);
  KNNKM_WS(ctx, dirty2, int32_t, "fit_dirty2", K);
  KNNKM_TRY(ks_fx_scales(ctx, jmax, m, k32, K, cs));
  KNNKM_TRY(ks_fill_i32(ctx, dirty, K, 0));
  KNNKM_TRY(ks_fill_i32(ctx, dirty2, K, 0));

  // The sweeps run on a working copy of X (and of the graph) in the cluster
  // order of the initial partition: rows are then read as streams, and the
  // neighbours of a sample, which mostly share its cluster, have nearby ids.
  // Assignments do not depend on the numbering of the samples; the update
  // sums each cluster's members in the copy's order.
  const bool use_graph = !(m == 1 && all_dense) && G_ids;
  KNNKM_WS(ctx, perm, int32_t, "fit_perm", n);
  KNNKM_WS(ctx, inv, int32_t, "fit_inv", n);
  KNNKM_WS(ctx, Xp, float, "fit_xp", n * (int64_t)d);
  KNNKM_WS(ctx, labp, int32_t, "fit_labp", n);
  int32_t* Gp = nullptr;
  if (use_graph) {
    Gp = (int32_t*)knnkm_ws(ctx, "fit_gp", sizeof(int32_t) * (size_t)n * kappa);
    if (!Gp) return KNNKM_ENOMEM;
  }
  KNNKM_HIP(ctx, hipMemcpyAsync(perm, mem, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
  const bool vec = (d % 4 == 0) && (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
  k_permute_rows<<<grid_for(n * (vec ? d / 4 : d), 256, 16384), 256, 0, ctx->stream>>>(X, d, ldx, perm, n,
                                                                                       vec ? 1 : 0, Xp);
  k_perm_inverse<<<grid_for(n, 256, 8192), 256, 0, ctx->stream>>>(perm, n, inv);
  if (use_graph)
    k_permute_graph<<<grid_for(n * kappa, 256, 16384), 256, 0, ctx->stream>>>(G_ids, kappa, perm, inv, n, Gp);
  k_gather_i32<<<grid_for(n, 256, 8192), 256, 0, ctx->stream>>>(labels, perm, n, labp);
  KNNKM_TRY(knnkm_check(ctx, "fit working copy"));
  // Active sets: after the first sweep a sample is looked at only when its
  // candidate set changed (it or a neighbour moved: bit 1 of its flag) or it
  // may have to move for another reason: narrow rows list the samples that
  // had several candidates (bit 0 from the sweep) and skip those none of
  // whose candidate centroids changed; wide rows, where nearly every sample
  // has several candidates, list only the samples with a changed candidate
  // centroid (bit 0 from the update: a member of a dirty cluster, or a
  // sample listing one in its graph row).  Every other sample has the inputs
  // of its last decision and keeps its label (same results).  One flag array
  // per label buffer: the flags next to a label array mark the samples the
  // sweep reading it looks at.
  const bool use_act = ctx->active_sets && use_graph && n * (int64_t)kappa < INT32_MAX;
  int32_t *rev_off = nullptr, *rev_src = nullptr;
  uint8_t *act_p = nullptr, *act_2 = nullptr;
  // wide rows: the labels of the graph entries, kept current by the updates,
  // which the active-set sweeps read in place of scattered neighbour labels
  int32_t* nlab = nullptr;
  int32_t* lcnt = nullptr;  // list counters, one per flag array
  int64_t* dmass = nullptr;  // members of the clusters an update made dirty
  if (use_act) {
    lcnt = (int32_t*)knnkm_ws(ctx, "fit_list_counts", 2 * sizeof(int32_t));
    dmass = (int64_t*)knnkm_ws(ctx, "fit_dirty_mass", sizeof(int64_t));
    if (!lcnt || !dmass) return KNNKM_ENOMEM;
    KNNKM_TRY(ks_fill_i32(ctx, lcnt, 2, 0));
    rev_off = (int32_t*)knnkm_ws(ctx, "fit_rev_off", sizeof(int32_t) * (size_t)(n + 1));
    rev_src = (int32_t*)knnkm_ws(ctx, "fit_rev_src", sizeof(int32_t) * (size_t)n * kappa);
    act_p = (uint8_t*)knnkm_ws(ctx, "fit_act_p", (size_t)(n + 3) / 4 * 4);
    act_2 = (uint8_t*)knnkm_ws(ctx, "fit_act_2", (size_t)(n + 3) / 4 * 4);
    if (!rev_off || !rev_src || !act_p || !act_2) return KNNKM_ENOMEM;
    if (ctx->wide_pd && ks_assign_pd_ok(d, kappa) && !all_dense) {
      nlab = (int32_t*)knnkm_ws(ctx, "fit_nlab", sizeof(int32_t) * (size_t)n * kappa);
      if (!nlab) return KNNKM_ENOMEM;
    }
    KNNKM_TRY(ks_reverse_graph(ctx, Gp, n, kappa, rev_off, rev_src));
    // both flag arrays start clear (the first sweep writes every flag of
    // its output array; the padding bytes stay zero)
    KNNKM_TRY(ks_fill_i32(ctx, (int32_t*)act_p, (n + 3) / 4, 0));
    KNNKM_TRY(ks_fill_i32(ctx, (int32_t*)act_2, (n + 3) / 4, 0));
  }
  auto act_for = [&](const int32_t* lab) -> uint8_t* {
    return use_act ? (lab == labp ? act_p : act_2) : nullptr;
  };
  auto cnt_for = [&](const int32_t* lab) -> int32_t* {
    return use_act ? (lab == labp ? lcnt : lcnt + 1) : nullptr;
  };
  auto dirty_for = [&](const int32_t* lab) -> int32_t* { return lab == labp ? dirty : dirty2; };
  // Wide rows: every evaluated sample leaves bounds of its distances (an
  // upper bound to its centroid, a lower bound to the cluster of each graph
  // entry) and every update the movement of each changed centroid, so the
  // clusters that the triangle inequality still rules out need no distance.
  const bool drift = use_act && ctx->wide_pd && ks_assign_pd_ok(d, kappa) && !all_dense;
  float *bnd_u = nullptr, *bnd_lb = nullptr, *cdelta = nullptr;
  // and the shadow of the centroids read by the early-abandon steps
  CShadow sw;
  if (ctx->wide_pd && ks_assign_pd_ok(d, kappa) && !all_dense) {
    KNNKM_TRY(ks_shadow_alloc(ctx, "fit", K, d, &sw));
    KNNKM_TRY(ks_c_shadow(ctx, C, K, d, nullptr, sw));
  }
  if (drift) {
    bnd_u = (float*)knnkm_ws(ctx, "fit_bnd_u", sizeof(float) * (size_t)n);
    bnd_lb = (float*)knnkm_ws(ctx, "fit_bnd_lb", sizeof(float) * (size_t)n * (kappa + 1));
    cdelta = (float*)knnkm_ws(ctx, "fit_delta", sizeof(float) * (size_t)K);
    if (!bnd_u || !bnd_lb || !cdelta) return KNNKM_ENOMEM;
  }
  mark(3);

  // one sweep: assignment, update, distortion of every job
  auto sweep = [&](const int32_t* cu, int32_t* nx, int64_t* mv, bool first, int64_t* ev,
                   int64_t* ac) -> knnkm_status {
    // moved counters are cleared once per fit (eager sweeps: one slot each)
    // or by the bookkeeping kernel (graph replays)
    // (with drift bounds the flags of the next sweep come from the update's
    // marks alone)
    return ks_assign(ctx, Xp, n, d, d, C, K, Gp, kappa, cu, nx, nullptr, mv, nullptr, m == 1 && all_dense,
                     J.job_of, k32, first ? KS_USE_FIT_FIRST : KS_USE_FIT, ev, first ? nullptr : act_for(cu),
                     drift ? nullptr : act_for(nx), ac, cnt_for(cu), cnt_for(nx), false, first ? nullptr : dirty_for(cu), bnd_u,
                     bnd_lb, first ? nullptr : cdelta, sw, first ? nullptr : nlab);
  };
  // The first sweep moves a large share of the samples away from the
  // initial partition: its update rebuilds the sums from a label sort and
  // the segmented float64 sums (as at initialisation) and converts them to
  // fixed point (and so does the second's when it still moves more than
  // n/8); later sweeps apply only their moves.
  auto update = [&](int32_t* cu, const int32_t* nx, double* tr, bool full, const int64_t* mv) -> knnkm_status {
    if (full) {
      KNNKM_TRY(ks_label_sort(ctx, nx, n, K, counts, off, mem));
      KNNKM_TRY(ks_segsum(ctx, Xp, n, d, d, K, counts, off, mem, C, sums0, Iterm, cdelta));
      KNNKM_TRY(ks_fx_from_f64(ctx, sums0, K, d, cs, Dfx));
      // the moves' marks, or every row once the moved samples' reverse
      // lists (kappa entries each on average) would cover n
      if (use_act)
        KNNKM_TRY(ks_mark_moved(ctx, n, cu, nx, rev_off, rev_src, act_for(nx), mv, (n + kappa) / (kappa + 1), kappa));
      // every centroid was recomputed
      KNNKM_TRY(ks_fill_i32(ctx, dirty_for(nx), K, 1));
      KNNKM_TRY(ks_fill_i32(ctx, dirty_for(cu), K, 0));
      KNNKM_TRY(ks_c_shadow(ctx, C, K, d, nullptr, sw));
      if (nlab) KNNKM_TRY(ks_entry_labels(ctx, Gp, n, kappa, nx, nlab));
      if (drift)
        KNNKM_TRY(ks_mark_dirty(ctx, n, nx, dirty_for(nx), rev_off, rev_src, act_for(nx), nullptr, 0, J.job_of, k32,
                                kappa));
    } else {
      KNNKM_TRY(ks_fx_update(ctx, Xp, n, d, cu, nx, cs, Dfx, K, counts, dirty_for(nx), C, Iterm, rev_off, rev_src,
                             act_for(nx), dirty_for(cu), cdelta, drift ? dmass : nullptr, sw, nullptr, nlab, kappa));
      // scattered marks while the dirty clusters' members and the rows
      // listing them stay below about 2n; every sample beyond that
      if (drift)
        KNNKM_TRY(ks_mark_dirty(ctx, n, nx, dirty_for(nx), rev_off, rev_src, act_for(nx), dmass,
                                2 * n / (kappa + 1), J.job_of, k32, kappa));
    }
    KNNKM_TRY(launch_trace(ctx, Iterm, k64, sxx, J.n_off, m, kmax, trpart, tr));
    return knnkm_check(ctx, "fit iteration");
  };
  ctx->fit_evals = nullptr;
  ctx->fit_actives = nullptr;
  ctx->fit_moved = nullptr;
  const bool time_all = ctx->timing >= 2;
  // with every assignment timed, also count the samples each one looked at
  // and the samples whose distances it evaluated
  int64_t *evals = nullptr, *actives = nullptr;
  if (time_all) {
    evals = (int64_t*)knnkm_ws(ctx, "fit_evals", sizeof(int64_t) * (size_t)(T + 1));
    actives = (int64_t*)knnkm_ws(ctx, "fit_actives", sizeof(int64_t) * (size_t)(T + 1));
    if (!evals || !actives) return KNNKM_ENOMEM;
  }
  int32_t* cur = labp;
  int32_t* nxt = lab2;
  int it = 0;
  auto eager = [&](int t) -> knnkm_status {
    if (time_all) mark(6 + 2 * (t - 1));
    KNNKM_TRY(sweep(cur, nxt, moved + t, t == 1, evals ? evals + t : nullptr, actives ? actives + t : nullptr));
    if (time_all) {
      mark(7 + 2 * (t - 1));
      ctx->assign_n = t;
    }
    // the first sweep's update rebuilds the sums; so does the second's when
    // it moved more than n/8 samples (decided on the host, and only for the
    // eagerly run sweeps, so every path of the fit takes the same updates)
    bool full = t == 1;
    if (t == 2) {
      int64_t mv = 0;
      KNNKM_HIP(ctx, hipMemcpyAsync(&mv, moved + t, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
      KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
      full = mv > n / 8;
    }
    KNNKM_TRY(update(cur, nxt, trace_dev + (int64_t)t * m, full, moved + t));
    std::swap(cur, nxt);
    it = t;
    return KNNKM_OK;
  };
  const bool early = p->early_stop && m == 1;
  // Iterations 1-2 run eagerly (they size every workspace buffer); without
  // early stopping the rest replays a captured graph of two sweeps, whose
  // bookkeeping kernel files the moved count and the distortions of each
  // sweep under a device-side iteration counter.
  int t = 1;
  bool converged = false;
  for (; t <= T && (early || t <= 2) && !converged; ++t) {
    KNNKM_TRY(eager(t));
    if (early) {
      int64_t mv = -1;
      KNNKM_HIP(ctx, hipMemcpyAsync(&mv, moved + t, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
      KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
      converged = mv == 0;
    }
  }
  if (!early && t + 1 <= T && ctx->graphs && !time_all) {
    KNNKM_WS(ctx, book_it, int32_t, "fit_book_it", 1);
    KNNKM_WS(ctx, mv_slot, int64_t, "fit_mv_slot", 1);
    KNNKM_WS(ctx, tr_slot, double, "fit_tr_slot", m);
    KNNKM_TRY(ks_fill_i32(ctx, book_it, 1, t));
    KNNKM_TRY(ks_fill_i64(ctx, mv_slot, 1, 0));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool ok = true;
    if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      ctx->cap_stream = nullptr;
      ok = false;
    }
    if (ok) {
      hipStream_t user = ctx->stream;
      ctx->stream = ctx->cap_stream;
      ok = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        ctx->capturing = true;
        knnkm_status st = sweep(cur, nxt, mv_slot, false, nullptr, nullptr);
        if (st == KNNKM_OK) st = update(cur, nxt, tr_slot, false, nullptr);
        if (st == KNNKM_OK) {
          k_fit_book<<<1, 256, 0, ctx->stream>>>(mv_slot, moved, tr_slot, trace_dev, m, book_it);
          st = sweep(nxt, cur, mv_slot, false, nullptr, nullptr);
        }
        if (st == KNNKM_OK) st = update(nxt, cur, tr_slot, false, nullptr);
        if (st == KNNKM_OK) k_fit_book<<<1, 256, 0, ctx->stream>>>(mv_slot, moved, tr_slot, trace_dev, m, book_it);
        ctx->capturing = false;
        ok = hipStreamEndCapture(ctx->stream, &graph) == hipSuccess && st == KNNKM_OK && graph;
      }
      ctx->stream = user;
      (void)hipGetLastError();
      if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
      (void)hipGetLastError();
    }
    if (ok) {
      // pairs of sweeps; cur/nxt end where they started
      for (; t + 1 <= T; t += 2) {
        KNNKM_HIP(ctx, hipGraphLaunch(exec, ctx->stream));
        it = t + 1;
      }
      KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    // a capture that could not be made leaves the remaining sweeps to the
    // eager path below (same kernels, same results)
  }
  for (; t <= T && !converged; ++t) KNNKM_TRY(eager(t));
  mark(4);
  // labels back in the caller's numbering
  k_scatter_i32<<<grid_for(n, 256, 8192), 256, 0, ctx->stream>>>(cur, perm, n, labels);
  KNNKM_TRY(knnkm_check(ctx, "fit labels"));
  *iters_run = it;
  ctx->fit_iters = it;
  ctx->fit_evals = evals;
  ctx->fit_actives = actives;
  ctx->fit_moved = m == 1 ? moved : nullptr;
  return KNNKM_OK;
}

// Resume: counts the labels outside [0, k).
__global__ void k_check_labels(const int32_t* __restrict__ lab, int64_t n, int32_t k,
                               unsigned long long* __restrict__ bad) {
  unsigned long long c = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += (lab[i] < 0 || lab[i] >= k) ? 1ull : 0ull;
  if (c) atomicAdd(bad, c);
}

extern "C" knnkm_status knnkm_enable_active_sets(knnkm_ctx* ctx, int32_t on) {
  if (!ctx) return KNNKM_EINVAL;
  ctx->active_sets = on != 0;
  return KNNKM_OK;
}

extern "C" knnkm_status knn_kmeans_fit(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                       int32_t k, const int32_t* G_ids, const knnkm_params* p,
                                       int32_t* labels, float* C, int32_t* counts, double* trace_host,
                                       int32_t* iters_run_host) {
  if (!ctx) return KNNKM_EINVAL;
  if (ctx->sticky) return KNNKM_EDEVICE;
  KNNKM_TRY(check_data(ctx, X, n, d, ldx, "knn_kmeans_fit"));
  KNNKM_TRY(check_params(ctx, p, "knn_kmeans_fit"));
  if (k < 1 || k > n) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_kmeans_fit: need 1 <= k <= n");
  const int kappa = p->kappa;
  const bool dense = kappa >= k;
  if (kappa < 1 || (!dense && kappa > n - 1))
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_kmeans_fit: need 1 <= kappa <= n-1");
  if (!dense && kappa > KNNKM_MAX_KAPPA)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "knn_kmeans_fit: kappa=%d > %d", kappa, KNNKM_MAX_KAPPA);
  if (!labels || !C || !counts || (!dense && !G_ids))
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_kmeans_fit: null pointer");
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  Jobs J;
  J.m = 1;
  J.n = n;
  J.n_host = {n};
  J.n_off_host = {0, n};
  J.seed_host = {p->seed};
  KNNKM_TRY(upload_jobs(ctx, J, "one"));
  if (p->init == KNNKM_INIT_LABELS) {
    KNNKM_WS(ctx, bad, int64_t, "fit_bad_labels", 1);
    KNNKM_TRY(ks_fill_i64(ctx, bad, 1, 0));
    k_check_labels<<<grid_for(n, 256, 4096), 256, 0, ctx->stream>>>(labels, n, k, (unsigned long long*)bad);
    int64_t nbad = 0;
    KNNKM_HIP(ctx, hipMemcpyAsync(&nbad, bad, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (nbad) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_kmeans_fit: %lld input labels outside [0, %d)",
                                (long long)nbad, k);
  }
  KNNKM_WS(ctx, trace, double, "fit_trace", (int64_t)p->max_iters + 1);
  int it = 0;
  KNNKM_TRY(fit_impl(ctx, X, d, ldx, J, std::vector<int32_t>{k}, G_ids, p, labels, C, counts, trace, &it));
  if (trace_host)
    KNNKM_HIP(ctx, hipMemcpyAsync(trace_host, trace, sizeof(double) * (size_t)(it + 1), hipMemcpyDeviceToHost,
                                  ctx->stream));
  KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (iters_run_host) *iters_run_host = it;
  return knnkm_check(ctx, "knn_kmeans_fit");
}

extern "C" knnkm_status knn_build(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                  const knnkm_params* p, int32_t* G_ids, float* G_d2) {
  if (!ctx) return KNNKM_EINVAL;
  if (ctx->sticky) return KNNKM_EDEVICE;
  KNNKM_TRY(check_data(ctx, X, n, d, ldx, "knn_build"));
  KNNKM_TRY(check_params(ctx, p, "knn_build"));
  const int kappa = p->kappa;
  if (kappa < 1 || kappa > n - 1) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_build: need 1 <= kappa <= n-1");
  if (kappa > KNNKM_MAX_KAPPA)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "knn_build: kappa=%d > %d", kappa, KNNKM_MAX_KAPPA);
  if (!G_ids || !G_d2) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_build: null pointer");
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  Jobs J;
  J.m = 1;
  J.n = n;
  J.n_host = {n};
  J.n_off_host = {0, n};
  J.seed_host = {p->seed};
  KNNKM_TRY(upload_jobs(ctx, J, "one"));
  return build_impl(ctx, X, d, ldx, J, p, G_ids, G_d2);
}

extern "C" knnkm_status knnkm_fit_batched(knnkm_ctx* ctx, const float* X, int32_t d, int64_t ldx, int32_t m,
                                          const int64_t* n_off_host, const int32_t* k_host,
                                          const uint64_t* seeds_host, const knnkm_params* p, int32_t* G_ids,
                                          float* G_d2, int32_t* labels, float* C, int32_t* counts,
                                          double* trace_host) {
  if (!ctx) return KNNKM_EINVAL;
  if (ctx->sticky) return KNNKM_EDEVICE;
  if (m < 1 || !n_off_host || !k_host || !seeds_host)
    return knnkm_fail(ctx, KNNKM_EINVAL, "knnkm_fit_batched: need m >= 1 and job tables");
  KNNKM_TRY(check_params(ctx, p, "knnkm_fit_batched"));
  if (p->init == KNNKM_INIT_LABELS)
    return knnkm_fail(ctx, KNNKM_EINVAL, "knnkm_fit_batched: init from labels is knn_kmeans_fit only");
  const int kappa = p->kappa;
  if (kappa < 1 || kappa > KNNKM_MAX_KAPPA)
    return knnkm_fail(ctx, kappa < 1 ? KNNKM_EINVAL : KNNKM_EUNSUPPORTED, "knnkm_fit_batched: kappa=%d", kappa);
  if (n_off_host[0] != 0) return knnkm_fail(ctx, KNNKM_EINVAL, "knnkm_fit_batched: n_off[0] must be 0");
  Jobs J;
  J.m = m;
  std::vector<int32_t> kq(m);
  int64_t ktot = 0;
  for (int q = 0; q < m; ++q) {
    const int64_t nq = n_off_host[q + 1] - n_off_host[q];
    if (nq < 2 || kappa > nq - 1)
      return knnkm_fail(ctx, KNNKM_EINVAL, "knnkm_fit_batched: job %d has %lld rows (need >= kappa+1)", q,
                        (long long)nq);
    if (k_host[q] < 1 || k_host[q] > nq)
      return knnkm_fail(ctx, KNNKM_EINVAL, "knnkm_fit_batched: job %d needs 1 <= k <= n", q);
    J.n_host.push_back(nq);
    kq[q] = k_host[q];
    ktot += k_host[q];
  }
  J.n = n_off_host[m];
  J.n_off_host.assign(n_off_host, n_off_host + m + 1);
  J.seed_host.assign(seeds_host, seeds_host + m);
  KNNKM_TRY(check_data(ctx, X, J.n, d, ldx, "knnkm_fit_batched"));
  if (ktot > INT32_MAX) return knnkm_fail(ctx, KNNKM_EINVAL, "knnkm_fit_batched: too many clusters");
  if (!G_ids || !G_d2 || !labels || !C || !counts)
    return knnkm_fail(ctx, KNNKM_EINVAL, "knnkm_fit_batched: null pointer");
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  KNNKM_TRY(upload_jobs(ctx, J, "batch"));
  KNNKM_TRY(build_impl(ctx, X, d, ldx, J, p, G_ids, G_d2));
  KNNKM_WS(ctx, trace, double, "batch_trace", ((int64_t)p->max_iters + 1) * m);
  KNNKM_WS(ctx, glab, int32_t, "batch_labels", J.n);
  int it = 0;
  KNNKM_TRY(fit_impl(ctx, X, d, ldx, J, kq, G_ids, p, glab, C, counts, trace, &it));
  // job-local labels
  {
    int32_t *k32, K;
    int64_t* k64;
    KNNKM_TRY(upload_koff(ctx, kq, "fit", &k32, &k64, &K));
    if (J.job_of)
      k_local_labels<<<grid_for(J.n, 256, 8192), 256, 0, ctx->stream>>>(glab, J.job_of, k32, J.n, labels);
    else
      KNNKM_HIP(ctx, hipMemcpyAsync(labels, glab, sizeof(int32_t) * J.n, hipMemcpyDeviceToDevice, ctx->stream));
  }
  if (trace_host) {
    std::vector<double> tr((size_t)(it + 1) * m);
    KNNKM_HIP(ctx, hipMemcpyAsync(tr.data(), trace, sizeof(double) * tr.size(), hipMemcpyDeviceToHost,
                                  ctx->stream));
    KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < m; ++q)
      for (int t = 0; t <= it; ++t) trace_host[(int64_t)q * (p->max_iters + 1) + t] = tr[(size_t)t * m + q];
  }
  KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return knnkm_check(ctx, "knnkm_fit_batched");
}

// Alg. 2 as printed (boost form), data-parallel rounds (boost.hip): one job.
// trace_dev receives E_0..E_t (Eqn. 4 through Eqn. 2); *rounds_run the
// rounds done (the last one proposed nothing, or t = max_iters).
static knnkm_status boost_impl(knnkm_ctx* ctx, const float* X, int32_t d, int64_t ldx, Jobs& J, int32_t k,
                               const int32_t* G_ids, const knnkm_params* p, int32_t* labels, float* C,
                               int32_t* counts, double* trace_dev, int* rounds_run) {
  const int kappa = p->kappa;
  const int T = p->max_iters;
  const int64_t n = J.n;
  int32_t *k32, K;
  int64_t* k64;
  KNNKM_TRY(upload_koff(ctx, std::vector<int32_t>{k}, "boost", &k32, &k64, &K));
  KNNKM_TRY(init_partition(ctx, X, d, ldx, J, std::vector<int32_t>{k}, p, K, k32, labels, C));
  KNNKM_WS(ctx, rowsq, double, "fit_rowsq", n);
  KNNKM_WS(ctx, sxx, double, "fit_sxx", 1);
  KNNKM_WS(ctx, jmax, uint32_t, "fit_jmax", 1);
  KNNKM_TRY(ks_row_stats(ctx, X, n, d, ldx, 1, nullptr, rowsq, jmax));
  k_range_sum<<<1, 1024, 0, ctx->stream>>>(rowsq, J.n_off, sxx);
  KNNKM_WS(ctx, cs, int32_t, "fit_scale", K);
  KNNKM_TRY(ks_fx_scales(ctx, jmax, 1, k32, K, cs));
  KNNKM_WS(ctx, off, int32_t, "fit_offsets", (int64_t)K + 1);
  KNNKM_WS(ctx, mem, int32_t, "fit_members", n);
  KNNKM_TRY(ks_label_sort(ctx, labels, n, K, counts, off, mem));
  KNNKM_WS(ctx, Dfx, uint64_t, "fit_dfx", (int64_t)K * d * 2);
  KNNKM_WS(ctx, C64, double, "boost_c64", (int64_t)K * d);
  KNNKM_WS(ctx, Iterm, double, "fit_iterm", K);
  KNNKM_TRY(ks_fx_exact_sums(ctx, X, ldx, d, K, off, mem, cs, Dfx));
  KNNKM_TRY(ks_fx_finalize_all(ctx, Dfx, K, d, cs, counts, C, Iterm, C64));
  KNNKM_WS(ctx, trpart, double, "fit_trace_part", TR_SLICES);
  KNNKM_TRY(launch_trace(ctx, Iterm, k64, sxx, J.n_off, 1, K, trpart, trace_dev));
  KNNKM_TRY(knnkm_check(ctx, "boost initialisation"));
  // the moves read rows by position with stride d: a contiguous copy when
  // the caller's rows are strided
  const float* Xc = X;
  if (ldx != d) {
    KNNKM_WS(ctx, xc, float, "boost_rows", n * (int64_t)d);
    KNNKM_HIP(ctx, hipMemcpy2DAsync(xc, sizeof(float) * d, X, sizeof(float) * ldx, sizeof(float) * d, n,
                                    hipMemcpyDeviceToDevice, ctx->stream));
    Xc = xc;
  }
  KNNKM_WS(ctx, nxt, int32_t, "fit_labels2", n);
  KNNKM_WS(ctx, prop, int32_t, "boost_prop", n);
  // active lists: after a round only the samples with a changed cluster
  // among their own and their neighbours' (members of a dirty cluster and
  // the samples listing one in their graph rows) propose again
  if (n * (int64_t)kappa >= INT32_MAX)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "knn_boost_fit: n * kappa must stay below 2^31");
  KNNKM_WS(ctx, rev_off, int32_t, "fit_rev_off", n + 1);
  KNNKM_WS(ctx, rev_src, int32_t, "fit_rev_src", n * (int64_t)kappa);
  KNNKM_WS(ctx, act, uint8_t, "fit_act_p", (n + 3) / 4 * 4);
  KNNKM_WS(ctx, list, int32_t, "as_act_list", n);
  KNNKM_WS(ctx, lcount, int32_t, "fit_list_counts", 1);
  KNNKM_WS(ctx, dmass, int64_t, "fit_dirty_mass", 1);
  KNNKM_TRY(ks_reverse_graph(ctx, G_ids, n, kappa, rev_off, rev_src));
  KNNKM_TRY(ks_fill_i32(ctx, (int32_t*)act, (n + 3) / 4, 0));
  KNNKM_WS(ctx, win, uint64_t, "boost_win", K);
  KNNKM_WS(ctx, dirty, int32_t, "fit_dirty", K);
  KNNKM_WS(ctx, dirty2, int32_t, "fit_dirty2", K);
  KNNKM_WS(ctx, nprop, int64_t, "boost_nprop", (int64_t)T + 1);
  KNNKM_TRY(ks_fill_i32(ctx, dirty, K, 0));
  KNNKM_TRY(ks_fill_i32(ctx, dirty2, K, 0));
  KNNKM_TRY(ks_fill_i64(ctx, nprop, (int64_t)T + 1, 0));
  int32_t *dset = dirty, *dclear = dirty2;
  int t = 0;
  for (t = 1; t <= T; ++t) {
    KNNKM_TRY(ks_boost_propose(ctx, X, n, d, ldx, G_ids, kappa, labels, counts, C64, prop, t > 1 ? list : nullptr,
                               lcount));
    KNNKM_TRY(ks_boost_select(ctx, n, labels, prop, K, p->seed, t, win, nxt, nprop + t));
    // the applied moves into D (exact), sizes, centroids, means, Eqn. 2 terms
    KNNKM_TRY(ks_fx_update(ctx, Xc, n, d, labels, nxt, cs, Dfx, K, counts, dset, C, Iterm, nullptr, nullptr,
                           nullptr, dclear, nullptr, dmass, CShadow{}, C64));
    KNNKM_HIP(ctx, hipMemcpyAsync(labels, nxt, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
    KNNKM_TRY(ks_mark_dirty(ctx, n, labels, dset, rev_off, rev_src, act, dmass, 2 * n / (kappa + 1), nullptr, nullptr,
                            kappa));
    KNNKM_TRY(ks_act_compact(ctx, n, act, list, lcount));
    std::swap(dset, dclear);
    KNNKM_TRY(launch_trace(ctx, Iterm, k64, sxx, J.n_off, 1, K, trpart, trace_dev + t));
    int64_t np = 0;
    KNNKM_HIP(ctx, hipMemcpyAsync(&np, nprop + t, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (np == 0) break;
  }
  *rounds_run = std::min(t, T);
  return knnkm_check(ctx, "boost rounds");
}

extern "C" knnkm_status knn_boost_fit(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, int32_t k,
                                      const int32_t* G_ids, const knnkm_params* p, int32_t* labels, float* C,
                                      int32_t* counts, double* trace_host, int32_t* rounds_run_host) {
  if (!ctx) return KNNKM_EINVAL;
  if (ctx->sticky) return KNNKM_EDEVICE;
  KNNKM_TRY(check_data(ctx, X, n, d, ldx, "knn_boost_fit"));
  KNNKM_TRY(check_params(ctx, p, "knn_boost_fit"));
  if (k < 1 || k > n) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_boost_fit: need 1 <= k <= n");
  const int kappa = p->kappa;
  if (kappa < 1 || kappa > n - 1) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_boost_fit: need 1 <= kappa <= n-1");
  if (kappa > KNNKM_MAX_KAPPA)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "knn_boost_fit: kappa=%d > %d", kappa, KNNKM_MAX_KAPPA);
  if (p->max_iters > 0xFFFF) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_boost_fit: max_iters > 65535");
  if (!labels || !C || !counts || !G_ids) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_boost_fit: null pointer");
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  Jobs J;
  J.m = 1;
  J.n = n;
  J.n_host = {n};
  J.n_off_host = {0, n};
  J.seed_host = {p->seed};
  KNNKM_TRY(upload_jobs(ctx, J, "one"));
  if (p->init == KNNKM_INIT_LABELS) {
    KNNKM_WS(ctx, bad, int64_t, "fit_bad_labels", 1);
    KNNKM_TRY(ks_fill_i64(ctx, bad, 1, 0));
    k_check_labels<<<grid_for(n, 256, 4096), 256, 0, ctx->stream>>>(labels, n, k, (unsigned long long*)bad);
    int64_t nbad = 0;
    KNNKM_HIP(ctx, hipMemcpyAsync(&nbad, bad, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (nbad) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_boost_fit: %lld input labels outside [0, %d)",
                                (long long)nbad, k);
  }
  KNNKM_WS(ctx, trace, double, "fit_trace", (int64_t)p->max_iters + 1);
  int t = 0;
  KNNKM_TRY(boost_impl(ctx, X, d, ldx, J, k, G_ids, p, labels, C, counts, trace, &t));
  if (trace_host)
    KNNKM_HIP(ctx, hipMemcpyAsync(trace_host, trace, sizeof(double) * (size_t)(t + 1), hipMemcpyDeviceToHost,
                                  ctx->stream));
  KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (rounds_run_host) *rounds_run_host = t;
  return knnkm_check(ctx, "knn_boost_fit");
}
