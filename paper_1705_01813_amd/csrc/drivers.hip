// Host drivers: the GK-means^- fit (Alg. 2, Lloyd form) and the KNN graph
// construction (Alg. 3).  Every step runs in this library's kernels on the
// context stream; the host only sequences launches.
#include "common.h"

// k distinct sample ids by Floyd's algorithm (one thread; bitmap membership).
__global__ void k_random_init_ids(int64_t n, int32_t k, uint64_t seed, uint32_t* __restrict__ bitmap,
                                  int32_t* __restrict__ ids) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const uint64_t key = sm_key(seed, sm_stream(RNG_RANDOM_INIT, 0, 0));
  const int64_t base = n - k;
  for (int64_t j = base; j < n; ++j) {
    const int64_t t = sm_below(sm_draw(key, (uint64_t)(j - base)), (uint32_t)(j + 1));
    const bool seen = (bitmap[t >> 5] >> (t & 31)) & 1u;
    const int64_t v = seen ? j : t;
    bitmap[v >> 5] |= 1u << (v & 31);
    ids[j - base] = (int32_t)v;
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

// E_t = (sum ||x||^2 - I) / n  (Eqn. 4 through the Eqn. 2 identity)
__global__ void k_trace(const double* __restrict__ sxx, const double* __restrict__ isum, double inv_n,
                        double* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = (sxx[0] - isum[0]) * inv_n;
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
  if (p->init != KNNKM_INIT_TWOMEANS && p->init != KNNKM_INIT_RANDOM)
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
  const int T = p->max_iters;
  KNNKM_WS(ctx, lab2, int32_t, "fit_labels2", n);
  KNNKM_WS(ctx, off, int32_t, "fit_offsets", (int64_t)k + 1);
  KNNKM_WS(ctx, mem, int32_t, "fit_members", n);
  KNNKM_WS(ctx, Iterm, double, "fit_iterm", k);
  KNNKM_WS(ctx, scal, double, "fit_scalars", 2);
  KNNKM_WS(ctx, trace, double, "fit_trace", (int64_t)T + 1);
  KNNKM_WS(ctx, moved, int64_t, "fit_moved", (int64_t)T + 1);
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

  // initial partition
  if (p->init == KNNKM_INIT_RANDOM) {
    KNNKM_WS(ctx, bitmap, uint32_t, "fit_bitmap", (n + 31) / 32);
    KNNKM_WS(ctx, ids, int32_t, "fit_init_ids", k);
    KNNKM_TRY(ks_fill_i32(ctx, (int32_t*)bitmap, (n + 31) / 32, 0));
    k_random_init_ids<<<1, 64, 0, ctx->stream>>>(n, k, p->seed, bitmap, ids);
    k_gather_rows<<<grid_for((int64_t)k * d, 256, 4096), 256, 0, ctx->stream>>>(X, d, ldx, ids, k, C);
    KNNKM_TRY(knnkm_check(ctx, "random init"));
    KNNKM_TRY(ks_assign(ctx, X, n, d, ldx, C, k, nullptr, k, nullptr, labels, nullptr, nullptr, nullptr,
                        true));
  } else {
    KNNKM_TRY(ks_twomeans(ctx, X, n, d, ldx, k, p->seed, KNNKM_ROUND_FIT, p->bisect_iters, labels));
    KNNKM_TRY(ks_fill_i32(ctx, (int32_t*)C, (int64_t)k * d, 0));
  }
  KNNKM_TRY(ks_sqdist_sum(ctx, X, n, d, ldx, nullptr, nullptr, scal, 1.0));
  KNNKM_TRY(ks_label_sort(ctx, labels, n, k, counts, off, mem));
  KNNKM_TRY(ks_segsum(ctx, X, n, d, ldx, k, counts, off, mem, C, nullptr, Iterm));
  KNNKM_TRY(ks_sum_f64(ctx, Iterm, k, scal + 1));
  k_trace<<<1, 64, 0, ctx->stream>>>(scal, scal + 1, 1.0 / (double)n, trace);
  mark(3);

  int32_t* cur = labels;
  int32_t* nxt = lab2;
  int it = 0;
  for (int t = 1; t <= T; ++t) {
    mark(6 + 2 * (t - 1));
    KNNKM_TRY(ks_assign(ctx, X, n, d, ldx, C, k, G_ids, kappa, cur, nxt, nullptr, moved + t, mem, dense));
    mark(7 + 2 * (t - 1));
    if (ctx->timing) ctx->assign_n = t;
    KNNKM_TRY(ks_label_sort(ctx, nxt, n, k, counts, off, mem));
    KNNKM_TRY(ks_segsum(ctx, X, n, d, ldx, k, counts, off, mem, C, nullptr, Iterm));
    KNNKM_TRY(ks_sum_f64(ctx, Iterm, k, scal + 1));
    k_trace<<<1, 64, 0, ctx->stream>>>(scal, scal + 1, 1.0 / (double)n, trace + t);
    KNNKM_TRY(knnkm_check(ctx, "fit iteration"));
    std::swap(cur, nxt);
    it = t;
    if (p->early_stop) {
      int64_t mv = -1;
      KNNKM_HIP(ctx, hipMemcpyAsync(&mv, moved + t, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
      KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
      if (mv == 0) break;
    }
  }
  mark(4);
  if (cur != labels)
    KNNKM_HIP(ctx, hipMemcpyAsync(labels, cur, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice,
                                  ctx->stream));
  if (trace_host)
    KNNKM_HIP(ctx, hipMemcpyAsync(trace_host, trace, sizeof(double) * (size_t)(it + 1),
                                  hipMemcpyDeviceToHost, ctx->stream));
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
  const int32_t k0 = (int32_t)std::max<int64_t>(1, n / p->xi);
  // phase events 0 (start) and 1 (end)
  auto mark = [&](int e) {
    if (ctx->timing) {
      hipEvent_t h = knnkm_event(ctx, e);
      if (h) (void)hipEventRecord(h, ctx->stream);
    }
  };
  if (ctx->timing) ctx->build_ev = 0;
  mark(0);
  KNNKM_TRY(ks_graph_init(ctx, X, n, d, ldx, kappa, p->seed, G_ids, G_d2));
  if (p->tau == 0) {
    mark(1);
    return KNNKM_OK;
  }
  KNNKM_WS(ctx, lab, int32_t, "kb_labels", n);
  KNNKM_WS(ctx, lab2, int32_t, "kb_labels2", n);
  KNNKM_WS(ctx, counts, int32_t, "kb_counts", k0);
  KNNKM_WS(ctx, off, int32_t, "kb_offsets", (int64_t)k0 + 1);
  KNNKM_WS(ctx, mem, int32_t, "kb_members", n);
  KNNKM_WS(ctx, C, float, "kb_centroids", (int64_t)k0 * d);
  const bool dense = kappa >= k0;
  for (int t = 0; t < p->tau; ++t) {
    KNNKM_TRY(ks_twomeans(ctx, X, n, d, ldx, k0, p->seed, t, p->bisect_iters, lab));
    KNNKM_TRY(ks_label_sort(ctx, lab, n, k0, counts, off, mem));
    KNNKM_TRY(ks_segsum(ctx, X, n, d, ldx, k0, counts, off, mem, C, nullptr, nullptr));
    KNNKM_TRY(ks_assign(ctx, X, n, d, ldx, C, k0, G_ids, kappa, lab, lab2, nullptr, nullptr, mem, dense));
    KNNKM_TRY(ks_refine(ctx, X, n, d, ldx, lab2, k0, p->precision, G_ids, G_d2, kappa));
  }
  mark(1);
  return KNNKM_OK;
}
