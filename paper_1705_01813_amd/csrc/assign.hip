// Graph-restricted assignment (Alg. 2 candidate collection; Lloyd form of
// Sec. 4.2): each sample compares itself only with the centroids of the
// clusters its kappa neighbours belong to, plus its own cluster.
//
// One wavefront per sample; lane l holds dimensions l, l+64, ... of x_i.
//  * Candidate collection: lanes 0..kappa read the labels of the sample and
//    of its neighbours (coalesced row of G, then label gathers); duplicates are
//    removed with a ballot loop that peels one distinct label per step, so the
//    candidate ids come out wave-uniform and the centroid rows are read with a
//    scalar base address.
//  * Distances are evaluated in float32 (fixed lane -> dimension order, then a
//    butterfly reduction) while the smallest and second smallest values are
//    tracked.  When the two are closer than the rigorous float32 error bound,
//    every candidate inside that margin is re-evaluated in float64 and the tie
//    rule (stay unless strictly better; smallest id among equal minima) is
//    applied to the float64 values.  Decisions therefore match a float64
//    evaluation and do not depend on the launch configuration.
//  * Samples are visited in the order given by `order` (the previous
//    partition's members, so consecutive waves share candidate centroids);
//    blocks are remapped so that each XCD walks a contiguous range of it.
#include <cfloat>

#include "common.h"

#define ASSIGN_WAVES 4
#define ASSIGN_PER_BLOCK 64

template <int T>
struct SampleRow {
  float x[T];
};

template <int T>
__device__ inline float eval32(const SampleRow<T>& s, const float* __restrict__ cr, int d, int lane) {
  float acc = 0.f;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    int dim = lane + 64 * t;
    if (dim < d) {
      float df = s.x[t] - cr[dim];
      acc = fmaf(df, df, acc);
    }
  }
  return wave_sum(acc);
}

template <int T>
__device__ inline double eval64(const SampleRow<T>& s, const float* __restrict__ cr, int d, int lane) {
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    int dim = lane + 64 * t;
    if (dim < d) {
      double df = (double)s.x[t] - (double)cr[dim];
      acc = fma(df, df, acc);
    }
  }
  return wave_sum(acc);
}

// Visit the distinct candidate labels of a sample, calling f(q) with a
// wave-uniform q.  Entry 0 is the sample's own label, entries 1..kappa the
// labels of its neighbours.
struct CandSet {
  int v[3];
  bool valid[3];
};

__device__ inline void load_cands(CandSet& cs, const int* __restrict__ G, int64_t i, int kappa,
                                  const int* __restrict__ lab_in, int cur, int lane) {
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    int e = lane + 64 * s;
    cs.valid[s] = e <= kappa;
    cs.v[s] = -1;
    if (e == 0)
      cs.v[s] = cur;
    else if (e <= kappa)
      cs.v[s] = lab_in[G[i * kappa + (e - 1)]];
  }
}

template <typename F>
__device__ inline void for_each_cand(const CandSet& cs, F&& f) {
  bool pend[3] = {cs.valid[0], cs.valid[1], cs.valid[2]};
  while (true) {
    uint64_t m0 = __ballot(pend[0]);
    uint64_t m1 = __ballot(pend[1]);
    uint64_t m2 = __ballot(pend[2]);
    int q;
    if (m0)
      q = __builtin_amdgcn_readlane(cs.v[0], __builtin_ctzll(m0));
    else if (m1)
      q = __builtin_amdgcn_readlane(cs.v[1], __builtin_ctzll(m1));
    else if (m2)
      q = __builtin_amdgcn_readlane(cs.v[2], __builtin_ctzll(m2));
    else
      break;
#pragma unroll
    for (int s = 0; s < 3; ++s)
      if (pend[s] && cs.v[s] == q) pend[s] = false;
    f(q);
  }
}

template <int T>
__global__ __launch_bounds__(256) void k_assign(
    const float* __restrict__ X, int n, int d, int64_t ldx, const float* __restrict__ C, int k,
    const int* __restrict__ G, int kappa, const int* __restrict__ lab_in, int* __restrict__ lab_out,
    float* __restrict__ best_out, unsigned long long* __restrict__ moved_acc,
    const int* __restrict__ order, int dense, int nchunks, double rel) {
  __shared__ unsigned int block_moved;
  if (threadIdx.x == 0) block_moved = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // XCD-aware chunk mapping: hardware places block b on XCD b % 8.
  const int per_xcd = gridDim.x / 8;
  const int chunk = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  unsigned int my_moved = 0;
  if (chunk < nchunks) {
    const int64_t start = (int64_t)chunk * ASSIGN_PER_BLOCK;
    const int64_t end = min((int64_t)n, start + ASSIGN_PER_BLOCK);
    for (int64_t idx = start + w; idx < end; idx += ASSIGN_WAVES) {
      const int64_t i = order ? (int64_t)order[idx] : idx;
      SampleRow<T> s;
      const float* xr = X + i * ldx;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        int dim = lane + 64 * t;
        s.x[t] = dim < d ? xr[dim] : 0.f;
      }
      const int cur = lab_in ? lab_in[i] : -1;
      CandSet cs;
      if (!dense) load_cands(cs, G, i, kappa, lab_in, cur, lane);

      // pass 1: float32 distances, best and second best
      float b1 = FLT_MAX, b2 = FLT_MAX;
      int q1 = -1;
      auto pass1 = [&](int q) {
        float dq = eval32<T>(s, C + (int64_t)q * d, d, lane);
        if (dq < b1 || (dq == b1 && q < q1)) {
          if (q1 >= 0) b2 = fminf(b2, b1);
          b1 = dq;
          q1 = q;
        } else {
          b2 = fminf(b2, dq);
        }
      };
      if (dense)
        for (int q = 0; q < k; ++q) pass1(q);
      else
        for_each_cand(cs, pass1);

      const double thr = (double)b1 * (1.0 + rel) / (1.0 - rel) + 1e-30;
      int result = q1;
      float bestv = b1;
      if ((double)b2 <= thr) {
        // pass 2: float64 re-evaluation of every candidate inside the margin
        double m64 = DBL_MAX, cur64 = -1.0;
        int q64 = -1;
        auto pass2 = [&](int q) {
          float dq = eval32<T>(s, C + (int64_t)q * d, d, lane);
          if ((double)dq <= thr) {
            double e = eval64<T>(s, C + (int64_t)q * d, d, lane);
            if (q == cur) cur64 = e;
            if (e < m64 || (e == m64 && q < q64)) {
              m64 = e;
              q64 = q;
            }
          }
        };
        if (dense)
          for (int q = 0; q < k; ++q) pass2(q);
        else
          for_each_cand(cs, pass2);
        if (cur >= 0 && cur64 >= 0.0 && cur64 == m64) {
          result = cur;
          bestv = (float)cur64;
        } else {
          result = q64;
          bestv = (float)m64;
        }
      }
      if (lane == 0) {
        lab_out[i] = result;
        if (best_out) best_out[i] = bestv;
      }
      if (cur >= 0 && result != cur) my_moved++;
    }
  }
  if (moved_acc) {
    if (lane == 0 && my_moved) atomicAdd(&block_moved, my_moved);
    __syncthreads();
    if (threadIdx.x == 0 && block_moved) atomicAdd(moved_acc, (unsigned long long)block_moved);
  }
}

knnkm_status ks_assign(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                       const float* C, int32_t k, const int32_t* G_ids, int32_t kappa,
                       const int32_t* labels_in, int32_t* labels_out, float* best_d2,
                       int64_t* n_moved, const int32_t* order, bool dense) {
  if (n_moved) KNNKM_TRY(ks_fill_i64(ctx, n_moved, 1, 0));
  if (n == 0) return KNNKM_OK;
  const int T = (d + 63) / 64;
  const int nchunks = (int)((n + ASSIGN_PER_BLOCK - 1) / ASSIGN_PER_BLOCK);
  const int grid = ((nchunks + 7) / 8) * 8;
  const double rel = (double)(T + 10) * 0x1p-23;
  unsigned long long* acc = (unsigned long long*)n_moved;
#define LAUNCH(TT)                                                                             \
  k_assign<TT><<<grid, 256, 0, ctx->stream>>>(X, (int)n, d, ldx, C, k, G_ids, kappa, labels_in, \
                                              labels_out, best_d2, acc, order, dense ? 1 : 0,   \
                                              nchunks, rel)
  switch (T) {
    case 1: LAUNCH(1); break;
    case 2: LAUNCH(2); break;
    case 3: LAUNCH(3); break;
    case 4: LAUNCH(4); break;
    case 5: LAUNCH(5); break;
    case 6: LAUNCH(6); break;
    case 7: LAUNCH(7); break;
    case 8: LAUNCH(8); break;
    default: return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "knn_assign: d=%d > %d", d, KNNKM_MAX_D);
  }
#undef LAUNCH
  return knnkm_check(ctx, "knn_assign");
}

extern "C" knnkm_status knn_assign(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                   const float* C, int32_t k, const int32_t* G_ids, int32_t kappa,
                                   const int32_t* labels_in, int32_t* labels_out, float* best_d2,
                                   int64_t* n_moved) {
  if (!ctx) return KNNKM_EINVAL;
  if (ctx->sticky) return KNNKM_EDEVICE;
  if (n < 1 || n > INT32_MAX) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_assign: n=%lld out of range", (long long)n);
  if (d < 1 || ldx < d) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_assign: need d >= 1 and ldx >= d");
  if (d > KNNKM_MAX_D) return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "knn_assign: d=%d > %d", d, KNNKM_MAX_D);
  if (k < 1 || k > n) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_assign: need 1 <= k <= n");
  const bool dense = kappa >= k;
  if (kappa < 1 || (!dense && kappa > n - 1))
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_assign: need 1 <= kappa <= n-1");
  if (!dense && kappa > KNNKM_MAX_KAPPA)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "knn_assign: kappa=%d > %d", kappa, KNNKM_MAX_KAPPA);
  if (!X || !C || !labels_in || !labels_out || (!dense && !G_ids))
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_assign: null pointer");
  if (labels_in == labels_out) return knnkm_fail(ctx, KNNKM_EINVAL, "knn_assign: labels_in aliases labels_out");
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  return ks_assign(ctx, X, n, d, ldx, C, k, G_ids, kappa, labels_in, labels_out, best_d2, n_moved,
                   nullptr, dense);
}
