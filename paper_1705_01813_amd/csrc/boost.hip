// Boost form of GK-means (Alg. 2 as printed; Sec. 3.1, Eqn. 3), data-parallel.
//
// Alg. 2 moves a sample x from its cluster u to the cluster v of its
// neighbours that maximises the gain of I = sum_r D_r'D_r / n_r (Eqn. 2), as
// soon as that gain (Eqn. 3) is positive.  In the weighted form of Eqn. 3,
//   dI = n_u/(n_u-1) ||x - c_u||^2 - n_v/(n_v+1) ||x - c_v||^2
// (the first term 0 when the move empties u), with c_r = D_r / n_r.
//
// A round: every sample computes its best move against the same state
// (k_boost_propose; a sample none of whose clusters -- its own, those of its
// neighbours -- changed since its last proposal keeps it); each cluster keeps, among the proposals touching it as
// source or target, the one with the largest priority key (k_boost_bid); a
// proposal that keeps both of its clusters is applied (k_boost_apply).  No
// two applied moves share a cluster, so each one's gain is unchanged by the
// others and I rises by exactly their sum: a round is the same moves made one
// after the other by Alg. 2.
//
// Decisions are taken in the arithmetic that the oracle fixes, so that they
// agree bit for bit: the float64 means c_r = D_r / n_r of the exact
// fixed-point sums, every squared distance summed over the dimensions in
// order by one lane with one rounding per operation (no fused multiply-add),
// the coefficients as float64 quotients; the best target is the smallest
// weighted distance (smallest id among equal ones) and the move is proposed
// when the own weighted distance is strictly larger.
#include <cfloat>
#include <climits>

#include "common.h"

namespace {

constexpr uint64_t BOOST_PURPOSE = 4;  // random-number stream of the priorities

// Weighted squared distance of the row in LDS to the float64 mean of a
// cluster of nr members: coefficient nr/(nr-1) for the own cluster (0 when
// nr = 1), nr/(nr+1) for a target.
__device__ double boost_weighted(const float* __restrict__ xs, const double* __restrict__ c, int d, int nr, bool own) {
#pragma clang fp contract(off)
  double dist = 0.0;
  for (int j = 0; j < d; ++j) {
    const double df = (double)xs[j] - c[j];
    dist = dist + df * df;
  }
  const double n = (double)nr;
  const double coef = own ? (nr > 1 ? n / (n - 1.0) : 0.0) : n / (n + 1.0);
  return coef * dist;
}

// One wavefront per sample; lane e takes graph entries e, e + 64, ... (entry
// 0: the own cluster), each by itself over all dimensions.
__global__ __launch_bounds__(256) void k_boost_propose(const float* __restrict__ X, int64_t n, int d, int64_t ldx,
                                                       const int32_t* __restrict__ G, int kappa,
                                                       const int32_t* __restrict__ lab,
                                                       const int32_t* __restrict__ cnt,
                                                       const double* __restrict__ C64, int32_t* __restrict__ prop,
                                                       const int32_t* __restrict__ list,
                                                       const int32_t* __restrict__ count) {
  __shared__ float xs[4][KNNKM_MAX_D];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t m = list ? (int64_t)*count : n;
  for (int64_t li = blockIdx.x * 4 + w; li < m; li += (int64_t)gridDim.x * 4) {
    const int64_t i = list ? (int64_t)(list[li] & 0x7FFFFFFF) : li;
    for (int j = lane; j < d; j += 64) xs[w][j] = X[i * ldx + j];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int u = lab[i];
    double wu = 0.0, bw = DBL_MAX;
    int br = INT_MAX;
    for (int e0 = 0; e0 <= kappa; e0 += 64) {
      const int e = e0 + lane;
      if (e == 0) {
        wu = boost_weighted(xs[w], C64 + (int64_t)u * d, d, cnt[u], true);
      } else if (e <= kappa) {
        const int r = lab[G[i * kappa + (e - 1)]];
        if (r != u) {
          const double wr = boost_weighted(xs[w], C64 + (int64_t)r * d, d, cnt[r], false);
          if (wr < bw || (wr == bw && r < br)) {
            bw = wr;
            br = r;
          }
        }
      }
    }
    wu = __shfl(wu, 0, 64);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ow = __shfl_xor(bw, o, 64);
      const int orr = __shfl_xor(br, o, 64);
      if (ow < bw || (ow == bw && orr < br)) {
        bw = ow;
        br = orr;
      }
    }
    if (lane == 0) prop[i] = (br != INT_MAX && wu > bw) ? br : -1;
    // every lane has read the row before the next sample overwrites it
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

__device__ inline uint64_t boost_key(uint64_t seed, int32_t round, int64_t i) {
  const uint64_t h = sm_draw(sm_key(seed, sm_stream(BOOST_PURPOSE, (uint64_t)round, (uint64_t)i)), 0);
  return ((h >> 32) << 32) | (uint64_t)(uint32_t)i;
}

// Bids of every proposal on its two clusters; *nprop += proposals.
__global__ __launch_bounds__(256) void k_boost_bid(int64_t n, const int32_t* __restrict__ lab,
                                                   const int32_t* __restrict__ prop, uint64_t seed, int32_t round,
                                                   unsigned long long* __restrict__ win,
                                                   unsigned long long* __restrict__ nprop) {
  __shared__ unsigned int block_prop;
  if (threadIdx.x == 0) block_prop = 0;
  __syncthreads();
  unsigned int my = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int v = prop[i];
    if (v < 0) continue;
    ++my;
    const unsigned long long key = boost_key(seed, round, i);
    atomicMax(&win[lab[i]], key);
    atomicMax(&win[v], key);
  }
  if (my) atomicAdd(&block_prop, my);
  __syncthreads();
  if (threadIdx.x == 0 && block_prop) atomicAdd(nprop, (unsigned long long)block_prop);
}

__global__ void k_boost_apply(int64_t n, const int32_t* __restrict__ lab, const int32_t* __restrict__ prop,
                              uint64_t seed, int32_t round, const unsigned long long* __restrict__ win,
                              int32_t* __restrict__ next) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int u = lab[i], v = prop[i];
    int out = u;
    if (v >= 0) {
      const unsigned long long key = boost_key(seed, round, i);
      if (win[u] == key && win[v] == key) out = v;
    }
    next[i] = out;
  }
}

}  // namespace

knnkm_status ks_boost_propose(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, const int32_t* G,
                              int32_t kappa, const int32_t* labels, const int32_t* counts, const double* C64,
                              int32_t* prop, const int32_t* list, const int32_t* count) {
  if (n <= 0) return KNNKM_OK;
  k_boost_propose<<<grid_for(n, 4, 65536), 256, 0, ctx->stream>>>(X, n, d, ldx, G, kappa, labels, counts, C64, prop,
                                                                  list, count);
  return knnkm_check(ctx, "boost proposals");
}

knnkm_status ks_boost_select(knnkm_ctx* ctx, int64_t n, const int32_t* labels, const int32_t* prop, int32_t K,
                             uint64_t seed, int32_t round, uint64_t* win, int32_t* next, int64_t* nprop) {
  KNNKM_TRY(ks_fill_i64(ctx, (int64_t*)win, K, 0));
  k_boost_bid<<<grid_for(n, 256, 8192), 256, 0, ctx->stream>>>(n, labels, prop, seed, round,
                                                               (unsigned long long*)win, (unsigned long long*)nprop);
  k_boost_apply<<<grid_for(n, 256, 8192), 256, 0, ctx->stream>>>(n, labels, prop, seed, round,
                                                                 (const unsigned long long*)win, next);
  return knnkm_check(ctx, "boost selection");
}
