// Graph-restricted assignment (Alg. 2 candidate collection; Lloyd form of
// Sec. 4.2): each sample compares itself only with the centroids of the
// clusters its kappa neighbours belong to, plus its own cluster.
//
// A row group of L lanes handles one sample (V dimensions per lane), so a
// wavefront works on 64/L samples at once:
//  * Candidate collection: the group's lanes read the sample's own label and
//    the labels of its kappa neighbours (coalesced graph row, then label
//    gathers), S entries per lane.  Distinct labels are peeled one per step
//    with a ballot restricted to the group, so every candidate is
//    group-uniform and its centroid row is read as one contiguous segment.
//  * Distances are evaluated in float32 (fixed lane -> dimension order, fixed
//    DPP reduction tree) while the smallest and second smallest values are
//    tracked.  When the two are closer than the rigorous float32 error bound,
//    every candidate inside that margin is re-evaluated in float64 and the tie
//    rule (stay unless strictly better; smallest id among equal minima) is
//    applied to the float64 values, so decisions match a float64 evaluation.
//  * Samples are visited in the order given by `order` (the previous
//    partition's members, so neighbouring groups share candidate centroids);
//    blocks are remapped so that each XCD walks a contiguous range of it.
#include <algorithm>
#include <cfloat>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "rowgroup.h"

#define MAX_SLOTS 8

template <int V>
__device__ inline float dist32(const float (&x)[V], const float (&c)[V]) {
  float acc = 0.f;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const float df = x[e] - c[e];
    acc = fmaf(df, df, acc);
  }
  return acc;
}
template <int V>
__device__ inline float part32(const float (&x)[V], const float* __restrict__ cr, int j, int d, bool vec) {
  float c[V];
  load_row<V>(c, cr, j, d, vec);
  return dist32<V>(x, c);
}

template <int V>
__device__ inline double part64(const float (&x)[V], const float* __restrict__ cr, int j, int d, bool vec) {
  float c[V];
  load_row<V>(c, cr, j, d, vec);
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const double df = (double)x[e] - (double)c[e];
    acc = fma(df, df, acc);
  }
  return acc;
}

// Visit the distinct candidate labels of the group's sample in a fixed order
// (first occurrence among entries 0..kappa, entry 0 = own label), calling
// f(q) with a group-uniform q.
template <int L, int SM, typename F>
__device__ inline void for_each_cand(const int (&v)[SM], const bool (&valid)[SM], uint64_t gmask, F&& f) {
  bool pend[SM];
#pragma unroll
  for (int s = 0; s < SM; ++s) pend[s] = valid[s];
  while (true) {
    int q = -1;
#pragma unroll
    for (int s = 0; s < SM; ++s) {
      if (q < 0) {
        const uint64_t m = __ballot(pend[s]) & gmask;
        if (m) q = __shfl(v[s], (int)__builtin_ctzll(m), 64);
      }
    }
    if (q < 0) break;
#pragma unroll
    for (int s = 0; s < SM; ++s)
      if (pend[s] && v[s] == q) pend[s] = false;
    f(q);
  }
}

// The same visit, with the centroid row slice of the next candidate loaded
// while the current one is used: f(q, c) gets candidate q and its dims
// [j*V, j*V + V) of C.
template <int L, int V, int SM, typename F>
__device__ inline void for_each_cand_row(const int (&v)[SM], const bool (&valid)[SM], uint64_t gmask,
                                         const float* __restrict__ C, int d, int j, bool vec, F&& f) {
  bool pend[SM];
#pragma unroll
  for (int s = 0; s < SM; ++s) pend[s] = valid[s];
  auto next = [&]() -> int {
    int q = -1;
#pragma unroll
    for (int s = 0; s < SM; ++s) {
      if (q < 0) {
        const uint64_t m = __ballot(pend[s]) & gmask;
        if (m) q = __shfl(v[s], (int)__builtin_ctzll(m), 64);
      }
    }
    if (q >= 0) {
#pragma unroll
      for (int s = 0; s < SM; ++s)
        if (pend[s] && v[s] == q) pend[s] = false;
    }
    return q;
  };
  int q = next();
  if (q < 0) return;
  float c[V];
  load_row<V>(c, C + (int64_t)q * d, j, d, vec);
  while (true) {
    const int qn = next();
    float cn[V];
    if (qn >= 0) load_row<V>(cn, C + (int64_t)qn * d, j, d, vec);
    f(q, c);
    if (qn < 0) break;
    q = qn;
#pragma unroll
    for (int e = 0; e < V; ++e) c[e] = cn[e];
  }
}

// The candidate visits of GS samples of a group advanced together: each step
// takes the next candidate of every sample still visiting (use[p]) and loads
// its centroid slice while the previous ones are used.  Every sample sees
// its own candidates in its own order.  f(p, q, c).
template <int L, int V, int SM, int GS, typename F>
__device__ inline void for_each_cand_rows(const int (&v)[GS][SM], const bool (&valid)[GS][SM],
                                          const bool (&use)[GS], uint64_t gmask, const float* __restrict__ C,
                                          int d, int j, bool vec, F&& f) {
  bool pend[GS][SM];
#pragma unroll
  for (int p = 0; p < GS; ++p)
#pragma unroll
    for (int s = 0; s < SM; ++s) pend[p][s] = use[p] && valid[p][s];
  auto next = [&](int p) -> int {
    int q = -1;
#pragma unroll
    for (int s = 0; s < SM; ++s) {
      if (q < 0) {
        const uint64_t m = __ballot(pend[p][s]) & gmask;
        if (m) q = __shfl(v[p][s], (int)__builtin_ctzll(m), 64);
      }
    }
    if (q >= 0) {
#pragma unroll
      for (int s = 0; s < SM; ++s)
        if (pend[p][s] && v[p][s] == q) pend[p][s] = false;
    }
    return q;
  };
  int q[GS];
  float c[GS][V];
  bool any = false;
#pragma unroll
  for (int p = 0; p < GS; ++p) {
    q[p] = next(p);
    if (q[p] >= 0) {
      load_row<V>(c[p], C + (int64_t)q[p] * d, j, d, vec);
      any = true;
    }
  }
  while (any) {  // group-uniform
    int qn[GS];
    float cn[GS][V];
#pragma unroll
    for (int p = 0; p < GS; ++p) {
      qn[p] = q[p] >= 0 ? next(p) : -1;
      if (qn[p] >= 0) load_row<V>(cn[p], C + (int64_t)qn[p] * d, j, d, vec);
    }
    any = false;
#pragma unroll
    for (int p = 0; p < GS; ++p) {
      if (q[p] >= 0) f(p, q[p], c[p]);
      q[p] = qn[p];
      if (q[p] >= 0) {
        any = true;
#pragma unroll
        for (int e = 0; e < V; ++e) c[p][e] = cn[p][e];
      }
    }
  }
}

// One row group (L lanes) per sample, GS samples per group at a time: the
// loads of each dependency level (sample ids; rows, own labels and graph
// rows; neighbour labels) are issued for all GS samples before any is used,
// so a wavefront keeps several sample rows in flight.  SM candidate slots
// per lane (SM * L >= kappa + 1).
//
// A sample whose neighbours all share its own cluster has that cluster as its
// only candidate, so it stays without any distance being evaluated (unless
// best distances are requested).  With LAZY the sample's row is loaded only
// when a distance is needed, after its neighbour labels are known (fewer
// bytes, one more dependent step); without it the row is loaded first.
// eval_acc counts the samples whose distances were evaluated.
//
// Active sets (fit sweeps): act_in (nullable) marks the samples to look at;
// any other sample is known to have its own cluster as the only candidate
// and keeps its label.  act_out (nullable) receives 1 for every sample whose
// distances were evaluated (it had several candidates, so it is looked at
// again next sweep) and 0 otherwise; the update then marks the samples whose
// own or neighbours' labels change.
template <int L, int V, int GS, int SM, int LAZY>
__global__ __launch_bounds__(256) void k_assign(
    const float* __restrict__ X, int n, int d, int64_t ldx, const float* __restrict__ C, int k,
    const int* __restrict__ G, int kappa, const int* __restrict__ lab_in, int* __restrict__ lab_out,
    float* __restrict__ best_out, unsigned long long* __restrict__ moved_acc,
    unsigned long long* __restrict__ eval_acc, const int* __restrict__ order, int dense, int nchunks, int pb,
    double rel, int vec_x, int vec_c, const int* __restrict__ job_of, const int* __restrict__ kbase,
    const uint8_t* __restrict__ act_in, uint8_t* __restrict__ act_out) {
  constexpr int GW = 64 / L;           // samples per wavefront and pass
  constexpr int PASS = 4 * GW * GS;    // samples per block and pass
  __shared__ unsigned int block_moved, block_eval;
  if (threadIdx.x == 0) {
    block_moved = 0;
    block_eval = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane / L, j = lane % L;
  const uint64_t gmask = group_mask<L>(g);
  // XCD-aware chunk mapping: hardware places block b on XCD b % 8.
  const int per_xcd = gridDim.x / 8;
  const int chunk = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  unsigned int my_moved = 0, my_eval = 0;
  if (chunk < nchunks) {
    const int64_t start = (int64_t)chunk * pb;
    const int64_t end = min((int64_t)n, start + pb);
    for (int64_t base = start; base < end; base += PASS) {
      int64_t ii[GS];
      bool act[GS], live[GS];
#pragma unroll
      for (int p = 0; p < GS; ++p) {
        const int64_t idx = base + w * GW + g + p * 4 * GW;
        act[p] = idx < end;
        ii[p] = act[p] ? (order ? (int64_t)order[idx] : idx) : 0;
      }
#pragma unroll
      for (int p = 0; p < GS; ++p) live[p] = act[p] && (!act_in || act_in[ii[p]] != 0);
      float x[GS][V];
      int cur[GS], kb[GS], kc[GS], nb[GS][SM];
      bool dense_i[GS];
#pragma unroll
      for (int p = 0; p < GS; ++p) {
        const int64_t i = ii[p];
        if (live[p] && !LAZY) {
          load_row<V>(x[p], X + i * ldx, j, d, vec_x);
        } else {
#pragma unroll
          for (int e = 0; e < V; ++e) x[p][e] = 0.f;
        }
        cur[p] = (act[p] && lab_in) ? lab_in[i] : -1;
        kb[p] = 0;
        kc[p] = k;
        dense_i[p] = dense;
        if (job_of && live[p]) {
          const int q = job_of[i];
          kb[p] = kbase[q];
          kc[p] = kbase[q + 1] - kb[p];
          dense_i[p] = dense || kappa >= kc[p];
        }
#pragma unroll
        for (int s = 0; s < SM; ++s) {
          const int e = j + L * s;
          nb[p][s] = (live[p] && !dense_i[p] && e >= 1 && e <= kappa) ? G[i * kappa + (e - 1)] : -1;
        }
      }
      int cv[GS][SM];
      bool valid[GS][SM];
#pragma unroll
      for (int p = 0; p < GS; ++p)
#pragma unroll
        for (int s = 0; s < SM; ++s) {
          const int e = j + L * s;
          valid[p][s] = live[p] && !dense_i[p] && e <= kappa;
          cv[p][s] = !valid[p][s] ? -1 : (e == 0 ? cur[p] : lab_in[nb[p][s]]);
        }
      // the own cluster as the only candidate decides the sample
      bool single[GS];
#pragma unroll
      for (int p = 0; p < GS; ++p) {
        bool other = false;
#pragma unroll
        for (int s = 0; s < SM; ++s) other = other || (valid[p][s] && cv[p][s] != cur[p]);
        single[p] = live[p] && !dense_i[p] && !best_out && cur[p] >= 0 && (__ballot(other) & gmask) == 0;
      }
      if (LAZY) {
#pragma unroll
        for (int p = 0; p < GS; ++p)
          if (live[p] && !single[p]) load_row<V>(x[p], X + ii[p] * ldx, j, d, vec_x);
      }

#pragma unroll
      for (int p = 0; p < GS; ++p) {
        if (!act[p]) continue;       // group-uniform
        if (!live[p] || single[p]) {  // group-uniform
          if (j == 0) {
            lab_out[ii[p]] = cur[p];
            if (act_out) act_out[ii[p]] = 0;
          }
          continue;
        }
        if (j == 0) my_eval++;
        // pass 1: float32 distances, best and second best
        float b1 = FLT_MAX, b2 = FLT_MAX;
        int q1 = -1;
        auto pass1 = [&](int q, float dq) {
          if (dq < b1 || (dq == b1 && q < q1)) {
            if (q1 >= 0) b2 = fminf(b2, b1);
            b1 = dq;
            q1 = q;
          } else {
            b2 = fminf(b2, dq);
          }
        };
        if (dense_i[p])
          for (int q = kb[p]; q < kb[p] + kc[p]; ++q)
            pass1(q, group_sum<L>(part32<V>(x[p], C + (int64_t)q * d, j, d, vec_c)));
        else
          for_each_cand_row<L, V, SM>(cv[p], valid[p], gmask, C, d, j, vec_c,
                                      [&](int q, const float (&c)[V]) { pass1(q, group_sum<L>(dist32<V>(x[p], c))); });

        const double thr = (double)b1 * (1.0 + rel) / (1.0 - rel) + 1e-30;
        int result = q1;
        float bestv = b1;
        if ((double)b2 <= thr) {
          // pass 2: float64 re-evaluation of every candidate inside the margin
          double m64 = DBL_MAX, cur64 = -1.0;
          int q64 = -1;
          auto pass2 = [&](int q) {
            const float* cr = C + (int64_t)q * d;
            const float dq = group_sum<L>(part32<V>(x[p], cr, j, d, vec_c));
            if ((double)dq <= thr) {
              const double e = group_sum<L>(part64<V>(x[p], cr, j, d, vec_c));
              if (q == cur[p]) cur64 = e;
              if (e < m64 || (e == m64 && q < q64)) {
                m64 = e;
                q64 = q;
              }
            }
          };
          if (dense_i[p])
            for (int q = kb[p]; q < kb[p] + kc[p]; ++q) pass2(q);
          else
            for_each_cand<L, SM>(cv[p], valid[p], gmask, pass2);
          if (cur[p] >= 0 && cur64 >= 0.0 && cur64 == m64) {
            result = cur[p];
            bestv = (float)cur64;
          } else {
            result = q64;
            bestv = (float)m64;
          }
        }
        if (j == 0) {
          lab_out[ii[p]] = result;
          if (best_out) best_out[ii[p]] = bestv;
          if (act_out) act_out[ii[p]] = 1;
          if (cur[p] >= 0 && result != cur[p]) my_moved++;
        }
      }
    }
  }
  if (moved_acc || eval_acc) {
    if (my_moved) atomicAdd(&block_moved, my_moved);
    if (my_eval) atomicAdd(&block_eval, my_eval);
    __syncthreads();
    if (threadIdx.x == 0 && moved_acc && block_moved) atomicAdd(moved_acc, (unsigned long long)block_moved);
    if (threadIdx.x == 0 && eval_acc && block_eval) atomicAdd(eval_acc, (unsigned long long)block_eval);
  }
}

// Active-set sweeps.  A sample's flag has bit 0 when it had several
// candidates in the last sweep and bit 1 when its own or a neighbour's label
// changed since.  k_act_compact lists the positions whose flag is set (bit 1
// carried in the sign bit of the entry) and clears the flags it read, which
// makes that array the clean output of the next sweep.  A block takes CPB = 4 x 16 x 64 consecutive positions and
// reserves its share of the list with one atomic (blocks land in varying
// order; decisions do not depend on the order of the list).
__global__ __launch_bounds__(256) void k_act_compact(int64_t n, uint8_t* __restrict__ act, int32_t* __restrict__ list,
                                                     int32_t* __restrict__ count, int32_t* __restrict__ clear_other) {
  // a lane reads the flags of four consecutive positions as one word (the
  // flag arrays are padded to a multiple of four bytes)
  constexpr int RW = 4;  // rounds of 256 positions per wavefront
  __shared__ int32_t wtot[4], wbase[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // the other list's counter is free during this sweep: clear it for the next
  if (clear_other && blockIdx.x == 0 && threadIdx.x == 0) *clear_other = 0;
  const int64_t base = ((int64_t)blockIdx.x * 4 + w) * (RW * 256);
  const int64_t nw = (n + 3) / 4;
  uint32_t* act4 = reinterpret_cast<uint32_t*>(act);
  uint64_t m[RW][4], c[RW][4];
  int32_t tot = 0;
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const int64_t wi = base / 4 + r * 64 + lane;
    uint32_t f = 0;
    if (wi < nw) {
      f = act4[wi];
      if (f) act4[wi] = 0;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const bool in = 4 * wi + b < n;  // padding bytes past the last position never count
      const uint32_t fb = in ? (f >> (8 * b)) & 0xFFu : 0u;
      m[r][b] = __ballot(fb != 0);
      c[r][b] = __ballot((fb & 2u) != 0);
      tot += (int32_t)__popcll(m[r][b]);
    }
  }
  if (lane == 0) wtot[w] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int32_t all = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    int32_t at = all ? atomicAdd(count, all) : 0;
    for (int q = 0; q < 4; ++q) {
      wbase[q] = at;
      at += wtot[q];
    }
  }
  __syncthreads();
  int32_t at = wbase[w];
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if ((m[r][b] >> lane) & 1ull) {
        const int64_t p = base + 4 * (r * 64 + lane) + b;
        list[at + __popcll(m[r][b] & lanes_below())] =
            (int32_t)((uint32_t)p | (((c[r][b] >> lane) & 1ull) ? 0x80000000u : 0u));
      }
      at += (int32_t)__popcll(m[r][b]);
    }
}

// bits[r / 32] bit r % 32 = (flags[r] != 0), for r < K (the last word's
// bits past K are 0)
__global__ __launch_bounds__(256) void k_pack_flags(const int32_t* __restrict__ flags, int32_t K,
                                                    uint32_t* __restrict__ bits) {
  const int lane = threadIdx.x & 63;
  for (int64_t b = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63); b < K; b += (int64_t)gridDim.x * 256) {
    const int64_t r = b + lane;
    const uint64_t m = __ballot(r < K && flags[r] != 0);
    if (lane == 0) bits[b >> 5] = (uint32_t)m;
    if (lane == 32) bits[(b >> 5) + 1] = (uint32_t)(m >> 32);
  }
}

// The listed samples, GS per row group (grid-stride over the list), each
// through the same candidate collection, float32 pass and float64 pass as
// k_assign with one sample per group, so labels are the same bits.  The
// candidate loops of a group's samples advance together (the next centroid
// row of every sample is loaded while the current ones reduce), so a group
// keeps GS dependent load chains in flight (GS = 2 where a row group is a
// whole wavefront, d > 256: one sample per wavefront leaves its loads too
// serial; smaller groups keep GS = 1 and their higher occupancy).  Labels
// of unlisted samples are not written: the update keeps both label arrays
// equal outside the samples a sweep moves.  act_out as in k_assign.  A
// listed sample whose candidate set is unchanged (bit 1 clear) and none of
// whose candidate centroids changed in the last update (cbits, one bit per
// cluster; null: all changed) has all the inputs of its last decision, to
// stay, so it stays without a distance being evaluated.
template <int L, int V, int SM, int GS>
__global__ __launch_bounds__(256) void k_assign_list(
    const float* __restrict__ X, int d, int64_t ldx, const float* __restrict__ C, int k,
    const int* __restrict__ G, int kappa, const int* __restrict__ lab_in, int* __restrict__ lab_out,
    unsigned long long* __restrict__ moved_acc, unsigned long long* __restrict__ eval_acc,
    const int32_t* __restrict__ list, const int32_t* __restrict__ count, double rel, int vec_x, int vec_c,
    const int* __restrict__ job_of, const int* __restrict__ kbase, uint8_t* __restrict__ act_out,
    int64_t* __restrict__ n_listed, const uint32_t* __restrict__ cbits) {
  constexpr int GW = 64 / L;
  __shared__ unsigned int block_moved, block_eval;
  if (threadIdx.x == 0) {
    block_moved = 0;
    block_eval = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane / L, j = lane % L;
  const uint64_t gmask = group_mask<L>(g);
  const int cnt = *count;
  if (n_listed && blockIdx.x == 0 && threadIdx.x == 0) *n_listed = cnt;
  const int ngroups = gridDim.x * 4 * GW;
  unsigned int my_moved = 0, my_eval = 0;
  // wave-uniform trip count: groups of a wavefront stay in step
  for (int base = (blockIdx.x * 4 + w) * GW * GS; base < cnt; base += ngroups * GS) {
    bool live[GS], changed[GS], dn[GS], eval[GS];
    int64_t i[GS];
    int cur[GS], kb[GS], kc[GS];
    int cv[GS][SM];
    bool valid[GS][SM];
#pragma unroll
    for (int p = 0; p < GS; ++p) {
      const int li = base + p * GW + g;
      live[p] = li < cnt;  // group-uniform
      const uint32_t ent = live[p] ? (uint32_t)list[li] : 0u;
      changed[p] = (ent >> 31) != 0;
      i[p] = (int64_t)(ent & 0x7FFFFFFFu);
    }
#pragma unroll
    for (int p = 0; p < GS; ++p) {
      cur[p] = live[p] ? lab_in[i[p]] : -1;
      kb[p] = 0;
      kc[p] = k;
      dn[p] = false;
      if (job_of && live[p]) {
        const int q = job_of[i[p]];
        kb[p] = kbase[q];
        kc[p] = kbase[q + 1] - kb[p];
        dn[p] = kappa >= kc[p];
      }
    }
    int nb[GS][SM];
#pragma unroll
    for (int p = 0; p < GS; ++p)
#pragma unroll
      for (int s = 0; s < SM; ++s) {
        const int e = j + L * s;
        nb[p][s] = (live[p] && !dn[p] && e >= 1 && e <= kappa) ? G[i[p] * kappa + (e - 1)] : -1;
      }
#pragma unroll
    for (int p = 0; p < GS; ++p)
#pragma unroll
      for (int s = 0; s < SM; ++s) {
        const int e = j + L * s;
        valid[p][s] = live[p] && !dn[p] && e <= kappa;
        cv[p][s] = !valid[p][s] ? -1 : (e == 0 ? cur[p] : lab_in[nb[p][s]]);
      }
#pragma unroll
    for (int p = 0; p < GS; ++p) {
      bool other = false;
#pragma unroll
      for (int s = 0; s < SM; ++s) other = other || (valid[p][s] && cv[p][s] != cur[p]);
      const bool single = live[p] && !dn[p] && cur[p] >= 0 && (__ballot(other) & gmask) == 0;
      bool cand_dirty = true;
      if (!changed[p] && !dn[p] && cbits) {
        bool any = false;
#pragma unroll
        for (int s = 0; s < SM; ++s) any = any || (valid[p][s] && bit_of(cbits, cv[p][s]));
        cand_dirty = (__ballot(any) & gmask) != 0;
      }
      eval[p] = false;
      if (live[p] && single) {  // group-uniform
        if (j == 0) {
          lab_out[i[p]] = cur[p];
          if (act_out) act_out[i[p]] = 0;
        }
      } else if (live[p] && !cand_dirty) {  // same inputs as its last decision: stays
        if (j == 0) {
          lab_out[i[p]] = cur[p];
          if (act_out) act_out[i[p]] = 1;
        }
      } else if (live[p]) {
        eval[p] = true;
      }
    }
    float x[GS][V];
#pragma unroll
    for (int p = 0; p < GS; ++p)
      if (eval[p]) load_row<V>(x[p], X + i[p] * ldx, j, d, vec_x);
    // pass 1: float32 distances, best and second best of every sample
    float b1[GS], b2[GS];
    int q1[GS];
#pragma unroll
    for (int p = 0; p < GS; ++p) {
      b1[p] = b2[p] = FLT_MAX;
      q1[p] = -1;
    }
    auto pass1 = [&](int p, int q, float dq) {
      if (dq < b1[p] || (dq == b1[p] && q < q1[p])) {
        if (q1[p] >= 0) b2[p] = fminf(b2[p], b1[p]);
        b1[p] = dq;
        q1[p] = q;
      } else {
        b2[p] = fminf(b2[p], dq);
      }
    };
    {
      bool sparse[GS];
#pragma unroll
      for (int p = 0; p < GS; ++p) {
        sparse[p] = eval[p] && !dn[p];
        if (eval[p] && dn[p])
          for (int q = kb[p]; q < kb[p] + kc[p]; ++q)
            pass1(p, q, group_sum<L>(part32<V>(x[p], C + (int64_t)q * d, j, d, vec_c)));
      }
      for_each_cand_rows<L, V, SM, GS>(cv, valid, sparse, gmask, C, d, j, vec_c,
                                       [&](int p, int q, const float (&c)[V]) {
                                         pass1(p, q, group_sum<L>(dist32<V>(x[p], c)));
                                       });
    }
#pragma unroll
    for (int p = 0; p < GS; ++p) {
      if (!eval[p]) continue;  // group-uniform
      const double thr = (double)b1[p] * (1.0 + rel) / (1.0 - rel) + 1e-30;
      int result = q1[p];
      if ((double)b2[p] <= thr) {
        double m64 = DBL_MAX, cur64 = -1.0;
        int q64 = -1;
        auto pass2 = [&](int q) {
          const float* cr = C + (int64_t)q * d;
          const float dq = group_sum<L>(part32<V>(x[p], cr, j, d, vec_c));
          if ((double)dq <= thr) {
            const double e = group_sum<L>(part64<V>(x[p], cr, j, d, vec_c));
            if (q == cur[p]) cur64 = e;
            if (e < m64 || (e == m64 && q < q64)) {
              m64 = e;
              q64 = q;
            }
          }
        };
        if (dn[p])
          for (int q = kb[p]; q < kb[p] + kc[p]; ++q) pass2(q);
        else
          for_each_cand<L, SM>(cv[p], valid[p], gmask, pass2);
        result = (cur[p] >= 0 && cur64 >= 0.0 && cur64 == m64) ? cur[p] : q64;
      }
      if (j == 0) {
        lab_out[i[p]] = result;
        if (act_out) act_out[i[p]] = 1;
        my_eval++;
        if (cur[p] >= 0 && result != cur[p]) my_moved++;
      }
    }
  }
  if (moved_acc || eval_acc) {
    if (my_moved) atomicAdd(&block_moved, my_moved);
    if (my_eval) atomicAdd(&block_eval, my_eval);
    __syncthreads();
    if (threadIdx.x == 0 && moved_acc && block_moved) atomicAdd(moved_acc, (unsigned long long)block_moved);
    if (threadIdx.x == 0 && eval_acc && block_eval) atomicAdd(eval_acc, (unsigned long long)block_eval);
  }
}

// Launch shapes (GS samples per row group and pass, pb samples per block).
// Every shape gives the same results: a sample's arithmetic depends on (L, V)
// only.  The default, two samples per group and 64 per block, was measured
// best at 1M x 128; the autotuner below times the candidates on the first
// large call of each (group shape, size bin) and keeps the fastest.
struct AssignCfg {
  int gs = 2, pb = 64, lazy = 0;  // lazy: sample rows loaded only when a distance is needed
};
static const AssignCfg kAssignCandidates[] = {{1, 64, 0}, {2, 64, 0}, {4, 64, 0}, {1, 128, 0}, {2, 128, 0},
                                              {4, 128, 0}, {1, 64, 1},  {2, 64, 1},  {1, 128, 1}, {2, 128, 1}};

template <int L, int V, int SM>
static void launch_assign(knnkm_ctx* ctx, AssignCfg cfg, const float* X, int64_t n, int32_t d, int64_t ldx,
                          const float* C, int32_t k, const int32_t* G_ids, int32_t kappa,
                          const int32_t* labels_in, int32_t* labels_out, float* best_d2,
                          unsigned long long* acc, unsigned long long* eacc, const int32_t* order, bool dense,
                          double rel, bool vec_x, bool vec_c, const int32_t* job_of, const int32_t* kbase,
                          const uint8_t* act_in, uint8_t* act_out) {
  const int nchunks = (int)((n + cfg.pb - 1) / cfg.pb);
  const int grid = ((nchunks + 7) / 8) * 8;
#define LG(GG, LZ)                                                                                          \
  k_assign<L, V, GG, SM, LZ><<<grid, 256, 0, ctx->stream>>>(X, (int)n, d, ldx, C, k, G_ids, kappa, labels_in,  \
                                                            labels_out, best_d2, acc, eacc, order, dense ? 1 : 0, \
                                                            nchunks, cfg.pb, rel, vec_x ? 1 : 0, vec_c ? 1 : 0,   \
                                                            job_of, kbase, act_in, act_out)
  if (cfg.lazy) {
    if (cfg.gs == 1)
      LG(1, 1);
    else
      LG(2, 1);
  } else if (cfg.gs == 1) {
    LG(1, 0);
  } else if (cfg.gs == 4) {
    LG(4, 0);
  } else {
    LG(2, 0);
  }
#undef LG
}

template <int L, int V>
static void launch_assign_sm(knnkm_ctx* ctx, int S, AssignCfg cfg, const float* X, int64_t n, int32_t d,
                             int64_t ldx, const float* C, int32_t k, const int32_t* G_ids, int32_t kappa,
                             const int32_t* labels_in, int32_t* labels_out, float* best_d2,
                             unsigned long long* acc, unsigned long long* eacc, const int32_t* order, bool dense,
                             double rel, bool vec_x, bool vec_c, const int32_t* job_of, const int32_t* kbase,
                             const uint8_t* act_in, uint8_t* act_out) {
#define LS(SS)                                                                                            \
  launch_assign<L, V, SS>(ctx, cfg, X, n, d, ldx, C, k, G_ids, kappa, labels_in, labels_out, best_d2, acc, \
                          eacc, order, dense, rel, vec_x, vec_c, job_of, kbase, act_in, act_out)
  if (S <= 1)
    LS(1);
  else if (S <= 2)
    LS(2);
  else if (S <= 4)
    LS(4);
  else
    LS(8);
#undef LS
}

// Process-wide table of tuned shapes: key (device, L, V, slots, dense,
// size bin) -> shape and its time.
struct AssignTuned {
  AssignCfg cfg;
  float us = 0.f;
};
static std::mutex g_tune_mu;
static std::map<uint64_t, AssignTuned> g_tuned;

static const char* const kUseName[4] = {"call", "build", "fit1", "fit"};

static uint64_t tune_key(int dev, int L, int V, int S, bool dense, int use, int64_t n) {
  int bin = 0;
  while ((int64_t)1 << (bin + 1) <= n) ++bin;
  return ((uint64_t)(dev & 0xFF) << 40) | ((uint64_t)L << 32) | ((uint64_t)V << 24) | ((uint64_t)S << 16) |
         ((uint64_t)(use & 3) << 9) | ((uint64_t)(dense ? 1 : 0) << 8) | (uint64_t)bin;
}

extern "C" knnkm_status knnkm_autotune_table(char* buf, int64_t len, int64_t* needed) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  std::string out;
  for (auto& kv : g_tuned) {
    char line[160];
    const uint64_t k = kv.first;
    snprintf(line, sizeof(line),
             "knn_assign device=%d L=%d V=%d slots=%d dense=%d n_bin=2^%d use=%s gs=%d pb=%d lazy=%d us=%.1f\n",
             (int)((k >> 40) & 0xFF), (int)((k >> 32) & 0xFF), (int)((k >> 24) & 0xFF), (int)((k >> 16) & 0xFF),
             (int)((k >> 8) & 0x1), (int)(k & 0xFF), kUseName[(k >> 9) & 0x3], kv.second.cfg.gs, kv.second.cfg.pb,
             kv.second.cfg.lazy, kv.second.us);
    out += line;
  }
  if (buf && len > 0) {
    const size_t m = std::min<size_t>(out.size(), (size_t)len - 1);
    std::memcpy(buf, out.data(), m);
    buf[m] = 0;
  }
  if (needed) *needed = (int64_t)out.size() + 1;
  return KNNKM_OK;
}

extern "C" knnkm_status knnkm_autotune(knnkm_ctx* ctx, int32_t on) {
  if (!ctx) return KNNKM_EINVAL;
  ctx->autotune = on != 0;
  return KNNKM_OK;
}

extern "C" knnkm_status knnkm_enable_partial_distances(knnkm_ctx* ctx, int32_t on) {
  if (!ctx) return KNNKM_EINVAL;
  if (on < 0 || on > 3) return knnkm_fail(ctx, KNNKM_EINVAL, "partial distances: %d is not 0, 1, 2 or 3", on);
  ctx->wide_pd = on != 0;
  ctx->pd_shadow = on == 1 ? 2 : (on == 3 ? 1 : 0);
  return KNNKM_OK;
}

extern "C" knnkm_status knnkm_set_assign_shape(knnkm_ctx* ctx, int32_t gs, int32_t pb, int32_t lazy) {
  if (!ctx) return KNNKM_EINVAL;
  const bool ok = gs == 0 || ((pb == 64 || pb == 128) && ((lazy == 0 && (gs == 1 || gs == 2 || gs == 4)) ||
                                                          (lazy == 1 && (gs == 1 || gs == 2))));
  if (!ok)
    return knnkm_fail(ctx, KNNKM_EINVAL, "set_assign_shape: gs=%d pb=%d lazy=%d is not a launch shape", gs, pb,
                      lazy);
  ctx->assign_gs = gs;
  ctx->assign_pb = pb;
  ctx->assign_lazy = lazy;
  return KNNKM_OK;
}

// The centroid shadow of the context's kind (none: kind 0) for K rows of d
// dimensions, in the workspace under names starting with `tag`.
knnkm_status ks_shadow_alloc(knnkm_ctx* ctx, const char* tag, int32_t K, int32_t d, CShadow* sw) {
  *sw = CShadow{};
  if (ctx->pd_shadow == 0) return KNNKM_OK;
  const size_t per = ctx->pd_shadow == 2 ? 1 : 2;  // bytes per element
  char name[40];
  snprintf(name, sizeof(name), "%s_cshadow", tag);
  void* rows = knnkm_ws(ctx, name, per * (size_t)K * d);
  snprintf(name, sizeof(name), "%s_ceps", tag);
  float* eps = (float*)knnkm_ws(ctx, name, sizeof(float) * (size_t)K);
  float* scale = nullptr;
  if (ctx->pd_shadow == 2) {
    snprintf(name, sizeof(name), "%s_cscale", tag);
    scale = (float*)knnkm_ws(ctx, name, sizeof(float) * (size_t)K);
  }
  if (!rows || !eps || (ctx->pd_shadow == 2 && !scale)) return KNNKM_ENOMEM;
  sw->rows = rows;
  sw->eps = eps;
  sw->scale = scale;
  sw->kind = ctx->pd_shadow;
  return KNNKM_OK;
}

knnkm_status ks_act_compact(knnkm_ctx* ctx, int64_t n, uint8_t* act, int32_t* list, int32_t* count) {
  KNNKM_TRY(ks_fill_i32(ctx, count, 1, 0));
  k_act_compact<<<(unsigned)((n + 4095) / 4096), 256, 0, ctx->stream>>>(n, act, list, count, nullptr);
  return knnkm_check(ctx, "active list");
}

knnkm_status ks_assign(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                       const float* C, int32_t k, const int32_t* G_ids, int32_t kappa,
                       const int32_t* labels_in, int32_t* labels_out, float* best_d2,
                       int64_t* n_moved, const int32_t* order, bool dense, const int32_t* job_of,
                       const int32_t* kbase, int use, int64_t* n_eval, const uint8_t* act_in, uint8_t* act_out,
                       int64_t* n_active, int32_t* list_count, int32_t* list_count_other, bool zero_moved,
                       const int32_t* cdirty, float* bnd_u, float* bnd_lb, const float* cdelta, CShadow sw,
                       const int32_t* nlab) {
  if (n_moved && zero_moved) KNNKM_TRY(ks_fill_i64(ctx, n_moved, 1, 0));
  if (n_eval) KNNKM_TRY(ks_fill_i64(ctx, n_eval, 1, 0));
  if (n_active && !(act_in && !best_d2 && !order && !dense)) KNNKM_TRY(ks_fill_i64(ctx, n_active, 1, n));
  if (n == 0) return KNNKM_OK;
  const bool all_dense = dense;
  int L, V;
  pick_group(d, all_dense ? 1 : (kappa + 1 + MAX_SLOTS - 1) / MAX_SLOTS, &L, &V);
  const int S = all_dense ? 1 : (kappa + 1 + L - 1) / L;
  // float32 evaluation: V products and sums per lane, log2(L) reduction
  // levels, one rounding of each difference; twice the worst-case bound.
  int lv = 0;
  while ((1 << lv) < L) ++lv;
  const double rel = (double)(V + lv + 3) * 0x1p-23;
  const bool vec_x = (d % 4 == 0) && (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
  const bool vec_c = (d % 4 == 0) && ((uintptr_t)C % 16 == 0);
  unsigned long long* acc = (unsigned long long*)n_moved;
  unsigned long long* eacc = (unsigned long long*)n_eval;
#define LA(LL, VV)                                                                                         \
  launch_assign_sm<LL, VV>(ctx, S, cfg, X, n, d, ldx, C, k, G_ids, kappa, labels_in, labels_out, best_d2, acc, \
                           eacc, order, dense, rel, vec_x, vec_c, job_of, kbase, act_in, act_out)
  // wide rows: one wavefront per sample with early-abandoned partial
  // distances (same decisions; best distances come from the kernels below)
  const bool wide = ctx->wide_pd && ks_assign_pd_ok(d, kappa) && !all_dense && labels_in && !best_d2;
  if (act_in && !best_d2 && !order && !all_dense) {
    // active-set sweep: list the flagged samples, then assign them
    KNNKM_WS(ctx, list, int32_t, "as_act_list", n);
    int32_t* cnt = list_count;
    if (!cnt) {
      cnt = (int32_t*)knnkm_ws(ctx, "as_act_count", sizeof(int32_t));
      if (!cnt) return KNNKM_ENOMEM;
      KNNKM_TRY(ks_fill_i32(ctx, cnt, 1, 0));
    }
    k_act_compact<<<(unsigned)((n + 4095) / 4096), 256, 0, ctx->stream>>>(n, const_cast<uint8_t*>(act_in), list, cnt,
                                                                          list_count_other);
    // the changed-centroid flags as one bit per cluster: the listed samples
    // look them up for every candidate, and a bit array small enough to stay
    // in the caches turns those scattered reads into cache hits
    uint32_t* cbits = nullptr;
    if (cdirty) {
      cbits = (uint32_t*)knnkm_ws(ctx, "as_cbits", sizeof(uint32_t) * (((size_t)k + 63) / 64) * 2);
      if (!cbits) return KNNKM_ENOMEM;
      k_pack_flags<<<grid_for(k, 256, 65535), 256, 0, ctx->stream>>>(cdirty, k, cbits);
    }
    if (wide)
      return ks_assign_pd(ctx, X, n, d, ldx, C, k, G_ids, kappa, labels_in, labels_out, acc, eacc, nullptr, job_of,
                          kbase, nullptr, act_out, list, cnt, n_active, cbits, 0, bnd_u, bnd_lb, cdelta, sw, nlab);
    const unsigned grid = (unsigned)std::max(1, ctx->num_cus * 8);
#define LP(LL, VV, SS)                                                                                        \
  k_assign_list<LL, VV, SS, ((LL) >= 64 ? 2 : 1)><<<grid, 256, 0, ctx->stream>>>(X, d, ldx, C, k, G_ids, kappa, labels_in, labels_out, \
                                                           acc, eacc, list, cnt, rel, vec_x ? 1 : 0,            \
                                                           vec_c ? 1 : 0, job_of, kbase, act_out, n_active,    \
                                                           cbits)
#define LPS(LL, VV)     \
  if (S <= 1)           \
    LP(LL, VV, 1);      \
  else if (S <= 2)      \
    LP(LL, VV, 2);      \
  else if (S <= 4)      \
    LP(LL, VV, 4);      \
  else                  \
    LP(LL, VV, 8);
    if (V == 4) {
      switch (L) {
        case 4: LPS(4, 4) break;
        case 8: LPS(8, 4) break;
        case 16: LPS(16, 4) break;
        case 32: LPS(32, 4) break;
        default: LPS(64, 4) break;
      }
    } else {
      switch (L) {
        case 4: LPS(4, 8) break;
        case 8: LPS(8, 8) break;
        case 16: LPS(16, 8) break;
        case 32: LPS(32, 8) break;
        default: LPS(64, 8) break;
      }
    }
#undef LPS
#undef LP
    return knnkm_check(ctx, "knn_assign (active set)");
  }
  auto launch = [&](AssignCfg cfg) {
  if (V == 4) {
    switch (L) {
      case 4: LA(4, 4); break;
      case 8: LA(8, 4); break;
      case 16: LA(16, 4); break;
      case 32: LA(32, 4); break;
      default: LA(64, 4); break;
    }
  } else {
    switch (L) {
      case 4: LA(4, 8); break;
      case 8: LA(8, 8); break;
      case 16: LA(16, 8); break;
      case 32: LA(32, 8); break;
      default: LA(64, 8); break;
    }
  }
  };
#undef LA
  if (wide) {
    // a caller's assignment reads the context's kind of shadow too, built
    // here from its centroids
    if (use == KS_USE_CALL && sw.kind == 0 && ctx->pd_shadow != 0) {
      KNNKM_TRY(ks_shadow_alloc(ctx, "as", k, d, &sw));
      KNNKM_TRY(ks_c_shadow(ctx, C, k, d, nullptr, sw));
    }
    return ks_assign_pd(ctx, X, n, d, ldx, C, k, G_ids, kappa, labels_in, labels_out, acc, eacc, order, job_of,
                        kbase, act_in, act_out, nullptr, nullptr, nullptr, nullptr, 64, bnd_u, bnd_lb, nullptr, sw);
  }
  // shape: tuned entry, else (large call, tuning allowed, not inside a
  // graph capture) time every candidate once, else the default
  const int Sb = S <= 1 ? 1 : (S <= 2 ? 2 : (S <= 4 ? 4 : 8));
  const uint64_t key = tune_key(ctx->device, L, V, Sb, all_dense, use, n);
  AssignCfg cfg;
  bool found = false;
  if (ctx->assign_gs > 0) {
    cfg.gs = ctx->assign_gs;
    cfg.pb = ctx->assign_pb;
    cfg.lazy = ctx->assign_lazy;
    found = true;
  } else {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      cfg = it->second.cfg;
      found = true;
    }
  }
  if (!found && ctx->autotune && !ctx->capturing && n >= (1 << 16)) {
    for (int q = 0; q < 2; ++q)
      if (!ctx->tune_ev[q] && hipEventCreate(&ctx->tune_ev[q]) != hipSuccess) {
        (void)hipGetLastError();
        ctx->tune_ev[q] = nullptr;
      }
    hipEvent_t e0 = ctx->tune_ev[0], e1 = ctx->tune_ev[1];
    if (e0 && e1) {
      float best = 1e30f;
      for (const AssignCfg& c : kAssignCandidates) {
        if (n_moved) KNNKM_TRY(ks_fill_i64(ctx, n_moved, 1, 0));
        if (n_eval) KNNKM_TRY(ks_fill_i64(ctx, n_eval, 1, 0));
        KNNKM_HIP(ctx, hipEventRecord(e0, ctx->stream));
        launch(c);
        KNNKM_HIP(ctx, hipEventRecord(e1, ctx->stream));
        KNNKM_TRY(knnkm_check(ctx, "knn_assign tuning"));
        KNNKM_HIP(ctx, hipEventSynchronize(e1));
        float ms = 0.f;
        KNNKM_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          cfg = c;
        }
      }
      std::lock_guard<std::mutex> g(g_tune_mu);
      g_tuned[key] = AssignTuned{cfg, best * 1000.f};
      if (n_moved) KNNKM_TRY(ks_fill_i64(ctx, n_moved, 1, 0));
      if (n_eval) KNNKM_TRY(ks_fill_i64(ctx, n_eval, 1, 0));
    }
  }
  launch(cfg);
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
