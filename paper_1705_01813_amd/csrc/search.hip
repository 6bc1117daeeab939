// Best-first (beam) search over the KNN graph for approximate nearest
// neighbours of query rows (Sec. 4.3 notes the graph serves this search; no
// algorithm is given there, so the usual one is used).
//
// One wavefront per query.  The search keeps one sorted list of at most ef
// entries (d2, id, expanded), seeded with n_entry entry points (Floyd's
// sampling keyed by the seed and the query index); it repeatedly expands the
// first unexpanded entry -- the graph neighbours of that point not seen
// before get their distances and are merged into the list, which keeps its
// ef smallest -- and stops when every entry is expanded or max_visits points
// have been looked at.  This is the classic two-heap beam search (every
// candidate outside the list is farther than the list's farthest, so the
// classic loop stops or skips there), in the order it expands.
//
// Points are compared by (d2, id), d2 the squared distance summed over the
// dimensions in order in float64 with one rounding per operation, rounded
// once to float32 (the keys of the graph) -- each distance by one lane.
// Points seen are kept in an open-addressing hash filled to at most about
// half by the visit limit: up to 1,920 visits 4,096 slots in LDS; above,
// 16,384 slots in global memory, one table per resident wavefront of a
// persistent grid (cleared per query), so that the LDS holds only the query
// and the list and many queries run at once.
#include <cfloat>
#include <climits>

#include "common.h"

namespace {

constexpr uint64_t SR_PURPOSE = 5;  // random-number stream of the entry points
constexpr int SR_SMALL_VISITS = 1920;  // visit limit of the 4,096-slot hash
constexpr int SR_GH_BLOCKS_PER_CU = 8;  // workgroups of four queries per compute unit (global tables)

template <int HB>  // log2 of the hash slots in LDS (0: the hash is elsewhere)
struct SRWave {
  float q[KNNKM_MAX_D];
  int32_t hash[HB ? 1 << HB : 1];
  float lk[KNNKM_SEARCH_MAX_EF];
  int32_t li[KNNKM_SEARCH_MAX_EF];
  int32_t lx[KNNKM_SEARCH_MAX_EF];
  int32_t ent[KNNKM_SEARCH_MAX_ENTRY];
};

__device__ inline bool sr_lt(float ka, int ia, float kb, int ib) { return ka < kb || (ka == kb && ia < ib); }

__device__ inline void sr_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Inserts id; true if it was not there yet.
template <int HB>
__device__ inline bool sr_insert(int32_t* hash, int32_t id) {
  uint32_t h = ((uint32_t)id * 2654435761u) >> (32 - HB);
  while (true) {
    const int32_t prev = atomicCAS(&hash[h], -1, id);
    if (prev == -1) return true;
    if (prev == id) return false;
    h = (h + 1) & ((1u << HB) - 1);
  }
}

// float32 of the float64 squared distance, dimensions in order.
__device__ inline float sr_key(const float* __restrict__ q, const float* __restrict__ x, int d) {
#pragma clang fp contract(off)
  double acc = 0.0;
  for (int j = 0; j < d; ++j) {
    const double df = (double)q[j] - (double)x[j];
    acc = acc + df * df;
  }
  return (float)acc;
}

// Merges the candidates held by the lanes with `in` set (key ck, id ci) into
// the sorted list (slots l and l + 64 held by lane l: k0/i0/x0, k1/i1/x1;
// cnt entries), keeping the ef smallest; new entries are unexpanded.
template <class W>
__device__ inline void sr_merge(W& sh, bool in, float ck, int ci, int ef, int& cnt, float& k0, int& i0,
                                int& x0, float& k1, int& i1, int& x1) {
  const int lane = threadIdx.x & 63;
  uint64_t M = __ballot(in);
  if (!M) return;
  const int E = __popcll(M);
  // position of a candidate: list entries before it (binary search in LDS)
  // plus candidates before it
  int pos = 0;
  if (in) {
    int lo = 0, hi = cnt;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sr_lt(sh.lk[mid], sh.li[mid], ck, ci)) lo = mid + 1; else hi = mid;
    }
    pos = lo;
  }
  int add0 = 0, add1 = 0;
  for (uint64_t R = M; R; R &= R - 1) {
    const int b = (int)__builtin_ctzll(R);
    const float qk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ck), b));
    const int qi = __builtin_amdgcn_readlane(ci, b);
    pos += (in && sr_lt(qk, qi, ck, ci)) ? 1 : 0;
    add0 += sr_lt(qk, qi, k0, i0) ? 1 : 0;
    add1 += sr_lt(qk, qi, k1, i1) ? 1 : 0;
  }
  sr_sync();  // every lane has read the old list
  if (lane < cnt && lane + add0 < ef) {
    sh.lk[lane + add0] = k0;
    sh.li[lane + add0] = i0;
    sh.lx[lane + add0] = x0;
  }
  if (lane + 64 < cnt && lane + 64 + add1 < ef) {
    sh.lk[lane + 64 + add1] = k1;
    sh.li[lane + 64 + add1] = i1;
    sh.lx[lane + 64 + add1] = x1;
  }
  if (in && pos < ef) {
    sh.lk[pos] = ck;
    sh.li[pos] = ci;
    sh.lx[pos] = 0;
  }
  sr_sync();
  cnt = min(ef, cnt + E);
  k0 = lane < cnt ? sh.lk[lane] : FLT_MAX;
  i0 = lane < cnt ? sh.li[lane] : INT_MAX;
  x0 = lane < cnt ? sh.lx[lane] : 1;
  k1 = lane + 64 < cnt ? sh.lk[lane + 64] : FLT_MAX;
  i1 = lane + 64 < cnt ? sh.li[lane + 64] : INT_MAX;
  x1 = lane + 64 < cnt ? sh.lx[lane + 64] : 1;
}

// HB: log2 of the hash slots; WPB: queries (wavefronts) per workgroup; GH:
// the hash in global memory (vis: 2^HB slots per wavefront of the grid),
// else in LDS.
template <int HB, int WPB, bool GH>
__global__ __launch_bounds__(64 * WPB) void k_graph_search(const float* __restrict__ X, int64_t n, int d,
                                                           int64_t ldx, const int32_t* __restrict__ G, int kappa,
                                                           const float* __restrict__ Q, int64_t m, int64_t ldq,
                                                           int ef, int top_k, int max_visits, int n_entry,
                                                           uint64_t seed, int32_t* __restrict__ out_ids,
                                                           float* __restrict__ out_d2, int32_t* __restrict__ vis) {
  __shared__ SRWave<GH ? 0 : HB> shw[WPB];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  SRWave<GH ? 0 : HB>& sh = shw[w];
  int32_t* hash = GH ? vis + (((int64_t)blockIdx.x * WPB + w) << HB) : sh.hash;
  for (int64_t qi = (int64_t)blockIdx.x * WPB + w; qi < m; qi += (int64_t)gridDim.x * WPB) {
    for (int j = lane; j < d; j += 64) sh.q[j] = Q[qi * ldq + j];
    if constexpr (GH) {
      // 16-byte stores, every one complete before the first insert (the
      // table is this wavefront's alone: a workgroup-scope release suffices)
      for (int j = lane * 4; j < (1 << HB); j += 256) *reinterpret_cast<int4*>(hash + j) = make_int4(-1, -1, -1, -1);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    } else {
      for (int j = lane; j < (1 << HB); j += 64) hash[j] = -1;
    }
    // entry points (Floyd's sampling, one draw per step)
    const int ne = (int)min<int64_t>(n_entry, n);
    if (lane == 0) {
      const uint64_t key = sm_key(seed, sm_stream(SR_PURPOSE, 0, (uint64_t)qi));
      const int64_t base = n - ne;
      for (int c = 0; c < ne; ++c) {
        const int64_t j = base + c;
        const int64_t t = (int64_t)sm_below(sm_draw(key, (uint64_t)c), (uint32_t)(j + 1));
        bool seen = false;
        for (int e = 0; e < c; ++e) seen = seen || sh.ent[e] == t;
        sh.ent[c] = (int32_t)(seen ? j : t);
      }
    }
    sr_sync();
    int cnt = 0;
    float k0 = FLT_MAX, k1 = FLT_MAX;
    int i0 = INT_MAX, i1 = INT_MAX, x0 = 1, x1 = 1;
    {
      const bool in = lane < ne;
      int id = 0;
      float key = FLT_MAX;
      if (in) {
        id = sh.ent[lane];
        sr_insert<HB>(hash, id);
        key = sr_key(sh.q, X + (int64_t)id * ldx, d);
      }
      sr_merge(sh, in, key, id, ef, cnt, k0, i0, x0, k1, i1, x1);
    }
    int visited = ne;
    while (true) {
      const uint64_t M0 = __ballot(lane < cnt && !x0), M1 = __ballot(lane + 64 < cnt && !x1);
      if ((!M0 && !M1) || visited >= max_visits) break;
      const int t = M0 ? (int)__builtin_ctzll(M0) : 64 + (int)__builtin_ctzll(M1);
      const int c = t < 64 ? __builtin_amdgcn_readlane(i0, t) : __builtin_amdgcn_readlane(i1, t - 64);
      if (lane == (t & 63)) {
        if (t < 64) x0 = 1; else x1 = 1;
      }
      // the list in LDS for the merges' binary searches
      if (lane < cnt) {
        sh.lk[lane] = k0;
        sh.li[lane] = i0;
        sh.lx[lane] = x0;
      }
      if (lane + 64 < cnt) {
        sh.lk[lane + 64] = k1;
        sh.li[lane + 64] = i1;
        sh.lx[lane + 64] = x1;
      }
      sr_sync();
      for (int e0 = 0; e0 < kappa; e0 += 64) {
        const int e = e0 + lane;
        const int b = e < kappa ? G[(int64_t)c * kappa + e] : -1;
        const bool fresh = b >= 0 && b < n && sr_insert<HB>(hash, b);
        visited += __popcll(__ballot(fresh));
        float key = FLT_MAX;
        if (fresh) key = sr_key(sh.q, X + (int64_t)b * ldx, d);
        sr_merge(sh, fresh, key, b, ef, cnt, k0, i0, x0, k1, i1, x1);
      }
    }
    const int64_t o = qi * top_k;
    if (lane < top_k) {
      out_ids[o + lane] = lane < cnt ? i0 : -1;
      out_d2[o + lane] = lane < cnt ? k0 : INFINITY;
    }
    if (lane + 64 < top_k) {
      out_ids[o + lane + 64] = lane + 64 < cnt ? i1 : -1;
      out_d2[o + lane + 64] = lane + 64 < cnt ? k1 : INFINITY;
    }
    sr_sync();  // the next query overwrites the wave's LDS
  }
}

}  // namespace

extern "C" knnkm_status knn_graph_search(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                         const int32_t* G_ids, int32_t kappa, const float* Q, int64_t m,
                                         int64_t ldq, int32_t ef, int32_t top_k, int32_t max_visits,
                                         int32_t n_entry, uint64_t seed, int32_t* out_ids, float* out_d2) {
  if (!ctx) return KNNKM_EINVAL;
  if (ctx->sticky) return KNNKM_EDEVICE;
  if (!X || !G_ids || !Q || !out_ids || !out_d2)
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_graph_search: null pointer");
  if (n < 1 || n > INT32_MAX || d < 1 || ldx < d || ldq < d || m < 0)
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_graph_search: need n >= 1, d >= 1, ldx >= d, ldq >= d, m >= 0");
  if (d > KNNKM_MAX_D) return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "knn_graph_search: d=%d > %d", d, KNNKM_MAX_D);
  if (kappa < 1 || kappa > KNNKM_MAX_KAPPA)
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_graph_search: kappa=%d not in [1, %d]", kappa, KNNKM_MAX_KAPPA);
  if (ef < 1 || ef > KNNKM_SEARCH_MAX_EF || top_k < 1 || top_k > ef)
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_graph_search: need 1 <= top_k <= ef <= %d", KNNKM_SEARCH_MAX_EF);
  if (max_visits < 1 || max_visits > KNNKM_SEARCH_MAX_VISITS)
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_graph_search: max_visits not in [1, %d]", KNNKM_SEARCH_MAX_VISITS);
  if (n_entry < 1 || n_entry > KNNKM_SEARCH_MAX_ENTRY)
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_graph_search: n_entry not in [1, %d]", KNNKM_SEARCH_MAX_ENTRY);
  if (ctx->dry || m == 0) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  if (max_visits <= SR_SMALL_VISITS) {
    k_graph_search<12, 4, false><<<grid_for(m, 4, 65536), 256, 0, ctx->stream>>>(
        X, n, d, ldx, G_ids, kappa, Q, m, ldq, ef, top_k, max_visits, n_entry, seed, out_ids, out_d2, nullptr);
  } else {
    // a persistent grid of SR_GH_BLOCKS_PER_CU workgroups per compute unit,
    // one 64 KB table per wavefront
    const int blocks = grid_for(m, 4, std::max(1, ctx->num_cus) * SR_GH_BLOCKS_PER_CU);
    int32_t* vis = (int32_t*)knnkm_ws(ctx, "search_visited", sizeof(int32_t) * ((size_t)blocks * 4 << 14));
    if (!vis) return KNNKM_ENOMEM;
    k_graph_search<14, 4, true><<<blocks, 256, 0, ctx->stream>>>(
        X, n, d, ldx, G_ids, kappa, Q, m, ldq, ef, top_k, max_visits, n_entry, seed, out_ids, out_d2, vis);
  }
  return knnkm_check(ctx, "knn_graph_search");
}
