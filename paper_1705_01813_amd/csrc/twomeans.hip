// Two-means tree (Alg. 1) as a level-synchronous balanced bisection.
//
// Every split is exactly ceil(s/2) / floor(s/2), so the shape of the tree —
// the offset and size of every node at every depth and which nodes split at
// the last, partial depth — depends on (n, k) only.  The host computes it
// once (TMPlan) and the device moves sample ids between node segments:
// perm[] holds the ids of each node contiguously, ascending inside a node.
//
// Per depth:
//   seed      two distinct members per splitting node (counter-based draws)
//   accum x I Lloyd 2-means steps: side of each member from
//             delta = ||x-c_u||^2 - ||x-c_v||^2 = sum_j (c_v-c_u)_j (2x - c_u - c_v)_j
//             in float64 (u when delta <= 0), float64 sums per side per tile
//   final     per node, tile partials added in tile order; centroid = float32
//             of the float64 mean; an empty side keeps its centroid
//   delta     the same delta with the final centroids, stored as an ordered key
//   split     the first ceil(s/2) members in (delta, id) order go left:
//             nodes of <= TM_SMALL members sort (delta, id) in LDS; larger nodes
//             find the threshold key by an 8-digit radix select and partition
//             tile by tile, members equal to it going left in position
//             (= id) order up to the remaining rank
// A node to split of at most the finish limit (1,024 members by default) is
// the root of a subtree that one block finishes with the ids in LDS
// (k_tm_finish): the same steps, arithmetic and order for every later depth.
// Leaves are numbered left to right.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "rowgroup.h"

#define TM_TILE 1024    // positions per tile of the per-member passes
#define TM_SMALL 2048   // nodes up to this size split inside one block
#define TM_CHUNK 16     // tiles per chunk of the two-stage node reduction
#define TM_SEL_PASSES 8  // 8-bit digits of the 64-bit delta key
#define TM_FINISH_DEFAULT TM_TILE  // largest subtree root that one block finishes

struct TMLevel {
  int depth;
  int nsplit;            // split nodes at this depth
  int split_base;        // into plan.split_* arrays
  int ntiles, tile_base; // tiles of split nodes
  int nbig, big_base;    // split nodes with size > TM_SMALL
  int nbigtiles, bigtile_base;
  int nsmall, small_base;  // split nodes with size <= TM_SMALL
  int ncopy, copy_base;    // unsplit nodes (copied unchanged)
  int nchunks, chunk_base; // groups of up to TM_CHUNK tiles of one node
  int max_node_tiles;      // largest number of tiles of one split node
  int nfin, fin_base;      // subtrees finished by one block, rooted at this depth
};

// One split of a subtree that a single block finishes (k_tm_finish): the node
// at `off` (relative to the subtree's first position) of `size` members.
struct TMFinOp {
  int64_t heap;   // heap index of the node inside its job's tree (seed stream)
  int32_t off, size, job, depth;
};

struct TMPlan {
  int64_t n = -1;
  int32_t k = -1;
  std::vector<TMLevel> levels;
  // host arrays (uploaded into one device buffer)
  std::vector<int32_t> split_off, split_size, split_tile_begin, split_tile_end;  // per split node
  std::vector<int64_t> split_heap;
  std::vector<int32_t> split_job;                          // job of each split node
  std::vector<int64_t> key;                                // (n_j, k_j) of every job
  std::vector<int32_t> tile_split, tile_start, tile_len;  // per tile: local split index, range
  std::vector<int32_t> big_split;                         // local split index of big nodes
  std::vector<int32_t> bigtile;                           // tile index (global) of big-node tiles
  std::vector<int32_t> bigtile_big;                       // local big index of those tiles
  std::vector<int32_t> small_split;                       // local split index of small nodes
  std::vector<int32_t> copy_off, copy_size;               // unsplit nodes
  std::vector<int32_t> leaf_off;                          // k+1
  std::vector<int32_t> big_btb, big_bte;                  // per big node: range in the bigtile list
  std::vector<int32_t> split_cb, split_ce;                // per split node: range of its chunks
  std::vector<int32_t> chunk_tb, chunk_te;                // per chunk: range of its tiles
  std::vector<int32_t> fin_off, fin_size, fin_ob, fin_oe;  // per finished subtree: rows, op range
  std::vector<TMFinOp> fin_ops;                           // splits of the subtrees, depth order each
  int max_split = 0, max_tiles = 0, max_big = 0, max_chunks = 0;
  // device copies
  void* dev = nullptr;
  size_t dev_bytes = 0;
  const int32_t *d_split_off, *d_split_size, *d_split_tile_begin, *d_split_tile_end, *d_tile_split,
      *d_tile_start, *d_tile_len, *d_big_split, *d_bigtile, *d_bigtile_big, *d_small_split,
      *d_copy_off, *d_copy_size, *d_leaf_off, *d_big_btb, *d_big_bte, *d_split_cb, *d_split_ce,
      *d_chunk_tb, *d_chunk_te, *d_split_job, *d_fin_off, *d_fin_size, *d_fin_ob, *d_fin_oe;
  const int64_t* d_split_heap;
  const TMFinOp* d_fin_ops;
};

// The device tables live in the context workspace ("tm_plan0", "tm_plan1":
// one buffer per cached plan).
void tm_plan_free(TMPlan* p) { delete p; }

// Tree shapes of several independent jobs (job j: rows [off_j, off_j + n_j),
// k_j leaves), merged depth by depth so one launch per step covers every job
// that still splits; a job whose tree is complete is carried over as a copy.
// With finish_max > 0, a split node of at most finish_max (<= TM_TILE)
// members becomes the root of a subtree that one block finishes: its splits
// at this and every later depth leave the per-depth lists and become that
// subtree's ops.
static void build_plan(TMPlan& P, const std::vector<int64_t>& jn, const std::vector<int32_t>& jk,
                       int finish_max) {
  P = TMPlan();
  const int nj = (int)jn.size();
  P.key.clear();
  int64_t total = 0;
  for (int q = 0; q < nj; ++q) {
    P.key.push_back(jn[q]);
    P.key.push_back(jk[q]);
    total += jn[q];
  }
  P.key.push_back(finish_max);
  P.n = total;
  std::vector<std::vector<int64_t>> joff(nj), jsize(nj);
  std::vector<std::vector<int32_t>> jroot(nj);  // per node: finished subtree holding it, or -1
  std::vector<std::vector<TMFinOp>> rops;       // per finished subtree: its splits
  {
    int64_t at = 0;
    for (int q = 0; q < nj; ++q) {
      joff[q] = {at};
      jsize[q] = {jn[q]};
      jroot[q] = {-1};
      at += jn[q];
    }
  }
  auto unfinished = [&]() {
    for (int q = 0; q < nj; ++q)
      if ((int64_t)joff[q].size() < jk[q]) return true;
    return false;
  };
  int depth = 0;
  while (unfinished()) {
    TMLevel L{};
    L.depth = depth;
    L.split_base = (int)P.split_off.size();
    L.tile_base = (int)P.tile_split.size();
    L.big_base = (int)P.big_split.size();
    L.bigtile_base = (int)P.bigtile.size();
    L.small_base = (int)P.small_split.size();
    L.copy_base = (int)P.copy_off.size();
    L.chunk_base = (int)P.chunk_tb.size();
    L.fin_base = (int)P.fin_off.size();
    L.max_node_tiles = 0;
    for (int q = 0; q < nj; ++q) {
    std::vector<int64_t>& off = joff[q];
    std::vector<int64_t>& size = jsize[q];
    std::vector<int32_t>& root = jroot[q];
    const int m = (int)off.size();
    const int32_t k = jk[q];
    if ((int64_t)m >= k) {  // this job's tree is complete: carry its rows over
      P.copy_off.push_back((int32_t)off[0]);
      int64_t sz = 0;
      for (int64_t v : size) sz += v;
      P.copy_size.push_back((int32_t)sz);
      continue;
    }
    std::vector<char> split(m, 1);
    if (2 * (int64_t)m > k) {
      std::vector<int> ord(m);
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return size[a] > size[b]; });
      std::fill(split.begin(), split.end(), 0);
      for (int j = 0; j < k - m; ++j) split[ord[j]] = 1;
    }
    std::vector<int64_t> noff, nsize;
    std::vector<int32_t> nroot;
    for (int i = 0; i < m; ++i) {
      int32_t rt = root[i];
      if (rt < 0 && split[i] && size[i] <= finish_max) {
        rt = (int32_t)P.fin_off.size();
        P.fin_off.push_back((int32_t)off[i]);
        P.fin_size.push_back((int32_t)size[i]);
        rops.emplace_back();
      }
      if (rt >= 0) {
        if (split[i]) {
          TMFinOp op;
          op.heap = ((int64_t)1 << depth) + i;
          op.off = (int32_t)(off[i] - P.fin_off[rt]);
          op.size = (int32_t)size[i];
          op.job = q;
          op.depth = depth;
          rops[rt].push_back(op);
          const int64_t h = (size[i] + 1) / 2;
          noff.push_back(off[i]);
          nsize.push_back(h);
          noff.push_back(off[i] + h);
          nsize.push_back(size[i] - h);
          nroot.push_back(rt);
          nroot.push_back(rt);
        } else {
          noff.push_back(off[i]);
          nsize.push_back(size[i]);
          nroot.push_back(rt);
        }
        continue;
      }
      if (split[i]) {
        const int local = (int)P.split_off.size() - L.split_base;
        P.split_off.push_back((int32_t)off[i]);
        P.split_size.push_back((int32_t)size[i]);
        P.split_heap.push_back(((int64_t)1 << depth) + i);
        P.split_job.push_back(q);
        P.split_tile_begin.push_back((int32_t)P.tile_split.size() - L.tile_base);
        const bool big = size[i] > TM_SMALL;
        const int bigl = (int)P.big_split.size() - L.big_base;
        if (big) {
          P.big_split.push_back(local);
          P.big_btb.push_back((int32_t)P.bigtile.size() - L.bigtile_base);
        } else {
          P.small_split.push_back(local);
        }
        for (int64_t s = 0; s < size[i]; s += TM_TILE) {
          const int tl = (int)P.tile_split.size() - L.tile_base;
          P.tile_split.push_back(local);
          P.tile_start.push_back((int32_t)(off[i] + s));
          P.tile_len.push_back((int32_t)std::min<int64_t>(TM_TILE, size[i] - s));
          if (big) {
            P.bigtile.push_back(tl);
            P.bigtile_big.push_back(bigl);
          }
        }
        P.split_tile_end.push_back((int32_t)P.tile_split.size() - L.tile_base);
        if (big) P.big_bte.push_back((int32_t)P.bigtile.size() - L.bigtile_base);
        {
          const int tb = P.split_tile_begin.back(), te = P.split_tile_end.back();
          L.max_node_tiles = std::max(L.max_node_tiles, te - tb);
          P.split_cb.push_back((int32_t)P.chunk_tb.size() - L.chunk_base);
          for (int t = tb; t < te; t += TM_CHUNK) {
            P.chunk_tb.push_back(t);
            P.chunk_te.push_back(std::min(te, t + TM_CHUNK));
          }
          P.split_ce.push_back((int32_t)P.chunk_tb.size() - L.chunk_base);
        }
        const int64_t h = (size[i] + 1) / 2;
        noff.push_back(off[i]);
        nsize.push_back(h);
        noff.push_back(off[i] + h);
        nsize.push_back(size[i] - h);
        nroot.push_back(-1);
        nroot.push_back(-1);
      } else {
        P.copy_off.push_back((int32_t)off[i]);
        P.copy_size.push_back((int32_t)size[i]);
        noff.push_back(off[i]);
        nsize.push_back(size[i]);
        nroot.push_back(-1);
      }
    }
    off.swap(noff);
    size.swap(nsize);
    root.swap(nroot);
    }
    L.nfin = (int)P.fin_off.size() - L.fin_base;
    L.nsplit = (int)P.split_off.size() - L.split_base;
    L.ntiles = (int)P.tile_split.size() - L.tile_base;
    L.nbig = (int)P.big_split.size() - L.big_base;
    L.nbigtiles = (int)P.bigtile.size() - L.bigtile_base;
    L.nsmall = (int)P.small_split.size() - L.small_base;
    L.ncopy = (int)P.copy_off.size() - L.copy_base;
    L.nchunks = (int)P.chunk_tb.size() - L.chunk_base;
    P.max_chunks = std::max(P.max_chunks, L.nchunks);
    P.max_split = std::max(P.max_split, L.nsplit);
    P.max_tiles = std::max(P.max_tiles, L.ntiles);
    P.max_big = std::max(P.max_big, L.nbig);
    P.levels.push_back(L);
    ++depth;
  }
  for (const auto& ops : rops) {
    P.fin_ob.push_back((int32_t)P.fin_ops.size());
    P.fin_ops.insert(P.fin_ops.end(), ops.begin(), ops.end());
    P.fin_oe.push_back((int32_t)P.fin_ops.size());
  }
  // leaves of all jobs, left to right, job after job
  P.leaf_off.clear();
  for (int q = 0; q < nj; ++q)
    for (int64_t v : joff[q]) P.leaf_off.push_back((int32_t)v);
  P.k = (int32_t)P.leaf_off.size();
  P.leaf_off.push_back((int32_t)total);
}

static knnkm_status upload_plan(knnkm_ctx* ctx, TMPlan& P, const char* ws_name) {
  std::vector<std::pair<const void*, size_t>> parts = {
      {P.split_off.data(), P.split_off.size() * 4},   {P.split_size.data(), P.split_size.size() * 4},
      {P.split_tile_begin.data(), P.split_tile_begin.size() * 4},
      {P.split_tile_end.data(), P.split_tile_end.size() * 4},
      {P.tile_split.data(), P.tile_split.size() * 4}, {P.tile_start.data(), P.tile_start.size() * 4},
      {P.tile_len.data(), P.tile_len.size() * 4},     {P.big_split.data(), P.big_split.size() * 4},
      {P.bigtile.data(), P.bigtile.size() * 4},       {P.bigtile_big.data(), P.bigtile_big.size() * 4},
      {P.small_split.data(), P.small_split.size() * 4}, {P.copy_off.data(), P.copy_off.size() * 4},
      {P.copy_size.data(), P.copy_size.size() * 4},   {P.leaf_off.data(), P.leaf_off.size() * 4},
      {P.split_heap.data(), P.split_heap.size() * 8},
      {P.big_btb.data(), P.big_btb.size() * 4},       {P.big_bte.data(), P.big_bte.size() * 4},
      {P.split_cb.data(), P.split_cb.size() * 4},     {P.split_ce.data(), P.split_ce.size() * 4},
      {P.chunk_tb.data(), P.chunk_tb.size() * 4},     {P.chunk_te.data(), P.chunk_te.size() * 4},
      {P.split_job.data(), P.split_job.size() * 4},
      {P.fin_off.data(), P.fin_off.size() * 4},       {P.fin_size.data(), P.fin_size.size() * 4},
      {P.fin_ob.data(), P.fin_ob.size() * 4},         {P.fin_oe.data(), P.fin_oe.size() * 4},
      {P.fin_ops.data(), P.fin_ops.size() * sizeof(TMFinOp)}};
  size_t total = 0;
  std::vector<size_t> at;
  for (auto& p : parts) {
    total = (total + 15) & ~(size_t)15;
    at.push_back(total);
    total += p.second;
  }
  total += 16;
  P.dev = knnkm_ws(ctx, ws_name, total);
  if (!P.dev) return KNNKM_ENOMEM;
  P.dev_bytes = total;
  std::vector<char> host(total, 0);
  for (size_t i = 0; i < parts.size(); ++i)
    if (parts[i].second) std::memcpy(host.data() + at[i], parts[i].first, parts[i].second);
  KNNKM_HIP(ctx, hipMemcpyAsync(P.dev, host.data(), total, hipMemcpyHostToDevice, ctx->stream));
  // `host` is released on return
  KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const char* b = (const char*)P.dev;
  P.d_split_off = (const int32_t*)(b + at[0]);
  P.d_split_size = (const int32_t*)(b + at[1]);
  P.d_split_tile_begin = (const int32_t*)(b + at[2]);
  P.d_split_tile_end = (const int32_t*)(b + at[3]);
  P.d_tile_split = (const int32_t*)(b + at[4]);
  P.d_tile_start = (const int32_t*)(b + at[5]);
  P.d_tile_len = (const int32_t*)(b + at[6]);
  P.d_big_split = (const int32_t*)(b + at[7]);
  P.d_bigtile = (const int32_t*)(b + at[8]);
  P.d_bigtile_big = (const int32_t*)(b + at[9]);
  P.d_small_split = (const int32_t*)(b + at[10]);
  P.d_copy_off = (const int32_t*)(b + at[11]);
  P.d_copy_size = (const int32_t*)(b + at[12]);
  P.d_leaf_off = (const int32_t*)(b + at[13]);
  P.d_split_heap = (const int64_t*)(b + at[14]);
  P.d_big_btb = (const int32_t*)(b + at[15]);
  P.d_big_bte = (const int32_t*)(b + at[16]);
  P.d_split_cb = (const int32_t*)(b + at[17]);
  P.d_split_ce = (const int32_t*)(b + at[18]);
  P.d_chunk_tb = (const int32_t*)(b + at[19]);
  P.d_chunk_te = (const int32_t*)(b + at[20]);
  P.d_split_job = (const int32_t*)(b + at[21]);
  P.d_fin_off = (const int32_t*)(b + at[22]);
  P.d_fin_size = (const int32_t*)(b + at[23]);
  P.d_fin_ob = (const int32_t*)(b + at[24]);
  P.d_fin_oe = (const int32_t*)(b + at[25]);
  P.d_fin_ops = (const TMFinOp*)(b + at[26]);
  return KNNKM_OK;
}

// ------------------------------------------------------------------ kernels --
__global__ void k_iota(int32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}

// One wave per split node: seed centroids from two distinct members.
__global__ __launch_bounds__(256) void k_tm_seed(const float* __restrict__ X, int d, int64_t ldx,
                                                 const int32_t* __restrict__ perm, int nsplit,
                                                 const int32_t* __restrict__ s_off,
                                                 const int32_t* __restrict__ s_size,
                                                 const int64_t* __restrict__ s_heap,
                                                 const int32_t* __restrict__ s_job,
                                                 const uint64_t* __restrict__ seeds, uint64_t seed1,
                                                 int round_tag, float* __restrict__ cent) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nsplit) return;
  const uint32_t s = (uint32_t)s_size[j];
  const uint64_t seed = seeds ? seeds[s_job[j]] : seed1;
  const uint64_t key = sm_key(seed, sm_stream(RNG_TWOMEANS, (uint64_t)round_tag, (uint64_t)s_heap[j]));
  const uint32_t r0 = sm_below(sm_draw(key, 0), s);
  uint32_t r1 = sm_below(sm_draw(key, 1), s - 1);
  if (r1 >= r0) r1 += 1;
  const float* xu = X + (int64_t)perm[s_off[j] + r0] * ldx;
  const float* xv = X + (int64_t)perm[s_off[j] + r1] * ldx;
  float* cu = cent + (int64_t)j * 2 * d;
  for (int dim = lane; dim < d; dim += 64) {
    cu[dim] = xu[dim];
    cu[d + dim] = xv[dim];
  }
}

// delta = sum_j (c_v - c_u)_j (2 x_j - c_u - c_v)_j over the group's dims, with
// w = c_v - c_u and s = c_u + c_v held per lane in float64 (every product of
// these float32-derived values is exact in float64; only the sums round).
template <int V>
__device__ inline double tm_part(const float (&x)[V], const double (&wv)[V], const double (&sv)[V]) {
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < V; ++e) acc = fma(wv[e], fma(2.0, (double)x[e], -sv[e]), acc);
  return acc;
}

template <int V>
__device__ inline void tm_node_consts(const float* __restrict__ cu, const float* __restrict__ cv, int j, int d,
                                      double (&wv)[V], double (&sv)[V]) {
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const int dim = j * V + e;
    const double u = dim < d ? (double)cu[dim] : 0.0, v = dim < d ? (double)cv[dim] : 0.0;
    wv[e] = v - u;
    sv[e] = u + v;
  }
}

// Rows at positions p, p + step, ..., p + (U-1) step of a node (those below
// len), all loaded before any is used so that U row loads are in flight per
// group; ids[q] is the sample at node position q.
template <int V, int U>
__device__ inline void tm_load_rows(float (&x)[U][V], const float* __restrict__ X, int64_t ldx,
                                    const int32_t* ids, int p, int step, int len, int j, int d,
                                    bool vec) {
  int32_t id[U];
#pragma unroll
  for (int u = 0; u < U; ++u) id[u] = p + u * step < len ? ids[p + u * step] : -1;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (id[u] >= 0) {
      load_row<V>(x[u], X + (int64_t)id[u] * ldx, j, d, vec);
    } else {
#pragma unroll
      for (int e = 0; e < V; ++e) x[u][e] = 0.f;
    }
  }
}

#define TM_UNROLL 4
#define TM_FIN_UNROLL 3  // fewer in flight per group in the finisher: four blocks per CU fit

// One block per tile: side of each member, float64 sums per side.  Group gid
// of the block takes tile positions gid, gid + NG, ...; the NG group sums are
// then added in group order.
template <int L, int V>
__global__ __launch_bounds__(256) void k_tm_accum(const float* __restrict__ X, int d, int64_t ldx,
                                                  const int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ t_split,
                                                  const int32_t* __restrict__ t_start,
                                                  const int32_t* __restrict__ t_len,
                                                  const float* __restrict__ cent,
                                                  double* __restrict__ partial,
                                                  int32_t* __restrict__ pcnt, int vec) {
  constexpr int NG = 4 * (64 / L);
  __shared__ double sh[NG][2][L * V];
  __shared__ int32_t shc[NG][2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = lane % L, gid = w * (64 / L) + lane / L;
  const int tile = blockIdx.x;
  const int js = t_split[tile];
  const int start = t_start[tile], len = t_len[tile];
  const float* cu = cent + (int64_t)js * 2 * d;
  double wv[V], sv[V];
  tm_node_consts<V>(cu, cu + d, j, d, wv, sv);
  double au[V], av[V];
#pragma unroll
  for (int e = 0; e < V; ++e) au[e] = av[e] = 0.0;
  int cnu = 0, cnv = 0;
  for (int p = gid; p < len; p += TM_UNROLL * NG) {
    float x[TM_UNROLL][V];
    tm_load_rows<V, TM_UNROLL>(x, X, ldx, perm + start, p, NG, len, j, d, vec);
#pragma unroll
    for (int u = 0; u < TM_UNROLL; ++u) {
      if (p + u * NG < len) {  // members in position order, as one row at a time
        const double delta = group_sum<L>(tm_part<V>(x[u], wv, sv));
        if (delta <= 0.0) {
          ++cnu;
#pragma unroll
          for (int e = 0; e < V; ++e) au[e] += (double)x[u][e];
        } else {
          ++cnv;
#pragma unroll
          for (int e = 0; e < V; ++e) av[e] += (double)x[u][e];
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < V; ++e) {
    sh[gid][0][j * V + e] = au[e];
    sh[gid][1][j * V + e] = av[e];
  }
  if (j == 0) {
    shc[gid][0] = cnu;
    shc[gid][1] = cnv;
  }
  __syncthreads();
  double* out = partial + (int64_t)tile * 2 * d;
  for (int e = threadIdx.x; e < 2 * d; e += 256) {
    const int side = e / d, dim = e % d;
    double s = 0.0;
    for (int q = 0; q < NG; ++q) s += sh[q][side][dim];
    out[e] = s;
  }
  if (threadIdx.x < 2) {
    int c = 0;
    for (int q = 0; q < NG; ++q) c += shc[q][threadIdx.x];
    pcnt[tile * 2 + threadIdx.x] = c;
  }
}

// Chunk partial = ordered sum of its tiles: one block per (chunk, 64 of the
// 2d coordinates); per coordinate wavefront w sums tiles w, w + 4, ... in
// order, then ((w0 + w1) + w2) + w3.
__global__ __launch_bounds__(256) void k_tm_chunk(int d, const int32_t* __restrict__ c_tb,
                                                  const int32_t* __restrict__ c_te,
                                                  const double* __restrict__ partial,
                                                  const int32_t* __restrict__ pcnt,
                                                  double* __restrict__ cpart, int32_t* __restrict__ ccnt) {
  __shared__ double sh[4][64];
  __shared__ int32_t shc[8];
  const int c = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tb = c_tb[c], te = c_te[c];
  const int e = 64 * blockIdx.y + lane;
  if (e < 2 * d) {
    double a = 0.0;
    for (int t = tb + w; t < te; t += 4) a += partial[(int64_t)t * 2 * d + e];
    sh[w][lane] = a;
  }
  if (blockIdx.y == 0 && lane == 0) {
    int nu = 0, nv = 0;
    for (int t = tb + w; t < te; t += 4) {
      nu += pcnt[2 * t];
      nv += pcnt[2 * t + 1];
    }
    shc[2 * w] = nu;
    shc[2 * w + 1] = nv;
  }
  __syncthreads();
  if (w == 0 && e < 2 * d) cpart[(int64_t)c * 2 * d + e] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
  if (blockIdx.y == 0 && threadIdx.x < 2)
    ccnt[2 * c + threadIdx.x] = shc[threadIdx.x] + shc[2 + threadIdx.x] + shc[4 + threadIdx.x] + shc[6 + threadIdx.x];
}

// New centroids of the split nodes from their partials (tiles, or chunks of
// tiles for nodes with many tiles), added in a fixed order: one block per
// (split node, 64 of its 2d mean coordinates); per coordinate wavefront w
// sums the node's tiles or chunks w, w + 4, ... in order, then
// ((w0 + w1) + w2) + w3.
__global__ __launch_bounds__(256) void k_tm_final(int d, const int32_t* __restrict__ s_tb,
                                                  const int32_t* __restrict__ s_te,
                                                  const double* __restrict__ partial,
                                                  const int32_t* __restrict__ pcnt,
                                                  float* __restrict__ cent) {
  __shared__ double sh[4][64];
  __shared__ int32_t shc[8];
  const int js = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tb = s_tb[js], te = s_te[js];
  const int e = 64 * blockIdx.y + lane;
  if (e < 2 * d) {
    double a = 0.0;
    for (int t = tb + w; t < te; t += 4) a += partial[(int64_t)t * 2 * d + e];
    sh[w][lane] = a;
  }
  if (lane == 0) {
    int nu = 0, nv = 0;
    for (int t = tb + w; t < te; t += 4) {
      nu += pcnt[2 * t];
      nv += pcnt[2 * t + 1];
    }
    shc[2 * w] = nu;
    shc[2 * w + 1] = nv;
  }
  __syncthreads();
  if (w == 0 && e < 2 * d) {
    const int cnt = e < d ? shc[0] + shc[2] + shc[4] + shc[6] : shc[1] + shc[3] + shc[5] + shc[7];
    const double a = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
    if (cnt > 0) cent[(int64_t)js * 2 * d + e] = (float)(a / (double)cnt);
  }
}

// delta keys of every member of every split node (position-indexed).
template <int L, int V>
__global__ __launch_bounds__(256) void k_tm_delta(const float* __restrict__ X, int d, int64_t ldx,
                                                  const int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ t_split,
                                                  const int32_t* __restrict__ t_start,
                                                  const int32_t* __restrict__ t_len,
                                                  const float* __restrict__ cent,
                                                  uint64_t* __restrict__ keys, int vec) {
  constexpr int NG = 4 * (64 / L);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = lane % L, gid = w * (64 / L) + lane / L;
  const int tile = blockIdx.x;
  const int js = t_split[tile];
  const int start = t_start[tile], len = t_len[tile];
  const float* cu = cent + (int64_t)js * 2 * d;
  double wv[V], sv[V];
  tm_node_consts<V>(cu, cu + d, j, d, wv, sv);
  for (int p = gid; p < len; p += TM_UNROLL * NG) {
    float x[TM_UNROLL][V];
    tm_load_rows<V, TM_UNROLL>(x, X, ldx, perm + start, p, NG, len, j, d, vec);
#pragma unroll
    for (int u = 0; u < TM_UNROLL; ++u) {
      if (p + u * NG < len) {
        const double delta = group_sum<L>(tm_part<V>(x[u], wv, sv));
        if (j == 0) keys[start + p + u * NG] = dkey(delta);
      }
    }
  }
}

// Composite order (key, id).
__device__ inline bool kv_le(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib) {
  return ka < kb || (ka == kb && ia <= ib);
}

// Block-level stable partition of positions [off, off+s): members with
// (key,id) <= threshold go to [off, off+h) in order, the rest to [off+h, off+s).
__device__ void tm_partition_block(const int32_t* __restrict__ perm, const uint64_t* __restrict__ keys,
                                   int off, int s, int h, uint64_t tk, int32_t ti,
                                   int32_t* __restrict__ perm_out, int32_t* sh_scan) {
  const int per = (s + 255) / 256;
  const int p0 = off + threadIdx.x * per;
  const int p1 = min(off + s, p0 + per);
  int cnt = 0;
  for (int p = p0; p < p1; ++p) cnt += kv_le(keys[p], perm[p], tk, ti) ? 1 : 0;
  sh_scan[threadIdx.x] = cnt;
  __syncthreads();
  // exclusive scan of 256 counts (simple, thread 0 sequential is fine for 256)
  if (threadIdx.x == 0) {
    int run = 0;
    for (int j = 0; j < 256; ++j) {
      int c = sh_scan[j];
      sh_scan[j] = run;
      run += c;
    }
  }
  __syncthreads();
  int lpos = off + sh_scan[threadIdx.x];
  int rpos = off + h + ((p0 - off) - sh_scan[threadIdx.x]);
  for (int p = p0; p < p1; ++p) {
    const int32_t id = perm[p];
    if (kv_le(keys[p], id, tk, ti))
      perm_out[lpos++] = id;
    else
      perm_out[rpos++] = id;
  }
}

// Nodes of at most TM_SMALL members: bitonic sort of (key, id) in LDS to find
// the ceil(s/2)-th pair, then a stable partition.
__global__ __launch_bounds__(256) void k_tm_split_small(const int32_t* __restrict__ perm,
                                                        const uint64_t* __restrict__ keys,
                                                        const int32_t* __restrict__ small_split,
                                                        const int32_t* __restrict__ s_off,
                                                        const int32_t* __restrict__ s_size,
                                                        int32_t* __restrict__ perm_out) {
  __shared__ uint64_t sk[TM_SMALL];
  __shared__ int32_t si[TM_SMALL];
  __shared__ int32_t sh_scan[256];
  const int j = small_split[blockIdx.x];
  const int off = s_off[j], s = s_size[j];
  int P = 1;
  while (P < s) P <<= 1;
  for (int e = threadIdx.x; e < P; e += 256) {
    if (e < s) {
      sk[e] = keys[off + e];
      si[e] = perm[off + e];
    } else {
      sk[e] = ~0ull;
      si[e] = INT32_MAX;
    }
  }
  __syncthreads();
  for (int kk = 2; kk <= P; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int e = threadIdx.x; e < P; e += 256) {
        const int x = e ^ jj;
        if (x > e) {
          const bool up = (e & kk) == 0;
          const bool gt = !kv_le(sk[e], si[e], sk[x], si[x]);
          if (gt == up) {
            uint64_t tk = sk[e];
            sk[e] = sk[x];
            sk[x] = tk;
            int32_t ti = si[e];
            si[e] = si[x];
            si[x] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  const int h = (s + 1) / 2;
  const uint64_t tk = sk[h - 1];
  const int32_t ti = si[h - 1];
  __syncthreads();
  tm_partition_block(perm, keys, off, s, h, tk, ti, perm_out, sh_scan);
}

// Nodes larger than one tile: radix select of the ceil(s/2)-th smallest
// delta key, 8 bits per pass.  The members whose key equals it are ordered
// by id, and a node holds its members in ascending id order (every split is
// a stable partition of an ascending sequence), so the ones that go left are
// the first h' of them in position order, h' being the rank left inside the
// last bucket: the partition counts them instead of selecting on the id.
struct SelState {
  uint64_t pk;  // decided high bits of the key
  int32_t h;    // rank still to find inside the current bucket (1-based)
};

__device__ inline int sel_digit(uint64_t key, int pass) { return (int)((key >> (56 - 8 * pass)) & 255); }
__device__ inline bool sel_match(uint64_t key, int pass, const SelState& st) {
  if (pass == 0) return true;
  const int sh = 64 - 8 * pass;
  return (key >> sh) == (st.pk >> sh);
}

// Selection state and histograms are kept per pass: st[p * nbig + b] is the
// prefix decided before pass p of big node b, hist[(p * nbig + b) * 256 + .]
// the digit counts of pass p.  Each pass's blocks derive their own state from
// the previous pass's finished histogram, so no block waits for another.
__global__ __launch_bounds__(256) void k_tm_sel_init(int nbig, const int32_t* __restrict__ big_split,
                                                     const int32_t* __restrict__ s_size,
                                                     SelState* st, int32_t* hist) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nbig; b += gridDim.x * blockDim.x) {
    st[b].pk = 0;
    st[b].h = (s_size[big_split[b]] + 1) / 2;
  }
  for (int64_t e = blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)nbig * 256 * TM_SEL_PASSES;
       e += gridDim.x * blockDim.x)
    hist[e] = 0;
}

// Whole block: the state after `pass` from the state before it and that
// pass's histogram: the bucket holding the rank-h member is the digit whose
// exclusive prefix count is < h <= inclusive count.
__device__ inline SelState sel_next(const SelState& s, const int32_t* __restrict__ hh, int pass,
                                    int32_t* sh8, SelState* shs) {
  const int32_t c = hh[threadIdx.x];
  int32_t tot;
  const int32_t ex = block_scan_excl_256(c, sh8, &tot);
  if (c > 0 && ex < s.h && s.h <= ex + c) {
    SelState t = s;
    t.h -= ex;
    t.pk |= (uint64_t)threadIdx.x << (56 - 8 * pass);
    *shs = t;
  }
  __syncthreads();
  const SelState r = *shs;
  __syncthreads();
  return r;
}

// One block per tile of a big node: state for this pass (the first tile's
// block stores it), then the histogram of the current digit over the members
// that match the decided prefix, added into the node's histogram of the pass.
__global__ __launch_bounds__(256) void k_tm_sel_pass(const int32_t* __restrict__ perm,
                                                     const uint64_t* __restrict__ keys,
                                                     const int32_t* __restrict__ bigtile,
                                                     const int32_t* __restrict__ bigtile_big,
                                                     const int32_t* __restrict__ big_btb,
                                                     const int32_t* __restrict__ t_start,
                                                     const int32_t* __restrict__ t_len, int pass, int nbig,
                                                     SelState* __restrict__ st, int32_t* __restrict__ hist) {
  __shared__ int32_t h[256];
  __shared__ int32_t sh8[8];
  __shared__ SelState shs;
  h[threadIdx.x] = 0;
  const int tile = bigtile[blockIdx.x];
  const int b = bigtile_big[blockIdx.x];
  SelState s;
  if (pass == 0) {
    s = st[b];
  } else {
    s = sel_next(st[(int64_t)(pass - 1) * nbig + b], hist + ((int64_t)(pass - 1) * nbig + b) * 256, pass - 1,
                 sh8, &shs);
    if (blockIdx.x == big_btb[b] && threadIdx.x == 0) st[(int64_t)pass * nbig + b] = s;
  }
  __syncthreads();
  const int start = t_start[tile], len = t_len[tile];
  for (int p = threadIdx.x; p < len; p += 256) {
    const uint64_t key = keys[start + p];
    if (sel_match(key, pass, s)) atomicAdd(&h[sel_digit(key, pass)], 1);
  }
  __syncthreads();
  const int c = h[threadIdx.x];
  if (c) atomicAdd(&hist[((int64_t)pass * nbig + b) * 256 + threadIdx.x], c);
}

// One block per tile of a big node: the node's threshold key (the state
// after the last pass; the first tile's block stores it) and the tile's
// numbers of members below it and equal to it.
__global__ __launch_bounds__(256) void k_tm_part_count(const uint64_t* __restrict__ keys,
                                                       const int32_t* __restrict__ bigtile,
                                                       const int32_t* __restrict__ bigtile_big,
                                                       const int32_t* __restrict__ big_btb,
                                                       const int32_t* __restrict__ t_start,
                                                       const int32_t* __restrict__ t_len, int nbig,
                                                       SelState* __restrict__ st, const int32_t* __restrict__ hist,
                                                       int32_t* __restrict__ tile_less, int32_t* __restrict__ tile_tie) {
  __shared__ int32_t cl, ct;
  __shared__ int32_t sh8[8];
  __shared__ SelState shs;
  if (threadIdx.x == 0) cl = ct = 0;
  const int tile = bigtile[blockIdx.x];
  const int b = bigtile_big[blockIdx.x];
  constexpr int LAST = TM_SEL_PASSES - 1;
  const SelState s = sel_next(st[(int64_t)LAST * nbig + b], hist + ((int64_t)LAST * nbig + b) * 256, LAST,
                              sh8, &shs);
  if (blockIdx.x == big_btb[b] && threadIdx.x == 0) st[(int64_t)TM_SEL_PASSES * nbig + b] = s;
  const int start = t_start[tile], len = t_len[tile];
  int less = 0, tie = 0;
  for (int p = threadIdx.x; p < len; p += 256) {
    const uint64_t key = keys[start + p];
    less += key < s.pk ? 1 : 0;
    tie += key == s.pk ? 1 : 0;
  }
  atomicAdd(&cl, less);
  atomicAdd(&ct, tie);
  __syncthreads();
  if (threadIdx.x == 0) {
    tile_less[blockIdx.x] = cl;
    tile_tie[blockIdx.x] = ct;
  }
}

// One block per big node: exclusive scans of both counts over its tiles.
__global__ __launch_bounds__(256) void k_tm_part_scan(const int32_t* __restrict__ big_btb,
                                                      const int32_t* __restrict__ big_bte,
                                                      int32_t* __restrict__ tile_less,
                                                      int32_t* __restrict__ tile_tie) {
  __shared__ int32_t sh[8];
  const int b = blockIdx.x;
  const int tb = big_btb[b], te = big_bte[b];
  int32_t carry_l = 0, carry_t = 0;
  for (int base = tb; base < te; base += 256) {
    const int t = base + threadIdx.x;
    int32_t tot;
    const int32_t ex_l = block_scan_excl_256(t < te ? tile_less[t] : 0, sh, &tot);
    if (t < te) tile_less[t] = carry_l + ex_l;
    carry_l += tot;
    const int32_t ex_t = block_scan_excl_256(t < te ? tile_tie[t] : 0, sh, &tot);
    if (t < te) tile_tie[t] = carry_t + ex_t;
    carry_t += tot;
  }
}

// Stable partition of a big node, tile by tile: a member goes left when its
// key is below the threshold, or equal to it and among the first h' such
// members of the node in position order.  Each thread takes a contiguous
// chunk of the tile; lefts_before = less_before + min(ties_before, h').
__global__ __launch_bounds__(256) void k_tm_part_write(const int32_t* __restrict__ perm,
                                                       const uint64_t* __restrict__ keys,
                                                       const int32_t* __restrict__ bigtile,
                                                       const int32_t* __restrict__ bigtile_big,
                                                       const int32_t* __restrict__ big_split,
                                                       const int32_t* __restrict__ s_off,
                                                       const int32_t* __restrict__ s_size,
                                                       const int32_t* __restrict__ t_start,
                                                       const int32_t* __restrict__ t_len,
                                                       const SelState* __restrict__ st,
                                                       const int32_t* __restrict__ less_base,
                                                       const int32_t* __restrict__ tie_base,
                                                       int32_t* __restrict__ perm_out) {
  __shared__ int32_t sh8[8];
  const int tile = bigtile[blockIdx.x];
  const int b = bigtile_big[blockIdx.x];
  const SelState s = st[b];
  const uint64_t tk = s.pk;
  const int hp = s.h;
  const int j = big_split[b];
  const int off = s_off[j], h = (s_size[j] + 1) / 2;
  const int start = t_start[tile], len = t_len[tile];
  const int per = (len + 255) / 256;
  const int p0 = start + threadIdx.x * per;
  const int p1 = min(start + len, p0 + per);
  int cl = 0, ct = 0;
  for (int p = p0; p < p1; ++p) {
    const uint64_t key = keys[p];
    cl += key < tk ? 1 : 0;
    ct += key == tk ? 1 : 0;
  }
  int32_t tot;
  int lb = less_base[blockIdx.x] + block_scan_excl_256(cl, sh8, &tot);
  int tb = tie_base[blockIdx.x] + block_scan_excl_256(ct, sh8, &tot);
  for (int p = p0; p < p1; ++p) {
    const int32_t id = perm[p];
    const uint64_t key = keys[p];
    const int lefts_before = lb + min(tb, hp);
    const bool left = key < tk || (key == tk && tb < hp);
    if (left)
      perm_out[off + lefts_before] = id;
    else
      perm_out[off + h + (p - off) - lefts_before] = id;
    lb += key < tk ? 1 : 0;
    tb += key == tk ? 1 : 0;
  }
}

__global__ void k_tm_copy(const int32_t* __restrict__ perm, const int32_t* __restrict__ c_off,
                          const int32_t* __restrict__ c_size, int32_t* __restrict__ perm_out) {
  const int j = blockIdx.x;
  const int off = c_off[j], s = c_size[j];
  for (int p = threadIdx.x; p < s; p += blockDim.x) perm_out[off + p] = perm[off + p];
}

__global__ void k_tm_labels(const int32_t* __restrict__ perm, const int32_t* __restrict__ leaf_off,
                            int32_t k, int32_t* __restrict__ labels) {
  for (int r = blockIdx.x; r < k; r += gridDim.x)
    for (int p = leaf_off[r] + threadIdx.x; p < leaf_off[r + 1]; p += blockDim.x) labels[perm[p]] = r;
}

// One block per subtree of at most TM_TILE members: every remaining split of
// the subtree, depth after depth, with the member ids held in LDS.  Each step
// does the same arithmetic in the same order as the per-depth kernels above
// (group gid of the block sums positions gid, gid + NG, ... of the node; the
// group sums are added in group order; a one-tile node's mean passes through
// the same additions of zero as the per-node reduction), so the tree is
// bitwise the one the per-depth path builds.  The final ids go to both
// permutation buffers, so the ping-pong copies of later depths see them.
template <int L, int V>
__global__ __launch_bounds__(256, 4) void k_tm_finish(const float* __restrict__ X, int d, int64_t ldx,
                                                   int32_t* __restrict__ perm_a, int32_t* __restrict__ perm_b,
                                                   const int32_t* __restrict__ f_off,
                                                   const int32_t* __restrict__ f_size,
                                                   const int32_t* __restrict__ f_ob,
                                                   const int32_t* __restrict__ f_oe,
                                                   const TMFinOp* __restrict__ ops,
                                                   const uint64_t* __restrict__ seeds, uint64_t seed1,
                                                   int round_tag, int iters, int vec) {
  constexpr int NG = 4 * (64 / L);
  constexpr int W = L * V;
  constexpr int ACC_BYTES = NG * W * 8;  // one side's group sums at a time
  constexpr int SORT_BYTES = TM_TILE * 12;
  __shared__ int32_t sid[TM_TILE];
  __shared__ uint64_t skey[TM_TILE];
  __shared__ float scent[2 * KNNKM_MAX_D];
  // group sums, or the sort buffers, or the partition's output
  __shared__ __align__(16) char sraw[ACC_BYTES > SORT_BYTES ? ACC_BYTES : SORT_BYTES];
  __shared__ int32_t shc[NG][2];
  __shared__ int32_t sscan[8];
  double(*acc)[W] = reinterpret_cast<double(*)[W]>(sraw);
  uint64_t* sk = reinterpret_cast<uint64_t*>(sraw);
  int32_t* si = reinterpret_cast<int32_t*>(sraw + TM_TILE * 8);
  int32_t* sid2 = reinterpret_cast<int32_t*>(sraw);

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = lane % L, gid = w * (64 / L) + lane / L;
  const int R0 = f_off[blockIdx.x], S = f_size[blockIdx.x];
  for (int p = threadIdx.x; p < S; p += 256) sid[p] = perm_a[R0 + p];
  __syncthreads();
  for (int o = f_ob[blockIdx.x]; o < f_oe[blockIdx.x]; ++o) {
    const TMFinOp op = ops[o];
    const int off = op.off, s = op.size;
    {  // seeds: two distinct members
      const uint64_t seed = seeds ? seeds[op.job] : seed1;
      const uint64_t key = sm_key(seed, sm_stream(RNG_TWOMEANS, (uint64_t)round_tag, (uint64_t)op.heap));
      const uint32_t r0 = sm_below(sm_draw(key, 0), (uint32_t)s);
      uint32_t r1 = sm_below(sm_draw(key, 1), (uint32_t)s - 1);
      if (r1 >= r0) r1 += 1;
      const float* xu = X + (int64_t)sid[off + r0] * ldx;
      const float* xv = X + (int64_t)sid[off + r1] * ldx;
      for (int dim = threadIdx.x; dim < d; dim += 256) {
        scent[dim] = xu[dim];
        scent[d + dim] = xv[dim];
      }
    }
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
      double wv[V], sv[V];
      tm_node_consts<V>(scent, scent + d, j, d, wv, sv);
      double au[V], av[V];
#pragma unroll
      for (int e = 0; e < V; ++e) au[e] = av[e] = 0.0;
      int cnu = 0, cnv = 0;
      for (int p = gid; p < s; p += TM_FIN_UNROLL * NG) {
        float x[TM_FIN_UNROLL][V];
        tm_load_rows<V, TM_FIN_UNROLL>(x, X, ldx, sid + off, p, NG, s, j, d, vec);
#pragma unroll
        for (int u = 0; u < TM_FIN_UNROLL; ++u) {
          if (p + u * NG < s) {
            const double delta = group_sum<L>(tm_part<V>(x[u], wv, sv));
            if (delta <= 0.0) {
              ++cnu;
#pragma unroll
              for (int e = 0; e < V; ++e) au[e] += (double)x[u][e];
            } else {
              ++cnv;
#pragma unroll
              for (int e = 0; e < V; ++e) av[e] += (double)x[u][e];
            }
          }
        }
      }
      if (j == 0) {
        shc[gid][0] = cnu;
        shc[gid][1] = cnv;
      }
      for (int side = 0; side < 2; ++side) {
#pragma unroll
        for (int e = 0; e < V; ++e) acc[gid][j * V + e] = side ? av[e] : au[e];
        __syncthreads();
        for (int dim = threadIdx.x; dim < d; dim += 256) {
          double t = 0.0;
          for (int q = 0; q < NG; ++q) t += acc[q][dim];
          const double sum = (((0.0 + t) + 0.0) + 0.0) + 0.0;
          int cnt = 0;
          for (int q = 0; q < NG; ++q) cnt += shc[q][side];
          if (cnt > 0) scent[side * d + dim] = (float)(sum / (double)cnt);
        }
        __syncthreads();
      }
    }
    {  // delta keys with the final centroids
      double wv[V], sv[V];
      tm_node_consts<V>(scent, scent + d, j, d, wv, sv);
      for (int p = gid; p < s; p += TM_FIN_UNROLL * NG) {
        float x[TM_FIN_UNROLL][V];
        tm_load_rows<V, TM_FIN_UNROLL>(x, X, ldx, sid + off, p, NG, s, j, d, vec);
#pragma unroll
        for (int u = 0; u < TM_FIN_UNROLL; ++u) {
          if (p + u * NG < s) {
            const double delta = group_sum<L>(tm_part<V>(x[u], wv, sv));
            if (j == 0) skey[off + p + u * NG] = dkey(delta);
          }
        }
      }
    }
    __syncthreads();
    // threshold: the ceil(s/2)-th smallest (key, id), by a bitonic sort
    int P2 = 1;
    while (P2 < s) P2 <<= 1;
    for (int e = threadIdx.x; e < P2; e += 256) {
      sk[e] = e < s ? skey[off + e] : ~0ull;
      si[e] = e < s ? sid[off + e] : INT32_MAX;
    }
    __syncthreads();
    for (int kk = 2; kk <= P2; kk <<= 1) {
      for (int jj = kk >> 1; jj > 0; jj >>= 1) {
        for (int e = threadIdx.x; e < P2; e += 256) {
          const int x = e ^ jj;
          if (x > e) {
            const bool up = (e & kk) == 0;
            const bool gt = !kv_le(sk[e], si[e], sk[x], si[x]);
            if (gt == up) {
              const uint64_t tk = sk[e];
              sk[e] = sk[x];
              sk[x] = tk;
              const int32_t ti = si[e];
              si[e] = si[x];
              si[x] = ti;
            }
          }
        }
        __syncthreads();
      }
    }
    const int h = (s + 1) / 2;
    const uint64_t tk = sk[h - 1];
    const int32_t ti = si[h - 1];
    // stable partition of the node's positions: (key, id) <= threshold first
    const int per = (s + 255) / 256;
    const int p0 = threadIdx.x * per, p1 = min(s, p0 + per);
    int cnt = 0;
    for (int p = p0; p < p1; ++p) cnt += kv_le(skey[off + p], sid[off + p], tk, ti) ? 1 : 0;
    int32_t tot;
    const int32_t before = block_scan_excl_256(cnt, sscan, &tot);
    int lpos = off + before, rpos = off + h + (min(p0, s) - before);
    for (int p = p0; p < p1; ++p) {
      const int32_t id = sid[off + p];
      if (kv_le(skey[off + p], id, tk, ti))
        sid2[lpos++] = id;
      else
        sid2[rpos++] = id;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < s; p += 256) sid[off + p] = sid2[off + p];
    __syncthreads();
  }
  for (int p = threadIdx.x; p < S; p += 256) {
    perm_a[R0 + p] = sid[p];
    perm_b[R0 + p] = sid[p];
  }
}

// ------------------------------------------------------------------ driver --
template <int L, int V>
static void launch_accum(knnkm_ctx* ctx, const TMPlan& P, const TMLevel& Lv, const float* X, int d,
                         int64_t ldx, const int32_t* perm, const float* cent, double* partial,
                         int32_t* pcnt, bool vec) {
  k_tm_accum<L, V><<<Lv.ntiles, 256, 0, ctx->stream>>>(X, d, ldx, perm, P.d_tile_split + Lv.tile_base,
                                                       P.d_tile_start + Lv.tile_base,
                                                       P.d_tile_len + Lv.tile_base, cent, partial, pcnt,
                                                       vec ? 1 : 0);
}
template <int L, int V>
static void launch_delta(knnkm_ctx* ctx, const TMPlan& P, const TMLevel& Lv, const float* X, int d,
                         int64_t ldx, const int32_t* perm, const float* cent, uint64_t* keys, bool vec) {
  k_tm_delta<L, V><<<Lv.ntiles, 256, 0, ctx->stream>>>(X, d, ldx, perm, P.d_tile_split + Lv.tile_base,
                                                       P.d_tile_start + Lv.tile_base,
                                                       P.d_tile_len + Lv.tile_base, cent, keys,
                                                       vec ? 1 : 0);
}

template <int L, int V>
static void launch_finish(knnkm_ctx* ctx, const TMPlan& P, const TMLevel& Lv, const float* X, int d,
                          int64_t ldx, int32_t* perm, int32_t* perm_next, const uint64_t* seeds,
                          uint64_t seed1, int round_tag, int iters, bool vec) {
  k_tm_finish<L, V><<<Lv.nfin, 256, 0, ctx->stream>>>(
      X, d, ldx, perm, perm_next, P.d_fin_off + Lv.fin_base, P.d_fin_size + Lv.fin_base,
      P.d_fin_ob + Lv.fin_base, P.d_fin_oe + Lv.fin_base, P.d_fin_ops, seeds, seed1, round_tag, iters,
      vec ? 1 : 0);
}

// Dispatch on the row-group shape chosen for d.
#define TM_DISPATCH(FN, ...)                     \
  do {                                           \
    if (gV == 4) {                               \
      switch (gL) {                              \
        case 4: FN<4, 4>(__VA_ARGS__); break;    \
        case 8: FN<8, 4>(__VA_ARGS__); break;    \
        case 16: FN<16, 4>(__VA_ARGS__); break;  \
        case 32: FN<32, 4>(__VA_ARGS__); break;  \
        default: FN<64, 4>(__VA_ARGS__); break;  \
      }                                          \
    } else {                                     \
      switch (gL) {                              \
        case 4: FN<4, 8>(__VA_ARGS__); break;    \
        case 8: FN<8, 8>(__VA_ARGS__); break;    \
        case 16: FN<16, 8>(__VA_ARGS__); break;  \
        case 32: FN<32, 8>(__VA_ARGS__); break;  \
        default: FN<64, 8>(__VA_ARGS__); break;  \
      }                                          \
    }                                            \
  } while (0)

knnkm_status ks_twomeans_multi(knnkm_ctx* ctx, const float* X, int32_t d, int64_t ldx,
                               const std::vector<int64_t>& jn, const std::vector<int32_t>& jk,
                               const uint64_t* seeds_dev, uint64_t seed1, int32_t round_tag, int32_t iters,
                               int32_t* labels) {
  std::vector<int64_t> key;
  int64_t n = 0;
  for (size_t q = 0; q < jn.size(); ++q) {
    key.push_back(jn[q]);
    key.push_back(jk[q]);
    n += jn[q];
  }
  key.push_back(ctx->tm_finish_max);
  int slot = -1;
  for (int s = 0; s < 2; ++s)
    if (ctx->tm_plan[s] && ctx->tm_plan[s]->key == key) slot = s;
  if (slot < 0) {
    slot = !ctx->tm_plan[0] ? 0 : (!ctx->tm_plan[1] ? 1 : (ctx->tm_plan_used[0] <= ctx->tm_plan_used[1] ? 0 : 1));
    // the replaced plan's tables may still be read by queued work
    KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    tm_plan_free(ctx->tm_plan[slot]);
    ctx->tm_plan[slot] = new TMPlan();
    build_plan(*ctx->tm_plan[slot], jn, jk, ctx->tm_finish_max);
    KNNKM_TRY(upload_plan(ctx, *ctx->tm_plan[slot], slot == 0 ? "tm_plan0" : "tm_plan1"));
  }
  ctx->tm_plan_used[slot] = ++ctx->tm_plan_clock;
  const TMPlan& P = *ctx->tm_plan[slot];
  const int32_t k = P.k;
  if (d > KNNKM_MAX_D) return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "twomeans: d=%d > %d", d, KNNKM_MAX_D);
  int gL, gV;
  pick_group(d, 1, &gL, &gV);
  const bool vec = (d % 4 == 0) && (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
  KNNKM_WS(ctx, permbuf, int32_t, "tm_perm", 2 * n);
  KNNKM_WS(ctx, keys, uint64_t, "tm_keys", n);
  KNNKM_WS(ctx, cent, float, "tm_cent", (int64_t)std::max(1, P.max_split) * 2 * d);
  KNNKM_WS(ctx, partial, double, "tm_partial", (int64_t)std::max(1, P.max_tiles) * 2 * d);
  KNNKM_WS(ctx, pcnt, int32_t, "tm_pcnt", (int64_t)std::max(1, P.max_tiles) * 2);
  KNNKM_WS(ctx, sel, SelState, "tm_sel", (int64_t)std::max(1, P.max_big) * (TM_SEL_PASSES + 1));
  KNNKM_WS(ctx, hist, int32_t, "tm_hist", (int64_t)std::max(1, P.max_big) * 256 * TM_SEL_PASSES);
  KNNKM_WS(ctx, tless, int32_t, "tm_tless", std::max(1, P.max_tiles));
  KNNKM_WS(ctx, ttie, int32_t, "tm_ttie", std::max(1, P.max_tiles));
  KNNKM_WS(ctx, cpart, double, "tm_cpart", (int64_t)std::max(1, P.max_chunks) * 2 * d);
  KNNKM_WS(ctx, ccnt, int32_t, "tm_ccnt", (int64_t)std::max(1, P.max_chunks) * 2);
  int32_t* perm = permbuf;
  int32_t* perm_next = permbuf + n;
  k_iota<<<grid_for(n, 256, 4096), 256, 0, ctx->stream>>>(perm, n);
  KNNKM_TRY(knnkm_check(ctx, "twomeans iota"));
  for (const TMLevel& L : P.levels) {
    const int32_t* s_off = P.d_split_off + L.split_base;
    const int32_t* s_size = P.d_split_size + L.split_base;
    const unsigned gw = (unsigned)((L.nsplit + 3) / 4);
    if (L.nfin)
      TM_DISPATCH(launch_finish, ctx, P, L, X, d, ldx, perm, perm_next, seeds_dev, seed1, round_tag, iters,
                  vec);
    if (L.nsplit)
      k_tm_seed<<<gw, 256, 0, ctx->stream>>>(X, d, ldx, perm, L.nsplit, s_off, s_size,
                                             P.d_split_heap + L.split_base, P.d_split_job + L.split_base,
                                             seeds_dev, seed1, round_tag, cent);
    for (int it = 0; it < iters && L.nsplit; ++it) {
      TM_DISPATCH(launch_accum, ctx, P, L, X, d, ldx, perm, cent, partial, pcnt, vec);
      if (L.max_node_tiles > TM_CHUNK) {
        // nodes with many tiles: tiles -> chunks -> node, each stage in fixed order
        k_tm_chunk<<<dim3(L.nchunks, (2 * d + 63) / 64), 256, 0, ctx->stream>>>(
            d, P.d_chunk_tb + L.chunk_base, P.d_chunk_te + L.chunk_base, partial, pcnt, cpart, ccnt);
        k_tm_final<<<dim3(L.nsplit, (2 * d + 63) / 64), 256, 0, ctx->stream>>>(
            d, P.d_split_cb + L.split_base, P.d_split_ce + L.split_base, cpart, ccnt, cent);
      } else {
        k_tm_final<<<dim3(L.nsplit, (2 * d + 63) / 64), 256, 0, ctx->stream>>>(
            d, P.d_split_tile_begin + L.split_base, P.d_split_tile_end + L.split_base, partial, pcnt, cent);
      }
    }
    if (L.nsplit) TM_DISPATCH(launch_delta, ctx, P, L, X, d, ldx, perm, cent, keys, vec);
    KNNKM_TRY(knnkm_check(ctx, "twomeans level"));
    if (L.nsmall)
      k_tm_split_small<<<L.nsmall, 256, 0, ctx->stream>>>(perm, keys, P.d_small_split + L.small_base,
                                                          s_off, s_size, perm_next);
    if (L.nbig) {
      const int32_t* bt = P.d_bigtile + L.bigtile_base;
      const int32_t* btb = P.d_bigtile_big + L.bigtile_base;
      const int32_t* bs = P.d_big_split + L.big_base;
      const int32_t* ts = P.d_tile_start + L.tile_base;
      const int32_t* tl = P.d_tile_len + L.tile_base;
      k_tm_sel_init<<<grid_for((int64_t)L.nbig * 256 * TM_SEL_PASSES, 256, 4096), 256, 0, ctx->stream>>>(
          L.nbig, bs, s_size, sel, hist);
      for (int pass = 0; pass < TM_SEL_PASSES; ++pass)
        k_tm_sel_pass<<<L.nbigtiles, 256, 0, ctx->stream>>>(perm, keys, bt, btb, P.d_big_btb + L.big_base, ts, tl,
                                                            pass, L.nbig, sel, hist);
      k_tm_part_count<<<L.nbigtiles, 256, 0, ctx->stream>>>(keys, bt, btb, P.d_big_btb + L.big_base, ts, tl,
                                                            L.nbig, sel, hist, tless, ttie);
      k_tm_part_scan<<<L.nbig, 256, 0, ctx->stream>>>(P.d_big_btb + L.big_base, P.d_big_bte + L.big_base,
                                                      tless, ttie);
      k_tm_part_write<<<L.nbigtiles, 256, 0, ctx->stream>>>(perm, keys, bt, btb, bs, s_off, s_size, ts, tl,
                                                            sel + (int64_t)TM_SEL_PASSES * L.nbig, tless, ttie,
                                                            perm_next);
    }
    if (L.ncopy)
      k_tm_copy<<<L.ncopy, 256, 0, ctx->stream>>>(perm, P.d_copy_off + L.copy_base,
                                                  P.d_copy_size + L.copy_base, perm_next);
    KNNKM_TRY(knnkm_check(ctx, "twomeans split"));
    std::swap(perm, perm_next);
  }
  k_tm_labels<<<grid_for(k, 1, 65536), 256, 0, ctx->stream>>>(perm, P.d_leaf_off, k, labels);
  return knnkm_check(ctx, "twomeans labels");
}

knnkm_status ks_twomeans(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                         int32_t k, uint64_t seed, int32_t round_tag, int32_t iters,
                         int32_t* labels) {
  return ks_twomeans_multi(ctx, X, d, ldx, std::vector<int64_t>{n}, std::vector<int32_t>{k}, nullptr, seed,
                           round_tag, iters, labels);
}

extern "C" knnkm_status knnkm_twomeans(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d,
                                       int64_t ldx, int32_t k, uint64_t seed, int32_t round_tag,
                                       int32_t bisect_iters, int32_t* labels) {
  if (!ctx) return KNNKM_EINVAL;
  if (ctx->sticky) return KNNKM_EDEVICE;
  if (!X || !labels) return knnkm_fail(ctx, KNNKM_EINVAL, "twomeans: null pointer");
  if (n < 1 || n > INT32_MAX) return knnkm_fail(ctx, KNNKM_EINVAL, "twomeans: n out of range");
  if (d < 1 || ldx < d) return knnkm_fail(ctx, KNNKM_EINVAL, "twomeans: need d >= 1 and ldx >= d");
  if (d > KNNKM_MAX_D) return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "twomeans: d=%d > %d", d, KNNKM_MAX_D);
  if (k < 1 || k > n) return knnkm_fail(ctx, KNNKM_EINVAL, "twomeans: need 1 <= k <= n");
  if (bisect_iters < 0) return knnkm_fail(ctx, KNNKM_EINVAL, "twomeans: bisect_iters < 0");
  if (round_tag < 0 || round_tag > 0xFFFF) return knnkm_fail(ctx, KNNKM_EINVAL, "twomeans: round_tag");
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  return ks_twomeans(ctx, X, n, d, ldx, k, seed, round_tag, bisect_iters, labels);
}

extern "C" knnkm_status knnkm_enable_subtree_finish(knnkm_ctx* ctx, int32_t on) {
  if (!ctx) return KNNKM_EINVAL;
  if (on < 0 || on > TM_TILE)
    return knnkm_fail(ctx, KNNKM_EINVAL, "subtree finish: %d is not 0, 1 or a root size 2..%d", on, TM_TILE);
  ctx->tm_finish_max = on == 1 ? TM_FINISH_DEFAULT : on;
  return KNNKM_OK;
}
