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
//             find the threshold by a 12-digit radix select over the 96-bit
//             (delta key, id) and partition tile by tile
// Leaves are numbered left to right.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "rowgroup.h"

#define TM_TILE 1024    // positions per tile of the per-member passes
#define TM_SMALL 2048   // nodes up to this size split inside one block
#define TM_CHUNK 16     // tiles per chunk of the two-stage node reduction

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
  int max_split = 0, max_tiles = 0, max_big = 0, max_chunks = 0;
  // device copies
  void* dev = nullptr;
  size_t dev_bytes = 0;
  const int32_t *d_split_off, *d_split_size, *d_split_tile_begin, *d_split_tile_end, *d_tile_split,
      *d_tile_start, *d_tile_len, *d_big_split, *d_bigtile, *d_bigtile_big, *d_small_split,
      *d_copy_off, *d_copy_size, *d_leaf_off, *d_big_btb, *d_big_bte, *d_split_cb, *d_split_ce,
      *d_chunk_tb, *d_chunk_te, *d_split_job;
  const int64_t* d_split_heap;
};

// The device tables live in the context workspace ("tm_plan").
void tm_plan_free(TMPlan* p) { delete p; }

// Tree shapes of several independent jobs (job j: rows [off_j, off_j + n_j),
// k_j leaves), merged depth by depth so one launch per step covers every job
// that still splits; a job whose tree is complete is carried over as a copy.
static void build_plan(TMPlan& P, const std::vector<int64_t>& jn, const std::vector<int32_t>& jk) {
  P = TMPlan();
  const int nj = (int)jn.size();
  P.key.clear();
  int64_t total = 0;
  for (int q = 0; q < nj; ++q) {
    P.key.push_back(jn[q]);
    P.key.push_back(jk[q]);
    total += jn[q];
  }
  P.n = total;
  std::vector<std::vector<int64_t>> joff(nj), jsize(nj);
  {
    int64_t at = 0;
    for (int q = 0; q < nj; ++q) {
      joff[q] = {at};
      jsize[q] = {jn[q]};
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
    L.max_node_tiles = 0;
    for (int q = 0; q < nj; ++q) {
    std::vector<int64_t>& off = joff[q];
    std::vector<int64_t>& size = jsize[q];
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
    for (int i = 0; i < m; ++i) {
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
      } else {
        P.copy_off.push_back((int32_t)off[i]);
        P.copy_size.push_back((int32_t)size[i]);
        noff.push_back(off[i]);
        nsize.push_back(size[i]);
      }
    }
    off.swap(noff);
    size.swap(nsize);
    }
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
  // leaves of all jobs, left to right, job after job
  P.leaf_off.clear();
  for (int q = 0; q < nj; ++q)
    for (int64_t v : joff[q]) P.leaf_off.push_back((int32_t)v);
  P.k = (int32_t)P.leaf_off.size();
  P.leaf_off.push_back((int32_t)total);
}

static knnkm_status upload_plan(knnkm_ctx* ctx, TMPlan& P) {
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
      {P.split_job.data(), P.split_job.size() * 4}};
  size_t total = 0;
  std::vector<size_t> at;
  for (auto& p : parts) {
    total = (total + 15) & ~(size_t)15;
    at.push_back(total);
    total += p.second;
  }
  total += 16;
  P.dev = knnkm_ws(ctx, "tm_plan", total);
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
  for (int p = gid; p < len; p += NG) {
    float x[V];
    load_row<V>(x, X + (int64_t)perm[start + p] * ldx, j, d, vec);
    const double delta = group_sum<L>(tm_part<V>(x, wv, sv));
    if (delta <= 0.0) {
      ++cnu;
#pragma unroll
      for (int e = 0; e < V; ++e) au[e] += (double)x[e];
    } else {
      ++cnv;
#pragma unroll
      for (int e = 0; e < V; ++e) av[e] += (double)x[e];
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

// Partial sums of the entries [tb, te) of `src` in a fixed order: wave w adds
// entries w, w+4, ... in order into sh[w][.] and its counts into shc[w][.];
// callers add the four wave sums in wave order.
__device__ void tm_sum_range(int d, int tb, int te, const double* __restrict__ src,
                             const int32_t* __restrict__ scnt, double* sh /*[4][2d]*/, int32_t* shc /*[4][2]*/) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int e = lane; e < 2 * d; e += 64) {
    double s = 0.0;
    for (int t = tb + w; t < te; t += 4) s += src[(int64_t)t * 2 * d + e];
    sh[w * 2 * d + e] = s;
  }
  if (lane == 0) {
    int nu = 0, nv = 0;
    for (int t = tb + w; t < te; t += 4) {
      nu += scnt[2 * t];
      nv += scnt[2 * t + 1];
    }
    shc[2 * w] = nu;
    shc[2 * w + 1] = nv;
  }
  __syncthreads();
}

// One block per chunk of tiles: chunk partial = ordered sum of its tiles.
__global__ __launch_bounds__(256) void k_tm_chunk(int d, const int32_t* __restrict__ c_tb,
                                                  const int32_t* __restrict__ c_te,
                                                  const double* __restrict__ partial,
                                                  const int32_t* __restrict__ pcnt,
                                                  double* __restrict__ cpart, int32_t* __restrict__ ccnt) {
  __shared__ double sh[4 * 2 * KNNKM_MAX_D];
  __shared__ int32_t shc[8];
  const int c = blockIdx.x;
  tm_sum_range(d, c_tb[c], c_te[c], partial, pcnt, sh, shc);
  for (int e = threadIdx.x; e < 2 * d; e += 256)
    cpart[(int64_t)c * 2 * d + e] = ((sh[e] + sh[2 * d + e]) + sh[4 * d + e]) + sh[6 * d + e];
  if (threadIdx.x < 2)
    ccnt[2 * c + threadIdx.x] = shc[threadIdx.x] + shc[2 + threadIdx.x] + shc[4 + threadIdx.x] + shc[6 + threadIdx.x];
}

// One block per split node: new centroids from its partials (tiles, or
// chunks of tiles for nodes with many tiles), added in a fixed order.
__global__ __launch_bounds__(256) void k_tm_final(int d, const int32_t* __restrict__ s_tb,
                                                  const int32_t* __restrict__ s_te,
                                                  const double* __restrict__ partial,
                                                  const int32_t* __restrict__ pcnt,
                                                  float* __restrict__ cent) {
  __shared__ double sh[4 * 2 * KNNKM_MAX_D];
  __shared__ int32_t shc[8];
  const int js = blockIdx.x;
  tm_sum_range(d, s_tb[js], s_te[js], partial, pcnt, sh, shc);
  const int cu_n = shc[0] + shc[2] + shc[4] + shc[6];
  const int cv_n = shc[1] + shc[3] + shc[5] + shc[7];
  for (int e = threadIdx.x; e < 2 * d; e += 256) {
    const double s = ((sh[e] + sh[2 * d + e]) + sh[4 * d + e]) + sh[6 * d + e];
    const int cnt = e < d ? cu_n : cv_n;
    if (cnt > 0) cent[(int64_t)js * 2 * d + e] = (float)(s / (double)cnt);
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
  for (int p = gid; p < len; p += NG) {
    float x[V];
    load_row<V>(x, X + (int64_t)perm[start + p] * ldx, j, d, vec);
    const double delta = group_sum<L>(tm_part<V>(x, wv, sv));
    if (j == 0) keys[start + p] = dkey(delta);
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

// Radix select over 96-bit (key, id) for nodes larger than one tile.
struct SelState {
  uint64_t pk;  // decided high bits of the key
  uint32_t pi;  // decided high bits of the id
  int32_t h;    // rank still to find inside the current bucket (1-based)
};

__device__ inline int sel_digit(uint64_t key, int32_t id, int pass) {
  if (pass < 8) return (int)((key >> (56 - 8 * pass)) & 255);
  return (int)(((uint32_t)id >> (24 - 8 * (pass - 8))) & 255);
}
__device__ inline bool sel_match(uint64_t key, int32_t id, int pass, const SelState& st) {
  if (pass == 0) return true;
  if (pass <= 8) {
    const int sh = 64 - 8 * pass;
    return (key >> sh) == (st.pk >> sh);
  }
  if (key != st.pk) return false;
  const int sh = 32 - 8 * (pass - 8);
  return ((uint32_t)id >> sh) == (st.pi >> sh);
}

__global__ __launch_bounds__(256) void k_tm_sel_init(int nbig, const int32_t* __restrict__ big_split,
                                                     const int32_t* __restrict__ s_size,
                                                     SelState* st, int32_t* hist) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nbig; b += gridDim.x * blockDim.x) {
    st[b].pk = 0;
    st[b].pi = 0;
    st[b].h = (s_size[big_split[b]] + 1) / 2;
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nbig * 256; e += gridDim.x * blockDim.x)
    hist[e] = 0;
}

__global__ __launch_bounds__(256) void k_tm_sel_hist(const int32_t* __restrict__ perm,
                                                     const uint64_t* __restrict__ keys,
                                                     const int32_t* __restrict__ bigtile,
                                                     const int32_t* __restrict__ bigtile_big,
                                                     const int32_t* __restrict__ t_start,
                                                     const int32_t* __restrict__ t_len, int pass,
                                                     const SelState* __restrict__ st,
                                                     int32_t* __restrict__ hist) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int tile = bigtile[blockIdx.x];
  const int b = bigtile_big[blockIdx.x];
  const SelState s = st[b];
  const int start = t_start[tile], len = t_len[tile];
  for (int p = threadIdx.x; p < len; p += 256) {
    const uint64_t key = keys[start + p];
    const int32_t id = perm[start + p];
    if (sel_match(key, id, pass, s)) atomicAdd(&h[sel_digit(key, id, pass)], 1);
  }
  __syncthreads();
  const int c = h[threadIdx.x];
  if (c) atomicAdd(&hist[b * 256 + threadIdx.x], c);
}

// One 256-thread block per big node: the bucket holding the rank-h element is
// the digit whose exclusive prefix count is < h <= inclusive count.
__global__ __launch_bounds__(256) void k_tm_sel_pick(int pass, SelState* st, int32_t* hist) {
  __shared__ int32_t sh[8];
  const int b = blockIdx.x;
  int32_t* hh = hist + b * 256;
  const int32_t c = hh[threadIdx.x];
  const SelState s = st[b];
  int32_t tot;
  const int32_t ex = block_scan_excl_256(c, sh, &tot);
  if (c > 0 && ex < s.h && s.h <= ex + c) {
    SelState t = s;
    t.h -= ex;
    const int dg = threadIdx.x;
    if (pass < 8)
      t.pk |= (uint64_t)dg << (56 - 8 * pass);
    else
      t.pi |= (uint32_t)dg << (24 - 8 * (pass - 8));
    st[b] = t;
  }
  hh[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_tm_part_count(const int32_t* __restrict__ perm,
                                                       const uint64_t* __restrict__ keys,
                                                       const int32_t* __restrict__ bigtile,
                                                       const int32_t* __restrict__ bigtile_big,
                                                       const int32_t* __restrict__ t_start,
                                                       const int32_t* __restrict__ t_len,
                                                       const SelState* __restrict__ st,
                                                       int32_t* __restrict__ tile_left) {
  __shared__ int32_t c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  const int tile = bigtile[blockIdx.x];
  const SelState s = st[bigtile_big[blockIdx.x]];
  const int start = t_start[tile], len = t_len[tile];
  int mine = 0;
  for (int p = threadIdx.x; p < len; p += 256)
    mine += kv_le(keys[start + p], perm[start + p], s.pk, (int32_t)s.pi) ? 1 : 0;
  atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) tile_left[blockIdx.x] = c;
}

// Exclusive scan of the left counts over the tiles of each big node.
// One block per big node: exclusive scan of the left counts of its tiles.
__global__ __launch_bounds__(256) void k_tm_part_scan(const int32_t* __restrict__ big_btb,
                                                      const int32_t* __restrict__ big_bte,
                                                      int32_t* __restrict__ tile_left) {
  __shared__ int32_t sh[8];
  const int b = blockIdx.x;
  const int tb = big_btb[b], te = big_bte[b];
  int32_t carry = 0;
  for (int base = tb; base < te; base += 256) {
    const int t = base + threadIdx.x;
    const int32_t c = t < te ? tile_left[t] : 0;
    int32_t tot;
    const int32_t ex = block_scan_excl_256(c, sh, &tot);
    if (t < te) tile_left[t] = carry + ex;
    carry += tot;
  }
}

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
                                                       const int32_t* __restrict__ tile_left_base,
                                                       int32_t* __restrict__ perm_out) {
  __shared__ int32_t sh_scan[256];
  const int tile = bigtile[blockIdx.x];
  const int b = bigtile_big[blockIdx.x];
  const SelState s = st[b];
  const int j = big_split[b];
  const int off = s_off[j], h = (s_size[j] + 1) / 2;
  const int start = t_start[tile], len = t_len[tile];
  const int per = (len + 255) / 256;
  const int p0 = start + threadIdx.x * per;
  const int p1 = min(start + len, p0 + per);
  int cnt = 0;
  for (int p = p0; p < p1; ++p) cnt += kv_le(keys[p], perm[p], s.pk, (int32_t)s.pi) ? 1 : 0;
  sh_scan[threadIdx.x] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int e = 0; e < 256; ++e) {
      int c = sh_scan[e];
      sh_scan[e] = run;
      run += c;
    }
  }
  __syncthreads();
  const int lefts_before = tile_left_base[blockIdx.x] + sh_scan[threadIdx.x];
  int lpos = off + lefts_before;
  int rpos = off + h + ((p0 - off) - lefts_before);
  for (int p = p0; p < p1; ++p) {
    const int32_t id = perm[p];
    if (kv_le(keys[p], id, s.pk, (int32_t)s.pi))
      perm_out[lpos++] = id;
    else
      perm_out[rpos++] = id;
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
  if (!ctx->tm_plan || ctx->tm_plan->key != key) {
    KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    tm_plan_free(ctx->tm_plan);
    ctx->tm_plan = new TMPlan();
    build_plan(*ctx->tm_plan, jn, jk);
    KNNKM_TRY(upload_plan(ctx, *ctx->tm_plan));
  }
  const TMPlan& P = *ctx->tm_plan;
  const int32_t k = P.k;
  if (d > KNNKM_MAX_D) return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "twomeans: d=%d > %d", d, KNNKM_MAX_D);
  int gL, gV;
  pick_group(d, 1, &gL, &gV);
  const bool vec = (d % 4 == 0) && (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
  KNNKM_WS(ctx, permbuf, int32_t, "tm_perm", 2 * n);
  KNNKM_WS(ctx, keys, uint64_t, "tm_keys", n);
  KNNKM_WS(ctx, cent, float, "tm_cent", (int64_t)P.max_split * 2 * d);
  KNNKM_WS(ctx, partial, double, "tm_partial", (int64_t)P.max_tiles * 2 * d);
  KNNKM_WS(ctx, pcnt, int32_t, "tm_pcnt", (int64_t)P.max_tiles * 2);
  KNNKM_WS(ctx, sel, SelState, "tm_sel", std::max(1, P.max_big));
  KNNKM_WS(ctx, hist, int32_t, "tm_hist", (int64_t)std::max(1, P.max_big) * 256);
  KNNKM_WS(ctx, tleft, int32_t, "tm_tleft", std::max(1, P.max_tiles));
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
    if (L.nsplit)
      k_tm_seed<<<gw, 256, 0, ctx->stream>>>(X, d, ldx, perm, L.nsplit, s_off, s_size,
                                             P.d_split_heap + L.split_base, P.d_split_job + L.split_base,
                                             seeds_dev, seed1, round_tag, cent);
    for (int it = 0; it < iters; ++it) {
      TM_DISPATCH(launch_accum, ctx, P, L, X, d, ldx, perm, cent, partial, pcnt, vec);
      if (L.max_node_tiles > TM_CHUNK) {
        // nodes with many tiles: tiles -> chunks -> node, each stage in fixed order
        k_tm_chunk<<<L.nchunks, 256, 0, ctx->stream>>>(d, P.d_chunk_tb + L.chunk_base,
                                                       P.d_chunk_te + L.chunk_base, partial, pcnt, cpart,
                                                       ccnt);
        k_tm_final<<<L.nsplit, 256, 0, ctx->stream>>>(d, P.d_split_cb + L.split_base,
                                                      P.d_split_ce + L.split_base, cpart, ccnt, cent);
      } else {
        k_tm_final<<<L.nsplit, 256, 0, ctx->stream>>>(d, P.d_split_tile_begin + L.split_base,
                                                      P.d_split_tile_end + L.split_base, partial, pcnt,
                                                      cent);
      }
    }
    TM_DISPATCH(launch_delta, ctx, P, L, X, d, ldx, perm, cent, keys, vec);
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
      k_tm_sel_init<<<grid_for((int64_t)L.nbig * 256, 256, 1024), 256, 0, ctx->stream>>>(L.nbig, bs, s_size,
                                                                                    sel, hist);
      for (int pass = 0; pass < 12; ++pass) {
        k_tm_sel_hist<<<L.nbigtiles, 256, 0, ctx->stream>>>(perm, keys, bt, btb, ts, tl, pass, sel, hist);
        k_tm_sel_pick<<<L.nbig, 256, 0, ctx->stream>>>(pass, sel, hist);
      }
      k_tm_part_count<<<L.nbigtiles, 256, 0, ctx->stream>>>(perm, keys, bt, btb, ts, tl, sel, tleft);
      k_tm_part_scan<<<L.nbig, 256, 0, ctx->stream>>>(P.d_big_btb + L.big_base, P.d_big_bte + L.big_base,
                                                      tleft);
      k_tm_part_write<<<L.nbigtiles, 256, 0, ctx->stream>>>(perm, keys, bt, btb, bs, s_off, s_size, ts, tl,
                                                            sel, tleft, perm_next);
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
