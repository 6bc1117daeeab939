// KNN graph construction pieces (Alg. 3).
//
// graph_init: random initial lists.  One wavefront per row: Floyd's sampling
//   of kappa distinct values of [0, n-1) (one counter-based draw per step,
//   membership by ballot over the lanes that hold the chosen ids), shifted
//   past the row's own id; squared distances in float64 (rounded to float32);
//   the row is ordered by (d2, id) through per-lane ranks.
//
// refine: the exhaustive comparison inside every cluster and the list
//   update.  A cluster of at most 64 members (32 when d is large) is one tile
//   handled by one 512-thread block:
//     1. the samples are staged in LDS (float32, 16-byte aligned rows);
//     2. the Gram block runs on MFMA (float32 16x16x4, or bfloat16 16x16x32
//        in the precision form), 16 x 16 tiles spread over the 8 waves;
//     3. d^2 estimates ||x||^2 + ||y||^2 - 2 x.y minus a rigorous error bound
//        are compared with the row's current kappa-th distance; survivors go
//        to a compact list;
//     4. survivors get their exact distance (float64 direct difference from
//        LDS by row groups, rounded to float32);
//     5. each row (one wave) drops survivors already in its list (visited
//        pairs) and merges the rest by per-lane ranks, writing the graph row.
//   Clusters larger than a tile and of at most 128 members get the exact
//   distances of all their pairs (refine_exact.hip); larger ones go through a
//   screen over 64 x 64 member blocks and a per-row merge (below); clusters
//   too large for that item count fall back to row blocks walking the
//   cluster's column blocks.  Every row belongs to
//   exactly one cluster, so rows are updated without atomics.  Both precisions
//   produce the same graph: the screen only removes pairs that provably cannot
//   enter, and a row's result is the kappa smallest (d2, id) of its old list
//   and its cluster, independent of the order in which pairs are examined.
#include <cfloat>

#include "merge.h"
#include "rowgroup.h"

// ------------------------------------------------------------- graph init --
template <int T>
__global__ __launch_bounds__(256) void k_graph_init(const float* __restrict__ X, int n, int d,
                                                    int64_t ldx, int kappa, uint64_t seed,
                                                    int32_t* __restrict__ G_ids,
                                                    float* __restrict__ G_d2,
                                                    const int32_t* __restrict__ job_of,
                                                    const int64_t* __restrict__ n_off,
                                                    const uint64_t* __restrict__ seeds) {
  const int lane = threadIdx.x & 63;
  const int64_t gi_row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gi_row >= n) return;
  // job-local view: rows [row0, row0 + nj) with the job's own seed
  int64_t row0 = 0, nj = n;
  uint64_t jseed = seed;
  if (job_of) {
    const int q = job_of[gi_row];
    row0 = n_off[q];
    nj = n_off[q + 1] - row0;
    jseed = seeds[q];
  }
  const int64_t i = gi_row - row0;
  const uint64_t key = sm_key(jseed, sm_stream(RNG_GRAPH_INIT, 0, (uint64_t)i));
  const uint32_t m = (uint32_t)(nj - 1);
  const uint32_t fbase = m - (uint32_t)kappa;
  int v0 = -1, v1 = -1;  // chosen value for slot lane, lane+64
  for (int c = 0; c < kappa; ++c) {
    const uint32_t j = fbase + (uint32_t)c;
    const int t = (int)sm_below(sm_draw(key, (uint64_t)c), j + 1);
    const bool seen = (__ballot(v0 == t) | __ballot(v1 == t)) != 0ull;
    const int v = seen ? (int)j : t;
    if (c < 64) {
      if (lane == c) v0 = v;
    } else if (lane == c - 64) {
      v1 = v;
    }
  }
  // shift past the row's own id, then to global ids
  int id0 = v0 >= 0 ? (int)(v0 + (v0 >= i ? 1 : 0) + row0) : -1;
  int id1 = v1 >= 0 ? (int)(v1 + (v1 >= i ? 1 : 0) + row0) : -1;
  // distances: one float64 reduction per entry
  float x[T];
  const float* xr = X + gi_row * ldx;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    int dim = lane + 64 * t;
    x[t] = dim < d ? xr[dim] : 0.f;
  }
  float k0 = FLT_MAX, k1 = FLT_MAX;
  for (int c = 0; c < kappa; ++c) {
    const int j = c < 64 ? __builtin_amdgcn_readlane(id0, c) : __builtin_amdgcn_readlane(id1, c - 64);
    const float* yr = X + (int64_t)j * ldx;
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      int dim = lane + 64 * t;
      if (dim < d) {
        double df = (double)x[t] - (double)yr[dim];
        acc = fma(df, df, acc);
      }
    }
    const float kv = (float)wave_sum(acc);
    if (c < 64) {
      if (lane == c) k0 = kv;
    } else if (lane == c - 64) {
      k1 = kv;
    }
  }
  // ranks by (key, id)
  int r0 = 0, r1 = 0;
  for (int c = 0; c < kappa; ++c) {
    float kc;
    int ic;
    if (c < 64) {
      kc = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(k0), c));
      ic = __builtin_amdgcn_readlane(id0, c);
    } else {
      kc = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(k1), c - 64));
      ic = __builtin_amdgcn_readlane(id1, c - 64);
    }
    r0 += (kc < k0 || (kc == k0 && ic < id0)) ? 1 : 0;
    r1 += (kc < k1 || (kc == k1 && ic < id1)) ? 1 : 0;
  }
  int32_t* gi = G_ids + gi_row * kappa;
  float* gd = G_d2 + gi_row * kappa;
  if (lane < kappa) {
    gi[r0] = id0;
    gd[r0] = k0;
  }
  if (lane + 64 < kappa) {
    gi[r1] = id1;
    gd[r1] = k1;
  }
}

knnkm_status ks_graph_init(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                           int32_t kappa, uint64_t seed, int32_t* G_ids, float* G_d2,
                           const int32_t* job_of, const int64_t* n_off, const uint64_t* seeds) {
  const int T = (d + 63) / 64;
  const unsigned grid = (unsigned)((n + 3) / 4);
#define GI(TT)                                                                                    \
  k_graph_init<TT><<<grid, 256, 0, ctx->stream>>>(X, (int)n, d, ldx, kappa, seed, G_ids, G_d2, job_of, \
                                                  n_off, seeds)
  switch (T) {
    case 1: GI(1); break;
    case 2: GI(2); break;
    case 3: GI(3); break;
    case 4: GI(4); break;
    case 5: GI(5); break;
    case 6: GI(6); break;
    case 7: GI(7); break;
    case 8: GI(8); break;
    default: return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "graph_init: d=%d > %d", d, KNNKM_MAX_D);
  }
#undef GI
  return knnkm_check(ctx, "graph_init");
}

// ----------------------------------------------------------------- refine --
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

__device__ inline bool key_lt(float ka, int ia, float kb, int ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// LDS layout of a refine tile (byte offsets, regions laid end to end):
//   xi [RB][ld] float rows, xj [RB][ld] (the same region when `single`),
//   km [RB][RB] float exact keys, ni/nj/thr [RB] float, ids_i/ids_j [RB] int,
//   pcount [4] int, plist [RB*RB] uint16 survivors, rk/ri [RB][kappa] the
//   graph rows of the block (float keys, int ids), mh [8][MG_SLOTS] int the
//   merge's id tables (one per wavefront).
struct TileLayout {
  int ld;
  size_t xi, xj, km, ni, nj, thr, ids_i, ids_j, pcount, plist, rk, ri, mh, bytes;
  __host__ __device__ TileLayout(int RB, int dpad, bool single, int kappa) {
    ld = dpad + 4;  // 16-byte aligned rows
    const size_t rows = (size_t)RB * ld * 4;
    size_t at = 0;
    xi = at;
    at += rows;
    xj = single ? xi : at;
    if (!single) at += rows;
    km = at;
    at += (size_t)RB * RB * 4;
    ni = at;
    at += (size_t)RB * 4;
    nj = single ? ni : at;
    if (!single) at += (size_t)RB * 4;
    thr = at;
    at += (size_t)RB * 4;
    ids_i = at;
    at += (size_t)RB * 4;
    ids_j = at;
    at += (size_t)RB * 4;
    pcount = at;
    at += 16;
    plist = at;
    at += (size_t)RB * RB * 2;
    at = (at + 15) & ~(size_t)15;
    rk = at;
    at += (size_t)RB * kappa * 4;
    ri = at;
    at += (size_t)RB * kappa * 4;
    mh = at;
    at += (size_t)8 * MG_SLOTS * 4;
    bytes = at;
  }
};

// Stage rows [r0, r0 + nr) of a cluster (members c0 + r) into LDS, zero
// padded to RB rows of dpad floats.
template <int RB>
__device__ inline void stage_rows(float* __restrict__ xs, int ld, const float* __restrict__ X, int64_t ldx,
                                  const int32_t* __restrict__ members, int c0, int r0, int nr, int d,
                                  int dpad, bool vec) {
  const int q4 = dpad / 4;
  for (int e = threadIdx.x; e < RB * q4; e += blockDim.x) {
    const int r = e / q4, t = 4 * (e % q4);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r < nr) {
      const float* row = X + (int64_t)members[c0 + r0 + r] * ldx;
      if (vec && t < d) {
        v = *reinterpret_cast<const float4*>(row + t);
      } else {
        v.x = t < d ? row[t] : 0.f;
        v.y = t + 1 < d ? row[t + 1] : 0.f;
        v.z = t + 2 < d ? row[t + 2] : 0.f;
        v.w = t + 3 < d ? row[t + 3] : 0.f;
      }
    }
    *reinterpret_cast<float4*>(xs + r * ld + t) = v;
  }
}

// Lane j of a row group reads the staged row in float4 chunks j, j + L, ...
// (consecutive lanes, consecutive 16 bytes: no LDS bank conflicts).
template <int L, int V>
__device__ inline float4 row_chunk(const float* __restrict__ row, int j, int u, int dpad) {
  const int c = 4 * (j + L * u);
  return c < dpad ? *reinterpret_cast<const float4*>(row + c) : make_float4(0.f, 0.f, 0.f, 0.f);
}

// float32 squared norms of RB staged rows, one row group per row.
template <int RB, int L, int V>
__device__ inline void row_norms(const float* __restrict__ xs, int ld, int dpad, float* __restrict__ nrm) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NG = 512 / L;
  const int j = lane % L, gid = w * (64 / L) + lane / L;
  for (int r = gid; r < RB; r += NG) {
    float a = 0.f;
#pragma unroll
    for (int u = 0; u < V / 4; ++u) {
      const float4 v = row_chunk<L, V>(xs + r * ld, j, u, dpad);
      a = fmaf(v.x, v.x, a);
      a = fmaf(v.y, v.y, a);
      a = fmaf(v.z, v.z, a);
      a = fmaf(v.w, v.w, a);
    }
    a = group_sum<L>(a);
    if (j == 0) nrm[r] = a;
  }
}

// Exhaustive comparison inside clusters (Alg. 3 inner loops), one block of
// 512 threads per (cluster, block of RB rows).  SINGLE: the whole cluster
// (2 <= s <= RB) is one tile, its rows serve as both sides of the Gram block.
// Otherwise (clusters too large for the screen items) the block walks the cluster's
// column blocks of RB members.  Per (row block, column block):
//   Gram on MFMA (16 x 16 tiles over 8 waves) -> screen against the rows'
//   current kappa-th distance with a rigorous margin -> survivor list ->
//   exact float64 squared distances (row groups) -> per-row merge (one wave
//   per row, lane c = candidate column c) written straight to the graph.
template <bool BF16, int L, int V, int RB, bool SINGLE>
__global__ __launch_bounds__(512) void k_refine_tile(const float* __restrict__ X, int d, int64_t ldx, int dpad,
                                                     int kappa, int32_t k, const int32_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ members,
                                                     const int32_t* __restrict__ wb_off, int64_t max_items,
                                                     int smin, float err_c, int vec, int32_t* __restrict__ G_ids,
                                                     float* __restrict__ G_d2) {
  extern __shared__ __align__(16) char smem[];
  const TileLayout lay(RB, dpad, SINGLE, kappa);
  const int ld = lay.ld;
  float* rk = (float*)(smem + lay.rk);
  int32_t* ri = (int32_t*)(smem + lay.ri);
  float* xi = (float*)(smem + lay.xi);
  float* xj = (float*)(smem + lay.xj);
  float* km = (float*)(smem + lay.km);
  float* ni = (float*)(smem + lay.ni);
  float* nj = (float*)(smem + lay.nj);
  float* thr = (float*)(smem + lay.thr);
  int32_t* ids_i = (int32_t*)(smem + lay.ids_i);
  int32_t* ids_j = (int32_t*)(smem + lay.ids_j);
  int32_t* pcount = (int32_t*)(smem + lay.pcount);
  uint16_t* plist = (uint16_t*)(smem + lay.plist);
  int32_t* mh = (int32_t*)(smem + lay.mh);

  int cl, i0, s;
  if (SINGLE) {
    cl = blockIdx.x;
    i0 = 0;
    s = offsets[cl + 1] - offsets[cl];
    if (s < 2 || s <= smin || s > RB) return;  // another launch takes clusters of <= smin
  } else {
    const int64_t item = blockIdx.x;
    if (item >= max_items || item >= wb_off[k]) return;
    int lo = 0, hi = k;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (wb_off[mid] <= item) lo = mid; else hi = mid;
    }
    cl = lo;
    s = offsets[cl + 1] - offsets[cl];
    i0 = (int)(item - wb_off[cl]) * RB;
  }
  const int c0 = offsets[cl];
  const int nrows = min(RB, s - i0);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int NG = 512 / L;
  const int j = lane % L, gid = w * (64 / L) + lane / L;

  if (tid < RB) {
    const int id = tid < nrows ? members[c0 + i0 + tid] : -1;
    ids_i[tid] = id;
    thr[tid] = tid < nrows ? G_d2[(int64_t)id * kappa + kappa - 1] : -FLT_MAX;
  }
  stage_rows<RB>(xi, ld, X, ldx, members, c0, i0, nrows, d, dpad, vec);
  for (int e = tid; e < 8 * MG_SLOTS; e += 512) mh[e] = -1;
  for (int e = tid; e < nrows * kappa; e += 512) {
    const int r = e / kappa, q = e % kappa;
    const int64_t g = (int64_t)members[c0 + i0 + r] * kappa + q;
    rk[e] = G_d2[g];
    ri[e] = G_ids[g];
  }
  __syncthreads();
  row_norms<RB, L, V>(xi, ld, dpad, ni);

  for (int j0 = 0; j0 < s; j0 += RB) {
    const int ncols = SINGLE ? nrows : min(RB, s - j0);
    if (!SINGLE) {
      if (tid < RB) ids_j[tid] = tid < ncols ? members[c0 + j0 + tid] : -1;
      stage_rows<RB>(xj, ld, X, ldx, members, c0, j0, ncols, d, dpad, vec);
    } else if (tid < RB) {
      ids_j[tid] = ids_i[tid];
    }
    for (int e = tid; e < RB * RB; e += 512) km[e] = FLT_MAX;
    if (tid == 0) pcount[0] = 0;
    __syncthreads();
    if (!SINGLE) {
      row_norms<RB, L, V>(xj, ld, dpad, nj);
      __syncthreads();
    }
    // Gram tiles and screen
    constexpr int TPS = RB / 16;
    for (int t = w; t < TPS * TPS; t += 8) {
      const int tr = 16 * (t / TPS), tc = 16 * (t % TPS);
      if (tr >= nrows || tc >= ncols) continue;  // wave-uniform
      f4_t acc = {0.f, 0.f, 0.f, 0.f};
      const float* ar = xi + (tr + (lane & 15)) * ld;
      const float* br = xj + (tc + (lane & 15)) * ld;
      if (BF16) {
        for (int k0 = 0; k0 < dpad; k0 += 32) {
          bf8_t a, b;
          const int kb = k0 + 8 * (lane >> 4);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            a[e] = (__bf16)ar[kb + e];
            b[e] = (__bf16)br[kb + e];
          }
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        }
      } else {
        for (int k0 = 0; k0 < dpad; k0 += 4) {
          const int kk = k0 + (lane >> 4);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[kk], br[kk], acc, 0, 0, 0);
        }
      }
      const int c = tc + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = tr + 4 * (lane >> 4) + e;
        if (r < nrows && c < ncols && ids_i[r] != ids_j[c]) {
          const float sn = ni[r] + nj[c];
          const float lb = sn - 2.f * acc[e] - err_c * sn;
          const float th = thr[r];
          if (lb <= th + th * 0x1p-22f + 1e-30f) plist[atomicAdd(pcount, 1)] = (uint16_t)(r * RB + c);
        }
      }
    }
    __syncthreads();
    // exact float64 distances of the survivors, one row group per pair
    const int np = pcount[0];
    for (int p = gid; p < np; p += NG) {
      const int rc = plist[p];
      const int r = rc / RB, c = rc % RB;
      double a = 0.0;
#pragma unroll
      for (int u = 0; u < V / 4; ++u) {
        const float4 p4 = row_chunk<L, V>(xi + r * ld, j, u, dpad);
        const float4 q4 = row_chunk<L, V>(xj + c * ld, j, u, dpad);
        double df = (double)p4.x - (double)q4.x;
        a = fma(df, df, a);
        df = (double)p4.y - (double)q4.y;
        a = fma(df, df, a);
        df = (double)p4.z - (double)q4.z;
        a = fma(df, df, a);
        df = (double)p4.w - (double)q4.w;
        a = fma(df, df, a);
      }
      a = group_sum<L>(a);
      if (j == 0) km[rc] = (float)a;
    }
    __syncthreads();
    // merge: one wave per row; lane c holds candidate column c
    for (int r = w; r < nrows; r += 8) {
      float* rowk = rk + r * kappa;
      int32_t* rowi = ri + r * kappa;
      const float ck[1] = {lane < RB ? km[r * RB + lane] : FLT_MAX};
      if (!__ballot(ck[0] < FLT_MAX)) continue;  // no survivor for this row
      const int cid[1] = {lane < RB ? ids_j[lane] : -1};
      const bool valid[1] = {ck[0] < FLT_MAX};
      const MergeRow old = merge_load(rowk, rowi, kappa);
      merge_row<1>(rowk, rowi, kappa, old, ck, cid, valid, mh + MG_SLOTS * w, thr + r);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
  }
  // write the block's rows back
  for (int e = tid; e < nrows * kappa; e += 512) {
    const int r = e / kappa, q = e % kappa;
    const int64_t g = (int64_t)ids_i[r] * kappa + q;
    G_d2[g] = rk[e];
    G_ids[g] = ri[e];
  }
}

// ------------------------------------------- large clusters: screen + merge --
// Clusters larger than one tile are processed in two kernels per round.
//  screen: one item per (cluster, row block I, column block J) of 64 x 64
//    members, taken by a persistent grid.  The Gram block is accumulated on
//    MFMA over 64-dimension slices staged in LDS; every pair whose lower bound
//    passes the row's kappa-th distance at the start of the round is appended
//    to the row's survivor slots (at most SC_CAP per row; a row with more
//    survivors is compared with its whole cluster by the merge).
//  merge: one wavefront per row with survivors: exact float64 distances of
//    the survivors not yet in the row, merged into the row by (d2, id).
// The merged row is the kappa smallest (d2, id) of the old row and the
// cluster, whatever the order in which survivors were found, so the graph is
// the same as with the one-block-per-tile kernel.
#define SC_RB 64   // rows and columns per item
#define SC_KC 64   // dimensions per staged slice
#define SC_LD (SC_KC + 4)
#define SC_CAP 64  // survivor slots per row and round

__global__ void k_screen_items(const int32_t* __restrict__ counts, int32_t k, int lo, int hi, int32_t* items) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < k;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int s = counts[r];
    const int t = (s + SC_RB - 1) / SC_RB;
    items[r] = (s > lo && s <= hi) ? t * t : 0;
  }
}

// float32 squared norms of all rows (the screening bound covers any
// summation order of the d products)
__global__ __launch_bounds__(256) void k_row_norms(const float* __restrict__ X, int64_t n, int d, int64_t ldx,
                                                   float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
    float a = 0.f;
    for (int t = lane; t < d; t += 64) a = fmaf(X[i * ldx + t], X[i * ldx + t], a);
    a = wave_sum(a);
    if (lane == 0) out[i] = a;
  }
}

template <bool BF16>
__global__ __launch_bounds__(256) void k_refine_screen(const float* __restrict__ X, int d, int64_t ldx, int dpad,
                                                       int kappa, int32_t k, const int32_t* __restrict__ offsets,
                                                       const int32_t* __restrict__ members,
                                                       const int32_t* __restrict__ item_off,
                                                       const float* __restrict__ nrm, float err_c, int vec,
                                                       const float* __restrict__ G_d2, int32_t* __restrict__ cnt,
                                                       int32_t* __restrict__ slots) {
  __shared__ __align__(16) float xi[SC_RB * SC_LD];
  __shared__ __align__(16) float xj[SC_RB * SC_LD];
  __shared__ int32_t ids_i[SC_RB], ids_j[SC_RB];
  __shared__ float thr[SC_RB], ni[SC_RB], nj[SC_RB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t total = item_off[k];
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    int lo = 0, hi = k;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (item_off[mid] <= item) lo = mid; else hi = mid;
    }
    const int cl = lo;
    const int c0 = offsets[cl], s = offsets[cl + 1] - c0;
    const int t = (s + SC_RB - 1) / SC_RB;
    const int local = (int)(item - item_off[cl]);
    const int i0 = (local / t) * SC_RB, j0 = (local % t) * SC_RB;
    const int nr = min(SC_RB, s - i0), nc = min(SC_RB, s - j0);
    __syncthreads();  // the previous item is done with the shared arrays
    if (tid < SC_RB) {
      const int id = tid < nr ? members[c0 + i0 + tid] : -1;
      ids_i[tid] = id;
      thr[tid] = id >= 0 ? G_d2[(int64_t)id * kappa + kappa - 1] : -FLT_MAX;
      ni[tid] = id >= 0 ? nrm[id] : 0.f;
    } else if (tid < 2 * SC_RB) {
      const int q = tid - SC_RB;
      const int id = q < nc ? members[c0 + j0 + q] : -1;
      ids_j[q] = id;
      nj[q] = id >= 0 ? nrm[id] : 0.f;
    }
    f4_t acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < dpad; k0 += SC_KC) {
      __syncthreads();
      // stage the slice [k0, k0 + SC_KC) of both row blocks (zero padded)
      for (int e = tid; e < 2 * SC_RB * (SC_KC / 4); e += 256) {
        const int side = e / (SC_RB * (SC_KC / 4));
        const int rem = e - side * (SC_RB * (SC_KC / 4));
        const int r = rem / (SC_KC / 4), c = 4 * (rem % (SC_KC / 4));
        const int id = side ? ids_j[r] : ids_i[r];
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        const int col = k0 + c;
        if (id >= 0) {
          const float* row = X + (int64_t)id * ldx;
          if (vec && col < d) {
            v = *reinterpret_cast<const float4*>(row + col);
          } else {
            v.x = col < d ? row[col] : 0.f;
            v.y = col + 1 < d ? row[col + 1] : 0.f;
            v.z = col + 2 < d ? row[col + 2] : 0.f;
            v.w = col + 3 < d ? row[col + 3] : 0.f;
          }
        }
        *reinterpret_cast<float4*>((side ? xj : xi) + r * SC_LD + c) = v;
      }
      __syncthreads();
      // wave w: tiles 16 x 16 of rows 16w..16w+15 and the 4 column tiles
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float* ar = xi + (16 * w + (lane & 15)) * SC_LD;
        const float* br = xj + (16 * q + (lane & 15)) * SC_LD;
        if (BF16) {
#pragma unroll
          for (int kk = 0; kk < SC_KC; kk += 32) {
            bf8_t a, b;
            const int kb = kk + 8 * (lane >> 4);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              a[e] = (__bf16)ar[kb + e];
              b[e] = (__bf16)br[kb + e];
            }
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
          }
        } else {
#pragma unroll
          for (int kk = 0; kk < SC_KC; kk += 4) {
            const int c = kk + (lane >> 4);
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[c], br[c], acc[q], 0, 0, 0);
          }
        }
      }
    }
    // screen: lane holds rows 16w + 4(lane>>4) + e of column 16q + (lane&15)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 16 * q + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * w + 4 * (lane >> 4) + e;
        if (r < nr && c < nc && ids_i[r] != ids_j[c]) {
          const float sn = ni[r] + nj[c];
          const float lb = sn - 2.f * acc[q][e] - err_c * sn;
          const float th = thr[r];
          if (lb <= th + th * 0x1p-22f + 1e-30f) {
            const int id = ids_i[r];
            const int slot = atomicAdd(&cnt[id], 1);
            if (slot < SC_CAP) slots[(int64_t)id * SC_CAP + slot] = ids_j[c];
          }
        }
      }
    }
  }
}

// One wavefront per row with survivors; exact distances of 64/L candidates
// at a time, one row group of L lanes each.
template <int L>
__global__ __launch_bounds__(256) void k_refine_merge(const float* __restrict__ X, int d, int64_t ldx, int kappa,
                                                      const int32_t* __restrict__ labels,
                                                      const int32_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ members, int64_t n,
                                                      const int32_t* __restrict__ cnt,
                                                      const int32_t* __restrict__ slots, int vec,
                                                      int32_t* __restrict__ G_ids, float* __restrict__ G_d2) {
  __shared__ float rks[4][KNNKM_MAX_KAPPA];
  __shared__ int32_t ris[4][KNNKM_MAX_KAPPA];
  __shared__ float kys[4][64];
  constexpr int G = 64 / L;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane / L, j = lane % L;
  float* rowk = rks[w];
  int32_t* rowi = ris[w];
  float* keys = kys[w];
  for (int64_t i = blockIdx.x * 4 + w; i < n; i += (int64_t)gridDim.x * 4) {
    const int c = cnt[i];
    if (c == 0) continue;  // wave-uniform
    for (int q = lane; q < kappa; q += 64) {
      rowk[q] = G_d2[i * kappa + q];
      rowi[q] = G_ids[i * kappa + q];
    }
    __builtin_amdgcn_wave_barrier();
    const bool over = c > SC_CAP;
    int64_t m0 = 0, total = c;
    if (over) {
      const int l = labels[i];
      m0 = offsets[l];
      total = offsets[l + 1] - m0;
    }
    const float* xr = X + i * ldx;
    bool changed = false;
    for (int64_t base = 0; base < total; base += 64) {
      const int64_t tt = base + lane;
      int cid = -1;
      if (tt < total) cid = over ? members[m0 + tt] : slots[i * SC_CAP + tt];
      if (cid == (int)i) cid = -1;
      bool valid = cid >= 0;
      if (!__ballot(valid)) continue;
      const float e0k = lane < kappa ? rowk[lane] : FLT_MAX;
      const int e0i = lane < kappa ? rowi[lane] : INT32_MAX;
      const float e1k = lane + 64 < kappa ? rowk[lane + 64] : FLT_MAX;
      const int e1i = lane + 64 < kappa ? rowi[lane + 64] : INT32_MAX;
      for (int q = 0; q < kappa; ++q) {
        const int qi = q < 64 ? __builtin_amdgcn_readlane(e0i, q) : __builtin_amdgcn_readlane(e1i, q - 64);
        valid = valid && qi != cid;  // a visited pair is already in the row
      }
      uint64_t M = __ballot(valid);
      if (!M) continue;
      // exact float64 distances: group g takes the g-th and the (G+g)-th
      // pending candidates (both rows in flight); lane j of the group reads
      // float4 chunks j, j + L, ... of the rows, summed in that order
      for (uint64_t rest = M; rest;) {
        int q0 = -1, q1 = -1;
#pragma unroll
        for (int gg = 0; gg < 2 * G; ++gg) {
          if (rest) {
            const int b = (int)__builtin_ctzll(rest);
            rest &= rest - 1;
            if (gg == g) q0 = b;
            if (gg == G + g) q1 = b;
          }
        }
        double a0 = 0.0, a1 = 0.0;
        const int jd0 = __shfl(cid, q0 < 0 ? 0 : q0, 64);  // all lanes take part
        const int jd1 = __shfl(cid, q1 < 0 ? 0 : q1, 64);
        const float* xc0 = X + (int64_t)(q0 >= 0 ? jd0 : (int)i) * ldx;
        const float* xc1 = X + (int64_t)(q1 >= 0 ? jd1 : (int)i) * ldx;
        if (q0 >= 0) {
          if (vec) {
            for (int c4 = 4 * j; c4 < d; c4 += 4 * L) {
              const float4 p4 = *reinterpret_cast<const float4*>(xr + c4);
              const float4 u4 = *reinterpret_cast<const float4*>(xc0 + c4);
              const float4 v4 = *reinterpret_cast<const float4*>(xc1 + c4);
              double df = (double)p4.x - (double)u4.x;
              a0 = fma(df, df, a0);
              df = (double)p4.y - (double)u4.y;
              a0 = fma(df, df, a0);
              df = (double)p4.z - (double)u4.z;
              a0 = fma(df, df, a0);
              df = (double)p4.w - (double)u4.w;
              a0 = fma(df, df, a0);
              df = (double)p4.x - (double)v4.x;
              a1 = fma(df, df, a1);
              df = (double)p4.y - (double)v4.y;
              a1 = fma(df, df, a1);
              df = (double)p4.z - (double)v4.z;
              a1 = fma(df, df, a1);
              df = (double)p4.w - (double)v4.w;
              a1 = fma(df, df, a1);
            }
          } else {
            for (int t = j; t < d; t += L) {
              const double p = (double)xr[t];
              double df = p - (double)xc0[t];
              a0 = fma(df, df, a0);
              df = p - (double)xc1[t];
              a1 = fma(df, df, a1);
            }
          }
        }
        a0 = group_sum<L>(a0);
        a1 = group_sum<L>(a1);
        if (q0 >= 0 && j == 0) keys[q0] = (float)a0;
        if (q1 >= 0 && j == 0) keys[q1] = (float)a1;
      }
      __builtin_amdgcn_wave_barrier();
      const float ck = valid ? keys[lane] : FLT_MAX;
      int pos_c = 0, add0 = 0, add1 = 0;
      for (int q = 0; q < kappa; ++q) {
        const float qk = q < 64 ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(e0k), q))
                                : __int_as_float(__builtin_amdgcn_readlane(__float_as_int(e1k), q - 64));
        const int qi = q < 64 ? __builtin_amdgcn_readlane(e0i, q) : __builtin_amdgcn_readlane(e1i, q - 64);
        pos_c += key_lt(qk, qi, ck, cid) ? 1 : 0;
      }
      while (M) {
        const int q = (int)__builtin_ctzll(M);
        M &= M - 1;
        const float qk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ck), q));
        const int qi = __builtin_amdgcn_readlane(cid, q);
        pos_c += key_lt(qk, qi, ck, cid) ? 1 : 0;
        add0 += key_lt(qk, qi, e0k, e0i) ? 1 : 0;
        add1 += key_lt(qk, qi, e1k, e1i) ? 1 : 0;
      }
      changed = changed || __ballot(valid && pos_c < kappa);
      __builtin_amdgcn_wave_barrier();
      if (lane < kappa && lane + add0 < kappa) {
        rowk[lane + add0] = e0k;
        rowi[lane + add0] = e0i;
      }
      if (lane + 64 < kappa && lane + 64 + add1 < kappa) {
        rowk[lane + 64 + add1] = e1k;
        rowi[lane + 64 + add1] = e1i;
      }
      if (valid && pos_c < kappa) {
        rowk[pos_c] = ck;
        rowi[pos_c] = cid;
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (changed) {
      for (int q = lane; q < kappa; q += 64) {
        G_d2[i * kappa + q] = rowk[q];
        G_ids[i * kappa + q] = rowi[q];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

static size_t refine_tile_lds(int d, int RB, bool single, int kappa) {
  return TileLayout(RB, (d + 31) / 32 * 32, single, kappa).bytes;
}

#define LDS_BUDGET (160 * 1024)
// clusters larger than one tile and at most this size: exact all-pairs kernel
#define RX_MAX 128

// Largest tile edge in {64, 32, 16} whose layout fits in LDS (0: none).
static int pick_rb(int d, bool single, int kappa) {
  for (int rb = 64; rb >= 16; rb >>= 1)
    if (refine_tile_lds(d, rb, single, kappa) <= LDS_BUDGET) return rb;
  return 0;
}

// Row blocks of the multi-tile kernel: clusters larger than one tile only.
__global__ void k_row_blocks(const int32_t* __restrict__ counts, int32_t k, int single_max, int rb,
                             int32_t* wb) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < k;
       r += (int64_t)gridDim.x * blockDim.x)
    wb[r] = counts[r] > single_max ? (counts[r] + rb - 1) / rb : 0;
}

template <bool BF16, int L, int V, int RB, bool SINGLE>
static void launch_tile(knnkm_ctx* ctx, unsigned grid, const float* X, int d, int64_t ldx, int dpad,
                        int kappa, int32_t k, const int32_t* off, const int32_t* mem, const int32_t* wb,
                        int64_t max_items, int smin, float err_c, bool vec, int32_t* G_ids, float* G_d2) {
  const size_t lds = refine_tile_lds(d, RB, SINGLE, kappa);
  hipFuncSetAttribute((const void*)k_refine_tile<BF16, L, V, RB, SINGLE>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  k_refine_tile<BF16, L, V, RB, SINGLE><<<grid, 512, lds, ctx->stream>>>(
      X, d, ldx, dpad, kappa, k, off, mem, wb, max_items, smin, err_c, vec ? 1 : 0, G_ids, G_d2);
}

template <bool BF16, int L, int V>
static knnkm_status launch_refine(knnkm_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, int dpad,
                                  int kappa, int32_t k, const int32_t* off, const int32_t* mem,
                                  const int32_t* wb, int rb1, int rb2, float err_c, bool vec,
                                  int32_t* G_ids, float* G_d2, bool multi) {
  // one tile per cluster of at most rb1 = 16 members
  launch_tile<BF16, L, V, 16, true>(ctx, k, X, d, ldx, dpad, kappa, k, off, mem, nullptr, 0, 0, err_c, vec, G_ids,
                                    G_d2);
  KNNKM_TRY(knnkm_check(ctx, "graph refine (one-tile clusters)"));
  if (!multi) return KNNKM_OK;
  // larger clusters: blocks of rb2 rows walking blocks of rb2 columns; the
  // sum over clusters of ceil(s / rb2) is at most n / rb2 + k
  const int64_t max_items = n / rb2 + k + 1;
  const unsigned g = (unsigned)max_items;
  switch (rb2) {
    case 64: launch_tile<BF16, L, V, 64, false>(ctx, g, X, d, ldx, dpad, kappa, k, off, mem, wb, max_items, 0, err_c, vec, G_ids, G_d2); break;
    case 32: launch_tile<BF16, L, V, 32, false>(ctx, g, X, d, ldx, dpad, kappa, k, off, mem, wb, max_items, 0, err_c, vec, G_ids, G_d2); break;
    default: launch_tile<BF16, L, V, 16, false>(ctx, g, X, d, ldx, dpad, kappa, k, off, mem, wb, max_items, 0, err_c, vec, G_ids, G_d2); break;
  }
  return knnkm_check(ctx, "graph refine (multi-tile clusters)");
}

knnkm_status ks_row_norms(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, float* out) {
  k_row_norms<<<grid_for(n, 4, 16384), 256, 0, ctx->stream>>>(X, n, d, ldx, out);
  return knnkm_check(ctx, "row norms");
}

knnkm_status ks_refine(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                       const int32_t* labels, int32_t k, int32_t precision, int32_t* G_ids,
                       float* G_d2, int32_t kappa, const float* norms) {
  // one-tile kernel for clusters of at most 16 members; 17-128 members take
  // the float64 Gram kernels (measured faster for 17-64 members at d = 128
  // and d = 512)
  const int rb1 = std::min(16, pick_rb(d, true, kappa)), rb2 = pick_rb(d, false, kappa);
  if (!rb1 || !rb2)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "graph refine: d=%d with kappa=%d does not fit in LDS", d,
                      kappa);
  KNNKM_WS(ctx, counts, int32_t, "rf_counts", k);
  KNNKM_WS(ctx, off, int32_t, "rf_offsets", (int64_t)k + 1);
  KNNKM_WS(ctx, mem, int32_t, "rf_members", n);
  KNNKM_WS(ctx, wb, int32_t, "rf_wb", (int64_t)k + 1);
  KNNKM_WS(ctx, items, int32_t, "rf_items", (int64_t)k + 1);
  KNNKM_WS(ctx, cnt, int32_t, "rf_survivor_counts", n);
  KNNKM_WS(ctx, slots, int32_t, "rf_survivors", n * SC_CAP);
  KNNKM_TRY(ks_label_sort(ctx, labels, n, k, counts, off, mem));
  const int dpad = (d + 31) / 32 * 32;
  const bool vec = (d % 4 == 0) && (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
  // clusters of RX_MAX < s <= RX_BIG_HI: the tiled exact kernels
  static_assert(RX_BIG_LO == RX_MAX, "the tiled exact kernels take over where the mid-sized one ends");
  bool big = false, above = true;
  KNNKM_TRY(ks_refine_big(ctx, X, n, d, ldx, kappa, k, counts, off, mem, vec, G_ids, G_d2, &big, &above));
  // with no cluster past the tiled kernels' range, the screen, its merge and
  // the multi-tile kernel have nothing to do
  const bool rest = !big || above;
  // Screening bound (squared-distance units, relative to ||x||^2 + ||y||^2):
  // twice the worst-case rounding of the float32 Gram, the float32 norms and
  // the final additions; plus the bfloat16 rounding of both operands.
  const double u = 0x1p-24;
  double err = (2.0 * dpad + 8.0) * u;
  if (precision == KNNKM_BF16_RERANK) err += 2.0 * (0x1p-7 + 0x1p-15);
  const float err_c = (float)(2.0 * err);
  int gL, gV;
  pick_group(d, 1, &gL, &gV);
  if (rest) {
    // clusters of lo_screen < s <= hi: screen + merge, with the item count
    // within int32 (items <= t_max * (n / 64 + k)); larger ones: row blocks of
    // the multi-tile kernel
    const int64_t denom = n / SC_RB + k + 1;
    const int64_t t_max = std::max<int64_t>(1, std::min<int64_t>(46340, INT32_MAX / denom));
    const int hi = (int)std::min<int64_t>(t_max * SC_RB, INT32_MAX);
    // clusters of rb1 < s <= RX_MAX: exact all-pairs kernel (below)
    const int lo_screen = big ? RX_BIG_HI : std::max(rb1, RX_MAX);
    const int multi_lo = big ? std::max(hi, RX_BIG_HI) : hi;
    k_screen_items<<<grid_for(k, 256, 4096), 256, 0, ctx->stream>>>(counts, k, lo_screen, hi, items);
    k_row_blocks<<<grid_for(k, 256, 4096), 256, 0, ctx->stream>>>(counts, k, multi_lo, rb2, wb);
    KNNKM_TRY(knnkm_check(ctx, "refine blocks"));
    KNNKM_TRY(ks_scan_exclusive(ctx, items, items, k, true));
    KNNKM_TRY(ks_scan_exclusive(ctx, wb, wb, k, true));
    KNNKM_TRY(ks_fill_i32(ctx, cnt, n, 0));
    const float* nrm = norms;
    if (!nrm) {
      KNNKM_WS(ctx, own, float, "rf_norms", n);
      KNNKM_TRY(ks_row_norms(ctx, X, n, d, ldx, own));
      nrm = own;
    }
    const unsigned gs = (unsigned)std::max(1, ctx->num_cus * 8);
    if (precision == KNNKM_BF16_RERANK)
      k_refine_screen<true><<<gs, 256, 0, ctx->stream>>>(X, d, ldx, dpad, kappa, k, off, mem, items, nrm, err_c,
                                                         vec ? 1 : 0, G_d2, cnt, slots);
    else
      k_refine_screen<false><<<gs, 256, 0, ctx->stream>>>(X, d, ldx, dpad, kappa, k, off, mem, items, nrm, err_c,
                                                          vec ? 1 : 0, G_d2, cnt, slots);
    KNNKM_TRY(knnkm_check(ctx, "graph refine screen"));
    {
      const unsigned gm = (unsigned)grid_for(n, 4, 16384);
#define RM(LL)                                                                                       \
    k_refine_merge<LL><<<gm, 256, 0, ctx->stream>>>(X, d, ldx, kappa, labels, off, mem, n, cnt, slots, \
                                                    vec ? 1 : 0, G_ids, G_d2)
      switch (gL) {
        case 4: RM(4); break;
        case 8: RM(8); break;
        case 16: RM(16); break;
        case 32: RM(32); break;
        default: RM(64); break;
      }
#undef RM
    }
    KNNKM_TRY(knnkm_check(ctx, "graph refine merge"));
  }
  if (rb1 < RX_MAX)
    KNNKM_TRY(ks_refine_exact(ctx, X, n, d, ldx, kappa, k, off, mem, rb1, RX_MAX, vec, G_ids, G_d2));
#define RF(BF, LL, VV)                                                                                    \
  return launch_refine<BF, LL, VV>(ctx, X, n, d, ldx, dpad, kappa, k, off, mem, wb, rb1, rb2, err_c, vec, \
                                   G_ids, G_d2, rest)
#define RF_L(BF, VV)                \
  switch (gL) {                     \
    case 4: RF(BF, 4, VV);          \
    case 8: RF(BF, 8, VV);          \
    case 16: RF(BF, 16, VV);        \
    case 32: RF(BF, 32, VV);        \
    default: RF(BF, 64, VV);        \
  }
  if (precision == KNNKM_BF16_RERANK) {
    if (gV == 4) { RF_L(true, 4) } else { RF_L(true, 8) }
  } else {
    if (gV == 4) { RF_L(false, 4) } else { RF_L(false, 8) }
  }
#undef RF_L
#undef RF
}

extern "C" knnkm_status knnkm_graph_init(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d,
                                         int64_t ldx, int32_t kappa, uint64_t seed, int32_t* G_ids,
                                         float* G_d2) {
  if (!ctx) return KNNKM_EINVAL;
  if (ctx->sticky) return KNNKM_EDEVICE;
  if (!X || !G_ids || !G_d2) return knnkm_fail(ctx, KNNKM_EINVAL, "graph_init: null pointer");
  if (n < 2 || n > INT32_MAX) return knnkm_fail(ctx, KNNKM_EINVAL, "graph_init: need 2 <= n < 2^31");
  if (d < 1 || ldx < d) return knnkm_fail(ctx, KNNKM_EINVAL, "graph_init: need d >= 1 and ldx >= d");
  if (d > KNNKM_MAX_D) return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "graph_init: d=%d > %d", d, KNNKM_MAX_D);
  if (kappa < 1 || kappa > n - 1) return knnkm_fail(ctx, KNNKM_EINVAL, "graph_init: need 1 <= kappa <= n-1");
  if (kappa > KNNKM_MAX_KAPPA)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "graph_init: kappa=%d > %d", kappa, KNNKM_MAX_KAPPA);
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  return ks_graph_init(ctx, X, n, d, ldx, kappa, seed, G_ids, G_d2);
}

extern "C" knnkm_status knnkm_graph_refine(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d,
                                           int64_t ldx, const int32_t* labels, int32_t k,
                                           int32_t precision, int32_t* G_ids, float* G_d2,
                                           int32_t kappa) {
  if (!ctx) return KNNKM_EINVAL;
  if (ctx->sticky) return KNNKM_EDEVICE;
  if (!X || !labels || !G_ids || !G_d2) return knnkm_fail(ctx, KNNKM_EINVAL, "graph_refine: null pointer");
  if (n < 2 || n > INT32_MAX) return knnkm_fail(ctx, KNNKM_EINVAL, "graph_refine: need 2 <= n < 2^31");
  if (d < 1 || ldx < d) return knnkm_fail(ctx, KNNKM_EINVAL, "graph_refine: need d >= 1 and ldx >= d");
  if (d > KNNKM_MAX_D) return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "graph_refine: d=%d > %d", d, KNNKM_MAX_D);
  if (k < 1 || k > n) return knnkm_fail(ctx, KNNKM_EINVAL, "graph_refine: need 1 <= k <= n");
  if (kappa < 1 || kappa > n - 1) return knnkm_fail(ctx, KNNKM_EINVAL, "graph_refine: need 1 <= kappa <= n-1");
  if (kappa > KNNKM_MAX_KAPPA)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "graph_refine: kappa=%d > %d", kappa, KNNKM_MAX_KAPPA);
  if (precision != KNNKM_FP32 && precision != KNNKM_BF16_RERANK)
    return knnkm_fail(ctx, KNNKM_EINVAL, "graph_refine: unknown precision %d", precision);
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  return ks_refine(ctx, X, n, d, ldx, labels, k, precision, G_ids, G_d2, kappa);
}
