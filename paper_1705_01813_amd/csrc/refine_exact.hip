// Exhaustive comparison inside mid-sized clusters (Alg. 3 inner loops) with
// exact keys for every pair: one block of 256 threads per cluster of
// smin < s <= SMAX members (SMAX = 64 or 128); further down, the same keys
// tiled over pairs of 64-member blocks for clusters of up to 1024 members.
//
// At the cluster sizes graph construction produces (about xi = 50 members)
// a screen of the Gram block leaves too many survivors for a separate exact
// re-rank to pay off, so every pair gets its key here:
//  1. the members' rows stream through LDS in slices (float32, transposed,
//     double-buffered: the next slice is in registers while the current one
//     is used), and the float64 Gram block G = X_S X_S^T of the cluster is
//     accumulated on MFMA (v_mfma_f64_16x16x4, the 16 x 16 tiles of the
//     upper triangle spread over the four wavefronts);
//  2. d2 = G_ii + G_jj - 2 G_ij in float64, with a rigorous bound of its
//     error; its float32 rounding is kept when the whole error interval
//     rounds to the same float32 value -- that value is then the float32
//     rounding of the exact squared distance, which the direct float64
//     difference also gives -- and otherwise (near ties with a rounding
//     boundary, near-duplicate rows, where G_ii + G_jj cancels) the pair is
//     recomputed by a float64 direct difference over its two rows;
//  3. one wavefront per member merges the cluster's other members that are
//     not yet in its list, keeping the kappa smallest (d2, id) -- the same
//     list as any other order of comparison (merge.h).
#include <cfloat>
#include <cmath>

#include "common.h"
#include "merge.h"

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

// float32 neighbours of a finite positive float32 value
__device__ inline float f32_next(float f) { return __uint_as_float(__float_as_uint(f) + 1u); }
__device__ inline float f32_prev(float f) { return __uint_as_float(__float_as_uint(f) - 1u); }

constexpr int RX_UNC_CAP = 256;  // uncertified pairs listed per cluster

// SPLIT: the keys go to global memory (keys, row r of the cluster at
// member position c0 + r, stride SMAX; columns s and beyond and the diagonal
// are left unwritten) and k_refine_rows merges them, with the occupancy the
// Gram's registers would deny the merge; the block then needs no key block
// in LDS.  Else the block merges them itself.
template <int SMAX, int SL, bool SPLIT>
__global__ __launch_bounds__(256) void k_refine_gram(const float* __restrict__ X, int d, int64_t ldx, int kappa,
                                                     int32_t k, const int32_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ members, int smin, int vec,
                                                     int32_t* __restrict__ G_ids, float* __restrict__ G_d2,
                                                     float* __restrict__ keys) {
  constexpr int TG = SMAX / 16;              // tile rows of the Gram block
  constexpr int MAXT = TG * (TG + 1) / 2;    // tiles of its upper triangle
  constexpr int TPW = (MAXT + 3) / 4;        // tiles per wavefront
  constexpr int NC = SMAX / 64;              // candidates per lane in the merge
  constexpr int NF4 = SMAX * (SL / 4);       // float4 per slice
  constexpr int PER = (NF4 + 255) / 256;     // per thread
  // slice row stride: the four k rows an MFMA operand read touches start 16
  // banks apart
  constexpr int XS = SMAX + 16;
  __shared__ __align__(16) float xs[2 * SL * XS];  // two slices, dimension-major
  __shared__ float km[SPLIT ? 1 : SMAX * SMAX];      // keys (in global memory with SPLIT)
  __shared__ double nrm[SMAX];                       // diagonal of the Gram block
  __shared__ int32_t ids[SMAX];
  __shared__ int nunc;                 // uncertified pairs
  __shared__ int16_t unc[RX_UNC_CAP];  // the first of them, r * SMAX + c
  const int cl = blockIdx.x;
  if (cl >= k) return;
  const int c0 = offsets[cl];
  const int s = offsets[cl + 1] - c0;
  if (s <= smin || s > SMAX || s < 2) return;  // block-uniform
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid < SMAX) ids[tid] = tid < s ? members[c0 + tid] : -1;
  if (tid == 0) nunc = 0;
  // this wavefront's tiles: the active ones (I <= J < ceil(s/16)) in
  // row-major order, every fourth
  const int ta = (s + 15) / 16;
  const int nta = ta * (ta + 1) / 2;
  int ti[TPW], tj[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    int t = w + 4 * q, a = 0;
    if (t >= nta) t = -1;
    while (t >= 0 && t >= ta - a) {
      t -= ta - a;
      ++a;
    }
    ti[q] = t < 0 ? -1 : a;
    tj[q] = t < 0 ? -1 : a + t;
  }
  d4_t acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = d4_t{0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  // two slices' loads in flight in registers (ra, rb) while a third is read
  // from LDS
  float4 ra[PER], rb[PER];
  auto fetch = [&](float4 (&nxt)[PER], int t0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      const int r = e % SMAX, t = t0 + 4 * (e / SMAX);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < NF4 && r < s && t < d) {
        const float* row = X + (int64_t)ids[r] * ldx;
        if (vec) {
          v = *reinterpret_cast<const float4*>(row + t);
        } else {
          v.x = row[t];
          v.y = t + 1 < d ? row[t + 1] : 0.f;
          v.z = t + 2 < d ? row[t + 2] : 0.f;
          v.w = t + 3 < d ? row[t + 3] : 0.f;
        }
      }
      nxt[u] = v;
    }
  };
  auto store = [&](const float4 (&nxt)[PER], float* buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      if (e >= NF4) continue;
      const int r = e % SMAX, q4 = e / SMAX;
      buf[(4 * q4) * XS + r] = nxt[u].x;
      buf[(4 * q4 + 1) * XS + r] = nxt[u].y;
      buf[(4 * q4 + 2) * XS + r] = nxt[u].z;
      buf[(4 * q4 + 3) * XS + r] = nxt[u].w;
    }
  };
  const int nsl = (d + SL - 1) / SL;  // slices
  fetch(ra, 0);
  store(ra, xs);
  if (nsl > 1) fetch(ra, SL);
  if (nsl > 2) fetch(rb, 2 * SL);
  __syncthreads();
  int cur = 0;
  const int kr = lane >> 4, rc = lane & 15;  // MFMA operands: k row, tile row or column
  auto gram_slice = [&](const float* buf) {
#pragma unroll
    for (int kk = 0; kk < SL; kk += 4) {
      const float* kb = buf + (kk + kr) * XS + rc;
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        if (ti[q] < 0) continue;  // wave-uniform
        const double a = (double)kb[16 * ti[q]];
        const double b = (double)kb[16 * tj[q]];
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
      }
    }
  };
  // slice i in LDS; the next two in ra / rb, their roles alternating
  for (int i = 0; i < nsl; i += 2) {
    gram_slice(xs + cur * (SL * XS));
    if (i + 1 < nsl) store(ra, xs + (cur ^ 1) * (SL * XS));
    if (i + 3 < nsl) fetch(ra, (i + 3) * SL);
    __syncthreads();
    cur ^= 1;
    if (i + 1 >= nsl) break;
    gram_slice(xs + cur * (SL * XS));
    if (i + 2 < nsl) store(rb, xs + (cur ^ 1) * (SL * XS));
    if (i + 4 < nsl) fetch(rb, (i + 4) * SL);
    __syncthreads();
    cur ^= 1;
  }
  // the output of a tile: lane l holds rows (l >> 4) + 4v, column l & 15
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    if (ti[q] < 0 || ti[q] != tj[q]) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (kr + 4 * v == rc) nrm[16 * ti[q] + rc] = acc[q][v];
  }
  __syncthreads();
  // keys; an uncertified one is marked and recomputed below.  Error of d2
  // (float64 Gram expansion over K summed products): at most
  // (2K + 16) 2^-53 (G_ii + G_jj).
  const double gam = (2.0 * (double)((d + SL - 1) / SL * SL) + 16.0) * 0x1p-53;
  // f: the float32 rounding of d2 from the Gram entry g; true when certified
  auto certify = [&](double g, int r, int c, float& f) {
    const double nn = nrm[r] + nrm[c];
    const double D = nn - 2.0 * g;
    const double E = gam * nn + 1e-300;
    f = (float)D;
    bool ok = D - E > 0.0 && f > 0.f && f < FLT_MAX;
    if (ok) {
      const double lo = 0.5 * ((double)f32_prev(f) + (double)f);
      const double hi = 0.5 * ((double)f + (double)f32_next(f));
      ok = D - E > lo && D + E < hi;
    }
    return ok;
  };
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    if (ti[q] < 0) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * ti[q] + kr + 4 * v, c = 16 * tj[q] + rc;
      if (r < c && c < s) {
        float f;
        const bool ok = certify(acc[q][v], r, c, f);
        if constexpr (!SPLIT) {
          km[r * SMAX + c] = f;
          km[c * SMAX + r] = f;
        }
        if (!ok) {
          const int u = atomicAdd(&nunc, 1);
          if (u < RX_UNC_CAP) unc[u] = (int16_t)(r * SMAX + c);
        }
      }
    }
  }
  __syncthreads();
  const int nu = nunc;  // block-uniform
  // SPLIT: every key is written to global memory once -- the certified ones
  // here (none when every pair is recomputed below), the others below
  float* kout = SPLIT ? keys + (int64_t)c0 * SMAX : nullptr;
  if constexpr (SPLIT) {
    if (nu <= RX_UNC_CAP) {
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        if (ti[q] < 0) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * ti[q] + kr + 4 * v, c = 16 * tj[q] + rc;
          float f;
          if (r < c && c < s && certify(acc[q][v], r, c, f)) {
            kout[r * SMAX + c] = f;
            kout[c * SMAX + r] = f;
          }
        }
      }
    }
  }
  // uncertified pairs: float64 direct difference of the two rows, one
  // wavefront per pair (lane j: dimensions j, j + 64, ...; fixed order).
  // Past the list's capacity every pair of the cluster is recomputed.
  if (nu > 0) {
    const int np = nu <= RX_UNC_CAP ? nu : s * s;
    for (int p = w; p < np; p += 4) {
      int pr, pc;
      if (nu <= RX_UNC_CAP) {
        pr = unc[p] / SMAX;
        pc = unc[p] % SMAX;
      } else {
        pr = p / s;
        pc = p % s;
        if (pr >= pc) continue;  // wave-uniform
      }
      const float* xa = X + (int64_t)ids[pr] * ldx;
      const float* xb = X + (int64_t)ids[pc] * ldx;
      double a = 0.0;
      for (int t = lane; t < d; t += 64) {
        const double df = (double)xa[t] - (double)xb[t];
        a = fma(df, df, a);
      }
      a = wave_sum(a);
      if (lane == 0) {
        if constexpr (SPLIT) {
          kout[pr * SMAX + pc] = (float)a;
          kout[pc * SMAX + pr] = (float)a;
        } else {
          km[pr * SMAX + pc] = (float)a;
          km[pc * SMAX + pr] = (float)a;
        }
      }
    }
    if constexpr (!SPLIT) __syncthreads();
  }
  if constexpr (SPLIT) return;
  // merge: one wavefront per member; lane l holds candidates l, l + 64, ...
  // (the next member's row is loaded while one is merged); the id tables in
  // the slice buffers, free now
  static_assert(2 * SL * XS >= 4 * MG_SLOTS, "id tables fit in the slice buffers");
  int32_t* hs = reinterpret_cast<int32_t*>(xs) + MG_SLOTS * w;
  for (int e = lane; e < MG_SLOTS; e += 64) hs[e] = -1;
  MergeRow cur_row = {FLT_MAX, FLT_MAX, INT32_MAX, INT32_MAX};
  if (w < s) cur_row = merge_load(G_d2 + (int64_t)ids[w] * kappa, G_ids + (int64_t)ids[w] * kappa, kappa);
  for (int r = w; r < s; r += 4) {
    MergeRow nxt_row = cur_row;
    if (r + 4 < s)
      nxt_row = merge_load(G_d2 + (int64_t)ids[r + 4] * kappa, G_ids + (int64_t)ids[r + 4] * kappa, kappa);
    float ck[NC];
    int cid[NC];
    bool valid[NC];
#pragma unroll
    for (int h = 0; h < NC; ++h) {
      const int c = lane + 64 * h;
      valid[h] = c < s && c != r;
      ck[h] = valid[h] ? km[r * SMAX + c] : FLT_MAX;
      cid[h] = valid[h] ? ids[c] : -1;
    }
    const int64_t row = (int64_t)ids[r] * kappa;
    merge_row<NC>(G_d2 + row, G_ids + row, kappa, cur_row, ck, cid, valid, hs);
    cur_row = nxt_row;
  }
}

// The merge of k_refine_gram<SMAX, SL, true>'s keys: one block per cluster
// of smin < s <= SMAX members, one wavefront per member row (w, w + 4, ...),
// the next row's entries and keys loaded while one is merged; the same
// merge, in the same order per row, as the fused kernel.
template <int SMAX>
__global__ __launch_bounds__(256) void k_refine_rows(const float* __restrict__ keys, int32_t k,
                                                     const int32_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ members, int smin, int kappa,
                                                     int32_t* __restrict__ G_ids, float* __restrict__ G_d2) {
  constexpr int NC = SMAX / 64;
  const int cl = blockIdx.x;
  if (cl >= k) return;
  const int c0 = offsets[cl];
  const int s = offsets[cl + 1] - c0;
  if (s <= smin || s > SMAX || s < 2) return;  // block-uniform
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __shared__ int32_t mgh[4][MG_SLOTS];
  int32_t* hs = mgh[w];
  for (int e = lane; e < MG_SLOTS; e += 64) hs[e] = -1;
  // the cluster's member ids, candidate slot h of this lane
  int mid[NC];
#pragma unroll
  for (int h = 0; h < NC; ++h) mid[h] = lane + 64 * h < s ? members[c0 + lane + 64 * h] : -1;
  // keys of row r (columns s and beyond and the diagonal unwritten; masked
  // by valid below)
  auto load_keys = [&](int r, float (&out)[NC]) {
#pragma unroll
    for (int h = 0; h < NC; ++h) out[h] = keys[(int64_t)(c0 + r) * SMAX + lane + 64 * h];
  };
  MergeRow cur_row = {FLT_MAX, FLT_MAX, INT32_MAX, INT32_MAX};
  float cur_k[NC];
  if (w < s) {
    const int64_t row = (int64_t)members[c0 + w] * kappa;
    cur_row = merge_load(G_d2 + row, G_ids + row, kappa);
    load_keys(w, cur_k);
  }
  for (int r = w; r < s; r += 4) {
    MergeRow nxt_row = cur_row;
    float nxt_k[NC];
#pragma unroll
    for (int h = 0; h < NC; ++h) nxt_k[h] = cur_k[h];
    if (r + 4 < s) {
      const int64_t row = (int64_t)members[c0 + r + 4] * kappa;
      nxt_row = merge_load(G_d2 + row, G_ids + row, kappa);
      load_keys(r + 4, nxt_k);
    }
    float ck[NC];
    int cid[NC];
    bool valid[NC];
#pragma unroll
    for (int h = 0; h < NC; ++h) {
      const int c = lane + 64 * h;
      valid[h] = c < s && c != r;
      ck[h] = valid[h] ? cur_k[h] : FLT_MAX;
      cid[h] = valid[h] ? mid[h] : -1;
    }
    const int64_t row = (int64_t)members[c0 + r] * kappa;
    merge_row<NC>(G_d2 + row, G_ids + row, kappa, cur_row, ck, cid, valid, hs);
    cur_row = nxt_row;
#pragma unroll
    for (int h = 0; h < NC; ++h) cur_k[h] = nxt_k[h];
  }
}


// ------------------------------------------------ clusters of 129...1024 --
// The same exact keys for clusters of RX_BIG_LO < s <= RX_BIG_HI members,
// tiled: one block of 256 threads per pair of 64-member blocks (I <= J) of
// a cluster.  The block stages the two blocks' rows (I first, then J) as
// the mid-sized kernel does, forms the 64 x 64 float64 Gram block between
// them on MFMA (for I == J its upper triangle), the rows' float64 squared
// norms from the same slices (one thread per row, dimensions in order), and
// writes every certified key of the block, both ways, to global memory
// (keys: the cluster's rows at row_off, stride sw); the uncertified ones
// are recomputed from the rows.  Each key is written once.
constexpr int BX_RB = 64;  // members per side of a block

template <int SL>
__global__ __launch_bounds__(256) void k_refine_gram_big(const float* __restrict__ X, int d, int64_t ldx,
                                                         int32_t k, const int32_t* __restrict__ offsets,
                                                         const int32_t* __restrict__ members,
                                                         const int32_t* __restrict__ item_off,
                                                         const int32_t* __restrict__ row_off, int sw, int vec,
                                                         float* __restrict__ keys) {
  constexpr int R = 2 * BX_RB;            // staged rows: block I, then block J
  constexpr int TPW = 4;                  // tiles per wavefront (16 of 16 x 16, or 10 for I == J)
  constexpr int NF4 = R * (SL / 4);       // float4 per slice
  constexpr int PER = (NF4 + 255) / 256;  // per thread
  constexpr int XS = R + 16;
  __shared__ __align__(16) float xs[2 * SL * XS];
  __shared__ double nrm[R];
  __shared__ int32_t ids[R];
  __shared__ int nunc;
  __shared__ int16_t unc[RX_UNC_CAP];  // staged r * R + c
  const int64_t item = blockIdx.x;
  if (item >= item_off[k]) return;
  int lo = 0, hi = k;  // the cluster: the last c with item_off[c] <= item
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (item_off[mid] <= item) lo = mid; else hi = mid;
  }
  const int cl = lo;
  const int c0 = offsets[cl];
  const int s = offsets[cl + 1] - c0;
  const int T = (s + BX_RB - 1) / BX_RB;
  int pr0 = (int)(item - item_off[cl]), I = 0;  // row-major upper triangle of T x T
  while (pr0 >= T - I) {
    pr0 -= T - I;
    ++I;
  }
  const int J = I + pr0;
  const bool diag = I == J;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // member of staged row r; -1 past s (and for the J half when I == J)
  auto member_of = [&](int r) { return r < BX_RB ? BX_RB * I + r : BX_RB * J + r - BX_RB; };
  if (tid < R) {
    const int m = member_of(tid);
    ids[tid] = (tid < BX_RB || !diag) && m < s ? members[c0 + m] : -1;
  }
  if (tid == 0) nunc = 0;
  // tiles (16-row groups a of the I half, b of the J half or, for I == J,
  // b >= a of the I half); a group whose first member is past s is skipped
  int ti[TPW], tj[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    int t = w + 4 * q, a, b;
    if (!diag) {
      a = t / 4;
      b = 4 + t % 4;
    } else if (t < 10) {
      a = 0;
      while (t >= 4 - a) {
        t -= 4 - a;
        ++a;
      }
      b = a + t;
    } else {
      a = b = -1;
    }
    if (a >= 0 && (member_of(16 * a) >= s || member_of(16 * b) >= s)) a = b = -1;
    ti[q] = a;
    tj[q] = b;
  }
  d4_t acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = d4_t{0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  float4 ra[PER], rb[PER];
  auto fetch = [&](float4 (&nxt)[PER], int t0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      const int r = e % R, t = t0 + 4 * (e / R);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < NF4 && ids[r] >= 0 && t < d) {
        const float* row = X + (int64_t)ids[r] * ldx;
        if (vec) {
          v = *reinterpret_cast<const float4*>(row + t);
        } else {
          v.x = row[t];
          v.y = t + 1 < d ? row[t + 1] : 0.f;
          v.z = t + 2 < d ? row[t + 2] : 0.f;
          v.w = t + 3 < d ? row[t + 3] : 0.f;
        }
      }
      nxt[u] = v;
    }
  };
  auto store = [&](const float4 (&nxt)[PER], float* buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      if (e >= NF4) continue;
      const int r = e % R, q4 = e / R;
      buf[(4 * q4) * XS + r] = nxt[u].x;
      buf[(4 * q4 + 1) * XS + r] = nxt[u].y;
      buf[(4 * q4 + 2) * XS + r] = nxt[u].z;
      buf[(4 * q4 + 3) * XS + r] = nxt[u].w;
    }
  };
  const int nsl = (d + SL - 1) / SL;
  fetch(ra, 0);
  store(ra, xs);
  if (nsl > 1) fetch(ra, SL);
  if (nsl > 2) fetch(rb, 2 * SL);
  __syncthreads();
  int cur = 0;
  const int kr = lane >> 4, rc = lane & 15;
  double nacc = 0.0;  // thread tid < R: squared norm of staged row tid
  auto gram_slice = [&](const float* buf) {
#pragma unroll
    for (int kk = 0; kk < SL; kk += 4) {
      const float* kb = buf + (kk + kr) * XS + rc;
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        if (ti[q] < 0) continue;  // wave-uniform
        const double a = (double)kb[16 * ti[q]];
        const double b = (double)kb[16 * tj[q]];
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
      }
    }
    if (tid < R) {
#pragma unroll
      for (int kk = 0; kk < SL; ++kk) {
        const double v = (double)buf[kk * XS + tid];
        nacc = fma(v, v, nacc);
      }
    }
  };
  for (int i = 0; i < nsl; i += 2) {
    gram_slice(xs + cur * (SL * XS));
    if (i + 1 < nsl) store(ra, xs + (cur ^ 1) * (SL * XS));
    if (i + 3 < nsl) fetch(ra, (i + 3) * SL);
    __syncthreads();
    cur ^= 1;
    if (i + 1 >= nsl) break;
    gram_slice(xs + cur * (SL * XS));
    if (i + 2 < nsl) store(rb, xs + (cur ^ 1) * (SL * XS));
    if (i + 4 < nsl) fetch(rb, (i + 4) * SL);
    __syncthreads();
    cur ^= 1;
  }
  if (tid < R) nrm[tid] = nacc;
  __syncthreads();
  // error of d2: as in the mid-sized kernel, with the norms summed in order
  const double gam = (2.0 * (double)((d + SL - 1) / SL * SL) + 16.0) * 0x1p-53;
  auto certify = [&](double g, int r, int c, float& f) {
    const double nn = nrm[r] + nrm[c];
    const double D = nn - 2.0 * g;
    const double E = gam * nn + 1e-300;
    f = (float)D;
    bool ok = D - E > 0.0 && f > 0.f && f < FLT_MAX;
    if (ok) {
      const double lo_ = 0.5 * ((double)f32_prev(f) + (double)f);
      const double hi_ = 0.5 * ((double)f + (double)f32_next(f));
      ok = D - E > lo_ && D + E < hi_;
    }
    return ok;
  };
  // staged pair (r, c) of this block: r in the I half, c in the J half (or
  // c > r in the I half when I == J), both members below s
  auto in_block = [&](int r, int c) {
    if (r >= BX_RB || member_of(r) >= s) return false;
    if (diag) return c < BX_RB && c > r && member_of(c) < s;
    return c >= BX_RB && member_of(c) < s;
  };
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    if (ti[q] < 0) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * ti[q] + kr + 4 * v, c = 16 * tj[q] + rc;
      float f;
      if (in_block(r, c) && !certify(acc[q][v], r, c, f)) {
        const int u = atomicAdd(&nunc, 1);
        if (u < RX_UNC_CAP) unc[u] = (int16_t)(r * R + c);
      }
    }
  }
  __syncthreads();
  const int nu = nunc;  // block-uniform
  float* kout = keys + (int64_t)row_off[cl] * sw;
  if (nu <= RX_UNC_CAP) {
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      if (ti[q] < 0) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * ti[q] + kr + 4 * v, c = 16 * tj[q] + rc;
        float f;
        if (in_block(r, c) && certify(acc[q][v], r, c, f)) {
          const int mr = member_of(r), mc = member_of(c);
          kout[(int64_t)mr * sw + mc] = f;
          kout[(int64_t)mc * sw + mr] = f;
        }
      }
    }
  }
  // uncertified pairs (past the list's capacity: every pair of the block)
  if (nu > 0) {
    const int np = nu <= RX_UNC_CAP ? nu : R * R;
    for (int p = w; p < np; p += 4) {
      int pr, pc;
      if (nu <= RX_UNC_CAP) {
        pr = unc[p] / R;
        pc = unc[p] % R;
      } else {
        pr = p / R;
        pc = p % R;
        if (!in_block(pr, pc)) continue;  // wave-uniform
      }
      const float* xa = X + (int64_t)ids[pr] * ldx;
      const float* xb = X + (int64_t)ids[pc] * ldx;
      double a = 0.0;
      for (int t = lane; t < d; t += 64) {
        const double df = (double)xa[t] - (double)xb[t];
        a = fma(df, df, a);
      }
      a = wave_sum(a);
      if (lane == 0) {
        const int mr = member_of(pr), mc = member_of(pc);
        kout[(int64_t)mr * sw + mc] = (float)a;
        kout[(int64_t)mc * sw + mr] = (float)a;
      }
    }
  }
}

// The merge of k_refine_gram_big's keys: one wavefront per member row of
// the clusters (rows at row_off, in cluster order; four per block, the grid
// striding over them); the row is held in LDS and merged with 64 candidates
// at a time (keys of the next 64 loaded while one group is merged), then
// written back if it changed -- the same list as any other order of
// comparison.
__global__ __launch_bounds__(256) void k_refine_rows_big(const float* __restrict__ keys, int sw, int32_t k,
                                                         const int32_t* __restrict__ offsets,
                                                         const int32_t* __restrict__ members,
                                                         const int32_t* __restrict__ row_off, int kappa,
                                                         int32_t* __restrict__ G_ids, float* __restrict__ G_d2) {
  __shared__ float rks[4][KNNKM_MAX_KAPPA];
  __shared__ int32_t ris[4][KNNKM_MAX_KAPPA];
  __shared__ int32_t mgh[4][MG_SLOTS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  float* rowk = rks[w];
  int32_t* rowi = ris[w];
  int32_t* hs = mgh[w];
  for (int e = lane; e < MG_SLOTS; e += 64) hs[e] = -1;
  const int64_t total = row_off[k];
  // wave-uniform loop (no block barrier inside)
  for (int64_t gr = (int64_t)blockIdx.x * 4 + w; gr < total; gr += (int64_t)gridDim.x * 4) {
    int lo = 0, hi = k;  // the cluster: the last c with row_off[c] <= gr
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (row_off[mid] <= gr) lo = mid; else hi = mid;
    }
    const int cl = lo;
    const int c0 = offsets[cl];
    const int s = offsets[cl + 1] - c0;
    const int r = (int)(gr - row_off[cl]);
    const float* kr = keys + ((int64_t)row_off[cl] + r) * sw;
    const int64_t g = (int64_t)members[c0 + r] * kappa;
    for (int q = lane; q < kappa; q += 64) {
      rowk[q] = G_d2[g + q];
      rowi[q] = G_ids[g + q];
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    bool changed = false;
    float nk = kr[lane];
    for (int cb = 0; cb < s; cb += 64) {
      const float kv = nk;
      if (cb + 64 < s) nk = kr[cb + 64 + lane];
      const int c = cb + lane;
      const bool valid[1] = {c < s && c != r};
      const float ck[1] = {valid[0] ? kv : FLT_MAX};
      const int cid[1] = {valid[0] ? members[c0 + c] : -1};
      const MergeRow old = merge_load(rowk, rowi, kappa);
      if (merge_row<1>(rowk, rowi, kappa, old, ck, cid, valid, hs)) changed = true;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    if (changed)
      for (int q = lane; q < kappa; q += 64) {
        G_d2[g + q] = rowk[q];
        G_ids[g + q] = rowi[q];
      }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// tot[2]: the largest size in (lo, hi]; tot[3]: clusters above hi
__global__ void k_big_items(const int32_t* __restrict__ counts, int32_t k, int lo, int hi, int32_t* items,
                            int32_t* rows, int32_t* tot) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < k; c += (int64_t)gridDim.x * blockDim.x) {
    const int s = counts[c];
    const bool in = s > lo && s <= hi;
    const int t = (s + BX_RB - 1) / BX_RB;
    items[c] = in ? t * (t + 1) / 2 : 0;
    rows[c] = in ? s : 0;
    if (in) atomicMax(&tot[2], s);
    if (s > hi) atomicAdd(&tot[3], 1);
  }
}

__global__ void k_big_totals(const int32_t* items_total, const int32_t* rows_total, int32_t* tot) {
  if (threadIdx.x == 0) {
    tot[0] = *items_total;
    tot[1] = *rows_total;
  }
}

}  // namespace

knnkm_status ks_refine_exact(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, int32_t kappa,
                             int32_t k, const int32_t* offsets, const int32_t* members, int32_t smin,
                             int32_t smax, bool vec, int32_t* G_ids, float* G_d2) {
  if (smax > 128) return knnkm_fail(ctx, KNNKM_EINVAL, "refine_exact: clusters of at most 128 members");
  if (k <= 0 || smin >= smax) return KNNKM_OK;
  if (smin < 64)
    k_refine_gram<64, 32, false><<<(unsigned)k, 256, 0, ctx->stream>>>(X, d, ldx, kappa, k, offsets, members, smin,
                                                                    vec ? 1 : 0, G_ids, G_d2, nullptr);
  if (smax > 64) {
    // keys of every member row at stride 128 (a cluster's rows at its member
    // positions), then the merge
    float* keys = (float*)knnkm_ws(ctx, "rx_keys", sizeof(float) * (size_t)n * 128);
    if (!keys) return KNNKM_ENOMEM;
    const int s0 = std::max(smin, 64);
    k_refine_gram<128, 8, true><<<(unsigned)k, 256, 0, ctx->stream>>>(X, d, ldx, kappa, k, offsets, members, s0,
                                                                    vec ? 1 : 0, G_ids, G_d2, keys);
    k_refine_rows<128><<<(unsigned)k, 256, 0, ctx->stream>>>(keys, k, offsets, members, s0, kappa, G_ids, G_d2);
  }
  return knnkm_check(ctx, "graph refine (exact, mid-sized clusters)");
}


knnkm_status ks_refine_big(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, int32_t kappa,
                           int32_t k, const int32_t* counts, const int32_t* offsets, const int32_t* members,
                           bool vec, int32_t* G_ids, float* G_d2, bool* handled, bool* above) {
  *handled = false;
  *above = true;
  if (ctx->capturing || k <= 0) return KNNKM_OK;
  KNNKM_WS(ctx, items, int32_t, "bx_items", (int64_t)k + 1);
  KNNKM_WS(ctx, rows, int32_t, "bx_rows", (int64_t)k + 1);
  KNNKM_WS(ctx, tot, int32_t, "bx_tot", 4);
  KNNKM_TRY(ks_fill_i32(ctx, tot, 4, 0));
  k_big_items<<<grid_for(k, 256, 4096), 256, 0, ctx->stream>>>(counts, k, RX_BIG_LO, RX_BIG_HI, items, rows,
                                                               tot);
  KNNKM_TRY(knnkm_check(ctx, "refine (large clusters): items"));
  KNNKM_TRY(ks_scan_exclusive(ctx, items, items, k, true));
  KNNKM_TRY(ks_scan_exclusive(ctx, rows, rows, k, true));
  k_big_totals<<<1, 64, 0, ctx->stream>>>(items + k, rows + k, tot);
  int32_t h[4] = {0, 0, 0, 0};
  KNNKM_HIP(ctx, hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  KNNKM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *handled = true;  // the screen path now leaves these clusters alone
  *above = h[3] > 0;
  if (h[0] == 0) return KNNKM_OK;
  // one launch of at most 2^32 threads
  if ((int64_t)h[0] * 256 >= ((int64_t)1 << 32)) {
    *handled = false;
    return KNNKM_OK;
  }
  const int sw = (h[2] + 63) / 64 * 64;
  float* keys = (float*)knnkm_ws(ctx, "bx_keys", sizeof(float) * (size_t)h[1] * (size_t)sw);
  if (!keys) return KNNKM_ENOMEM;
  k_refine_gram_big<8><<<(unsigned)h[0], 256, 0, ctx->stream>>>(X, d, ldx, k, offsets, members, items, rows, sw,
                                                              vec ? 1 : 0, keys);
  KNNKM_TRY(knnkm_check(ctx, "refine (large clusters): keys"));
  const unsigned gm = (unsigned)std::min<int64_t>(((int64_t)h[1] + 3) / 4, (int64_t)1 << 20);
  k_refine_rows_big<<<gm, 256, 0, ctx->stream>>>(keys, sw, k, offsets, members, rows, kappa, G_ids, G_d2);
  return knnkm_check(ctx, "refine (large clusters): merge");
}
