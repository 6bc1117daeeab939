// Centroid update (Sec. 1: each centroid becomes the average of its members;
// Eqn. 2: composite vectors D_r and sizes n_r) and distortion (Eqn. 4).
//
//  * label sort: stable LSD radix sort of sample ids by label (8-bit digits,
//    1024 ids per block, per-wave match masks for stable ranks) giving the CSR
//    partition offsets[k+1] / members[n] with ids ascending inside a cluster.
//  * segmented sums: every cluster is cut into chunks of 64 members; one
//    wavefront sums a chunk in float64 (rows read as float4, 64/LR rows at a
//    time with LR lanes per row; each lane adds its rows in member order and
//    the row slots are combined by a fixed butterfly); a second kernel adds
//    the chunk partials of a cluster in chunk order, so the result is
//    identical on every run.
//  * distortion: float64 per sample, fixed per-block order, fixed final sum.
#include <mutex>

#include "common.h"

#define RS_TILE 1024
#define SEG_CHUNK 64

// ------------------------------------------------------------ label sort --
// Cluster sizes.  Runs of equal labels inside a wavefront's 64 consecutive
// samples are counted with one atomic (labels of cluster-ordered data come in
// long runs).
__global__ void k_label_hist(const int32_t* __restrict__ labels, int64_t n, int32_t* counts) {
  const int lane = threadIdx.x & 63;
  for (int64_t base = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) - lane; base < n;
       base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + lane;
    const bool valid = i < n;
    const int lab = valid ? labels[i] : -1;
    const int prev = __shfl_up(lab, 1, 64);
    const bool head = valid && (lane == 0 || lab != prev);
    const uint64_t heads = __ballot(head);
    const uint64_t alive = __ballot(valid);
    if (head) {
      const uint64_t later = lane == 63 ? 0ull : (heads >> (lane + 1));
      const int run_end = later ? lane + 1 + (int)__builtin_ctzll(later) : 64 - (int)__builtin_clzll(alive);
      atomicAdd(&counts[lab], run_end - lane);
    }
  }
}

__global__ __launch_bounds__(256) void k_rs_count(const int32_t* __restrict__ keys, int64_t n,
                                                  int shift, int nblocks, int32_t* hist) {
  __shared__ int32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int j = 0; j < 4; ++j) {
    int64_t idx = base + threadIdx.x + 256 * j;
    if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__device__ inline uint64_t match_digit(int dg, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    bool bit = (dg >> b) & 1;
    uint64_t bb = __ballot(valid && bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

// Stable scatter: wave w of a block owns ids [base + 256w, base + 256w + 256)
// and walks them in order, 64 at a time.
__global__ __launch_bounds__(256) void k_rs_scatter(const int32_t* __restrict__ keys_in,
                                                    const int32_t* __restrict__ vals_in, int64_t n,
                                                    int shift, int nblocks,
                                                    const int32_t* __restrict__ hist_scan,
                                                    int32_t* __restrict__ keys_out,
                                                    int32_t* __restrict__ vals_out) {
  __shared__ int32_t wcnt[4][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = 0; j < 4; ++j) wcnt[j][threadIdx.x] = 0;
  __syncthreads();
  const int64_t wbase = (int64_t)blockIdx.x * RS_TILE + w * 256;
  for (int r = 0; r < 4; ++r) {
    int64_t idx = wbase + r * 64 + lane;
    bool valid = idx < n;
    int dg = valid ? (keys_in[idx] >> shift) & 255 : 0;
    uint64_t m = match_digit(dg, valid);
    if (valid && lane == (int)__builtin_ctzll(m)) atomicAdd(&wcnt[w][dg], __popcll(m));
  }
  __syncthreads();
  {
    int dg = threadIdx.x;
    int32_t run = hist_scan[(int64_t)dg * nblocks + blockIdx.x];
    for (int j = 0; j < 4; ++j) {
      int32_t c = wcnt[j][dg];
      wcnt[j][dg] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int r = 0; r < 4; ++r) {
    int64_t idx = wbase + r * 64 + lane;
    bool valid = idx < n;
    int32_t key = valid ? keys_in[idx] : 0;
    int dg = (key >> shift) & 255;
    uint64_t m = match_digit(dg, valid);
    int32_t base = valid ? wcnt[w][dg] : 0;
    if (valid) {
      int32_t pos = base + __popcll(m & lanes_below());
      if (keys_out) keys_out[pos] = key;
      vals_out[pos] = vals_in ? vals_in[idx] : (int32_t)idx;
    }
    __builtin_amdgcn_wave_barrier();
    if (valid && lane == (int)__builtin_ctzll(m)) wcnt[w][dg] = base + __popcll(m);
    __builtin_amdgcn_wave_barrier();
  }
}

knnkm_status ks_label_sort(knnkm_ctx* ctx, const int32_t* labels, int64_t n, int32_t k,
                           int32_t* counts, int32_t* offsets, int32_t* members) {
  KNNKM_TRY(ks_fill_i32(ctx, counts, k, 0));
  k_label_hist<<<grid_for(n, 256, 8192), 256, 0, ctx->stream>>>(labels, n, counts);
  KNNKM_TRY(knnkm_check(ctx, "label hist"));
  KNNKM_TRY(ks_scan_exclusive(ctx, counts, offsets, k, true));
  int bits = 0;
  while (bits < 31 && ((int64_t)1 << bits) < k) ++bits;
  int passes = (bits + 7) / 8;
  if (passes == 0) passes = 1;  // one cluster: still materialise members = 0..n-1
  const int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
  KNNKM_WS(ctx, hist, int32_t, "rs_hist", (int64_t)256 * nblocks + 1);
  KNNKM_WS(ctx, kbuf, int32_t, "rs_keys", 2 * n);
  KNNKM_WS(ctx, vbuf, int32_t, "rs_vals", 2 * n);
  const int32_t* kin = labels;
  const int32_t* vin = nullptr;
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    int32_t* kout = last ? nullptr : kbuf + (p & 1) * n;
    int32_t* vout = last ? members : vbuf + (p & 1) * n;
    k_rs_count<<<nblocks, 256, 0, ctx->stream>>>(kin, n, 8 * p, nblocks, hist);
    KNNKM_TRY(knnkm_check(ctx, "radix count"));
    KNNKM_TRY(ks_scan_exclusive(ctx, hist, hist, (int64_t)256 * nblocks, false));
    k_rs_scatter<<<nblocks, 256, 0, ctx->stream>>>(kin, vin, n, 8 * p, nblocks, hist, kout, vout);
    KNNKM_TRY(knnkm_check(ctx, "radix scatter"));
    kin = kout;
    vin = vout;
  }
  return KNNKM_OK;
}

// ---------------------------------------------------------- segmented sum --
__global__ void k_chunk_counts(const int32_t* __restrict__ counts, int32_t k, int32_t* cc) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < k;
       r += (int64_t)gridDim.x * blockDim.x)
    cc[r] = (counts[r] + SEG_CHUNK - 1) / SEG_CHUNK;
}

template <int T>
__global__ __launch_bounds__(256) void k_seg_partial(const float* __restrict__ X, int d, int64_t ldx,
                                                     int32_t k, const int32_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ members,
                                                     const int32_t* __restrict__ chunk_off,
                                                     int64_t max_chunks, double* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= max_chunks) return;
  const int32_t total = chunk_off[k];
  if (c >= total) return;
  // cluster r: chunk_off[r] <= c < chunk_off[r+1]
  int lo = 0, hi = k;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= c) lo = mid; else hi = mid;
  }
  const int r = lo;
  const int64_t p0 = offsets[r] + (c - chunk_off[r]) * SEG_CHUNK;
  const int64_t p1 = min((int64_t)offsets[r + 1], p0 + SEG_CHUNK);
  double acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = 0.0;
  int64_t p = p0;
  for (; p + 4 <= p1; p += 4) {
    const float* r0 = X + (int64_t)members[p] * ldx;
    const float* r1 = X + (int64_t)members[p + 1] * ldx;
    const float* r2 = X + (int64_t)members[p + 2] * ldx;
    const float* r3 = X + (int64_t)members[p + 3] * ldx;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      int dim = lane + 64 * t;
      if (dim < d) {
        float v0 = r0[dim], v1 = r1[dim], v2 = r2[dim], v3 = r3[dim];
        acc[t] += (double)v0;
        acc[t] += (double)v1;
        acc[t] += (double)v2;
        acc[t] += (double)v3;
      }
    }
  }
  for (; p < p1; ++p) {
    const float* r0 = X + (int64_t)members[p] * ldx;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      int dim = lane + 64 * t;
      if (dim < d) acc[t] += (double)r0[dim];
    }
  }
  double* out = partial + c * d;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    int dim = lane + 64 * t;
    if (dim < d) out[dim] = acc[t];
  }
}

// Wide rows (d > 256, rows 16-byte aligned): the same chunk sums, each lane
// reading four consecutive dimensions per 16-byte load (dimensions
// 4 lane + 256 t + j); every dimension is still summed over the chunk's
// members in order, so the partials are those of k_seg_partial.
template <int T4>
__global__ __launch_bounds__(256) void k_seg_partial4(const float* __restrict__ X, int d, int64_t ldx,
                                                      int32_t k, const int32_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ members,
                                                      const int32_t* __restrict__ chunk_off,
                                                      int64_t max_chunks, double* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= max_chunks) return;
  const int32_t total = chunk_off[k];
  if (c >= total) return;
  int lo = 0, hi = k;  // cluster r: chunk_off[r] <= c < chunk_off[r+1]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= c) lo = mid; else hi = mid;
  }
  const int r = lo;
  const int64_t p0 = offsets[r] + (c - chunk_off[r]) * SEG_CHUNK;
  const int64_t p1 = min((int64_t)offsets[r + 1], p0 + SEG_CHUNK);
  double acc[T4][4];
#pragma unroll
  for (int t = 0; t < T4; ++t) acc[t][0] = acc[t][1] = acc[t][2] = acc[t][3] = 0.0;
  auto add = [&](double (&a)[4], float4 v) {
    a[0] += (double)v.x;
    a[1] += (double)v.y;
    a[2] += (double)v.z;
    a[3] += (double)v.w;
  };
  int64_t p = p0;
  for (; p + 4 <= p1; p += 4) {
    const float* r0 = X + (int64_t)members[p] * ldx;
    const float* r1 = X + (int64_t)members[p + 1] * ldx;
    const float* r2 = X + (int64_t)members[p + 2] * ldx;
    const float* r3 = X + (int64_t)members[p + 3] * ldx;
#pragma unroll
    for (int t = 0; t < T4; ++t) {
      const int dim = 4 * lane + 256 * t;
      if (dim < d) {
        const float4 v0 = *reinterpret_cast<const float4*>(r0 + dim);
        const float4 v1 = *reinterpret_cast<const float4*>(r1 + dim);
        const float4 v2 = *reinterpret_cast<const float4*>(r2 + dim);
        const float4 v3 = *reinterpret_cast<const float4*>(r3 + dim);
        add(acc[t], v0);
        add(acc[t], v1);
        add(acc[t], v2);
        add(acc[t], v3);
      }
    }
  }
  for (; p < p1; ++p) {
    const float* r0 = X + (int64_t)members[p] * ldx;
#pragma unroll
    for (int t = 0; t < T4; ++t) {
      const int dim = 4 * lane + 256 * t;
      if (dim < d) add(acc[t], *reinterpret_cast<const float4*>(r0 + dim));
    }
  }
  double* out = partial + c * d;
#pragma unroll
  for (int t = 0; t < T4; ++t) {
    const int dim = 4 * lane + 256 * t;
    if (dim < d) {
      out[dim] = acc[t][0];
      out[dim + 1] = acc[t][1];
      out[dim + 2] = acc[t][2];
      out[dim + 3] = acc[t][3];
    }
  }
}

template <int T>
__global__ __launch_bounds__(256) void k_seg_final(int d, int32_t k, const int32_t* __restrict__ counts,
                                                   const int32_t* __restrict__ chunk_off,
                                                   const double* __restrict__ partial,
                                                   float* __restrict__ C, double* __restrict__ sums,
                                                   double* __restrict__ Iterm, float* __restrict__ delta) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= k) return;
  const int32_t cnt = counts[r];
  double s[T];
#pragma unroll
  for (int t = 0; t < T; ++t) s[t] = 0.0;
  for (int32_t c = chunk_off[r]; c < chunk_off[r + 1]; ++c) {
    const double* pr = partial + (int64_t)c * d;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      int dim = lane + 64 * t;
      if (dim < d) s[t] += pr[dim];
    }
  }
  double sq = 0.0, mv = 0.0;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    int dim = lane + 64 * t;
    if (dim < d) {
      if (sums) sums[r * d + dim] = s[t];
      if (cnt > 0) {
        const float c = (float)(s[t] / (double)cnt);
        if (delta) {
          const double df = (double)c - (double)C[r * d + dim];  // exact: two float32 values
          mv = fma(df, df, mv);
        }
        C[r * d + dim] = c;
      }
      sq = fma(s[t], s[t], sq);
    }
  }
  sq = wave_sum(sq);
  if (lane == 0 && Iterm) Iterm[r] = cnt > 0 ? sq / (double)cnt : 0.0;
  // movement of the centroid (upper bound, float32), for the drift bounds
  // of the assignment
  if (delta) {
    mv = wave_sum(mv);
    if (lane == 0) delta[r] = f32_round_up(sqrt(mv) * (1.0 + 0x1p-40));
  }
}

knnkm_status ks_segsum(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                       int32_t k, const int32_t* counts, const int32_t* offsets,
                       const int32_t* members, float* C, double* sums, double* Iterm, float* delta) {
  KNNKM_WS(ctx, cc, int32_t, "seg_chunk_off", (int64_t)k + 1);
  k_chunk_counts<<<grid_for(k, 256, 4096), 256, 0, ctx->stream>>>(counts, k, cc);
  KNNKM_TRY(knnkm_check(ctx, "chunk counts"));
  KNNKM_TRY(ks_scan_exclusive(ctx, cc, cc, k, true));
  const int64_t max_chunks = (int64_t)k + (n + SEG_CHUNK - 1) / SEG_CHUNK;
  KNNKM_WS(ctx, partial, double, "seg_partial", max_chunks * d);
  const int T = (d + 63) / 64;
  const unsigned gp = (unsigned)((max_chunks + 3) / 4), gf = (unsigned)((k + 3) / 4);
  const bool wide4 = d > 256 && d % 4 == 0 && ldx % 4 == 0 && (uintptr_t)X % 16 == 0;
#define SEG(TT)                                                                                        \
  if (wide4)                                                                                           \
    k_seg_partial4<2><<<gp, 256, 0, ctx->stream>>>(X, d, ldx, k, offsets, members, cc, max_chunks,    \
                                                   partial);                                           \
  else                                                                                                 \
    k_seg_partial<TT><<<gp, 256, 0, ctx->stream>>>(X, d, ldx, k, offsets, members, cc, max_chunks,    \
                                                   partial);                                           \
  k_seg_final<TT><<<gf, 256, 0, ctx->stream>>>(d, k, counts, cc, partial, C, sums, Iterm, delta)
  switch (T) {
    case 1: SEG(1); break;
    case 2: SEG(2); break;
    case 3: SEG(3); break;
    case 4: SEG(4); break;
    case 5: SEG(5); break;
    case 6: SEG(6); break;
    case 7: SEG(7); break;
    case 8: SEG(8); break;
    default: return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "d=%d > %d", d, KNNKM_MAX_D);
  }
#undef SEG
  return knnkm_check(ctx, "segsum");
}

// ------------------------------------------------------------- distortion --
// One wave per sample: float64 ||x_i - C_{l_i}||^2 (or ||x_i||^2 when C is
// null).  Block b covers samples [256b, 256b+256); wave w takes every 4th.
template <int T>
__global__ __launch_bounds__(256) void k_sqdist_blocks(const float* __restrict__ X, int64_t n, int d,
                                                       int64_t ldx, const float* __restrict__ C,
                                                       const int32_t* __restrict__ labels,
                                                       double* __restrict__ partial) {
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * 256;
  double tot = 0.0;
  for (int j = w; j < 256; j += 4) {
    int64_t i = base + j;
    if (i >= n) break;
    const float* xr = X + i * ldx;
    const float* cr = C ? C + (int64_t)labels[i] * d : nullptr;
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      int dim = lane + 64 * t;
      if (dim < d) {
        double df = (double)xr[dim] - (cr ? (double)cr[dim] : 0.0);
        acc = fma(df, df, acc);
      }
    }
    tot += wave_sum(acc);
  }
  if (lane == 0) sh[w] = tot;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ void k_scale_f64(double* v, double s) {
  if (threadIdx.x == 0) v[0] *= s;
}

// sum_i ||x_i - C_{l_i}||^2 (scaled by `scale`) into *out.
knnkm_status ks_sqdist_sum(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                           const float* C, const int32_t* labels, double* out, double scale) {
  const int64_t blocks = (n + 255) / 256;
  KNNKM_WS(ctx, part, double, "dist_part", blocks);
  const int T = (d + 63) / 64;
#define DL(TT) k_sqdist_blocks<TT><<<(unsigned)blocks, 256, 0, ctx->stream>>>(X, n, d, ldx, C, labels, part)
  switch (T) {
    case 1: DL(1); break;
    case 2: DL(2); break;
    case 3: DL(3); break;
    case 4: DL(4); break;
    case 5: DL(5); break;
    case 6: DL(6); break;
    case 7: DL(7); break;
    case 8: DL(8); break;
    default: return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "d=%d > %d", d, KNNKM_MAX_D);
  }
#undef DL
  KNNKM_TRY(knnkm_check(ctx, "distortion blocks"));
  KNNKM_TRY(ks_sum_f64(ctx, part, blocks, out));
  if (scale != 1.0) {
    k_scale_f64<<<1, 64, 0, ctx->stream>>>(out, scale);
    return knnkm_check(ctx, "distortion scale");
  }
  return KNNKM_OK;
}

static knnkm_status check_common(knnkm_ctx* ctx, const char* who, const float* X, int64_t n, int32_t d,
                                 int64_t ldx, int32_t k) {
  if (!ctx) return KNNKM_EINVAL;
  if (ctx->sticky) return KNNKM_EDEVICE;
  if (!X) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: X is null", who);
  if (n < 1 || n > INT32_MAX) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: n out of range", who);
  if (d < 1 || ldx < d) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: need d >= 1 and ldx >= d", who);
  if (d > KNNKM_MAX_D) return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "%s: d=%d > %d", who, d, KNNKM_MAX_D);
  if (k < 1 || k > n) return knnkm_fail(ctx, KNNKM_EINVAL, "%s: need 1 <= k <= n", who);
  return KNNKM_OK;
}

extern "C" knnkm_status centroid_update(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d,
                                        int64_t ldx, const int32_t* labels, int32_t k, float* C,
                                        int32_t* counts, double* sums) {
  KNNKM_TRY(check_common(ctx, "centroid_update", X, n, d, ldx, k));
  if (!labels || !C || !counts) return knnkm_fail(ctx, KNNKM_EINVAL, "centroid_update: null pointer");
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  KNNKM_WS(ctx, off, int32_t, "cu_offsets", (int64_t)k + 1);
  KNNKM_WS(ctx, mem, int32_t, "cu_members", n);
  KNNKM_TRY(ks_label_sort(ctx, labels, n, k, counts, off, mem));
  return ks_segsum(ctx, X, n, d, ldx, k, counts, off, mem, C, sums, nullptr);
}

extern "C" knnkm_status distortion(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                   const float* C, int32_t k, const int32_t* labels, double* E) {
  KNNKM_TRY(check_common(ctx, "distortion", X, n, d, ldx, k));
  if (!labels || !C || !E) return knnkm_fail(ctx, KNNKM_EINVAL, "distortion: null pointer");
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  return ks_sqdist_sum(ctx, X, n, d, ldx, C, labels, E, 1.0 / (double)n);
}

// ------------------------------------------------ allocation-free distortion --
// distortion_noalloc keeps its per-block partial sums (and, past 65,536
// blocks, the partials of their sum) in this fixed array instead of the
// context workspace.  Each device holds its own copy until the process ends;
// host code uses only the device address resolved below, never the array's
// name.  Every call overwrites what it reads, so nothing needs clearing; calls
// that overlap on one device race on it.
#define NOALLOC_SCRATCH_DOUBLES (1 << 19) /* 4 MiB */
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
static std::mutex g_scratch_mu;
static double* g_scratch_dev[64] = {};  // per device, resolved once

knnkm_status ks_noalloc_setup(knnkm_ctx* ctx) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (ctx->device < 0 || ctx->device >= 64)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "device %d: the fixed scratch supports devices 0..63", ctx->device);
  if (g_scratch_dev[ctx->device]) return KNNKM_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return knnkm_fail(ctx, KNNKM_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  }
  g_scratch_dev[ctx->device] = (double*)ptr;
  return KNNKM_OK;
}

extern "C" knnkm_status distortion_noalloc(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                           const float* C, int32_t k, const int32_t* labels, double* E) {
  KNNKM_TRY(check_common(ctx, "distortion_noalloc", X, n, d, ldx, k));
  if (!labels || !C || !E) return knnkm_fail(ctx, KNNKM_EINVAL, "distortion_noalloc: null pointer");
  const int64_t blocks = (n + 255) / 256;
  const int64_t tiles = blocks > 65536 ? (blocks + 8191) / 8192 : 0;
  if (blocks + tiles > NOALLOC_SCRATCH_DOUBLES)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED,
                      "distortion_noalloc: n=%lld needs %lld scratch doubles, the fixed scratch holds %d "
                      "(n <= 134,201,344)",
                      (long long)n, (long long)(blocks + tiles), NOALLOC_SCRATCH_DOUBLES);
  if (ctx->dry) return KNNKM_OK;
  KNNKM_HIP(ctx, hipSetDevice(ctx->device));
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    part = g_scratch_dev[ctx->device];
  }
  if (!part) return knnkm_fail(ctx, KNNKM_EDEVICE, "distortion_noalloc: scratch not resolved for this device");
  const int T = (d + 63) / 64;
#define DL(TT) k_sqdist_blocks<TT><<<(unsigned)blocks, 256, 0, ctx->stream>>>(X, n, d, ldx, C, labels, part)
  switch (T) {
    case 1: DL(1); break;
    case 2: DL(2); break;
    case 3: DL(3); break;
    case 4: DL(4); break;
    case 5: DL(5); break;
    case 6: DL(6); break;
    case 7: DL(7); break;
    default: DL(8); break;
  }
#undef DL
  KNNKM_TRY(knnkm_check(ctx, "distortion_noalloc blocks"));
  KNNKM_TRY(ks_sum_f64_with(ctx, part, blocks, part + blocks, E));
  k_scale_f64<<<1, 64, 0, ctx->stream>>>(E, 1.0 / (double)n);
  return knnkm_check(ctx, "distortion_noalloc scale");
}
