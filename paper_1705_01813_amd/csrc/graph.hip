// KNN graph construction pieces (Alg. 3).
//
// graph_init: random initial lists.  One wavefront per row: Floyd's sampling
//   of kappa distinct values of [0, n-1) (one counter-based draw per step,
//   membership by ballot over the lanes that hold the chosen ids), shifted
//   past the row's own id; squared distances in float64 (rounded to float32);
//   the row is ordered by (d2, id) through per-lane ranks.
//
// refine: the exhaustive comparison inside every cluster and the list
//   update.  Work item = (cluster, block of 32 rows); the block walks all
//   32-member column blocks of its cluster:
//     1. the 32 row and 32 column samples are staged in LDS (float32);
//     2. their 32 x 32 Gram block runs on MFMA (float32 16x16x4, or bfloat16
//        16x16x32 in the precision form), four 16 x 16 tiles, one per wave;
//     3. d^2 estimates ||x||^2 + ||y||^2 - 2 x.y minus a rigorous error bound
//        are compared with the row's current kappa-th distance; pairs already
//        in the row (visited) are dropped;
//     4. survivors get their exact distance (float64 direct difference from
//        LDS, rounded to float32);
//     5. each row merges its survivors into its sorted list (per-lane ranks).
//   Every row belongs to exactly one cluster, so rows are updated without
//   atomics.  Both precisions produce the same graph: the screen only removes
//   pairs that provably cannot enter.
#include <cfloat>

#include "common.h"

// ------------------------------------------------------------- graph init --
template <int T>
__global__ __launch_bounds__(256) void k_graph_init(const float* __restrict__ X, int n, int d,
                                                    int64_t ldx, int kappa, uint64_t seed,
                                                    int32_t* __restrict__ G_ids,
                                                    float* __restrict__ G_d2) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const uint64_t key = sm_key(seed, sm_stream(RNG_GRAPH_INIT, 0, (uint64_t)i));
  const uint32_t m = (uint32_t)(n - 1);
  const uint32_t base = m - (uint32_t)kappa;
  int v0 = -1, v1 = -1;  // chosen value for slot lane, lane+64
  for (int c = 0; c < kappa; ++c) {
    const uint32_t j = base + (uint32_t)c;
    const int t = (int)sm_below(sm_draw(key, (uint64_t)c), j + 1);
    const bool seen = (__ballot(v0 == t) | __ballot(v1 == t)) != 0ull;
    const int v = seen ? (int)j : t;
    if (c < 64) {
      if (lane == c) v0 = v;
    } else if (lane == c - 64) {
      v1 = v;
    }
  }
  // shift past the row's own id
  int id0 = v0 >= 0 ? v0 + (v0 >= i ? 1 : 0) : -1;
  int id1 = v1 >= 0 ? v1 + (v1 >= i ? 1 : 0) : -1;
  // distances: one float64 reduction per entry
  float x[T];
  const float* xr = X + i * ldx;
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
  int32_t* gi = G_ids + i * kappa;
  float* gd = G_d2 + i * kappa;
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
                           int32_t kappa, uint64_t seed, int32_t* G_ids, float* G_d2) {
  const int T = (d + 63) / 64;
  const unsigned grid = (unsigned)((n + 3) / 4);
#define GI(TT) k_graph_init<TT><<<grid, 256, 0, ctx->stream>>>(X, (int)n, d, ldx, kappa, seed, G_ids, G_d2)
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
#define RB 32  // rows / columns per block

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

struct RefineLDS {
  // layout (dynamic LDS):
  //   xi[RB][ld], xj[RB][ld]   float32 samples, ld = dpad + 1
  //   rk[RB][kappa], ri[RB][kappa]  current row lists
  //   ck[RB][RB], ci[RB][RB]   survivors per row
  //   ni[RB], nj[RB], cnt[RB], thr[RB]
  //   ids_i[RB], ids_j[RB]
};

__device__ inline bool key_lt(float ka, int ia, float kb, int ib) {
  return ka < kb || (ka == kb && ia < ib);
}

template <bool BF16>
__global__ __launch_bounds__(256) void k_refine(const float* __restrict__ X, int d, int64_t ldx,
                                                int dpad, int kappa, int32_t k,
                                                const int32_t* __restrict__ offsets,
                                                const int32_t* __restrict__ members,
                                                const int32_t* __restrict__ wb_off,
                                                int64_t max_items, float err_c,
                                                int32_t* __restrict__ G_ids,
                                                float* __restrict__ G_d2) {
  extern __shared__ __align__(16) char smem[];
  const int ld = dpad + 1;
  float* xi = (float*)smem;
  float* xj = xi + RB * ld;
  float* rk = xj + RB * ld;
  int32_t* ri = (int32_t*)(rk + RB * kappa);
  float* ck = (float*)(ri + RB * kappa);
  int32_t* ci = (int32_t*)(ck + RB * RB);
  float* ni = (float*)(ci + RB * RB);
  float* nj = ni + RB;
  float* thr = nj + RB;
  int32_t* cnt = (int32_t*)(thr + RB);
  int32_t* ids_i = cnt + RB;
  int32_t* ids_j = ids_i + RB;

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t item = blockIdx.x;
  if (item >= max_items) return;
  const int32_t total = wb_off[k];
  if (item >= total) return;
  int lo = 0, hi = k;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (wb_off[mid] <= item) lo = mid; else hi = mid;
  }
  const int cl = lo;
  const int c0 = offsets[cl], s = offsets[cl + 1] - c0;
  const int rb0 = (int)(item - wb_off[cl]) * RB;
  const int nrows = min(RB, s - rb0);

  // stage rows, their lists and norms
  for (int r = threadIdx.x; r < RB; r += 256) {
    ids_i[r] = r < nrows ? members[c0 + rb0 + r] : -1;
    cnt[r] = 0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < RB * dpad; e += 256) {
    const int r = e / dpad, t = e % dpad;
    xi[r * ld + t] = (r < nrows && t < d) ? X[(int64_t)ids_i[r] * ldx + t] : 0.f;
  }
  for (int e = threadIdx.x; e < RB * kappa; e += 256) {
    const int r = e / kappa, c = e % kappa;
    if (r < nrows) {
      rk[e] = G_d2[(int64_t)ids_i[r] * kappa + c];
      ri[e] = G_ids[(int64_t)ids_i[r] * kappa + c];
    }
  }
  __syncthreads();
  for (int r = w; r < RB; r += 4) {
    float a = 0.f;
    for (int t = lane; t < dpad; t += 64) a = fmaf(xi[r * ld + t], xi[r * ld + t], a);
    a = wave_sum(a);
    if (lane == 0) {
      ni[r] = a;
      thr[r] = r < nrows ? rk[r * kappa + kappa - 1] : -FLT_MAX;
    }
  }
  __syncthreads();

  for (int cb0 = 0; cb0 < s; cb0 += RB) {
    const int ncols = min(RB, s - cb0);
    for (int r = threadIdx.x; r < RB; r += 256) ids_j[r] = r < ncols ? members[c0 + cb0 + r] : -1;
    __syncthreads();
    for (int e = threadIdx.x; e < RB * dpad; e += 256) {
      const int r = e / dpad, t = e % dpad;
      xj[r * ld + t] = (r < ncols && t < d) ? X[(int64_t)ids_j[r] * ldx + t] : 0.f;
    }
    __syncthreads();
    for (int r = w; r < RB; r += 4) {
      float a = 0.f;
      for (int t = lane; t < dpad; t += 64) a = fmaf(xj[r * ld + t], xj[r * ld + t], a);
      a = wave_sum(a);
      if (lane == 0) nj[r] = a;
    }
    __syncthreads();

    // Gram tile of this wave: rows 16*(w>>1).., cols 16*(w&1)..
    const int tr = 16 * (w >> 1), tc = 16 * (w & 1);
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
    // screen: lane holds column tc + (lane & 15), rows tr + 4*(lane>>4) + e
    {
      const int c = tc + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = tr + 4 * (lane >> 4) + e;
        if (r < nrows && c < ncols) {
          const int idi = ids_i[r], idj = ids_j[c];
          if (idi != idj) {
            const float sn = ni[r] + nj[c];
            const float est = sn - 2.f * acc[e];
            const float lb = est - err_c * sn;
            const float th = thr[r];
            if (lb <= th + th * 0x1p-22f + 1e-30f) {
              bool dup = false;
              for (int q = 0; q < kappa; ++q) dup |= (ri[r * kappa + q] == idj);
              if (!dup) {
                const int slot = atomicAdd(&cnt[r], 1);
                ci[r * RB + slot] = c;  // column index for now
              }
            }
          }
        }
      }
    }
    __syncthreads();
    // exact distances of survivors: thread per (row, slot)
    for (int e = threadIdx.x; e < RB * RB; e += 256) {
      const int r = e / RB, slot = e % RB;
      if (slot < cnt[r]) {
        const int c = ci[r * RB + slot];
        const float* a = xi + r * ld;
        const float* b = xj + c * ld;
        double acc2 = 0.0;
        for (int t = 0; t < d; ++t) {
          const double df = (double)a[t] - (double)b[t];
          acc2 = fma(df, df, acc2);
        }
        ck[r * RB + slot] = (float)acc2;
        ci[r * RB + slot] = ids_j[c];
      }
    }
    __syncthreads();
    // merge: one wave per row
    for (int r = w; r < RB; r += 4) {
      const int m = cnt[r];
      if (r < nrows && m > 0) {
        const float cv = lane < m ? ck[r * RB + lane] : FLT_MAX;
        const int cid = lane < m ? ci[r * RB + lane] : INT32_MAX;
        // row entries in two slots
        const float e0k = lane < kappa ? rk[r * kappa + lane] : FLT_MAX;
        const int e0i = lane < kappa ? ri[r * kappa + lane] : INT32_MAX;
        const float e1k = lane + 64 < kappa ? rk[r * kappa + lane + 64] : FLT_MAX;
        const int e1i = lane + 64 < kappa ? ri[r * kappa + lane + 64] : INT32_MAX;
        int pos_c = 0;  // candidate rank among row entries and other candidates
        for (int q = 0; q < kappa; ++q) {
          const float qk = rk[r * kappa + q];
          const int qi = ri[r * kappa + q];
          pos_c += key_lt(qk, qi, cv, cid) ? 1 : 0;
        }
        int add0 = 0, add1 = 0;
        for (int q = 0; q < m; ++q) {
          const float qk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cv), q));
          const int qi = __builtin_amdgcn_readlane(cid, q);
          pos_c += key_lt(qk, qi, cv, cid) ? 1 : 0;
          add0 += key_lt(qk, qi, e0k, e0i) ? 1 : 0;
          add1 += key_lt(qk, qi, e1k, e1i) ? 1 : 0;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < kappa && lane + add0 < kappa) {
          rk[r * kappa + lane + add0] = e0k;
          ri[r * kappa + lane + add0] = e0i;
        }
        if (lane + 64 < kappa && lane + 64 + add1 < kappa) {
          rk[r * kappa + lane + 64 + add1] = e1k;
          ri[r * kappa + lane + 64 + add1] = e1i;
        }
        if (lane < m && pos_c < kappa) {
          rk[r * kappa + pos_c] = cv;
          ri[r * kappa + pos_c] = cid;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) thr[r] = rk[r * kappa + kappa - 1];
      }
      if (lane == 0) cnt[r] = 0;
    }
    __syncthreads();
  }
  // write rows back
  for (int e = threadIdx.x; e < RB * kappa; e += 256) {
    const int r = e / kappa, c = e % kappa;
    if (r < nrows) {
      G_d2[(int64_t)ids_i[r] * kappa + c] = rk[e];
      G_ids[(int64_t)ids_i[r] * kappa + c] = ri[e];
    }
  }
}

__global__ void k_row_blocks(const int32_t* __restrict__ counts, int32_t k, int32_t* wb) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < k;
       r += (int64_t)gridDim.x * blockDim.x)
    wb[r] = (counts[r] + RB - 1) / RB;
}

size_t refine_lds_bytes(int d, int kappa) {
  const int dpad = (d + 31) / 32 * 32;
  const int ld = dpad + 1;
  return (size_t)4 * (2 * RB * ld + 2 * RB * kappa + 2 * RB * RB + 4 * RB + 2 * RB);
}

knnkm_status ks_refine(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                       const int32_t* labels, int32_t k, int32_t precision, int32_t* G_ids,
                       float* G_d2, int32_t kappa) {
  const size_t lds = refine_lds_bytes(d, kappa);
  if (lds > 160 * 1024)
    return knnkm_fail(ctx, KNNKM_EUNSUPPORTED, "graph refine: d=%d with kappa=%d needs %zu B of LDS", d,
                      kappa, lds);
  KNNKM_WS(ctx, counts, int32_t, "rf_counts", k);
  KNNKM_WS(ctx, off, int32_t, "rf_offsets", (int64_t)k + 1);
  KNNKM_WS(ctx, mem, int32_t, "rf_members", n);
  KNNKM_WS(ctx, wb, int32_t, "rf_wb", (int64_t)k + 1);
  KNNKM_TRY(ks_label_sort(ctx, labels, n, k, counts, off, mem));
  k_row_blocks<<<grid_for(k, 256, 4096), 256, 0, ctx->stream>>>(counts, k, wb);
  KNNKM_TRY(knnkm_check(ctx, "refine blocks"));
  KNNKM_TRY(ks_scan_exclusive(ctx, wb, wb, k, true));
  const int64_t max_items = (int64_t)k + (n + RB - 1) / RB;
  const int dpad = (d + 31) / 32 * 32;
  // Screening bound (squared-distance units, relative to ||x||^2 + ||y||^2),
  // twice the worst-case rounding analysis; see the design notes.
  const double u = 0x1p-24;
  double err = (2.0 * dpad + 8.0) * u;
  if (precision == KNNKM_BF16_RERANK) err += 2.0 * (0x1p-7 + 0x1p-15);
  const float err_c = (float)(2.0 * err);
  if (precision == KNNKM_BF16_RERANK) {
    hipFuncSetAttribute((const void*)k_refine<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_refine<true><<<(unsigned)max_items, 256, lds, ctx->stream>>>(X, d, ldx, dpad, kappa, k, off, mem, wb,
                                                                   max_items, err_c, G_ids, G_d2);
  } else {
    hipFuncSetAttribute((const void*)k_refine<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_refine<false><<<(unsigned)max_items, 256, lds, ctx->stream>>>(X, d, ldx, dpad, kappa, k, off, mem, wb,
                                                                    max_items, err_c, G_ids, G_d2);
  }
  return knnkm_check(ctx, "graph refine");
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
