// Incremental centroid update for the fit sweeps (Sec. 1 Lloyd update written
// with the composite vectors D_r of Eqn. 2: a sample that moves from u to v
// subtracts its row from D_u and adds it to D_v, as in the paper's own
// update of D_u and D_v for a move).
//
// D_r is held per (cluster, dimension) as a 128-bit two's-complement fixed
// point number, value * 2^s with one exponent s per job chosen from the
// job's largest |x| so that no sum can overflow (n |x| 2^s < 2^125).  Adding
// a float32 row value is exact (its 24-bit significand lands on integer bits
// unless it is 2^71 times smaller than the job's largest value), and integer
// additions are associative, so the sums are exact and independent of the
// order in which the moves are applied (atomics in any order give the same
// bits).  Only the moved samples are touched each sweep; a cluster whose
// members changed gets C_r = float32(D_r / n_r) (rounded to float64 first)
// and the Eqn. 2 term ||D_r||^2 / n_r.
#include "fixed128.h"
#include "rowgroup.h"

// Multi-word atomic add: the carry out of the low word is known from the
// value the low-word atomic returns.
__device__ inline void fx_atomic_add(uint64_t* p, uint64_t hi, uint64_t lo) {
  if (lo) {
    const uint64_t old = atomicAdd((unsigned long long*)p, (unsigned long long)lo);
    if (old + lo < old) hi += 1;
  }
  if (hi) atomicAdd((unsigned long long*)(p + 1), (unsigned long long)hi);
}

// Per-row statistics in one pass over X: ||x_i||^2 in float64 (the Eqn. 2
// identity of the distortion) and the largest |x| of every job, as the bits
// of a non-negative float (ordered like the floats, so an atomic max of the
// bits is exact in any order).  Row groups of L lanes (V dimensions each)
// take a contiguous run of rows per wavefront; each lane keeps a running
// maximum that is reduced and published when its row's job changes (rare)
// and at the end, where a block combines its groups first, so one atomic
// per block and job reaches memory (many atomics on one job's word would
// serialise).
template <int L, int V>
__global__ __launch_bounds__(256) void k_row_stats(const float* __restrict__ X, int64_t n, int d, int64_t ldx,
                                                   int vec, const int32_t* __restrict__ job_of,
                                                   double* __restrict__ rowsq, uint32_t* __restrict__ jmax) {
  constexpr int GW = 64 / L;
  __shared__ int32_t sjob[4 * GW];
  __shared__ float smax[4 * GW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane / L, j = lane % L;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t per = ((n + nwaves - 1) / nwaves + GW - 1) / GW * GW;
  const int64_t i0 = wave * per, i1 = min(n, i0 + per);
  float mx = 0.f;
  int job = -1;
  for (int64_t r0 = i0; r0 < i1; r0 += GW) {
    const int64_t i = r0 + g;
    const bool act = i < i1;  // group-uniform
    if (!act) continue;
    const int q = job_of ? job_of[i] : 0;
    if (q != job) {  // group-uniform
      if (job >= 0) {
        const float wm = group_max<L>(mx);
        if (j == 0) atomicMax(&jmax[job], __float_as_uint(wm));
      }
      job = q;
      mx = 0.f;
    }
    float x[V];
    load_row<V>(x, X + i * ldx, j, d, vec != 0);
    double a = 0.0;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      mx = fmaxf(mx, fabsf(x[e]));
      a = fma((double)x[e], (double)x[e], a);
    }
    a = group_sum<L>(a);
    if (j == 0) rowsq[i] = a;
  }
  float gm = 0.f;
  if (job >= 0) gm = group_max<L>(mx);  // group-uniform
  if (j == 0) {
    sjob[w * GW + g] = job;
    smax[w * GW + g] = gm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int cj = -1;
    float cm = 0.f;
    for (int t = 0; t < 4 * GW; ++t) {
      const int q = sjob[t];
      if (q < 0) continue;
      if (q != cj) {
        if (cj >= 0) atomicMax(&jmax[cj], __float_as_uint(cm));
        cj = q;
        cm = 0.f;
      }
      cm = fmaxf(cm, smax[t]);
    }
    if (cj >= 0) atomicMax(&jmax[cj], __float_as_uint(cm));
  }
}

// scale exponent of every cluster from its job's largest |x|: s = 94 - e
// with max |x| < 2^e (0 for a job of zeros)
__global__ void k_cluster_scale(const uint32_t* __restrict__ jmax, const int32_t* __restrict__ k_off, int m,
                                int32_t K, int32_t* __restrict__ cs) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < K; r += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = m;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (k_off[mid] <= r) lo = mid; else hi = mid;
    }
    const float mxv = __uint_as_float(jmax[lo]);
    int e = 0;
    if (mxv > 0.f) (void)frexpf(mxv, &e);
    cs[r] = mxv > 0.f ? 94 - e : 0;
  }
}

__global__ void k_fx_from_f64(const double* __restrict__ sums, int64_t kd, int d, const int32_t* __restrict__ cs,
                              uint64_t* __restrict__ D) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < kd; e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t hi, lo;
    fx_of_double(sums[e], cs[e / d], hi, lo);
    D[2 * e] = lo;
    D[2 * e + 1] = hi;
  }
}

// Active sets: a moved sample, and every sample that has it as a neighbour
// (reverse lists rev_off/rev_src of the fixed graph), have a new candidate
// set for the next sweep; bit 1 of their flag says so.  Bit 0 says that a
// candidate centroid of the sample changed (k_mark_dirty).  Within one
// kernel every writer of a flag sets the same bit of a value no other
// kernel is writing at the time, so all of them store the same byte and the
// order of the stores does not matter.
template <int BIT>
__device__ inline void mark_one(uint8_t* __restrict__ act_out, int64_t x) { act_out[x] = act_out[x] | BIT; }
// Whole wave: the marks of every selected sample of the wave (lane q holds
// position p and `moved`), the wave's marks laid end to end over the lanes
// (sample q owns entries [ex_q, ex_q + 1 + its reverse-list length); its
// first entry is the sample itself), so all of them are in flight at once.
// A reverse-list entry is the graph entry (row * kappa + position) that
// lists the sample.  With nlab (the labels of every graph entry, row-major
// n x kappa) those entries also receive the sample's new label lab_new.
template <int BIT = 2>
__device__ inline void mark_moved_wave(bool moved, int64_t p, const int32_t* __restrict__ rev_off,
                                       const int32_t* __restrict__ rev_src, uint8_t* __restrict__ act_out,
                                       int lane, int kappa, int32_t* __restrict__ nlab = nullptr, int lab_new = 0) {
  int32_t r0 = 0, c = 0;
  if (moved) {
    r0 = rev_off[p];
    c = 1 + rev_off[p + 1] - r0;
  }
  int32_t inc = c;  // inclusive scan of the entry counts over the lanes
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  const int32_t total = __shfl(inc, 63, 64);
  for (int32_t e0 = 0; e0 < total; e0 += 64) {  // wave-uniform: every lane takes part in the shuffles
    const int32_t e = e0 + lane;
    int q = 0;  // owner: the first lane whose inclusive count exceeds e
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
      if (__shfl(inc, q + step - 1, 64) <= e) q += step;
    q = min(q, 63);
    const int32_t local = e - (__shfl(inc, q, 64) - __shfl(c, q, 64));
    const int32_t rq = __shfl(r0, q, 64);
    const int64_t pq = __shfl(p, q, 64);
    const int32_t src = e < total && local > 0 ? rev_src[rq + local - 1] : 0;
    if (e < total) mark_one<BIT>(act_out, local == 0 ? pq : (int64_t)(src / kappa));
    if (nlab) {  // wave-uniform
      const int lq = __shfl(lab_new, q, 64);
      if (e < total && local > 0) nlab[src] = lq;
    }
  }
}

// 128-bit two's-complement accumulation in registers
__device__ inline void add128(uint64_t& h, uint64_t& l, uint64_t bh, uint64_t bl) {
  const uint64_t nl = l + bl;
  h += bh + (nl < l ? 1ull : 0ull);
  l = nl;
}

// Every moved sample: its row out of D[old], into D[new]; sizes and dirty
// flags of both clusters.  With act_out (active sets) also its marks, its
// new label written over the old one in cur, so that the two label arrays
// agree outside the samples the next sweep writes, and (nlab non-null) into
// the graph-entry labels of the rows that list it.  A wavefront scans
// 64 positions and takes its moved samples in order, lanes over the
// dimensions (DPL per lane); consecutive moved samples that leave the same
// cluster (or join the same one), common in the cluster-ordered working
// copy, are summed in registers first and reach D with one atomic per run
// and dimension (integer sums: the same bits in any grouping).
template <int DPL>
__global__ __launch_bounds__(256) void k_fx_moves(const float* __restrict__ X, int64_t n, int d,
                                                  int32_t* __restrict__ cur, const int32_t* __restrict__ nxt,
                                                  const int32_t* __restrict__ cs, uint64_t* __restrict__ D,
                                                  int32_t* __restrict__ counts, int32_t* __restrict__ dirty,
                                                  const int32_t* __restrict__ rev_off,
                                                  const int32_t* __restrict__ rev_src, uint8_t* __restrict__ act_out,
                                                  int32_t* __restrict__ nlab, int kappa) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
    const int64_t p = base + lane;
    int a = -1, b = -1;
    if (p < n) {
      a = cur[p];
      b = nxt[p];
    }
    const bool moved = p < n && a != b;
    if (moved) {
      atomicAdd(&counts[a], -1);
      atomicAdd(&counts[b], 1);
      atomicOr(&dirty[a], 1);
      atomicOr(&dirty[b], 1);
      if (act_out) cur[p] = b;
    }
    uint64_t M = __ballot(moved);
    if (!M) continue;  // wave-uniform
    if (act_out) mark_moved_wave(moved, p, rev_off, rev_src, act_out, lane, kappa, nlab, b);
    int run_from = -1, run_to = -1;
    uint64_t fh[DPL], fl[DPL], th[DPL], tl[DPL];
#pragma unroll
    for (int e = 0; e < DPL; ++e) fh[e] = fl[e] = th[e] = tl[e] = 0;
    auto flush = [&](uint64_t (&h)[DPL], uint64_t (&l)[DPL], int r) {
#pragma unroll
      for (int e = 0; e < DPL; ++e) {
        const int t = lane + 64 * e;
        if (t < d) fx_atomic_add(D + 2 * ((int64_t)r * d + t), h[e], l[e]);
        h[e] = l[e] = 0;
      }
    };
    // the next moved sample's row is loaded while this one is converted
    float xn[DPL];
    auto load = [&](int q) {
      const float* row = X + (base + q) * (int64_t)d;
#pragma unroll
      for (int e = 0; e < DPL; ++e) xn[e] = lane + 64 * e < d ? row[lane + 64 * e] : 0.f;
    };
    load((int)__builtin_ctzll(M));
    for (; M; M &= M - 1) {
      const int q = (int)__builtin_ctzll(M);
      float xr[DPL];
#pragma unroll
      for (int e = 0; e < DPL; ++e) xr[e] = xn[e];
      if (M & (M - 1)) load((int)__builtin_ctzll(M & (M - 1)));
      const int from = __shfl(a, q, 64), to = __shfl(b, q, 64);
      if (from != run_from) {
        if (run_from >= 0) flush(fh, fl, run_from);
        run_from = from;
      }
      if (to != run_to) {
        if (run_to >= 0) flush(th, tl, run_to);
        run_to = to;
      }
      const int s = cs[to];  // both clusters belong to the sample's job
#pragma unroll
      for (int e = 0; e < DPL; ++e) {
        const int t = lane + 64 * e;
        if (t < d) {
          uint64_t hi, lo;
          fx_of_double((double)xr[e], s, hi, lo);
          add128(th[e], tl[e], hi, lo);
          fx_neg(hi, lo);
          add128(fh[e], fl[e], hi, lo);
        }
      }
    }
    flush(fh, fl, run_from);
    flush(th, tl, run_to);
  }
}

// Active-set marks of the moved samples alone (the sweep whose sums are
// rebuilt rather than updated), with their labels synchronised as above.
// When the sweep moved at least all_at samples (their reverse lists then
// cover most rows), every row is marked instead of the moved samples and the
// rows listing them: a superset of the marks, so the next sweep's results are
// the same, for one streaming pass instead of scattered marks.
__global__ __launch_bounds__(256) void k_mark_moved(int64_t n, int32_t* __restrict__ cur,
                                                    const int32_t* __restrict__ nxt,
                                                    const int32_t* __restrict__ rev_off,
                                                    const int32_t* __restrict__ rev_src, uint8_t* __restrict__ act_out,
                                                    const int64_t* __restrict__ moved, int64_t all_at, int kappa) {
  const int lane = threadIdx.x & 63;
  const bool all = *moved >= all_at;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
    const int64_t p = base + lane;
    int b = 0;
    const bool mv = p < n && cur[p] != (b = nxt[p]);
    if (mv) cur[p] = b;
    if (all) {
      if (p < n) mark_one<2>(act_out, p);
    } else if (__ballot(mv)) {
      mark_moved_wave(mv, p, rev_off, rev_src, act_out, lane, kappa);
    }
  }
}

// Active-set marks of changed centroids: every sample in a dirty cluster
// (labels lab, after the update) and every sample that lists it in its graph
// row has that cluster among its candidates, so bit 0 of their flags is set;
// a sample none of whose candidate centroids changed and whose candidate set
// is the same (bit 1 clear) has every input of its last decision and is not
// looked at.  A sample of a job with no more clusters than kappa has all of
// them as candidates and is always marked (job_of/kbase: jobs of a batch,
// null for one job).  With mass (the members of all dirty clusters) null or
// at least all_at, every sample is marked instead: one streaming pass in
// place of scattered marks that would cover most rows.
__global__ __launch_bounds__(256) void k_mark_dirty(int64_t n, const int32_t* __restrict__ lab,
                                                    const int32_t* __restrict__ dirty,
                                                    const int32_t* __restrict__ rev_off,
                                                    const int32_t* __restrict__ rev_src, uint8_t* __restrict__ act_out,
                                                    const int64_t* __restrict__ mass, int64_t all_at,
                                                    const int32_t* __restrict__ job_of,
                                                    const int32_t* __restrict__ kbase, int kappa) {
  const int lane = threadIdx.x & 63;
  const bool all = !mass || *mass >= all_at;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
    const int64_t p = base + lane;
    if (all) {
      if (p < n) mark_one<1>(act_out, p);
      continue;
    }
    bool sel = p < n && dirty[lab[p]] != 0;
    if (p < n && !sel && job_of) {
      const int q = job_of[p];
      sel = kappa >= kbase[q + 1] - kbase[q];
    }
    if (__ballot(sel)) mark_moved_wave<1>(sel, p, rev_off, rev_src, act_out, lane, kappa);
  }
}

// Reverse lists of a graph of n rows with kappa ids each: rev_src holds, for
// every target p in rev_off[p] .. rev_off[p+1], the graph entries (row *
// kappa + position, n * kappa < 2^31) that list p (in no particular order).
// Ids outside [0, n) are left out.
__global__ void k_rev_count(const int32_t* __restrict__ G, int64_t ne, int64_t n, int32_t* __restrict__ cnt) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t t = G[e];
    if (t >= 0 && t < n) atomicAdd(&cnt[t], 1);
  }
}
__global__ void k_rev_fill(const int32_t* __restrict__ G, int64_t ne, int64_t n, int kappa,
                           const int32_t* __restrict__ off, int32_t* __restrict__ cursor, int32_t* __restrict__ src) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t t = G[e];
    if (t < 0 || t >= n) continue;
    const int32_t pos = atomicAdd(&cursor[t], 1);
    src[off[t] + pos] = (int32_t)e;
  }
}

// Label of every graph entry: nlab[e] = lab[G[e]] (-1 for ids outside [0, n)).
__global__ void k_entry_labels(const int32_t* __restrict__ G, int64_t ne, int64_t n, const int32_t* __restrict__ lab,
                               int32_t* __restrict__ nlab) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t t = G[e];
    nlab[e] = t >= 0 && t < n ? lab[t] : -1;
  }
}

// Clusters whose members changed (dirty, set by this sweep's moves and kept
// for the next sweep's assignment): centroid (unchanged when empty) and the
// Eqn. 2 term; one wavefront per cluster.  dirty_clear, the previous
// sweep's flags, is cleared on the way; mass (nullable, cleared before)
// receives the number of members of all dirty clusters; sw (kind 0: none)
// the shadow of each new centroid and its bound; C64 (nullable) the float64
// mean D_r / n_r.  dirty null: every cluster.
__global__ __launch_bounds__(256) void k_fx_finalize(const uint64_t* __restrict__ D, int32_t K, int d,
                                                     const int32_t* __restrict__ cs,
                                                     const int32_t* __restrict__ counts,
                                                     const int32_t* __restrict__ dirty,
                                                     int32_t* __restrict__ dirty_clear, float* __restrict__ C,
                                                     double* __restrict__ Iterm, float* __restrict__ delta,
                                                     unsigned long long* __restrict__ mass, CShadow sw,
                                                     double* __restrict__ C64) {
  uint16_t* __restrict__ Cb = sw.kind == 1 ? (uint16_t*)sw.rows : nullptr;
  const int lane = threadIdx.x & 63;
  for (int64_t r = blockIdx.x * 4 + (threadIdx.x >> 6); r < K; r += (int64_t)gridDim.x * 4) {
    if (dirty_clear && lane == 0) dirty_clear[r] = 0;
    if (dirty && !dirty[r]) continue;  // wave-uniform
    const int cnt = counts[r];
    if (mass && lane == 0 && cnt > 0) atomicAdd(mass, (unsigned long long)cnt);
    const int s = cs[r];
    double sq = 0.0, mv = 0.0, e2 = 0.0;
    for (int t = lane; t < d; t += 64) {
      const int64_t e = r * d + t;
      const double v = fx_to_double(D[2 * e + 1], D[2 * e], s);
      if (cnt > 0) {
        const float c = (float)(v / (double)cnt);
        if (delta) {
          const double df = (double)c - (double)C[e];  // exact: two float32 values
          mv = fma(df, df, mv);
        }
        C[e] = c;
        if (C64) C64[e] = v / (double)cnt;
        if (Cb) {
          const uint16_t h = bf16_rne(c);
          Cb[e] = h;
          const double dq = (double)(c - __uint_as_float((uint32_t)h << 16));  // exact
          e2 = fma(dq, dq, e2);
        }
      }
      sq = fma(v, v, sq);
    }
    sq = wave_sum(sq);
    if (Cb && cnt > 0) {
      e2 = wave_sum(e2);
      if (lane == 0) sw.eps[r] = f32_round_up(sqrt(e2) * (1.0 + 0x1p-40));
    }
    // (the lanes read back the elements of the row they wrote)
    if (sw.kind == 2 && cnt > 0) i8_shadow_row(C + r * d, d, (uint8_t*)sw.rows + r * d, &sw.scale[r], &sw.eps[r]);
    if (lane == 0) Iterm[r] = cnt > 0 ? sq / (double)cnt : 0.0;
    if (delta) {
      mv = wave_sum(mv);
      if (lane == 0) delta[r] = f32_round_up(sqrt(mv) * (1.0 + 0x1p-40));
    }
  }
}

knnkm_status ks_row_stats(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, int m,
                          const int32_t* job_of, double* rowsq, uint32_t* jmax) {
  KNNKM_TRY(ks_fill_i32(ctx, (int32_t*)jmax, m, 0));
  int L, V;
  pick_group(d, 1, &L, &V);
  const int vec = (d % 4 == 0) && (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
  const unsigned grid = grid_for(n, 1024, 1024);
#define RS(LL, VV) k_row_stats<LL, VV><<<grid, 256, 0, ctx->stream>>>(X, n, d, ldx, vec, job_of, rowsq, jmax)
  if (V == 4) {
    switch (L) {
      case 4: RS(4, 4); break;
      case 8: RS(8, 4); break;
      case 16: RS(16, 4); break;
      case 32: RS(32, 4); break;
      default: RS(64, 4); break;
    }
  } else {
    switch (L) {
      case 4: RS(4, 8); break;
      case 8: RS(8, 8); break;
      case 16: RS(16, 8); break;
      case 32: RS(32, 8); break;
      default: RS(64, 8); break;
    }
  }
#undef RS
  return knnkm_check(ctx, "row statistics");
}

knnkm_status ks_fx_scales(knnkm_ctx* ctx, const uint32_t* jmax, int m, const int32_t* k_off, int32_t K,
                          int32_t* cs) {
  k_cluster_scale<<<grid_for(K, 256, 4096), 256, 0, ctx->stream>>>(jmax, k_off, m, K, cs);
  return knnkm_check(ctx, "fixed-point scales");
}

knnkm_status ks_fx_from_f64(knnkm_ctx* ctx, const double* sums, int32_t K, int32_t d, const int32_t* cs,
                            uint64_t* D) {
  const int64_t kd = (int64_t)K * d;
  k_fx_from_f64<<<grid_for(kd, 256, 16384), 256, 0, ctx->stream>>>(sums, kd, d, cs, D);
  return knnkm_check(ctx, "fixed-point sums");
}

knnkm_status ks_fx_update(knnkm_ctx* ctx, const float* Xp, int64_t n, int32_t d, int32_t* cur,
                          const int32_t* nxt, const int32_t* cs, uint64_t* D, int32_t K, int32_t* counts,
                          int32_t* dirty, float* C, double* Iterm, const int32_t* rev_off, const int32_t* rev_src,
                          uint8_t* act_out, int32_t* dirty_clear, float* delta, int64_t* mass, CShadow sw,
                          double* C64, int32_t* nlab, int32_t kappa) {
  if (mass) KNNKM_TRY(ks_fill_i64(ctx, mass, 1, 0));
#define MV(DD)                                                                                           \
  k_fx_moves<DD><<<grid_for(n, 256, 8192), 256, 0, ctx->stream>>>(Xp, n, d, cur, nxt, cs, D, counts, dirty, \
                                                                  rev_off, rev_src, act_out, nlab, kappa)
  if (d <= 64)
    MV(1);
  else if (d <= 128)
    MV(2);
  else if (d <= 256)
    MV(4);
  else
    MV(8);
#undef MV
  k_fx_finalize<<<grid_for(K, 4, 16384), 256, 0, ctx->stream>>>(D, K, d, cs, counts, dirty, dirty_clear, C, Iterm,
                                                                delta, (unsigned long long*)mass, sw, C64);
  return knnkm_check(ctx, "incremental update");
}

knnkm_status ks_mark_moved(knnkm_ctx* ctx, int64_t n, int32_t* cur, const int32_t* nxt, const int32_t* rev_off,
                           const int32_t* rev_src, uint8_t* act_out, const int64_t* moved, int64_t all_at,
                           int32_t kappa) {
  k_mark_moved<<<grid_for(n, 256, 8192), 256, 0, ctx->stream>>>(n, cur, nxt, rev_off, rev_src, act_out, moved,
                                                                all_at, kappa);
  return knnkm_check(ctx, "active-set marks");
}

// D_r of every cluster from its members (CSR off/mem), exactly: each row's
// value converted to the cluster's fixed point and added as a 128-bit
// integer; one wavefront per cluster, lanes over the dimensions.
__global__ __launch_bounds__(256) void k_fx_exact_sums(const float* __restrict__ X, int64_t ldx, int d, int32_t K,
                                                       const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ mem,
                                                       const int32_t* __restrict__ cs, uint64_t* __restrict__ D) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = blockIdx.x * 4 + (threadIdx.x >> 6); r < K; r += (int64_t)gridDim.x * 4) {
    const int s = cs[r];
    for (int t = lane; t < d; t += 64) {
      uint64_t h = 0, l = 0;
      for (int q = off[r]; q < off[r + 1]; ++q) {
        uint64_t bh, bl;
        fx_of_double((double)X[(int64_t)mem[q] * ldx + t], s, bh, bl);
        add128(h, l, bh, bl);
      }
      D[2 * (r * d + t)] = l;
      D[2 * (r * d + t) + 1] = h;
    }
  }
}

knnkm_status ks_fx_exact_sums(knnkm_ctx* ctx, const float* X, int64_t ldx, int32_t d, int32_t K, const int32_t* off,
                              const int32_t* mem, const int32_t* cs, uint64_t* D) {
  k_fx_exact_sums<<<grid_for(K, 4, 16384), 256, 0, ctx->stream>>>(X, ldx, d, K, off, mem, cs, D);
  return knnkm_check(ctx, "exact fixed-point sums");
}

knnkm_status ks_fx_finalize_all(knnkm_ctx* ctx, const uint64_t* D, int32_t K, int32_t d, const int32_t* cs,
                                const int32_t* counts, float* C, double* Iterm, double* C64) {
  k_fx_finalize<<<grid_for(K, 4, 16384), 256, 0, ctx->stream>>>(D, K, d, cs, counts, nullptr, nullptr, C, Iterm,
                                                                nullptr, nullptr, CShadow{}, C64);
  return knnkm_check(ctx, "centroids from fixed-point sums");
}

knnkm_status ks_mark_dirty(knnkm_ctx* ctx, int64_t n, const int32_t* lab, const int32_t* dirty,
                           const int32_t* rev_off, const int32_t* rev_src, uint8_t* act_out, const int64_t* mass,
                           int64_t all_at, const int32_t* job_of, const int32_t* kbase, int32_t kappa) {
  k_mark_dirty<<<grid_for(n, 256, 8192), 256, 0, ctx->stream>>>(n, lab, dirty, rev_off, rev_src, act_out, mass,
                                                                all_at, job_of, kbase, kappa);
  return knnkm_check(ctx, "active-set marks of changed centroids");
}

knnkm_status ks_entry_labels(knnkm_ctx* ctx, const int32_t* G, int64_t n, int32_t kappa, const int32_t* lab,
                             int32_t* nlab) {
  const int64_t ne = n * (int64_t)kappa;
  k_entry_labels<<<grid_for(ne, 256, 16384), 256, 0, ctx->stream>>>(G, ne, n, lab, nlab);
  return knnkm_check(ctx, "graph-entry labels");
}

knnkm_status ks_reverse_graph(knnkm_ctx* ctx, const int32_t* G, int64_t n, int32_t kappa, int32_t* rev_off,
                              int32_t* rev_src) {
  KNNKM_WS(ctx, cursor, int32_t, "rev_cursor", n);
  const int64_t ne = n * (int64_t)kappa;
  KNNKM_TRY(ks_fill_i32(ctx, rev_off, n + 1, 0));
  KNNKM_TRY(ks_fill_i32(ctx, cursor, n, 0));
  k_rev_count<<<grid_for(ne, 256, 16384), 256, 0, ctx->stream>>>(G, ne, n, rev_off);
  KNNKM_TRY(knnkm_check(ctx, "reverse graph counts"));
  KNNKM_TRY(ks_scan_exclusive(ctx, rev_off, rev_off, n, true));
  k_rev_fill<<<grid_for(ne, 256, 16384), 256, 0, ctx->stream>>>(G, ne, n, kappa, rev_off, cursor, rev_src);
  return knnkm_check(ctx, "reverse graph");
}
