// Graph-restricted assignment for wide rows (256 < d <= 512): one wavefront
// per sample, candidate distances by partial sums with early abandoning.
//
// The decision is the one of Alg. 2's Lloyd form (Sec. 4.2): the sample moves
// to the closest centroid among the clusters of its kappa neighbours and its
// own, staying unless a candidate is strictly closer, smallest id among equal
// minima.  At this width the candidates of one sample are nearly all distinct
// and hardly shared with the samples next to it, so every candidate costs one
// gathered centroid row and the sweep is bound by those gathers; most
// candidates are far from the sample, and a sum of squares over the first
// dimensions already exceeds the distance to the closest centroid.  So:
//  * every graph entry holding another cluster is a candidate slot (a
//    cluster held by several entries is evaluated once per entry, with the
//    same bits each time; at this width that is a few percent of the
//    entries, less than sorting them out would cost);
//  * an upper bound ub of the squared distance to the closest centroid comes
//    first, from the full float32 distance of the own centroid and, in a
//    full sweep, of the first slot (the cluster of the nearest entry holding
//    another one, the likeliest to be the closest; in the sweeps on active
//    sets a sample mostly stays), their loads in flight together;
//  * a sample with at most PD_DIRECT candidates left takes their full
//    float32 distances at once (one load level);
//  * otherwise the candidates advance breadth first, a chunk of dimensions
//    at a time (pd_chunk_full / pd_chunk_list), GL lanes per candidate and
//    PD_SB batches of candidates' loads in flight per wavefront, reading the
//    shadow of the centroids when there is one (8-bit codes with a step per
//    row, or bfloat16; eps bounds each shadow row's distance to the float32
//    row) and the float32 rows otherwise: each chunk adds to a running
//    float32 partial sum P, and a candidate is dropped as soon as a rigorous
//    lower bound of its squared distance over the dimensions so far,
//    (sqrt(P (1 - rel)) - eps)^2 by the triangle inequality, exceeds ub (the
//    candidate then cannot be the closest nor tie with it);
//  * with the shadow, a survivor of every chunk has its distance bracketed
//    by (sqrt(P (1 -+ rel)) -+ eps)^2, and only those whose lower end is
//    within the smallest upper end (and ub) remain;
//  * the remaining candidates get full float32 distances from the float32
//    rows;
//  * best and second best over the full distances, and when they are within
//    the rigorous float32 error margin, float64 re-evaluation of every
//    survivor inside it with the tie rule, as in the narrow kernels.
// Decisions therefore equal those of a float64 evaluation of every candidate;
// no centroid row is read past the chunk that rules it out.
#include <cfloat>

#include "rowgroup.h"

namespace {

// dimensions per early-abandon step (within the error bound pd_rel of the
// shadow kind): 64 of float32, 128 of bfloat16 (32 bytes per lane and
// candidate); of 8-bit codes 256 in full sweeps (32 bytes per lane: fewer
// dependent steps for the many candidates alive there) and 128 on active
// sets (16 bytes per lane: finer abandoning for the few)
template <int SK>
constexpr int pd_chunk_full() { return SK == 2 ? 256 : (SK ? 128 : 64); }
template <int SK>
constexpr int pd_chunk_list() { return SK ? 128 : 64; }

// candidate batches whose loads are in flight together: full sweeps 4 (more
// would cost a wavefront per SIMD), active-set sweeps 6
constexpr int PD_SB_FULL = 4;
constexpr int PD_SB_LIST = 6;
constexpr int PD_EX = 4;      // full float32 rows in flight together
constexpr int PD_DIRECT = 4;  // at most this many candidates: full distances at once

struct alignas(16) PDWave {
  float x[512];       // the sample's row
  int32_t cand[64];   // cluster of slot s (slot 0: the own one)
  float full[64];     // float32 full distance of slot (FLT_MAX: not taken)
  float lb[64];       // lower bound of the squared distance of slot
  float part[64];     // running partial sum of slot
  int32_t al[2][64];  // slots alive at this chunk and at the next
};

// Result of one decision: the label; u, an upper bound of the distance (not
// squared) to the chosen centroid; and, per lane e, a lower bound of the
// distance to the cluster of graph entry e (0 where that cluster is the
// chosen one or the entry is unused).
struct PDResult {
  int label;
  float u;
  float lb;  // lane-held
};

// Orders this wavefront's LDS writes before its later LDS reads by other
// lanes (a wavefront's LDS operations execute in order; this keeps the
// compiler from moving them across).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Sum over aligned groups of GL lanes (GL in {4, 8}); every lane of a group
// ends with the same bits.
template <int GL>
__device__ inline float gl_sum(float v) {
  v += dpp_f32<DPP_QUAD_XOR1>(v);
  v += dpp_f32<DPP_QUAD_XOR2>(v);
  if (GL >= 8) v += dpp_f32<DPP_ROW_HALF_MIRROR>(v);
  return v;
}

// bfloat16 (bit pattern) to float32, exact
__device__ inline float bf16_f32(uint32_t h) { return __uint_as_float(h << 16); }

// Rigorous lower bound of a squared distance from a float32 partial sum P
// (relative error at most rel) of the squared differences to a row within
// eps (Euclidean) of the true row: (sqrt(P (1 - rel)) - eps)^2, rounded down.
__device__ inline double pd_lower(float P, double rel, float eps) {
  const double t = sqrt((double)P * (1.0 - rel)) * (1.0 - 0x1p-50) - (double)eps;
  return t > 0.0 ? t * t * (1.0 - 0x1p-50) : 0.0;
}

// Rigorous upper bound of the squared distance from the float32 sum P of the
// squared differences to a row within eps of the true row over every
// dimension: (sqrt(P (1 + rel)) + eps)^2, rounded up.
__device__ inline double pd_upper(float P, double rel, float eps) {
  const double t = sqrt((double)P * (1.0 + rel)) * (1.0 + 0x1p-50) + (double)eps;
  return t * t * (1.0 + 0x1p-50);
}

// Full float32 distances (64-lane layout) of the row in LDS to the float32
// centroids of up to PD_EX slots taken from `pick` (index -> slot, -1 none),
// their loads in flight together; lane 0 stores full and lb of each slot.
template <typename Pick>
__device__ __attribute__((always_inline)) inline void pd_exact(PDWave& sh, int ne, Pick pick, const float* __restrict__ C, int d, bool vec_c,
                                double rel) {
  const int lane = threadIdx.x & 63;
  for (int e0 = 0; e0 < ne; e0 += PD_EX) {
    int sl[PD_EX];
    float c[PD_EX][8];
#pragma unroll
    for (int u = 0; u < PD_EX; ++u) {
      sl[u] = e0 + u < ne ? pick(e0 + u) : -1;
      if (sl[u] >= 0) load_row<8>(c[u], C + (int64_t)sh.cand[sl[u]] * d, lane, d, vec_c);
    }
#pragma unroll
    for (int u = 0; u < PD_EX; ++u) {
      if (sl[u] < 0) break;  // wave-uniform
      float acc = 0.f;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float df = sh.x[lane * 8 + e] - c[u][e];
        acc = fmaf(df, df, acc);
      }
      const float v = group_sum<64>(acc);
      if (lane == 0) {
        sh.full[sl[u]] = v;
        sh.lb[sl[u]] = f32_round_down((double)v * (1.0 - rel));
      }
    }
  }
}

// The decision of one sample, by the whole wavefront (every argument
// wave-uniform except lane-held ones).  cv: the candidate label held by lane
// e (entry e: 0 own, 1..kappa neighbours; -1 unused).  skip (lane-held): the
// entry's cluster is already known to be strictly farther than the own
// centroid, so it takes no part (its lane's lb is left to the caller).
// sw: the shadow of C read in the chunk steps (SK = sw.kind; 0: the float32
// rows).
// pilot: the first slot's full distance is taken with the own one.  Returns
// the label and the bounds of PDResult: every candidate's squared distance
// is bracketed by rigorous bounds (a dropped one from below by its partial
// sum), so they hold for the exact distances.
template <int GL, int SK, int CHK, int PD_SB>
__device__ __attribute__((always_inline)) inline PDResult pd_decide(PDWave& sh, const float* __restrict__ xrow,
                                                                    int d, bool vec_x, const float* __restrict__ C,
                                                                    bool vec_c, CShadow sw, bool vec_b, int cur,
                                                                    int cv, double rel, bool skip, bool pilot) {
  const float* __restrict__ eps = sw.eps;
  const int lane = threadIdx.x & 63;
  // slots: 0 the own cluster, then the entries holding another one in entry
  // order; an entry holding the own cluster maps to slot 0
  const int mine = (cv >= 0 && !(skip && lane > 0)) ? cv : -1;
  const bool isc = lane > 0 && mine >= 0 && mine != cur;
  const uint64_t cm = __ballot(isc);
  const int A0 = __popcll(cm);
  const int myslot = mine < 0 ? -1 : (isc ? 1 + __popcll(cm & lanes_below()) : 0);
  // the own centroid in full, and with a pilot the first slot's: their rows
  // are loaded together with the sample's row (lane j: dims [8j, 8j+8)),
  // which then goes to LDS for the chunk steps; the distances are formed as
  // pd_exact forms them
  const int np = pilot ? min(A0, 1) : 0;
  float x[8], co[8], cp[8];
  load_row<8>(x, xrow, lane, d, vec_x);
  load_row<8>(co, C + (int64_t)cur * d, lane, d, vec_c);
  if (np) load_row<8>(cp, C + (int64_t)__builtin_amdgcn_readlane(mine, (int)__builtin_ctzll(cm)) * d, lane, d, vec_c);
#pragma unroll
  for (int e = 0; e < 8; ++e) sh.x[lane * 8 + e] = x[e];
  sh.full[lane] = FLT_MAX;
  sh.lb[lane] = FLT_MAX;
  sh.part[lane] = 0.f;
  if (isc) {
    sh.cand[myslot] = mine;
    sh.al[0][myslot - 1] = myslot;
  }
  if (lane == 0) sh.cand[0] = cur;
  wave_lds_sync();
  {
    float acc = 0.f, accp = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float df = x[e] - co[e];
      acc = fmaf(df, df, acc);
    }
    const float v = group_sum<64>(acc);
    float vp = FLT_MAX;
    if (np) {  // wave-uniform
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float df = x[e] - cp[e];
        accp = fmaf(df, df, accp);
      }
      vp = group_sum<64>(accp);
    }
    if (lane == 0) {
      sh.full[0] = v;
      sh.lb[0] = f32_round_down((double)v * (1.0 - rel));
      if (np) {
        sh.full[1] = vp;
        sh.lb[1] = f32_round_down((double)vp * (1.0 - rel));
      }
    }
  }
  wave_lds_sync();
  const double ub = (double)fminf(sh.full[0], np ? sh.full[1] : FLT_MAX) * (1.0 + rel) + 1e-30;
  constexpr int NG = 64 / GL;        // candidates per batch
  constexpr int PL = CHK / GL;  // dimensions per lane and chunk
  static_assert(PL * (SK == 2 ? 1 : (SK == 1 ? 2 : 4)) == 32 || (SK == 2 && PL == 16),
                "32 bytes per lane and chunk (16 of 8-bit codes on active sets)");
  const int g = lane / GL, jj = lane % GL;
  const int nch = (d + CHK - 1) / CHK;
  // the other slots, breadth first (al[0] lists slots 1..A0; the first np
  // are done).  With the shadow, the survivors of the last chunk go to the
  // next list for their float32 distances; without it they have them.
  int A = A0 - np, buf = 0;
  if (A > 0 && A <= PD_DIRECT) {
    // few candidates left: their float32 distances in one load level in
    // place of the chunk steps, the bracket and the survivors' rows
    pd_exact(sh, A, [&](int e) { return sh.al[0][e + np]; }, C, d, vec_c, rel);
    wave_lds_sync();
    A = 0;
  }
  for (int ch = 0; ch < nch && A > 0; ++ch) {
    const bool last = ch == nch - 1;
    const int base = ch * CHK + jj * PL;
    int nA = 0;
    for (int s0 = 0; s0 < A; s0 += NG * PD_SB) {
      int slot[PD_SB];
      // the chunk of each batch's candidate per lane: 8 float32 values, 16
      // bfloat16 (two per word) or 16 or 32 codes (four per word), and the
      // code step of the candidate
      constexpr int NW = SK == 2 ? PL / 4 : (SK == 1 ? PL / 2 : PL);
      uint32_t cq[PD_SB][NW];
      float sc[PD_SB];
#pragma unroll
      for (int u = 0; u < PD_SB; ++u) {
        const int idx = s0 + u * NG + g;
        slot[u] = idx < A ? sh.al[buf][ch == 0 ? idx + np : idx] : -1;
      }
#pragma unroll
      for (int u = 0; u < PD_SB; ++u) {
#pragma unroll
        for (int e = 0; e < NW; ++e) cq[u][e] = SK == 2 ? 0x80808080u : 0u;
        sc[u] = 0.f;
        if (slot[u] < 0) continue;
        const int64_t q = sh.cand[slot[u]];
        if constexpr (SK == 2) {
          const uint8_t* br = (const uint8_t*)sw.rows + q * d;
          sc[u] = sw.scale[q];
          if (vec_b && base + PL <= d) {
#pragma unroll
            for (int h = 0; h < PL / 16; ++h) {
              const uint4 v = *reinterpret_cast<const uint4*>(br + base + 16 * h);
              cq[u][4 * h] = v.x;
              cq[u][4 * h + 1] = v.y;
              cq[u][4 * h + 2] = v.z;
              cq[u][4 * h + 3] = v.w;
            }
          } else {
#pragma unroll
            for (int e = 0; e < PL; ++e) {
              const uint32_t b = base + e < d ? br[base + e] : 128u;  // code 128: the value 0
              cq[u][e / 4] = (cq[u][e / 4] & ~(0xFFu << (8 * (e % 4)))) | (b << (8 * (e % 4)));
            }
          }
        } else if constexpr (SK == 1) {
          const uint16_t* br = (const uint16_t*)sw.rows + q * d;
          if (vec_b && base + PL <= d) {
#pragma unroll
            for (int h = 0; h < PL / 8; ++h) {
              const uint4 v = *reinterpret_cast<const uint4*>(br + base + 8 * h);
              cq[u][4 * h] = v.x;
              cq[u][4 * h + 1] = v.y;
              cq[u][4 * h + 2] = v.z;
              cq[u][4 * h + 3] = v.w;
            }
          } else {
#pragma unroll
            for (int e = 0; e < PL; e += 2) {
              const uint32_t lo = base + e < d ? br[base + e] : 0u;
              const uint32_t hi = base + e + 1 < d ? br[base + e + 1] : 0u;
              cq[u][e / 2] = lo | (hi << 16);
            }
          }
        } else {
          const float* cr = C + q * d;
#pragma unroll
          for (int e = 0; e < PL; e += 4) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (vec_c && base + e < d) {
              v = *reinterpret_cast<const float4*>(cr + base + e);
            } else {
              v.x = base + e < d ? cr[base + e] : 0.f;
              v.y = base + e + 1 < d ? cr[base + e + 1] : 0.f;
              v.z = base + e + 2 < d ? cr[base + e + 2] : 0.f;
              v.w = base + e + 3 < d ? cr[base + e + 3] : 0.f;
            }
            cq[u][e] = __float_as_uint(v.x);
            cq[u][e + 1] = __float_as_uint(v.y);
            cq[u][e + 2] = __float_as_uint(v.z);
            cq[u][e + 3] = __float_as_uint(v.w);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < PD_SB; ++u) {
        if (s0 + u * NG >= A) break;  // wave-uniform: no candidate left in this batch
        float acc = 0.f;
        if (slot[u] >= 0) {
#pragma unroll
          for (int e = 0; e < PL; e += 4) {
            const float4 xq = *reinterpret_cast<const float4*>(&sh.x[base + e]);
            float df0, df1, df2, df3;
            if constexpr (SK == 2) {
              // x - s (u - 128) with one rounding (the shadow value is the
              // exact product)
              const uint32_t w4 = cq[u][e / 4];
              const float ns = -sc[u];
              df0 = fmaf(ns, (float)(w4 & 0xFFu) - 128.f, xq.x);
              df1 = fmaf(ns, (float)((w4 >> 8) & 0xFFu) - 128.f, xq.y);
              df2 = fmaf(ns, (float)((w4 >> 16) & 0xFFu) - 128.f, xq.z);
              df3 = fmaf(ns, (float)(w4 >> 24) - 128.f, xq.w);
            } else if constexpr (SK == 1) {
              df0 = xq.x - bf16_f32(cq[u][e / 2] & 0xFFFFu);
              df1 = xq.y - bf16_f32(cq[u][e / 2] >> 16);
              df2 = xq.z - bf16_f32(cq[u][e / 2 + 1] & 0xFFFFu);
              df3 = xq.w - bf16_f32(cq[u][e / 2 + 1] >> 16);
            } else {
              df0 = xq.x - __uint_as_float(cq[u][e]);
              df1 = xq.y - __uint_as_float(cq[u][e + 1]);
              df2 = xq.z - __uint_as_float(cq[u][e + 2]);
              df3 = xq.w - __uint_as_float(cq[u][e + 3]);
            }
            acc = fmaf(df0, df0, acc);
            acc = fmaf(df1, df1, acc);
            acc = fmaf(df2, df2, acc);
            acc = fmaf(df3, df3, acc);
          }
        }
        const float sum = gl_sum<GL>(acc);
        bool keep = false;
        if (slot[u] >= 0) {
          const float P = sh.part[slot[u]] + sum;
          const double lo = SK ? pd_lower(P, rel, eps[sh.cand[slot[u]]]) : (double)P * (1.0 - rel);
          if (lo > ub) {
            if (jj == 0) sh.lb[slot[u]] = f32_round_down(lo);
          } else if (last && !SK) {
            if (jj == 0) {
              sh.full[slot[u]] = P;
              sh.lb[slot[u]] = f32_round_down(lo);
            }
          } else {
            keep = true;
            if (jj == 0) {
              sh.part[slot[u]] = P;
              if (last) sh.lb[slot[u]] = f32_round_down(lo);
            }
          }
        }
        const uint64_t km = __ballot(keep && jj == 0);
        if (keep && jj == 0) sh.al[buf ^ 1][nA + __popcll(km & lanes_below())] = slot[u];
        nA += __popcll(km);
      }
    }
    wave_lds_sync();
    A = nA;
    buf ^= 1;
  }
  if (SK && A > 0) {
    // the survivors' shadow distances bracket their distances: only those
    // whose lower bound is within the smallest upper bound (and ub) can be
    // the closest or tie with it
    const int sl = lane < A ? sh.al[buf][lane] : -1;
    double lo = DBL_MAX, hi = DBL_MAX;
    if (sl >= 0) {
      const float P = sh.part[sl];
      const float e = eps[sh.cand[sl]];
      lo = pd_lower(P, rel, e);
      hi = pd_upper(P, rel, e);
    }
    double m = hi;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
    m = fmin(m, ub);
    const bool stay = sl >= 0 && lo <= m;
    const uint64_t M = __ballot(stay);
    if (stay) sh.al[buf ^ 1][__popcll(M & lanes_below())] = sl;
    A = __popcll(M);
    buf ^= 1;
    wave_lds_sync();
  }
  // the remaining survivors' float32 distances
  if (A > 0) {
    pd_exact(sh, A, [&](int e) { return sh.al[buf][e]; }, C, d, vec_c, rel);
    wave_lds_sync();
  }
  PDResult r;
  r.lb = 0.f;
  {
    // best and second best over the full distances (lane t reads slot t; the
    // tie rule makes the result independent of the order of the fold)
    const float fl = lane <= A0 ? sh.full[lane] : FLT_MAX;
    const int ql = lane <= A0 ? sh.cand[lane] : -1;
    float b1 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(fl))), b2 = FLT_MAX;
    int q1 = cur;
    for (uint64_t F = __ballot(lane >= 1 && fl != FLT_MAX); F; F &= F - 1) {
      const int t = (int)__builtin_ctzll(F);
      const float dq = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fl), t));
      const int qq = __builtin_amdgcn_readlane(ql, t);
      if (qq == q1) continue;  // a cluster held by several entries
      if (dq < b1 || (dq == b1 && qq < q1)) {
        b2 = fminf(b2, b1);
        b1 = dq;
        q1 = qq;
      } else {
        b2 = fminf(b2, dq);
      }
    }
    const double thr = (double)b1 * (1.0 + rel) / (1.0 - rel) + 1e-30;
    int res = q1;
    double dres = (double)b1 * (1.0 + rel) + 1e-30;  // upper bound of the chosen squared distance
    if ((double)b2 <= thr) {
      // float64 re-evaluation of every survivor inside the margin
      double m64 = DBL_MAX, cur64 = -1.0;
      int q64 = -1;
      for (uint64_t F = __ballot(fl != FLT_MAX && (double)fl <= thr); F; F &= F - 1) {
        const int t = (int)__builtin_ctzll(F);
        const int qq = __builtin_amdgcn_readlane(ql, t);
        float c[8];
        load_row<8>(c, C + (int64_t)qq * d, lane, d, vec_c);
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const double df = (double)sh.x[lane * 8 + e] - (double)c[e];
          acc = fma(df, df, acc);
        }
        const double e64 = group_sum<64>(acc);
        if (qq == cur) cur64 = e64;
        if (e64 < m64 || (e64 == m64 && qq < q64)) {
          m64 = e64;
          q64 = qq;
        }
      }
      res = (cur64 >= 0.0 && cur64 == m64) ? cur : q64;
      dres = m64 * (1.0 + 0x1p-40) + 1e-300;
    }
    r.label = res;
    r.u = f32_round_up(sqrt(dres) * (1.0 + 0x1p-50));
  }
  if (myslot >= 0 && mine != r.label) {
    const float lq = sh.lb[myslot];
    r.lb = lq == FLT_MAX ? 0.f : f32_round_down(sqrt((double)lq) * (1.0 - 0x1p-50));
  }
  wave_lds_sync();  // every lane has read the slots before the next sample writes them
  return r;
}

// Candidate label of lane e for sample i (entry 0: own label; 1..kappa:
// neighbour labels; for a sample whose job has no more clusters than kappa,
// every cluster of its job, own first).
__device__ inline int pd_candidate(int lane, int64_t i, int cur, const int* __restrict__ G, int kappa,
                                   const int* __restrict__ lab_in, bool dense, int kb, int kc) {
  if (lane == 0) return cur;
  if (dense) {
    if (lane >= kc) return -1;
    const int v = kb + lane - 1;
    return v < cur ? v : v + 1;
  }
  return lane <= kappa ? lab_in[G[i * kappa + (lane - 1)]] : -1;
}

// Full sweep: block b takes pb consecutive positions of `order` (or of the
// identity), wave w of it the positions w, w+4, ...  Same arguments and
// outputs as k_assign without best distances.
template <int GL, int SK>
__global__ __launch_bounds__(256) void k_assign_pd(
    const float* __restrict__ X, int n, int d, int64_t ldx, const float* __restrict__ C, int k,
    const int* __restrict__ G, int kappa, const int* __restrict__ lab_in, int* __restrict__ lab_out,
    unsigned long long* __restrict__ moved_acc, unsigned long long* __restrict__ eval_acc,
    const int* __restrict__ order, int nchunks, int pb, double rel, int vec_x, int vec_c,
    const int* __restrict__ job_of, const int* __restrict__ kbase, const uint8_t* __restrict__ act_in,
    uint8_t* __restrict__ act_out, float* __restrict__ bnd_u, float* __restrict__ bnd_lb, CShadow sw, int vec_b) {
  __shared__ PDWave sh[4];
  __shared__ unsigned int block_moved, block_eval;
  if (threadIdx.x == 0) {
    block_moved = 0;
    block_eval = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int per_xcd = gridDim.x / 8;
  const int chunk = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  unsigned int my_moved = 0, my_eval = 0;
  if (chunk < nchunks) {
    const int64_t start = (int64_t)chunk * pb;
    const int64_t end = min((int64_t)n, start + pb);
    for (int64_t idx = start + w; idx < end; idx += 4) {
      const int64_t i = order ? (int64_t)order[idx] : idx;
      const int cur = lab_in[i];
      if (act_in && act_in[i] == 0) {
        if (lane == 0) {
          lab_out[i] = cur;
          if (act_out) act_out[i] = 0;
        }
        continue;
      }
      int kb = 0, kc = k;
      if (job_of) {
        const int q = job_of[i];
        kb = kbase[q];
        kc = kbase[q + 1] - kb;
      }
      const bool dense = kappa >= kc;
      const int cv = pd_candidate(lane, i, cur, G, kappa, lab_in, dense, kb, kc);
      const bool other = cv >= 0 && cv != cur;
      if (!dense && __ballot(other) == 0) {  // the own cluster is the only candidate
        if (lane == 0) {
          lab_out[i] = cur;
          if (act_out) act_out[i] = 0;
        }
        continue;
      }
      const PDResult r = pd_decide<GL, SK, pd_chunk_full<SK>(), PD_SB_FULL>(sh[w], X + i * ldx, d, vec_x, C, vec_c,
                                                                             sw, vec_b, cur, cv, rel, false, true);
      if (bnd_u && lane <= kappa) bnd_lb[i * (kappa + 1) + lane] = r.lb;
      if (lane == 0) {
        lab_out[i] = r.label;
        if (act_out) act_out[i] = 1;
        if (bnd_u) bnd_u[i] = r.u;
        ++my_eval;
        if (r.label != cur) ++my_moved;
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

// Active-set sweep over the listed positions (entries as k_act_compact writes
// them: position, bit 31 = own or a neighbour's label changed), grid-stride,
// NS listed samples per wavefront and step: the loads of each dependent level
// (list entries; own labels and graph rows; neighbour labels; changed flags
// of the candidate clusters) are issued for all NS samples before any is
// used, then the samples are decided one after the other.  nlab (nullable):
// the labels of the graph entries (row-major, n x kappa, equal to lab_in of
// the entries' ids), read in place of the graph row and the scattered
// neighbour labels.  Same outputs as k_assign_list.
template <int GL, int NS, int SK>
__global__ __launch_bounds__(256) void k_assign_list_pd(
    const float* __restrict__ X, int d, int64_t ldx, const float* __restrict__ C, int k,
    const int* __restrict__ G, int kappa, const int* __restrict__ lab_in, int* __restrict__ lab_out,
    unsigned long long* __restrict__ moved_acc, unsigned long long* __restrict__ eval_acc,
    const int32_t* __restrict__ list, const int32_t* __restrict__ count, double rel, int vec_x, int vec_c,
    const int* __restrict__ job_of, const int* __restrict__ kbase, uint8_t* __restrict__ act_out,
    int64_t* __restrict__ n_listed, const uint32_t* __restrict__ cbits, float* __restrict__ bnd_u,
    float* __restrict__ bnd_lb, const float* __restrict__ delta, CShadow sw, int vec_b,
    const int32_t* __restrict__ nlab) {
  __shared__ PDWave sh[4];
  __shared__ unsigned int block_moved, block_eval;
  if (threadIdx.x == 0) {
    block_moved = 0;
    block_eval = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cnt = *count;
  if (n_listed && blockIdx.x == 0 && threadIdx.x == 0) *n_listed = cnt;
  unsigned int my_moved = 0, my_eval = 0;
  const int stride = gridDim.x * 4 * NS;
  for (int li0 = (blockIdx.x * 4 + w) * NS; li0 < cnt; li0 += stride) {
    bool live[NS], changed[NS], dense[NS];
    int64_t ii[NS];
    int cur[NS], kb[NS], kc[NS], nb[NS], cv[NS];
    bool dq[NS];
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      live[p] = li0 + p < cnt;  // wave-uniform
      const uint32_t ent = live[p] ? (uint32_t)list[li0 + p] : 0u;
      changed[p] = (ent >> 31) != 0;
      ii[p] = (int64_t)(ent & 0x7FFFFFFFu);
    }
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      const int64_t i = ii[p];
      cur[p] = live[p] ? lab_in[i] : 0;
      kb[p] = 0;
      kc[p] = k;
      if (job_of && live[p]) {
        const int q = job_of[i];
        kb[p] = kbase[q];
        kc[p] = kbase[q + 1] - kb[p];
      }
      // (with the graph-entry labels nb holds the entry's label, not its id)
      const bool ent = live[p] && lane >= 1 && lane <= kappa;
      nb[p] = !ent ? -1 : (nlab ? nlab[i * kappa + (lane - 1)] : G[i * kappa + (lane - 1)]);
    }
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      dense[p] = kappa >= kc[p];
      if (!live[p]) {
        cv[p] = -1;
      } else if (lane == 0) {
        cv[p] = cur[p];
      } else if (dense[p]) {
        const int v = kb[p] + lane - 1;
        cv[p] = lane >= kc[p] ? -1 : (v < cur[p] ? v : v + 1);
      } else {
        cv[p] = nlab ? nb[p] : (nb[p] >= 0 ? lab_in[nb[p]] : -1);
      }
    }
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      const bool look = live[p] && !changed[p] && !dense[p] && cbits && cv[p] >= 0;
      dq[p] = look && bit_of(cbits, cv[p]);
    }
    // the decisions, one sample after the other (one copy of the decision
    // code: the sample's values are selected, not indexed)
    auto pick = [&](const auto(&a)[NS], int p) {
      auto v = a[0];
#pragma unroll
      for (int q = 1; q < NS; ++q)
        if (p == q) v = a[q];
      return v;
    };
#pragma unroll 1
    for (int p = 0; p < NS; ++p) {
      if (!pick(live, p)) continue;  // wave-uniform
      const int64_t i = pick(ii, p);
      const int c = pick(cv, p), own = pick(cur, p);
      const bool chg = pick(changed, p), dn = pick(dense, p), dirt = pick(dq, p);
      const bool other = c >= 0 && c != own;
      if (!dn && __ballot(other) == 0) {
        if (lane == 0) {
          lab_out[i] = own;
          if (act_out) act_out[i] = 0;
        }
        continue;
      }
      bool skip = false;
      float lb_drift = 0.f;
      if (!chg && !dn && cbits) {
        // the same candidates as in the last sweep and none of their
        // centroids changed: the last decision, to stay, stands
        if (__ballot(dirt) == 0) {
          if (lane == 0) {
            lab_out[i] = own;
            if (act_out) act_out[i] = 1;
          }
          continue;
        }
        if (bnd_u) {
          // drift bounds (triangle inequality): the own centroid moved by at
          // most delta[own], the centroid of entry e by at most its delta; an
          // entry whose lower bound, less its movement, still exceeds the own
          // centroid's upper bound, plus its movement, is strictly farther
          // (movements are read for the changed clusters only: most of a late
          // sweep's candidates are unchanged, and each read is a scattered line)
          const float de = dirt ? delta[c] : 0.f;
          const float u_p = bnd_u[i];
          const float lb_p = lane <= kappa ? bnd_lb[i * (kappa + 1) + lane] : 0.f;
          const double U = ((double)u_p + (double)__shfl(de, 0, 64)) * (1.0 + 0x1p-50);
          const double Le = lane <= kappa ? ((double)lb_p - (double)de) * (1.0 - 0x1p-50) : 0.0;
          skip = c < 0 || c == own || Le > U;
          lb_drift = f32_round_down(Le);
          if (__ballot(!skip) == 0) {  // every other cluster is strictly farther: stays
            if (lane <= kappa) bnd_lb[i * (kappa + 1) + lane] = c == own ? 0.f : lb_drift;
            if (lane == 0) {
              lab_out[i] = own;
              if (act_out) act_out[i] = 1;
              bnd_u[i] = f32_round_up(U);
            }
            continue;
          }
        }
      }
      // (a listed sample mostly stays: no pilot)
      const PDResult r = pd_decide<GL, SK, pd_chunk_list<SK>(), PD_SB_LIST>(sh[w], X + i * ldx, d, vec_x, C, vec_c,
                                                                             sw, vec_b, own, c, rel, skip, false);
      if (bnd_u && lane <= kappa) {
        // skipped entries keep their drifted bounds (the chosen cluster is at
        // least as close as the own one, so they remain valid lower bounds)
        const bool keep = skip && lane > 0 && c >= 0 && c != own && c != r.label;
        bnd_lb[i * (kappa + 1) + lane] = keep ? lb_drift : r.lb;
      }
      if (lane == 0) {
        lab_out[i] = r.label;
        if (act_out) act_out[i] = 1;
        if (bnd_u) bnd_u[i] = r.u;
        ++my_eval;
        if (r.label != own) ++my_moved;
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

}  // namespace

// Relative error bound used by the wide kernel, in units of 2^-24 to first
// order: a rounded difference squared (2) plus the products summed per lane
// and the reduction levels; full distances 8 + 6, float32 chunks 8 + 3 plus up
// to eight chunk additions, bfloat16 chunks 16 + 3 plus up to four: at most
// 25; chunks of 8-bit codes 32 + 3 plus up to two (or 16 + 3 plus up to
// four): 39.  The bound is twice that.
static double pd_rel(int kind) { return (kind == 2 ? 39.0 : 25.0) * 0x1p-23; }

bool ks_assign_pd_ok(int32_t d, int32_t kappa) { return d > 256 && d <= 512 && kappa <= 63; }

// Shadow of centroid rows (all, or those with dirty[r] set): one wavefront
// per row.  bfloat16: eps[r] = ||c_r - bf16(c_r)|| rounded up (every
// difference is exact in float32, its square in float64); 8-bit codes:
// i8_shadow_row.
__global__ __launch_bounds__(256) void k_c_shadow(const float* __restrict__ C, int32_t K, int d,
                                                  const int32_t* __restrict__ dirty, CShadow sw) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = blockIdx.x * 4 + (threadIdx.x >> 6); r < K; r += (int64_t)gridDim.x * 4) {
    if (dirty && !dirty[r]) continue;  // wave-uniform
    if (sw.kind == 2) {
      i8_shadow_row(C + r * d, d, (uint8_t*)sw.rows + r * d, &sw.scale[r], &sw.eps[r]);
      continue;
    }
    uint16_t* Cb = (uint16_t*)sw.rows;
    double e2 = 0.0;
    for (int t = lane; t < d; t += 64) {
      const float c = C[r * d + t];
      const uint16_t h = bf16_rne(c);
      Cb[r * d + t] = h;
      const double df = (double)(c - __uint_as_float((uint32_t)h << 16));
      e2 = fma(df, df, e2);
    }
    e2 = wave_sum(e2);
    if (lane == 0) sw.eps[r] = f32_round_up(sqrt(e2) * (1.0 + 0x1p-40));
  }
}

knnkm_status ks_c_shadow(knnkm_ctx* ctx, const float* C, int32_t K, int32_t d, const int32_t* dirty, CShadow sw) {
  if (K <= 0 || sw.kind == 0) return KNNKM_OK;
  k_c_shadow<<<grid_for(K, 4, 16384), 256, 0, ctx->stream>>>(C, K, d, dirty, sw);
  return knnkm_check(ctx, "centroid shadow");
}

knnkm_status ks_assign_pd(knnkm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, const float* C,
                          int32_t k, const int32_t* G_ids, int32_t kappa, const int32_t* labels_in,
                          int32_t* labels_out, unsigned long long* acc, unsigned long long* eacc,
                          const int32_t* order, const int32_t* job_of, const int32_t* kbase,
                          const uint8_t* act_in, uint8_t* act_out, const int32_t* list, const int32_t* list_count,
                          int64_t* n_listed, const uint32_t* cbits, int pb, float* bnd_u, float* bnd_lb,
                          const float* delta, CShadow sw, const int32_t* nlab) {
  if ((bnd_u != nullptr) != (bnd_lb != nullptr) || (list && bnd_u && cbits && !delta))
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_assign (wide rows): incomplete drift bounds");
  if (sw.kind < 0 || sw.kind > 2 || (sw.kind && (!sw.rows || !sw.eps || (sw.kind == 2 && !sw.scale))))
    return knnkm_fail(ctx, KNNKM_EINVAL, "knn_assign (wide rows): incomplete centroid shadow");
  const bool vec_x = (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0) && (d % 4 == 0);
  const bool vec_c = (d % 4 == 0) && ((uintptr_t)C % 16 == 0);
  // 16-byte shadow loads: rows of whole 16-byte units from an aligned base
  const bool vec_b = (d % (sw.kind == 2 ? 16 : 8) == 0) && ((uintptr_t)sw.rows % 16 == 0);
  const double rel = pd_rel(sw.kind);
  if (list) {
    const unsigned grid = (unsigned)std::max(1, ctx->num_cus * 8);
    // listed samples interleaved per wavefront: 2 unless the context fixes
    // the assignment shape to one sample per group
#define LPD(NS, SK)                                                                                           \
  k_assign_list_pd<8, NS, SK><<<grid, 256, 0, ctx->stream>>>(X, d, ldx, C, k, G_ids, kappa, labels_in, labels_out, \
                                                        acc, eacc, list, list_count, rel, vec_x ? 1 : 0,      \
                                                        vec_c ? 1 : 0, job_of, kbase, act_out, n_listed,      \
                                                        cbits, bnd_u, bnd_lb, delta, sw, vec_b ? 1 : 0, nlab)
#define LPD_K(NS)            \
  switch (sw.kind) {         \
    case 1: LPD(NS, 1); break; \
    case 2: LPD(NS, 2); break; \
    default: LPD(NS, 0); break; \
  }
    if (ctx->assign_gs == 1) {
      LPD_K(1);
    } else {
      LPD_K(2);
    }
#undef LPD_K
#undef LPD
    return knnkm_check(ctx, "knn_assign (wide rows, active set)");
  }
  const int nchunks = (int)((n + pb - 1) / pb);
  const int grid = ((nchunks + 7) / 8) * 8;
#define FPD(SK)                                                                                                    \
  k_assign_pd<8, SK><<<grid, 256, 0, ctx->stream>>>(X, (int)n, d, ldx, C, k, G_ids, kappa, labels_in, labels_out, \
                                                    acc, eacc, order, nchunks, pb, rel, vec_x ? 1 : 0,           \
                                                    vec_c ? 1 : 0, job_of, kbase, act_in, act_out, bnd_u, bnd_lb, \
                                                    sw, vec_b ? 1 : 0)
  switch (sw.kind) {
    case 1: FPD(1); break;
    case 2: FPD(2); break;
    default: FPD(0); break;
  }
#undef FPD
  return knnkm_check(ctx, "knn_assign (wide rows)");
}
