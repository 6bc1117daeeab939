// List update of Alg. 3 for one graph row, by one wavefront: the row keeps
// the kappa smallest (d2, id) of its old entries and the candidates (other
// members of its cluster with their exact keys) whose ids it does not hold
// yet (a pair already in the row was visited).
//
// Lane l holds candidate slots l, l + 64, ... (NC of them).  Only candidates
// that come before the row's kappa-th entry can enter, so a row none of whose
// candidates does is left as it is after one comparison per slot (the
// kappa-th entry read from the lane holding it).  Otherwise the old row is
// staged in LDS; each entering candidate finds its position
// among the old entries by binary search and looks for its id among all of
// them (a row passed in by the caller may hold any keys, so the search does
// not rely on where its key would put the id); the entering candidates are
// then ranked among themselves and the old entries shifted.
#pragma once
#include <cfloat>

#include "common.h"

__device__ inline bool mg_lt(float ka, int ia, float kb, int ib) { return ka < kb || (ka == kb && ia < ib); }

// The old entries of a row as the lanes hold them: lane l has entries l and
// l + 64 (FLT_MAX / INT32_MAX past kappa).  Loaded by the caller, so that the
// next row's loads can be in flight while one row is merged.
struct MergeRow {
  float e0k, e1k;
  int e0i, e1i;
};

__device__ inline MergeRow merge_load(const float* __restrict__ rowk, const int32_t* __restrict__ rowi, int kappa) {
  const int lane = threadIdx.x & 63;
  MergeRow m;
  m.e0k = lane < kappa ? rowk[lane] : FLT_MAX;
  m.e0i = lane < kappa ? rowi[lane] : INT32_MAX;
  m.e1k = lane + 64 < kappa ? rowk[lane + 64] : FLT_MAX;
  m.e1i = lane + 64 < kappa ? rowi[lane + 64] : INT32_MAX;
  return m;
}

// rowk/rowi: the row (global memory), read and written by this wavefront
// only; old: its entries (merge_load).  sk/si: LDS scratch of kappa floats
// and ints for this wavefront.
template <int NC>
__device__ inline void merge_row(float* __restrict__ rowk, int32_t* __restrict__ rowi, int kappa, const MergeRow& old,
                                 const float (&ck)[NC], const int (&cid)[NC], const bool (&valid)[NC],
                                 float* __restrict__ sk, int32_t* __restrict__ si) {
  const int lane = threadIdx.x & 63;
  const float e0k = old.e0k, e1k = old.e1k;
  const int e0i = old.e0i, e1i = old.e1i;
  // the kappa-th entry, from the lane that holds it
  const int tl = (kappa - 1) & 63;
  const bool hi_half = kappa > 64;
  const float tk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hi_half ? e1k : e0k), tl));
  const int tid_ = __builtin_amdgcn_readlane(hi_half ? e1i : e0i, tl);
  bool enter[NC];
  bool any = false;
#pragma unroll
  for (int h = 0; h < NC; ++h) {
    enter[h] = valid[h] && mg_lt(ck[h], cid[h], tk, tid_);
    any = any || enter[h];
  }
  if (__ballot(any) == 0) return;  // nothing can enter: the row stays
  if (lane < kappa) {
    sk[lane] = e0k;
    si[lane] = e0i;
  }
  if (lane + 64 < kappa) {
    sk[lane + 64] = e1k;
    si[lane + 64] = e1i;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  int pos[NC];
#pragma unroll
  for (int h = 0; h < NC; ++h) {
    pos[h] = 0;
    if (!enter[h]) continue;
    // entries before (ck, cid): the first q with !(entry_q < cand)
    int lo = 0, hi = kappa;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (mg_lt(sk[mid], si[mid], ck[h], cid[h])) lo = mid + 1; else hi = mid;
    }
    pos[h] = lo;
  }
  // visited: the id is already in the row (uniform LDS addresses: broadcast)
  for (int q = 0; q < kappa; ++q) {
    const int qi = si[q];
#pragma unroll
    for (int h = 0; h < NC; ++h) enter[h] = enter[h] && qi != cid[h];
  }
  // ranks among the entering candidates, shifts of the old entries
  int add0 = 0, add1 = 0;
  bool anyin = false;
#pragma unroll
  for (int g = 0; g < NC; ++g) {
    uint64_t M = __ballot(enter[g]);
    anyin = anyin || M != 0;
    while (M) {
      const int b = (int)__builtin_ctzll(M);
      M &= M - 1;
      const float qk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ck[g]), b));
      const int qi = __builtin_amdgcn_readlane(cid[g], b);
#pragma unroll
      for (int h = 0; h < NC; ++h) pos[h] += mg_lt(qk, qi, ck[h], cid[h]) ? 1 : 0;
      add0 += mg_lt(qk, qi, e0k, e0i) ? 1 : 0;
      add1 += mg_lt(qk, qi, e1k, e1i) ? 1 : 0;
    }
  }
  if (!anyin) return;  // wave-uniform: every entering candidate was visited
  // every lane has read the row before any lane writes it
  if (lane < kappa && lane + add0 < kappa) {
    rowk[lane + add0] = e0k;
    rowi[lane + add0] = e0i;
  }
  if (lane + 64 < kappa && lane + 64 + add1 < kappa) {
    rowk[lane + 64 + add1] = e1k;
    rowi[lane + 64 + add1] = e1i;
  }
#pragma unroll
  for (int h = 0; h < NC; ++h)
    if (enter[h] && pos[h] < kappa) {
      rowk[pos[h]] = ck[h];
      rowi[pos[h]] = cid[h];
    }
}
