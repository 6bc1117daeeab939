// List update of Alg. 3 for one graph row, by one wavefront: the row keeps
// the kappa smallest (d2, id) of its old entries and the candidates (other
// members of its cluster with their exact keys) whose ids it does not hold
// yet (a pair already in the row was visited).
//
// Lane l holds the row's entries l and l + 64 and candidate slots l, l + 64,
// ... (NC of them).  Every (d2, id) is compared as one 64-bit integer whose
// order is that of (d2, id) (mg_key).  Only candidates that come before the
// row's kappa-th entry can enter, so a row none of whose candidates does is
// left as it is after one comparison per slot.  Otherwise the visited
// entering candidates are dropped in parallel -- the row's ids go into a
// small open-addressing table in LDS, one per wavefront, which every
// entering candidate probes for its id.  With many more entering than the
// row holds, those that cannot be among the kappa smallest are dropped
// after a bisection on the keys' high words.  The remaining ones are taken
// one at a time (broadcast from their lane): each counts, in one pass, the
// old entries and the other entering candidates before it (its position)
// and adds itself to the shift of every old entry after it.  The row's old
// entries are in ascending (d2, id) order (the graph's invariant), so these
// counts are the positions in the merged row.
#pragma once
#include <cfloat>
#include <cstdint>

#include "common.h"

__device__ inline bool mg_lt(float ka, int ia, float kb, int ib) { return ka < kb || (ka == kb && ia < ib); }

// 64-bit key ordered as (d2, id) under mg_lt for every d2 that is not NaN:
// the float's bits made monotone (negative values complemented, the sign bit
// set on the others, -0 taken as +0) above the id with its sign bit flipped.
__device__ inline uint64_t mg_key(float k, int id) {
  uint32_t b = __float_as_uint(k);
  if (b == 0x80000000u) b = 0u;
  b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((uint64_t)b << 32) | (uint32_t)(id ^ (int)0x80000000);
}

// Per-wavefront id table: MG_SLOTS entries, -1 when empty (the caller fills
// it with -1 once; merge_row leaves it empty).  At most KNNKM_MAX_KAPPA ids
// are in it at a time, so a probe meets an empty slot; the loops are bounded
// by the table size all the same.
#define MG_SLOTS 256
static_assert(MG_SLOTS >= 2 * KNNKM_MAX_KAPPA, "id table at most half full");

__device__ inline int mg_slot(int id) { return (int)(((uint32_t)id * 2654435761u) >> 24) & (MG_SLOTS - 1); }

__device__ inline int mg_insert(int32_t* hs, int id) {
  int s = mg_slot(id);
  for (int t = 0; t < MG_SLOTS; ++t) {
    if (atomicCAS(&hs[s], -1, id) == -1) return s;
    s = (s + 1) & (MG_SLOTS - 1);
  }
  return -1;
}

__device__ inline bool mg_has(const int32_t* hs, int id) {
  int s = mg_slot(id);
  for (int t = 0; t < MG_SLOTS; ++t) {
    const int v = hs[s];
    if (v == id) return true;
    if (v == -1) return false;
    s = (s + 1) & (MG_SLOTS - 1);
  }
  return false;
}

__device__ inline uint64_t mg_readlane(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

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

// rowk/rowi: the row (global memory or LDS), read and written by this
// wavefront only; old: its entries (merge_load).  Candidate ids are
// non-negative and below INT32_MAX where valid.  hs: this wavefront's id
// table (LDS, MG_SLOTS entries, empty).  kth (optional): receives the row's
// new kappa-th key when the row changes.  Returns whether it changed.
template <int NC>
__device__ inline bool merge_row(float* __restrict__ rowk, int32_t* __restrict__ rowi, int kappa, const MergeRow& old,
                                 const float (&ck)[NC], const int (&cid)[NC], const bool (&valid)[NC],
                                 int32_t* __restrict__ hs, float* kth = nullptr) {
  const int lane = threadIdx.x & 63;
  const bool two = kappa > 64;  // wave-uniform: entries past 64 in use
  const uint64_t o0 = mg_key(old.e0k, old.e0i);
  const uint64_t o1 = two ? mg_key(old.e1k, old.e1i) : ~0ull;
  // the kappa-th entry, from the lane that holds it
  const uint64_t tk = mg_readlane(two ? o1 : o0, (kappa - 1) & 63);
  uint64_t cq[NC];
  bool enter[NC];
  bool any = false;
#pragma unroll
  for (int h = 0; h < NC; ++h) {
    cq[h] = mg_key(ck[h], cid[h]);
    enter[h] = valid[h] && cq[h] < tk;
    any = any || enter[h];
  }
  if (__ballot(any) == 0) return false;  // nothing can enter: the row stays
  // visited: the candidate's id is already in the row
  const int s0 = lane < kappa ? mg_insert(hs, old.e0i) : -1;
  const int s1 = two && lane + 64 < kappa ? mg_insert(hs, old.e1i) : -1;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int h = 0; h < NC; ++h)
    if (enter[h] && mg_has(hs, cid[h])) enter[h] = false;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (s0 >= 0) hs[s0] = -1;
  if (s1 >= 0) hs[s1] = -1;
  // young lists (far more entering candidates than the list holds): drop the
  // candidates whose key's high word exceeds t, the least value with at least
  // kappa keys (old entries and entering candidates) of high word <= t --
  // kappa keys precede each of them, so none can enter and none moves an
  // entry that stays.  t by bisection between 0 and the kappa-th entry's.
  int ne = 0;
#pragma unroll
  for (int g = 0; g < NC; ++g) ne += __builtin_popcountll(__ballot(enter[g]));
  if (ne > kappa + 24) {
    const uint32_t oh0 = lane < kappa ? (uint32_t)(o0 >> 32) : 0xFFFFFFFFu;
    const uint32_t oh1 = two && lane + 64 < kappa ? (uint32_t)(o1 >> 32) : 0xFFFFFFFFu;
    uint32_t ch[NC];
#pragma unroll
    for (int h = 0; h < NC; ++h) ch[h] = enter[h] ? (uint32_t)(cq[h] >> 32) : 0xFFFFFFFFu;
    uint32_t lo = 0, hi = (uint32_t)(tk >> 32);
    for (int it = 0; it < 32 && lo < hi; ++it) {
      const uint32_t mid = lo + (hi - lo) / 2;
      int cnt = __builtin_popcountll(__ballot(oh0 <= mid)) + __builtin_popcountll(__ballot(oh1 <= mid));
#pragma unroll
      for (int h = 0; h < NC; ++h) cnt += __builtin_popcountll(__ballot(ch[h] <= mid));
      if (cnt >= kappa) hi = mid; else lo = mid + 1;
    }
#pragma unroll
    for (int h = 0; h < NC; ++h)
      if (enter[h] && ch[h] > lo) enter[h] = false;
  }
  // positions of the entering candidates, shifts of the old entries
  int pos[NC];
#pragma unroll
  for (int h = 0; h < NC; ++h) pos[h] = 0;
  int add0 = 0, add1 = 0;
  bool anyin = false;
#pragma unroll
  for (int g = 0; g < NC; ++g) {
    uint64_t M = __ballot(enter[g]);
    anyin = anyin || M != 0;
    while (M) {
      const int b = (int)__builtin_ctzll(M);
      M &= M - 1;
      const uint64_t q = mg_readlane(cq[g], b);
#pragma unroll
      for (int h = 0; h < NC; ++h) pos[h] += q < cq[h] ? 1 : 0;
      add0 += q < o0 ? 1 : 0;
      int before = __builtin_popcountll(__ballot(o0 < q));
      if (two) {
        add1 += q < o1 ? 1 : 0;
        before += __builtin_popcountll(__ballot(o1 < q));
      }
      if (lane == b) pos[g] += before;
    }
  }
  if (!anyin) return false;  // wave-uniform: every entering candidate was visited
  if (lane < kappa && lane + add0 < kappa) {
    rowk[lane + add0] = old.e0k;
    rowi[lane + add0] = old.e0i;
    if (kth && lane + add0 == kappa - 1) *kth = old.e0k;
  }
  if (two && lane + 64 < kappa && lane + 64 + add1 < kappa) {
    rowk[lane + 64 + add1] = old.e1k;
    rowi[lane + 64 + add1] = old.e1i;
    if (kth && lane + 64 + add1 == kappa - 1) *kth = old.e1k;
  }
#pragma unroll
  for (int h = 0; h < NC; ++h)
    if (enter[h] && pos[h] < kappa) {
      rowk[pos[h]] = ck[h];
      rowi[pos[h]] = cid[h];
      if (kth && pos[h] == kappa - 1) *kth = ck[h];
    }
  return true;
}
