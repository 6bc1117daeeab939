// Row groups: L consecutive lanes of a wavefront hold one sample row, lane j
// of the group holding dimensions [j*V, j*V + V).  A wavefront therefore works
// on 64/L rows at once, and sums over a row reduce inside the group with DPP
// (quad permutes and row mirrors inside a 16-lane row), ds_swizzle (xor 16)
// and ds_bpermute (xor 32).  The reduction tree is fixed, so every lane of a
// group ends with the bitwise same value and results do not depend on the
// launch configuration beyond the choice of (L, V), which depends on d only.
#pragma once
#include "common.h"

#define DPP_QUAD_XOR1 0xB1
#define DPP_QUAD_XOR2 0x4E
#define DPP_ROW_HALF_MIRROR 0x141
#define DPP_ROW_MIRROR 0x140
#define SWZ_XOR16 0x401F

template <int CTRL>
__device__ inline float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float swz16_f32(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), SWZ_XOR16));
}
__device__ inline double swz16_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)b, SWZ_XOR16);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), SWZ_XOR16);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the L lanes of the group (L in {1,2,4,8,16,32,64}).
template <int L>
__device__ inline float group_sum(float v) {
  if (L >= 2) v += dpp_f32<DPP_QUAD_XOR1>(v);
  if (L >= 4) v += dpp_f32<DPP_QUAD_XOR2>(v);
  if (L >= 8) v += dpp_f32<DPP_ROW_HALF_MIRROR>(v);
  if (L >= 16) v += dpp_f32<DPP_ROW_MIRROR>(v);
  if (L >= 32) v += swz16_f32(v);
  if (L >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}
template <int L>
__device__ inline double group_sum(double v) {
  if (L >= 2) v += dpp_f64<DPP_QUAD_XOR1>(v);
  if (L >= 4) v += dpp_f64<DPP_QUAD_XOR2>(v);
  if (L >= 8) v += dpp_f64<DPP_ROW_HALF_MIRROR>(v);
  if (L >= 16) v += dpp_f64<DPP_ROW_MIRROR>(v);
  if (L >= 32) v += swz16_f64(v);
  if (L >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

template <int L>
__device__ inline float group_max(float v) {
  if (L >= 2) v = fmaxf(v, dpp_f32<DPP_QUAD_XOR1>(v));
  if (L >= 4) v = fmaxf(v, dpp_f32<DPP_QUAD_XOR2>(v));
  if (L >= 8) v = fmaxf(v, dpp_f32<DPP_ROW_HALF_MIRROR>(v));
  if (L >= 16) v = fmaxf(v, dpp_f32<DPP_ROW_MIRROR>(v));
  if (L >= 32) v = fmaxf(v, swz16_f32(v));
  if (L >= 64) v = fmaxf(v, __shfl_xor(v, 32, 64));
  return v;
}

template <int L>
__device__ inline uint64_t group_mask(int g) {
  return L == 64 ? ~0ull : (((1ull << L) - 1ull) << (g * L));
}

// Load dims [j*V, j*V+V) of a row (zeros beyond d).  vec: d % 4 == 0 and the
// row start 16-byte aligned.
template <int V>
__device__ inline void load_row(float (&x)[V], const float* __restrict__ row, int j, int d, bool vec) {
  const int base = j * V;
  if (vec) {
#pragma unroll
    for (int e = 0; e < V; e += 4) {
      if (base + e < d) {
        const float4 q = *reinterpret_cast<const float4*>(row + base + e);
        x[e] = q.x;
        x[e + 1] = q.y;
        x[e + 2] = q.z;
        x[e + 3] = q.w;
      } else {
        x[e] = x[e + 1] = x[e + 2] = x[e + 3] = 0.f;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) x[e] = (base + e < d) ? row[base + e] : 0.f;
  }
}

// Host: group shape for dimension d (and at least `min_lanes` lanes).
inline void pick_group(int d, int min_lanes, int* L, int* V) {
  int l = 4;
  while (l < 64 && l * 8 < d) l <<= 1;
  while (l < 64 && l < min_lanes) l <<= 1;
  *L = l;
  *V = (l * 4 >= d) ? 4 : 8;
}
