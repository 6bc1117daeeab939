// Exact 128-bit two's-complement fixed point for the composite vectors D_r
// of Eqn. 2 (value * 2^s, one exponent s per job): conversion from a double
// and correctly rounded conversion back.  Usable from host and device code,
// so the same functions are checked on the CPU against 128-bit integers.
#pragma once
#include <cmath>
#include <cstdint>

#ifdef __HIPCC__
#define FX_HD __host__ __device__
#else
#define FX_HD
#endif

// The conversions below work on 32-bit words only.  A form of the
// fixed-point-to-double conversion written with 64-bit variable shifts was
// exact when run alone but gave nondeterministic extra high bits when
// inlined in the finalize loop on gfx950, so no 64-bit variable shift is
// used here.

// fixed-point value of a double times 2^s (magnitude truncated toward zero
// below the last integer bit), as (hi, lo) two's complement
FX_HD inline void fx_of_double(double v, int s, uint64_t& hi, uint64_t& lo) {
  hi = lo = 0;
  if (v == 0.0) return;
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t bh = (uint32_t)(b >> 32), bl = (uint32_t)b;
  const int ex = (int)((bh >> 20) & 0x7FFu);
  uint32_t m1 = bh & 0xFFFFFu;
  const uint32_t m0 = bl;
  int e;
  if (ex == 0) {
    e = -1074;
  } else {
    m1 |= 0x100000u;
    e = ex - 1075;
  }
  const int sh = e + s;  // |v| 2^s = (m1:m0) 2^sh, below 2^125 by the choice of s
  uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
  if (sh >= 0) {
    const int q = sh >> 5, r = sh & 31;
    const uint32_t t0 = m0 << r;
    const uint32_t t1 = r ? (m1 << r) | (m0 >> (32 - r)) : m1;
    const uint32_t t2 = r ? m1 >> (32 - r) : 0u;
    if (q == 0) {
      w0 = t0; w1 = t1; w2 = t2;
    } else if (q == 1) {
      w1 = t0; w2 = t1; w3 = t2;
    } else if (q == 2) {
      w2 = t0; w3 = t1;
    } else if (q == 3) {
      w3 = t0;
    }
  } else if (sh > -64) {
    const int q = (-sh) >> 5, r = (-sh) & 31;
    if (q == 0) {
      w0 = r ? (m0 >> r) | (m1 << (32 - r)) : m0;
      w1 = r ? m1 >> r : m1;
    } else {
      w0 = m1 >> r;
    }
  }
  lo = ((uint64_t)w1 << 32) | w0;
  hi = ((uint64_t)w3 << 32) | w2;
  if (bh >> 31) {
    lo = ~lo;
    hi = ~hi;
    lo += 1;
    if (lo == 0) hi += 1;
  }
}

FX_HD inline void fx_neg(uint64_t& hi, uint64_t& lo) {
  lo = ~lo;
  hi = ~hi;
  lo += 1;
  if (lo == 0) hi += 1;
}

// Round (hi, lo) * 2^-s to the nearest double: the 64 bits below the leading
// one, a sticky bit for everything further down, then one rounding.
FX_HD inline double fx_to_double(uint64_t hi, uint64_t lo, int s) {
  const bool neg = (int64_t)hi < 0;
  if (neg) fx_neg(hi, lo);
  const uint32_t w0 = (uint32_t)lo, w1 = (uint32_t)(lo >> 32), w2 = (uint32_t)hi, w3 = (uint32_t)(hi >> 32);
  uint32_t a, b, c, rest;
  int top;  // index of the leading nonzero word
  if (w3) {
    top = 3; a = w3; b = w2; c = w1; rest = w0;
  } else if (w2) {
    top = 2; a = w2; b = w1; c = w0; rest = 0;
  } else if (w1) {
    top = 1; a = w1; b = w0; c = 0; rest = 0;
  } else if (w0) {
    top = 0; a = w0; b = 0; c = 0; rest = 0;
  } else {
    return 0.0;
  }
  const int z = __builtin_clz(a);  // a != 0
  uint32_t t1, t0;
  if (z == 0) {
    t1 = a; t0 = b; rest |= c;
  } else {
    t1 = (a << z) | (b >> (32 - z));
    t0 = (b << z) | (c >> (32 - z));
    rest |= c << z;
  }
  if (rest) t0 |= 1u;  // sticky, 11 bits below the double's last place
  const double m = (double)t1 * 4294967296.0 + (double)t0;  // the one rounding
  const int e = 32 * top - 32 - z;  // value = (t1:t0) 2^e
  return ldexp(neg ? -m : m, e - s);
}
