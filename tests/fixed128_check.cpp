// Host check of the 128-bit fixed-point conversions used by the incremental
// centroid update, against the compiler's own 128-bit integer arithmetic:
// long double scaling (64-bit significand, exact for a double times 2^s)
// truncated to __int128, and the correctly rounded __int128 -> double
// conversion.  Also checks, on the same cases, an earlier form of the
// fixed-point -> double conversion written with 64-bit variable shifts
// (fx_to_double_shift64 below), which the library no longer uses.  Prints the
// number of mismatches; exit status 1 on any.  Built both plainly and with
// the address and undefined-behaviour sanitizers by the test that runs it.
#include <cstdio>
#include <random>

#include "../paper_1705_01813_amd/csrc/fixed128.h"

static __int128 want_of_double(double v, int s) {
  const long double a = std::ldexp((long double)std::fabs(v), s);
  const unsigned __int128 mag = (unsigned __int128)a;
  return v < 0 ? -(__int128)mag : (__int128)mag;
}

// The earlier conversion: the 64 bits below the leading one taken with 64-bit
// shifts of the two words, a sticky bit for the rest, one rounding through
// (double) of a 64-bit integer, then two exact power-of-two scalings.
static double fx_to_double_shift64(uint64_t hi, uint64_t lo, int s) {
  const bool neg = (int64_t)hi < 0;
  if (neg) fx_neg(hi, lo);
  double m;
  if (hi == 0) {
    m = (double)lo;
  } else {
    const int lz = __builtin_clzll(hi);
    const int sh = 64 - lz;
    uint64_t top = lz ? ((hi << lz) | (lo >> (64 - lz))) : hi;
    const uint64_t rest = sh >= 64 ? lo : (lo & ((1ull << sh) - 1));
    if (rest) top |= 1;
    m = std::ldexp((double)top, sh);
  }
  return std::ldexp(neg ? -m : m, -s);
}

static __int128 join(uint64_t hi, uint64_t lo) { return (__int128)(((unsigned __int128)hi << 64) | lo); }

static long bad_shift64 = 0;

static long check_to(__int128 x, int s) {
  const double want = std::ldexp((double)x, -s);
  const uint64_t hi = (uint64_t)((unsigned __int128)x >> 64), lo = (uint64_t)x;
  bad_shift64 += fx_to_double_shift64(hi, lo, s) != want;
  return fx_to_double(hi, lo, s) != want;
}

int main(int argc, char** argv) {
  const long N = argc > 1 ? std::atol(argv[1]) : 2000000;
  std::mt19937_64 g(20170505);
  long bad_of = 0, bad_to = 0;
  // edge cases: zeros, subnormals, powers of two, all-ones words, ties
  const double specials[] = {0.0, -0.0, 0x1p-1074, -0x1p-1074, 0x1p-1022, 1.0, -1.0, 0x1.fffffffffffffp0,
                             0x1p30, -0x1p30, 3.0e-8, -7.25};
  for (double v : specials)
    for (int s = 0; s <= 120; ++s) {
      if (std::fabs(v) * std::ldexp(1.0, s) >= 0x1p125) continue;
      uint64_t hi, lo;
      fx_of_double(v, s, hi, lo);
      bad_of += join(hi, lo) != want_of_double(v, s);
    }
  for (int b = 0; b < 125; ++b) {
    const unsigned __int128 one = (unsigned __int128)1 << b;
    for (int k = -1; k <= 1; ++k) {
      const __int128 x = (__int128)(one + k);
      bad_to += check_to(x, 90) + check_to(-x, 90);
    }
    // exact ties at the 53-bit boundary, with and without a sticky bit below
    if (b >= 60) {
      // a random (b+1)-bit value with its top bit set (b = 60..62 shift right)
      const unsigned __int128 top = (unsigned __int128)g() | ((unsigned __int128)1 << 63);
      const unsigned __int128 base = b >= 63 ? top << (b - 63) : top >> (63 - b);
      const unsigned __int128 half = (unsigned __int128)1 << (b - 53);
      bad_to += check_to((__int128)(base | half), 7) + check_to((__int128)((base | half) + 1), 7);
    }
  }
  for (long i = 0; i < N; ++i) {
    const int s = (int)(g() % 121);
    const int ee = (int)(g() % 140) - 120 - ((g() & 1) ? 0 : 900);
    double v = std::ldexp((double)(g() >> 11) * 0x1p-53 + 0.5, ee);
    if (g() & 1) v = -v;
    if (std::fabs(v) * std::ldexp(1.0, s) < 0x1p125) {
      uint64_t hi, lo;
      fx_of_double(v, s, hi, lo);
      bad_of += join(hi, lo) != want_of_double(v, s);
    }
    const int bits = (int)(g() % 126);
    unsigned __int128 m = ((unsigned __int128)g() << 64) | g();
    m = bits ? m >> (128 - bits) : 0;
    if (g() & 1) m &= ~(unsigned __int128)0 << (g() % 100);
    const __int128 x = (g() & 1) ? -(__int128)m : (__int128)m;
    bad_to += check_to(x, (int)(g() % 121));
  }
  std::printf("fx_of_double mismatches %ld, fx_to_double mismatches %ld, shift64 form mismatches %ld\n", bad_of,
              bad_to, bad_shift64);
  return (bad_of || bad_to || bad_shift64) ? 1 : 0;
}
