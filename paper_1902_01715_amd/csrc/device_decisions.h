// Device forms of the set-up decision primitives: the quantiser of decision
// quantities and the node hash of the independent-set order.  Both are the
// host's operations bit for bit (integer arithmetic; IEEE rounding only where
// the host rounds the same way).  Included by the set-up kernel files, which
// are compiled with -ffp-contract=off.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace aspamg {

// s rounded to `bits` significant bits, ties to even: the host quantiser of
// the set-up decisions, for the device (normal values by integer operations on
// the significand; zero, subnormal and non-finite values by frexp / ldexp).
__device__ __forceinline__ double quantize_dev(double s, int bits) {
  uint64_t u = (uint64_t)__double_as_longlong(s);
  const uint64_t ex = (u >> 52) & 0x7FF;
  if (ex == 0 || ex == 0x7FF) {
    if (s == 0.0 || !isfinite(s)) return s;
    int e;
    const double m = frexp(s, &e);
    const double r = nearbyint(ldexp(m, bits));
    return ldexp(r, e - bits);
  }
  const int drop = 53 - bits;
  const uint64_t mask = (1ULL << drop) - 1, half = 1ULL << (drop - 1);
  const uint64_t rem = u & mask;
  u &= ~mask;
  if (rem > half || (rem == half && ((u >> drop) & 1))) u += 1ULL << drop;
  return __longlong_as_double((long long)u);
}

// splitmix64 finaliser of x + golden gamma: the key of the independent-set order
__device__ __forceinline__ uint64_t mix64_dev(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

}  // namespace aspamg
