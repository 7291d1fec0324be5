// Semirings of the product (Sec. II-A: the algorithms need nothing beyond a
// semiring's two operations, so they apply to any of them).  A product term
// is mul(A(i,k), B(k,j)); the terms of one output entry are combined with
// the semiring's addition.  Every accumulator is an 8-byte slot whose
// all-zero bit pattern means "no term yet", so tables and accumulator
// regions are cleared to zero whatever the semiring:
//   plus-times: the float64 sum (the ordinary product);
//   min-plus  : the float64 minimum, kept as the complement of an
//               order-preserving unsigned image of the value, so that an
//               unsigned atomic max combines terms and 0 is above every
//               value (the tropical product: shortest paths);
//   or-and    : no value at all -- every structural entry is true, written
//               as 1 (the pattern product).
// Structure is kept apart from the slot (hash keys or occupancy bitmaps),
// so an entry exists wherever a term exists, as in the plain product.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spgemm.h"

namespace spg {

struct SrPlusTimes {
  static constexpr int kId = SPGEMM_SR_PLUS_TIMES;
  __device__ static __forceinline__ double mul(double a, double b) { return a * b; }
  __device__ static __forceinline__ void acc(double *slot, double t) { atomicAdd(slot, t); }
  // the same combination by one thread, on a slot in a register
  __device__ static __forceinline__ void acc_plain(double &slot, double t) { slot += t; }
  __device__ static __forceinline__ double out(double slot) { return slot; }
};

// Order-preserving map of float64 onto uint64 (negative values: all bits
// flipped; others: sign bit set), and its inverse.
__device__ __forceinline__ uint64_t ord_key(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double ord_val(uint64_t k) {
  const uint64_t b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)b);
}

struct SrMinPlus {
  static constexpr int kId = SPGEMM_SR_MIN_PLUS;
  __device__ static __forceinline__ double mul(double a, double b) { return a + b; }
  __device__ static __forceinline__ void acc(double *slot, double t) {
    atomicMax((unsigned long long *)slot, (unsigned long long)~ord_key(t));
  }
  __device__ static __forceinline__ void acc_plain(double &slot, double t) {
    const uint64_t s = (uint64_t)__double_as_longlong(slot), k = ~ord_key(t);
    slot = __longlong_as_double((long long)(k > s ? k : s));
  }
  __device__ static __forceinline__ double out(double slot) {
    return ord_val(~(uint64_t)__double_as_longlong(slot));
  }
};

struct SrOrAnd {
  static constexpr int kId = SPGEMM_SR_OR_AND;
  __device__ static __forceinline__ double mul(double, double) { return 1.0; }
  __device__ static __forceinline__ void acc(double *, double) {}
  __device__ static __forceinline__ void acc_plain(double &, double) {}
  __device__ static __forceinline__ double out(double) { return 1.0; }
};

// Terms passed through unchanged (the merge adds entries of partial
// products, which are already semiring products).
struct MulFirst {
  __device__ static __forceinline__ double mul(double a, double) { return a; }
};

}  // namespace spg
