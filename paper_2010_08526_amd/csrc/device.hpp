// Wavefront-level building blocks for gfx950 (64-lane wavefronts, GFX9 DPP).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spg {

constexpr int kWave = 64;
constexpr int32_t kEmpty = -1;  // empty hash-table key

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Orders this lane's LDS accesses against the other lanes of its wavefront
// (a compiler barrier plus the wave-scope fence; a wavefront's LDS accesses
// execute in issue order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// DPP move; lanes whose source lies outside the row, or whose row is masked
// off, receive 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp0(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}

// Value of lane l - 1 in lane l (0 in lane 0): the wavefront shift right by
// one lane (DPP wave_shr:1), a VALU move with no LDS round trip.
__device__ __forceinline__ int wave_prev(int v) { return dpp0<0x138>(v); }

// Inclusive prefix sum over the 64 lanes: Hillis-Steele inside each 16-lane
// row (row_shr 1, 2, 4, 8), then row 0's total into row 1 and row 2's total
// into row 3 (row_bcast:15), then lane 31's running total into rows 2 and 3
// (row_bcast:31).
__device__ __forceinline__ int wave_incl_add(int v) {
  v += dpp0<0x111>(v);
  v += dpp0<0x112>(v);
  v += dpp0<0x114>(v);
  v += dpp0<0x118>(v);
  v += dpp0<0x142, 0xa>(v);
  v += dpp0<0x143, 0xc>(v);
  return v;
}

// Per-thread counts -> exclusive offset within the workgroup; `total` gets
// the workgroup's sum.  Contains a barrier.
template <int NW>
__device__ __forceinline__ int block_excl(int c, int *s_w, int &total) {
  const int w = threadIdx.x / kWave, l = lane();
  const int incl = wave_incl_add(c);
  if (l == kWave - 1) s_w[w] = incl;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int z = 0; z < NW; z++) {
    const int v = s_w[z];
    if (z < w) before += v;
    tot += v;
  }
  total = tot;
  return before + incl - c;
}

// Inclusive prefix maximum of non-negative values (0 is the identity).
__device__ __forceinline__ int wave_incl_max(int v) {
  v = max(v, dpp0<0x111>(v));
  v = max(v, dpp0<0x112>(v));
  v = max(v, dpp0<0x114>(v));
  v = max(v, dpp0<0x118>(v));
  v = max(v, dpp0<0x142, 0xa>(v));
  v = max(v, dpp0<0x143, 0xc>(v));
  return v;
}

__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  return __longlong_as_double((long long)readlane64((int64_t)__double_as_longlong(v), l));
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ int wave_sum_i32(int v) { return readlane(wave_incl_add(v), 63); }

// Number of set lanes of `mask` below this lane.
__device__ __forceinline__ int mbcnt(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Fibonacci hashing (multiplier floor(2^32 / golden ratio)) mapped onto
// [0, T) by the high half of a 32x32 product, so T need not be a power of 2.
__device__ __forceinline__ uint32_t hash_slot(int32_t key, uint32_t T) {
  uint32_t h = (uint32_t)key * 2654435769u;
  return (uint32_t)(((uint64_t)h * T) >> 32);
}

// Load-balanced traversal of up to 64 variable-length segments held one per
// lane (length `len`, 0 allowed).  The segments' elements are numbered
// 0..total-1 in lane order; in rounds of 64, lane t handles element
// fb + t and calls body(owner, e) with the owning lane and e, the element's
// number counted from the start of the owner's segment plus the owner's
// exclusive prefix (callers pre-subtract that prefix from their per-segment
// base).  The owner of each element is found by marking segment starts in a
// 64-entry LDS array (`mark`, all zero on entry and on exit) and taking an
// inclusive prefix maximum across lanes.  Returns the total element count.
template <class Body>
__device__ __forceinline__ int wave_flatten(int len, int *mark, Body &&body) {
  const int l = lane();
  const int incl = wave_incl_add(len);
  const int excl = incl - len;
  const int total = readlane(incl, 63);
  int carry = 0;
  for (int fb = 0; fb < total; fb += kWave) {
    if (len > 0 && excl >= fb && excl < fb + kWave) mark[excl - fb] = l + 1;
    wave_sync();
    const int mk = mark[l];
    mark[l] = 0;
    const int own = max(wave_incl_max(mk), carry);
    carry = readlane(own, 63);
    const int e = fb + l;
    if (e < total) body(own - 1, e);
    wave_sync();
  }
  return total;
}

// Load through a pointer that addresses device (global) memory.  A pointer
// read from LDS or from memory is generic to the compiler, which then emits
// flat loads; those also count against the LDS wait counter, so every later
// LDS access waits for them and loads meant to overlap do not.
template <class T>
__device__ __forceinline__ T ld_global(const T *p) {
  return *(const __attribute__((address_space(1))) T *)p;
}

// Returns v unchanged, but the compiler cannot move a use of the result above
// this point: a gathered value used only after every gather of a batch has
// been issued keeps those loads in flight together (no wait between them).
template <class T>
__device__ __forceinline__ T opaque(T v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Device-side status word: first writer wins, value kept for the host.
__device__ __forceinline__ void flag_error(int32_t *status, int code) { atomicCAS(status, 0, code); }

}  // namespace spg
