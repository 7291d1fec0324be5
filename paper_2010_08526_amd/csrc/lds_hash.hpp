// LDS hash tables: open addressing, linear probing, key kEmpty = free slot.
#pragma once

#include "device.hpp"

namespace spg {

// Inserts `key`; returns true if this call created it.  Each probe is one
// compare-and-swap (it finds the key, claims a free slot, or moves on), so
// a new key costs one LDS round trip per probe rather than a load and a swap.
__device__ __forceinline__ bool ht_insert_key(int32_t *keys, uint32_t T, int32_t key) {
  uint32_t h = hash_slot(key, T);
  for (uint32_t probe = 0; probe < T; probe++) {
    const int32_t old = atomicCAS(&keys[h], kEmpty, key);
    if (old == kEmpty) return true;
    if (old == key) return false;
    h = (h + 1 == T) ? 0 : h + 1;
  }
  return false;  // unreachable with tables at most half full
}

// Adds `v` to the slot of `key`, creating it if needed.
__device__ __forceinline__ void ht_accumulate(int32_t *keys, double *vals, uint32_t T, int32_t key, double v) {
  uint32_t h = hash_slot(key, T);
  for (uint32_t probe = 0; probe < T; probe++) {
    const int32_t old = atomicCAS(&keys[h], kEmpty, key);
    if (old == kEmpty || old == key) {
      atomicAdd(&vals[h], v);
      return;
    }
    h = (h + 1 == T) ? 0 : h + 1;
  }
}

// As ht_accumulate, combining values with the addition of semiring SR
// (SR::acc on the slot; slots start all zero).
template <class SR>
__device__ __forceinline__ void ht_accumulate_sr(int32_t *keys, double *vals, uint32_t T, int32_t key, double v) {
  uint32_t h = hash_slot(key, T);
  for (uint32_t probe = 0; probe < T; probe++) {
    const int32_t old = atomicCAS(&keys[h], kEmpty, key);
    if (old == kEmpty || old == key) {
      SR::acc(&vals[h], v);
      return;
    }
    h = (h + 1 == T) ? 0 : h + 1;
  }
}

// As ht_accumulate_sr, and a call that claims a free slot appends the slot
// to `slots` (at most `cap` of them; *n counts every claim), so the table can
// be read out, and cleared, by walking the claimed slots only.
template <class SR>
__device__ __forceinline__ void ht_accumulate_list(int32_t *keys, double *vals, uint32_t T, int32_t key, double v,
                                                   uint16_t *slots, int *n, int cap) {
  uint32_t h = hash_slot(key, T);
  for (uint32_t probe = 0; probe < T; probe++) {
    const int32_t old = atomicCAS(&keys[h], kEmpty, key);
    if (old == kEmpty || old == key) {
      if (old == kEmpty) {
        const int q = atomicAdd(n, 1);
        if (q < cap) slots[q] = (uint16_t)h;
      }
      SR::acc(&vals[h], v);
      return;
    }
    h = (h + 1 == T) ? 0 : h + 1;
  }
}

// As ht_accumulate_sr on a table whose free slots hold 0: keys are stored
// as key + 1 (key < INT32_MAX), so an all-zero table is empty and a pass
// that reads the table out can leave it empty by writing zeros.
template <class SR>
__device__ __forceinline__ void ht_accumulate_z(int32_t *keys, double *vals, uint32_t T, int32_t key, double v) {
  const int32_t kk = key + 1;
  uint32_t h = hash_slot(key, T);
  for (uint32_t probe = 0; probe < T; probe++) {
    const int32_t old = atomicCAS(&keys[h], 0, kk);
    if (old == 0 || old == kk) {
      SR::acc(&vals[h], v);
      return;
    }
    h = (h + 1 == T) ? 0 : h + 1;
  }
}

// Value stored under `key`, or 0 if absent (tables are read-only here).
__device__ __forceinline__ double ht_lookup(const int32_t *keys, const double *vals, uint32_t T, int32_t key) {
  uint32_t h = hash_slot(key, T);
  for (uint32_t probe = 0; probe < T; probe++) {
    const int32_t k = keys[h];
    if (k == key) return vals[h];
    if (k == kEmpty) return 0.0;
    h = (h + 1 == T) ? 0 : h + 1;
  }
  return 0.0;
}

}  // namespace spg
