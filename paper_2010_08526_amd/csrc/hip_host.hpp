// Host-side helpers shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace spg {

int hip_fail(hipError_t e);
int read_header(WsHeader *dev, hipStream_t st, WsHeader *out);  // synchronizes st
int device_cus();
// keep_tag: the zero_region_tag of the caller's accumulator region (the
// header's clean_tag survives only if it equals it), 0, or kKeepAnyTag
int launch_init_header(WsHeader *h, uint64_t keep_tag, hipStream_t st);
int launch_set_tag(WsHeader *h, uint64_t tag, hipStream_t st);
// zeroes the bin counters and work-queue cursors only (status, tags kept)
int launch_reset_counters(WsHeader *h, hipStream_t st);
// Row sort of C's columns into (ro, vo) with column lists in `lists`
// (3 * C->ncols int32) and counters in hdr's bin_count[0..2] (zero on
// entry).  Columns that esc_class(skip_flops[j], nnz_j, skip_cf) places in
// an expand-sort-compress kernel are skipped (skip_flops NULL: none).
int sort_column_lists(const spgemm_csc *C, int32_t *ro, void *vo, int32_t *lists, WsHeader *hdr,
                      const int64_t *skip_flops, double skip_cf, hipStream_t st);
int g_min_bin_value();  // the spgemm_debug_min_bin setting
BinCaps bin_caps(int which);  // 0: symbolic, 1: numeric / merge / masked product
// colptr_out[0] = 0, colptr_out[i+1] = counts[0] + ... + counts[i]; bsum holds n / 8192 + 2 int64
int launch_colptr_scan(const int64_t *counts, int64_t n, int64_t *colptr_out, int64_t *bsum, hipStream_t st);

inline unsigned grid_of(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

#define HIPCHK(x)                              \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)
#define LAUNCHCHK()                            \
  do {                                         \
    hipError_t e_ = hipGetLastError();         \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

}  // namespace spg
