// Host-only part of the library: status text, argument checks, workspace
// sizing and the batch planner.  Nothing here touches a GPU, so all of it
// can be exercised on a machine without one.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace spg {

static thread_local int g_last_hip_error = 0;
void set_hip_error(int code) { g_last_hip_error = code; }

int dtype_bytes(int32_t dtype) {
  if (dtype == SPGEMM_F32) return 4;
  if (dtype == SPGEMM_F64) return 8;
  return 0;
}

int check_csc(const spgemm_csc *M, bool need_values) {
  if (!M) return SPGEMM_E_INVAL;
  if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0) return SPGEMM_E_INVAL;
  if (M->nrows > INT32_MAX) return SPGEMM_E_OVERFLOW;
  if (!M->colptr) return SPGEMM_E_INVAL;
  if (M->nnz > 0 && !M->rowidx) return SPGEMM_E_INVAL;
  if (need_values) {
    if (!dtype_bytes(M->dtype)) return SPGEMM_E_DTYPE;
    if (M->nnz > 0 && !M->values) return SPGEMM_E_INVAL;
  } else if (M->values && !dtype_bytes(M->dtype)) {
    return SPGEMM_E_DTYPE;
  }
  return SPGEMM_OK;
}

int check_ws(const void *ws, size_t ws_bytes, size_t need) {
  if (!ws) return SPGEMM_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return SPGEMM_E_WORKSPACE;
  if (ws_bytes < need) return SPGEMM_E_WORKSPACE;
  return SPGEMM_OK;
}

int ws_layout(int op, const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t c1, int32_t n_layers,
              WsLayout *L) {
  if (!L) return SPGEMM_E_INVAL;
  *L = WsLayout();
  size_t off = kHeaderBytes;
  switch (op) {
    case SPGEMM_OP_SYMBOLIC:
    case SPGEMM_OP_NUMERIC:
    case SPGEMM_OP_BATCHED_FORWARD:
    case SPGEMM_OP_MERGE: {
      if (!A) return SPGEMM_E_INVAL;
      int64_t ncol;
      if (op == SPGEMM_OP_MERGE) {
        ncol = A->ncols;
        if (n_layers < 1 || n_layers > kMaxParts) return SPGEMM_E_INVAL;
      } else {
        if (!B || c0 < 0 || c1 < c0 || c1 > B->ncols || n_layers < 1) return SPGEMM_E_INVAL;
        ncol = c1 - c0;
      }
      if (A->nrows < 0 || A->nrows > INT32_MAX) return SPGEMM_E_OVERFLOW;
      L->ncol = ncol;
      L->m = A->nrows;
      const bool numeric = op == SPGEMM_OP_NUMERIC || op == SPGEMM_OP_BATCHED_FORWARD;
      const int64_t P = num_slabs(A->nrows);
      // columns of A one call reads: one layer of ceil(k / n_layers) columns
      const int64_t kcols = (A->ncols + n_layers - 1) / n_layers;
      // (entries of the slabbed copy are addressed with 32-bit indices)
      const bool slabs = numeric && A->nrows > kNumCap[kNumBins - 2] && P <= kMaxSlabs && A->nnz <= INT32_MAX &&
                         sizeof(int32_t) * (uint64_t)(P + 1) * (uint64_t)kcols <= kMaxSlabOffBytes;
      if (slabs) {
        // the slabbed copy of A depends only on A and the layer: it comes
        // first, so that calls on other column ranges find it at the same
        // offsets (and may reuse it)
        L->P = P;
        L->slab_off = off;
        off = align_up(off + sizeof(int32_t) * (size_t)(L->P + 1) * (size_t)kcols);
        L->slab_pack = off;
        off = align_up(off + sizeof(uint64_t) * (size_t)L->P * (size_t)kcols);
        L->slab_ent = off;
        off = align_up(off + kSlabEntBytes[A->dtype == SPGEMM_F64 ? 1 : 0] * (size_t)A->nnz);
      }
      L->bins = off;
      // numeric: two more lists, for the row-sorted product's columns formed
      // by expand-sort-compress
      off = align_up(off + sizeof(int32_t) * (kNumBins + (op == SPGEMM_OP_NUMERIC ? 2 : 0)) * (size_t)ncol);
      if (op == SPGEMM_OP_MERGE) {
        L->parts = off;
        off = align_up(off + kPartDescBytes * (size_t)n_layers);
      }
      if (slabs) {
        L->hv_cur = off;
        off = align_up(off + sizeof(int32_t) * (size_t)ncol);
        L->hv_items = off;
        off = align_up(off + 4 * (size_t)hv_item_cap(ncol, P));
        L->hv_wide = off;
        off = align_up(off + sizeof(int32_t) * (size_t)ncol);
      } else if (op == SPGEMM_OP_MERGE && A->nrows > kNumCap[kNumBins - 2] && P <= kMaxSlabs) {
        // heavy merge columns: slab buckets of up to kMbBucket entries
        const int64_t icap = hv_item_cap(ncol, P);
        const int64_t hcap = std::max<int64_t>(1, icap / P);
        L->P = P;
        // a column holds at most one entry per row and part
        int64_t cap = std::min<int64_t>(kMbBucket, ncol);
        cap = std::min<int64_t>(kMbBucket, cap * n_layers);
        L->mb_cap = std::min<int64_t>(kMbBucket, cap * A->nrows);
        L->mb_len = off;
        off = align_up(off + sizeof(int64_t) * (size_t)ncol);
        L->mb_base = off;
        off = align_up(off + sizeof(int64_t) * (size_t)(ncol + 1));
        L->scan = off;
        off = align_up(off + sizeof(int64_t) * (size_t)(ncol / 8192 + 2));
        L->slab_off = off;
        off = align_up(off + sizeof(int32_t) * (size_t)hcap * (size_t)(P + 1));
        L->hv_items = off;
        off = align_up(off + 4 * (size_t)icap);
        L->hv_cur = off;
        off = align_up(off + sizeof(int32_t) * (size_t)ncol);
        L->slab_ri = off;
        off = align_up(off + sizeof(int32_t) * (size_t)L->mb_cap);
        L->slab_v = off;
        off = align_up(off + sizeof(double) * (size_t)L->mb_cap);
      } else if ((op == SPGEMM_OP_NUMERIC || op == SPGEMM_OP_MERGE) && A->nrows > kNumCap[kNumBins - 2]) {
        L->slots = heavy_slots(A->nrows);
        L->nseg = (A->nrows + kHeavySeg - 1) / kHeavySeg;
        L->heavy_vals = off;
        off = align_up(off + sizeof(double) * (size_t)L->slots * (size_t)A->nrows);
        L->heavy_flags = off;
        off = align_up(off + (size_t)L->slots * (size_t)A->nrows);
        L->heavy_segcnt = off;
        off = align_up(off + sizeof(int64_t) * (size_t)L->slots * (size_t)L->nseg);
      }
      if ((op == SPGEMM_OP_SYMBOLIC || op == SPGEMM_OP_NUMERIC) && n_layers > 1) {
        // the entries of B(:, c0:c1) in one inner-dimension layer, as a CSC matrix
        if (B->nnz < 0) return SPGEMM_E_INVAL;
        L->bl_cap = B->nnz;
        L->bl_cnt = off;
        off = align_up(off + sizeof(int64_t) * (size_t)ncol);
        L->bl_cp = off;
        off = align_up(off + sizeof(int64_t) * (size_t)(ncol + 1));
        L->bl_scan = off;
        off = align_up(off + sizeof(int64_t) * (size_t)(ncol / 8192 + 2));
        L->bl_ri = off;
        off = align_up(off + sizeof(int32_t) * (size_t)B->nnz);
        if (op == SPGEMM_OP_NUMERIC) {
          L->bl_v = off;
          off = align_up(off + sizeof(double) * (size_t)B->nnz);
        }
      }
      if (op == SPGEMM_OP_BATCHED_FORWARD) {
        L->scan = off;
        off = align_up(off + sizeof(int64_t) * (size_t)(ncol / 8192 + 2));
      }
      break;
    }
    case SPGEMM_OP_TRANSPOSE: {
      if (!A) return SPGEMM_E_INVAL;
      if (A->nrows < 0 || A->nrows > INT32_MAX) return SPGEMM_E_OVERFLOW;
      L->m = A->nrows;
      L->bins = off;  // int64 row counts, then cursors
      off = align_up(off + sizeof(int64_t) * (size_t)A->nrows);
      L->scan = off;
      off = align_up(off + sizeof(int64_t) * (size_t)(A->nrows / 8192 + 2));
      break;
    }
    case SPGEMM_OP_MASKED_XTY: {
      if (!A || !B) return SPGEMM_E_INVAL;
      if (B->nrows < 0 || B->nrows > INT32_MAX) return SPGEMM_E_OVERFLOW;
      L->ncol = B->ncols;
      L->m = B->nrows;
      L->bins = off;
      off = align_up(off + sizeof(int32_t) * kNumBins * (size_t)B->ncols);
      if (B->nrows > kNumCap[kNumBins - 2]) {
        L->slots = heavy_slots(B->nrows);
        L->heavy_vals = off;
        off = align_up(off + sizeof(double) * (size_t)L->slots * (size_t)B->nrows);
      }
      break;
    }
    case SPGEMM_OP_BATCHED_BACKWARD: {  // A, B of the product
      if (!A || !B) return SPGEMM_E_INVAL;
      if (A->nrows < 0 || A->nrows > INT32_MAX) return SPGEMM_E_OVERFLOW;
      L->ncol = B->ncols;
      L->m = A->nrows;
      L->bins = off;
      off = align_up(off + sizeof(int32_t) * kNumBins * (size_t)B->ncols);
      L->heavy_vals = off;  // float64 accumulators of dA
      off = align_up(off + sizeof(double) * (size_t)A->nnz);
      break;
    }
    case SPGEMM_OP_PRUNE: {  // A = the matrix pruned
      if (!A) return SPGEMM_E_INVAL;
      if (A->ncols < 0) return SPGEMM_E_INVAL;
      const size_t n = (size_t)A->ncols;
      L->ncol = A->ncols;
      L->pr_cnt = off;
      off = align_up(off + sizeof(int64_t) * n);
      L->pr_cutv = off;
      off = align_up(off + sizeof(uint64_t) * n);
      L->pr_cutr = off;
      off = align_up(off + sizeof(uint32_t) * n);
      L->scan = off;
      off = align_up(off + sizeof(int64_t) * (n / 8192 + 2));
      break;
    }
    case SPGEMM_OP_SORT: {  // A = the matrix sorted: column lists of three length classes
      if (!A) return SPGEMM_E_INVAL;
      if (A->ncols < 0) return SPGEMM_E_INVAL;
      L->ncol = A->ncols;
      L->m = A->nrows;
      L->bins = off;
      off = align_up(off + sizeof(int32_t) * 3 * (size_t)A->ncols);
      break;
    }
    case SPGEMM_OP_COLPTR: {
      if (c0 < 0 || c1 < c0) return SPGEMM_E_INVAL;
      int64_t n = c1 - c0;
      L->scan = off;
      off = align_up(off + sizeof(int64_t) * (size_t)(n / 8192 + 2));
      break;
    }
    default:
      return SPGEMM_E_INVAL;
  }
  L->total = off;
  return SPGEMM_OK;
}

}  // namespace spg

using namespace spg;

extern "C" {

const char *spgemm_status_string(int status) {
  switch (status) {
    case SPGEMM_OK: return "ok";
    case SPGEMM_E_INVAL: return "invalid argument";
    case SPGEMM_E_SHAPE: return "shape mismatch";
    case SPGEMM_E_DTYPE: return "unsupported or mixed dtype";
    case SPGEMM_E_BUDGET: return "memory budget too small";
    case SPGEMM_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case SPGEMM_E_HIP: return "HIP runtime error";
    case SPGEMM_E_OVERFLOW: return "size overflows the index types";
    case SPGEMM_E_DEVICE: return "device-side check failed";
    default: return "unknown status";
  }
}

int spgemm_last_hip_error(void) { return g_last_hip_error; }

int spgemm_workspace_size(int op, const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t c1,
                          int32_t n_layers, size_t *bytes_host) {
  if (!bytes_host) return SPGEMM_E_INVAL;
  WsLayout L;
  int st = ws_layout(op, A, B, c0, c1, n_layers, &L);
  if (st != SPGEMM_OK) return st;
  *bytes_host = L.total;
  return SPGEMM_OK;
}

int spgemm_plan_batches(const int64_t *nnz_host, int64_t ncols, int32_t n_layers, int32_t value_bytes,
                        uint64_t input_bytes, uint64_t budget_bytes, uint64_t reserve_bytes, int32_t max_batches,
                        int64_t *bounds_host, int32_t *nbatches_host, int64_t *batch_nnz_host) {
  if (ncols < 0 || n_layers < 1 || max_batches < 1 || !bounds_host || !nbatches_host) return SPGEMM_E_INVAL;
  if (ncols > 0 && !nnz_host) return SPGEMM_E_INVAL;
  if (value_bytes != 4 && value_bytes != 8) return SPGEMM_E_DTYPE;
  if (input_bytes > budget_bytes || reserve_bytes > budget_bytes - input_bytes) return SPGEMM_E_BUDGET;
  const uint64_t avail = budget_bytes - input_bytes - reserve_bytes;
  if (avail == 0) return SPGEMM_E_BUDGET;
  const int rows = n_layers > 1 ? n_layers + 1 : 1;
  const uint64_t r = 4 + (uint64_t)value_bytes;
  const size_t n = (size_t)ncols;

  // Memory of every output column and its prefix sums.
  std::vector<uint64_t> pre(n + 1, 0);
  uint64_t maxcol = 0;
  for (size_t j = 0; j < n; j++) {
    uint64_t mem;
    if (n_layers == 1) {
      int64_t u = nnz_host[j];
      if (u < 0) return SPGEMM_E_INVAL;
      mem = r * (uint64_t)u + 8;
    } else {
      uint64_t parts = 0;
      for (int l = 0; l < n_layers; l++) {
        int64_t u = nnz_host[(size_t)l * n + j];
        if (u < 0) return SPGEMM_E_INVAL;
        parts += (uint64_t)u;
      }
      int64_t u = nnz_host[(size_t)n_layers * n + j];
      if (u < 0) return SPGEMM_E_INVAL;
      mem = r * parts + 8 * (uint64_t)n_layers + r * (uint64_t)u + 8;
    }
    if (mem > avail) return SPGEMM_E_BUDGET;
    maxcol = std::max(maxcol, mem);
    pre[j + 1] = pre[j] + mem;
  }
  const uint64_t total = pre[n];

  // Greedy packing from the left under `cap`: every batch extends to the
  // last column that keeps it within cap.  Returns the number of batches
  // (at least 1) and optionally the bounds.
  auto greedy = [&](uint64_t cap, int64_t *bounds, int64_t limit) -> int64_t {
    size_t pos = 0;
    int64_t cnt = 0;
    if (bounds) bounds[0] = 0;
    while (pos < n) {
      // largest e in (pos, n] with pre[e] - pre[pos] <= cap
      size_t e = (size_t)(std::upper_bound(pre.begin() + pos + 1, pre.end(), pre[pos] + cap) - pre.begin()) - 1;
      pos = e;
      cnt++;
      if (bounds && cnt <= limit) bounds[cnt] = (int64_t)pos;
    }
    if (cnt == 0) {
      cnt = 1;
      if (bounds) bounds[1] = 0;
    }
    return cnt;
  };

  const int64_t b = greedy(avail, nullptr, 0);
  if (b > max_batches) return SPGEMM_E_BUDGET;
  uint64_t lo = std::max(maxcol, (total + (uint64_t)b - 1) / (uint64_t)b);
  uint64_t hi = avail;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (greedy(mid, nullptr, 0) <= b)
      hi = mid;
    else
      lo = mid + 1;
  }
  greedy(lo, bounds_host, b);
  *nbatches_host = (int32_t)b;
  if (batch_nnz_host) {
    for (int64_t i = 0; i < b; i++) {
      for (int rr = 0; rr < rows; rr++) {
        int64_t s = 0;
        for (int64_t j = bounds_host[i]; j < bounds_host[i + 1]; j++) s += nnz_host[(size_t)rr * n + (size_t)j];
        batch_nnz_host[i * rows + rr] = s;
      }
    }
  }
  return SPGEMM_OK;
}

}  // extern "C"
