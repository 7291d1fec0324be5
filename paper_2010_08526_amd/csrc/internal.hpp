// Internal declarations shared by the host-only translation unit (host.cpp)
// and the HIP translation unit (kernels.hip).  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/spgemm.h"

namespace spg {

// ----------------------------------------------------------------------------
// Hash-table bins.  A column is placed in the first bin whose capacity
// covers its bound on distinct output rows: min(flops, nrows) in the
// symbolic pass, the exact count from the symbolic pass in the numeric pass
// and the merge.  Tables are sized to at least twice the capacity (load
// factor <= 0.5, linear probing).
//   wave bins : one 64-lane wavefront per column, table private to it (LDS)
//   block bins: one workgroup per column, table shared by its waves (LDS)
//   last bin  : "heavy" -- symbolic uses an LDS bitmap over row windows,
//               numeric and merge use dense float64 accumulators in global
//               memory (the workspace), several workgroups per column.
// ----------------------------------------------------------------------------
constexpr int kNumBins = 6;
// symbolic (keys only, 4 bytes per slot)
constexpr int64_t kSymCap[kNumBins - 1] = {32, 128, 512, 2048, 16384};
// numeric / merge (int32 key + float64 value, 12 bytes per slot)
constexpr int64_t kNumCap[kNumBins - 1] = {32, 128, 512, 2048, 5120};

// Largest capacity each LDS bin's table allows (half its slots).
constexpr int64_t kSymTableCap[kNumBins - 1] = {32, 128, 512, 2048, 16384};
constexpr int64_t kNumTableCap[kNumBins - 1] = {32, 128, 512, 2048, 5120};

// Bin thresholds passed to the binning kernels (monotone, each at most the
// table capacity of its bin).
struct BinCaps {
  int64_t cap[kNumBins - 1];
};

constexpr int kMaxParts = 4096;  // merge: parts per call

// Row-sorted product (spgemm_numeric_sorted): a column with at most
// kEscBlockTerms product terms whose compression ratio flops / nnz is at
// most cf_max is formed by expand-sort-compress (every term placed in LDS,
// sorted by row, equal rows combined in order), one wavefront per column up
// to kEscWaveTerms terms, one workgroup above; every other column is hashed
// and sorted afterwards.  Returns the kernel class (0, 1) or -1 (hashed).
constexpr int64_t kEscWaveTerms = 64;
constexpr int64_t kEscBlockTerms = 4096;
constexpr int esc_class(int64_t flops, int64_t nnz, double cf_max) {
  return (nnz <= 0 || flops > kEscBlockTerms || (double)flops > cf_max * (double)nnz) ? -1
         : (flops <= kEscWaveTerms ? 0 : 1);
}
constexpr size_t kPartDescBytes = 24;  // device-side copy of one part's pointers
constexpr int64_t kBitmapRows = 1 << 20;  // heavy symbolic: rows per LDS bitmap window (128 KiB)
constexpr int64_t kHeavySeg = 16384;  // global heavy path: rows per compaction segment
constexpr int kMaxAdeg = 1 << 25;  // per-column degree of the left operand handled per chunk

// Heavy numeric columns: the left operand's entries are bucketed by row slab
// of 2^kSlabShift rows.  A heavy column is cut into independent items: runs of
// consecutive slabs whose flop bounds add up to at most kHvCap (an LDS hash
// table of kHvSlots slots), or one slab whose bound exceeds kHvCap (a dense
// LDS accumulator of kSlabRows rows).  Columns with more than kHvWideT
// entries in B(:,j) skip the bounds: they are formed kHvWideSlabs slabs at a
// time on a larger dense LDS accumulator (one workgroup per CU).
constexpr int kSlabShift = 12;
constexpr int64_t kSlabRows = int64_t(1) << kSlabShift;
constexpr int kMaxSlabs = 2048;  // rows up to kMaxSlabs * kSlabRows use slabs
constexpr uint64_t kMaxSlabOffBytes = uint64_t(8) << 30;  // cap on the slab offset table
constexpr int kSegLenBits = kSlabShift + 1;  // a segment of one slab holds at most kSlabRows entries
constexpr int kHvSlots = 2560;
constexpr int kHvCap = kHvSlots / 2;
constexpr int64_t kHvWideT = 1024;
constexpr uint64_t kHvItemBytes = uint64_t(64) << 20;  // item list of one chunk of heavy columns
constexpr size_t kSlabEntBytes[2] = {8, 16};  // one slabbed entry of A (row and value): float32, float64
constexpr int64_t kMbBucket = int64_t(1) << 29;  // merge: entries bucketed at once (heavy columns)

inline int64_t num_slabs(int64_t m) { return (m + kSlabRows - 1) / kSlabRows; }

// Slot table capacity (slots of 4 bytes) for ncol columns and P slabs: a
// chunk of at most this many slots over P heavy columns is planned at once.
inline int64_t hv_item_cap(int64_t ncol, int64_t P) {
  const int64_t lim = (int64_t)(kHvItemBytes / 4);
  int64_t c = ncol * P;
  if (c > lim) c = lim;
  if (c < P) c = P;
  return c;
}

// Workspace header: one 4 KiB block at offset 0.
struct WsHeader {
  int32_t status;  // 0 = ok; nonzero = a device-side check failed
  int32_t pad0;
  uint64_t clean_tag;  // zero_region_tag of the accumulator region known to be all zero; 0 = none
  int32_t bin_count[kNumBins];
  int32_t items;        // heavy items listed for the current chunk
  int32_t item_cursor;  // work-queue position over those items
  int32_t cursor[kNumBins];  // work-queue positions of the persistent kernels
  int32_t nwide;        // wide heavy columns listed for the current chunk
  int32_t wide_cursor;  // work-queue position over their items
  int32_t mb_cursor;    // merge: work-queue position over the chunk's heavy columns (bucketing)
  int32_t split_cursor; // numeric: work-queue position over the columns of A (slabbed copy)
  uint64_t left_tag;    // fingerprint (| 1) of the source of the slabbed copy of A in the workspace; 0 = none
  uint64_t left_new;    // fingerprint of the current call's left operand (summed by k_left_sum)
  int32_t esc_count[2];  // row-sorted product: columns listed for the two expand-sort-compress kernels
};
constexpr size_t kHeaderBytes = 4096;

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Number of heavy accumulator slots (columns accumulated at once) for m rows:
// about 1 GiB of float64 values plus one flag byte per row and slot.
inline int64_t heavy_slots(int64_t m) {
  if (m <= 0) return 1;
  int64_t s = (int64_t(1) << 30) / (9 * m);
  if (s < 8) s = 8;
  if (s > 256) s = 256;
  return s;
}

struct WsLayout {
  size_t bins = 0;        // int32 [kNumBins][ncol]
  size_t heavy_vals = 0;  // double [slots][m]
  size_t heavy_flags = 0; // uint8 [slots][m]
  size_t heavy_segcnt = 0;// int64 [slots][nseg]
  size_t scan = 0;        // int64 block sums
  size_t parts = 0;       // merge: part descriptors
  size_t slab_off = 0;    // numeric: int32 [kcols][P+1] slab offsets of the left operand
  size_t slab_ent = 0;    // numeric: [nnzA] slabbed entries of A (row and value side by side)
  size_t slab_ri = 0;     // merge: int32 [mb_cap] bucketed rows
  size_t slab_v = 0;      // merge: 8-byte [mb_cap] bucketed values
  size_t slab_pack = 0;   // numeric: uint64 [P][kcols] slab segments, slab-major (start << kSegLenBits | len)
  size_t hv_cur = 0;      // numeric: int32 [ncol] output cursor per heavy column
  size_t hv_items = 0;    // numeric: uint32 [hv_item_cap] heavy item slots of one chunk
  size_t hv_wide = 0;     // numeric: int32 [ncol] wide heavy columns of one chunk
  size_t mb_len = 0;      // merge: int64 [ncol] entries of every heavy column over the parts
  size_t mb_base = 0;     // merge: int64 [ncol+1] their exclusive scan
  int64_t mb_cap = 0;     // merge: entries of the bucket region (slab_ri / slab_v)
  size_t bl_cnt = 0;      // layers: int64 [ncol] entries of one layer per column
  size_t bl_cp = 0;       // layers: int64 [ncol+1] column pointers of the layer's share of B
  size_t bl_scan = 0;     // layers: int64 block sums of that scan
  size_t bl_ri = 0;       // layers: int32 [nnz(B)] rows of the layer's share of B
  size_t bl_v = 0;        // layers: 8-byte [nnz(B)] values (numeric only)
  int64_t bl_cap = 0;     // layers: entries the two arrays hold (0 = no split)
  size_t pr_cnt = 0;      // prune: int64 [ncol] entries each column keeps
  size_t pr_cutv = 0;     // prune: uint64 [ncol] value key of the smallest kept entry
  size_t pr_cutr = 0;     // prune: uint32 [ncol] row key of the smallest kept entry
  int64_t P = 0;          // numeric: slabs (0 = heavy columns use global accumulators)
  size_t total = 0;
  int64_t slots = 0, nseg = 0, ncol = 0, m = 0;
};

// Zero-filled accumulator regions.  The global heavy path (product and
// merge) and the masked product keep their dense accumulators all zero
// between calls (each call clears what it used), so a call may skip the fill
// when the header's clean_tag says the region it is about to use was left
// zero by a call with the same region.  The tag names the region: its kind,
// offsets, slot count and rows.  Every call that initialises the header
// passes the tag of its own region (or 0 if it has none, which clears the
// tag: its layout may put other data there); kKeepAnyTag is for calls that
// write nothing but the header.
constexpr uint64_t kKeepAnyTag = ~0ull;
enum : uint64_t { kTagProduct = 0x70726f64ull, kTagMasked = 0x6d787479ull };
inline uint64_t zero_region_tag(uint64_t kind, const WsLayout &L) {
  if (L.slots <= 0 || L.heavy_vals == 0) return 0;
  uint64_t t = kind;
  const uint64_t parts[6] = {(uint64_t)L.heavy_vals, (uint64_t)L.heavy_flags, (uint64_t)L.heavy_segcnt,
                             (uint64_t)L.slots,      (uint64_t)L.m,           (uint64_t)L.nseg};
  for (uint64_t x : parts) {
    t = (t ^ x) * 0x9e3779b97f4a7c15ull;
    t ^= t >> 29;
  }
  t |= 1;  // never 0 (no region)
  return t == kKeepAnyTag ? t - 2 : t;
}

// Computes the layout; returns SPGEMM_OK or an error status.
int ws_layout(int op, const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t c1, int32_t n_layers,
              WsLayout *out);

// Host-side argument checks shared by the entry points.
int check_csc(const spgemm_csc *M, bool need_values);
int check_ws(const void *ws, size_t ws_bytes, size_t need);
int dtype_bytes(int32_t dtype);

void set_hip_error(int code);

}  // namespace spg
