// HIP kernels and GPU-facing entry points of the SpGEMM library (gfx950).
//
// C = A*B over (+, *) in CSC, one output column at a time (Gustavson's
// column formula, Sec. II-C).  Three passes, each sort-free (Sec. IV-D):
//   symbolic: per-column flops and exact distinct-row counts (Alg. 3,
//             LocalSymbolic) from hash tables of row keys;
//   numeric : hash-table accumulation of A(i,k)*B(k,j) and compaction of
//             the table into the output column in table order;
//   merge   : hash-table addition of the same column of several partial
//             products (Merge-Layer / Merge-Fiber, Alg. 1 and Alg. 2).
// Columns are binned by their bound on distinct rows; see internal.hpp.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <mutex>
#include <type_traits>
#include <vector>

#include "device.hpp"
#include "internal.hpp"
#include "lds_hash.hpp"
#include "hip_host.hpp"
#include "profile.hpp"
#include "semiring.hpp"

namespace spg {

// ============================================================================
// Per-wave scratch for the load-balanced traversal.
// ============================================================================
struct SegScratch {
  int mark[kWave];      // start masks of 32 rounds (flatten_rounds)
  int64_t off[kWave];   // element base of the o-th nonempty short segment minus its exclusive prefix
  double scale[kWave];  // B(k,j) of that segment
};

struct PartDesc {  // one merge input, stored in the workspace
  const int64_t *cp;
  const int32_t *ri;
  const void *v;
};

struct MergeScratch {
  int mark[kWave];           // start masks of 32 rounds (flatten_rounds)
  const int32_t *ri[kWave];  // rows of the o-th nonempty short segment, minus its exclusive prefix
  const void *v[kWave];      // its values, likewise
};

template <class VT>
struct ProductArgs {
  const int64_t *Acp;
  const int32_t *Ari;
  const VT *Av;
  const int64_t *Bcp;
  const int32_t *Bri;
  const VT *Bv;
  int64_t klo, khi, kdim, m, nnzA;
};

// Traversal of the rounds of one chunk of segments.  The caller lists the
// chunk's nonempty segments in lane order (the ordinal of a segment is the
// number of nonempty segments in lower lanes) and load/value take that
// ordinal.  Rounds r with (r + r_base) % r_stride == r_rank are processed,
// so that a group of r_stride waves can share one column; r_stride = 1
// processes every round.  One 64-bit word per round marks where segments
// start (32 rounds per refill of the words, in the caller's mark array), so
// the owner of element e is (segments starting before the round) + (starts
// in the round at or below e) - 1: a ballot, a population count and a mask
// count.  Rounds are taken kPipe at a time in three phases: owners, then
// every gather (load(o, e, row, raw) issues the loads of element e of
// segment o and must not use their results), then every insert
// (ins(row, value(o, raw))), so that a wavefront keeps kPipe independent
// global loads in flight.
constexpr int kPipe = 8;

template <class RawT, class Load, class Value, class Ins>
__device__ __forceinline__ void flatten_rounds(int len, int excl, int total, int *mark, int64_t r_base,
                                               int64_t r_rank, int64_t r_stride, uint32_t m, int32_t *status,
                                               Load &&load, Value &&value, Ins &&ins) {
  constexpr int kGroup = kWave / 2;  // rounds per refill of the start masks (mark holds 32 words)
  const int l = lane();
  uint64_t *rmask = reinterpret_cast<uint64_t *>(mark);
  const int rs = (int)r_stride;
  int r0 = (int)((r_rank - r_base) % r_stride);
  if (r0 < 0) r0 += rs;
  const int nround = (total + kWave - 1) / kWave;
  for (int g = 0; g < nround; g += kGroup) {
    if (l < kGroup) rmask[l] = 0ull;
    wave_sync();
    const int rr = (excl >> 6) - g;
    if (len > 0 && rr >= 0 && rr < kGroup) atomicOr((unsigned long long *)&rmask[rr], 1ull << (excl & 63));
    wave_sync();
    const int gend = min(nround, g + kGroup);
    int rf = (r0 - g) % rs;
    if (rf < 0) rf += rs;
    for (int r = g + rf; r < gend; r += kPipe * rs) {
      int own_[kPipe], e_[kPipe];
#pragma unroll
      for (int u = 0; u < kPipe; u++) {
        const int ru = r + u * rs;
        own_[u] = -1;
        e_[u] = 0;
        if (ru < gend) {
          const int fb = ru * kWave;
          const uint64_t mm = rmask[ru - g];
          const int carry = __popcll(__ballot(len > 0 && excl < fb));
          const int e = fb + l;
          if (e < total) {
            own_[u] = carry + mbcnt(mm) + (int)((mm >> l) & 1ull) - 1;
            e_[u] = e;
          }
        }
      }
      int32_t row_[kPipe];
      RawT raw_[kPipe];
#pragma unroll
      for (int u = 0; u < kPipe; u++) {
        row_[u] = -1;
        raw_[u] = RawT(0);
        if (own_[u] >= 0) load(own_[u], e_[u], row_[u], raw_[u]);
      }
#pragma unroll
      for (int u = 0; u < kPipe; u++) {
        if (own_[u] >= 0) {
          const int32_t row = opaque(row_[u]);
          if ((uint32_t)row < m)
            ins(row, value(own_[u], opaque(raw_[u])));
          else
            flag_error(status, 3);
        }
      }
    }
    wave_sync();  // every lane has read the masks before they are rewritten
  }
}

// Long segments (at least kLongSeg elements) bypass the owner search: the
// whole wavefront streams them in blocks of kBlk elements, element
// blk*kBlk + t*64 + lane for t < kVec, so every load instruction reads 64
// consecutive entries and each lane keeps kVec loads in flight (values are
// scaled only after every load of the block is issued).  Blocks are
// numbered from unit_base and split among r_stride waves like rounds.
constexpr int kLongSeg = 256;
constexpr int kVec = 8;
constexpr int kBlk = kWave * kVec;

template <bool VALUES, class VT, class Mul = SrPlusTimes, class Ins>
__device__ __forceinline__ void stream_segment(const int32_t *__restrict__ ri, const VT *__restrict__ v,
                                               double scale, int len, int64_t unit_base, int64_t r_rank,
                                               int64_t r_stride, uint32_t m, int32_t *status, Ins &&ins) {
  const int l = lane();
  const int64_t nblk = (len + kBlk - 1) / kBlk;
  int64_t b0 = (r_rank - unit_base) % r_stride;
  if (b0 < 0) b0 += r_stride;
  for (int64_t blk = b0; blk < nblk; blk += r_stride) {
    const int e0 = (int)blk * kBlk + l;
    if ((blk + 1) * kBlk <= len) {  // uniform: a whole block, no lane conditions on the loads
      int32_t row[kVec];
      VT raw[kVec];
#pragma unroll
      for (int t = 0; t < kVec; t++) {
        row[t] = ld_global(ri + e0 + t * kWave);
        raw[t] = VALUES ? ld_global(v + e0 + t * kWave) : VT(0);
      }
#pragma unroll
      for (int t = 0; t < kVec; t++) {
        const int32_t r = opaque(row[t]);
        if ((uint32_t)r < m)
          ins(r, VALUES ? Mul::mul((double)opaque(raw[t]), scale) : 0.0);
        else
          flag_error(status, 3);
      }
      continue;
    }
    int32_t row[kVec];
    VT raw[kVec];
#pragma unroll
    for (int t = 0; t < kVec; t++) {
      const int e = e0 + t * kWave;
      row[t] = 0;
      raw[t] = VT(0);
      if (e < len) {
        row[t] = ld_global(ri + e);
        if (VALUES) raw[t] = ld_global(v + e);
      }
    }
#pragma unroll
    for (int t = 0; t < kVec; t++) {
      if (e0 + t * kWave < len) {
        const int32_t r = opaque(row[t]);
        if ((uint32_t)r < m)
          ins(r, VALUES ? Mul::mul((double)opaque(raw[t]), scale) : 0.0);
        else
          flag_error(status, 3);
      }
    }
  }
}

// Row-slab view of the left operand: entries of each column k in [klo,khi)
// grouped by slab (row >> kSlabShift); slab s of column k occupies
// [Acp[k] + off[(k-klo)*(P+1)+s], Acp[k] + off[(k-klo)*(P+1)+s+1]) of the
// slabbed row/value copies.  sa, sb select the slab range [sa, sb).
struct SlabSel {
  const int32_t *off;
  int P, sa, sb;
};

// Visits every product term A(i,k)*B(k,j) of output column `col` with
// k in [klo, khi): ins(i, A(i,k)*B(k,j)) (values in float64).  Chunks of 64
// entries of B(:,col) are split among waves: chunk c is read by waves with
// (c % c_stride) == c_rank when c_stride > 1 and r_stride == 1; with
// r_stride > 1 every wave reads every chunk and the rounds are split.  With
// SLAB, only the terms whose row lies in the selected slabs are visited
// (a.Ari/a.Av then point at the slabbed copies).
// A column and the first chunk of its B entries loaded ahead of the column's
// turn, in dependent steps placed where the current column has other work:
// lp_cols (B's column pointers), lp_b (the chunk's rows and values of B),
// lp_a (A's column pointers of those rows).  The column pointers are loaded
// per lane (vector loads, so they do not hold up LDS waits) and made uniform
// in lp_b.
template <class VT>
struct LightPre {
  int64_t pbeg, pend;
  int32_t k;
  VT bv;
  int64_t a0, a1;
};

__device__ __forceinline__ int64_t first_lane64(int64_t v) {
  return (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v) |
         ((int64_t)__builtin_amdgcn_readfirstlane((int)((uint64_t)v >> 32)) << 32);
}

template <bool VALUES, class VT>
__device__ __forceinline__ void lp_cols(const ProductArgs<VT> &a, int64_t col, LightPre<VT> &pre) {
  const int64_t z = opaque((int64_t)0);  // a per-lane address: a vector load
  pre.pbeg = ld_global(a.Bcp + col + z);
  pre.pend = ld_global(a.Bcp + col + 1 + z);
}

// The chunk is the one wave w of nw reads first: w when the column has at
// least 2 nw chunks (the waves split the chunks), else chunk 0.
template <bool VALUES, class VT>
__device__ __forceinline__ void lp_b(const ProductArgs<VT> &a, LightPre<VT> &pre, int w, int nw) {
  pre.pbeg = first_lane64(pre.pbeg);
  pre.pend = first_lane64(pre.pend);
  const int64_t nchunks = (pre.pend - pre.pbeg + kWave - 1) / kWave;
  const int64_t p = pre.pbeg + (nchunks >= 2 * nw ? (int64_t)w * kWave : 0) + lane();
  pre.k = -1;
  pre.bv = VT(0);
  if (p < pre.pend) {
    pre.k = a.Bri[p];
    if (VALUES) pre.bv = a.Bv[p];
  }
}

template <bool VALUES, class VT>
__device__ __forceinline__ void lp_a(const ProductArgs<VT> &a, LightPre<VT> &pre) {
  const int32_t k = pre.k;
  pre.a0 = 0;
  pre.a1 = 0;
  if (k >= 0 && (int64_t)k < a.kdim && k >= a.klo && k < a.khi) {
    pre.a0 = a.Acp[k];
    pre.a1 = a.Acp[k + 1];
  }
}

template <bool VALUES, class VT, bool SLAB = false, class Mul = SrPlusTimes, class Ins>
__device__ __forceinline__ void traverse_product(const ProductArgs<VT> &a, int64_t col, int64_t c_rank,
                                                 int64_t c_stride, int64_t r_rank, int64_t r_stride,
                                                 SegScratch &sc, int32_t *status, Ins &&ins,
                                                 SlabSel sl = SlabSel{nullptr, 0, 0, 0},
                                                 const LightPre<VT> *pre = nullptr) {
  // pre (non-SLAB): the column's B range and this wave's first chunk,
  // loaded ahead by lp_cols / lp_b / lp_a
  const int l = lane();
  const int64_t pbeg = pre ? pre->pbeg : a.Bcp[col], pend = pre ? pre->pend : a.Bcp[col + 1];
  int64_t rounds_before = 0;
  for (int64_t base = pbeg + c_rank * kWave; base < pend; base += c_stride * kWave) {
    const int64_t p = base + l;
    const bool first_pre = !SLAB && pre && base == pbeg + c_rank * kWave;  // uniform
    int len = 0;
    int64_t off = 0;
    double b = 0.0;
    if (p < pend) {
      const int32_t k = first_pre ? pre->k : a.Bri[p];
      if ((uint64_t)(uint32_t)k >= (uint64_t)a.kdim || k < 0) {
        flag_error(status, 1);
      } else if (k >= a.klo && k < a.khi) {
        const int64_t a0 = first_pre ? pre->a0 : a.Acp[k];
        int64_t d;
        if (SLAB) {
          const int32_t *o = sl.off + (int64_t)(k - a.klo) * (sl.P + 1);
          const int32_t s0 = o[sl.sa];
          d = o[sl.sb] - s0;
          off = a0 + s0;
        } else {
          d = (first_pre ? pre->a1 : a.Acp[k + 1]) - a0;
          off = a0;
        }
        if (d < 0 || d >= kMaxAdeg) {
          flag_error(status, 2);
          off = 0;
        } else {
          len = (int)d;
          if (VALUES) b = (double)(first_pre ? pre->bv : a.Bv[p]);
        }
      }
    }
    // short segments: load-balanced rounds
    const bool lg = len >= kLongSeg;
    const int ls = lg ? 0 : len;
    const int incl = wave_incl_add(ls);
    const int excl = incl - ls;
    const int total = readlane(incl, 63);
    if (total > 0) {
      const uint64_t nz = __ballot(ls > 0);
      if (ls > 0) {  // the nonempty short segments in lane order
        const int o = mbcnt(nz);
        sc.off[o] = off - excl;
        if (VALUES) sc.scale[o] = b;
      }
      wave_sync();
      int oob = 0;
      flatten_rounds<VT>(
          ls, excl, total, sc.mark, rounds_before, r_rank, r_stride, (uint32_t)a.m, status,
          [&](int o, int e, int32_t &row, VT &raw) {
            int64_t q = sc.off[o] + e;
            oob |= (uint64_t)q >= (uint64_t)a.nnzA ? 1 : 0;
            q = (uint64_t)q >= (uint64_t)a.nnzA ? 0 : q;  // a bounded read; the status word records the fault
            row = a.Ari[q];
            if (VALUES) raw = a.Av[q];
          },
          [&](int o, VT raw) { return VALUES ? Mul::mul((double)raw, sc.scale[o]) : 0.0; }, ins);
      if (__ballot(oob) && l == 0) flag_error(status, 5);
      rounds_before += (total + kWave - 1) / kWave;
      wave_sync();
    }
    // long segments: streamed one at a time by the whole wave
    uint64_t lm = __ballot(lg);
    while (lm) {
      const int L = __builtin_ctzll(lm);
      lm &= lm - 1;
      const int64_t so = readlane64(off, L);
      const int sn = readlane(len, L);
      const double sb = VALUES ? readlane_f64(b, L) : 0.0;
      if (so < 0 || so + sn > a.nnzA) {
        flag_error(status, 5);
        continue;
      }
      stream_segment<VALUES, VT, Mul>(a.Ari + so, VALUES ? a.Av + so : nullptr, sb, sn, rounds_before, r_rank, r_stride,
                                 (uint32_t)a.m, status, ins);
      rounds_before += (sn + kBlk - 1) / kBlk;
    }
  }
}

// A whole workgroup of nw waves on one column: columns with many chunks of
// B(:,col) split the chunks among the waves; columns with few chunks (a
// handful of long segments is typical of heavy columns) split the rounds of
// every chunk instead, so that no wave idles.  (Splitting fewer chunks among
// groups of waves loses more to uneven chunks than it saves in re-reads.)
template <bool VALUES, class VT, bool SLAB = false, class Mul = SrPlusTimes, class Ins>
__device__ __forceinline__ void traverse_product_block(const ProductArgs<VT> &a, int64_t col, int w, int nw,
                                                       SegScratch &sc, int32_t *status, Ins &&ins,
                                                       SlabSel sl = SlabSel{nullptr, 0, 0, 0},
                                                       const LightPre<VT> *pre = nullptr) {
  const int64_t nchunks = ((pre ? pre->pend - pre->pbeg : a.Bcp[col + 1] - a.Bcp[col]) + kWave - 1) / kWave;
  if (nchunks >= 2 * nw)
    traverse_product<VALUES, VT, SLAB, Mul>(a, col, w, nw, 0, 1, sc, status, ins, sl, pre);
  else
    traverse_product<VALUES, VT, SLAB, Mul>(a, col, 0, 1, w, nw, sc, status, ins, sl, pre);
}

// Visits every stored entry of column `col` of the parts: ins(i, value).
// Parts are taken 64 at a time (one per lane); rounds are numbered across
// chunks and split among r_stride waves.
template <class VT, class Ins>
__device__ __forceinline__ void traverse_merge(const PartDesc *P, int nparts, int64_t m, int64_t col,
                                               int64_t r_rank, int64_t r_stride, MergeScratch &sc,
                                               int32_t *status, Ins &&ins) {
  const int l = lane();
  int64_t rounds_before = 0;
  for (int c0 = 0; c0 < nparts; c0 += kWave) {
    const int p = c0 + l;
    int len = 0;
    const int32_t *ri = nullptr;
    const VT *v = nullptr;
    if (p < nparts) {
      const int64_t a0 = ld_global(P[p].cp + col);
      const int64_t d = ld_global(P[p].cp + (col + 1)) - a0;
      if (d < 0 || d >= kMaxAdeg) {
        flag_error(status, 2);
      } else {
        len = (int)d;
        ri = P[p].ri + a0;
        v = (const VT *)P[p].v + a0;
      }
    }
    const bool lg = len >= kLongSeg;
    const int ls = lg ? 0 : len;
    const int incl = wave_incl_add(ls);
    const int excl = incl - ls;
    const int total = readlane(incl, 63);
    if (total > 0) {
      const uint64_t nz = __ballot(ls > 0);
      if (ls > 0) {  // the nonempty short segments in lane order
        const int o = mbcnt(nz);
        sc.ri[o] = ri - excl;
        sc.v[o] = (const void *)(v - excl);
      }
      wave_sync();
      flatten_rounds<VT>(
          ls, excl, total, sc.mark, rounds_before, r_rank, r_stride, (uint32_t)m, status,
          [&](int o, int e, int32_t &row, VT &raw) {
            row = ld_global(sc.ri[o] + e);
            raw = ld_global((const VT *)sc.v[o] + e);
          },
          [&](int, VT raw) { return (double)raw; }, ins);
      rounds_before += (total + kWave - 1) / kWave;
      wave_sync();
    }
    uint64_t lm = __ballot(lg);
    while (lm) {
      const int L = __builtin_ctzll(lm);
      lm &= lm - 1;
      const int32_t *sri = (const int32_t *)readlane64((int64_t)ri, L);
      const VT *sv = (const VT *)readlane64((int64_t)v, L);
      const int sn = readlane(len, L);
      stream_segment<true, VT, MulFirst>(sri, sv, 1.0, sn, rounds_before, r_rank, r_stride, (uint32_t)m, status, ins);
      rounds_before += (sn + kBlk - 1) / kBlk;
    }
  }
}

// ============================================================================
// Small kernels: header init, fills.
// ============================================================================
__global__ void k_init_header(WsHeader *h, uint64_t keep_tag, int keep_status = 0, int keep_left = 0) {
  if (threadIdx.x == 0) {
    if (!keep_status) h->status = 0;
    if (!keep_left) h->left_tag = 0;  // every other operation may overwrite the slabbed copy
    h->left_new = 0;
    for (int b = 0; b < kNumBins; b++) h->bin_count[b] = 0;
    for (int b = 0; b < kNumBins; b++) h->cursor[b] = 0;
    h->esc_count[0] = h->esc_count[1] = 0;
    h->split_cursor = 0;
    h->items = 0;
    h->item_cursor = 0;
    h->nwide = 0;
    h->wide_cursor = 0;
    if (keep_tag != kKeepAnyTag && h->clean_tag != keep_tag) h->clean_tag = 0;
  }
}

__global__ void k_set_tag(WsHeader *h, uint64_t tag) {
  if (threadIdx.x == 0) h->clean_tag = tag;
}

__global__ void k_fill_zero(uint4 *p, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_zero_i64(int64_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

struct PartsChunk {
  PartDesc d[kWave];
};
__global__ void k_store_parts(PartDesc *dst, PartsChunk src, int n) {
  if ((int)threadIdx.x < n) dst[threadIdx.x] = src.d[threadIdx.x];
}

// ============================================================================
// Binning: per output column, its bound on distinct rows and its bin.
//   SYM: bound = min(flops, m); writes flops_out (optional); columns with no
//        product term get nnz 0 here and no bin.
//   NUM: bound = exact count from c_colptr; empty columns get no bin.
// One wavefront per column, 16 columns per wave, one block-level append per
// bin and block.
// ============================================================================
__device__ __forceinline__ int bin_of(int64_t bound, const BinCaps &caps) {
#pragma unroll
  for (int b = 0; b < kNumBins - 1; b++) {
    if (bound <= caps.cap[b]) return b;
  }
  return kNumBins - 1;
}

constexpr int kBinColsPerWave = 16;

template <bool SYM>
__global__ __launch_bounds__(256) void k_bin(const int64_t *Acp, const int64_t *Bcp, const int32_t *Bri,
                                             int64_t c0, int64_t ncol, int64_t klo, int64_t khi, int64_t kdim,
                                             int64_t m, const int64_t *c_colptr, int64_t *flops_out,
                                             int64_t *nnz_out, int32_t *bins, WsHeader *hdr, int min_bin,
                                             BinCaps caps, const int64_t *esc_flops, double esc_cf) {
  // lists kNumBins and kNumBins + 1: the row-sorted product's
  // expand-sort-compress columns (numeric only, when esc_flops is given)
  constexpr int NL = kNumBins + 2;
  __shared__ int s_cnt[NL];
  __shared__ int s_base[NL];
  __shared__ int s_bin[4 * kBinColsPerWave];
  __shared__ int s_pos[4 * kBinColsPerWave];
  const int w = threadIdx.x / kWave, l = lane();
  if (threadIdx.x < NL) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int t = 0; t < kBinColsPerWave; t++) {
    const int slot = w * kBinColsPerWave + t;
    const int64_t jj = ((int64_t)blockIdx.x * 4 + w) * kBinColsPerWave + t;
    int bin = -1;
    if (jj < ncol) {
      int64_t bound;
      if (SYM) {
        const int64_t col = c0 + jj;
        int64_t f = 0;
        for (int64_t p = Bcp[col] + l; p < Bcp[col + 1]; p += kWave) {
          const int32_t k = Bri[p];
          if (k < 0 || (int64_t)k >= kdim) {
            flag_error(&hdr->status, 1);
          } else if (k >= klo && k < khi) {
            f += Acp[k + 1] - Acp[k];
          }
        }
        f = wave_sum_i64(f);
        if (l == 0 && flops_out) flops_out[jj] = f;
        bound = f < m ? f : m;
        if (bound == 0 && l == 0) nnz_out[jj] = 0;
      } else {
        bound = c_colptr[jj + 1] - c_colptr[jj];
      }
      if (bound > 0) bin = max(bin_of(bound, caps), min_bin);
      if (!SYM && esc_flops && bound > 0) {
        const int e = esc_class(esc_flops[jj], bound, esc_cf);
        if (e >= 0) bin = kNumBins + e;
      }
    }
    if (l == 0) {
      s_bin[slot] = bin;
      s_pos[slot] = bin >= 0 ? atomicAdd(&s_cnt[bin], 1) : 0;
    }
  }
  __syncthreads();
  if (threadIdx.x < NL) {
    const int b = threadIdx.x;
    const int c = s_cnt[b];
    s_base[b] = c ? atomicAdd(b < kNumBins ? &hdr->bin_count[b] : &hdr->esc_count[b - kNumBins], c) : 0;
  }
  __syncthreads();
  if (threadIdx.x < 4 * kBinColsPerWave) {
    const int slot = threadIdx.x;
    const int bin = s_bin[slot];
    if (bin >= 0) {
      const int64_t jj = ((int64_t)blockIdx.x * 4 + slot / kBinColsPerWave) * kBinColsPerWave + slot % kBinColsPerWave;
      bins[(int64_t)bin * ncol + s_base[bin] + s_pos[slot]] = (int32_t)jj;
    }
  }
}

// ============================================================================
// Symbolic kernels.
// ============================================================================
// One wavefront per column, TBL-slot table private to the wave.
template <int TBL>
__global__ __launch_bounds__(256) void k_sym_wave(ProductArgs<float> a, int64_t c0, const int32_t *list,
                                                  const int32_t *count_p, int64_t *nnz_out, int32_t *status) {
  __shared__ int32_t s_keys[4][TBL];
  __shared__ SegScratch s_sc[4];
  const int w = threadIdx.x / kWave, l = lane();
  const int count = *count_p;
  int32_t *keys = s_keys[w];
  SegScratch &sc = s_sc[w];
  sc.mark[l] = 0;
  // the next column's B range and first chunk are loaded while one is counted
  const int64_t stride = (int64_t)gridDim.x * 4;  // 64-bit: no overflow near 2^31 columns
  int64_t idx = (int64_t)blockIdx.x * 4 + w;
  const int64_t z = opaque((int64_t)0);  // per-lane addresses: vector loads
  LightPre<float> pre;
  int32_t jn = 0;
  if (idx < count) {
    jn = __builtin_amdgcn_readfirstlane(ld_global(list + idx + z));
    lp_cols<false, float>(a, c0 + jn, pre);
    lp_b<false, float>(a, pre, 0, 1);
    lp_a<false, float>(a, pre);
  }
  int32_t jn2 = idx + stride < count ? ld_global(list + idx + stride + z) : 0;
  for (; idx < count; idx += stride) {
    const int32_t jj = jn;
    const LightPre<float> cur = pre;
    const bool more = idx + stride < count;  // uniform
    if (more) {
      jn = __builtin_amdgcn_readfirstlane(jn2);
      lp_cols<false, float>(a, c0 + jn, pre);
      jn2 = idx + 2 * stride < count ? ld_global(list + idx + 2 * stride + z) : 0;
    }
    for (int s = l; s < TBL; s += kWave) keys[s] = kEmpty;
    wave_sync();
    int cnt = 0;
    traverse_product<false, float>(
        a, c0 + jj, 0, 1, 0, 1, sc, status,
        [&](int32_t row, double) { cnt += ht_insert_key(keys, TBL, row) ? 1 : 0; }, SlabSel{nullptr, 0, 0, 0},
        &cur);
    if (more) lp_b<false, float>(a, pre, 0, 1);
    cnt = wave_sum_i32(cnt);
    if (l == 0) nnz_out[jj] = cnt;
    if (more) lp_a<false, float>(a, pre);
    wave_sync();
  }
}

// One workgroup per column, TBL-slot table shared by its waves.
template <int TBL, int THREADS>
__global__ __launch_bounds__(THREADS) void k_sym_block(ProductArgs<float> a, int64_t c0, const int32_t *list,
                                                       const int32_t *count_p, int64_t *nnz_out, int32_t *status) {
  constexpr int NW = THREADS / kWave;
  __shared__ int32_t s_keys[TBL];
  __shared__ SegScratch s_sc[NW];
  __shared__ int s_cnt;
  const int w = threadIdx.x / kWave, l = lane();
  const int count = *count_p;
  s_sc[w].mark[l] = 0;
  // the next column's B range and each wave's first chunk are loaded while
  // one is counted
  const int64_t z = opaque((int64_t)0);  // per-lane addresses: vector loads
  int64_t item = blockIdx.x;  // 64-bit: no overflow near 2^31 columns
  LightPre<float> pre;
  int32_t jn = 0;
  if (item < count) {
    jn = __builtin_amdgcn_readfirstlane(ld_global(list + item + z));
    lp_cols<false, float>(a, c0 + jn, pre);
    lp_b<false, float>(a, pre, w, NW);
    lp_a<false, float>(a, pre);
  }
  int32_t jn2 = item + (int64_t)gridDim.x < count ? ld_global(list + item + (int64_t)gridDim.x + z) : 0;
  for (; item < count; item += gridDim.x) {
    const int32_t jj = jn;
    const LightPre<float> cur = pre;
    const bool more = item + (int64_t)gridDim.x < count;  // uniform
    if (more) {
      jn = __builtin_amdgcn_readfirstlane(jn2);
      lp_cols<false, float>(a, c0 + jn, pre);
      jn2 = item + 2 * (int64_t)gridDim.x < count ? ld_global(list + item + 2 * (int64_t)gridDim.x + z) : 0;
    }
    for (int s = threadIdx.x; s < TBL; s += THREADS) s_keys[s] = kEmpty;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    int cnt = 0;
    traverse_product_block<false, float>(
        a, c0 + jj, w, NW, s_sc[w], status,
        [&](int32_t row, double) { cnt += ht_insert_key(s_keys, TBL, row) ? 1 : 0; }, SlabSel{nullptr, 0, 0, 0},
        &cur);
    if (more) lp_b<false, float>(a, pre, w, NW);
    cnt = wave_sum_i32(cnt);
    if (l == 0) atomicAdd(&s_cnt, cnt);
    __syncthreads();
    if (threadIdx.x == 0) nnz_out[jj] = s_cnt;
    if (more) lp_a<false, float>(a, pre);
    __syncthreads();
  }
}

// Heavy columns: exact count with an LDS bitmap over windows of kBitmapRows
// rows (one pass over the column's terms per window).
constexpr int kBmWords = (int)(kBitmapRows / 32);
__global__ __launch_bounds__(1024) void k_sym_bitmap(ProductArgs<float> a, int64_t c0, const int32_t *list,
                                                     const int32_t *count_p, int *cursor, int64_t *nnz_out,
                                                     int32_t *status) {
  constexpr int NW = 1024 / kWave;
  __shared__ uint32_t s_bm[kBmWords];
  __shared__ SegScratch s_sc[NW];
  __shared__ unsigned long long s_cnt;
  __shared__ int s_item;
  const int w = threadIdx.x / kWave, l = lane();
  const int count = *count_p;
  s_sc[w].mark[l] = 0;
  for (;;) {  // columns taken from a work queue (heaviest work is uneven)
  if (threadIdx.x == 0) {
    s_cnt = 0;
    s_item = atomicAdd(cursor, 1);
  }
  __syncthreads();
  const int item = s_item;
  if (item >= count) break;
  const int32_t jj = list[item];
  for (int64_t r0 = 0; r0 < a.m; r0 += kBitmapRows) {
    const int words = (int)((min((int64_t)kBitmapRows, a.m - r0) + 31) / 32);
    for (int s = threadIdx.x; s < words; s += 1024) s_bm[s] = 0;
    __syncthreads();
    traverse_product_block<false, float>(a, c0 + jj, w, NW, s_sc[w], status, [&](int32_t row, double) {
      const int64_t r = (int64_t)row - r0;
      if (r >= 0 && r < kBitmapRows) atomicOr(&s_bm[r >> 5], 1u << (r & 31));
    });
    __syncthreads();
    int c = 0;
    for (int s = threadIdx.x; s < words; s += 1024) c += __popc(s_bm[s]);
    c = wave_sum_i32(c);
    if (l == 0) atomicAdd(&s_cnt, (unsigned long long)c);
    __syncthreads();
  }
  if (threadIdx.x == 0) nnz_out[jj] = (int64_t)s_cnt;
  __syncthreads();
  }
}

// ============================================================================
// Numeric and merge kernels (float64 accumulation, output in VT).
// ============================================================================
// Source selector: the product terms of A*B, or the entries of the parts.
template <class VT, class SR = SrPlusTimes>
struct ProductSrc {
  using Sr = SR;
  static constexpr bool kMerge = false;
  ProductArgs<VT> a;
  int64_t c0;
  using Pre = LightPre<VT>;
  __device__ __forceinline__ void pre_cols(int64_t jj, Pre &pre) const { lp_cols<true, VT>(a, c0 + jj, pre); }
  __device__ __forceinline__ void pre_b(Pre &pre, int w, int nw) const { lp_b<true, VT>(a, pre, w, nw); }
  __device__ __forceinline__ void pre_a(Pre &pre) const { lp_a<true, VT>(a, pre); }
  // one wave on the whole column, its first chunk loaded ahead
  template <class Ins>
  __device__ __forceinline__ void visit_pre(int64_t jj, const Pre &pre, void *scratch, int32_t *status,
                                            Ins &&ins) const {
    traverse_product<true, VT, false, SR>(a, c0 + jj, 0, 1, 0, 1, *(SegScratch *)scratch, status, ins,
                                          SlabSel{nullptr, 0, 0, 0}, &pre);
  }
  // the waves of a workgroup on one column (chunks or rounds split)
  template <class Ins>
  __device__ __forceinline__ void visit_pre_block(int64_t jj, const Pre &pre, int w, int nw, void *scratch,
                                                  int32_t *status, Ins &&ins) const {
    traverse_product_block<true, VT, false, SR>(a, c0 + jj, w, nw, *(SegScratch *)scratch, status, ins,
                                                SlabSel{nullptr, 0, 0, 0}, &pre);
  }
  template <class Ins>
  __device__ __forceinline__ void visit(int64_t jj, int64_t c_rank, int64_t c_stride, int64_t r_rank,
                                        int64_t r_stride, void *scratch, int32_t *status, Ins &&ins) const {
    if (c_stride > 1 && r_stride == 1)
      traverse_product_block<true, VT, false, SR>(a, c0 + jj, (int)c_rank, (int)c_stride, *(SegScratch *)scratch,
                                                  status, ins);
    else
      traverse_product<true, VT, false, SR>(a, c0 + jj, c_rank, c_stride, r_rank, r_stride, *(SegScratch *)scratch,
                                            status, ins);
  }
  static constexpr size_t kScratch = sizeof(SegScratch);
};

template <class VT, class SR = SrPlusTimes>
struct MergeSrc {
  using Sr = SR;
  static constexpr bool kMerge = true;
  const PartDesc *P;
  int nparts;
  int64_t m;
  struct Pre {};  // the part descriptors are the input: nothing to load ahead
  __device__ __forceinline__ void pre_cols(int64_t, Pre &) const {}
  __device__ __forceinline__ void pre_b(Pre &, int, int) const {}
  __device__ __forceinline__ void pre_a(Pre &) const {}
  template <class Ins>
  __device__ __forceinline__ void visit_pre(int64_t jj, const Pre &, void *scratch, int32_t *status,
                                            Ins &&ins) const {
    visit(jj, 0, 1, 0, 1, scratch, status, ins);
  }
  template <class Ins>
  __device__ __forceinline__ void visit_pre_block(int64_t jj, const Pre &, int w, int nw, void *scratch,
                                                  int32_t *status, Ins &&ins) const {
    visit(jj, w, nw, 0, 1, scratch, status, ins);
  }
  template <class Ins>
  __device__ __forceinline__ void visit(int64_t jj, int64_t c_rank, int64_t c_stride, int64_t r_rank,
                                        int64_t r_stride, void *scratch, int32_t *status, Ins &&ins) const {
    // one chunk holds every part; the waves of a group split its rounds
    traverse_merge<VT>(P, nparts, m, jj, c_rank + r_rank * c_stride, c_stride * r_stride, *(MergeScratch *)scratch,
                       status, ins);
  }
  static constexpr size_t kScratch = sizeof(MergeScratch);
};

constexpr size_t kScratchBytes = sizeof(SegScratch) > sizeof(MergeScratch) ? sizeof(SegScratch) : sizeof(MergeScratch);

template <class VT>
__device__ __forceinline__ void init_mark(void *scratch) {
  ((int *)scratch)[lane()] = 0;  // both scratch layouts start with mark[64]
}

// Writes the occupied slots [s_lo, s_hi) of a table, in slot order, to
// consecutive output positions from o on (one wave; positions at or beyond
// `end` are not written), and leaves the slots it reads empty (key kEmpty,
// value 0), so a table stays clear between columns without a clearing pass.
// Returns the position after the last entry.
template <class VT, class SR>
__device__ __forceinline__ int64_t compact_run(int32_t *keys, double *vals, int s_lo, int s_hi, int64_t o,
                                               int64_t end, int32_t *out_ri, VT *out_v) {
  const int l = lane();
  for (int s0 = s_lo; s0 < s_hi; s0 += kWave) {
    const int s = s0 + l;
    const int32_t key = s < s_hi ? keys[s] : kEmpty;
    const bool occ = key != kEmpty;
    const uint64_t mask = __ballot(occ);
    const int64_t q = o + mbcnt(mask);
    if (occ) {
      const double x = vals[s];
      keys[s] = kEmpty;
      vals[s] = 0.0;
      if (q < end) {
        out_ri[q] = key;
        out_v[q] = (VT)SR::out(x);
      }
    }
    o += __popcll(mask);
  }
  return o;
}

template <int TBL, class VT, class Src>
__global__ __launch_bounds__(256) void k_num_wave(Src src, const int32_t *list, const int32_t *count_p,
                                                  const int64_t *c_colptr, int32_t *out_ri, VT *out_v,
                                                  int32_t *status) {
  static_assert(TBL % 4 == 0, "tables cleared 16 bytes at a time");
  __shared__ __align__(16) int32_t s_keys[4][TBL];
  __shared__ __align__(16) double s_vals[4][TBL];
  __shared__ __align__(16) char s_sc[4][kScratchBytes];
  const int w = threadIdx.x / kWave, l = lane();
  const int count = *count_p;
  int32_t *keys = s_keys[w];
  double *vals = s_vals[w];
  init_mark<VT>(s_sc[w]);
  // cleared once: every compaction leaves the table empty again
  for (int s = l; s < TBL / 4; s += kWave) reinterpret_cast<int4 *>(keys)[s] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
  for (int s = l; s < TBL / 2; s += kWave) reinterpret_cast<double2 *>(vals)[s] = make_double2(0.0, 0.0);
  // columns idx, idx + stride, ...: while one is processed, the next one's
  // output range, B range and first chunk are loaded (Src::pre_*), and the
  // list entry of the one after
  const int64_t stride = (int64_t)gridDim.x * 4;  // 64-bit: no overflow near 2^31 columns
  int64_t idx = (int64_t)blockIdx.x * 4 + w;
  const int64_t z = opaque((int64_t)0);  // per-lane addresses: vector loads
  typename Src::Pre pre;
  int32_t jn = 0;
  int64_t cb = 0, ce = 0;
  if (idx < count) {
    jn = __builtin_amdgcn_readfirstlane(ld_global(list + idx + z));
    src.pre_cols(jn, pre);
    cb = ld_global(c_colptr + jn + z);
    ce = ld_global(c_colptr + jn + 1 + z);
    src.pre_b(pre, 0, 1);
    src.pre_a(pre);
  }
  int32_t jn2 = idx + stride < count ? ld_global(list + idx + stride + z) : 0;
  for (; idx < count; idx += stride) {
    const int32_t jj = jn;
    const int64_t base = first_lane64(cb), cap = first_lane64(ce) - base;
    const typename Src::Pre cur = pre;
    const bool more = idx + stride < count;  // uniform
    if (more) {
      jn = __builtin_amdgcn_readfirstlane(jn2);
      src.pre_cols(jn, pre);
      cb = ld_global(c_colptr + jn + z);
      ce = ld_global(c_colptr + jn + 1 + z);
      jn2 = idx + 2 * stride < count ? ld_global(list + idx + 2 * stride + z) : 0;
    }
    wave_sync();
    src.visit_pre(jj, cur, s_sc[w], status,
                  [&](int32_t row, double v) { ht_accumulate_sr<typename Src::Sr>(keys, vals, TBL, row, v); });
    if (more) src.pre_b(pre, 0, 1);
    wave_sync();
    // one wave owns the column: output positions follow a running count
    // (a wave's table is small enough to scan; a list of claimed slots would
    // cost a workgroup per CU)
    const int64_t o = compact_run<VT, typename Src::Sr>(keys, vals, 0, TBL, base, base + cap, out_ri, out_v);
    if (more) src.pre_a(pre);
    if (l == 0 && o - base != cap) flag_error(status, 4);
    wave_sync();
  }
}

template <int TBL, int THREADS, class VT, class Src>
__global__ __launch_bounds__(THREADS) void k_num_block(Src src, const int32_t *list, const int32_t *count_p,
                                                       const int64_t *c_colptr, int32_t *out_ri, VT *out_v,
                                                       int32_t *status) {
  constexpr int NW = THREADS / kWave;
  static_assert(TBL % 4 == 0, "tables cleared 16 bytes at a time");
  static_assert(TBL <= 65536, "slot numbers fit 16 bits");
  __shared__ __align__(16) int32_t s_keys[TBL];
  __shared__ __align__(16) double s_vals[TBL];
  __shared__ __align__(16) char s_sc[NW][kScratchBytes];
  __shared__ uint16_t s_list[TBL / 2];  // claimed slots, in claim order
  __shared__ int s_n;
  const int w = threadIdx.x / kWave, l = lane();
  const int count = *count_p;
  init_mark<VT>(s_sc[w]);
  if (threadIdx.x == 0) s_n = 0;
  // cleared once: every compaction leaves the table empty again
  for (int s = threadIdx.x; s < TBL / 4; s += THREADS)
    reinterpret_cast<int4 *>(s_keys)[s] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
  for (int s = threadIdx.x; s < TBL / 2; s += THREADS) reinterpret_cast<double2 *>(s_vals)[s] = make_double2(0.0, 0.0);
  // columns item, item + gridDim.x, ...: the next column's output range, B
  // range and each wave's first chunk are loaded while one is processed
  const int64_t z = opaque((int64_t)0);  // per-lane addresses: vector loads
  int64_t item = blockIdx.x;  // 64-bit: no overflow near 2^31 columns
  typename Src::Pre pre;
  int32_t jn = 0;
  int64_t cb = 0, ce = 0;
  if (item < count) {
    jn = __builtin_amdgcn_readfirstlane(ld_global(list + item + z));
    src.pre_cols(jn, pre);
    cb = ld_global(c_colptr + jn + z);
    ce = ld_global(c_colptr + jn + 1 + z);
    src.pre_b(pre, w, NW);
    src.pre_a(pre);
  }
  int32_t jn2 = item + (int64_t)gridDim.x < count ? ld_global(list + item + (int64_t)gridDim.x + z) : 0;
  for (; item < count; item += gridDim.x) {
    const int32_t jj = jn;
    const int64_t base = first_lane64(cb), cap = first_lane64(ce) - base;
    const typename Src::Pre cur = pre;
    const bool more = item + (int64_t)gridDim.x < count;  // uniform
    if (more) {
      jn = __builtin_amdgcn_readfirstlane(jn2);
      src.pre_cols(jn, pre);
      cb = ld_global(c_colptr + jn + z);
      ce = ld_global(c_colptr + jn + 1 + z);
      jn2 = item + 2 * (int64_t)gridDim.x < count ? ld_global(list + item + 2 * (int64_t)gridDim.x + z) : 0;
    }
    __syncthreads();
    src.visit_pre_block(jj, cur, w, NW, s_sc[w], status, [&](int32_t row, double v) {
      ht_accumulate_list<typename Src::Sr>(s_keys, s_vals, TBL, row, v, s_list, &s_n, TBL / 2);
    });
    if (more) src.pre_b(pre, w, NW);
    __syncthreads();
    // the claimed slots, in claim order, to consecutive output positions;
    // each slot is left empty again
    const int n = s_n;
    const int nl = min(n, TBL / 2);
    for (int i = threadIdx.x; i < nl; i += THREADS) {
      const int sl = s_list[i];
      const int32_t key = s_keys[sl];
      const double x = s_vals[sl];
      s_keys[sl] = kEmpty;
      s_vals[sl] = 0.0;
      if (i < cap) {
        out_ri[base + i] = key;
        out_v[base + i] = (VT)Src::Sr::out(x);
      }
    }
    if (more) src.pre_a(pre);
    if (threadIdx.x == 0 && n != cap) flag_error(status, 4);
    __syncthreads();
    if (threadIdx.x == 0) s_n = 0;  // read by every thread before the barrier above
  }
}

// ----------------------------------------------------------------------------
// Row-sorted product, columns of low compression ratio: expand-sort-compress.
// Every product term of the column is placed in LDS as (row, float64 term),
// the terms are sorted by row with a bitonic network, and each run of equal
// rows is combined in sorted order and written at its rank among the runs:
// the column comes out in ascending row order with no hash table and no
// second pass over the output.  Where nearly every term has a row of its own
// (flops close to nnz) this is the cheaper way to a sorted column, the role
// the heap kernel plays in the CPU hybrid (Sec. V); columns with many
// repeated rows are cheaper to hash and sort afterwards.  Placement is
// deterministic (terms in B-entry order, each A column in storage order),
// and so is the order in which a run is combined.
// ----------------------------------------------------------------------------
// Bitonic sort of (key, val) across the 64 lanes, ascending by key.
__device__ __forceinline__ void wave_bitonic(int32_t &key, double &val) {
  const int l = lane();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int s = k >> 1; s > 0; s >>= 1) {
      const int32_t ok = __shfl_xor(key, s, kWave);
      const double ov = __shfl_xor(val, s, kWave);
      const bool up = (l & k) == 0;   // this block of k lanes sorts ascending
      const bool low = (l & s) == 0;  // the lower lane of the pair keeps the smaller key when ascending
      if (low == up ? ok < key : ok > key) {
        key = ok;
        val = ov;
      }
    }
  }
}

// One wavefront per column of at most kEscWaveTerms terms.
template <class VT, class SR>
__global__ __launch_bounds__(256) void k_esc_wave(ProductArgs<VT> a, int64_t c0, const int32_t *list,
                                                  const int32_t *count_p, const int64_t *c_colptr, int32_t *out_ri,
                                                  VT *out_v, int32_t *status) {
  __shared__ int s_mark[4][kWave];
  __shared__ int32_t s_row[4][kWave];
  __shared__ double s_val[4][kWave];
  const int w = threadIdx.x / kWave, l = lane();
  const int count = *count_p;
  s_mark[w][l] = 0;
  wave_sync();
  for (int64_t idx = (int64_t)blockIdx.x * 4 + w; idx < count; idx += (int64_t)gridDim.x * 4) {
    const int64_t jj = list[idx];
    const int64_t bb = a.Bcp[c0 + jj], be = a.Bcp[c0 + jj + 1];
    const int64_t base = c_colptr[jj], cap = c_colptr[jj + 1] - base;
    int n = 0;  // terms placed (uniform)
    bool bad = false;
    for (int64_t p0 = bb; p0 < be; p0 += kWave) {
      const int64_t p = p0 + l;
      int len = 0;
      int64_t ab = 0;
      double bv = 0.0;
      if (p < be) {
        const int32_t k = a.Bri[p];
        if (k >= a.klo && k < a.khi) {
          ab = a.Acp[k];
          len = (int)min<int64_t>(a.Acp[k + 1] - ab, kEscWaveTerms + 1);
          bv = (double)a.Bv[p];
        }
      }
      const int incl = wave_incl_add(len), excl = incl - len;
      const int tot = readlane(incl, kWave - 1);
      if (n + tot > kEscWaveTerms) {  // more terms than the flops the column was listed with
        bad = true;
        break;
      }
      if (tot == 0) continue;
      // owner of term e of this chunk: the last lane whose segment starts at or below e
      if (len > 0) s_mark[w][excl] = l + 1;
      wave_sync();
      const int mk = s_mark[w][l];
      s_mark[w][l] = 0;
      const int own = max(wave_incl_max(mk) - 1, 0);
      const int64_t oab = __shfl(ab, own, kWave);
      const int oex = __shfl(excl, own, kWave);
      const double obv = __shfl(bv, own, kWave);
      if (l < tot) {
        const int64_t q = oab + (l - oex);
        s_row[w][n + l] = a.Ari[q];
        s_val[w][n + l] = SR::mul((double)a.Av[q], obv);
      }
      n += tot;
      wave_sync();
    }
    if (bad) {
      if (l == 0) flag_error(status, 4);
      continue;
    }
    int32_t key = l < n ? s_row[w][l] : INT32_MAX;  // padding sorts last (rows are below INT32_MAX)
    double val = l < n ? s_val[w][l] : 0.0;
    wave_bitonic(key, val);
    wave_sync();
    s_row[w][l] = key;
    s_val[w][l] = val;
    wave_sync();
    const bool head = l < n && (l == 0 || s_row[w][l - 1] != key);
    double acc = 0.0;  // all-zero slot: no term yet
    if (head) {
      SR::acc_plain(acc, val);
      for (int t = l + 1; t < n && s_row[w][t] == key; t++) SR::acc_plain(acc, s_val[w][t]);
    }
    const uint64_t hm = __ballot(head);
    const int r = mbcnt(hm);
    if (head && r < cap) {
      out_ri[base + r] = key;
      out_v[base + r] = (VT)SR::out(acc);
    }
    if (l == 0 && __popcll(hm) != cap) flag_error(status, 4);
    wave_sync();  // the next column overwrites s_row, s_val
  }
}

// One workgroup per column of up to kEscBlockTerms terms: B(:,j) in chunks
// of 256 entries, each chunk's terms placed by all threads (the owner of a
// term found by binary search over the chunk's exclusive prefix), then a
// bitonic sort in LDS and the runs combined tile by tile.
template <class VT, class SR>
__global__ __launch_bounds__(256) void k_esc_block(ProductArgs<VT> a, int64_t c0, const int32_t *list,
                                                   const int32_t *count_p, const int64_t *c_colptr, int32_t *out_ri,
                                                   VT *out_v, int32_t *status) {
  constexpr int T = 256, NW = T / kWave, N = (int)kEscBlockTerms;
  __shared__ int32_t s_row[N];
  __shared__ double s_val[N];
  __shared__ int s_ex[T];
  __shared__ int64_t s_ab[T];
  __shared__ double s_bv[T];
  __shared__ int s_w[NW];
  const int tid = threadIdx.x;
  const int count = *count_p;
  for (int64_t item = blockIdx.x; item < count; item += gridDim.x) {
    const int64_t jj = list[item];
    const int64_t bb = a.Bcp[c0 + jj], be = a.Bcp[c0 + jj + 1];
    const int64_t base = c_colptr[jj], cap = c_colptr[jj + 1] - base;
    int n = 0;  // terms placed (uniform)
    bool bad = false;
    for (int64_t p0 = bb; p0 < be; p0 += T) {
      const int64_t p = p0 + tid;
      int len = 0;
      int64_t ab = 0;
      double bv = 0.0;
      if (p < be) {
        const int32_t k = a.Bri[p];
        if (k >= a.klo && k < a.khi) {
          ab = a.Acp[k];
          len = (int)min<int64_t>(a.Acp[k + 1] - ab, N + 1);
          bv = (double)a.Bv[p];
        }
      }
      int tot;
      const int ex = block_excl<NW>(len, s_w, tot);
      if (n + tot > N) {  // more terms than the flops the column was listed with
        bad = true;
        break;
      }
      s_ex[tid] = ex;
      s_ab[tid] = ab;
      s_bv[tid] = bv;
      __syncthreads();
      const int np = (int)min<int64_t>(T, be - p0);
      for (int q = tid; q < tot; q += T) {
        int lo = 0, hi = np - 1;  // the last entry whose segment starts at or below q
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_ex[mid] <= q) lo = mid;
          else hi = mid - 1;
        }
        const int64_t qa = s_ab[lo] + (q - s_ex[lo]);
        s_row[n + q] = a.Ari[qa];
        s_val[n + q] = SR::mul((double)a.Av[qa], s_bv[lo]);
      }
      n += tot;
      __syncthreads();  // s_ex, s_ab, s_bv, s_w are reused by the next chunk
    }
    if (bad) {
      if (tid == 0) flag_error(status, 4);
      __syncthreads();
      continue;
    }
    int M = 128;
    while (M < n) M <<= 1;
    for (int t = n + tid; t < M; t += T) {
      s_row[t] = INT32_MAX;  // padding sorts last
      s_val[t] = 0.0;
    }
    __syncthreads();
    for (int k = 2; k <= M; k <<= 1) {
      for (int s = k >> 1; s > 0; s >>= 1) {
        for (int t = tid; t < M / 2; t += T) {
          const int lo = ((t & ~(s - 1)) << 1) | (t & (s - 1));  // lower element of pair t at distance s
          const int hi = lo + s;
          const bool up = (lo & k) == 0;
          const int32_t kl = s_row[lo], kh = s_row[hi];
          if ((kl > kh) == up) {
            const double vl = s_val[lo];
            s_row[lo] = kh;
            s_row[hi] = kl;
            s_val[lo] = s_val[hi];
            s_val[hi] = vl;
          }
        }
        __syncthreads();
      }
    }
    int done = 0;  // runs written so far (uniform)
    for (int t0 = 0; t0 < n; t0 += T) {
      const int t = t0 + tid;
      const int32_t key = t < n ? s_row[t] : INT32_MAX;
      const bool head = t < n && (t == 0 || s_row[t - 1] != key);
      int tot;
      const int r = done + block_excl<NW>(head ? 1 : 0, s_w, tot);
      if (head) {
        double acc = 0.0;  // all-zero slot: no term yet
        for (int u = t; u < n && s_row[u] == key; u++) SR::acc_plain(acc, s_val[u]);
        if (r < cap) {
          out_ri[base + r] = key;
          out_v[base + r] = (VT)SR::out(acc);
        }
      }
      done += tot;
      __syncthreads();  // s_w is reused by the next tile
    }
    if (tid == 0 && done != cap) flag_error(status, 4);
    __syncthreads();  // the next column overwrites s_row, s_val
  }
}

// ----------------------------------------------------------------------------
// Heavy columns, LDS path.  First the left operand's columns k in [klo,khi)
// are bucketed by row slab (a counting sort on row >> kSlabShift inside each
// column; one wavefront per column).
// ----------------------------------------------------------------------------
// The slabbed copy of A (k_slab_split, k_seg_pack) depends only on A's
// columns [klo, khi) and the slab count, so consecutive numeric calls on one
// workspace (the batches of one product) can share it.  k_left_sum forms a
// fingerprint of those columns on the device: every column pointer and
// every entry (row and value bits) is mixed with its position by the
// MurmurHash3 64-bit finalizer and summed, with A's pointers, sizes, the
// layer and the slab count in the seed.  The copy is rebuilt unless the
// workspace holds one made from a source with the same fingerprint; any
// other operation on the workspace clears the tag.
__device__ __host__ __forceinline__ uint64_t fmix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}
__device__ __forceinline__ uint64_t value_bits(float v) { return (uint64_t)__float_as_uint(v); }
__device__ __forceinline__ uint64_t value_bits(double v) { return (uint64_t)__double_as_longlong(v); }

template <class VT>
__global__ __launch_bounds__(256) void k_left_sum(const int64_t *Acp, const int32_t *Ari, const VT *Av, int64_t klo,
                                                  int64_t khi, uint64_t seed, WsHeader *h,
                                                  const int32_t *heavy_count) {
  if (*heavy_count == 0) return;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nth = (int64_t)gridDim.x * blockDim.x;
  uint64_t s = 0;
  for (int64_t k = klo + tid; k <= khi; k += nth) s += fmix64(seed ^ fmix64((uint64_t)k) ^ (uint64_t)Acp[k]);
  const int64_t e0 = Acp[klo], e1 = Acp[khi];
  for (int64_t p = e0 + tid; p < e1; p += nth)
    s += fmix64(seed + fmix64((uint64_t)p) + (((uint64_t)(uint32_t)Ari[p] << 32) ^ value_bits(Av[p])));
  for (int o = 32; o > 0; o >>= 1) s += (uint64_t)__shfl_xor((long long)s, o, kWave);
  if (lane() == 0) atomicAdd((unsigned long long *)&h->left_new, (unsigned long long)s);
}

__device__ __forceinline__ bool left_is_current(const WsHeader *h) { return h->left_tag == (h->left_new | 1ull); }

// After the copy is (re)built or found current: tag it, unless a check
// failed (then the copy is not trusted again).  No heavy columns: nothing
// was touched, the tag stays.
__global__ void k_left_forget(WsHeader *h) {
  if (threadIdx.x == 0) h->left_tag = 0;
}

__global__ void k_left_set(WsHeader *h, const int32_t *heavy_count) {
  if (threadIdx.x == 0 && *heavy_count != 0) h->left_tag = h->status == 0 ? (h->left_new | 1ull) : 0ull;
}

// One entry of the slabbed copy of the left operand: row and value side by
// side, so that one load fetches both.
template <class VT>
struct SlabEnt;
template <>
struct __align__(8) SlabEnt<float> {
  int32_t row;
  float v;
};
template <>
struct __align__(16) SlabEnt<double> {
  int32_t row;
  int32_t pad;
  double v;
};

constexpr int kSplitCols = 16;  // columns of A a wave takes from the work queue at once

template <class VT>
__global__ __launch_bounds__(256) void k_slab_split(const int64_t *Acp, const int32_t *Ari, const VT *Av,
                                                    int64_t klo, int64_t khi, int64_t m, int P, int32_t *soff,
                                                    SlabEnt<VT> *s_ent, const int32_t *heavy_count,
                                                    int32_t *status, WsHeader *hdr) {
  __shared__ int s_hist[4][kMaxSlabs + 1];
  const int w = threadIdx.x / kWave, l = lane();
  // a resident grid whose waves take columns from a work queue (column
  // lengths are uneven): a call whose copy is current, or that has no heavy
  // column, returns from a small grid
  if (*heavy_count == 0 || left_is_current(hdr)) return;
  int *h = s_hist[w];
  for (;;) {
    int q = 0;
    if (l == 0) q = atomicAdd(&hdr->split_cursor, kSplitCols);
    const int64_t kq = klo + readlane(q, 0);
    if (kq >= khi) break;
    const int64_t kend = min(khi, kq + kSplitCols);
    for (int64_t k = kq; k < kend; k++) {
      for (int t = l; t <= P; t += kWave) h[t] = 0;
      wave_sync();
      const int64_t a0 = Acp[k], a1 = Acp[k + 1];
      bool bad = false;
      for (int64_t p = a0 + l; p < a1; p += kWave) {
        const int32_t row = Ari[p];
        bad |= row < 0 || row >= m;
        const uint32_t sl = min((uint32_t)row >> kSlabShift, (uint32_t)(P - 1));
        atomicAdd(&h[sl], 1);
      }
      if (__ballot(bad) && l == 0) flag_error(status, 3);
      wave_sync();
      int32_t *o = soff + (k - klo) * (int64_t)(P + 1);
      int carry = 0;
      for (int t0 = 0; t0 < P; t0 += kWave) {
        const int t = t0 + l;
        const int c = t < P ? h[t] : 0;
        const int incl = wave_incl_add(c);
        if (t < P) {
          o[t] = carry + incl - c;
          h[t] = carry + incl - c;
        }
        carry += readlane(incl, 63);
      }
      if (l == 0) o[P] = carry;
      wave_sync();
      for (int64_t p = a0 + l; p < a1; p += kWave) {
        const int32_t row = Ari[p];
        const uint32_t sl = min((uint32_t)row >> kSlabShift, (uint32_t)(P - 1));
        const int pos = atomicAdd(&h[sl], 1);
        SlabEnt<VT> e;
        e.row = row;
        e.v = Av[p];
        s_ent[a0 + pos] = e;
      }
      wave_sync();  // the next column clears h
    }
  }
}

// Slab-major segment table: pack[s * kc + k] describes the entries of
// A(:,klo+k) in slab s as (absolute start << kSegLenBits) | length, so that
// one 8-byte load gives a segment.  Built from the slab offsets through
// 64 x 64 tiles in LDS (both sides coalesced).
__global__ __launch_bounds__(256) void k_seg_pack(const int32_t *off, const int64_t *Acp, int64_t klo, int64_t kc,
                                                  int P, uint64_t *pack, const int32_t *heavy_count,
                                                  const WsHeader *hdr) {
  __shared__ int32_t tile[64][66];
  __shared__ int64_t s_a0[64];
  if (*heavy_count == 0 || left_is_current(hdr)) return;
  // a persistent grid over the 64 x 64 tiles (k tiles fastest)
  const int64_t nkt = (kc + 63) / 64, ntile = nkt * ((P + 63) / 64);
  for (int64_t ti = blockIdx.x; ti < ntile; ti += gridDim.x) {
    const int64_t k0 = (ti % nkt) * 64;
    const int s0 = (int)(ti / nkt) * 64;
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    for (int r = ty; r < 64; r += 4) {  // rows k, columns s (65 of them: s0 .. s0 + 64)
      const int64_t k = k0 + r;
      if (k < kc) {
        const int sl = s0 + tx;
        if (sl <= P) tile[r][tx] = off[k * (P + 1) + sl];
        if (tx == 0 && s0 + 64 <= P) tile[r][64] = off[k * (P + 1) + s0 + 64];
      }
    }
    if (threadIdx.x < 64 && k0 + threadIdx.x < kc) s_a0[threadIdx.x] = Acp[klo + k0 + threadIdx.x];
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {  // rows s, columns k
      const int sl = s0 + r;
      const int64_t k = k0 + tx;
      if (sl < P && k < kc) {
        const int32_t b0 = tile[tx][r], b1 = tile[tx][r + 1];
        pack[(int64_t)sl * kc + k] = ((uint64_t)(s_a0[tx] + b0) << kSegLenBits) | (uint64_t)(uint32_t)(b1 - b0);
      }
    }
    __syncthreads();  // the next tile rewrites tile and s_a0
  }
}

// Heavy columns: independent slab items (the constants are in internal.hpp).
// The items of a chunk of Hc heavy columns live in a slot table
// slots[hl * P + t] (hl = column within the chunk): nonzero iff an item of
// that column starts at slab t; hv_enc packs its range [t, sb) and the dense
// flag.  Every column has at most one item starting at each slab.
constexpr uint32_t kHvValid = 1u << 31;
__device__ __forceinline__ uint32_t hv_enc(int sa, int sb, bool dense) {
  return kHvValid | (uint32_t)sa | ((uint32_t)sb << 12) | (dense ? (1u << 24) : 0u);
}
static_assert(kMaxSlabs < (1 << 12), "slab ids must fit 12 bits");

__global__ void k_hv_reset(WsHeader *h) {
  if (threadIdx.x == 0) {
    h->items = 0;
    h->item_cursor = 0;
    h->nwide = 0;
    h->wide_cursor = 0;
    h->mb_cursor = 0;
  }
}

// Planning: one workgroup per heavy column of the chunk [h0, h1) of the heavy
// list.  The flop bound of slab s is F_s = sum over k in B(:,col) of the
// entries of A(:,k) in slab s (read from the slab offsets: lanes along slabs,
// a loop over B(:,col)).  Slabs are then cut into items in order: a slab
// with F_s > kHvCap is a dense item, other slabs are joined while their
// bounds add up to at most kHvCap (one hash item).  Wide columns (more than
// kHvWideT entries in B(:,col)) are listed for k_hv_wide instead.  The
// column's P slots are written whole (zero where no item starts).
constexpr int kHvPlanThreads = 256;

__global__ __launch_bounds__(kHvPlanThreads) void k_hv_plan(const int64_t *Bcp, const int32_t *Bri, int64_t c0,
                                                            int64_t klo, int64_t khi, const int32_t *off, int P,
                                                            const int32_t *list, const int32_t *count_p, int64_t h0,
                                                            int64_t h1, uint32_t *slots, int32_t *wlist,
                                                            WsHeader *hdr) {
  constexpr int NW = kHvPlanThreads / kWave;
  __shared__ int s_F[kMaxSlabs];
  __shared__ uint32_t s_slot[kMaxSlabs];
  const int w = threadIdx.x / kWave, l = lane();
  const int64_t count = min((int64_t)*count_p, h1);
  for (int64_t h = h0 + blockIdx.x; h < count; h += gridDim.x) {
    const int64_t col = c0 + list[h];
    const int64_t pb = Bcp[col], pe = Bcp[col + 1];
    const bool wide = pe - pb > kHvWideT;
    for (int t = threadIdx.x; t < P; t += kHvPlanThreads) s_slot[t] = 0u;
    if (!wide) {
      for (int sb = w * kWave; sb < P; sb += NW * kWave) {
        const int s = sb + l;
        int64_t acc = 0;
        for (int64_t q0 = pb; q0 < pe; q0 += kWave) {
          const int32_t kv = q0 + l < pe ? Bri[q0 + l] : -1;
          const int nk = (int)min((int64_t)kWave, pe - q0);
          for (int i = 0; i < nk; i += 4) {
            int32_t lo_[4], hi_[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
              const int32_t k = readlane(kv, min(i + u, kWave - 1));
              const bool ok = i + u < nk && k >= klo && k < khi && s < P;
              const int32_t *o = off + (ok ? (int64_t)(k - klo) * (P + 1) : 0);
              lo_[u] = ok ? o[s] : 0;
              hi_[u] = ok ? o[s + 1] : 0;
            }
#pragma unroll
            for (int u = 0; u < 4; u++) acc += hi_[u] - lo_[u];
          }
        }
        if (s < P) s_F[s] = (int)min(acc, (int64_t)1 << 30);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (wide) {  // formed by k_hv_wide: listed, no slots
        wlist[atomicAdd(&hdr->nwide, 1)] = (int32_t)h;
      } else {
        int t = 0;
        while (t < P) {
          const int f = s_F[t];
          if (f == 0) {
            t++;
          } else if (f > kHvCap) {
            s_slot[t] = hv_enc(t, t + 1, true);
            t++;
          } else {
            int sum = f, t2 = t + 1;
            while (t2 < P && sum + s_F[t2] <= kHvCap) sum += s_F[t2++];
            s_slot[t] = hv_enc(t, t2, false);
            t = t2;
          }
        }
      }
    }
    __syncthreads();
    uint32_t *dst = slots + (h - h0) * (int64_t)P;
    for (int t = threadIdx.x; t < P; t += kHvPlanThreads) dst[t] = s_slot[t];
    __syncthreads();
  }
}

// Operands of the item kernels: the slabbed copy of A and B.  Rows of the
// slabbed copy were checked against m by k_slab_split.
template <class VT>
struct HvArgs {
  const int64_t *Acp;
  const SlabEnt<VT> *ent;  // slabbed entries (fewer than 2^31)
  const int64_t *Bcp;
  const int32_t *Bri;
  const VT *Bv;
  const uint64_t *pack;  // [P][khi-klo] slab segments (start << kSegLenBits | len), slab-major
  int64_t nnzA;
  int32_t klo, khi, kdim, P;
};

// Visits the terms A(i,k) B(k,col) of k in B(:,col) = entries [pbeg, pend)
// of B with i in slabs [sa, sb): ins(i, value).  Segment bounds are checked
// once per segment (the element reads need no check); returns nonzero if an
// index was out of range (that segment is skipped).  The nw waves of the
// workgroup split the chunks of 64 entries of B(:,col) when there are at
// least cs_min*nw of them, else they split the rounds of every chunk.
// Short segments are flattened into rounds of 64 elements: the nonempty
// ones are listed in order (entry base minus exclusive prefix, B value), and
// one 64-bit word per round marks the positions where a segment starts, so
// the owner of element e is (segments starting before the round) + (starts
// in the round at or below e) - 1: a ballot, a population count and a mask
// count, with no scan.  Rounds are taken in blocks of PIPE consecutive ones
// (dealt to the waves in turn when they share a chunk), whose gathers are
// kept in flight together; segments of kLongSeg or more elements are
// streamed by the whole wave.
constexpr int kHvPipe = 4;      // the item kernel
constexpr int kHvWidePipe = 8;  // the wide kernel (one workgroup per CU: deeper blocks pay)
constexpr int kHvVec = 4;
constexpr int kHvBlk = kWave * kHvVec;

// The first chunk of an item's B entries, as one wave reads it, loaded ahead
// of the item in two steps (hv_pre_b: the entries; hv_pre_seg: their segment
// words), so that the dependent loads B entry -> segment word of the next
// item run while the current one finishes.
template <class VT>
struct HvPre {
  int32_t k;
  VT bv;
  uint64_t g0, g1;
};

template <class VT>
__device__ __forceinline__ void hv_pre_b(const HvArgs<VT> &a, int64_t pbeg, int64_t pend, int w, int nw,
                                         int cs_min, HvPre<VT> &pre) {
  const int nchunk = (int)((pend - pbeg + kWave - 1) / kWave);
  const int c = nchunk >= cs_min * nw ? w : 0;
  const int64_t p = pbeg + (int64_t)c * kWave + lane();
  pre.k = -1;
  pre.bv = VT(0);
  if (p < pend) {
    pre.k = a.Bri[p];
    pre.bv = a.Bv[p];
  }
}

template <class VT>
__device__ __forceinline__ void hv_pre_seg(const HvArgs<VT> &a, int sa, int sb, HvPre<VT> &pre) {
  pre.g0 = 0;
  pre.g1 = 0;
  const int32_t k = pre.k;
  if (k >= a.klo && k < a.khi) {
    const int64_t kc = a.khi - a.klo;
    pre.g0 = a.pack[(int64_t)sa * kc + (k - a.klo)];
    if (sb != sa + 1) pre.g1 = a.pack[(int64_t)(sb - 1) * kc + (k - a.klo)];
  }
}

// Per-wave scratch of the traversal: the start mask of 64 consecutive
// rounds and the chunk's nonempty short segments.
template <class VT>
struct SegInfo;
template <>
struct __align__(8) SegInfo<float> {
  uint32_t offm;  // entry index of the segment's first element minus its exclusive prefix (mod 2^32)
  float b;        // B(k,j)
};
template <>
struct __align__(16) SegInfo<double> {
  uint32_t offm;
  uint32_t pad;
  double b;
};
template <class VT>
struct HvScratch {
  uint64_t rmask[kWave];
  SegInfo<VT> info[kWave];
};

// pre: the wave's first chunk loaded ahead (same pbeg, pend, sa, sb, w, nw,
// cs_min), or nullptr.
template <class VT, class Mul = SrPlusTimes, int PIPE = kHvPipe, class Ins>
__device__ __forceinline__ int hv_traverse(const HvArgs<VT> &a, int64_t pbeg, int64_t pend, int sa, int sb, int w,
                                           int nw, int cs_min, HvScratch<VT> &sc, const HvPre<VT> *pre,
                                           Ins &&ins) {
  static_assert(kWave % PIPE == 0, "round blocks do not straddle a start-mask refill");
  const int l = lane();
  const int nchunk = (int)((pend - pbeg + kWave - 1) / kWave);
  const bool csplit = nchunk >= cs_min * nw;
  const int c_rank = csplit ? w : 0, c_stride = csplit ? nw : 1;
  const int r_rank = csplit ? 0 : w, r_stride = csplit ? 1 : nw;
  int bad = 0;
  int units = 0;  // rounds and long-segment blocks before the current chunk
  for (int c = c_rank; c < nchunk; c += c_stride) {
    const int64_t p = pbeg + (int64_t)c * kWave + l;
    int len = 0;
    int64_t off = 0;
    double b = 0.0;
    int32_t k = -1;
    VT bv = VT(0);
    uint64_t g0 = 0, g1 = 0;
    if (pre && c == c_rank) {  // uniform
      k = pre->k;
      bv = pre->bv;
      g0 = pre->g0;
      g1 = pre->g1;
    } else if (p < pend) {
      k = a.Bri[p];
      bv = a.Bv[p];
      if (k >= a.klo && k < a.khi) {
        const int64_t kc = a.khi - a.klo;
        g0 = a.pack[(int64_t)sa * kc + (k - a.klo)];
        if (sb != sa + 1) g1 = a.pack[(int64_t)(sb - 1) * kc + (k - a.klo)];
      }
    }
    if (p < pend) {
      if (k >= a.klo && k < a.khi) {
        constexpr uint64_t kLenMask = (uint64_t(1) << kSegLenBits) - 1;
        // a hash item over several slabs ends where its last slab's segment ends
        const uint64_t ge = sb != sa + 1 ? g1 : g0;
        const int64_t end = (int64_t)(ge >> kSegLenBits) + (int64_t)(ge & kLenMask);
        b = (double)bv;
        off = (int64_t)(g0 >> kSegLenBits);
        const int64_t d = end - off;
        len = (int)min(max(d, (int64_t)-1), (int64_t)kMaxAdeg);
        if (d < 0 || len >= kMaxAdeg || off < 0 || off + len > a.nnzA) {
          bad = 1;
          len = 0;
          off = 0;
        }
      } else if (k < 0 || k >= a.kdim) {
        bad = 1;
      }
    }
    const bool lg = len >= kLongSeg;
    const int ls = lg ? 0 : len;
    const int incl = wave_incl_add(ls);
    const int excl = incl - ls;
    const int total = readlane(incl, 63);
    if (total > 0) {
      const uint64_t nz = __ballot(ls > 0);
      if (ls > 0) {
        SegInfo<VT> si;
        si.offm = (uint32_t)(uint64_t)(off - excl);
        si.b = bv;
        sc.info[mbcnt(nz)] = si;
      }
      const int nround = (total + kWave - 1) / kWave;
      int r0 = (r_rank - units) % r_stride;
      if (r0 < 0) r0 += r_stride;
      for (int g = 0; g < nround; g += kWave) {  // 64 rounds per start-mask refill
        sc.rmask[l] = 0ull;
        wave_sync();
        const int rr = (excl >> 6) - g;
        if (ls > 0 && rr >= 0 && rr < kWave) atomicOr((unsigned long long *)&sc.rmask[rr], 1ull << (excl & 63));
        wave_sync();
        const int gend = min(nround, g + kWave);
        // blocks of PIPE consecutive rounds, dealt to the waves in turn
        int rf = (r0 - g / PIPE) % r_stride;
        if (rf < 0) rf += r_stride;
        for (int r = g + rf * PIPE; r < gend; r += PIPE * r_stride) {
          const int rl = r + PIPE - 1;  // the block's last round
          if (rl < gend && (rl + 1) * kWave <= total) {  // uniform: every lane of every round holds an element
            int own_[PIPE];
#pragma unroll
            for (int u = 0; u < PIPE; u++) {
              const int ru = r + u;
              const uint64_t m = sc.rmask[ru - g];
              const int carry = __popcll(__ballot(ls > 0 && excl < ru * kWave));
              own_[u] = carry + mbcnt(m) + (int)((m >> l) & 1ull) - 1;
            }
            SegInfo<VT> inf_[PIPE];
#pragma unroll
            for (int u = 0; u < PIPE; u++) inf_[u] = sc.info[own_[u]];
            SlabEnt<VT> e_[PIPE];
#pragma unroll
            for (int u = 0; u < PIPE; u++) e_[u] = a.ent[inf_[u].offm + (uint32_t)((r + u) * kWave + l)];
#pragma unroll
            for (int u = 0; u < PIPE; u++)
              ins(opaque(e_[u].row), Mul::mul((double)opaque(e_[u].v), (double)inf_[u].b));
            continue;
          }
          int own_[PIPE];
#pragma unroll
          for (int u = 0; u < PIPE; u++) {
            const int ru = r + u;
            own_[u] = -1;
            if (ru < gend) {
              const int fb = ru * kWave;
              const uint64_t m = sc.rmask[ru - g];
              const int carry = __popcll(__ballot(ls > 0 && excl < fb));
              const int o = carry + mbcnt(m) + (int)((m >> l) & 1ull) - 1;
              if (fb + l < total) own_[u] = o;
            }
          }
          SegInfo<VT> inf_[PIPE];
#pragma unroll
          for (int u = 0; u < PIPE; u++)
            if (own_[u] >= 0) inf_[u] = sc.info[own_[u]];
          // gathers only; the loaded values are used after every load is issued
          SlabEnt<VT> e_[PIPE];
#pragma unroll
          for (int u = 0; u < PIPE; u++) {
            e_[u].row = 0;
            e_[u].v = VT(0);
            if (own_[u] >= 0) e_[u] = a.ent[inf_[u].offm + (uint32_t)((r + u) * kWave + l)];
          }
#pragma unroll
          for (int u = 0; u < PIPE; u++)
            if (own_[u] >= 0) ins(opaque(e_[u].row), Mul::mul((double)opaque(e_[u].v), (double)inf_[u].b));
        }
        wave_sync();
      }
      units += (nround + PIPE - 1) / PIPE;
    }
    uint64_t lm = __ballot(lg);
    while (lm) {
      const int L = __builtin_ctzll(lm);
      lm &= lm - 1;
      const int64_t so = readlane64(off, L);
      const int sn = readlane(len, L);
      const double sbv = readlane_f64(b, L);
      const int nblk = (sn + kHvBlk - 1) / kHvBlk;
      int b0 = (r_rank - units) % r_stride;
      if (b0 < 0) b0 += r_stride;
      for (int blk = b0; blk < nblk; blk += r_stride) {
        const int e0 = blk * kHvBlk + l;
        if ((blk + 1) * kHvBlk <= sn) {  // uniform: a whole block
          SlabEnt<VT> ev[kHvVec];
#pragma unroll
          for (int t = 0; t < kHvVec; t++) ev[t] = a.ent[so + e0 + t * kWave];
#pragma unroll
          for (int t = 0; t < kHvVec; t++) ins(opaque(ev[t].row), Mul::mul((double)opaque(ev[t].v), sbv));
          continue;
        }
        SlabEnt<VT> ev[kHvVec];
#pragma unroll
        for (int t = 0; t < kHvVec; t++) {
          const int e = e0 + t * kWave;
          ev[t].row = 0;
          ev[t].v = VT(0);
          if (e < sn) ev[t] = a.ent[so + e];
        }
#pragma unroll
        for (int t = 0; t < kHvVec; t++)
          if (e0 + t * kWave < sn) ins(opaque(ev[t].row), Mul::mul((double)opaque(ev[t].v), sbv));
      }
      units += nblk;
    }
  }
  return bad;
}

// Items: persistent workgroups take batches from a queue in slab-major
// order: batch i covers slab t = i / nb of the chunk's columns
// [64 (i % nb), 64 (i % nb) + 64), nb = ceil(Hc / 64), so that the
// workgroups of the device work on the same few slabs of A at a time and
// those slabs stay in L2.  The items of a batch (its nonzero slots) are
// formed one after another by the whole workgroup.  A dense item accumulates
// slab t in a float64 array of kSlabRows rows plus an occupancy bitmap; a
// hash item accumulates slabs [t, sb) in a kHvSlots-slot table.  Each wave
// owns a quarter of the rows (or slots), reserves room for its entries on
// the column's cursor and appends them in row (or slot) order.
constexpr int kHvThreads = 256;

// Item source of the numeric pass: the product terms of column c0 + jj.
template <class VT, class SR = SrPlusTimes>
struct HvProductSrc {
  using Sr = SR;
  HvArgs<VT> a;
  int64_t c0;
  int P;
  // the item's input range: the entries of B(:, c0 + jj)
  __device__ __forceinline__ void range(int64_t jj, int64_t, int, int, int64_t &lo, int64_t &hi) const {
    lo = a.Bcp[c0 + jj];
    hi = a.Bcp[c0 + jj + 1];
  }
  using Pre = HvPre<VT>;
  static constexpr int kCsMin = 1;
  __device__ __forceinline__ void pre_b(int64_t lo, int64_t hi, int w, int nw, Pre &pre) const {
    hv_pre_b<VT>(a, lo, hi, w, nw, kCsMin, pre);
  }
  __device__ __forceinline__ void pre_seg(int sa, int sb, Pre &pre) const { hv_pre_seg<VT>(a, sa, sb, pre); }
  using Scratch = HvScratch<VT>;
  template <class Ins>
  __device__ __forceinline__ int visit(int64_t lo, int64_t hi, int sa, int sb, int w, int nw, Scratch &sc,
                                       const Pre &pre, Ins &&ins) const {
    return hv_traverse<VT, SR>(a, lo, hi, sa, sb, w, nw, kCsMin, sc, &pre, ins);
  }
};

// Items are taken from the work queue in batches: the items starting at one
// slab in kItemCols consecutive heavy columns (one wave reads their slots).
constexpr int kItemCols = 64;
static_assert(kItemCols <= kWave, "one slot per lane");

template <class VT, class Src>
__global__ __launch_bounds__(kHvThreads) void k_hv_items(Src src, const int32_t *list,
                                                         const uint32_t *slots, int64_t h0, int64_t hc,
                                                         WsHeader *hdr, const int64_t *c_colptr, int32_t *hv_cur,
                                                         int32_t *out_ri, VT *out_v) {
  constexpr int NW = kHvThreads / kWave;
  constexpr int kWords = (int)(kSlabRows / 32);
  constexpr int kRowsPerWave = (int)kSlabRows / NW;
  constexpr int kWordsPerWave = kRowsPerWave / 32;
  constexpr int kSlotsPerWave = kHvSlots / NW;
  static_assert(kRowsPerWave % kWave == 0 && kWordsPerWave <= kWave, "dense rows split evenly over waves");
  static_assert(kSlotsPerWave % kWave == 0, "hash slots split evenly over waves");
  static_assert(kWords <= kHvThreads, "one bitmap word per thread");
  static_assert(kHvSlots * 12 <= kSlabRows * 8, "hash table fits the dense array");
  // dense items: float64 rows, a spare row, the occupancy bitmap and a spare
  // word (rows outside the slab go to the spares, so the insert needs no
  // branch; the spares are never read out)
  constexpr int kBitsOff = (int)kSlabRows * 8 + 16;
  __shared__ __align__(16) unsigned char s_tab[kBitsOff + kSlabRows / 8 + 16];
  __shared__ typename Src::Scratch s_sc[NW];
  __shared__ int s_batch;
  __shared__ uint32_t s_e[kWave];
  __shared__ int32_t s_jj[kWave];
  __shared__ int64_t s_lo[kWave], s_hi[kWave], s_cb[kWave];  // input range, output column start
  __shared__ int32_t s_cn[kWave];                             // output column length
  __shared__ unsigned long long s_mask;
  const int w = threadIdx.x / kWave, l = lane();
  int32_t *status = &hdr->status;
  const int P = src.P;
  const int64_t nheavy = hdr->bin_count[kNumBins - 1];
  hc = min(hc, max(nheavy - h0, (int64_t)0));  // the device count bounds a chunk sized on the host
  const int64_t nb = (hc + kItemCols - 1) / kItemCols;
  const int64_t nbatch = nb * P;
  double *acc = (double *)s_tab;
  uint32_t *bits = (uint32_t *)(s_tab + kBitsOff);
  int32_t *keys = (int32_t *)s_tab;  // hash items: key = row + 1, 0 = free
  double *vals = (double *)(s_tab + kHvSlots * 4);
  // The table is all zero between items: cleared once here, and every
  // compaction clears what the item wrote (dense rows with their bitmap
  // bits, occupied hash slots), so no item starts with a clearing pass.
  for (int q = threadIdx.x; q < (int)(sizeof(s_tab) / 16); q += kHvThreads)
    reinterpret_cast<uint4 *>(s_tab)[q] = make_uint4(0u, 0u, 0u, 0u);
  for (;;) {
    __syncthreads();  // the previous batch's s_batch, s_e, s_jj, s_mask are no longer read
    if (threadIdx.x == 0) s_batch = atomicAdd(&hdr->item_cursor, 1);
    __syncthreads();
    const int64_t bi = s_batch;
    if (bi >= nbatch) break;
    const int t = (int)(bi / nb);
    const int64_t hb = (bi % nb) * kItemCols;
    if (w == 0) {  // the batch's items: slot, column, input range and output column, one per lane
      const int64_t hl = hb + l;
      uint32_t e = 0u;
      int32_t jj = 0;
      if (l < kItemCols && hl < hc && h0 + hl < nheavy) {
        e = slots[hl * P + t];
        jj = list[h0 + hl];
      }
      int64_t lo = 0, hi = 0, cb = 0, cn = 0;
      const int sb0 = (int)((e >> 12) & 0xfffu);
      if ((e & kHvValid) != 0u && (int)(e & 0xfffu) == t && sb0 > t && sb0 <= P) {
        src.range(jj, hl, t, sb0, lo, hi);
        cb = c_colptr[jj];
        cn = c_colptr[jj + 1] - cb;
      }
      const uint64_t mk = __ballot((e & kHvValid) != 0u);
      s_e[l] = e;
      s_jj[l] = jj;
      s_lo[l] = lo;
      s_hi[l] = hi;
      s_cb[l] = cb;
      s_cn[l] = (int32_t)min(cn, (int64_t)INT32_MAX);
      if (l == 0) s_mask = mk;
    }
    __syncthreads();
    uint64_t mask = s_mask;
    // the first chunk of the next item is loaded ahead: its B entries while
    // the current item finishes its accumulation, their segment words after
    // its output is written
    typename Src::Pre pre;
    const auto pre_load = [&](int jn, bool seg_only) {
      const uint32_t en = s_e[jn];
      const int sbn = (int)((en >> 12) & 0xfffu);
      if ((int)(en & 0xfffu) != t || sbn <= t || sbn > P) return;  // malformed: the item is skipped
      if (!seg_only) src.pre_b(s_lo[jn], s_hi[jn], w, NW, pre);
      else src.pre_seg(t, sbn, pre);
    };
    if (mask) {
      pre_load(__builtin_ctzll(mask), false);
      pre_load(__builtin_ctzll(mask), true);
    }
    while (mask) {
      const int j = __builtin_ctzll(mask);
      mask &= mask - 1;
      const int jn = mask ? __builtin_ctzll(mask) : -1;
      const uint32_t e = s_e[j];
      const int64_t jj = s_jj[j];
      const int sb0 = (int)((e >> 12) & 0xfffu);
      const bool dense = ((e >> 24) & 1u) != 0;
      if ((int)(e & 0xfffu) != t || sb0 <= t || sb0 > P || (dense && sb0 != t + 1)) {
        if (threadIdx.x == 0) flag_error(status, 9);
        if (jn >= 0) {
          pre_load(jn, false);
          pre_load(jn, true);
        }
        continue;
      }
      const int64_t base = s_cb[j], cap = s_cn[j];
      const int64_t lo = s_lo[j], hi = s_hi[j];
      int bad;
      int c = 0;
      uint32_t word = 0u;  // dense: this lane's bitmap word of the wave's rows
      const uint32_t rb = (uint32_t)t << kSlabShift;
      if (dense) {
        int outside = 0;
        bad = src.visit(lo, hi, t, sb0, w, NW, s_sc[w], pre, [&](int32_t row, double v) {
          const uint32_t r0 = (uint32_t)row - rb;
          const bool in = r0 < (uint32_t)kSlabRows;
          const uint32_t r = in ? r0 : (uint32_t)kSlabRows;  // the spare row
          outside |= in ? 0 : 1;
          Src::Sr::acc(&acc[r], v);
          atomicOr(&bits[r >> 5], 1u << (r & 31));
        });
        bad |= outside;
        __syncthreads();
        // wave w owns rows [w * kRowsPerWave, +kRowsPerWave): bitmap words
        // w * kWordsPerWave + lane
        if (l < kWordsPerWave) word = bits[w * kWordsPerWave + l];
        c = __popc(word);
      } else {
        bad = src.visit(lo, hi, t, sb0, w, NW, s_sc[w], pre, [&](int32_t row, double v) {
          ht_accumulate_z<typename Src::Sr>(keys, vals, kHvSlots, row, v);
        });
        __syncthreads();
        // wave w owns slots [w * kSlotsPerWave, +kSlotsPerWave)
#pragma unroll
        for (int g = 0; g < kSlotsPerWave / kWave; g++) c += keys[w * kSlotsPerWave + g * kWave + l] != 0 ? 1 : 0;
      }
      if (jn >= 0) pre_load(jn, false);  // the next item's B entries
      if (__ballot(bad) && l == 0) flag_error(status, 5);
      // each wave reserves room for its own entries on the column's cursor
      // (no workgroup scan or barrier) and writes its rows or slots 64 at a
      // time to consecutive positions, clearing them in the table
      const int cw = readlane(wave_incl_add(c), kWave - 1);
      int pw = 0;
      if (l == 0 && cw) pw = atomicAdd(&hv_cur[jj], cw);
      pw = readlane(pw, 0);
      const bool fits = (int64_t)pw + cw <= cap;
      if (!fits && l == 0) flag_error(status, 4);
      int64_t o = base + pw;
      if (dense) {
#pragma unroll 4
        for (int g = 0; g < kRowsPerWave / kWave; g++) {
          const uint64_t mask = (uint64_t)(uint32_t)readlane((int)word, 2 * g) |
                                ((uint64_t)(uint32_t)readlane((int)word, 2 * g + 1) << 32);
          if (mask == 0ull) continue;
          const int r = w * kRowsPerWave + g * kWave + l;
          if ((mask >> l) & 1ull) {
            const double x = acc[r];
            acc[r] = 0.0;
            if (fits) {
              const int64_t q = o + mbcnt(mask);
              out_ri[q] = (int32_t)(rb + r);
              out_v[q] = (VT)Src::Sr::out(x);
            }
          }
          o += __popcll(mask);
        }
        if (l < kWordsPerWave) bits[w * kWordsPerWave + l] = 0u;
      } else {
#pragma unroll 2
        for (int g = 0; g < kSlotsPerWave / kWave; g++) {
          const int q = w * kSlotsPerWave + g * kWave + l;
          const int32_t key = keys[q];
          const bool occ = key != 0;
          const uint64_t mask = __ballot(occ);
          if (occ) {
            const double x = vals[q];
            keys[q] = 0;
            vals[q] = 0.0;
            if (fits) {
              const int64_t d = o + mbcnt(mask);
              out_ri[d] = key - 1;
              out_v[d] = (VT)Src::Sr::out(x);
            }
          }
          o += __popcll(mask);
        }
      }
      if (jn >= 0) pre_load(jn, true);  // and their segment words
      __syncthreads();
    }
  }
}

// ----------------------------------------------------------------------------
// Heavy merge columns.  The entries of column jj of all parts are bucketed
// by row slab into the workspace (one workgroup per column: slab histogram,
// scan, scatter), which gives the exact entries of every slab; slabs are cut
// into items as in the numeric pass (a slab with more than kHvCap entries is a
// dense item, other slabs are joined while their entries add up to at most
// kHvCap) and every item accumulates one contiguous range of the bucket.  The
// scatter fills each item's range through one cursor (entries of the item's
// slabs interleave there), so a column writes few streams at a time.
// ----------------------------------------------------------------------------
__global__ void k_mb_len(const PartDesc *parts, int nparts, const int32_t *list, const int32_t *count_p,
                         int64_t *len) {
  const int count = *count_p;
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < count; h += gridDim.x * blockDim.x) {
    const int64_t jj = list[h];
    int64_t sum = 0;
    for (int p = 0; p < nparts; p++) sum += ld_global(parts[p].cp + (jj + 1)) - ld_global(parts[p].cp + jj);
    len[h] = sum;
  }
}

constexpr int kMbThreads = 1024;

// Runs of equal slab ids across the lanes of a wavefront (sl < 0: no entry).
// Lane l heads a run if l == 0 or lane l-1 holds another id; run_head_lane
// gives the head of the lane's run, slab_run_head returns whether the lane
// heads a run of a valid id and that run's length.
__device__ __forceinline__ uint64_t run_heads(int sl) {
  const int l = lane();
  const int prev = wave_prev(sl);
  return __ballot(l == 0 || prev != sl);
}

__device__ __forceinline__ int run_head_lane(int sl) {
  const int l = lane();
  const uint64_t upto = l == 63 ? ~0ull : ((2ull << l) - 1);
  return 63 - __clzll((long long)(run_heads(sl) & upto));
}

__device__ __forceinline__ bool slab_run_head(int sl, int &len) {
  const int l = lane();
  const uint64_t heads = run_heads(sl);
  const uint64_t upto = l == 63 ? ~0ull : ((2ull << l) - 1);
  const uint64_t above = heads & ~upto;
  const int next = above ? __builtin_ctzll(above) : kWave;
  len = next - l;
  return ((heads >> l) & 1ull) && sl >= 0;
}

// The entries of column jj over a group of parts as one index space of
// 64-entry chunks: chunk q lies in part p with cpre[p] <= q < cpre[p+1].
constexpr int kMbParts = 256;  // parts whose column ranges sit in LDS at once
constexpr int kMbUnroll = 4;   // chunks whose loads a wave keeps in flight (scatter)
constexpr int kMbUnrollCount = 4;  // the same for the count pass (rows only)

struct MbParts {
  int64_t pb[kMbParts];
  const int32_t *ri[kMbParts];
  const void *v[kMbParts];
  int cpre[kMbParts + 1];
  int64_t plen[kMbParts];
};

// Loads the column ranges of parts [g0, g0 + n) for column jj (n <= kMbParts)
// and the chunk prefix; returns the number of chunks.  Contains barriers.
__device__ __forceinline__ int mb_load_parts(const PartDesc *parts, int g0, int n, int64_t jj, MbParts &mp,
                                             int *s_w) {
  constexpr int NW = kMbThreads / kWave;
  const int t = threadIdx.x;
  int nch = 0;
  if (t < n) {
    const PartDesc d = parts[g0 + t];
    const int64_t a0 = ld_global(d.cp + jj), a1 = ld_global(d.cp + (jj + 1));
    mp.pb[t] = a0;
    mp.ri[t] = d.ri;
    mp.v[t] = d.v;
    mp.plen[t] = max(a1 - a0, (int64_t)0);
    nch = (int)((mp.plen[t] + kWave - 1) / kWave);
  }
  int total;
  const int ex = block_excl<NW>(nch, s_w, total);
  if (t < n) mp.cpre[t] = ex;
  if (t == 0) mp.cpre[n] = total;
  __syncthreads();
  return total;
}

// Part of chunk q: the last p with cpre[p] <= q (binary search over n parts).
__device__ __forceinline__ int mb_part_of(const MbParts &mp, int n, int q) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (mp.cpre[mid] <= q)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <class VT>
__global__ __launch_bounds__(kMbThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_mb_bucket(const PartDesc *parts, int nparts, int64_t m, int P,
                                                          const int32_t *list, const int32_t *count_p, int64_t h0,
                                                          int64_t h1, const int32_t *ord, int64_t t0, int64_t t1,
                                                          int32_t *queue, const int64_t *base, int64_t ecap,
                                                          int32_t *soff, int32_t *brow, VT *bval, uint32_t *slots,
                                                          int32_t *status) {
  constexpr int NW = kMbThreads / kWave;
  constexpr int kPerT = kMaxSlabs / kMbThreads;
  static_assert(kMaxSlabs % kMbThreads == 0, "slabs split evenly over threads");
  static_assert(kMbParts <= kMbThreads, "one part per thread when loading ranges");
  __shared__ int s_cnt[kMaxSlabs];
  __shared__ int s_cur[kMaxSlabs];
  __shared__ uint32_t s_slot[kMaxSlabs];
  __shared__ int s_map[kMaxSlabs];  // slab -> first slab of its item
  __shared__ int s_w[NW];
  __shared__ MbParts s_mp;
  const int w = threadIdx.x / kWave, l = lane();
  __shared__ int s_next;
  const int64_t count = min((int64_t)*count_p, h1);
  const int64_t b0 = base[h0];
  // tasks from a work queue over ord[t0, t1), the chunk's tasks largest
  // first (a long task never starts late and holds the launch open).  A task
  // is (h << 2) | mode: mode 0 takes column h whole; a long column is split
  // into mode 1, its slabs below P / 2 placed from the start of its bucket
  // range, and mode 2, the other slabs placed against the end of the range
  // (the two halves need no count from each other).
  const int mid = P / 2;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(queue, 1);
    __syncthreads();
    const int32_t task = t0 + s_next < t1 ? ord[t0 + s_next] : -1;
    __syncthreads();  // s_next is written again for the next task
    if (task < 0) break;
    const int64_t h = task >> 2;
    const int mode = task & 3;
    if (h < h0 || h >= count) continue;  // uniform
    const int slo = mode == 2 ? mid : 0, shi = mode == 1 ? mid : P;  // this task's slabs
    const int64_t jj = list[h];
    const int64_t bb = base[h] - b0, elen = base[h + 1] - base[h];
    for (int t = threadIdx.x; t < kMaxSlabs; t += kMbThreads) {
      s_cnt[t] = 0;
      s_slot[t] = 0u;
    }
    __syncthreads();
    // ---- count entries per slab
    bool bad = false;
    for (int g0 = 0; g0 < nparts; g0 += kMbParts) {
      const int n = min(kMbParts, nparts - g0);
      const int nch = mb_load_parts(parts, g0, n, jj, s_mp, s_w);
      for (int q0 = w; q0 < nch; q0 += NW * kMbUnrollCount) {
        int32_t row_[kMbUnrollCount];
        bool ok_[kMbUnrollCount];
#pragma unroll
        for (int u = 0; u < kMbUnrollCount; u++) {
          const int q = q0 + u * NW;
          row_[u] = 0;
          ok_[u] = false;
          if (q < nch) {
            const int pp = mb_part_of(s_mp, n, q);
            const int64_t off = (int64_t)(q - s_mp.cpre[pp]) * kWave + l;
            if (off < s_mp.plen[pp]) {
              row_[u] = ld_global(s_mp.ri[pp] + (s_mp.pb[pp] + off));
              ok_[u] = true;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kMbUnrollCount; u++) {
          if (q0 + u * NW >= nch) break;  // uniform
          const int32_t row = opaque(row_[u]);
          int sl = -1;
          if (ok_[u]) {
            if (row >= 0 && (int64_t)row < m) {
              sl = row >> kSlabShift;
              if (sl < slo || sl >= shi) sl = -1;  // the other half's slab
            } else {
              bad = true;
            }
          }
          int len;
          if (slab_run_head(sl, len)) atomicAdd(&s_cnt[sl], len);
        }
      }
      __syncthreads();  // s_mp is reloaded by the next group
    }
    if (__ballot(bad) && l == 0) flag_error(status, 3);
    // exclusive scan over the slabs: thread t owns slabs [t*kPerT, (t+1)*kPerT)
    int loc = 0;
    for (int i = 0; i < kPerT; i++) loc += s_cnt[threadIdx.x * kPerT + i];
    int total;
    int run = block_excl<NW>(loc, s_w, total);
    int32_t *so = soff + (h - h0) * (int64_t)(P + 1);
    // the upper half is placed against the end of the column's range
    const int64_t boff = mode == 2 ? elen - total : 0;
    run += (int)boff;
    for (int i = 0; i < kPerT; i++) {
      const int t = threadIdx.x * kPerT + i;
      const int c = s_cnt[t];
      s_cur[t] = run;
      if (t >= slo && t < shi) so[t] = run;
      run += c;
    }
    if (threadIdx.x == 0 && mode != 1) so[P] = (int32_t)(boff + total);
    const int64_t lim = boff + total;  // positions of this task stay below lim
    const bool fits = bb + elen <= ecap && total <= elen;
    if (threadIdx.x == 0 && !fits) flag_error(status, 9);
    __syncthreads();
    if (w == 0) {  // items in slab order, formed by one wave 64 slabs at a time
      int t = slo;
      while (t < shi) {
        const int u = t + l;
        const int c = u < shi ? s_cnt[u] : 0;
        const uint64_t nz = __ballot(c > 0);
        if (nz == 0) {  // no entries in these slabs
          t += kWave;
          continue;
        }
        const int f = __builtin_ctzll(nz);
        if (f > 0) {  // skip to the next slab with entries
          t += f;
          continue;
        }
        const int ct = readlane(c, 0);
        if (ct > kHvCap) {
          if (l == 0) {
            s_slot[t] = hv_enc(t, t + 1, true);
            s_map[t] = t;
          }
          t++;
          continue;
        }
        // hash item [t, t2): the longest run of slabs whose entries add up to at most kHvCap
        const int e0 = s_cur[t];
        int t2 = t;
        for (;;) {
          const int v = t2 + l;
          const bool ok = v < shi && s_cur[v] + s_cnt[v] - e0 <= kHvCap;
          const uint64_t okm = __ballot(ok);  // a prefix of the lanes: the sums grow with v
          const int n = __popcll(okm);
          if (ok) s_map[v] = t;
          t2 += n;
          if (n < kWave) break;
        }
        if (l == 0) s_slot[t] = hv_enc(t, t2, false);
        t = t2;
      }
    }
    __syncthreads();
    uint32_t *dst = slots + (h - h0) * (int64_t)P;
    for (int t = slo + threadIdx.x; t < shi; t += kMbThreads) dst[t] = fits ? s_slot[t] : 0u;
    // ---- scatter into the items' ranges
    if (fits) {
      for (int g0 = 0; g0 < nparts; g0 += kMbParts) {
        const int n = min(kMbParts, nparts - g0);
        const int nch = mb_load_parts(parts, g0, n, jj, s_mp, s_w);
        for (int q0 = w; q0 < nch; q0 += NW * kMbUnroll) {
          int32_t row_[kMbUnroll];
          VT val_[kMbUnroll];
          bool ok_[kMbUnroll];
#pragma unroll
          for (int u = 0; u < kMbUnroll; u++) {
            const int q = q0 + u * NW;
            row_[u] = 0;
            val_[u] = VT(0);
            ok_[u] = false;
            if (q < nch) {
              const int pp = mb_part_of(s_mp, n, q);
              const int64_t off = (int64_t)(q - s_mp.cpre[pp]) * kWave + l;
              if (off < s_mp.plen[pp]) {
                row_[u] = ld_global(s_mp.ri[pp] + (s_mp.pb[pp] + off));
                val_[u] = ld_global((const VT *)s_mp.v[pp] + (s_mp.pb[pp] + off));
                ok_[u] = true;
              }
            }
          }
#pragma unroll
          for (int u = 0; u < kMbUnroll; u++) {
            if (q0 + u * NW >= nch) break;  // uniform
            const int32_t row = opaque(row_[u]);
            int sl = -1;
            if (ok_[u] && row >= 0 && (int64_t)row < m) {
              const int rs = row >> kSlabShift;
              if (rs >= slo && rs < shi) sl = s_map[rs];  // the item's range
            }
            int len;
            int pos = 0;
            if (slab_run_head(sl, len)) pos = atomicAdd(&s_cur[sl], len);
            // every lane of a run takes the head's position plus its distance to the head
            const int head = run_head_lane(sl);
            pos = __shfl(pos, head, kWave) + (l - head);
            if (sl >= 0 && pos >= 0 && pos < lim) {  // positions stay inside the task's counted range
              brow[bb + pos] = row;
              bval[bb + pos] = opaque(val_[u]);
            }
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// Item source of the merge: the bucket range of the item's slabs.
template <class VT, class SR = SrPlusTimes>
struct MbSrc {
  using Sr = SR;
  const int32_t *brow;
  const VT *bval;
  const int32_t *soff;
  const int64_t *base;
  int64_t h0;
  int P;
  // the item's input range: its slabs' part of the column's bucket
  __device__ __forceinline__ void range(int64_t, int64_t hl, int sa, int sb, int64_t &lo, int64_t &hi) const {
    const int32_t *so = soff + hl * (int64_t)(P + 1);
    const int64_t bb = base[h0 + hl] - base[h0];
    lo = bb + so[sa];
    hi = bb + so[sb];
  }
  struct Pre {};  // nothing to load ahead: the range is the item's input
  __device__ __forceinline__ void pre_b(int64_t, int64_t, int, int, Pre &) const {}
  __device__ __forceinline__ void pre_seg(int, int, Pre &) const {}
  using Scratch = HvScratch<VT>;  // unused: the entries of an item are contiguous
  template <class Ins>
  __device__ __forceinline__ int visit(int64_t e0, int64_t e1, int, int, int w, int nw, Scratch &, const Pre &,
                                       Ins &&ins) const {
    constexpr int kV = 4;
    const int l = lane();
    for (int64_t q0 = e0 + (int64_t)w * kWave * kV + l; q0 < e1; q0 += (int64_t)nw * kWave * kV) {
      int32_t row[kV];
      VT raw[kV];
#pragma unroll
      for (int t = 0; t < kV; t++) {
        const int64_t q = q0 + t * kWave;
        row[t] = 0;
        raw[t] = VT(0);
        if (q < e1) {
          row[t] = brow[q];
          raw[t] = bval[q];
        }
      }
#pragma unroll
      for (int t = 0; t < kV; t++)
        if (q0 + t * kWave < e1) ins(opaque(row[t]), (double)opaque(raw[t]));
    }
    return 0;
  }
};

// Wide heavy columns (more than kHvWideT entries in B(:,j)): items of
// kHvWideSlabs consecutive slabs on one dense float64 array of kHvWideRows
// rows (one workgroup of 16 waves per CU), so that the entries of B(:,j) are
// visited once per kHvWideSlabs slabs.  Items are taken in slab-major order:
// item i is slab group i / nw of the (i % nw)-th listed wide column.
constexpr int kHvWideSlabs = 4;
constexpr int64_t kHvWideRows = kSlabRows * kHvWideSlabs;
constexpr int kHvWideThreads = 1024;

template <class VT, class SR>
__global__ __launch_bounds__(kHvWideThreads) void k_hv_wide(HvArgs<VT> a, int64_t c0, const int32_t *list,
                                                            const int32_t *wlist, int64_t wcap, WsHeader *hdr,
                                                            const int64_t *c_colptr, int32_t *hv_cur,
                                                            int32_t *out_ri, VT *out_v) {
  constexpr int NW = kHvWideThreads / kWave;
  constexpr int kWords = (int)(kHvWideRows / 32);
  constexpr int kRowsPerWave = (int)kHvWideRows / NW;
  constexpr int kWordsPerWave = kRowsPerWave / 32;
  static_assert(kWords <= kHvWideThreads, "one bitmap word per thread");
  static_assert(kRowsPerWave % kWave == 0 && kWordsPerWave <= kWave, "rows split evenly over waves");
  __shared__ double s_acc[kHvWideRows];
  __shared__ uint32_t s_bits[kWords];
  __shared__ HvScratch<VT> s_sc[NW];
  __shared__ int s_item;
  const int w = threadIdx.x / kWave, l = lane();
  int32_t *status = &hdr->status;
  const int P = a.P;
  const int64_t nheavy = hdr->bin_count[kNumBins - 1];
  const int64_t nwide = min((int64_t)hdr->nwide, wcap);
  const int64_t nq = (P + kHvWideSlabs - 1) / kHvWideSlabs;
  const int64_t nitems = nwide * nq;
  for (;;) {
    __syncthreads();  // s_item of the previous item is no longer read
    if (threadIdx.x == 0) s_item = atomicAdd(&hdr->wide_cursor, 1);
    __syncthreads();
    const int64_t it = s_item;
    if (it >= nitems) break;
    const int q = (int)(it / nwide);
    const int64_t h = wlist[it % nwide];
    if (h < 0 || h >= nheavy) {
      if (threadIdx.x == 0) flag_error(status, 9);
      continue;
    }
    const int64_t jj = list[h];
    const int64_t col = c0 + jj;
    const int64_t base = c_colptr[jj], cap = c_colptr[jj + 1] - base;
    const int sa = q * kHvWideSlabs, sb = min(sa + kHvWideSlabs, P);
    const uint32_t rb = (uint32_t)sa << kSlabShift;
    for (int r = threadIdx.x; r < (int)kHvWideRows; r += kHvWideThreads) s_acc[r] = 0.0;
    if (threadIdx.x < kWords) s_bits[threadIdx.x] = 0u;
    __syncthreads();
    int outside = 0;
    int bad = hv_traverse<VT, SR, kHvWidePipe>(a, a.Bcp[col], a.Bcp[col + 1], sa, sb, w, NW, 1, s_sc[w], (const HvPre<VT> *)nullptr, [&](int32_t row, double v) {
      const uint32_t r = (uint32_t)row - rb;
      if (r < (uint32_t)kHvWideRows) {
        SR::acc(&s_acc[r], v);
        atomicOr(&s_bits[r >> 5], 1u << (r & 31));
      } else {
        outside = 1;
      }
    });
    bad |= outside;
    __syncthreads();
    if (__ballot(bad) && l == 0) flag_error(status, 5);
    // wave w owns rows [w * kRowsPerWave, +kRowsPerWave) and writes them 64
    // at a time to consecutive positions
    // (each wave reserves room for its own rows on the column's cursor)
    const int cw = readlane(wave_incl_add(l < kWordsPerWave ? __popc(s_bits[w * kWordsPerWave + l]) : 0), kWave - 1);
    int pw = 0;
    if (l == 0 && cw) pw = atomicAdd(&hv_cur[jj], cw);
    pw = readlane(pw, 0);
    if ((int64_t)pw + cw > cap) {
      if (l == 0) flag_error(status, 4);
    } else {
      int64_t o = base + pw;
#pragma unroll 4
      for (int g = 0; g < kRowsPerWave / kWave; g++) {
        const int r = w * kRowsPerWave + g * kWave + l;
        const bool occ = (s_bits[r >> 5] >> (r & 31)) & 1u;
        const uint64_t mask = __ballot(occ);
        if (occ) {
          const int64_t d = o + mbcnt(mask);
          out_ri[d] = (int32_t)(rb + r);
          out_v[d] = (VT)SR::out(s_acc[r]);
        }
        o += __popcll(mask);
      }
    }
  }
}

// Every heavy column received exactly its symbolic count.
__global__ void k_hv_check(const int32_t *list, const int32_t *count_p, const int64_t *c_colptr,
                           const int32_t *hv_cur, int32_t *status) {
  const int count = *count_p;
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < count; h += gridDim.x * blockDim.x) {
    const int64_t jj = list[h];
    if ((int64_t)hv_cur[jj] != c_colptr[jj + 1] - c_colptr[jj]) flag_error(status, 4);
  }
}

// Heavy columns: dense float64 accumulators in the workspace, one per slot;
// blocks (slot, part) share a column.  vals/flags are zero on entry and are
// reset by k_heavy_write.
template <class Src>
__global__ __launch_bounds__(256) void k_heavy_acc(Src src, const int32_t *list, int first, int nslots, int parts,
                                                   int64_t m, double *vals, uint8_t *flags, int32_t *status) {
  constexpr int NW = 4;
  __shared__ __align__(16) char s_sc[NW][kScratchBytes];
  const int w = threadIdx.x / kWave;
  const int slot = blockIdx.x / parts, part = blockIdx.x % parts;
  if (slot >= nslots) return;
  init_mark<float>(s_sc[w]);
  wave_sync();
  const int32_t jj = list[first + slot];
  double *dv = vals + (int64_t)slot * m;
  uint8_t *df = flags + (int64_t)slot * m;
  // chunks of B(:,j) are shared by all waves of the group; rounds are split
  src.visit(jj, 0, 1, (int64_t)part * NW + w, (int64_t)parts * NW, s_sc[w], status, [&](int32_t row, double v) {
    Src::Sr::acc(&dv[row], v);
    df[row] = 1;
  });
}

// Occupied rows per segment of kHeavySeg rows.
__global__ __launch_bounds__(256) void k_heavy_count(int nslots, int64_t m, int64_t nseg, const uint8_t *flags,
                                                     int64_t *segcnt) {
  __shared__ int s_cnt;
  const int64_t slot = blockIdx.x / nseg, seg = blockIdx.x % nseg;
  if (slot >= nslots) return;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const uint8_t *f = flags + slot * m;
  const int64_t r0 = seg * kHeavySeg, r1 = min(m, r0 + kHeavySeg);
  int c = 0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) c += f[r];
  c = wave_sum_i32(c);
  if (lane() == 0) atomicAdd(&s_cnt, c);
  __syncthreads();
  if (threadIdx.x == 0) segcnt[slot * nseg + seg] = s_cnt;
}

// Ordered compaction of one segment of a heavy column; resets its slots.
template <class VT, class SR>
__global__ __launch_bounds__(256) void k_heavy_write(const int32_t *list, int first, int nslots, int64_t m,
                                                     int64_t nseg, double *vals, uint8_t *flags,
                                                     const int64_t *segcnt, const int64_t *c_colptr,
                                                     int32_t *out_ri, VT *out_v, int32_t *status) {
  constexpr int PER = 16;  // rows per thread per tile
  constexpr int TILE = 256 * PER;
  __shared__ int64_t s_base;
  __shared__ int s_wsum[4];
  const int64_t slot = blockIdx.x / nseg, seg = blockIdx.x % nseg;
  if (slot >= nslots) return;
  const int w = threadIdx.x / kWave, l = lane();
  const int32_t jj = list[first + slot];
  const int64_t cbase = c_colptr[jj], cap = c_colptr[jj + 1] - cbase;
  if (threadIdx.x == 0) {
    int64_t pre = 0;
    for (int64_t s = 0; s < seg; s++) pre += segcnt[slot * nseg + s];
    s_base = pre;
    if (seg == nseg - 1 && pre + segcnt[slot * nseg + seg] != cap) flag_error(status, 4);
  }
  __syncthreads();
  int64_t pos = s_base;
  double *dv = vals + slot * m;
  uint8_t *df = flags + slot * m;
  const int64_t r0 = seg * kHeavySeg, r1 = min(m, r0 + kHeavySeg);
  for (int64_t t0 = r0; t0 < r1; t0 += TILE) {
    const int64_t my0 = t0 + (int64_t)threadIdx.x * PER;
    uint8_t f[PER];
    int c = 0;
#pragma unroll
    for (int i = 0; i < PER; i++) {
      f[i] = (my0 + i < r1) ? df[my0 + i] : 0;
      c += f[i];
    }
    // exclusive scan of c over the block
    const int incl = wave_incl_add(c);
    if (l == 63) s_wsum[w] = incl;
    __syncthreads();
    int wbase = 0, tot = 0;
    for (int q = 0; q < 4; q++) {
      if (q < w) wbase += s_wsum[q];
      tot += s_wsum[q];
    }
    int64_t o = pos + wbase + incl - c;
#pragma unroll
    for (int i = 0; i < PER; i++) {
      if (f[i]) {
        const int64_t r = my0 + i;
        if (o < cap) {
          out_ri[cbase + o] = (int32_t)r;
          out_v[cbase + o] = (VT)SR::out(dv[r]);
        }
        o++;
        dv[r] = 0.0;
        df[r] = 0;
      }
    }
    pos += tot;
    __syncthreads();
  }
}

// ============================================================================
// Exclusive scan of int64 counts into column pointers.
// ============================================================================
constexpr int kScanPer = 32, kScanThreads = 256, kScanBlock = kScanPer * kScanThreads;

__device__ __forceinline__ int64_t wave_incl_add_i64(int64_t v) {
  const int l = lane();
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t t = __shfl_up(v, o, kWave);
    if (l >= o) v += t;
  }
  return v;
}

// Exclusive block scan (256 threads); returns this thread's exclusive prefix
// and writes the block total to *total.
__device__ __forceinline__ int64_t block_excl_i64(int64_t v, int64_t *s_w, int64_t *total) {
  const int w = threadIdx.x / kWave, l = lane();
  const int64_t incl = wave_incl_add_i64(v);
  if (l == kWave - 1) s_w[w] = incl;
  __syncthreads();
  int64_t wb = 0, tot = 0;
  for (int q = 0; q < kScanThreads / kWave; q++) {
    if (q < w) wb += s_w[q];
    tot += s_w[q];
  }
  __syncthreads();
  *total = tot;
  return wb + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int64_t *x, int64_t n, int64_t *bsum) {
  __shared__ int64_t s_w[kScanThreads / kWave];
  const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
  int64_t s = 0;
  for (int i = 0; i < kScanPer; i++) {
    const int64_t idx = b0 + (int64_t)i * kScanThreads + threadIdx.x;
    if (idx < n) s += x[idx];
  }
  int64_t tot;
  block_excl_i64(s, s_w, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_bsums(int64_t *bsum, int64_t nb) {
  __shared__ int64_t s_w[kScanThreads / kWave];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nb ? bsum[i] : 0;
    int64_t tot;
    const int64_t ex = block_excl_i64(v, s_w, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_final(const int64_t *x, int64_t n, const int64_t *bsum,
                                                             int64_t *out) {
  __shared__ int64_t s_w[kScanThreads / kWave];
  const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
  const int64_t t0 = b0 + (int64_t)threadIdx.x * kScanPer;  // contiguous items per thread
  int64_t v[kScanPer];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; i++) {
    v[i] = (t0 + i < n) ? x[t0 + i] : 0;
    s += v[i];
  }
  int64_t tot;
  int64_t run = bsum[blockIdx.x] + block_excl_i64(s, s_w, &tot);
  if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; i++) {
    run += v[i];
    if (t0 + i < n) out[t0 + i + 1] = run;
  }
}

// ============================================================================
// Host side.
// ============================================================================
int hip_fail(hipError_t e) {
  set_hip_error((int)e);
  return SPGEMM_E_HIP;
}

struct HostPinned {
  WsHeader *hdr = nullptr;
};
static thread_local HostPinned g_pin;

// Testing hook: every column goes to at least this bin (0 = natural bins).
static int g_min_bin = 0;
// Bin thresholds in use (symbolic, numeric); tunable within the table sizes.
static BinCaps g_caps[2] = {BinCaps{{kSymCap[0], kSymCap[1], kSymCap[2], kSymCap[3], kSymCap[4]}},
                            BinCaps{{kNumCap[0], kNumCap[1], kNumCap[2], kNumCap[3], kNumCap[4]}}};
// Workgroups per compute unit of the persistent bin kernels' grids
// (symbolic, numeric and merge); tunable, never changing results.
constexpr int kBpcDefault[2][kNumBins - 1] = {{8, 8, 8, 8, 1}, {8, 8, 4, 4, 1}};
static int g_bpc[2][kNumBins - 1] = {{8, 8, 8, 8, 1}, {8, 8, 4, 4, 1}};

int read_header(WsHeader *dev, hipStream_t st, WsHeader *out) {
  if (!g_pin.hdr) HIPCHK(hipHostMalloc((void **)&g_pin.hdr, sizeof(WsHeader), hipHostMallocDefault));
  HIPCHK(hipMemcpyAsync(g_pin.hdr, dev, sizeof(WsHeader), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *out = *g_pin.hdr;
  return SPGEMM_OK;
}

int device_cus() {
  static int cus = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    if (cus <= 0) cus = 256;
  });
  return cus;
}

int g_min_bin_value() { return g_min_bin; }
BinCaps bin_caps(int which) { return g_caps[which ? 1 : 0]; }

int launch_set_tag(WsHeader *h, uint64_t tag, hipStream_t st) {
  hipLaunchKernelGGL(k_set_tag, dim3(1), dim3(64), 0, st, h, tag);
  LAUNCHCHK();
  return SPGEMM_OK;
}

int launch_reset_counters(WsHeader *h, hipStream_t st) {
  hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, st, h, kKeepAnyTag, 1, 1);
  LAUNCHCHK();
  return SPGEMM_OK;
}

int launch_init_header(WsHeader *h, uint64_t keep_tag, hipStream_t st) {
  hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, st, h, keep_tag, 0);
  LAUNCHCHK();
  return SPGEMM_OK;
}

int launch_colptr_scan(const int64_t *counts, int64_t n, int64_t *out, int64_t *bsum, hipStream_t s) {
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, s, out, (int64_t)1);
    LAUNCHCHK();
    return SPGEMM_OK;
  }
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  ProfScope prof("scan", s);
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, n, bsum);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kScanThreads), 0, s, bsum, nb);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, n, bsum, out);
  LAUNCHCHK();
  return SPGEMM_OK;
}


// One inner-dimension layer of the right operand: the entries of
// B(:, c0 + jj), jj < ncol, whose row k lies in [klo, khi), in their order, as
// a CSC matrix over the call's columns (column jj).  The passes of a layer
// then read only its share of B instead of skipping the other layers'
// entries column by column.  Rows outside [0, kdim) set status 1.
__global__ __launch_bounds__(256) void k_layer_count(const int64_t *Bcp, const int32_t *Bri, int64_t c0,
                                                     int64_t ncol, int64_t klo, int64_t khi, int64_t kdim,
                                                     int64_t *cnt, int32_t *status) {
  const int w = threadIdx.x / kWave, l = lane();
  for (int64_t jj = (int64_t)blockIdx.x * 4 + w; jj < ncol; jj += (int64_t)gridDim.x * 4) {
    const int64_t p0 = Bcp[c0 + jj], p1 = Bcp[c0 + jj + 1];
    int64_t c = 0;
    bool bad = false;
    for (int64_t b = p0; b < p1; b += kWave) {
      const int64_t p = b + l;
      bool in = false;
      if (p < p1) {
        const int32_t k = Bri[p];
        in = k >= klo && k < khi;
        bad |= k < 0 || k >= kdim;
      }
      c += __popcll(__ballot(in));
    }
    if (__ballot(bad) && l == 0) flag_error(status, 1);
    if (l == 0) cnt[jj] = c;
  }
}

template <class VT>
__global__ __launch_bounds__(256) void k_layer_fill(const int64_t *Bcp, const int32_t *Bri, const VT *Bv,
                                                    int64_t c0, int64_t ncol, int64_t klo, int64_t khi,
                                                    const int64_t *cp, int64_t cap, int32_t *ri_out, VT *v_out,
                                                    int32_t *status) {
  const int w = threadIdx.x / kWave, l = lane();
  for (int64_t jj = (int64_t)blockIdx.x * 4 + w; jj < ncol; jj += (int64_t)gridDim.x * 4) {
    const int64_t p0 = Bcp[c0 + jj], p1 = Bcp[c0 + jj + 1];
    int64_t o = cp[jj];
    const int64_t e = cp[jj + 1];
    if (o < 0 || e < o || e > cap) {  // more entries than B declares
      if (l == 0) flag_error(status, 8);
      continue;
    }
    for (int64_t b = p0; b < p1; b += kWave) {
      const int64_t p = b + l;
      int32_t k = -1;
      if (p < p1) k = Bri[p];
      const bool in = k >= klo && k < khi;
      const uint64_t mask = __ballot(in);
      const int64_t pos = o + mbcnt(mask);
      if (in && pos < e) {
        ri_out[pos] = k;
        if (v_out) v_out[pos] = Bv[p];
      }
      o += __popcll(mask);
    }
  }
}

// Builds the layer's share of B (columns [c0, c0 + ncol), rows [klo, khi)) in
// the workspace and describes it in *Bl (column jj of Bl is column c0 + jj
// of B; nnz is the capacity, an upper bound).
template <class VT>
static int build_layer(const spgemm_csc *B, int64_t c0, int64_t ncol, int64_t klo, int64_t khi, int64_t kdim,
                       bool values, const WsLayout &L, char *ws, hipStream_t st, spgemm_csc *Bl) {
  WsHeader *hdr = (WsHeader *)ws;
  int64_t *cnt = (int64_t *)(ws + L.bl_cnt);
  int64_t *cp = (int64_t *)(ws + L.bl_cp);
  {
    ProfScope prof("layer_split", st);
    hipLaunchKernelGGL(k_layer_count, dim3(grid_of(ncol, 4)), dim3(256), 0, st, B->colptr, B->rowidx, c0, ncol, klo,
                       khi, kdim, cnt, &hdr->status);
    LAUNCHCHK();
    int rc = launch_colptr_scan(cnt, ncol, cp, (int64_t *)(ws + L.bl_scan), st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_layer_fill<VT>, dim3(grid_of(ncol, 4)), dim3(256), 0, st, B->colptr, B->rowidx,
                       values ? (const VT *)B->values : (const VT *)nullptr, c0, ncol, klo, khi, (const int64_t *)cp,
                       L.bl_cap, (int32_t *)(ws + L.bl_ri), values ? (VT *)(ws + L.bl_v) : (VT *)nullptr,
                       &hdr->status);
    LAUNCHCHK();
  }
  *Bl = *B;
  Bl->ncols = ncol;
  Bl->nnz = L.bl_cap;
  Bl->colptr = cp;
  Bl->rowidx = (const int32_t *)(ws + L.bl_ri);
  Bl->values = values ? (const void *)(ws + L.bl_v) : nullptr;
  return SPGEMM_OK;
}

template <class VT>
static ProductArgs<VT> product_args(const spgemm_csc *A, const spgemm_csc *B, int64_t klo, int64_t khi) {
  ProductArgs<VT> a;
  a.Acp = A->colptr;
  a.Ari = A->rowidx;
  a.Av = (const VT *)A->values;
  a.Bcp = B->colptr;
  a.Bri = B->rowidx;
  a.Bv = (const VT *)B->values;
  a.klo = klo;
  a.khi = khi;
  a.kdim = A->ncols;
  a.m = A->nrows;
  a.nnzA = A->nnz;
  return a;
}

// One symbolic pass over inner range [klo, khi) writing one row of counts.
// Grid of a persistent bin kernel: the exact need when the bin's count is
// known on the host (cnt >= 0), else a fixed grid that fills the device.
static unsigned bin_grid(int cnt, bool wave_kernel, int blocks_per_cu) {
  const unsigned full = (unsigned)(blocks_per_cu * device_cus());
  if (cnt < 0) return full;
  const unsigned need = wave_kernel ? grid_of(cnt, 4) : (unsigned)cnt;
  return std::max(1u, std::min(need, full));
}

__global__ void k_flag_if_nonzero(const int32_t *count, int32_t *status, int code) {
  if (threadIdx.x == 0 && *count > 0) flag_error(status, code);
}

// Column pointers beyond the output capacity are clamped to it (their
// columns then fail the count check and are cut short); the status word
// records the overflow.
__global__ void k_clamp_colptr(int64_t *colptr, int64_t ncol, int64_t cap, int32_t *status) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= ncol; i += (int64_t)gridDim.x * blockDim.x) {
    if (colptr[i] > cap) {
      colptr[i] = cap;
      if (i == ncol) flag_error(status, 8);
    }
  }
}

// One workgroup per instance: copies instance i of a batch into the block
// diagonal at its row/column/entry offsets.
struct PackDesc {
  const int64_t *cp;
  const int32_t *ri;
  const void *v;
  int64_t ncols, nnz, row_off, col_off, nnz_off;
};

template <class VT>
__global__ __launch_bounds__(256) void k_pack(const PackDesc *d, int count, int64_t *cp_out, int32_t *ri_out,
                                              VT *v_out) {
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const PackDesc q = d[i];
    for (int64_t j = threadIdx.x; j < q.ncols; j += 256) cp_out[q.col_off + j] = q.nnz_off + ld_global(q.cp + j);
    for (int64_t p = threadIdx.x; p < q.nnz; p += 256) {
      ri_out[q.nnz_off + p] = (int32_t)(q.row_off + ld_global(q.ri + p));
      if (v_out) v_out[q.nnz_off + p] = ld_global((const VT *)q.v + p);
    }
  }
}

__global__ void k_pack_last(int64_t *cp_out, int64_t ncols, int64_t nnz) {
  if (threadIdx.x == 0) cp_out[ncols] = nnz;
}

// Counts of the bins: read back (one synchronization) or left on the device.
static int bin_counts(WsHeader *hdr, hipStream_t st, bool sync, int *cnt, WsHeader *h) {
  if (sync) {
    int rc = read_header(hdr, st, h);
    if (rc) return rc;
    for (int b = 0; b < kNumBins; b++) cnt[b] = h->bin_count[b];
  } else {
    for (int b = 0; b < kNumBins; b++) cnt[b] = -1;
    memset(h, 0, sizeof(*h));
  }
  return SPGEMM_OK;
}

// One symbolic pass over inner range [klo, khi) writing one row of counts.
static int symbolic_pass(const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t ncol, int64_t klo,
                         int64_t khi, int64_t *flops_out, int64_t *nnz_row, const WsLayout &L, char *ws,
                         hipStream_t st, bool sync, bool keep_status = false) {
  WsHeader *hdr = (WsHeader *)ws;
  int32_t *bins = (int32_t *)(ws + L.bins);
  hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, st, hdr, (uint64_t)0, keep_status ? 1 : 0);
  LAUNCHCHK();
  const int64_t per_block = 4 * kBinColsPerWave;
  {
    ProfScope prof_bin("bin_symbolic", st);
    hipLaunchKernelGGL(k_bin<true>, dim3(grid_of(ncol, per_block)), dim3(256), 0, st, A->colptr, B->colptr,
                       B->rowidx, c0, ncol, klo, khi, (int64_t)A->ncols, A->nrows, (const int64_t *)nullptr,
                       flops_out, nnz_row, bins, hdr, g_min_bin, g_caps[0], (const int64_t *)nullptr, 0.0);
    LAUNCHCHK();
  }
  int cnt[kNumBins];
  WsHeader h;
  int rc = bin_counts(hdr, st, sync, cnt, &h);
  if (rc) return rc;
  ProductArgs<float> a = product_args<float>(A, B, klo, khi);
  int32_t *status = &hdr->status;
  static const char *kSymNames[kNumBins] = {"sym_wave64", "sym_wave256", "sym_wave1024", "sym_block4096",
                                            "sym_block32768", "sym_bitmap"};
  for (int b = 0; b < kNumBins; b++) {
    if (cnt[b] == 0) continue;
    ProfScope prof(kSymNames[b], st);
    const int32_t *list = bins + (int64_t)b * ncol;
    const int32_t *cp = &hdr->bin_count[b];
    switch (b) {
      case 0: hipLaunchKernelGGL(k_sym_wave<64>, dim3(bin_grid(cnt[b], true, g_bpc[0][0])), dim3(256), 0, st, a, c0, list, cp, nnz_row, status); break;
      case 1: hipLaunchKernelGGL(k_sym_wave<256>, dim3(bin_grid(cnt[b], true, g_bpc[0][1])), dim3(256), 0, st, a, c0, list, cp, nnz_row, status); break;
      case 2: hipLaunchKernelGGL(k_sym_wave<1024>, dim3(bin_grid(cnt[b], true, g_bpc[0][2])), dim3(256), 0, st, a, c0, list, cp, nnz_row, status); break;
      case 3: hipLaunchKernelGGL((k_sym_block<4096, 256>), dim3(bin_grid(cnt[b], false, g_bpc[0][3])), dim3(256), 0, st, a, c0, list, cp, nnz_row, status); break;
      case 4: hipLaunchKernelGGL((k_sym_block<32768, 1024>), dim3(bin_grid(cnt[b], false, g_bpc[0][4])), dim3(1024), 0, st, a, c0, list, cp, nnz_row, status); break;
      default: hipLaunchKernelGGL(k_sym_bitmap, dim3(bin_grid(cnt[b], false, 1)), dim3(1024), 0, st, a, c0, list, cp, &hdr->cursor[b], nnz_row, status); break;
    }
    LAUNCHCHK();
  }
  return SPGEMM_OK;
}


// Numeric-style pass (product or merge) once the bins are filled.  cnt[b]
// < 0 means the count is only on the device (no host synchronization);
// then heavy columns must take the slab path (heavy_global = false), and a
// heavy column that would need the global path is reported as an error.
template <class VT, class Src>
static int accumulate_pass(const Src &src, const int *cnt, const WsHeader &h, const WsLayout &L, char *ws,
                           const int64_t *c_colptr, int32_t *out_ri, VT *out_v, hipStream_t st,
                           bool heavy_global = true) {
  WsHeader *hdr = (WsHeader *)ws;
  int32_t *bins = (int32_t *)(ws + L.bins);
  int32_t *status = &hdr->status;
  const int64_t ncol = L.ncol;
  static const char *kNumNames[kNumBins - 1] = {"num_wave64", "num_wave256", "num_wave1024", "num_block4096",
                                                "num_block10240"};
  static const char *kMrgNames[kNumBins - 1] = {"mrg_wave64", "mrg_wave256", "mrg_wave1024", "mrg_block4096",
                                                "mrg_block10240"};
  const char *const *names = Src::kMerge ? kMrgNames : kNumNames;
  for (int b = 0; b < kNumBins - 1; b++) {
    if (cnt[b] == 0) continue;
    ProfScope prof(names[b], st);
    const int32_t *list = bins + (int64_t)b * ncol;
    const int32_t *cp = &hdr->bin_count[b];
    switch (b) {
      case 0: hipLaunchKernelGGL((k_num_wave<64, VT, Src>), dim3(bin_grid(cnt[b], true, g_bpc[1][0])), dim3(256), 0, st, src, list, cp, c_colptr, out_ri, out_v, status); break;
      case 1: hipLaunchKernelGGL((k_num_wave<256, VT, Src>), dim3(bin_grid(cnt[b], true, g_bpc[1][1])), dim3(256), 0, st, src, list, cp, c_colptr, out_ri, out_v, status); break;
      case 2: hipLaunchKernelGGL((k_num_wave<1024, VT, Src>), dim3(bin_grid(cnt[b], true, g_bpc[1][2])), dim3(256), 0, st, src, list, cp, c_colptr, out_ri, out_v, status); break;
      case 3: hipLaunchKernelGGL((k_num_block<4096, 256, VT, Src>), dim3(bin_grid(cnt[b], false, g_bpc[1][3])), dim3(256), 0, st, src, list, cp, c_colptr, out_ri, out_v, status); break;
      default: hipLaunchKernelGGL((k_num_block<10240, 1024, VT, Src>), dim3(bin_grid(cnt[b], false, g_bpc[1][4])), dim3(1024), 0, st, src, list, cp, c_colptr, out_ri, out_v, status); break;
    }
    LAUNCHCHK();
  }
  const int heavy = cnt[kNumBins - 1];
  if (heavy != 0 && heavy_global) {
    if (heavy < 0) {  // no host count: the global path cannot be scheduled
      hipLaunchKernelGGL(k_flag_if_nonzero, dim3(1), dim3(64), 0, st, &hdr->bin_count[kNumBins - 1], status, 7);
      LAUNCHCHK();
      return SPGEMM_OK;
    }
    if (L.slots <= 0) return SPGEMM_E_INVAL;
    double *vals = (double *)(ws + L.heavy_vals);
    uint8_t *flags = (uint8_t *)(ws + L.heavy_flags);
    int64_t *segcnt = (int64_t *)(ws + L.heavy_segcnt);
    const uint64_t tag = zero_region_tag(kTagProduct, L);
    if (h.clean_tag != tag) {
      const int64_t bytes = (int64_t)(L.heavy_segcnt - L.heavy_vals);
      hipLaunchKernelGGL(k_fill_zero, dim3(4 * device_cus()), dim3(256), 0, st, (uint4 *)(ws + L.heavy_vals), bytes / 16);
      LAUNCHCHK();
      hipLaunchKernelGGL(k_set_tag, dim3(1), dim3(64), 0, st, hdr, tag);
      LAUNCHCHK();
    }
    const int32_t *list = bins + (int64_t)(kNumBins - 1) * ncol;
    ProfScope prof("heavy_global", st);
    for (int first = 0; first < heavy; first += (int)L.slots) {
      const int ns = (int)std::min<int64_t>(L.slots, heavy - first);
      int parts = (int)std::max<int64_t>(1, std::min<int64_t>(64, (4 * device_cus() + ns - 1) / ns));
      hipLaunchKernelGGL((k_heavy_acc<Src>), dim3(ns * parts), dim3(256), 0, st, src, list, first, ns, parts, L.m, vals,
                         flags, status);
      LAUNCHCHK();
      hipLaunchKernelGGL(k_heavy_count, dim3((unsigned)(ns * L.nseg)), dim3(256), 0, st, ns, L.m, L.nseg, flags, segcnt);
      LAUNCHCHK();
      hipLaunchKernelGGL((k_heavy_write<VT, typename Src::Sr>), dim3((unsigned)(ns * L.nseg)), dim3(256), 0, st, list, first, ns, L.m,
                         L.nseg, vals, flags, segcnt, c_colptr, out_ri, out_v, status);
      LAUNCHCHK();
    }
  }
  return SPGEMM_OK;
}

// Row-sorted product: the columns that expand-sort-compress forms (chosen
// by esc_class from the symbolic flops of the batch's columns and cf) are
// written in row order to ri / v; the others go to the numeric pass's output.
struct EscOut {
  const int64_t *flops;
  double cf;
  int32_t *ri;
  void *v;
};

template <class VT, class SR>
static int numeric_typed(const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t ncol, int64_t klo,
                         int64_t khi, const int64_t *c_colptr, int32_t *c_rowidx, void *c_values, const WsLayout &L,
                         char *ws, hipStream_t st, bool sync, bool keep_status = false,
                         const EscOut *esc = nullptr) {
  WsHeader *hdr = (WsHeader *)ws;
  int32_t *bins = (int32_t *)(ws + L.bins);
  hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, st, hdr, zero_region_tag(kTagProduct, L),
                     keep_status ? 1 : 0, 1);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_bin<false>, dim3(grid_of(ncol, 4 * kBinColsPerWave)), dim3(256), 0, st, A->colptr, B->colptr,
                     B->rowidx, c0, ncol, klo, khi, (int64_t)A->ncols, A->nrows, c_colptr, (int64_t *)nullptr,
                     (int64_t *)nullptr, bins, hdr, g_min_bin, g_caps[1], esc ? esc->flops : (const int64_t *)nullptr,
                     esc ? esc->cf : 0.0);
  LAUNCHCHK();
  int cnt[kNumBins];
  WsHeader h;
  int rc = bin_counts(hdr, st, sync, cnt, &h);
  if (rc) return rc;
  ProductSrc<VT, SR> src;
  src.a = product_args<VT>(A, B, klo, khi);
  src.c0 = c0;
  if (esc) {
    int32_t *status = &hdr->status;
    for (int e = 0; e < 2; e++) {
      const int ce = sync ? h.esc_count[e] : -1;
      if (ce == 0) continue;
      const int32_t *list = bins + (int64_t)(kNumBins + e) * ncol;
      const int32_t *cp = &hdr->esc_count[e];
      ProfScope prof(e == 0 ? "esc_wave" : "esc_block", st);
      if (e == 0)
        hipLaunchKernelGGL((k_esc_wave<VT, SR>), dim3(bin_grid(ce, true, 8)), dim3(256), 0, st, src.a, c0, list, cp,
                           c_colptr, esc->ri, (VT *)esc->v, status);
      else
        hipLaunchKernelGGL((k_esc_block<VT, SR>), dim3(bin_grid(ce, false, 3)), dim3(256), 0, st, src.a, c0, list,
                           cp, c_colptr, esc->ri, (VT *)esc->v, status);
      LAUNCHCHK();
    }
  }
  const bool slabs = L.P > 0;
  rc = accumulate_pass<VT>(src, cnt, h, L, ws, c_colptr, c_rowidx, (VT *)c_values, st, !slabs);
  if (rc) return rc;
  const int heavy = cnt[kNumBins - 1];
  if (slabs && heavy != 0) {
    int32_t *soff = (int32_t *)(ws + L.slab_off);
    SlabEnt<VT> *s_ent = (SlabEnt<VT> *)(ws + L.slab_ent);
    const int32_t *hc = &hdr->bin_count[kNumBins - 1];
    if (khi > klo) {
      ProfScope prof("slab_split", st);
      uint64_t seed = 0x5eed;
      for (uint64_t x : {(uint64_t)(uintptr_t)A->colptr, (uint64_t)(uintptr_t)A->rowidx, (uint64_t)(uintptr_t)A->values,
                         (uint64_t)A->nnz, (uint64_t)A->nrows, (uint64_t)klo, (uint64_t)khi, (uint64_t)L.P,
                         (uint64_t)sizeof(VT), (uint64_t)L.slab_off, (uint64_t)L.slab_pack})
        seed = fmix64(seed ^ x);
      hipLaunchKernelGGL(k_left_sum<VT>, dim3((unsigned)(4 * device_cus())), dim3(256), 0, st, A->colptr, A->rowidx,
                         (const VT *)A->values, klo, khi, seed, hdr, hc);
      LAUNCHCHK();
      const unsigned pgrid = (unsigned)(8 * device_cus());
      hipLaunchKernelGGL(k_slab_split<VT>, dim3(std::min(grid_of(khi - klo, 4), (unsigned)(4 * device_cus()))),
                         dim3(256), 0, st, A->colptr, A->rowidx, (const VT *)A->values, klo, khi, A->nrows, (int)L.P,
                         soff, s_ent, hc, &hdr->status, hdr);
      LAUNCHCHK();
      hipLaunchKernelGGL(k_seg_pack, dim3(std::min(grid_of(khi - klo, 64) * (unsigned)((L.P + 63) / 64), pgrid)), dim3(256), 0, st,
                         (const int32_t *)soff, A->colptr, klo, khi - klo, (int)L.P, (uint64_t *)(ws + L.slab_pack), hc,
                         (const WsHeader *)hdr);
      LAUNCHCHK();
      hipLaunchKernelGGL(k_left_set, dim3(1), dim3(64), 0, st, hdr, hc);
      LAUNCHCHK();
    }
    HvArgs<VT> ha;
    ha.Acp = A->colptr;
    ha.ent = s_ent;
    ha.Bcp = B->colptr;
    ha.Bri = B->rowidx;
    ha.Bv = (const VT *)B->values;
    ha.pack = (const uint64_t *)(ws + L.slab_pack);
    ha.nnzA = A->nnz;
    ha.klo = (int32_t)klo;
    ha.khi = (int32_t)khi;
    ha.kdim = (int32_t)A->ncols;
    ha.P = (int32_t)L.P;
    const int32_t *list = bins + (int64_t)(kNumBins - 1) * ncol;
    int32_t *hv_cur = (int32_t *)(ws + L.hv_cur);
    uint32_t *slots = (uint32_t *)(ws + L.hv_items);
    int32_t *wlist = (int32_t *)(ws + L.hv_wide);
    const int64_t icap = hv_item_cap(ncol, L.P);
    const int64_t H = std::max<int64_t>(1, icap / L.P);
    const int64_t hmax = heavy > 0 ? heavy : ncol;  // heavy < 0: the count is only on the device
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_of((ncol * 4 + 15) / 16, 256)), dim3(256), 0, st, (uint4 *)hv_cur,
                       (ncol * 4 + 15) / 16);
    LAUNCHCHK();
    for (int64_t h0 = 0; h0 < hmax; h0 += H) {
      const int64_t h1 = std::min(hmax, h0 + H);
      hipLaunchKernelGGL(k_hv_reset, dim3(1), dim3(64), 0, st, hdr);
      LAUNCHCHK();
      {
        ProfScope prof("heavy_plan", st);
        const unsigned pg = (unsigned)std::min<int64_t>(h1 - h0, 16 * (int64_t)device_cus());
        hipLaunchKernelGGL(k_hv_plan, dim3(pg), dim3(kHvPlanThreads), 0, st, B->colptr, B->rowidx, c0, klo, khi,
                           (const int32_t *)soff, (int)L.P, list, hc, h0, h1, slots, wlist, hdr);
        LAUNCHCHK();
      }
      {
        ProfScope prof("heavy_wide", st);
        hipLaunchKernelGGL((k_hv_wide<VT, SR>), dim3(device_cus()), dim3(kHvWideThreads), 0, st, ha, c0, list,
                           (const int32_t *)wlist, ncol, hdr, c_colptr, hv_cur, c_rowidx, (VT *)c_values);
        LAUNCHCHK();
      }
      ProfScope prof("heavy_items", st);
      HvProductSrc<VT, SR> hsrc{ha, c0, (int)L.P};
      hipLaunchKernelGGL((k_hv_items<VT, HvProductSrc<VT, SR>>), dim3(4 * device_cus()), dim3(kHvThreads), 0, st, hsrc, list,
                         (const uint32_t *)slots, h0, h1 - h0, hdr, c_colptr, hv_cur, c_rowidx, (VT *)c_values);
      LAUNCHCHK();
    }
    hipLaunchKernelGGL(k_hv_check, dim3(grid_of(hmax, 256)), dim3(256), 0, st, list, hc, c_colptr,
                       (const int32_t *)hv_cur, &hdr->status);
    LAUNCHCHK();
  }
  return SPGEMM_OK;
}

template <class VT, class SR>
static int merge_typed(const spgemm_csc *parts, int32_t n_parts, const int64_t *c_colptr, int32_t *c_rowidx,
                       void *c_values, const WsLayout &L, char *ws, hipStream_t st) {
  WsHeader *hdr = (WsHeader *)ws;
  int32_t *bins = (int32_t *)(ws + L.bins);
  PartDesc *pd = (PartDesc *)(ws + L.parts);
  hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, st, hdr, zero_region_tag(kTagProduct, L), 0);
  LAUNCHCHK();
  for (int c = 0; c < n_parts; c += kWave) {
    PartsChunk hc;
    memset(&hc, 0, sizeof(hc));
    const int nc = std::min(kWave, n_parts - c);
    for (int p = 0; p < nc; p++) hc.d[p] = PartDesc{parts[c + p].colptr, parts[c + p].rowidx, parts[c + p].values};
    hipLaunchKernelGGL(k_store_parts, dim3(1), dim3(64), 0, st, pd + c, hc, nc);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_bin<false>, dim3(grid_of(L.ncol, 4 * kBinColsPerWave)), dim3(256), 0, st,
                     (const int64_t *)nullptr, (const int64_t *)nullptr, (const int32_t *)nullptr, (int64_t)0, L.ncol,
                     (int64_t)0, (int64_t)0, (int64_t)0, L.m, c_colptr, (int64_t *)nullptr, (int64_t *)nullptr, bins,
                     hdr, g_min_bin, g_caps[1], (const int64_t *)nullptr, 0.0);
  LAUNCHCHK();
  int cnt[kNumBins];
  WsHeader h;
  int rc = bin_counts(hdr, st, true, cnt, &h);
  if (rc) return rc;
  MergeSrc<VT, SR> src;
  src.P = pd;
  src.nparts = n_parts;
  src.m = L.m;
  const int heavy = cnt[kNumBins - 1];
  const bool buckets = L.P > 0 && heavy > 0;
  rc = accumulate_pass<VT>(src, cnt, h, L, ws, c_colptr, c_rowidx, (VT *)c_values, st, !buckets);
  if (rc || !buckets) return rc;
  // heavy columns through the slab buckets
  const int32_t *list = bins + (int64_t)(kNumBins - 1) * L.ncol;
  const int32_t *hcnt = &hdr->bin_count[kNumBins - 1];
  int64_t *len = (int64_t *)(ws + L.mb_len);
  int64_t *base = (int64_t *)(ws + L.mb_base);
  int32_t *soff = (int32_t *)(ws + L.slab_off);
  uint32_t *slots = (uint32_t *)(ws + L.hv_items);
  int32_t *hv_cur = (int32_t *)(ws + L.hv_cur);
  int32_t *brow = (int32_t *)(ws + L.slab_ri);
  VT *bval = (VT *)(ws + L.slab_v);
  int32_t *status = &hdr->status;
  hipLaunchKernelGGL(k_mb_len, dim3(grid_of(heavy, 256)), dim3(256), 0, st, (const PartDesc *)pd, n_parts, list, hcnt,
                     len);
  LAUNCHCHK();
  rc = launch_colptr_scan(len, heavy, base, (int64_t *)(ws + L.scan), st);
  if (rc) return rc;
  std::vector<int64_t> hb((size_t)heavy + 1);
  HIPCHK(hipMemcpyAsync(hb.data(), base, sizeof(int64_t) * (heavy + 1), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_of((L.ncol * 4 + 15) / 16, 256)), dim3(256), 0, st, (uint4 *)hv_cur,
                     (L.ncol * 4 + 15) / 16);
  LAUNCHCHK();
  const int64_t hcap = std::max<int64_t>(1, hv_item_cap(L.ncol, L.P) / L.P);
  const int64_t ecap = L.mb_cap;
  // chunks of the heavy list whose entries fit the bucket region, and in
  // each chunk its bucketing tasks by decreasing size: a column whole, or a
  // long column as two tasks, one per half of its row slabs (task encoding
  // (h << 2) | mode, see k_mb_bucket), so that no single column holds the
  // launch open
  if (heavy >= (int64_t(1) << 29)) return SPGEMM_E_OVERFLOW;
  const int64_t split_min = std::max<int64_t>(int64_t(1) << 16, ecap / 2048);
  std::vector<int64_t> cuts{0}, tcuts{0};
  std::vector<int32_t> ord;
  ord.reserve((size_t)heavy);
  std::vector<std::pair<int64_t, int32_t>> tasks;
  for (int64_t h0 = 0; h0 < heavy;) {
    int64_t h1 = h0 + 1;
    while (h1 < heavy && h1 - h0 < hcap && hb[h1 + 1] - hb[h0] <= ecap) h1++;
    if (hb[h1] - hb[h0] > ecap) {  // one column's entries exceed the bucket region
      hipLaunchKernelGGL(k_flag_if_nonzero, dim3(1), dim3(64), 0, st, hcnt, status, 9);
      LAUNCHCHK();
      return SPGEMM_OK;
    }
    tasks.clear();
    for (int64_t h = h0; h < h1; h++) {
      const int64_t n = hb[h + 1] - hb[h];
      if (n >= split_min && L.P >= 2) {
        tasks.emplace_back((n + 1) / 2, (int32_t)((h << 2) | 1));
        tasks.emplace_back(n / 2, (int32_t)((h << 2) | 2));
      } else {
        tasks.emplace_back(n, (int32_t)(h << 2));
      }
    }
    std::stable_sort(tasks.begin(), tasks.end(), [](const std::pair<int64_t, int32_t> &x,
                                                     const std::pair<int64_t, int32_t> &y) { return x.first > y.first; });
    for (const auto &t : tasks) ord.push_back(t.second);
    cuts.push_back(h1);
    tcuts.push_back((int64_t)ord.size());
    h0 = h1;
  }
  // the lengths are no longer needed once scanned: their room (8 bytes per
  // column) holds the tasks (at most two per heavy column, 4 bytes each)
  int32_t *ord_d = (int32_t *)len;
  HIPCHK(hipMemcpyAsync(ord_d, ord.data(), sizeof(int32_t) * ord.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));  // `ord` is host memory freed on return
  for (size_t c = 0; c + 1 < cuts.size(); c++) {
    const int64_t h0 = cuts[c], h1 = cuts[c + 1];
    const int64_t t0 = tcuts[c], t1 = tcuts[c + 1];
    hipLaunchKernelGGL(k_hv_reset, dim3(1), dim3(64), 0, st, hdr);
    LAUNCHCHK();
    {
      ProfScope prof("merge_bucket", st);
      const unsigned g = (unsigned)std::min<int64_t>(t1 - t0, 4 * (int64_t)device_cus());
      hipLaunchKernelGGL(k_mb_bucket<VT>, dim3(g), dim3(kMbThreads), 0, st, (const PartDesc *)pd, n_parts, L.m,
                         (int)L.P, list, hcnt, h0, h1, (const int32_t *)ord_d, t0, t1, &hdr->mb_cursor,
                         (const int64_t *)base, ecap, soff, brow, bval, slots, status);
      LAUNCHCHK();
    }
    ProfScope prof("merge_items", st);
    MbSrc<VT, SR> msrc{brow, bval, soff, base, h0, (int)L.P};
    hipLaunchKernelGGL((k_hv_items<VT, MbSrc<VT, SR>>), dim3(4 * device_cus()), dim3(kHvThreads), 0, st, msrc, list,
                       (const uint32_t *)slots, h0, h1 - h0, hdr, c_colptr, hv_cur, c_rowidx, (VT *)c_values);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_hv_check, dim3(grid_of(heavy, 256)), dim3(256), 0, st, list, hcnt, c_colptr,
                     (const int32_t *)hv_cur, status);
  LAUNCHCHK();
  return SPGEMM_OK;
}

// Scratch of the allocation-free entry point: one fixed array per device
// (every module load gives each GPU its own copy), shared by every call on
// that device, so calls that overlap on one GPU race.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in):
// the device address comes from hipGetSymbolAddress, taken once per device
// with that device current and kept per device.
static __device__ __align__(256) unsigned char scratch[SPGEMM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
}  // namespace

static int noalloc_scratch(void **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SPGEMM_E_INVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || reinterpret_cast<uintptr_t>(p) % 256) return SPGEMM_E_WORKSPACE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SPGEMM_OK;
}

static_assert(sizeof(PartDesc) == kPartDescBytes, "part descriptor size");
static_assert(sizeof(SlabEnt<float>) == kSlabEntBytes[0] && sizeof(SlabEnt<double>) == kSlabEntBytes[1],
              "slabbed entry sizes");
static_assert(sizeof(WsHeader) <= 2048, "header too large");

}  // namespace spg

namespace spg {
// The numeric pass for the dtype of A and a semiring (keep_status: a
// layer's call keeps the status its share of B may have set).
static int numeric_dispatch(const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t ncol, int64_t klo,
                            int64_t khi, const int64_t *c_colptr, int32_t *c_rowidx, void *c_values, int32_t semiring,
                            const WsLayout &L, char *ws, hipStream_t s, bool keep_status,
                            const EscOut *esc = nullptr) {
  const bool f32 = A->dtype == SPGEMM_F32;
  // The bin counts are read back only when heavy columns may need the
  // global accumulators (their launches are sized on the host); otherwise
  // every kernel takes its count from the device and the call does not
  // synchronize the stream.
  const bool sync = L.slots > 0;
  switch (semiring) {
    case SPGEMM_SR_MIN_PLUS:
      return f32 ? numeric_typed<float, SrMinPlus>(A, B, c0, ncol, klo, khi, c_colptr, c_rowidx, c_values, L, ws, s,
                                                   sync, keep_status, esc)
                 : numeric_typed<double, SrMinPlus>(A, B, c0, ncol, klo, khi, c_colptr, c_rowidx, c_values, L, ws, s,
                                                    sync, keep_status, esc);
    case SPGEMM_SR_OR_AND:
      return f32 ? numeric_typed<float, SrOrAnd>(A, B, c0, ncol, klo, khi, c_colptr, c_rowidx, c_values, L, ws, s,
                                                 sync, keep_status, esc)
                 : numeric_typed<double, SrOrAnd>(A, B, c0, ncol, klo, khi, c_colptr, c_rowidx, c_values, L, ws, s,
                                                  sync, keep_status, esc);
    default:
      return f32 ? numeric_typed<float, SrPlusTimes>(A, B, c0, ncol, klo, khi, c_colptr, c_rowidx, c_values, L, ws,
                                                     s, sync, keep_status, esc)
                 : numeric_typed<double, SrPlusTimes>(A, B, c0, ncol, klo, khi, c_colptr, c_rowidx, c_values, L, ws,
                                                      s, sync, keep_status, esc);
  }
}
}  // namespace spg

using namespace spg;

extern "C" {

int spgemm_symbolic(const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t c1, int32_t n_layers,
                    int64_t *flops_out, int64_t *nnz_out, void *ws, size_t ws_bytes, void *stream) {
  int st = check_csc(A, false);
  if (!st) st = check_csc(B, false);
  if (st) return st;
  if (A->ncols != B->nrows) return SPGEMM_E_SHAPE;
  if (c0 < 0 || c1 < c0 || c1 > B->ncols || n_layers < 1) return SPGEMM_E_INVAL;
  if (c1 > c0 && !nnz_out) return SPGEMM_E_INVAL;
  WsLayout L;
  st = ws_layout(SPGEMM_OP_SYMBOLIC, A, B, c0, c1, n_layers, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  const int64_t ncol = c1 - c0;
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)ws;
  if (ncol == 0) {
    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, s, (WsHeader *)w, (uint64_t)0, 0);
    LAUNCHCHK();
    return SPGEMM_OK;
  }
  const int64_t kdim = A->ncols;
  if (n_layers == 1) return symbolic_pass(A, B, c0, ncol, 0, kdim, flops_out, nnz_out, L, w, s, true);
  const int64_t width = (kdim + n_layers - 1) / n_layers;
  for (int32_t l = 0; l < n_layers; l++) {
    const int64_t klo = std::min<int64_t>(kdim, (int64_t)l * width), khi = std::min<int64_t>(kdim, klo + width);
    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, s, (WsHeader *)w, (uint64_t)0, 0);
    LAUNCHCHK();
    spgemm_csc Bl;
    int rc = build_layer<float>(B, c0, ncol, klo, khi, kdim, false, L, w, s, &Bl);
    if (rc) return rc;
    rc = symbolic_pass(A, &Bl, 0, ncol, klo, khi, nullptr, nnz_out + (int64_t)l * ncol, L, w, s, true, true);
    if (rc) return rc;
  }
  return symbolic_pass(A, B, c0, ncol, 0, kdim, flops_out, nnz_out + (int64_t)n_layers * ncol, L, w, s, true);
}

int spgemm_numeric(const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t c1, int32_t layer,
                   int32_t n_layers, const int64_t *flops, const int64_t *c_colptr, int32_t *c_rowidx,
                   void *c_values, int32_t semiring, void *ws, size_t ws_bytes, void *stream) {
  if (semiring < SPGEMM_SR_PLUS_TIMES || semiring > SPGEMM_SR_OR_AND) return SPGEMM_E_INVAL;
  (void)flops;
  int st = check_csc(A, true);
  if (!st) st = check_csc(B, true);
  if (st) return st;
  if (A->dtype != B->dtype) return SPGEMM_E_DTYPE;
  if (A->ncols != B->nrows) return SPGEMM_E_SHAPE;
  if (c0 < 0 || c1 < c0 || c1 > B->ncols || n_layers < 1 || layer < 0 || layer >= n_layers) return SPGEMM_E_INVAL;
  WsLayout L;
  st = ws_layout(SPGEMM_OP_NUMERIC, A, B, c0, c1, n_layers, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  const int64_t ncol = c1 - c0;
  if (ncol > 0 && !c_colptr) return SPGEMM_E_INVAL;
  if (ncol == 0) {
    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, (hipStream_t)stream, (WsHeader *)ws, kKeepAnyTag, 0);
    LAUNCHCHK();
    return SPGEMM_OK;
  }
  const int64_t kdim = A->ncols;
  const int64_t width = (kdim + n_layers - 1) / n_layers;
  const int64_t klo = std::min<int64_t>(kdim, (int64_t)layer * width), khi = std::min<int64_t>(kdim, klo + width);
  hipStream_t s = (hipStream_t)stream;
  if (n_layers > 1) {  // the layer's share of B first, then the passes over it
    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, s, (WsHeader *)ws, zero_region_tag(kTagProduct, L), 0,
                       1);
    LAUNCHCHK();
    spgemm_csc Bl;
    st = A->dtype == SPGEMM_F32 ? build_layer<float>(B, c0, ncol, klo, khi, kdim, true, L, (char *)ws, s, &Bl)
                                : build_layer<double>(B, c0, ncol, klo, khi, kdim, true, L, (char *)ws, s, &Bl);
    if (st) return st;
    return numeric_dispatch(A, &Bl, 0, ncol, klo, khi, c_colptr, c_rowidx, c_values, semiring, L, (char *)ws, s,
                            true);
  }
  return numeric_dispatch(A, B, c0, ncol, klo, khi, c_colptr, c_rowidx, c_values, semiring, L, (char *)ws, s, false);
}

int spgemm_numeric_sorted(const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t c1, const int64_t *flops,
                          const int64_t *c_colptr, int32_t *c_rowidx, void *c_values, int32_t *tmp_rowidx,
                          void *tmp_values, double esc_cf_max, int32_t semiring, void *ws, size_t ws_bytes,
                          void *stream) {
  if (semiring < SPGEMM_SR_PLUS_TIMES || semiring > SPGEMM_SR_OR_AND) return SPGEMM_E_INVAL;
  if (!(esc_cf_max >= 0.0)) return SPGEMM_E_INVAL;  // NaN included
  int st = check_csc(A, true);
  if (!st) st = check_csc(B, true);
  if (st) return st;
  if (A->dtype != B->dtype) return SPGEMM_E_DTYPE;
  if (A->ncols != B->nrows) return SPGEMM_E_SHAPE;
  if (c0 < 0 || c1 < c0 || c1 > B->ncols) return SPGEMM_E_INVAL;
  WsLayout L;
  st = ws_layout(SPGEMM_OP_NUMERIC, A, B, c0, c1, 1, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  const int64_t ncol = c1 - c0;
  hipStream_t s = (hipStream_t)stream;
  if (ncol == 0) {
    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, s, (WsHeader *)ws, kKeepAnyTag, 0);
    LAUNCHCHK();
    return SPGEMM_OK;
  }
  if (!c_colptr || !c_rowidx || !c_values || !tmp_rowidx || !tmp_values) return SPGEMM_E_INVAL;
  if ((void *)tmp_rowidx == (void *)c_rowidx || tmp_values == c_values) return SPGEMM_E_INVAL;  // out of place
  const bool use_esc = esc_cf_max > 0.0;
  if (use_esc && !flops) return SPGEMM_E_INVAL;
  const EscOut esc{flops, esc_cf_max, c_rowidx, c_values};
  st = numeric_dispatch(A, B, c0, ncol, 0, A->ncols, c_colptr, tmp_rowidx, tmp_values, semiring, L, (char *)ws, s,
                        false, use_esc ? &esc : nullptr);
  if (st) return st;
  // the hashed columns, from the staging arrays into row order (the bin
  // lists are free again: the sort pass lists its columns there)
  st = launch_reset_counters((WsHeader *)ws, s);
  if (st) return st;
  spgemm_csc T = *A;
  T.ncols = ncol;
  T.colptr = c_colptr;
  T.rowidx = tmp_rowidx;
  T.values = tmp_values;
  return sort_column_lists(&T, c_rowidx, c_values, (int32_t *)((char *)ws + L.bins), (WsHeader *)ws,
                           use_esc ? flops : nullptr, esc_cf_max, s);
}

int spgemm_merge(const spgemm_csc *parts, int32_t n_parts, const int64_t *c_colptr, int32_t *c_rowidx,
                 void *c_values, int32_t semiring, void *ws, size_t ws_bytes, void *stream) {
  if (!parts || n_parts < 1 || n_parts > kMaxParts) return SPGEMM_E_INVAL;
  if (semiring < SPGEMM_SR_PLUS_TIMES || semiring > SPGEMM_SR_OR_AND) return SPGEMM_E_INVAL;
  for (int p = 0; p < n_parts; p++) {
    int st = check_csc(&parts[p], true);
    if (st) return st;
    if (parts[p].nrows != parts[0].nrows || parts[p].ncols != parts[0].ncols) return SPGEMM_E_SHAPE;
    if (parts[p].dtype != parts[0].dtype) return SPGEMM_E_DTYPE;
  }
  WsLayout L;
  int st = ws_layout(SPGEMM_OP_MERGE, &parts[0], nullptr, 0, 0, n_parts, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  if (L.ncol > 0 && !c_colptr) return SPGEMM_E_INVAL;
  if (L.ncol == 0) {
    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, (hipStream_t)stream, (WsHeader *)ws, kKeepAnyTag, 0);
    LAUNCHCHK();
    return SPGEMM_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool f32 = parts[0].dtype == SPGEMM_F32;
  char *w = (char *)ws;
  switch (semiring) {
    case SPGEMM_SR_MIN_PLUS:
      return f32 ? merge_typed<float, SrMinPlus>(parts, n_parts, c_colptr, c_rowidx, c_values, L, w, s)
                 : merge_typed<double, SrMinPlus>(parts, n_parts, c_colptr, c_rowidx, c_values, L, w, s);
    case SPGEMM_SR_OR_AND:
      return f32 ? merge_typed<float, SrOrAnd>(parts, n_parts, c_colptr, c_rowidx, c_values, L, w, s)
                 : merge_typed<double, SrOrAnd>(parts, n_parts, c_colptr, c_rowidx, c_values, L, w, s);
    default:
      return f32 ? merge_typed<float, SrPlusTimes>(parts, n_parts, c_colptr, c_rowidx, c_values, L, w, s)
                 : merge_typed<double, SrPlusTimes>(parts, n_parts, c_colptr, c_rowidx, c_values, L, w, s);
  }
}

int spgemm_colptr(const int64_t *counts, int64_t n, int64_t *colptr_out, void *ws, size_t ws_bytes, void *stream) {
  if (n < 0 || !colptr_out || (n > 0 && !counts)) return SPGEMM_E_INVAL;
  WsLayout L;
  int st = ws_layout(SPGEMM_OP_COLPTR, nullptr, nullptr, 0, n, 1, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)ws;
  st = launch_init_header((WsHeader *)w, 0, s);
  if (st) return st;
  return launch_colptr_scan(counts, n, colptr_out, (int64_t *)(w + L.scan), s);
}

int spgemm_batched_forward(const spgemm_csc *A, const spgemm_csc *B, int64_t nnz_cap, int64_t *flops_out,
                           int64_t *nnz_out, int64_t *c_colptr, int32_t *c_rowidx, void *c_values, void *ws,
                           size_t ws_bytes, void *stream) {
  int st = check_csc(A, true);
  if (!st) st = check_csc(B, true);
  if (st) return st;
  if (A->dtype != B->dtype) return SPGEMM_E_DTYPE;
  if (A->ncols != B->nrows) return SPGEMM_E_SHAPE;
  if (nnz_cap < 0 || !nnz_out || !c_colptr || (nnz_cap > 0 && (!c_rowidx || !c_values))) return SPGEMM_E_INVAL;
  WsLayout L;
  st = ws_layout(SPGEMM_OP_BATCHED_FORWARD, A, B, 0, B->ncols, 1, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)ws;
  const int64_t n = B->ncols;
  if (n == 0) {
    st = launch_init_header((WsHeader *)w, 0, s);
    if (st) return st;
    return launch_colptr_scan(nnz_out, 0, c_colptr, (int64_t *)(w + L.scan), s);
  }
  st = symbolic_pass(A, B, 0, n, 0, A->ncols, flops_out, nnz_out, L, w, s, false);
  if (st) return st;
  st = launch_colptr_scan(nnz_out, n, c_colptr, (int64_t *)(w + L.scan), s);
  if (st) return st;
  hipLaunchKernelGGL(k_clamp_colptr, dim3(std::max(1u, std::min(grid_of(n + 1, 256), 1024u))), dim3(256), 0, s,
                     c_colptr, n, nnz_cap, &((WsHeader *)w)->status);
  LAUNCHCHK();
  // the numeric pass keeps the status word, so an overflow found above is reported
  if (A->dtype == SPGEMM_F32)
    return numeric_typed<float, SrPlusTimes>(A, B, 0, n, 0, A->ncols, c_colptr, c_rowidx, c_values, L, w, s, false,
                                             true);
  return numeric_typed<double, SrPlusTimes>(A, B, 0, n, 0, A->ncols, c_colptr, c_rowidx, c_values, L, w, s, false,
                                            true);
}

int spgemm_batched_forward_noalloc(const spgemm_csc *A, const spgemm_csc *B, int64_t nnz_cap, int64_t *flops_out,
                                   int64_t *nnz_out, int64_t *c_colptr, int32_t *c_rowidx, void *c_values,
                                   void *stream) {
  int st = check_csc(A, true);
  if (!st) st = check_csc(B, true);
  if (st) return st;
  if (A->dtype != B->dtype) return SPGEMM_E_DTYPE;
  if (A->ncols != B->nrows) return SPGEMM_E_SHAPE;
  WsLayout L;
  st = ws_layout(SPGEMM_OP_BATCHED_FORWARD, A, B, 0, B->ncols, 1, &L);
  if (st) return st;
  if (L.total > (size_t)SPGEMM_NOALLOC_SCRATCH_BYTES) return SPGEMM_E_WORKSPACE;  // before any HIP call
  void *ws = nullptr;
  st = noalloc_scratch(&ws);
  if (st) return st;
  return spgemm_batched_forward(A, B, nnz_cap, flops_out, nnz_out, c_colptr, c_rowidx, c_values, ws,
                                (size_t)SPGEMM_NOALLOC_SCRATCH_BYTES, stream);
}

int spgemm_set_bin_caps(int32_t which, const int64_t *caps_host) {
  if (which == 2 || which == 3) {  // workgroups per compute unit of the bin kernels
    const int t = which - 2;
    int v[kNumBins - 1];
    for (int b = 0; b < kNumBins - 1; b++) {
      const int64_t x = caps_host ? caps_host[b] : kBpcDefault[t][b];
      if (x < 1 || x > 32) return SPGEMM_E_INVAL;
      v[b] = (int)x;
    }
    for (int b = 0; b < kNumBins - 1; b++) g_bpc[t][b] = v[b];
    return SPGEMM_OK;
  }
  if (which != 0 && which != 1) return SPGEMM_E_INVAL;
  const int64_t *table = which == 0 ? kSymTableCap : kNumTableCap;
  BinCaps c;
  for (int b = 0; b < kNumBins - 1; b++) c.cap[b] = caps_host ? caps_host[b] : table[b];
  for (int b = 0; b < kNumBins - 1; b++) {
    if (c.cap[b] < 1 || c.cap[b] > table[b]) return SPGEMM_E_INVAL;
    if (b > 0 && c.cap[b] < c.cap[b - 1]) return SPGEMM_E_INVAL;
  }
  g_caps[which] = c;
  return SPGEMM_OK;
}

int spgemm_batch_pack(const spgemm_csc *instances, int32_t count, int64_t *colptr_out, int32_t *rowidx_out,
                      void *values_out, int64_t *offsets_host, void *ws, size_t ws_bytes, void *stream) {
  if (!instances || count < 0 || !colptr_out || !offsets_host) return SPGEMM_E_INVAL;
  const int32_t dt = instances[0].dtype;
  int64_t rows = 0, cols = 0, nnz = 0;
  std::vector<PackDesc> d((size_t)std::max(count, 1));
  for (int i = 0; i < count; i++) {
    const spgemm_csc &q = instances[i];
    int st = check_csc(&q, values_out != nullptr);
    if (st) return st;
    if (values_out && q.dtype != dt) return SPGEMM_E_DTYPE;
    d[i] = PackDesc{q.colptr, q.rowidx, q.values, q.ncols, q.nnz, rows, cols, nnz};
    offsets_host[3 * i + 0] = rows;
    offsets_host[3 * i + 1] = cols;
    offsets_host[3 * i + 2] = nnz;
    rows += q.nrows;
    cols += q.ncols;
    nnz += q.nnz;
  }
  offsets_host[3 * count + 0] = rows;
  offsets_host[3 * count + 1] = cols;
  offsets_host[3 * count + 2] = nnz;
  if (rows > INT32_MAX) return SPGEMM_E_OVERFLOW;
  if (nnz > 0 && !rowidx_out) return SPGEMM_E_INVAL;
  const size_t need = sizeof(PackDesc) * (size_t)std::max(count, 1);
  int st = check_ws(ws, ws_bytes, need);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if (count > 0) {
    HIPCHK(hipMemcpyAsync(ws, d.data(), sizeof(PackDesc) * (size_t)count, hipMemcpyHostToDevice, s));
    const unsigned g = (unsigned)std::min(count, 8 * device_cus());
    if (values_out && dt == SPGEMM_F64)
      hipLaunchKernelGGL(k_pack<double>, dim3(g), dim3(256), 0, s, (const PackDesc *)ws, count, colptr_out, rowidx_out,
                         (double *)values_out);
    else
      hipLaunchKernelGGL(k_pack<float>, dim3(g), dim3(256), 0, s, (const PackDesc *)ws, count, colptr_out, rowidx_out,
                         (float *)values_out);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_pack_last, dim3(1), dim3(64), 0, s, colptr_out, cols, nnz);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));  // the descriptor staging buffer is pageable host memory
  return SPGEMM_OK;
}

int spgemm_debug_min_bin(int32_t bin) {
  if (bin < 0 || bin >= kNumBins) return SPGEMM_E_INVAL;
  g_min_bin = bin;
  return SPGEMM_OK;
}

int spgemm_ws_invalidate(void *ws, void *stream) {
  if (!ws) return SPGEMM_E_WORKSPACE;
  hipLaunchKernelGGL(k_left_forget, dim3(1), dim3(64), 0, (hipStream_t)stream, (WsHeader *)ws);
  LAUNCHCHK();
  return SPGEMM_OK;
}

int spgemm_ws_status_code(void *ws, void *stream, int32_t *code_host) {
  if (code_host) *code_host = 0;
  if (!ws) return SPGEMM_E_WORKSPACE;
  WsHeader h;
  hipStream_t s = (hipStream_t)stream;
  int rc = read_header((WsHeader *)ws, s, &h);
  if (rc) return rc;
  if (h.status != 0) {
    if (code_host) *code_host = h.status;
    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, s, (WsHeader *)ws, kKeepAnyTag, 0);
    return SPGEMM_E_DEVICE;
  }
  return SPGEMM_OK;
}

int spgemm_ws_status(void *ws, void *stream) { return spgemm_ws_status_code(ws, stream, nullptr); }

}  // extern "C"
