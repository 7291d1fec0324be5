// Per-column pruning of one output batch: the step an application applies
// to each batch of C before it moves on to the next (Sec. I and Sec. IV-B:
// Markov clustering keeps the k largest entries of every column; Sec. V-C:
// HipMCL prunes column by column).
//
// Candidates are the entries with value >= threshold, compared in float64
// (NaN is never a candidate).  With k >= 0 at most the k largest candidates
// are kept, equal values going to the smaller row; kept entries stay in
// their input order, so the hash-table order of the numeric pass carries
// over unchanged.
//
// One workgroup per column.  Every entry gets a composite key that orders
// it as the selection does: the value mapped onto an unsigned integer in
// numeric order (-0 folded onto +0), then the row mapped so that a smaller
// row ranks higher.  Rows are unique inside a column, so keys are too, and
// a most-significant-digit radix select ends with a cut key: an entry is
// kept iff it is a candidate and its key is at least the cut.  The first
// digit is wide (12 bits, a 4096-bucket LDS histogram that skips entries
// below a lower bound on the k-th largest key's digit) and its chosen bucket
// is usually settled by sorting its candidates in LDS; otherwise 8-bit
// digits (256-bucket histograms) follow.  A scan of the per-column counts
// gives the output column pointers, and a second kernel compacts the kept
// entries in order with one exchange of per-wave counts per 2048 entries
// that keep any (one flag per wave for those that keep none).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "hip_host.hpp"
#include "internal.hpp"
#include "profile.hpp"

namespace spg {
namespace {

constexpr int kPrThreads = 256;
constexpr int kPrWaves = kPrThreads / kWave;
constexpr int kPrMaxGrid = 65536;
constexpr int kSelUnroll = 8;    // select: coalesced loads per thread per step
constexpr int kFillUnroll = 8;   // compaction: coalesced slots per thread per step
constexpr int kPrDupRows = 10;  // status code: a row twice in one column

__device__ __forceinline__ uint64_t order_key(float v) {
  uint32_t b = __float_as_uint(v);
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? (uint64_t)(~b) : (uint64_t)(b | 0x80000000u);
}
__device__ __forceinline__ uint64_t order_key(double v) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  if (b == 0x8000000000000000ull) b = 0ull;
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
// rows in [0, 2^31 - 1] map onto [2^31 - 1, 0]: the smaller row, the larger key
__device__ __forceinline__ uint32_t row_key(int32_t r) { return 0x7FFFFFFFu - (uint32_t)r; }

// Digit d of the composite key, most significant first: VD digits of the
// value key, then 4 of the row key.
template <int VD>
__device__ __forceinline__ int key_digit(int d, uint64_t vk, uint32_t rk) {
  return d < VD ? (int)((vk >> (8 * (VD - 1 - d))) & 255u) : (int)((rk >> (8 * (3 - (d - VD)))) & 255u);
}
// Masks of the digits above d.
template <int VD>
__device__ __forceinline__ uint64_t value_mask(int d) {
  return d >= VD ? ~0ull : (d == 0 ? 0ull : (~0ull << (8 * (VD - d))));
}
template <int VD>
__device__ __forceinline__ uint32_t row_mask(int d) {
  return d <= VD ? 0u : (~0u << (8 * (4 - (d - VD))));
}

template <typename VT>
__device__ __forceinline__ bool candidate(VT v, double thr) {
  return (double)v >= thr;
}

// Adds one to s_hist[dig] for every lane with `act`.  The digit of the first
// such lane is added once for all lanes that share it (one LDS atomic
// instead of up to 64 serialized on one address: the leading digits of a
// column's keys fall mostly into one or two buckets); the other lanes add
// their own.  Called by the whole wave.
__device__ __forceinline__ void hist_add(int *s_hist, bool act, int dig) {
  const uint64_t m = __ballot(act);
  if (m == 0) return;
  const int src = __builtin_ctzll(m);
  const int lead = __builtin_amdgcn_readlane(dig, src);
  const bool same = act && dig == lead;
  const uint64_t ms = __ballot(same);
  if (lane() == src) atomicAdd(&s_hist[lead], __popcll(ms));
  if (act && !same) atomicAdd(&s_hist[dig], 1);
}

// Wide first digit: the top kWideBits of the value key (sign, exponent and
// the top mantissa bits of a float32), a 4096-bucket histogram; the bucket
// holding the k-th largest key is then resolved in LDS when it holds at most
// kStage candidates (gathered by a second pass, sorted by key), so most
// columns are read twice whatever their length.
constexpr int kWideBits = 12;
constexpr int kWideBuckets = 1 << kWideBits;
constexpr int kStage = 2048;

// Bitonic sort of s_v / s_r (n a power of two), descending by (value key,
// row key).  Contains barriers.
__device__ __forceinline__ void stage_sort_desc(uint64_t *s_v, uint32_t *s_r, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int s = k >> 1; s > 0; s >>= 1) {
      for (int t = threadIdx.x; t < n / 2; t += kPrThreads) {
        const int a = ((t & ~(s - 1)) << 1) | (t & (s - 1));  // lower element of pair t at distance s
        const int c = a + s;
        const bool down = (a & k) == 0;  // this block of k sorts descending
        const uint64_t va = s_v[a], vc = s_v[c];
        const uint32_t ra = s_r[a], rc = s_r[c];
        const bool lt = va < vc || (va == vc && ra < rc);  // key a below key c
        if (lt == down) {
          s_v[a] = vc;
          s_v[c] = va;
          s_r[a] = rc;
          s_r[c] = ra;
        }
      }
      __syncthreads();
    }
  }
}

// cnt[j]: entries column j keeps; (cutv[j], cutr[j]): the smallest kept key
// ((0, 0) keeps every candidate).  The histogram of the first digit also
// counts the candidates, so a column that keeps all of them is read once.
template <typename VT>
__global__ __launch_bounds__(kPrThreads) void k_prune_select(const int64_t *__restrict__ colptr,
                                                             const int32_t *__restrict__ rowidx,
                                                             const VT *__restrict__ vals, int64_t ncols, double thr,
                                                             int64_t nnz, int64_t k, int64_t *__restrict__ cnt,
                                                             uint64_t *__restrict__ cutv, uint32_t *__restrict__ cutr,
                                                             int32_t *status) {
  constexpr int VD = (int)sizeof(VT), ND = VD + 4;
  constexpr int kShift = 8 * VD - kWideBits;  // value key bits below the wide digit
  __shared__ int s_hist[256];
  __shared__ int s_sel[4];  // chosen digit, entries still needed inside it, selection complete, candidates
  // the wide histogram, then (same memory) the staged value keys of its chosen bucket
  __shared__ __align__(16) uint64_t s_wide[kWideBuckets / 2];
  __shared__ uint32_t s_srow[kStage];
  __shared__ int s_n;
  __shared__ int s_ncw[kPrWaves];  // candidates counted by each wave
  int *s_whist = reinterpret_cast<int *>(s_wide);
  const int t = threadIdx.x;
  for (int64_t j = blockIdx.x; j < ncols; j += gridDim.x) {
    int64_t b = colptr[j], e = colptr[j + 1];
    if (b < 0 || e < b || e > nnz) {  // pointers outside the arrays: the column counts as empty
      if (t == 0) flag_error(status, 5);
      b = e = 0;
    }
    // need: entries still to keep among those matching the prefix; until the
    // first digit has counted the candidates it stands for "all of them"
    int need = k >= 0 && k < INT32_MAX ? (int)k : INT32_MAX, above = 0, last = 0, kept = -1;
    uint64_t pv = 0;
    uint32_t pr = 0;
    bool fast = k > 0 && k < INT32_MAX;  // the wide digit first; cleared when the digit loop must run
    if (fast) {
      // A lower bound on the wide digit of the k-th largest key of a column
      // longer than one step: the k-th largest of the per-thread maxima of
      // the first step (k distinct entries at or above it), rounded down to
      // its bucket.  Buckets below it cannot hold one of the k largest keys
      // and are not counted (the candidates are counted apart).
      int lo_dig = 0;
      if (e - b > kSelUnroll * kPrThreads && k <= kPrThreads) {
        uint64_t mk = 0;
        bool has = false;
#pragma unroll
        for (int q = 0; q < kSelUnroll; q++) {
          // (an opaque index: these loads stay apart from the histogram loop's)
          const VT v = vals[opaque(b + q * kPrThreads + t)];
          if (candidate(v, thr)) {
            const uint64_t vk = order_key(v);
            mk = vk > mk ? vk : mk;
            has = true;
          }
        }
        for (int i = t; i < kWideBuckets; i += kPrThreads) s_whist[i] = 0;
        __syncthreads();
        if (has) atomicAdd(&s_whist[(int)(mk >> kShift)], 1);
        __syncthreads();
        if (t < kWave) {
          constexpr int PER = kWideBuckets / kWave;
          int sum = 0;
#pragma unroll 1
          for (int q = 0; q < PER; q++) sum += s_whist[kWideBuckets - 1 - PER * t - q];
          const int incl = wave_incl_add(sum);
          if (t == kWave - 1 && incl < need) s_sel[0] = 0;  // fewer maxima than k: no bound
          int acc = incl - sum;
          if (acc < need && need <= incl) {
#pragma unroll 1
            for (int q = 0; q < PER; q++) {
              acc += s_whist[kWideBuckets - 1 - PER * t - q];
              if (acc >= need) {
                s_sel[0] = kWideBuckets - 1 - PER * t - q;
                break;
              }
            }
          }
        }
        __syncthreads();
        lo_dig = s_sel[0];
      }
      for (int i = t; i < kWideBuckets; i += kPrThreads) s_whist[i] = 0;
      __syncthreads();
      int nc = 0;  // this thread's candidates
      for (int64_t c0 = b; c0 < e; c0 += kSelUnroll * kPrThreads) {
        VT vq[kSelUnroll];
#pragma unroll
        for (int q = 0; q < kSelUnroll; q++) {
          const int64_t p = c0 + q * kPrThreads + t;
          vq[q] = p < e ? vals[p] : VT(0);
        }
#pragma unroll
        for (int q = 0; q < kSelUnroll; q++) {
          const int64_t p = c0 + q * kPrThreads + t;
          const bool cand = p < e && candidate(vq[q], thr);
          const int dig = cand ? (int)(order_key(vq[q]) >> kShift) : 0;
          nc += cand ? 1 : 0;
          hist_add(s_whist, cand && dig >= lo_dig, dig);
        }
      }
      nc = wave_sum_i32(nc);
      if (lane() == 0) s_ncw[t / kWave] = nc;
      __syncthreads();
      if (t < kWave) {
        // lane l owns buckets 4095 - 64l ... 4032 - 64l, scanned from the top
        constexpr int PER = kWideBuckets / kWave;
        int sum = 0;
        for (int q = 0; q < PER; q++) sum += s_whist[kWideBuckets - 1 - PER * t - q];
        const int incl = wave_incl_add(sum);
        if (t == kWave - 1) {
          int tot = 0;
#pragma unroll
          for (int z = 0; z < kPrWaves; z++) tot += s_ncw[z];
          s_sel[3] = tot;
        }
        int acc = incl - sum;
        if (acc < need && need <= incl) {
          for (int q = 0; q < PER; q++) {
            const int h = s_whist[kWideBuckets - 1 - PER * t - q];
            if (acc + h >= need) {
              s_sel[0] = kWideBuckets - 1 - PER * t - q;
              s_sel[1] = need - acc;
              s_sel[2] = h;
              break;
            }
            acc += h;
          }
        }
      }
      __syncthreads();
      const int ncand = s_sel[3];
      if (ncand <= need) {  // every candidate is kept
        kept = ncand;
      } else if (s_sel[2] <= kStage) {
        // gather the chosen bucket's candidates, sort them, take the need-th largest
        const uint64_t bucket = (uint64_t)s_sel[0];
        const int rest = s_sel[1], nb = s_sel[2];
        __syncthreads();  // s_sel and the histogram are read; the stage reuses its memory
        if (t == 0) s_n = 0;
        __syncthreads();
        for (int64_t c0 = b; c0 < e; c0 += kSelUnroll * kPrThreads) {
          VT vq[kSelUnroll];
#pragma unroll
          for (int q = 0; q < kSelUnroll; q++) {
            const int64_t p = c0 + q * kPrThreads + t;
            vq[q] = p < e ? vals[p] : VT(0);
          }
#pragma unroll
          for (int q = 0; q < kSelUnroll; q++) {
            const int64_t p = c0 + q * kPrThreads + t;
            const uint64_t vk = order_key(vq[q]);
            const bool in = p < e && candidate(vq[q], thr) && (vk >> kShift) == bucket;
            const uint64_t m = __ballot(in);
            if (m == 0) continue;  // uniform
            int base = 0;
            if (lane() == 0) base = atomicAdd(&s_n, __popcll(m));
            base = readlane(base, 0);
            const int pos = base + mbcnt(m);
            if (in && pos < kStage) {
              s_wide[pos] = vk;
              s_srow[pos] = row_key(rowidx[p]);
            }
          }
        }
        __syncthreads();
        int n2 = kWave;
        while (n2 < nb) n2 <<= 1;
        for (int i = nb + t; i < n2; i += kPrThreads) {  // padding sorts last
          s_wide[i] = 0ull;
          s_srow[i] = 0u;
        }
        __syncthreads();
        stage_sort_desc(s_wide, s_srow, n2);
        above = need - rest;
        need = rest;
        pv = s_wide[rest - 1];
        pr = s_srow[rest - 1];
        kept = (int)k;
        __syncthreads();  // the stage is rewritten by the next column
      } else {
        fast = false;  // the bucket is too full to stage: the digit loop decides
        __syncthreads();
      }
    }
    for (int d = 0; d < ND && !fast; d++) {
      for (int i = t; i < 256; i += kPrThreads) s_hist[i] = 0;
      if (t == 0) {
        s_sel[0] = 0;
        s_sel[1] = need;
        s_sel[2] = 1;
      }
      __syncthreads();
      const uint64_t vm = value_mask<VD>(d);
      const uint32_t rm = row_mask<VD>(d);
      // kSelUnroll coalesced loads per thread in flight, then their digits;
      // the same trip count for every lane
      for (int64_t c0 = b; c0 < e; c0 += kSelUnroll * kPrThreads) {
        VT vq[kSelUnroll];
#pragma unroll
        for (int q = 0; q < kSelUnroll; q++) {
          const int64_t p = c0 + q * kPrThreads + t;
          vq[q] = p < e ? vals[p] : VT(0);
        }
#pragma unroll
        for (int q = 0; q < kSelUnroll; q++) {
          const int64_t p = c0 + q * kPrThreads + t;
          bool act = false;
          int dig = 0;
          if (p < e) {
            const VT v = vq[q];
            if (candidate(v, thr)) {
              const uint64_t vk = order_key(v);
              if (d < VD) {  // value digits: the row is not read
                act = (vk & vm) == pv;
                dig = key_digit<VD>(d, vk, 0u);
              } else if (vk == pv) {  // row digits, among entries of the chosen value
                const uint32_t rk = row_key(rowidx[p]);
                act = (rk & rm) == pr;
                dig = key_digit<VD>(d, vk, rk);
              }
            }
          }
          hist_add(s_hist, act, dig);
        }
      }
      __syncthreads();
      if (t < kWave) {
        // lane l owns buckets 255 - 4l ... 252 - 4l, scanned from the top
        int h[4], sum = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
          h[q] = s_hist[255 - 4 * t - q];
          sum += h[q];
        }
        const int incl = wave_incl_add(sum);
        if (d == 0 && t == kWave - 1) s_sel[3] = incl;
        int acc = incl - sum;
        if (acc < need && need <= incl) {
#pragma unroll
          for (int q = 0; q < 4; q++) {
            if (acc + h[q] >= need) {
              s_sel[0] = 255 - 4 * t - q;
              s_sel[1] = need - acc;
              s_sel[2] = h[q] == need - acc ? 1 : 0;
              break;
            }
            acc += h[q];
          }
        }
      }
      __syncthreads();
      if (d == 0) {
        const int ncand = s_sel[3];
        if (k < 0 || (int64_t)ncand <= k) {  // every candidate is kept
          kept = ncand;
          pv = 0;
          pr = 0;
          __syncthreads();
          break;
        }
        if (k == 0) {
          kept = 0;
          pv = ~0ull;
          pr = ~0u;
          __syncthreads();
          break;
        }
      }
      // 0 < k < candidates: the scan found the bucket of the k-th largest key
      const int dig = s_sel[0], rest = s_sel[1], done = s_sel[2];
      above += need - rest;
      need = rest;
      last = s_hist[dig];
      if (d < VD)
        pv |= (uint64_t)dig << (8 * (VD - 1 - d));
      else
        pr |= (uint32_t)dig << (8 * (3 - (d - VD)));
      __syncthreads();  // s_hist and s_sel are rewritten by the next digit or column
      if (done) break;
    }
    if (t == 0) {
      // selection: every key with the chosen prefix is kept; `above` outrank it, `last` share it
      if (kept < 0) {
        const int64_t all = (int64_t)above + last;
        kept = (int)(all < k ? all : k);
      }
      cnt[j] = kept;
      cutv[j] = pv;
      cutr[j] = pr;
    }
  }
}

// Compacts the kept entries of every column, in input order, to
// out_colptr[j] ... out_colptr[j + 1].  A column that holds more keys at the
// cut than its count (a row twice) writes only its count and flags status.
template <typename VT>
__global__ __launch_bounds__(kPrThreads) void k_prune_fill(
    const int64_t *__restrict__ colptr, const int32_t *__restrict__ rowidx, const VT *__restrict__ vals,
    int64_t ncols, int64_t nnz, double thr, const uint64_t *__restrict__ cutv, const uint32_t *__restrict__ cutr,
    const int64_t *__restrict__ out_colptr, int32_t *__restrict__ out_rowidx, VT *__restrict__ out_vals,
    int32_t *status) {
  __shared__ int s_cnt[kFillUnroll][kPrWaves];
  __shared__ int s_any[2][kPrWaves];
  const int t = threadIdx.x, w = t / kWave;
  int par = 0;
  for (int64_t j = blockIdx.x; j < ncols; j += gridDim.x) {
    int64_t b = colptr[j], e = colptr[j + 1];
    if (b < 0 || e < b || e > nnz) b = e = 0;  // flagged by the select kernel
    const int64_t o = out_colptr[j], lim = out_colptr[j + 1];
    const uint64_t cv = cutv[j];
    const uint32_t cr = cutr[j];
    int64_t run = 0;
    // kFillUnroll coalesced slots per thread per step (entry c0 + q * 256 + t
    // in slot q); an entry's place in input order is the kept count of the
    // earlier slots, then of earlier waves in its slot, then of lower lanes,
    // so one exchange of per-wave counts orders the whole step.  The row is
    // read only for an entry that is kept or ties the cut's value.
    for (int64_t c0 = b; c0 < e; c0 += kFillUnroll * kPrThreads) {
      VT v[kFillUnroll];
#pragma unroll
      for (int q = 0; q < kFillUnroll; q++) {
        const int64_t p = c0 + q * kPrThreads + t;
        v[q] = p < e ? vals[p] : VT(0);
      }
      uint32_t keep = 0;
#pragma unroll
      for (int q = 0; q < kFillUnroll; q++) {
        const int64_t p = c0 + q * kPrThreads + t;
        if (p < e && candidate(v[q], thr)) {
          const uint64_t vk = order_key(v[q]);
          if (vk > cv || (vk == cv && row_key(rowidx[p]) >= cr)) keep |= 1u << q;
        }
      }
      // a step in which no wave keeps an entry (the common case: k is
      // small against the column) only exchanges one flag per wave, through
      // two alternating flag sets (a set is rewritten two steps later, after
      // every wave has passed the barrier between)
      const bool wkeep = __ballot(keep != 0u) != 0ull;
      int *any_w = s_any[par];
      par ^= 1;
      if (lane() == 0) any_w[w] = wkeep ? 1 : 0;
      __syncthreads();
      bool any = false;
#pragma unroll
      for (int z = 0; z < kPrWaves; z++) any |= any_w[z] != 0;
      if (!any) continue;
      int below[kFillUnroll];
#pragma unroll
      for (int q = 0; q < kFillUnroll; q++) {
        const uint64_t m = __ballot((keep >> q) & 1u);
        below[q] = mbcnt(m);
        if (lane() == 0) s_cnt[q][w] = __popcll(m);
      }
      __syncthreads();
      int64_t base = o + run;
#pragma unroll
      for (int q = 0; q < kFillUnroll; q++) {
        int before = 0, tot = 0;
#pragma unroll
        for (int z = 0; z < kPrWaves; z++) {
          const int c = s_cnt[q][z];
          before += z < w ? c : 0;
          tot += c;
        }
        if ((keep >> q) & 1u) {
          const int64_t pos = base + before + below[q];
          if (pos < lim) {
            out_rowidx[pos] = rowidx[c0 + q * kPrThreads + t];
            out_vals[pos] = v[q];
          }
        }
        base += tot;
      }
      run = base - o;
      __syncthreads();  // s_cnt is written again by the next step
    }
    if (t == 0 && o + run != lim) flag_error(status, kPrDupRows);
  }
}

template <typename VT>
int prune_typed(const spgemm_csc *C, double thr, int64_t k, int64_t *out_colptr, int32_t *out_rowidx,
                void *out_values, const WsLayout &L, char *ws, hipStream_t st) {
  WsHeader *hdr = (WsHeader *)ws;
  int rc = launch_init_header(hdr, (uint64_t)0, st);
  if (rc) return rc;
  const int64_t n = C->ncols;
  int64_t *cnt = (int64_t *)(ws + L.pr_cnt);
  uint64_t *cutv = (uint64_t *)(ws + L.pr_cutv);
  uint32_t *cutr = (uint32_t *)(ws + L.pr_cutr);
  const unsigned grid = (unsigned)(n < kPrMaxGrid ? n : kPrMaxGrid);
  if (n > 0) {
    ProfScope prof("prune_select", st);
    hipLaunchKernelGGL(k_prune_select<VT>, dim3(grid), dim3(kPrThreads), 0, st, C->colptr, C->rowidx,
                       (const VT *)C->values, n, thr, C->nnz, k, cnt, cutv, cutr, &hdr->status);
    LAUNCHCHK();
  }
  rc = launch_colptr_scan(cnt, n, out_colptr, (int64_t *)(ws + L.scan), st);
  if (rc || n == 0) return rc;
  ProfScope prof("prune_fill", st);
  hipLaunchKernelGGL(k_prune_fill<VT>, dim3(grid), dim3(kPrThreads), 0, st, C->colptr, C->rowidx,
                     (const VT *)C->values, n, C->nnz, thr, (const uint64_t *)cutv, (const uint32_t *)cutr,
                     (const int64_t *)out_colptr, out_rowidx, (VT *)out_values, &hdr->status);
  LAUNCHCHK();
  return SPGEMM_OK;
}

}  // namespace
}  // namespace spg

using namespace spg;

extern "C" {

int spgemm_prune_topk(const spgemm_csc *C, double threshold, int64_t k, int64_t *out_colptr, int32_t *out_rowidx,
                      void *out_values, int64_t out_cap, void *ws, size_t ws_bytes, void *stream) {
  int st = check_csc(C, true);
  if (st) return st;
  if (!out_colptr || out_cap < 0) return SPGEMM_E_INVAL;
  // the output never holds more than min(nnz, k * ncols) entries
  int64_t bound = C->nnz;
  if (k >= 0 && (C->ncols == 0 || k <= bound / C->ncols) && k * C->ncols < bound) bound = k * C->ncols;
  if (out_cap < bound) return SPGEMM_E_INVAL;
  if (bound > 0 && (!out_rowidx || !out_values)) return SPGEMM_E_INVAL;
  WsLayout L;
  st = ws_layout(SPGEMM_OP_PRUNE, C, nullptr, 0, 0, 1, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if (C->dtype == SPGEMM_F32)
    return prune_typed<float>(C, threshold, k, out_colptr, out_rowidx, out_values, L, (char *)ws, s);
  return prune_typed<double>(C, threshold, k, out_colptr, out_rowidx, out_values, L, (char *)ws, s);
}

}  // extern "C"
