// Row-sorted output columns.  The paper keeps the final output of its
// column-wise merge (Merge-Fiber) sorted within each column (Sec. IV-D),
// while the sort-free hash kernels of this library write rows in table
// order; this pass turns any such output into row-sorted columns, so a
// caller that needs sorted columns pays for the ordering once, after the
// product (or after the merge), instead of inside every accumulation.
//
// Each column is sorted by row, values moving with their rows, from the
// input arrays into separate output arrays (the column pointers stay the
// same).  Rows must be unique within a column, as in every output of the
// library.  Columns are binned by length:
//   up to 64 entries  : one wave, a bitonic network across the lanes;
//   up to 4096        : one workgroup, a bitonic network in LDS;
//   longer            : one workgroup of 1024 threads, row windows of
//                       2^19 rows: the window's rows are marked in an LDS
//                       bitmap, a prefix count over the bitmap words gives
//                       every row its rank, and each entry is written
//                       straight to its sorted position (no data movement
//                       between passes; a window with no entry is skipped).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "hip_host.hpp"
#include "internal.hpp"
#include "profile.hpp"

namespace spg {
namespace {

constexpr int kSortWaveLen = 64;
constexpr int kSortBlockLen = 4096;
constexpr int kSortBlockThreads = 256;
constexpr int kSortHeavyThreads = 1024;
constexpr int kSortWinShift = 19;
constexpr int64_t kSortWinRows = int64_t(1) << kSortWinShift;
constexpr int kSortWinWords = (int)(kSortWinRows / 32);
constexpr int kSortDupCode = 11;  // status code: a row twice in one column, or a row outside [0, m)

// Column lists per length class: lists[c * ncols + i], counts in the
// header's first three bin counters.
// Columns formed in row order by expand-sort-compress (skip_flops given) are
// left out.
__global__ __launch_bounds__(256) void k_sort_bin(const int64_t *cp, int64_t n, int32_t *lists, WsHeader *hdr,
                                                  const int64_t *skip_flops, double skip_cf) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int cls = -1;
  if (j < n) {
    const int64_t len = cp[j + 1] - cp[j];
    cls = len <= 0 ? -1 : (len <= kSortWaveLen ? 0 : (len <= kSortBlockLen ? 1 : 2));
    if (skip_flops && esc_class(skip_flops[j], len, skip_cf) >= 0) cls = -1;
  }
  for (int c = 0; c < 3; c++) {
    const uint64_t mask = __ballot(cls == c);
    if (!mask) continue;
    int base = 0;
    if (lane() == 0) base = atomicAdd(&hdr->bin_count[c], __popcll(mask));
    base = readlane(base, 0);
    if (cls == c) lists[(int64_t)c * n + base + mbcnt(mask)] = (int32_t)j;
  }
}

template <class VT>
__device__ __forceinline__ VT shfl_xor_v(VT v, int m) {
  return __shfl_xor(v, m, kWave);
}

template <class VT>
__global__ __launch_bounds__(256) void k_sort_wave(const int64_t *cp, const int32_t *ri, const VT *v, int64_t m,
                                                   const int32_t *list, const int32_t *count_p, int32_t *ro, VT *vo,
                                                   int32_t *status) {
  const int count = *count_p;
  const int w = threadIdx.x / kWave, l = lane();
  for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < count; i += (int64_t)gridDim.x * 4) {
    const int64_t j = list[i];
    const int64_t b = cp[j];
    const int len = (int)(cp[j + 1] - b);
    int32_t key = INT32_MAX;  // padding sorts last (rows are below INT32_MAX)
    VT val = VT(0);
    if (l < len) {
      key = ri[b + l];
      val = v[b + l];
    }
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
      for (int s = k >> 1; s > 0; s >>= 1) {
        const int32_t ok = __shfl_xor(key, s, kWave);
        const VT ov = shfl_xor_v(val, s);
        const bool up = (l & k) == 0;     // this block of k lanes sorts ascending
        const bool low = (l & s) == 0;    // the lower lane of the pair keeps the smaller key when ascending
        if (low == up ? ok < key : ok > key) {
          key = ok;
          val = ov;
        }
      }
    }
    if (l < len) {
      ro[b + l] = key;
      vo[b + l] = val;
    }
    // sorted: a repeated row sits next to its twin
    const int32_t nxt = __shfl_down(key, 1, kWave);
    if (__ballot(l < len && ((l + 1 < len && nxt == key) || key < 0 || (int64_t)key >= m)) && l == 0)
      flag_error(status, kSortDupCode);
  }
}

template <class VT>
__global__ __launch_bounds__(kSortBlockThreads) void k_sort_block(const int64_t *cp, const int32_t *ri, const VT *v,
                                                                  int64_t m, const int32_t *list,
                                                                  const int32_t *count_p, int32_t *ro, VT *vo,
                                                                  int32_t *status) {
  __shared__ int32_t s_k[kSortBlockLen];
  __shared__ VT s_v[kSortBlockLen];
  const int count = *count_p;
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
    const int64_t j = list[i];
    const int64_t b = cp[j];
    const int len = (int)(cp[j + 1] - b);
    int N = 128;
    while (N < len) N <<= 1;
    for (int t = threadIdx.x; t < N; t += kSortBlockThreads) {
      s_k[t] = t < len ? ri[b + t] : INT32_MAX;
      s_v[t] = t < len ? v[b + t] : VT(0);
    }
    __syncthreads();
    for (int k = 2; k <= N; k <<= 1) {
      for (int s = k >> 1; s > 0; s >>= 1) {
        for (int t = threadIdx.x; t < N / 2; t += kSortBlockThreads) {
          const int a = ((t & ~(s - 1)) << 1) | (t & (s - 1));  // lower element of pair t at distance s
          const int c = a + s;
          const bool up = (a & k) == 0;
          const int32_t ka = s_k[a], kc = s_k[c];
          if ((ka > kc) == up) {
            const VT va = s_v[a];
            s_k[a] = kc;
            s_k[c] = ka;
            s_v[a] = s_v[c];
            s_v[c] = va;
          }
        }
        __syncthreads();
      }
    }
    bool bad = false;
    for (int t = threadIdx.x; t < len; t += kSortBlockThreads) {
      const int32_t k = s_k[t];
      ro[b + t] = k;
      vo[b + t] = s_v[t];
      bad |= (t + 1 < len && s_k[t + 1] == k) || k < 0 || (int64_t)k >= m;  // a repeated row sits next to its twin
    }
    if (__ballot(bad) && lane() == 0) flag_error(status, kSortDupCode);
    __syncthreads();  // the next column overwrites s_k, s_v
  }
}

template <class VT>
__global__ __launch_bounds__(kSortHeavyThreads) void k_sort_heavy(const int64_t *cp, const int32_t *ri, const VT *v,
                                                                  int64_t m, const int32_t *list,
                                                                  const int32_t *count_p, int32_t *ro, VT *vo,
                                                                  int32_t *status) {
  constexpr int NW = kSortHeavyThreads / kWave;
  constexpr int kWordsPerThread = kSortWinWords / kSortHeavyThreads;
  static_assert(kSortWinWords % kSortHeavyThreads == 0, "bitmap words split evenly over threads");
  __shared__ uint32_t s_bits[kSortWinWords];
  __shared__ int32_t s_pref[kSortWinWords];  // entries of the window in words before this one
  __shared__ int s_wtot[NW];
  __shared__ int s_lo, s_hi;
  const int w = threadIdx.x / kWave, l = lane();
  const int count = *count_p;
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
    const int64_t j = list[i];
    const int64_t b = cp[j], e = cp[j + 1];
    // the column's row range: windows that hold no entry are skipped
    int lo = INT32_MAX, hi = -1;
    for (int64_t p = b + threadIdx.x; p < e; p += kSortHeavyThreads) {
      const int32_t r = ri[p];
      lo = min(lo, r);
      hi = max(hi, r);
    }
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, kWave));
      hi = max(hi, __shfl_xor(hi, o, kWave));
    }
    if (threadIdx.x == 0) {
      s_lo = INT32_MAX;
      s_hi = -1;
    }
    __syncthreads();
    if (l == 0) {
      atomicMin(&s_lo, lo);
      atomicMax(&s_hi, hi);
    }
    __syncthreads();
    const int64_t rlo = max((int64_t)s_lo, (int64_t)0), rhi = min((int64_t)s_hi, m - 1);
    int64_t done = 0;
    for (int64_t w0 = (rlo >> kSortWinShift) << kSortWinShift; w0 <= rhi; w0 += kSortWinRows) {
      for (int q = threadIdx.x; q < kSortWinWords; q += kSortHeavyThreads) s_bits[q] = 0u;
      __syncthreads();
      for (int64_t p = b + threadIdx.x; p < e; p += kSortHeavyThreads) {
        const int64_t r = (int64_t)ri[p] - w0;
        if (r >= 0 && r < kSortWinRows) atomicOr(&s_bits[r >> 5], 1u << (r & 31));
      }
      __syncthreads();
      // exclusive prefix of the word counts: kWordsPerThread consecutive
      // words per thread, a scan over the threads
      const int q0 = threadIdx.x * kWordsPerThread;
      int c = 0;
#pragma unroll 8
      for (int q = 0; q < kWordsPerThread; q++) c += __popc(s_bits[q0 + q]);
      const int incl = wave_incl_add(c);
      if (l == kWave - 1) s_wtot[w] = incl;
      __syncthreads();
      int before = 0, tot = 0;
#pragma unroll
      for (int z = 0; z < NW; z++) {
        const int t = s_wtot[z];
        if (z < w) before += t;
        tot += t;
      }
      int run = before + incl - c;
#pragma unroll 8
      for (int q = 0; q < kWordsPerThread; q++) {
        s_pref[q0 + q] = run;
        run += __popc(s_bits[q0 + q]);
      }
      __syncthreads();
      for (int64_t p = b + threadIdx.x; p < e; p += kSortHeavyThreads) {
        const int32_t row = ri[p];
        const int64_t r = (int64_t)row - w0;
        if (r >= 0 && r < kSortWinRows) {
          const int q = (int)(r >> 5);
          const int64_t dst = b + done + s_pref[q] + __popc(s_bits[q] & ((1u << (r & 31)) - 1u));
          if (dst < e) {
            ro[dst] = row;
            vo[dst] = v[p];
          }
        }
      }
      done += tot;
      __syncthreads();  // the next window clears s_bits, s_pref, s_wtot
    }
    if (threadIdx.x == 0 && done != e - b) flag_error(status, kSortDupCode);
  }
}

template <class VT>
int sort_typed(const spgemm_csc *C, int32_t *ro, void *vo, int32_t *lists, WsHeader *hdr,
               const int64_t *skip_flops, double skip_cf, hipStream_t st) {
  const int64_t n = C->ncols;
  ProfScope prof("sort_columns", st);
  hipLaunchKernelGGL(k_sort_bin, dim3(grid_of(n, 256)), dim3(256), 0, st, C->colptr, n, lists, hdr, skip_flops,
                     skip_cf);
  LAUNCHCHK();
  const VT *v = (const VT *)C->values;
  const int cus = device_cus();
  hipLaunchKernelGGL(k_sort_wave<VT>, dim3(8 * cus), dim3(256), 0, st, C->colptr, C->rowidx, v, C->nrows, lists,
                     (const int32_t *)&hdr->bin_count[0], ro, (VT *)vo, &hdr->status);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_sort_block<VT>, dim3(4 * cus), dim3(kSortBlockThreads), 0, st, C->colptr, C->rowidx, v,
                     C->nrows, lists + n, (const int32_t *)&hdr->bin_count[1], ro, (VT *)vo, &hdr->status);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_sort_heavy<VT>, dim3(cus), dim3(kSortHeavyThreads), 0, st, C->colptr, C->rowidx, v, C->nrows,
                     lists + 2 * n, (const int32_t *)&hdr->bin_count[2], ro, (VT *)vo, &hdr->status);
  LAUNCHCHK();
  return SPGEMM_OK;
}

}  // namespace

int sort_column_lists(const spgemm_csc *C, int32_t *ro, void *vo, int32_t *lists, WsHeader *hdr,
                      const int64_t *skip_flops, double skip_cf, hipStream_t st) {
  if (C->dtype == SPGEMM_F32) return sort_typed<float>(C, ro, vo, lists, hdr, skip_flops, skip_cf, st);
  return sort_typed<double>(C, ro, vo, lists, hdr, skip_flops, skip_cf, st);
}

}  // namespace spg

using namespace spg;

extern "C" {

int spgemm_sort_columns(const spgemm_csc *C, int32_t *rowidx_out, void *values_out, void *ws, size_t ws_bytes,
                        void *stream) {
  int st = check_csc(C, true);
  if (st) return st;
  if (C->ncols > INT32_MAX) return SPGEMM_E_OVERFLOW;
  if (C->nnz > 0 && (!rowidx_out || !values_out)) return SPGEMM_E_INVAL;
  if (C->nnz > 0 && ((const void *)rowidx_out == (const void *)C->rowidx || values_out == C->values))
    return SPGEMM_E_INVAL;  // out of place only
  WsLayout L;
  st = ws_layout(SPGEMM_OP_SORT, C, nullptr, 0, 0, 1, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  if (C->ncols == 0) return launch_init_header((WsHeader *)ws, (uint64_t)0, (hipStream_t)stream);
  hipStream_t s = (hipStream_t)stream;
  st = launch_init_header((WsHeader *)ws, (uint64_t)0, s);
  if (st) return st;
  return sort_column_lists(C, rowidx_out, values_out, (int32_t *)((char *)ws + L.bins), (WsHeader *)ws, nullptr, 0.0,
                           s);
}

}  // extern "C"
