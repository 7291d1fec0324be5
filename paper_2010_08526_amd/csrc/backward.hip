// Kernels for the gradient of C = A*B with respect to the stored values of A
// and B, for a loss defined on the pattern of C (not part of the paper; the
// product itself follows Gustavson's column formula, Sec. II-C).
//
//   dB(k,j) = sum over i in A(:,k) of A(i,k) * dC(i,j),   (k,j) in P(B)
//   dA(i,k) = sum over j in B(k,:) of dC(i,j) * B(k,j),   (i,k) in P(A)
//
// Both are masked products out = (X^T Y) restricted to a pattern M:
//   dB  = masked_xty(X = A,   Y = dC,   M = P(B))
//   dA^T = masked_xty(X = B^T, Y = dC^T, M = P(A^T))
// Every dC(i,j) they need lies in P(C), so no term is lost by the mask.
// For each output column j the kernel loads Y(:,j) into an LDS hash table
// (row -> value) and forms one dot product per requested entry (k,j) of M
// against X(:,k); the work equals the forward flops plus nnz(Y).
//
// The transposes are sort-free: a row histogram, a scan, and a scatter
// with atomic cursors (entry order inside each output column is arbitrary).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "device.hpp"
#include "hip_host.hpp"
#include "internal.hpp"
#include "lds_hash.hpp"
#include "profile.hpp"

namespace spg {

// ============================================================================
// Transpose
// ============================================================================
__global__ void k_tr_zero(unsigned long long *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_tr_count(const int32_t *ri, int64_t nnz, int64_t m, unsigned long long *cnt, int32_t *status) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = ri[p];
    if ((uint32_t)r < (uint32_t)m)
      atomicAdd(&cnt[r], 1ull);
    else
      flag_error(status, 3);
  }
}

__global__ void k_tr_cursor(const int64_t *t_colptr, int64_t m, unsigned long long *cursor) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    cursor[i] = (unsigned long long)t_colptr[i];
}

// One wavefront per source column (grid-stride).
template <class VT>
__global__ __launch_bounds__(256) void k_tr_scatter(const int64_t *cp, const int32_t *ri, const VT *v, int64_t ncols,
                                                    int64_t m, unsigned long long *cursor, int32_t *t_ri, VT *t_v,
                                                    int64_t *perm) {
  const int l = lane();
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t j = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave; j < ncols; j += nwaves) {
    for (int64_t p = cp[j] + l; p < cp[j + 1]; p += kWave) {
      const int32_t r = ri[p];
      if ((uint32_t)r >= (uint32_t)m) continue;  // counted as an error by k_tr_count
      const unsigned long long pos = atomicAdd(&cursor[r], 1ull);
      t_ri[pos] = (int32_t)j;
      if (t_v) t_v[pos] = v[p];
      if (perm) perm[pos] = p;
    }
  }
}

// ============================================================================
// Permute
// ============================================================================
template <class T>
__global__ void k_permute(const T *src, const int64_t *perm, int64_t n, T *dst, int scatter) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = perm[i];
    if ((uint64_t)q >= (uint64_t)n) continue;
    if (scatter)
      dst[q] = src[i];
    else
      dst[i] = src[q];
  }
}

// ============================================================================
// Masked X^T Y
// ============================================================================
template <class VT>
struct MxtyArgs {
  const int64_t *Xcp;
  const int32_t *Xri;
  const VT *Xv;
  const int64_t *Ycp;
  const int32_t *Yri;
  const VT *Yv;
  const int64_t *Mcp;
  const int32_t *Mri;
  VT *out;
  int64_t m, kdim, nnzX;
};

// Binning by nnz(Y(:,j)) with the numeric bins' capacities; columns of M
// with no entry need no work.
constexpr int kMxColsPerWave = 16;
__global__ __launch_bounds__(256) void k_mxty_bin(const int64_t *Ycp, const int64_t *Mcp, int64_t ncol, int min_bin,
                                                  BinCaps caps, int32_t *bins, WsHeader *hdr) {
  __shared__ int s_cnt[kNumBins];
  __shared__ int s_base[kNumBins];
  __shared__ int s_bin[256];
  __shared__ int s_pos[256];
  const int t = threadIdx.x;
  if (t < kNumBins) s_cnt[t] = 0;
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + t;
  int bin = -1;
  if (j < ncol && Mcp[j + 1] > Mcp[j]) {
    const int64_t u = Ycp[j + 1] - Ycp[j];
    bin = kNumBins - 1;
#pragma unroll
    for (int b = kNumBins - 2; b >= 0; b--)
      if (u <= caps.cap[b]) bin = b;
    bin = max(bin, min_bin);
  }
  s_bin[t] = bin;
  s_pos[t] = bin >= 0 ? atomicAdd(&s_cnt[bin], 1) : 0;
  __syncthreads();
  if (t < kNumBins) s_base[t] = s_cnt[t] ? atomicAdd(&hdr->bin_count[t], s_cnt[t]) : 0;
  __syncthreads();
  if (bin >= 0) bins[(int64_t)bin * ncol + s_base[bin] + s_pos[t]] = (int32_t)j;
}

constexpr int kLongDot = 64;

// Scratch of one wave for the masked dot products and the fused backward:
// the segments of a chunk of 64 entries (a column of X or A each), flattened
// into rounds of 64 products.
struct FbScratch {
  int mark[kWave];
  int64_t off[kWave];   // first A entry of the lane's segment minus its exclusive prefix
  double scale[kWave];  // B(k,j) of the lane's segment (fused backward)
  double db[kWave];     // the segment's dot product, summed by LDS atomics
};
constexpr int kFbPipe = 4;  // rounds whose gathers are in flight together

// Dot products for the entries [pb, pe) of M(:,j) taken in chunks of 64
// (chunk c by the wave with c % c_stride == c_rank).  Short X columns are
// flattened into rounds of 64 products, one per lane (owners as in the
// forward traversal), and each entry's sum is gathered by LDS atomics; long
// ones are summed by the whole wave with a wave reduction.  look(row)
// returns Y(row, j).
template <class VT, class Look>
__device__ __forceinline__ void mxty_dots(const MxtyArgs<VT> &a, int64_t pb, int64_t pe, int c_rank, int c_stride,
                                          int32_t *status, FbScratch &sc, Look &&look) {
  const int l = lane();
  for (int64_t base = pb + (int64_t)c_rank * kWave; base < pe; base += (int64_t)c_stride * kWave) {
    const int64_t p = base + l;
    int64_t x0 = 0, x1 = 0;
    if (p < pe) {
      const int32_t k = a.Mri[p];
      if ((uint32_t)k >= (uint32_t)a.kdim) {
        flag_error(status, 1);
      } else {
        x0 = a.Xcp[k];
        x1 = a.Xcp[k + 1];
        if (x0 < 0 || x1 < x0 || x1 > a.nnzX) {
          flag_error(status, 5);
          x0 = x1 = 0;
        }
      }
    }
    const int len = (int)(x1 - x0);
    const bool lg = len >= kLongDot;
    const int ls = (p < pe && !lg) ? len : 0;
    const int incl = wave_incl_add(ls);
    const int excl = incl - ls;
    const int total = readlane(incl, kWave - 1);
    sc.off[l] = x0 - excl;
    sc.db[l] = 0.0;
    wave_sync();
    for (int r = 0; r * kWave < total; r += kFbPipe) {
      int own_[kFbPipe];
#pragma unroll
      for (int u = 0; u < kFbPipe; u++) {
        const int fb = (r + u) * kWave;
        own_[u] = -1;
        if (fb < total) {
          const int last = min(fb + kWave - 1, total - 1);
          const uint64_t started = __ballot(ls > 0 && excl <= fb);
          const int carry = started ? 64 - __clzll((long long)started) : 0;
          int own = carry;
          if (__ballot(ls > 0 && excl <= last) != started) {
            if (ls > 0 && excl > fb && excl < fb + kWave) sc.mark[excl - fb] = l + 1;
            wave_sync();
            const int mk = sc.mark[l];
            sc.mark[l] = 0;
            own = max(wave_incl_max(mk), carry);
            wave_sync();
          }
          if (fb + l < total) own_[u] = own - 1;
        }
      }
      int32_t row_[kFbPipe];
      VT xv_[kFbPipe];
#pragma unroll
      for (int u = 0; u < kFbPipe; u++) {
        row_[u] = -1;
        xv_[u] = VT(0);
        if (own_[u] >= 0) {
          const int64_t q = sc.off[own_[u]] + (r + u) * kWave + l;
          row_[u] = a.Xri[q];
          xv_[u] = a.Xv[q];
        }
      }
#pragma unroll
      for (int u = 0; u < kFbPipe; u++) {
        if (own_[u] >= 0) {
          const int32_t rt = opaque(row_[u]);
          if ((uint32_t)rt < (uint32_t)a.m)
            atomicAdd(&sc.db[own_[u]], (double)opaque(xv_[u]) * look(rt));
          else
            flag_error(status, 3);
        }
      }
    }
    wave_sync();
    if (p < pe && !lg) a.out[p] = (VT)sc.db[l];
    uint64_t lm = __ballot(p < pe && lg);
    while (lm) {
      const int L = __builtin_ctzll(lm);
      lm &= lm - 1;
      const int64_t lx0 = readlane64(x0, L), lx1 = readlane64(x1, L);
      double s = 0.0;
      for (int64_t q0 = lx0 + l; q0 < lx1; q0 += 4 * kWave) {
        int32_t r[4];
        VT xv[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const int64_t q = q0 + t * kWave;
          r[t] = 0;
          xv[t] = VT(0);
          if (q < lx1) {
            r[t] = a.Xri[q];
            xv[t] = a.Xv[q];
          }
        }
#pragma unroll
        for (int t = 0; t < 4; t++) {
          if (q0 + t * kWave < lx1) {
            const int32_t rt = opaque(r[t]);
            if ((uint32_t)rt < (uint32_t)a.m)
              s += (double)opaque(xv[t]) * look(rt);
            else
              flag_error(status, 3);
          }
        }
      }
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
      if (l == 0) a.out[base + L] = (VT)s;
    }
    wave_sync();  // sc is rewritten by the next chunk
  }
}

// One wavefront per column, TBL-slot table of Y(:,j) private to the wave.
template <int TBL, class VT>
__global__ __launch_bounds__(256) void k_mxty_wave(MxtyArgs<VT> a, const int32_t *list, const int32_t *count_p,
                                                   int32_t *status) {
  __shared__ int32_t s_keys[4][TBL];
  __shared__ double s_vals[4][TBL];
  __shared__ FbScratch s_fb[4];
  const int w = threadIdx.x / kWave, l = lane();
  const int count = *count_p;
  int32_t *keys = s_keys[w];
  double *vals = s_vals[w];
  s_fb[w].mark[l] = 0;
  for (int idx = blockIdx.x * 4 + w; idx < count; idx += gridDim.x * 4) {
    for (int s = l; s < TBL; s += kWave) {
      keys[s] = kEmpty;
      vals[s] = 0.0;
    }
    wave_sync();
    const int32_t j = list[idx];
    for (int64_t p = a.Ycp[j] + l; p < a.Ycp[j + 1]; p += kWave) {
      const int32_t r = a.Yri[p];
      if ((uint32_t)r < (uint32_t)a.m)
        ht_accumulate(keys, vals, TBL, r, (double)a.Yv[p]);
      else
        flag_error(status, 3);
    }
    wave_sync();
    mxty_dots(a, a.Mcp[j], a.Mcp[j + 1], 0, 1, status, s_fb[w], [&](int32_t r) { return ht_lookup(keys, vals, TBL, r); });
    wave_sync();
  }
}

// One workgroup per column, shared table.
template <int TBL, int THREADS, class VT>
__global__ __launch_bounds__(THREADS) void k_mxty_block(MxtyArgs<VT> a, const int32_t *list, const int32_t *count_p,
                                                        int32_t *status) {
  constexpr int NW = THREADS / kWave;
  __shared__ int32_t s_keys[TBL];
  __shared__ double s_vals[TBL];
  __shared__ FbScratch s_fb[NW];
  const int w = threadIdx.x / kWave;
  const int count = *count_p;
  s_fb[w].mark[lane()] = 0;
  for (int item = blockIdx.x; item < count; item += gridDim.x) {
    for (int s = threadIdx.x; s < TBL; s += THREADS) {
      s_keys[s] = kEmpty;
      s_vals[s] = 0.0;
    }
    __syncthreads();
    const int32_t j = list[item];
    for (int64_t p = a.Ycp[j] + threadIdx.x; p < a.Ycp[j + 1]; p += THREADS) {
      const int32_t r = a.Yri[p];
      if ((uint32_t)r < (uint32_t)a.m)
        ht_accumulate(s_keys, s_vals, TBL, r, (double)a.Yv[p]);
      else
        flag_error(status, 3);
    }
    __syncthreads();
    mxty_dots(a, a.Mcp[j], a.Mcp[j + 1], w, NW, status, s_fb[w], [&](int32_t r) { return ht_lookup(s_keys, s_vals, TBL, r); });
    __syncthreads();
  }
}

// Heavy columns: Y(:,j) scattered into a dense float64 column of the
// workspace (zero outside Y's rows), dots read it, then it is cleared.
template <class VT>
__global__ __launch_bounds__(256) void k_mxty_heavy_fill(MxtyArgs<VT> a, const int32_t *list, int first, int ns,
                                                         double *dense, int clear) {
  const int slot = blockIdx.y;
  if (slot >= ns) return;
  const int32_t j = list[first + slot];
  double *d = dense + (int64_t)slot * a.m;
  for (int64_t p = a.Ycp[j] + (int64_t)blockIdx.x * 256 + threadIdx.x; p < a.Ycp[j + 1];
       p += (int64_t)gridDim.x * 256) {
    const int32_t r = a.Yri[p];
    if ((uint32_t)r < (uint32_t)a.m) d[r] = clear ? 0.0 : (double)a.Yv[p];
  }
}

template <class VT>
__global__ __launch_bounds__(256) void k_mxty_heavy_dot(MxtyArgs<VT> a, const int32_t *list, int first, int ns,
                                                        const double *dense, int parts, int32_t *status) {
  __shared__ FbScratch s_fb[4];
  const int slot = blockIdx.x / parts, part = blockIdx.x % parts;
  if (slot >= ns) return;
  const int32_t j = list[first + slot];
  const double *d = dense + (int64_t)slot * a.m;
  const int w = threadIdx.x / kWave;
  s_fb[w].mark[lane()] = 0;
  mxty_dots(a, a.Mcp[j], a.Mcp[j + 1], part * 4 + w, parts * 4, status, s_fb[w], [&](int32_t r) { return d[r]; });
}

static unsigned mx_grid(int cnt, bool wave_kernel, int blocks_per_cu) {
  const unsigned full = (unsigned)(blocks_per_cu * device_cus());
  if (cnt < 0) return full;
  const unsigned need = wave_kernel ? grid_of(cnt, 4) : (unsigned)cnt;
  return std::max(1u, std::min(need, full));
}

__global__ void k_mx_flag_if_nonzero(const int32_t *count, int32_t *status, int code) {
  if (threadIdx.x == 0 && *count > 0) flag_error(status, code);
}

template <class VT>
static int mxty_typed(const spgemm_csc *X, const spgemm_csc *Y, const spgemm_csc *M, void *out, const WsLayout &L,
                      char *ws, hipStream_t st, bool sync) {
  WsHeader *hdr = (WsHeader *)ws;
  int32_t *bins = (int32_t *)(ws + L.bins);
  const int64_t n = Y->ncols;
  int rc = launch_init_header(hdr, zero_region_tag(kTagMasked, L), st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_mxty_bin, dim3(grid_of(n, 256)), dim3(256), 0, st, Y->colptr, M->colptr, n, g_min_bin_value(),
                     bin_caps(1), bins, hdr);
  LAUNCHCHK();
  WsHeader h;
  int cnt[kNumBins];
  if (sync) {
    rc = read_header(hdr, st, &h);
    if (rc) return rc;
    for (int b = 0; b < kNumBins; b++) cnt[b] = h.bin_count[b];
  } else {
    for (int b = 0; b < kNumBins; b++) cnt[b] = -1;
    memset(&h, 0, sizeof(h));
  }
  MxtyArgs<VT> a{X->colptr, X->rowidx, (const VT *)X->values, Y->colptr, Y->rowidx, (const VT *)Y->values,
                 M->colptr, M->rowidx, (VT *)out, Y->nrows, X->ncols, X->nnz};
  int32_t *status = &hdr->status;
  for (int b = 0; b < kNumBins - 1; b++) {
    if (cnt[b] == 0) continue;
    ProfScope prof("masked_xty", st);
    const int32_t *list = bins + (int64_t)b * n;
    const int32_t *cp = &hdr->bin_count[b];
    switch (b) {
      case 0: hipLaunchKernelGGL((k_mxty_wave<64, VT>), dim3(mx_grid(cnt[b], true, 8)), dim3(256), 0, st, a, list, cp, status); break;
      case 1: hipLaunchKernelGGL((k_mxty_wave<256, VT>), dim3(mx_grid(cnt[b], true, 8)), dim3(256), 0, st, a, list, cp, status); break;
      case 2: hipLaunchKernelGGL((k_mxty_wave<1024, VT>), dim3(mx_grid(cnt[b], true, 4)), dim3(256), 0, st, a, list, cp, status); break;
      case 3: hipLaunchKernelGGL((k_mxty_block<4096, 256, VT>), dim3(mx_grid(cnt[b], false, 4)), dim3(256), 0, st, a, list, cp, status); break;
      default: hipLaunchKernelGGL((k_mxty_block<10240, 1024, VT>), dim3(mx_grid(cnt[b], false, 1)), dim3(1024), 0, st, a, list, cp, status); break;
    }
    LAUNCHCHK();
  }
  const int heavy = cnt[kNumBins - 1];
  if (heavy < 0) {  // no host count: heavy columns cannot be scheduled here
    hipLaunchKernelGGL(k_mx_flag_if_nonzero, dim3(1), dim3(64), 0, st, &hdr->bin_count[kNumBins - 1], status, 7);
    LAUNCHCHK();
    return SPGEMM_OK;
  }
  if (heavy > 0) {
    if (L.slots <= 0) return SPGEMM_E_INVAL;
    double *dense = (double *)(ws + L.heavy_vals);
    const uint64_t tag = zero_region_tag(kTagMasked, L);
    if (h.clean_tag != tag) {
      hipLaunchKernelGGL(k_tr_zero, dim3(4 * device_cus()), dim3(256), 0, st, (unsigned long long *)dense,
                         L.slots * L.m);
      LAUNCHCHK();
      rc = launch_set_tag(hdr, tag, st);
      if (rc) return rc;
    }
    const int32_t *list = bins + (int64_t)(kNumBins - 1) * n;
    for (int first = 0; first < heavy; first += (int)L.slots) {
      const int ns = (int)std::min<int64_t>(L.slots, heavy - first);
      hipLaunchKernelGGL(k_mxty_heavy_fill<VT>, dim3(64, ns), dim3(256), 0, st, a, list, first, ns, dense, 0);
      LAUNCHCHK();
      const int parts = (int)std::max<int64_t>(1, std::min<int64_t>(64, (4 * device_cus() + ns - 1) / ns));
      hipLaunchKernelGGL(k_mxty_heavy_dot<VT>, dim3(ns * parts), dim3(256), 0, st, a, list, first, ns, dense, parts,
                         status);
      LAUNCHCHK();
      hipLaunchKernelGGL(k_mxty_heavy_fill<VT>, dim3(64, ns), dim3(256), 0, st, a, list, first, ns, dense, 1);
      LAUNCHCHK();
    }
  }
  return SPGEMM_OK;
}

// ============================================================================
// Fused gradient (graph-capturable): for each output column j, dC(:,j) goes
// into an LDS hash table; every entry (k,j) of B then gives
//   dB(k,j)  = sum over i in A(:,k) of A(i,k) * dC(i,j)     (a dot product)
//   dA(i,k) += B(k,j) * dC(i,j)  for i in A(:,k)           (float64 atomics)
// in one traversal of the product's terms, with no transpose.  dA is
// accumulated in a float64 workspace array and rounded once.
// ============================================================================
template <class VT>
struct FbArgs {
  const int64_t *Acp;
  const int32_t *Ari;
  const VT *Av;
  const int64_t *Bcp;
  const int32_t *Bri;
  const VT *Bv;
  const int64_t *Ccp;
  const int32_t *Cri;
  const VT *dC;
  VT *dB;
  double *dA;
  int64_t m, kdim, nnzA;
};


// Entries (k,j) of B(:,j), 64 per chunk (chunk c by the wave with
// c % c_stride == c_rank).  Segments A(:,k) shorter than kLongDot are
// flattened into rounds of 64 products, one per lane (owner of each product
// from a ballot, or an LDS marker and a max-scan when a segment starts inside
// the round), so a column with few entries of B still fills the wave; each
// product adds to dA(i,k) (float64 global atomics) and to its segment's
// dB(k,j) (float64 LDS atomics).  Long segments are walked by the whole wave
// with a wave reduction.  look(row) returns dC(row, j).
template <class VT, class Look>
__device__ __forceinline__ void fbwd_column(const FbArgs<VT> &a, int64_t j, int c_rank, int c_stride, int32_t *status,
                                            FbScratch &sc, Look &&look) {
  const int l = lane();
  const int64_t pb = a.Bcp[j], pe = a.Bcp[j + 1];
  for (int64_t base = pb + (int64_t)c_rank * kWave; base < pe; base += (int64_t)c_stride * kWave) {
    const int64_t p = base + l;
    int64_t x0 = 0, x1 = 0;
    double bkj = 0.0;
    if (p < pe) {
      const int32_t k = a.Bri[p];
      if ((uint32_t)k >= (uint32_t)a.kdim) {
        flag_error(status, 1);
      } else {
        x0 = a.Acp[k];
        x1 = a.Acp[k + 1];
        bkj = (double)a.Bv[p];
        if (x0 < 0 || x1 < x0 || x1 > a.nnzA) {
          flag_error(status, 5);
          x0 = x1 = 0;
        }
      }
    }
    const int len = (int)(x1 - x0);
    const bool lg = len >= kLongDot;
    const int ls = (p < pe && !lg) ? len : 0;
    const int incl = wave_incl_add(ls);
    const int excl = incl - ls;
    const int total = readlane(incl, kWave - 1);
    sc.off[l] = x0 - excl;
    sc.scale[l] = bkj;
    sc.db[l] = 0.0;
    wave_sync();
    for (int r = 0; r * kWave < total; r += kFbPipe) {
      int own_[kFbPipe];
#pragma unroll
      for (int u = 0; u < kFbPipe; u++) {
        const int fb = (r + u) * kWave;
        own_[u] = -1;
        if (fb < total) {
          const int last = min(fb + kWave - 1, total - 1);
          const uint64_t started = __ballot(ls > 0 && excl <= fb);
          const int carry = started ? 64 - __clzll((long long)started) : 0;
          int own = carry;
          if (__ballot(ls > 0 && excl <= last) != started) {
            if (ls > 0 && excl > fb && excl < fb + kWave) sc.mark[excl - fb] = l + 1;
            wave_sync();
            const int mk = sc.mark[l];
            sc.mark[l] = 0;
            own = max(wave_incl_max(mk), carry);
            wave_sync();
          }
          if (fb + l < total) own_[u] = own - 1;
        }
      }
      int64_t q_[kFbPipe];
      int32_t row_[kFbPipe];
      VT av_[kFbPipe];
#pragma unroll
      for (int u = 0; u < kFbPipe; u++) {
        q_[u] = sc.off[max(own_[u], 0)] + (r + u) * kWave + l;
        row_[u] = -1;
        av_[u] = VT(0);
        if (own_[u] >= 0) {
          row_[u] = a.Ari[q_[u]];
          av_[u] = a.Av[q_[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < kFbPipe; u++) {
        if (own_[u] >= 0) {
          const int32_t rt = opaque(row_[u]);
          if ((uint32_t)rt < (uint32_t)a.m) {
            const double g = look(rt);
            atomicAdd(&a.dA[q_[u]], sc.scale[own_[u]] * g);
            atomicAdd(&sc.db[own_[u]], (double)opaque(av_[u]) * g);
          } else {
            flag_error(status, 3);
          }
        }
      }
    }
    wave_sync();
    if (p < pe && !lg) a.dB[p] = (VT)sc.db[l];
    uint64_t lm = __ballot(p < pe && lg);
    while (lm) {
      const int L = __builtin_ctzll(lm);
      lm &= lm - 1;
      const int64_t lx0 = readlane64(x0, L), lx1 = readlane64(x1, L);
      const double lb = readlane_f64(bkj, L);
      double s = 0.0;
      for (int64_t q = lx0 + l; q < lx1; q += kWave) {
        const int32_t r = a.Ari[q];
        if ((uint32_t)r < (uint32_t)a.m) {
          const double g = look(r);
          s += (double)a.Av[q] * g;
          atomicAdd(&a.dA[q], lb * g);
        } else {
          flag_error(status, 3);
        }
      }
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
      if (l == 0) a.dB[base + L] = (VT)s;
    }
    wave_sync();  // sc is rewritten by the next chunk
  }
}

template <int TBL, class VT>
__global__ __launch_bounds__(256) void k_fbwd_wave(FbArgs<VT> a, const int32_t *list, const int32_t *count_p,
                                                   int32_t *status) {
  __shared__ int32_t s_keys[4][TBL];
  __shared__ double s_vals[4][TBL];
  __shared__ FbScratch s_fb[4];
  const int w = threadIdx.x / kWave, l = lane();
  const int count = *count_p;
  int32_t *keys = s_keys[w];
  double *vals = s_vals[w];
  s_fb[w].mark[l] = 0;
  for (int idx = blockIdx.x * 4 + w; idx < count; idx += gridDim.x * 4) {
    for (int s = l; s < TBL; s += kWave) {
      keys[s] = kEmpty;
      vals[s] = 0.0;
    }
    wave_sync();
    const int32_t j = list[idx];
    for (int64_t p = a.Ccp[j] + l; p < a.Ccp[j + 1]; p += kWave) {
      const int32_t r = a.Cri[p];
      if ((uint32_t)r < (uint32_t)a.m)
        ht_accumulate(keys, vals, TBL, r, (double)a.dC[p]);
      else
        flag_error(status, 3);
    }
    wave_sync();
    fbwd_column(a, j, 0, 1, status, s_fb[w], [&](int32_t r) { return ht_lookup(keys, vals, TBL, r); });
    wave_sync();
  }
}

template <int TBL, int THREADS, class VT>
__global__ __launch_bounds__(THREADS) void k_fbwd_block(FbArgs<VT> a, const int32_t *list, const int32_t *count_p,
                                                        int32_t *status) {
  constexpr int NW = THREADS / kWave;
  __shared__ int32_t s_keys[TBL];
  __shared__ double s_vals[TBL];
  __shared__ FbScratch s_fb[NW];
  const int w = threadIdx.x / kWave;
  const int count = *count_p;
  s_fb[w].mark[lane()] = 0;
  for (int item = blockIdx.x; item < count; item += gridDim.x) {
    for (int s = threadIdx.x; s < TBL; s += THREADS) {
      s_keys[s] = kEmpty;
      s_vals[s] = 0.0;
    }
    __syncthreads();
    const int32_t j = list[item];
    for (int64_t p = a.Ccp[j] + threadIdx.x; p < a.Ccp[j + 1]; p += THREADS) {
      const int32_t r = a.Cri[p];
      if ((uint32_t)r < (uint32_t)a.m)
        ht_accumulate(s_keys, s_vals, TBL, r, (double)a.dC[p]);
      else
        flag_error(status, 3);
    }
    __syncthreads();
    fbwd_column(a, j, w, NW, status, s_fb[w], [&](int32_t r) { return ht_lookup(s_keys, s_vals, TBL, r); });
    __syncthreads();
  }
}

__global__ void k_zero_f64(double *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

template <class VT>
__global__ void k_round(const double *src, int64_t n, VT *dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (VT)src[i];
}

template <class VT>
static int fbwd_typed(const spgemm_csc *A, const spgemm_csc *B, const spgemm_csc *C, const void *dC, void *dA,
                      void *dB, const WsLayout &L, char *ws, hipStream_t st) {
  WsHeader *hdr = (WsHeader *)ws;
  int32_t *bins = (int32_t *)(ws + L.bins);
  double *acc = (double *)(ws + L.heavy_vals);
  const int64_t n = C->ncols;
  int rc = launch_init_header(hdr, (uint64_t)0, st);
  if (rc) return rc;
  const unsigned gz = (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_of(A->nnz, 256), 8 * device_cus()));
  hipLaunchKernelGGL(k_zero_f64, dim3(gz), dim3(256), 0, st, acc, A->nnz);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_mxty_bin, dim3(grid_of(n, 256)), dim3(256), 0, st, C->colptr, B->colptr, n, g_min_bin_value(),
                     bin_caps(1), bins, hdr);
  LAUNCHCHK();
  FbArgs<VT> a{A->colptr, A->rowidx, (const VT *)A->values, B->colptr, B->rowidx, (const VT *)B->values,
               C->colptr, C->rowidx, (const VT *)dC, (VT *)dB, acc, C->nrows, A->ncols, A->nnz};
  int32_t *status = &hdr->status;
  for (int b = 0; b < kNumBins - 1; b++) {
    ProfScope prof("fused_backward", st);
    const int32_t *list = bins + (int64_t)b * n;
    const int32_t *cp = &hdr->bin_count[b];
    switch (b) {
      case 0: hipLaunchKernelGGL((k_fbwd_wave<64, VT>), dim3(mx_grid(-1, true, 8)), dim3(256), 0, st, a, list, cp, status); break;
      case 1: hipLaunchKernelGGL((k_fbwd_wave<256, VT>), dim3(mx_grid(-1, true, 8)), dim3(256), 0, st, a, list, cp, status); break;
      case 2: hipLaunchKernelGGL((k_fbwd_wave<1024, VT>), dim3(mx_grid(-1, true, 4)), dim3(256), 0, st, a, list, cp, status); break;
      case 3: hipLaunchKernelGGL((k_fbwd_block<4096, 256, VT>), dim3(mx_grid(-1, false, 4)), dim3(256), 0, st, a, list, cp, status); break;
      default: hipLaunchKernelGGL((k_fbwd_block<10240, 1024, VT>), dim3(mx_grid(-1, false, 1)), dim3(1024), 0, st, a, list, cp, status); break;
    }
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_mx_flag_if_nonzero, dim3(1), dim3(64), 0, st, &hdr->bin_count[kNumBins - 1], status, 7);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_round<VT>, dim3(gz), dim3(256), 0, st, acc, A->nnz, (VT *)dA);
  LAUNCHCHK();
  return SPGEMM_OK;
}

template <class VT>
static int transpose_typed(const spgemm_csc *X, int64_t *t_colptr, int32_t *t_rowidx, void *t_values, int64_t *perm,
                           const WsLayout &L, char *ws, hipStream_t st) {
  WsHeader *hdr = (WsHeader *)ws;
  int rc = launch_init_header(hdr, (uint64_t)0, st);
  if (rc) return rc;
  ProfScope prof("transpose", st);
  const int64_t m = X->nrows;
  unsigned long long *cnt = (unsigned long long *)(ws + L.bins);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_of(std::max(m, X->nnz), 256), 8 * device_cus()));
  hipLaunchKernelGGL(k_tr_zero, dim3(g), dim3(256), 0, st, cnt, m);
  LAUNCHCHK();
  if (X->nnz > 0) {
    hipLaunchKernelGGL(k_tr_count, dim3(g), dim3(256), 0, st, X->rowidx, X->nnz, m, cnt, &hdr->status);
    LAUNCHCHK();
  }
  rc = launch_colptr_scan((const int64_t *)cnt, m, t_colptr, (int64_t *)(ws + L.scan), st);
  if (rc) return rc;
  if (X->nnz > 0) {
    hipLaunchKernelGGL(k_tr_cursor, dim3(g), dim3(256), 0, st, t_colptr, m, cnt);
    LAUNCHCHK();
    const unsigned gs = (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_of(X->ncols, 4), 16 * device_cus()));
    hipLaunchKernelGGL(k_tr_scatter<VT>, dim3(gs), dim3(256), 0, st, X->colptr, X->rowidx,
                       t_values ? (const VT *)X->values : (const VT *)nullptr, X->ncols, m, cnt, t_rowidx, (VT *)t_values,
                       perm);
    LAUNCHCHK();
  }
  return SPGEMM_OK;
}

}  // namespace spg

using namespace spg;

extern "C" {

int spgemm_transpose(const spgemm_csc *X, int64_t *t_colptr, int32_t *t_rowidx, void *t_values, int64_t *perm,
                     void *ws, size_t ws_bytes, void *stream) {
  int st = check_csc(X, t_values != nullptr);
  if (st) return st;
  if (!t_colptr || (X->nnz > 0 && !t_rowidx)) return SPGEMM_E_INVAL;
  if (X->ncols > INT32_MAX) return SPGEMM_E_OVERFLOW;
  WsLayout L;
  st = ws_layout(SPGEMM_OP_TRANSPOSE, X, nullptr, 0, 0, 1, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if (t_values && X->dtype == SPGEMM_F64)
    return transpose_typed<double>(X, t_colptr, t_rowidx, t_values, perm, L, (char *)ws, s);
  return transpose_typed<float>(X, t_colptr, t_rowidx, t_values, perm, L, (char *)ws, s);
}

int spgemm_masked_xty(const spgemm_csc *X, const spgemm_csc *Y, const spgemm_csc *M, void *out_values, void *ws,
                      size_t ws_bytes, void *stream) {
  int st = check_csc(X, true);
  if (!st) st = check_csc(Y, true);
  if (!st) st = check_csc(M, false);
  if (st) return st;
  if (X->dtype != Y->dtype) return SPGEMM_E_DTYPE;
  if (X->nrows != Y->nrows || M->nrows != X->ncols || M->ncols != Y->ncols) return SPGEMM_E_SHAPE;
  if (M->nnz > 0 && !out_values) return SPGEMM_E_INVAL;
  WsLayout L;
  st = ws_layout(SPGEMM_OP_MASKED_XTY, X, Y, 0, Y->ncols, 1, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if (Y->ncols == 0 || M->nnz == 0) return launch_init_header((WsHeader *)ws, kKeepAnyTag, s);
  if (X->dtype == SPGEMM_F64) return mxty_typed<double>(X, Y, M, out_values, L, (char *)ws, s, true);
  return mxty_typed<float>(X, Y, M, out_values, L, (char *)ws, s, true);
}

int spgemm_batched_masked_xty(const spgemm_csc *X, const spgemm_csc *Y, const spgemm_csc *M, void *out_values,
                              void *ws, size_t ws_bytes, void *stream) {
  int st = check_csc(X, true);
  if (!st) st = check_csc(Y, true);
  if (!st) st = check_csc(M, false);
  if (st) return st;
  if (X->dtype != Y->dtype) return SPGEMM_E_DTYPE;
  if (X->nrows != Y->nrows || M->nrows != X->ncols || M->ncols != Y->ncols) return SPGEMM_E_SHAPE;
  if (M->nnz > 0 && !out_values) return SPGEMM_E_INVAL;
  WsLayout L;
  st = ws_layout(SPGEMM_OP_MASKED_XTY, X, Y, 0, Y->ncols, 1, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if (Y->ncols == 0 || M->nnz == 0) return launch_init_header((WsHeader *)ws, kKeepAnyTag, s);
  if (X->dtype == SPGEMM_F64) return mxty_typed<double>(X, Y, M, out_values, L, (char *)ws, s, false);
  return mxty_typed<float>(X, Y, M, out_values, L, (char *)ws, s, false);
}

int spgemm_batched_backward(const spgemm_csc *A, const spgemm_csc *B, const spgemm_csc *C, const void *dC_values,
                            void *dA_out, void *dB_out, void *ws, size_t ws_bytes, void *stream) {
  int st = check_csc(A, true);
  if (!st) st = check_csc(B, true);
  if (!st) st = check_csc(C, false);
  if (st) return st;
  if (A->dtype != B->dtype) return SPGEMM_E_DTYPE;
  if (A->ncols != B->nrows || C->nrows != A->nrows || C->ncols != B->ncols) return SPGEMM_E_SHAPE;
  if ((C->nnz > 0 && !dC_values) || (A->nnz > 0 && !dA_out) || (B->nnz > 0 && !dB_out)) return SPGEMM_E_INVAL;
  WsLayout L;
  st = ws_layout(SPGEMM_OP_BATCHED_BACKWARD, A, B, 0, B->ncols, 1, &L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if (A->dtype == SPGEMM_F64) return fbwd_typed<double>(A, B, C, dC_values, dA_out, dB_out, L, (char *)ws, s);
  return fbwd_typed<float>(A, B, C, dC_values, dA_out, dB_out, L, (char *)ws, s);
}

int spgemm_permute(const void *src, const int64_t *perm, int64_t n, int32_t dtype, int32_t scatter, void *dst,
                   void *stream) {
  if (n < 0 || (n > 0 && (!src || !perm || !dst))) return SPGEMM_E_INVAL;
  const int vb = dtype_bytes(dtype);
  if (!vb) return SPGEMM_E_DTYPE;
  if (n == 0) return SPGEMM_OK;
  hipStream_t s = (hipStream_t)stream;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_of(n, 256), 8 * device_cus()));
  if (vb == 8)
    hipLaunchKernelGGL(k_permute<double>, dim3(g), dim3(256), 0, s, (const double *)src, perm, n, (double *)dst,
                       (int)scatter);
  else
    hipLaunchKernelGGL(k_permute<float>, dim3(g), dim3(256), 0, s, (const float *)src, perm, n, (float *)dst,
                       (int)scatter);
  LAUNCHCHK();
  return SPGEMM_OK;
}

}  // extern "C"
