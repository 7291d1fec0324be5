/*
 * spgemm.h -- C ABI of the one-GPU, memory-constrained, sort-free SpGEMM
 * library for MI355X (gfx950).
 *
 * The library computes C = A*B over (+, *) with A (m x k), B (k x n) and C
 * in compressed sparse column (CSC) form, following "Communication-Avoiding
 * and Memory-Constrained Sparse Matrix-Matrix Multiplication at Extreme
 * Scale" (Hussain, Selvitopi, Buluc, Azad; arXiv 2010.08526):
 *   - the product is Gustavson's column formula, C(:,j) = sum over k with
 *     B(k,j) != 0 of A(:,k)*B(k,j) (Sec. II-C);
 *   - a symbolic pass counts the nonzeros of the output before any value is
 *     formed (Alg. 3, LocalSymbolic);
 *   - the output is formed in b batches of whole columns, b chosen from the
 *     available memory (Sec. IV-A, Eq. 2, Alg. 3 and Alg. 4);
 *   - local multiplication and merging use hash tables and never sort
 *     (Sec. IV-D, sort-free local SpGEMM and sort-free hash merging);
 *   - the inner dimension may be split into layers whose partial products
 *     are merged afterwards (Sec. III-B, Alg. 2, Merge-Layer/Merge-Fiber).
 *
 * Conventions shared by every entry point
 *   - Every function returns an int status (spgemm_status); nothing throws
 *     across the ABI.  Argument checks (NULLs, shapes, dtypes, sizes) run on
 *     the host before anything is launched.
 *   - Pointers inside spgemm_csc and all array arguments named *_out or
 *     c_* point to DEVICE memory unless the name ends in _host.  All device
 *     memory is owned by the caller; the library never allocates device
 *     memory.  Scratch memory is passed in as `ws` (device, at least
 *     `ws_bytes` bytes, 256-byte aligned) and sized by
 *     spgemm_workspace_size().
 *   - `stream` is a hipStream_t (NULL = the null stream).  Device work is
 *     enqueued asynchronously on it; calls return before it completes unless
 *     documented otherwise.  Calls on different streams must use different
 *     workspaces.
 *   - Row indices inside a column may come in any order but must be unique;
 *     outputs are written in hash-table order (unsorted), except where noted.
 *     Structure is structural: an output entry exists wherever some product
 *     term exists, even if its terms cancel to zero.
 *   - Values of A and B share one dtype; outputs take that dtype.  Float32
 *     inputs are accumulated in float64 inside the library and rounded once.
 */
#ifndef SPGEMM_H_
#define SPGEMM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPGEMM_OK = 0,
  SPGEMM_E_INVAL = -1,     /* NULL pointer, negative size, bad range, bad op */
  SPGEMM_E_SHAPE = -2,     /* inner dimensions or part shapes disagree */
  SPGEMM_E_DTYPE = -3,     /* unknown dtype or mixed dtypes */
  SPGEMM_E_BUDGET = -4,    /* memory budget cannot hold inputs, reserve or one column */
  SPGEMM_E_WORKSPACE = -5, /* ws NULL, misaligned or smaller than required */
  SPGEMM_E_HIP = -6,       /* a HIP call or launch failed; see spgemm_last_hip_error() */
  SPGEMM_E_OVERFLOW = -7,  /* a size does not fit the index types (rows > INT32_MAX, ...) */
  SPGEMM_E_DEVICE = -8     /* a device-side check failed (reported by spgemm_ws_status) */
} spgemm_status;

typedef enum { SPGEMM_F32 = 0, SPGEMM_F64 = 1 } spgemm_dtype;

/* Semiring of spgemm_numeric and spgemm_merge (Sec. II-A: the algorithms
 * use only a semiring's addition and multiplication, so they apply to any
 * semiring).  For every output entry (i,j) with at least one product term:
 *   PLUS_TIMES: C(i,j) = sum over k of A(i,k)*B(k,j)   (the ordinary product)
 *   MIN_PLUS  : C(i,j) = min over k of A(i,k)+B(k,j)   (tropical: shortest paths)
 *   OR_AND    : C(i,j) = 1                              (boolean: every stored
 *               entry is true, so the result is the pattern product)
 * Terms are formed and combined in float64 and rounded once to the output
 * dtype; min and the or-and result are exact, a min-plus term is one
 * float64 addition.  Structure is structural in every semiring (the same
 * pattern as the plus-times product).  A merge combines the parts' entries
 * with the semiring's addition. */
typedef enum { SPGEMM_SR_PLUS_TIMES = 0, SPGEMM_SR_MIN_PLUS = 1, SPGEMM_SR_OR_AND = 2 } spgemm_semiring;

/* A CSC matrix.  colptr[ncols+1] (int64, colptr[0] = 0, nondecreasing,
 * colptr[ncols] = nnz), rowidx[nnz] (int32, 0 <= row < nrows, unique within
 * a column, any order), values[nnz] of `dtype` (may be NULL where only the
 * pattern is read).  All three arrays are device memory. */
typedef struct spgemm_csc {
  int64_t nrows, ncols, nnz;
  const int64_t *colptr;
  const int32_t *rowidx;
  const void *values;
  int32_t dtype;
} spgemm_csc;

/* Operations for spgemm_workspace_size(). */
typedef enum {
  SPGEMM_OP_SYMBOLIC = 0,
  SPGEMM_OP_NUMERIC = 1,
  SPGEMM_OP_MERGE = 2,
  SPGEMM_OP_COLPTR = 3,
  SPGEMM_OP_MASKED_XTY = 4,
  SPGEMM_OP_TRANSPOSE = 5,
  SPGEMM_OP_BATCHED_FORWARD = 6,
  SPGEMM_OP_BATCHED_BACKWARD = 7,
  SPGEMM_OP_PRUNE = 8,
  SPGEMM_OP_SORT = 9
} spgemm_op;

/* Workspace bytes needed by one call of `op`.  Host only; never syncs.
 *   SYMBOLIC, NUMERIC: A, B and columns [c0,c1) as passed to that call;
 *                      n_layers as passed (>= 1).
 *   MERGE:             A = any one part (its nrows and ncols), B unused,
 *                      n_layers = number of parts.
 *   COLPTR:            c1 - c0 = number of counts; A, B unused (may be NULL).
 *   MASKED_XTY:        A = X, B = Y (M has Y's column count).
 *   TRANSPOSE:         A = the matrix to transpose.
 *   BATCHED_FORWARD:   A, B = the packed operands; c0 = 0, c1 = B.ncols.
 *   BATCHED_BACKWARD:  A, B = the operands of the product.
 *   PRUNE, SORT:       A = the matrix pruned or sorted; B unused.
 * The result depends only on shapes, never on device data. */
int spgemm_workspace_size(int op, const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t c1,
                          int32_t n_layers, size_t *bytes_host);

/* Symbolic pass (Alg. 3, LocalSymbolic, for one process; flops per Sec. II-A).
 * For every output column j in [c0,c1) of C = A*B:
 *   flops_out[j-c0] = sum over k in B(:,j) of nnz(A(:,k))   (int64; may be NULL),
 *   nnz_out[j-c0]   = number of distinct rows of C(:,j)      when n_layers == 1.
 * With n_layers = L > 1 the inner dimension [0,k) is split into L contiguous
 * ranges of width w = ceil(k/L) (layer l covers [l*w, min(k,(l+1)*w)), some
 * possibly empty; Sec. III-B, Alg. 2) and nnz_out holds (L+1) rows of
 * (c1-c0) int64 each: row l = nnz of column j of the layer product
 * A(:,K_l)*B(K_l,:), row L = nnz of C(:,j).  Counts come from hash tables,
 * not from bounds.  Synchronizes `stream` once per pass (per layer, and once
 * for row L) to read the per-bin column counts that size the launches; the
 * counts themselves stay on the device.  A row of B outside [0,k) sets the
 * workspace status (code 1) and the entry is skipped. */
int spgemm_symbolic(const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t c1, int32_t n_layers,
                    int64_t *flops_out, int64_t *nnz_out, void *ws, size_t ws_bytes, void *stream);

/* Batch planner (Eq. 2 and Alg. 3 with one process; Alg. 4 ColSplit).  Host
 * only; reads nothing from the device.
 * nnz_host: the symbolic counts copied to the host, same layout as nnz_out
 * (ncols columns; (L+1) rows if n_layers > 1).  Memory of output column j:
 *   L == 1: r*u_j + 8
 *   L  > 1: r*(sum over l of u_j^l) + 8*L  +  r*u_j + 8
 * with r = 4 + value_bytes (int32 row + value) and 8 bytes of column pointer
 * per column per stored matrix; with layers both the partials and the merged
 * output of a batch are resident.  The memory available to outputs is
 *   avail = budget_bytes - input_bytes - reserve_bytes.
 * The result is the smallest number b of contiguous column batches whose
 * memory each fits in avail (never below ceil(total/avail), the Eq. 2 bound),
 * split so that the largest batch is as small as possible (greedy packing
 * from the left under that smallest cap).  Outputs:
 *   bounds_host[0..b]  column bounds (bounds_host[0] = 0, bounds_host[b] = ncols),
 *   *nbatches_host     = b,
 *   batch_nnz_host     (may be NULL) [b * rows] totals of each count row per
 *                      batch (rows = L+1 if L > 1 else 1), batch-major.
 * bounds_host needs max_batches+1 entries, batch_nnz_host max_batches*rows.
 * Errors: SPGEMM_E_BUDGET when avail <= 0, when one column alone exceeds
 * avail, or when more than max_batches batches would be needed. */
int spgemm_plan_batches(const int64_t *nnz_host, int64_t ncols, int32_t n_layers, int32_t value_bytes,
                        uint64_t input_bytes, uint64_t budget_bytes, uint64_t reserve_bytes, int32_t max_batches,
                        int64_t *bounds_host, int32_t *nbatches_host, int64_t *batch_nnz_host);

/* Column pointers from counts: colptr_out[0] = 0 and
 * colptr_out[i+1] = counts[0] + ... + counts[i] for i < n (an exclusive
 * scan, int64).  counts and colptr_out are device arrays of n and n+1
 * entries.  Asynchronous. */
int spgemm_colptr(const int64_t *counts, int64_t n, int64_t *colptr_out, void *ws, size_t ws_bytes, void *stream);

/* Numeric pass: sort-free hash SpGEMM (Sec. IV-D).  Forms columns [c0,c1) of
 * the layer product A(:,K_layer)*B(K_layer,:) (n_layers = 1, layer = 0: the
 * full product) into c_rowidx/c_values at c_colptr[j-c0] .. c_colptr[j-c0+1],
 * which must come from the matching symbolic counts (spgemm_colptr of the
 * layer's row).  c_colptr has c1-c0+1 entries and may start at any offset.
 * Rows within each output column are in hash-table order.  `flops` is the
 * symbolic flops_out of the same columns (may be NULL).  Every kernel takes
 * its column counts from the device, so the call does not synchronize
 * `stream`, except for A with more than 8,388,608 rows, where the count of
 * columns above 5120 rows (formed on global accumulators) is read back to
 * size their launches.  With n_layers > 1 the layer's share of
 * B(:, c0:c1) is first compacted into the workspace.  A mismatch between
 * counts and the product sets the workspace status (spgemm_ws_status).
 * `semiring` is a spgemm_semiring (SPGEMM_E_INVAL otherwise). */
int spgemm_numeric(const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t c1, int32_t layer,
                   int32_t n_layers, const int64_t *flops, const int64_t *c_colptr, int32_t *c_rowidx,
                   void *c_values, int32_t semiring, void *ws, size_t ws_bytes, void *stream);

/* Sort-free hash merge (Sec. IV-D, sort-free hash merging; Merge in Alg. 1
 * and Alg. 2): C(:,j) = sum over parts of parts[p](:,j), entries with equal
 * row combined (added, for plus-times).  parts is a HOST array of n_parts descriptors (device arrays
 * inside), all with the same nrows, ncols and dtype, 1 <= n_parts <= 4096.
 * c_colptr (ncols+1) comes from the union counts (row L of the symbolic
 * output for the batch).  Output rows in hash-table order.  Synchronizes
 * `stream` to read the per-bin column counts and, for columns of more than
 * 5120 rows, their total entry counts (to cut them into chunks that fit the
 * workspace's bucket region).  Entries with equal row are combined with the
 * addition of `semiring` (a spgemm_semiring; SPGEMM_E_INVAL otherwise). */
int spgemm_merge(const spgemm_csc *parts, int32_t n_parts, const int64_t *c_colptr, int32_t *c_rowidx,
                 void *c_values, int32_t semiring, void *ws, size_t ws_bytes, void *stream);

/* ---- Gradient support.  For a loss defined on the pattern of C = A*B
 * (not part of the paper), with dC = dLoss/dC on P(C):
 *   dB = masked_xty(X = A,   Y = dC,   M = P(B))          aligned with B,
 *   dA = scatter of masked_xty(X = B^T, Y = dC^T, M = P(A^T)) back to A's
 *        storage through A^T's permutation.
 * Every dC(i,j) these need lies in P(C). ---- */

/* Sort-free transpose: X^T in CSC (X.ncols rows, X.nrows columns).
 * t_colptr[X.nrows+1], t_rowidx[X.nnz] (column ids of X, in arbitrary order
 * inside each column of X^T), t_values[X.nnz] of X's dtype (may be NULL:
 * pattern only), perm[X.nnz] (may be NULL): perm[q] = the position in X of
 * the entry stored at position q of X^T.  Requires X.ncols <= INT32_MAX.
 * Workspace: spgemm_workspace_size(SPGEMM_OP_TRANSPOSE, X, ...).  Rows of X
 * out of range set the workspace status and are dropped.  Asynchronous. */
int spgemm_transpose(const spgemm_csc *X, int64_t *t_colptr, int32_t *t_rowidx, void *t_values, int64_t *perm,
                     void *ws, size_t ws_bytes, void *stream);

/* Masked product out(k,j) = sum over i of X(i,k) * Y(i,j) for every stored
 * entry (k,j) of the pattern M, written at M's storage position
 * (out_values[M.nnz], X's dtype; X and Y share a dtype; M's values are not
 * read).  Shapes: X is m x K, Y is m x n, M is K x n.  Rows of Y(:,j) absent
 * from a term count as zero.  Per output column j, Y(:,j) is held in an LDS
 * hash table (or, above the largest table, a dense column of the workspace)
 * and each entry of M(:,j) is a dot product against X(:,k), accumulated in
 * float64 and rounded once.  Workspace: SPGEMM_OP_MASKED_XTY with A = X,
 * B = Y.  Asynchronous. */
int spgemm_masked_xty(const spgemm_csc *X, const spgemm_csc *Y, const spgemm_csc *M, void *out_values, void *ws,
                      size_t ws_bytes, void *stream);

/* Value permutation of n elements of `dtype`: scatter == 0 gathers
 * dst[i] = src[perm[i]]; scatter != 0 scatters dst[perm[i]] = src[i].  perm
 * entries outside [0, n) are skipped.  src and dst must not overlap.
 * Asynchronous; no workspace. */
int spgemm_permute(const void *src, const int64_t *perm, int64_t n, int32_t dtype, int32_t scatter, void *dst,
                   void *stream);

/* ---- Batched form (not part of the paper).  A batch of independent
 * products C_i = A_i * B_i is one product of block-diagonal operands: A_i
 * occupies rows [r_i, r_i + m_i) and columns [k_i, k_i + K_i) of A, B_i rows
 * [k_i, ...) and columns [c_i, c_i + n_i) of B, and C_i is then columns
 * [c_i, c_i + n_i) of C with rows shifted by r_i.  Every phase runs once
 * over all instances; binning by column balances uneven instances. ---- */

/* Packs `count` instances (host array of descriptors, device arrays inside)
 * into one block-diagonal CSC: colptr_out[sum ncols + 1], rowidx_out[sum nnz]
 * (rows shifted by the instance's row offset), values_out[sum nnz] (may be
 * NULL).  offsets_host[3*(count+1)] receives (row, column, entry) offsets of
 * every instance followed by the totals.  ws: at least 64*count bytes.
 * Packed rows must fit int32.  Blocks the host until done (the descriptor
 * table is staged from host memory). */
int spgemm_batch_pack(const spgemm_csc *instances, int32_t count, int64_t *colptr_out, int32_t *rowidx_out,
                      void *values_out, int64_t *offsets_host, void *ws, size_t ws_bytes, void *stream);

/* Whole product C = A*B with no host synchronization and launch grids that
 * do not depend on device data, so the call can be captured in a HIP graph
 * and replayed: symbolic pass (flops_out[B.ncols] may be NULL,
 * nnz_out[B.ncols] per-column counts), column pointers c_colptr[B.ncols+1],
 * numeric pass into c_rowidx/c_values of capacity nnz_cap entries.  The bin
 * kernels are persistent: a fixed grid pulls columns from device-side bins.
 * If nnz(C) exceeds nnz_cap the output is cut at the capacity and the
 * workspace status reports SPGEMM_E_DEVICE.  Columns above the largest LDS
 * table are supported when A has at most 8,388,608 rows (row-slab path);
 * otherwise they are reported through the status word.  No batch planner:
 * the caller sizes outputs (a previous symbolic pass gives nnz(C) exactly).
 * Workspace: SPGEMM_OP_BATCHED_FORWARD. */
int spgemm_batched_forward(const spgemm_csc *A, const spgemm_csc *B, int64_t nnz_cap, int64_t *flops_out,
                           int64_t *nnz_out, int64_t *c_colptr, int32_t *c_rowidx, void *c_values, void *ws,
                           size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as spgemm_batched_forward, with no workspace argument.  Its
 * scratch is a fixed device array of SPGEMM_NOALLOC_SCRATCH_BYTES inside the
 * library (one per GPU, held until the process ends); the call allocates
 * nothing and calls no allocating routine.  Inputs whose
 * SPGEMM_OP_BATCHED_FORWARD workspace exceeds that size are refused with
 * SPGEMM_E_WORKSPACE before anything is launched.  Every call on one GPU
 * shares that GPU's array and initialises what it reads, so calls that
 * overlap on one GPU (different streams, or host threads) race and must not
 * be issued; calls in sequence on one stream are safe.  `stream` must
 * belong to the current device.  Device-side failures are recorded in the
 * array's status word, which this entry point cannot return later: check
 * outputs (e.g. the last column pointer against nnz_cap) instead. */
#define SPGEMM_NOALLOC_SCRATCH_BYTES (64ull << 20)
int spgemm_batched_forward_noalloc(const spgemm_csc *A, const spgemm_csc *B, int64_t nnz_cap, int64_t *flops_out,
                                   int64_t *nnz_out, int64_t *c_colptr, int32_t *c_rowidx, void *c_values,
                                   void *stream);

/* spgemm_masked_xty with no host synchronization (graph-capturable, same
 * workspace).  Columns of Y above the largest LDS table are not supported
 * here and are reported through the workspace status. */
int spgemm_batched_masked_xty(const spgemm_csc *X, const spgemm_csc *Y, const spgemm_csc *M, void *out_values,
                              void *ws, size_t ws_bytes, void *stream);

/* Gradient of a loss on P(C), C = A*B, in one pass with no transpose and no
 * host synchronization (graph-capturable): for each output column j, dC(:,j)
 * (dC_values aligned with C's storage) is held in an LDS hash table and each
 * stored (k,j) of B yields
 *   dB(k,j)  = sum over i in A(:,k) of A(i,k) * dC(i,j)       -> dB_out[nnz(B)]
 *   dA(i,k) += B(k,j) * dC(i,j) for every i in A(:,k)          -> dA_out[nnz(A)]
 * dA is accumulated with float64 atomics in the workspace and rounded once
 * (summation order is not fixed, so dA may differ in the last bits between
 * calls).  C gives only the pattern (values not read).  Columns of C above
 * the largest LDS table are reported through the workspace status; the
 * transpose-based path (spgemm_transpose + spgemm_masked_xty) handles them.
 * Workspace: SPGEMM_OP_BATCHED_BACKWARD with A, B. */
int spgemm_batched_backward(const spgemm_csc *A, const spgemm_csc *B, const spgemm_csc *C, const void *dC_values,
                            void *dA_out, void *dB_out, void *ws, size_t ws_bytes, void *stream);

/* ---- Consumer of an output batch (Sec. I and Sec. IV-B: the application
 * prunes each batch of C before the next one; Markov clustering keeps the
 * k largest entries of every column, Sec. V-C).
 *
 * Per-column pruning of C (float32 or float64; rows unique inside each
 * column, in any order).  Candidates are entries whose value, converted to
 * float64, is >= threshold (NaN is never one; a NaN threshold keeps
 * nothing).  k < 0 keeps every candidate; otherwise the k largest
 * candidates of each column are kept, equal values going to the smaller row
 * (-0.0 equals 0.0).  Kept entries keep their input order and are written
 * to out_colptr[C.ncols + 1] (device, starts at 0), out_rowidx and
 * out_values (device, C's dtype, exact copies).  out_cap, the capacity of
 * the last two in entries, must be at least min(nnz(C), k * C.ncols)
 * (nnz(C) for k < 0): the output never holds more, so no host
 * synchronization is needed and the call can be captured in a graph.  The
 * arrays of C are only read; the outputs must not overlap them.
 * Workspace: spgemm_workspace_size(SPGEMM_OP_PRUNE, C, NULL, 0, 0, 1, ...).
 * Device-side checks (spgemm_ws_status_code): 5 column pointers outside
 * the arrays (that column is treated as empty), 10 a row twice in a column
 * that had more than k candidates (that column keeps its first k kept
 * entries; a column that keeps all its candidates is not checked).  Errors: SPGEMM_E_INVAL for a NULL
 * output or a capacity below the bound, SPGEMM_E_DTYPE, SPGEMM_E_WORKSPACE. */
int spgemm_prune_topk(const spgemm_csc *C, double threshold, int64_t k, int64_t *out_colptr, int32_t *out_rowidx,
                      void *out_values, int64_t out_cap, void *ws, size_t ws_bytes, void *stream);

/* ---- Row-sorted output (Sec. IV-D: the final output of the column-wise
 * merge, Merge-Fiber, is kept sorted within each column; the sort-free hash
 * kernels of this library write rows in table order instead).
 *
 * Sorts every column of C by row, values moving with their rows, into
 * rowidx_out / values_out (device arrays of C.nnz entries, distinct from C's
 * arrays: out of place; C's column pointers describe the result too).  Rows
 * must be unique within each column, as in every output of this library; a
 * repeated row or a row outside [0, C.nrows) sets the workspace status
 * (code 11), and in columns of more than 4096 entries leaves some positions
 * of that column unwritten (nothing outside the column is written).  Columns of
 * up to 64 entries are sorted by one wavefront, up to 4096 by one workgroup
 * in LDS, longer ones by row windows of 2^19 rows ranked through an LDS
 * bitmap.  Asynchronous, no host synchronization (graph-capturable).
 * Workspace: SPGEMM_OP_SORT with A = C. */
int spgemm_sort_columns(const spgemm_csc *C, int32_t *rowidx_out, void *values_out, void *ws, size_t ws_bytes,
                        void *stream);

/* Row-sorted numeric pass with a per-column choice of kernel (the hybrid of
 * Sec. V, discussion of Table VII: a column whose compression ratio
 * flops/nnz is low is formed in row order directly, which beats hashing it
 * and sorting it afterwards; Sec. IV-D keeps the final output sorted within
 * each column).  Forms columns [c0,c1) of A*B (one layer: the full product)
 * with each column in ascending row order, at c_colptr as spgemm_numeric
 * does (`flops` and `c_colptr` from the symbolic pass of the same columns).
 *   - a column with flops_j <= 4096 and flops_j <= esc_cf_max * nnz_j is
 *     formed by expand-sort-compress: every product term placed in LDS,
 *     sorted by row, runs of equal rows combined in row order (one
 *     wavefront per column up to 64 terms, one workgroup up to 4096), and
 *     written straight to c_rowidx / c_values;
 *   - every other column is formed by the hash kernels of spgemm_numeric
 *     into tmp_rowidx / tmp_values (device arrays addressed by the same
 *     column pointers, distinct from the outputs) and then sorted into
 *     c_rowidx / c_values by the kernels of spgemm_sort_columns.
 * esc_cf_max = 0 hashes every column (then `flops` may be NULL); it must be
 * >= 0 (SPGEMM_E_INVAL otherwise).  The choice changes speed only: values
 * equal the hashed ones up to the order in which a run's terms are
 * combined (plus-times), exactly otherwise.  `semiring` as in
 * spgemm_numeric.  Synchronizes the stream only where spgemm_numeric does.
 * A count mismatch sets the workspace status (code 4), as in
 * spgemm_numeric.  Workspace: SPGEMM_OP_NUMERIC with n_layers = 1. */
int spgemm_numeric_sorted(const spgemm_csc *A, const spgemm_csc *B, int64_t c0, int64_t c1, const int64_t *flops,
                          const int64_t *c_colptr, int32_t *c_rowidx, void *c_values, int32_t *tmp_rowidx,
                          void *tmp_values, double esc_cf_max, int32_t semiring, void *ws, size_t ws_bytes,
                          void *stream);

/* Bin thresholds (process-wide; used by calls launched afterwards): which = 0
 * for the symbolic pass, 1 for numeric, merge and masked products.
 * caps_host[5] are the largest bounds on distinct rows that go to bins 0..4
 * (wave tables of 64, 256, 1024 slots, workgroup tables of 4096 and
 * 32768 (symbolic) or 10240 (numeric) slots); larger columns go to the
 * heavy path.  They must be nondecreasing and at most each table's capacity
 * (32, 128, 512, 2048, 16384 symbolic; 32, 128, 512, 2048, 5120 numeric),
 * which are also the defaults (caps_host = NULL restores them).  Thresholds
 * change speed, never results.  SPGEMM_E_INVAL otherwise.
 * which = 2 (numeric, merge) and 3 (symbolic) set instead the launch shape
 * of the five bin kernels: caps_host[5] workgroups per compute unit of
 * their persistent grids, each in [1, 32] (defaults 8, 8, 4, 4, 1 numeric;
 * 8, 8, 8, 8, 1 symbolic; NULL restores them).  Launch shapes change speed,
 * never results. */
int spgemm_set_bin_caps(int32_t which, const int64_t *caps_host);

/* Per-kernel timing (process-wide, off by default; not under graph
 * capture).  spgemm_profile_enable(1) clears the records and brackets each
 * main kernel launch that follows with HIP events on its stream;
 * spgemm_profile_enable(0) stops recording and clears.  spgemm_profile_report
 * waits for the recorded events and writes one line per kernel name,
 * "name total_ms launches\n", into buf_host (SPGEMM_E_INVAL if it does not
 * fit). */
int spgemm_profile_enable(int32_t on);
int spgemm_profile_report(char *buf_host, size_t buf_bytes);

/* Synchronizes `stream` and reports the device-side status word of a
 * workspace used by the calls above: SPGEMM_OK, or SPGEMM_E_DEVICE if a
 * kernel found counts that disagree with the product or an index out of
 * range.  Clears the word.  The only call here that blocks the host. */
int spgemm_ws_status(void *ws, void *stream);

/* As spgemm_ws_status; *code_host (may be NULL) receives the device-side
 * code that was recorded first (0 if none): 1 an index of B(:,j) outside
 * A's columns, 2 a column of A longer than 2^25 entries, 3 a row index
 * outside [0, nrows), 4 a column whose entries disagree with its count from
 * the symbolic pass, 5 column pointers inconsistent with the arrays they
 * index, 7 a column above the largest LDS table in a call without a host
 * synchronization, 8 an output larger than the capacity given, 9 a
 * malformed internal work item, 10 a row twice in a pruned column that had
 * more than k candidates. */
int spgemm_ws_status_code(void *ws, void *stream, int32_t *code_host);

/* What a workspace keeps between calls: consecutive spgemm_numeric calls on
 * one workspace with the same left operand and layer share the copy of A
 * grouped by row slab that the heavy-column path builds (the copy is
 * rebuilt unless a fingerprint of A's columns of the layer, formed on the
 * device at every call from the column pointers, rows and value bits, equals
 * the one it was built from; every other operation of this library that
 * initialises the workspace header clears it, and spgemm_batch_pack
 * overwrites the header with its descriptor table, which leaves a stored
 * fingerprint no more likely to match than a fingerprint collision).
 * spgemm_ws_invalidate clears it explicitly, so that the next numeric call
 * rebuilds it: call it at the start of each product to time a product on
 * its own, and always after writing into a numeric workspace by any means
 * other than this library's calls.  Asynchronous: one small kernel on `stream`, no
 * allocation and no memset, so it can be captured in a graph. */
int spgemm_ws_invalidate(void *ws, void *stream);

/* Testing hook, process-wide, not thread-safe: from now on every column is
 * placed in bin `bin` or a later one (bins are ordered by table capacity,
 * 0 = smallest, 5 = heavy), so each kernel can be exercised on small
 * inputs.  0 restores the natural choice.  Affects results only through
 * output order.  SPGEMM_E_INVAL if bin is outside [0, 5]. */
int spgemm_debug_min_bin(int32_t bin);

/* Text of a status code (static storage). */
const char *spgemm_status_string(int status);

/* hipError_t code of the last failed HIP call in this thread (0 if none). */
int spgemm_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPGEMM_H_ */
