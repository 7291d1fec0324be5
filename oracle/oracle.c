/*
 * CPU oracle for C = A*B over (+, *) with CSC inputs.  TEST INFRASTRUCTURE
 * ONLY: nothing in the product path may link, load or call this file; only
 * the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Plain, slow and obviously correct by design.  Every routine follows a
 * definition in the paper:
 *   - Gustavson's column formula, C(:,j) = sum over k with B(k,j) != 0 of
 *     A(:,k) * B(k,j)  (Sec. II-C, the displayed column formula);
 *   - flops = the number of multiplications of A*B (Sec. II-A);
 *   - a layer's partial product D = A(:,K) * B(K,:) over a contiguous range
 *     K of the inner dimension, and merging = adding entries with equal
 *     (row, col) (Sec. III-A, Merge; Sec. III-B, Alg. 2);
 *   - a batch = a contiguous range of output columns (Sec. IV-B, Alg. 4).
 * The gradient routines follow from the product rule on the sum of squares
 * loss restricted to the pattern of C (not in the paper).
 *
 * Accumulation is a dense float64 array per output column (a sparse
 * accumulator in the sense of Gilbert, Moler and Schreiber 1992).  Values
 * arrive as float64; float32 inputs widen exactly, and the product of two
 * float32 values is exact in float64.  Output rows are sorted ascending:
 * this is only the oracle's canonical order for comparison.  Structure is
 * structural: an entry exists where some product term exists, even if the
 * terms cancel to zero.
 *
 * Parallelism: OpenMP over output columns (each column independent).
 * Return value of every entry point: 0 on success, -1 on a bad argument,
 * -2 on allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* flops of output columns [c0,c1) restricted to inner indices [klo,khi):
 * f[j-c0] = sum over k in B(:,j) with klo <= k < khi of nnz(A(:,k)). */
int orc_flops(const int64_t *Acp, const int64_t *Bcp, const int32_t *Bri, int64_t c0, int64_t c1,
              int64_t klo, int64_t khi, int64_t *f_out) {
  if (c1 < c0) return -1;
  for (int64_t j = c0; j < c1; j++) {
    int64_t f = 0;
    for (int64_t p = Bcp[j]; p < Bcp[j + 1]; p++) {
      int64_t k = Bri[p];
      if (k >= klo && k < khi) f += Acp[k + 1] - Acp[k];
    }
    f_out[j - c0] = f;
  }
  return 0;
}

/* Structural nnz of every output column j in [c0,c1) of A(:,K)*B(K,:),
 * K = [klo,khi).  m = rows of A. */
int orc_count(int64_t m, const int64_t *Acp, const int32_t *Ari, const int64_t *Bcp, const int32_t *Bri,
              int64_t c0, int64_t c1, int64_t klo, int64_t khi, int64_t *nnz_out, int nthreads) {
  if (c1 < c0 || m < 0) return -1;
  set_threads(nthreads);
  int err = 0;
#pragma omp parallel
  {
    unsigned char *mark = (unsigned char *)calloc((size_t)(m > 0 ? m : 1), 1);
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!mark || !touched) {
#pragma omp atomic write
      err = -2;
    } else {
#pragma omp for schedule(dynamic, 64)
      for (int64_t j = c0; j < c1; j++) {
        int64_t nt = 0;
        for (int64_t p = Bcp[j]; p < Bcp[j + 1]; p++) {
          int64_t k = Bri[p];
          if (k < klo || k >= khi) continue;
          for (int64_t q = Acp[k]; q < Acp[k + 1]; q++) {
            int32_t i = Ari[q];
            if (!mark[i]) {
              mark[i] = 1;
              touched[nt++] = i;
            }
          }
        }
        for (int64_t t = 0; t < nt; t++) mark[touched[t]] = 0;
        nnz_out[j - c0] = nt;
      }
    }
    free(mark);
    free(touched);
  }
  return err;
}

/* Values of the same product.  Ccp[0..c1-c0] are offsets into Cri/Cv/Cterms/Cabs
 * (Ccp[0] may be nonzero), sized by orc_count.  Per entry:
 *   Cri   row index, columns sorted ascending,
 *   Cv    sum of A(i,k)*B(k,j) accumulated in float64 in the order of B(:,j),
 *   Cterms number of product terms,
 *   Cabs  sum of |A(i,k)*B(k,j)| (the scale of the float32 error bound).
 * Cterms and Cabs may be NULL. */
int orc_fill(int64_t m, const int64_t *Acp, const int32_t *Ari, const double *Av, const int64_t *Bcp,
             const int32_t *Bri, const double *Bv, int64_t c0, int64_t c1, int64_t klo, int64_t khi,
             const int64_t *Ccp, int32_t *Cri, double *Cv, int32_t *Cterms, double *Cabs, int nthreads) {
  if (c1 < c0 || m < 0) return -1;
  set_threads(nthreads);
  int err = 0;
#pragma omp parallel
  {
    size_t mm = (size_t)(m > 0 ? m : 1);
    double *acc = (double *)calloc(mm, sizeof(double));
    double *aab = (double *)calloc(mm, sizeof(double));
    int32_t *terms = (int32_t *)calloc(mm, sizeof(int32_t));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * mm);
    if (!acc || !aab || !terms || !touched) {
#pragma omp atomic write
      err = -2;
    } else {
#pragma omp for schedule(dynamic, 64)
      for (int64_t j = c0; j < c1; j++) {
        int64_t nt = 0;
        for (int64_t p = Bcp[j]; p < Bcp[j + 1]; p++) {
          int64_t k = Bri[p];
          if (k < klo || k >= khi) continue;
          double b = Bv[p];
          for (int64_t q = Acp[k]; q < Acp[k + 1]; q++) {
            int32_t i = Ari[q];
            double prod = Av[q] * b;
            if (terms[i] == 0) touched[nt++] = i;
            terms[i] += 1;
            acc[i] += prod;
            aab[i] += fabs(prod);
          }
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        int64_t base = Ccp[j - c0];
        int64_t cap = Ccp[j - c0 + 1] - base;
        for (int64_t t = 0; t < nt; t++) {
          int32_t i = touched[t];
          if (t < cap) {
            Cri[base + t] = i;
            Cv[base + t] = acc[i];
            if (Cterms) Cterms[base + t] = terms[i];
            if (Cabs) Cabs[base + t] = aab[i];
          }
          acc[i] = 0.0;
          aab[i] = 0.0;
          terms[i] = 0;
        }
        if (nt != cap) {
#pragma omp atomic write
          err = -1;
        }
      }
    }
    free(acc);
    free(aab);
    free(terms);
    free(touched);
  }
  return err;
}

/* Masked product out(k,j) = sum over i of X(i,k) * Y(i,j), for every stored
 * (k,j) of the pattern M, written at M's storage slot.  X is m x K, Y is
 * m x n, M is K x n.  Y(:,j) is scattered into a dense float64 column and
 * each requested entry is a dot product against X(:,k). */
int orc_masked_xty(int64_t m, const int64_t *Xcp, const int32_t *Xri, const double *Xv, const int64_t *Ycp,
                   const int32_t *Yri, const double *Yv, int64_t n, const int64_t *Mcp, const int32_t *Mri,
                   double *out, int nthreads) {
  if (m < 0 || n < 0) return -1;
  set_threads(nthreads);
  int err = 0;
#pragma omp parallel
  {
    double *y = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    if (!y) {
#pragma omp atomic write
      err = -2;
    } else {
#pragma omp for schedule(dynamic, 64)
      for (int64_t j = 0; j < n; j++) {
        for (int64_t p = Ycp[j]; p < Ycp[j + 1]; p++) y[Yri[p]] = Yv[p];
        for (int64_t p = Mcp[j]; p < Mcp[j + 1]; p++) {
          int64_t k = Mri[p];
          double s = 0.0;
          for (int64_t q = Xcp[k]; q < Xcp[k + 1]; q++) s += Xv[q] * y[Xri[q]];
          out[p] = s;
        }
        for (int64_t p = Ycp[j]; p < Ycp[j + 1]; p++) y[Yri[p]] = 0.0;
      }
    }
    free(y);
  }
  return err;
}

/* Gradient of L(A,B) = sum over (i,j) in P(C) of g(C(i,j)) with respect to
 * the stored values of A, given dC(i,j) = dL/dC(i,j) on P(C):
 *   dA(i,k) = sum over j with (k,j) in P(B) of dC(i,j) * B(k,j),
 * one value per stored entry of A.  Runs serially over j (dA accumulates
 * across output columns).  dC is given as a CSC with C's pattern. */
int orc_grad_a(int64_t m, const int64_t *Acp, const int32_t *Ari, int64_t nnzA, const int64_t *Bcp,
               const int32_t *Bri, const double *Bv, int64_t n, const int64_t *Dcp, const int32_t *Dri,
               const double *Dv, double *dA) {
  if (m < 0 || n < 0 || nnzA < 0) return -1;
  double *g = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
  if (!g) return -2;
  for (int64_t q = 0; q < nnzA; q++) dA[q] = 0.0;
  for (int64_t j = 0; j < n; j++) {
    for (int64_t p = Dcp[j]; p < Dcp[j + 1]; p++) g[Dri[p]] = Dv[p];
    for (int64_t p = Bcp[j]; p < Bcp[j + 1]; p++) {
      int64_t k = Bri[p];
      double b = Bv[p];
      for (int64_t q = Acp[k]; q < Acp[k + 1]; q++) dA[q] += g[Ari[q]] * b;
    }
    for (int64_t p = Dcp[j]; p < Dcp[j + 1]; p++) g[Dri[p]] = 0.0;
  }
  free(g);
  return 0;
}

/* dB(k,j) = sum over i in A(:,k) of A(i,k) * dC(i,j), per stored (k,j) of B. */
int orc_grad_b(int64_t m, const int64_t *Acp, const int32_t *Ari, const double *Av, const int64_t *Bcp,
               const int32_t *Bri, int64_t n, const int64_t *Dcp, const int32_t *Dri, const double *Dv,
               double *dB, int nthreads) {
  return orc_masked_xty(m, Acp, Ari, Av, Dcp, Dri, Dv, n, Bcp, Bri, dB, nthreads);
}
