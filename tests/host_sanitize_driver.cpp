// Host-side checks of the library's host-only code (argument checks,
// workspace sizing, the batch planner of Eq. 2 / Alg. 3) under the address
// and undefined-behaviour sanitizers: built with g++ together with host.cpp
// by tests/test_host_sanitizers.py, run on the CPU.  Every array the planner
// writes is allocated at exactly the size the header documents, so a write
// past it is reported; the planner's invariants are checked on the way.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "spgemm.h"

static int fail(const char *what, long a, long b) {
  printf("FAIL %s (%ld, %ld)\n", what, a, b);
  return 1;
}

static int g_planned = 0, g_refused = 0;

static int check_plan(std::mt19937_64 &rng, int trial) {
  std::uniform_int_distribution<int> dn(0, 300), dl(1, 4), dv(0, 1), dmax(1, 70);
  const int64_t n = dn(rng);
  const int L = dl(rng) == 4 ? 3 : 1;
  const int rows = L > 1 ? L + 1 : 1;
  const int32_t vb = dv(rng) ? 4 : 8;
  std::vector<int64_t> nnz((size_t)rows * (size_t)n + 1);
  std::uniform_int_distribution<int64_t> du(0, trial % 3 == 0 ? 5 : 100000);
  for (auto &x : nnz) x = du(rng);
  uint64_t need = 0;
  for (int64_t j = 0; j < n; j++) {
    uint64_t parts = 0;
    for (int l = 0; l < (L > 1 ? L : 0); l++) parts += (uint64_t)nnz[(size_t)l * n + j];
    need += (4 + (uint64_t)vb) * (parts + (uint64_t)nnz[(size_t)(rows - 1) * n + j]) + 8 * (uint64_t)(L > 1 ? L + 1 : 1);
  }
  const uint64_t input = 1000, reserve = 500;
  std::uniform_int_distribution<uint64_t> dav(1, need / 3 + 2);
  const uint64_t budget = input + reserve + dav(rng) + (trial % 5 == 0 ? need : 0);
  const int32_t maxb = dmax(rng);
  int64_t *bounds = new int64_t[(size_t)maxb + 1];
  int64_t *bnnz = new int64_t[(size_t)maxb * (size_t)rows];
  int32_t nb = -1;
  const int st = spgemm_plan_batches(n ? nnz.data() : nullptr, n, L, vb, input, budget, reserve, maxb, bounds, &nb, bnnz);
  int bad = 0;
  if (st == SPGEMM_OK) {
    g_planned++;
    if (nb < 1 || nb > maxb) bad |= fail("batch count", nb, maxb);
    if (bounds[0] != 0 || bounds[nb] != n) bad |= fail("bounds cover the columns", bounds[0], bounds[nb]);
    for (int i = 0; i < nb && !bad; i++) {
      if (bounds[i + 1] < bounds[i]) bad |= fail("bounds nondecreasing", bounds[i], bounds[i + 1]);
      int64_t s = 0;
      for (int64_t j = bounds[i]; j < bounds[i + 1]; j++) s += nnz[(size_t)(rows - 1) * n + j];
      if (s != bnnz[(size_t)i * rows + rows - 1]) bad |= fail("batch counts", s, bnnz[(size_t)i * rows + rows - 1]);
    }
  } else if (st == SPGEMM_E_BUDGET) {
    g_refused++;
  } else {
    bad |= fail("planner status", st, 0);
  }
  delete[] bounds;
  delete[] bnnz;
  return bad;
}

static int check_sizes(std::mt19937_64 &rng) {
  std::uniform_int_distribution<int64_t> dm(0, 3000000), dk(0, 200000), dz(0, 5000000);
  std::uniform_int_distribution<int> dop(0, 11), dl(0, 20);
  int64_t dummy_cp[2] = {0, 0};
  int32_t dummy_ri[1] = {0};
  float dummy_v[1] = {0.0f};
  for (int t = 0; t < 3000; t++) {
    spgemm_csc A{dm(rng), dk(rng), dz(rng), dummy_cp, dummy_ri, dummy_v, (int32_t)(t % 3)};
    spgemm_csc B{A.ncols, dk(rng), dz(rng), dummy_cp, dummy_ri, dummy_v, A.dtype};
    const int op = dop(rng);
    const int64_t c0 = B.ncols ? (int64_t)(rng() % (uint64_t)B.ncols) : 0;
    const int64_t c1 = c0 + (B.ncols - c0 ? (int64_t)(rng() % (uint64_t)(B.ncols - c0 + 1)) : 0);
    size_t bytes = 0;
    const int st = spgemm_workspace_size(op, &A, t % 7 == 0 ? nullptr : &B, c0, c1, dl(rng), &bytes);
    if (st == SPGEMM_OK && bytes < 4096) return fail("workspace holds its header", (long)bytes, op);
    if (spgemm_status_string(st) == nullptr) return fail("status text", st, 0);
  }
  size_t b = 0;
  if (spgemm_workspace_size(SPGEMM_OP_SYMBOLIC, nullptr, nullptr, 0, 0, 1, &b) == SPGEMM_OK)
    return fail("null operands refused", 0, 0);
  for (int s = -10; s <= 2; s++)
    if (spgemm_status_string(s) == nullptr) return fail("status text", s, 0);
  return 0;
}

int main() {
  std::mt19937_64 rng(201008526);
  int bad = 0;
  for (int t = 0; t < 400 && !bad; t++) bad |= check_plan(rng, t);
  if (!bad) bad |= check_sizes(rng);
  if (bad) return 1;
  if (g_planned < 50 || g_refused < 10) return fail("planner cases reached", g_planned, g_refused);
  printf("planned %d, refused %d\nok\n", g_planned, g_refused);
  return 0;
}
