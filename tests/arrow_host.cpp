// Host build of the secular core SVD (rt_arrow.h) for the CPU tests: the same
// per-root and per-component functions the device runs on one wave, driven by
// loops, then sorted like the device wrapper.
#define RT_HD
#include "rt_arrow.h"

#include <algorithm>
#include <vector>

extern "C" int arrow_host(int r, int rows, const double *S, const double *a, double nu, double *sv, double *U,
                          double *V) {
  const int cols = r + 1;
  arrow::Problem P;
  int defl[arrow::N];
  if (!arrow::build(P, defl, S, a, nu, r, rows, cols)) return 0;
  int K[arrow::N];
  double tau[arrow::N], zh[arrow::N];
  for (int k = 0; k < P.m; ++k) arrow::root(P, k, K[k], tau[k]);
  for (int j = 0; j < P.m; ++j) zh[j] = arrow::zhat(P, j, K, tau);
  // unsorted columns: roots, then deflated rows
  std::vector<double> u((size_t)rows * rows, 0.0), v((size_t)cols * rows, 0.0), s(rows, 0.0);
  for (int k = 0; k < P.m; ++k) s[k] = arrow::vectors(P, k, K, tau, zh, r, &u[(size_t)k * rows], 1, &v[(size_t)k * cols], 1);
  int c = P.m;
  for (int j = 0; j < r; ++j)
    if (defl[j]) {
      u[(size_t)c * rows + j] = 1.0;
      v[(size_t)c * cols + j] = 1.0;
      s[c] = S[j];
      ++c;
    }
  std::vector<int> order(rows);
  for (int i = 0; i < rows; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return s[x] > s[y]; });
  // outputs: U rows x rows (row-major, column jj = jj-th triplet), V cols x rows
  for (int jj = 0; jj < rows; ++jj) {
    const int j = order[jj];
    sv[jj] = s[j];
    for (int i = 0; i < rows; ++i) U[i * rows + jj] = u[(size_t)j * rows + i];
    for (int i = 0; i < cols; ++i) V[i * rows + jj] = v[(size_t)j * cols + i];
  }
  return 1;
}
