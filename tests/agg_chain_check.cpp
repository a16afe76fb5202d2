// Host-side check of the elliptic relaxation's aggregation chain (agg_chain in
// paper_1006_0720_amd/csrc/k_amg.hip), driven by tests/test_agg_chain.py.
//
// Builds the chain for an anisotropic five-point operator on an N x N grid
// and checks, level by level, that the coarse values formed by the gather
// lists (each coarse entry the sum of the listed finer entries) equal the
// Galerkin product T^T A T with the tentative prolongator formed densely,
// that no entry of T^T A T is missing from the coarse pattern, that every row
// of the pattern is sorted, and that the member lists invert the aggregate
// map.  Prints the level sizes and the largest discrepancy; exit status 1 on
// any failure.
#include "../paper_1006_0720_amd/csrc/pdf_solvers.h"

#include <cmath>
#include <cstdio>
#include <map>
#include <vector>

using namespace pdfk;

int main(int argc, char **argv) {
  const int N = argc > 1 ? std::atoi(argv[1]) : 40, n = N * N;
  std::vector<int32_t> off(1, 0), col;
  std::vector<double> val;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      std::map<int, double> row;
      const int r = i * N + j;
      const double ax = 1.0 + 0.5 * (i % 3 == 0);  // stronger coupling along every third row
      row[r] = 2.0 + 2.0 * ax + 0.01 * ((r * 7) % 5);
      if (i > 0) row[r - N] = -1.0;
      if (i < N - 1) row[r + N] = -1.0;
      if (j > 0) row[r - 1] = -ax;
      if (j < N - 1) row[r + 1] = -ax;
      for (auto &kv : row) {
        col.push_back(kv.first);
        val.push_back(kv.second);
      }
      off.push_back((int32_t)col.size());
    }
  std::vector<AggHostLevel> lv;
  const bool ok = agg_chain(n, off, col, val, 20, lv);
  std::printf("built %d levels", ok ? 1 : 0);
  for (auto &L : lv) std::printf(" %d", L.n);
  std::printf("\n");
  if (!ok || lv.size() < 3) return 1;
  int bad = 0;
  double maxerr = 0.0;
  std::vector<double> v = val;
  for (size_t l = 0; l + 1 < lv.size(); ++l) {
    const AggHostLevel &F = lv[l], &C = lv[l + 1];
    std::vector<double> dense((size_t)C.n * C.n, 0.0);
    for (int i = 0; i < F.n; ++i)
      for (int j = F.off[i]; j < F.off[i + 1]; ++j) dense[(size_t)F.agg[i] * C.n + F.agg[F.col[j]]] += v[j];
    std::vector<double> vc(C.col.size(), 0.0);
    for (size_t J = 0; J < C.col.size(); ++J)
      for (int k = F.g_off[J]; k < F.g_off[J + 1]; ++k) vc[J] += v[F.g_idx[k]];
    for (int I = 0; I < C.n; ++I)
      for (int j = C.off[I]; j < C.off[I + 1]; ++j) {
        maxerr = std::fmax(maxerr, std::fabs(vc[j] - dense[(size_t)I * C.n + C.col[j]]));
        if (j > C.off[I] && C.col[j] <= C.col[j - 1]) ++bad;
        dense[(size_t)I * C.n + C.col[j]] = 0.0;
      }
    for (double x : dense)
      if (std::fabs(x) > 1e-12) ++bad;  // an entry of T^T A T outside the pattern
    for (int I = 0; I < C.n; ++I)
      for (int m = F.m_off[I]; m < F.m_off[I + 1]; ++m)
        if (F.agg[F.mem[m]] != I) ++bad;
    if ((int)F.mem.size() != F.n || (int)F.g_idx.size() != F.off[F.n]) ++bad;
    v = vc;
  }
  std::printf("max discrepancy %g, failures %d\n", maxerr, bad);
  return (bad == 0 && maxerr <= 1e-12) ? 0 : 1;
}
