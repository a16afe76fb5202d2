// Host-side check of the projection's multigrid hierarchy (amg_build in
// paper_1006_0720_amd/csrc/k_amg.hip), driven by tests/test_amg_host.py.
//
// Reads a symmetric CSR matrix (int32 n, nnz; int32 row offsets, columns;
// float64 values) and a right-hand side (float64 n), builds the hierarchy,
// and runs conjugate gradients on the CPU preconditioned by one V-cycle of it
// (the V-cycle the device kernels apply: a damped-Jacobi step from zero,
// restriction by P^T, the coarse correction, prolongation by P, a damped-Jacobi
// step; the coarsest level by its dense inverse).  Writes the iteration count,
// the level sizes and the solution.
#include "../paper_1006_0720_amd/csrc/pdf_solvers.h"

#include <cmath>
#include <cstdio>
#include <vector>

using namespace pdfk;
using Vec = std::vector<double>;

static void spmv(const std::vector<int32_t> &o, const std::vector<int32_t> &c, const Vec &v, const Vec &x, Vec &y) {
  const int n = (int)o.size() - 1;
  y.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = o[i]; j < o[i + 1]; ++j) s += v[j] * x[c[j]];
    y[i] = s;
  }
}

static void vcycle(const AmgHost &h, size_t l, const Vec &b, Vec &y) {
  const AmgHostLevel &L = h.lv[l];
  const int n = L.n;
  if (l + 1 == h.lv.size()) {
    y.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += h.cinv[(size_t)i * n + j] * b[j];
      y[i] = s;
    }
    return;
  }
  Vec x(n), r(n), t, bc, yc;
  for (int i = 0; i < n; ++i) x[i] = L.omega * L.dinv[i] * b[i];
  spmv(L.a_off, L.a_col, L.a_val, x, t);
  for (int i = 0; i < n; ++i) r[i] = b[i] - t[i];
  spmv(L.r_off, L.r_col, L.r_val, r, bc);
  vcycle(h, l + 1, bc, yc);
  spmv(L.p_off, L.p_col, L.p_val, yc, t);
  for (int i = 0; i < n; ++i) x[i] += t[i];
  spmv(L.a_off, L.a_col, L.a_val, x, t);
  y.resize(n);
  for (int i = 0; i < n; ++i) y[i] = x[i] + L.omega * L.dinv[i] * (b[i] - t[i]);
}

int main(int argc, char **argv) {
  if (argc != 4) return 2;
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hd[2];
  if (std::fread(hd, 4, 2, f) != 2) return 2;
  const int n = hd[0], nnz = hd[1];
  std::vector<int32_t> o(n + 1), c(nnz);
  Vec v(nnz), b(n);
  if (std::fread(o.data(), 4, n + 1, f) != (size_t)n + 1 || std::fread(c.data(), 4, nnz, f) != (size_t)nnz ||
      std::fread(v.data(), 8, nnz, f) != (size_t)nnz || std::fread(b.data(), 8, n, f) != (size_t)n)
    return 2;
  std::fclose(f);
  AmgHost h;
  if (!amg_build(n, o, c, v, h)) return 3;
  Vec x(n, 0.0), r = b, z, p, q;
  vcycle(h, 0, r, z);
  p = z;
  double rz = 0.0;
  for (int i = 0; i < n; ++i) rz += r[i] * z[i];
  const double bb = rz;
  int it = 0;
  for (; it < 1000 && rz > std::atof(argv[3]) * bb; ++it) {
    spmv(o, c, v, p, q);
    double pq = 0.0;
    for (int i = 0; i < n; ++i) pq += p[i] * q[i];
    const double a = rz / pq;
    for (int i = 0; i < n; ++i) {
      x[i] += a * p[i];
      r[i] -= a * q[i];
    }
    vcycle(h, 0, r, z);
    double rzn = 0.0;
    for (int i = 0; i < n; ++i) rzn += r[i] * z[i];
    const double be = rzn / rz;
    rz = rzn;
    for (int i = 0; i < n; ++i) p[i] = z[i] + be * p[i];
  }
  std::printf("iterations %d\nlevels", it);
  for (const auto &L : h.lv) std::printf(" %d", L.n);
  std::printf("\n");
  FILE *g = std::fopen(argv[2], "wb");
  if (!g || std::fwrite(x.data(), 8, n, g) != (size_t)n) return 2;
  std::fclose(g);
  return 0;
}
