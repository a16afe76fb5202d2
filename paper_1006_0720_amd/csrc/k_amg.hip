// Smoothed-aggregation algebraic multigrid (Vanek, Mandel & Brezina, 1996) as
// the preconditioner of the projection's conjugate gradients on gfx950.
//
// The paper solves the pressure Poisson problem (Ch.3, Sec. Solution of the
// Eulerian equations) with Jacobi-preconditioned conjugate gradients; on
// strongly graded meshes of a million triangles that needs thousands of
// iterations.  One V-cycle of this hierarchy replaces the Jacobi step: the
// iteration then converges in a few tens of steps, to the same solution.
//
// Hierarchy (built once on the host, the stiffness matrix being constant):
//   strength    |a_ij| >= theta sqrt(a_ii a_jj), theta = 0.08
//   aggregates  greedy: seeds whose strong neighbours are all free take them;
//               the rest join the aggregate they are most strongly tied to;
//               leftovers seed new aggregates
//   tentative   T[i, agg(i)] = 1 (the constants, the operator's null space,
//               are kept exactly on every level)
//   prolongator P = (I - omega D^-1 A) T, omega = 4 / (3 rho(D^-1 A))
//   coarse      A_c = P^T A P (Galerkin), until at most AMG_COARSE unknowns;
//               the coarsest is solved exactly by the dense inverse of
//               A_c + alpha 1 1^T (alpha = mean diagonal / n), which equals
//               the solve of A_c on right-hand sides of zero sum
// V-cycle on each level: one damped-Jacobi pre-smoothing step from zero,
// restriction of the residual by P^T, the coarse correction, one damped-Jacobi
// post-smoothing step.  Symmetric, so the preconditioned iteration stays a
// conjugate-gradient method.
#include <hip/hip_runtime.h>

#include "pdf_solvers.h"

#include <algorithm>
#include <cmath>

namespace pdfk {

namespace {

constexpr int32_t AMG_COARSE = 400;
constexpr double AMG_THETA = 0.08;

struct Csr {
  int32_t nr = 0, nc = 0;
  std::vector<int32_t> off, col;
  std::vector<double> val;
};

double diag_of(const Csr &a, int32_t i) {
  for (int32_t j = a.off[i]; j < a.off[i + 1]; ++j)
    if (a.col[j] == i) return a.val[j];
  return 0.0;
}

// largest eigenvalue of D^-1 A by power iteration (an estimate from below,
// raised by 10 %)
double spectral_radius(const Csr &a, const std::vector<double> &dinv) {
  const int32_t n = a.nr;
  std::vector<double> v((size_t)n), w((size_t)n);
  for (int32_t i = 0; i < n; ++i) v[i] = 1.0 + (double)((i * 7919) % 101) / 101.0;
  double rho = 1.0;
  for (int it = 0; it < 30; ++it) {
    double nw = 0.0, nv = 0.0;
    for (int32_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int32_t j = a.off[i]; j < a.off[i + 1]; ++j) s += a.val[j] * v[a.col[j]];
      w[i] = dinv[i] * s;
      nw += w[i] * w[i];
      nv += v[i] * v[i];
    }
    if (!(nw > 0.0)) break;
    rho = std::sqrt(nw / nv);
    const double sc = 1.0 / std::sqrt(nw);
    for (int32_t i = 0; i < n; ++i) v[i] = w[i] * sc;
  }
  return 1.1 * rho;
}

int32_t aggregate(const Csr &a, std::vector<int32_t> &agg) {
  const int32_t n = a.nr;
  std::vector<double> d((size_t)n);
  for (int32_t i = 0; i < n; ++i) d[i] = std::fabs(diag_of(a, i));
  auto strong = [&](int32_t i, int32_t j, double v) {
    return j != i && std::fabs(v) >= AMG_THETA * std::sqrt(d[i] * d[j]);
  };
  agg.assign((size_t)n, -1);
  int32_t na = 0;
  for (int32_t i = 0; i < n; ++i) {  // seeds
    if (agg[i] >= 0) continue;
    bool free = true;
    for (int32_t j = a.off[i]; j < a.off[i + 1] && free; ++j)
      if (strong(i, a.col[j], a.val[j]) && agg[a.col[j]] >= 0) free = false;
    if (!free) continue;
    agg[i] = na;
    for (int32_t j = a.off[i]; j < a.off[i + 1]; ++j)
      if (strong(i, a.col[j], a.val[j])) agg[a.col[j]] = na;
    ++na;
  }
  std::vector<int32_t> a1 = agg;
  for (int32_t i = 0; i < n; ++i) {  // join the most strongly tied aggregate
    if (a1[i] >= 0) continue;
    double best = -1.0;
    for (int32_t j = a.off[i]; j < a.off[i + 1]; ++j) {
      const int32_t c = a.col[j];
      if (a1[c] >= 0 && strong(i, c, a.val[j]) && std::fabs(a.val[j]) > best) {
        best = std::fabs(a.val[j]);
        agg[i] = a1[c];
      }
    }
  }
  for (int32_t i = 0; i < n; ++i) {  // leftovers seed new aggregates
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int32_t j = a.off[i]; j < a.off[i + 1]; ++j)
      if (strong(i, a.col[j], a.val[j]) && agg[a.col[j]] < 0) agg[a.col[j]] = na;
    ++na;
  }
  return na;
}

// c = a * b (Gustavson, one dense accumulator row)
Csr multiply(const Csr &a, const Csr &b) {
  Csr c;
  c.nr = a.nr;
  c.nc = b.nc;
  c.off.assign((size_t)a.nr + 1, 0);
  std::vector<int32_t> mark((size_t)b.nc, -1), cols;
  std::vector<double> acc((size_t)b.nc, 0.0);
  for (int32_t i = 0; i < a.nr; ++i) {
    cols.clear();
    for (int32_t j = a.off[i]; j < a.off[i + 1]; ++j) {
      const int32_t k = a.col[j];
      const double av = a.val[j];
      for (int32_t l = b.off[k]; l < b.off[k + 1]; ++l) {
        const int32_t q = b.col[l];
        if (mark[q] != i) {
          mark[q] = i;
          acc[q] = 0.0;
          cols.push_back(q);
        }
        acc[q] += av * b.val[l];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t q : cols) {
      c.col.push_back(q);
      c.val.push_back(acc[q]);
    }
    c.off[i + 1] = (int32_t)c.col.size();
  }
  return c;
}

Csr transpose(const Csr &a) {
  Csr t;
  t.nr = a.nc;
  t.nc = a.nr;
  t.off.assign((size_t)a.nc + 1, 0);
  for (int32_t c : a.col) t.off[c + 1]++;
  for (int32_t i = 0; i < a.nc; ++i) t.off[i + 1] += t.off[i];
  t.col.resize(a.col.size());
  t.val.resize(a.val.size());
  std::vector<int32_t> cur(t.off.begin(), t.off.end() - 1);
  for (int32_t i = 0; i < a.nr; ++i)
    for (int32_t j = a.off[i]; j < a.off[i + 1]; ++j) {
      const int32_t p = cur[a.col[j]]++;
      t.col[p] = i;
      t.val[p] = a.val[j];
    }
  return t;
}

// inverse of a dense symmetric positive definite matrix (row-major, n x n) by
// Cholesky; false if it is not positive definite
bool spd_inverse(std::vector<double> &m, int32_t n) {
  std::vector<double> l((size_t)n * n, 0.0);
  for (int32_t j = 0; j < n; ++j) {
    double s = m[(size_t)j * n + j];
    for (int32_t k = 0; k < j; ++k) s -= l[(size_t)j * n + k] * l[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    const double d = std::sqrt(s);
    l[(size_t)j * n + j] = d;
    for (int32_t i = j + 1; i < n; ++i) {
      double t = m[(size_t)i * n + j];
      for (int32_t k = 0; k < j; ++k) t -= l[(size_t)i * n + k] * l[(size_t)j * n + k];
      l[(size_t)i * n + j] = t / d;
    }
  }
  // columns of the inverse: L L^T x = e_c
  std::vector<double> y((size_t)n);
  for (int32_t c = 0; c < n; ++c) {
    for (int32_t i = 0; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int32_t k = 0; k < i; ++k) t -= l[(size_t)i * n + k] * y[k];
      y[i] = t / l[(size_t)i * n + i];
    }
    for (int32_t i = n - 1; i >= 0; --i) {
      double t = y[i];
      for (int32_t k = i + 1; k < n; ++k) t -= l[(size_t)k * n + i] * y[k];
      y[i] = t / l[(size_t)i * n + i];
    }
    for (int32_t i = 0; i < n; ++i) m[(size_t)i * n + c] = y[i];
  }
  return true;
}

}  // namespace

bool amg_build(int32_t n, const std::vector<int32_t> &off, const std::vector<int32_t> &col,
               const std::vector<double> &val, AmgHost &h) {
  h.lv.clear();
  Csr a;
  a.nr = a.nc = n;
  a.off = off;
  a.col = col;
  a.val = val;
  while ((int)h.lv.size() < AMG_MAXL - 1 && a.nr > AMG_COARSE) {
    AmgHostLevel L;
    L.n = a.nr;
    L.dinv.resize((size_t)a.nr);
    for (int32_t i = 0; i < a.nr; ++i) {
      const double d = diag_of(a, i);
      L.dinv[i] = d > 0.0 ? 1.0 / d : 0.0;
    }
    L.omega = 4.0 / (3.0 * spectral_radius(a, L.dinv));
    std::vector<int32_t> agg;
    const int32_t na = aggregate(a, agg);
    if (na >= a.nr || na < 1) break;  // no coarsening: stop here
    Csr p;  // P = (I - omega D^-1 A) T, row by row
    p.nr = a.nr;
    p.nc = na;
    p.off.assign((size_t)a.nr + 1, 0);
    std::vector<int32_t> mark((size_t)na, -1), cols;
    std::vector<double> acc((size_t)na, 0.0);
    for (int32_t i = 0; i < a.nr; ++i) {
      cols.clear();
      auto add = [&](int32_t q, double v) {
        if (mark[q] != i) {
          mark[q] = i;
          acc[q] = 0.0;
          cols.push_back(q);
        }
        acc[q] += v;
      };
      add(agg[i], 1.0);
      for (int32_t j = a.off[i]; j < a.off[i + 1]; ++j) add(agg[a.col[j]], -L.omega * L.dinv[i] * a.val[j]);
      std::sort(cols.begin(), cols.end());
      for (int32_t q : cols) {
        p.col.push_back(q);
        p.val.push_back(acc[q]);
      }
      p.off[i + 1] = (int32_t)p.col.size();
    }
    const Csr r = transpose(p);
    Csr ac = multiply(r, multiply(a, p));
    L.a_off = std::move(a.off);
    L.a_col = std::move(a.col);
    L.a_val = std::move(a.val);
    L.p_off = std::move(p.off);
    L.p_col = std::move(p.col);
    L.p_val = std::move(p.val);
    L.r_off = r.off;
    L.r_col = r.col;
    L.r_val = r.val;
    h.lv.push_back(std::move(L));
    a = std::move(ac);
  }
  // coarsest level: dense inverse of A + alpha 1 1^T
  AmgHostLevel L;
  L.n = a.nr;
  const int32_t nc = a.nr;
  if (nc > 4 * AMG_COARSE) return false;
  std::vector<double> m((size_t)nc * nc, 0.0);
  double dsum = 0.0;
  for (int32_t i = 0; i < nc; ++i)
    for (int32_t j = a.off[i]; j < a.off[i + 1]; ++j) {
      m[(size_t)i * nc + a.col[j]] += a.val[j];
      if (a.col[j] == i) dsum += a.val[j];
    }
  const double alpha = dsum / ((double)nc * nc);
  for (auto &v : m) v += alpha;
  if (!spd_inverse(m, nc)) return false;
  h.cinv = std::move(m);
  h.lv.push_back(std::move(L));
  return true;
}

// Plain-aggregation chain for the elliptic relaxation: the same strength
// rule and greedy aggregates as above, with the tentative prolongator
// (T[i, agg(i)] = 1), so that the Galerkin product T^T A T sums the entries of
// A over pairs of aggregates and the coarse values of every solve are plain
// sums of the finer ones.  The coarser patterns come from the aggregated
// stiffness matrix, whose values also decide the next level's aggregates.
bool agg_chain(int32_t n, const std::vector<int32_t> &off, const std::vector<int32_t> &col,
               const std::vector<double> &val, int32_t max_last, std::vector<AggHostLevel> &lv) {
  lv.clear();
  Csr a;
  a.nr = a.nc = n;
  a.off = off;
  a.col = col;
  a.val = val;
  for (;;) {
    AggHostLevel L;
    L.n = a.nr;
    L.off = a.off;
    L.col = a.col;
    if (a.nr <= max_last || (int)lv.size() + 1 >= ELL_MAXL) {
      lv.push_back(std::move(L));
      return a.nr <= max_last && a.nr > 0;
    }
    std::vector<int32_t> agg;
    const int32_t na = aggregate(a, agg);
    if (na >= a.nr || na < 1) return false;
    L.m_off.assign((size_t)na + 1, 0);
    for (int32_t i = 0; i < a.nr; ++i) L.m_off[agg[i] + 1]++;
    for (int32_t k = 0; k < na; ++k) L.m_off[k + 1] += L.m_off[k];
    L.mem.resize((size_t)a.nr);
    {
      std::vector<int32_t> cur(L.m_off.begin(), L.m_off.end() - 1);
      for (int32_t i = 0; i < a.nr; ++i) L.mem[cur[agg[i]]++] = i;
    }
    // coarse row I: the fine entries of its member rows, grouped by the
    // aggregate of their column
    Csr c;
    c.nr = c.nc = na;
    c.off.assign((size_t)na + 1, 0);
    L.g_off.assign(1, 0);
    std::vector<int32_t> mark((size_t)na, -1), slot((size_t)na, 0), cols;
    std::vector<std::vector<int32_t>> groups;
    for (int32_t I = 0; I < na; ++I) {
      cols.clear();
      for (int32_t m = L.m_off[I]; m < L.m_off[I + 1]; ++m) {
        const int32_t i = L.mem[m];
        for (int32_t j = a.off[i]; j < a.off[i + 1]; ++j) {
          const int32_t J = agg[a.col[j]];
          if (mark[J] != I) {
            mark[J] = I;
            slot[J] = (int32_t)cols.size();
            cols.push_back(J);
            if (groups.size() < cols.size()) groups.emplace_back();
            groups[cols.size() - 1].clear();
          }
          groups[slot[J]].push_back(j);
        }
      }
      std::vector<int32_t> order(cols.size());
      for (size_t k = 0; k < order.size(); ++k) order[k] = (int32_t)k;
      std::sort(order.begin(), order.end(), [&](int32_t u, int32_t v) { return cols[u] < cols[v]; });
      for (const int32_t k : order) {
        std::vector<int32_t> &g = groups[k];
        std::sort(g.begin(), g.end());
        double v = 0.0;
        for (const int32_t j : g) v += a.val[j];
        c.col.push_back(cols[k]);
        c.val.push_back(v);
        L.g_idx.insert(L.g_idx.end(), g.begin(), g.end());
        L.g_off.push_back((int32_t)L.g_idx.size());
      }
      c.off[I + 1] = (int32_t)c.col.size();
    }
    L.agg = std::move(agg);
    lv.push_back(std::move(L));
    a = std::move(c);
  }
}

namespace {

constexpr int AB = 256;

__global__ __launch_bounds__(AB) void k_amg_gather(int32_t n, const int32_t *masters, const double *rin, double *b,
                                                   const int *stop) {
  if (*stop) return;
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) b[k] = rin[masters[k]];
}

__global__ __launch_bounds__(AB) void k_amg_scatter(int32_t n, const int32_t *masters, const double *y, double *zout,
                                                    const int *stop) {
  if (*stop) return;
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) zout[masters[k]] = y[k];
}

// x = omega D^-1 b (one Jacobi step from zero)
__global__ __launch_bounds__(AB) void k_amg_smooth0(int32_t n, double omega, const double *dinv, const double *b,
                                                    double *x, const int *stop) {
  if (*stop) return;
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = omega * dinv[i] * b[i];
}

// Sparse products row by row, G lanes per row (G a power of two near the mean
// row length, chosen on the host): the lanes of a row read consecutive
// entries, then sum their partial products across the group.
template <int G>
__device__ __forceinline__ double row_dot(const int32_t *off, const int32_t *col, const double *val, const double *v,
                                          int32_t i, int g) {
  double s = 0.0;
  for (int32_t j = off[i] + g; j < off[i + 1]; j += G) s += val[j] * v[col[j]];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
  return s;
}

// r = b - A x
template <int G>
__global__ __launch_bounds__(AB) void k_amg_resid(int32_t n, const int32_t *off, const int32_t *col, const double *val,
                                                  const double *b, const double *x, double *r, const int *stop) {
  if (*stop) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t i = (int32_t)(t / G);
  const int g = (int)(t % G);
  if (i >= n) return;
  const double s = row_dot<G>(off, col, val, x, i, g);
  if (g == 0) r[i] = b[i] - s;
}

// y = M v (restriction by P^T)
template <int G>
__global__ __launch_bounds__(AB) void k_amg_spmv(int32_t n, const int32_t *off, const int32_t *col, const double *val,
                                                 const double *v, double *y, const int *stop) {
  if (*stop) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t i = (int32_t)(t / G);
  const int g = (int)(t % G);
  if (i >= n) return;
  const double s = row_dot<G>(off, col, val, v, i, g);
  if (g == 0) y[i] = s;
}

// x += P yc
template <int G>
__global__ __launch_bounds__(AB) void k_amg_prolong(int32_t n, const int32_t *off, const int32_t *col,
                                                    const double *val, const double *yc, double *x, const int *stop) {
  if (*stop) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t i = (int32_t)(t / G);
  const int g = (int)(t % G);
  if (i >= n) return;
  const double s = row_dot<G>(off, col, val, yc, i, g);
  if (g == 0) x[i] += s;
}

// y = x + omega D^-1 (b - A x)
template <int G>
__global__ __launch_bounds__(AB) void k_amg_post(int32_t n, const int32_t *off, const int32_t *col, const double *val,
                                                 double omega, const double *dinv, const double *b, const double *x,
                                                 double *y, const int *stop) {
  if (*stop) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t i = (int32_t)(t / G);
  const int g = (int)(t % G);
  if (i >= n) return;
  const double s = row_dot<G>(off, col, val, x, i, g);
  if (g == 0) y[i] = x[i] + omega * dinv[i] * (b[i] - s);
}

// y = Cinv b on the coarsest level: one wave per row
__global__ __launch_bounds__(64) void k_amg_dense(int32_t n, const double *cinv, const double *b, double *y,
                                                  const int *stop) {
  if (*stop) return;
  const int32_t i = blockIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int32_t j = threadIdx.x; j < n; j += 64) s += cinv[(size_t)i * n + j] * b[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) y[i] = s;
}

inline unsigned blocks(int32_t n) { return (unsigned)((n + AB - 1) / AB); }
inline unsigned blocks_g(int32_t n, int g) { return (unsigned)(((int64_t)n * g + AB - 1) / AB); }

// launch K<G> with the group size g (1, 2, 4, ..., 64)
#define AMG_LAUNCH_G(K, g, n, s, ...)                                                                   \
  do {                                                                                                  \
    switch (g) {                                                                                        \
      case 1: hipLaunchKernelGGL(K<1>, dim3(blocks_g(n, 1)), dim3(AB), 0, s, n, __VA_ARGS__); break;   \
      case 2: hipLaunchKernelGGL(K<2>, dim3(blocks_g(n, 2)), dim3(AB), 0, s, n, __VA_ARGS__); break;   \
      case 4: hipLaunchKernelGGL(K<4>, dim3(blocks_g(n, 4)), dim3(AB), 0, s, n, __VA_ARGS__); break;   \
      case 8: hipLaunchKernelGGL(K<8>, dim3(blocks_g(n, 8)), dim3(AB), 0, s, n, __VA_ARGS__); break;   \
      case 16: hipLaunchKernelGGL(K<16>, dim3(blocks_g(n, 16)), dim3(AB), 0, s, n, __VA_ARGS__); break; \
      case 32: hipLaunchKernelGGL(K<32>, dim3(blocks_g(n, 32)), dim3(AB), 0, s, n, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL(K<64>, dim3(blocks_g(n, 64)), dim3(AB), 0, s, n, __VA_ARGS__); break; \
    }                                                                                                   \
  } while (0)

void vcycle(hipStream_t s, const AmgDev &a, int l, const int *stop) {
  const AmgDevLevel &L = a.lv[l];
  if (l == a.nl - 1) {
    hipLaunchKernelGGL(k_amg_dense, dim3((unsigned)L.n), dim3(64), 0, s, L.n, a.cinv, L.b, L.y, stop);
    return;
  }
  const AmgDevLevel &C = a.lv[l + 1];
  hipLaunchKernelGGL(k_amg_smooth0, dim3(blocks(L.n)), dim3(AB), 0, s, L.n, L.omega, L.dinv, L.b, L.x, stop);
  AMG_LAUNCH_G(k_amg_resid, L.ga, L.n, s, L.a_off, L.a_col, L.a_val, L.b, L.x, L.r, stop);
  AMG_LAUNCH_G(k_amg_spmv, L.gr, C.n, s, L.r_off, L.r_col, L.r_val, L.r, C.b, stop);
  vcycle(s, a, l + 1, stop);
  AMG_LAUNCH_G(k_amg_prolong, L.gp, L.n, s, L.p_off, L.p_col, L.p_val, C.y, L.x, stop);
  AMG_LAUNCH_G(k_amg_post, L.ga, L.n, s, L.a_off, L.a_col, L.a_val, L.omega, L.dinv, L.b, L.x, L.y, stop);
}

}  // namespace

void launch_amg_apply(hipStream_t s, const AmgDev &a, const int32_t *masters, const double *rin, double *zout,
                      const int *stop) {
  const int32_t n0 = a.lv[0].n;
  hipLaunchKernelGGL(k_amg_gather, dim3(blocks(n0)), dim3(AB), 0, s, n0, masters, rin, a.lv[0].b, stop);
  vcycle(s, a, 0, stop);
  hipLaunchKernelGGL(k_amg_scatter, dim3(blocks(n0)), dim3(AB), 0, s, n0, masters, a.lv[0].y, zout, stop);
}

}  // namespace pdfk
