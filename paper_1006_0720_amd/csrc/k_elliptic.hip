// Elliptic relaxation for wp_ij on gfx950 (eq:elliptic-relaxation-Lagrangian
// with eq:L and eq:Cxi; wall condition wp_ij = -4.5 eps n_i n_j): linear
// finite elements on the triangles, all nine components at once, solved by
// preconditioned conjugate gradients warm-started from the previous solution
// (Ch.3, Sec. Solution of the Eulerian equations).  The paper preconditions
// by Jacobi; the default here is one V-cycle of a plain-aggregation
// multigrid hierarchy whose aggregates and patterns are fixed (built once
// from the stiffness matrix over the free masters) and whose values follow
// the matrix of every solve: level 0 copies the free-free block of M + L2 K,
// each coarser level sums the finer entries over pairs of aggregates (the
// Galerkin product with the tentative prolongator), and every level smooths
// with one Jacobi step before and after the coarse correction, its diagonal
// the l1 row sum with the off-diagonal part halved (k_mg_dinv); the last
// level takes a fixed number of such sweeps.  The V-cycle is a fixed
// symmetric positive definite operator, so the iteration stays a conjugate-
// gradient method and converges to the same solution, in several times fewer
// iterations on graded meshes.
//
// Per component c = 3i+j the system over the master nodes is
//   sum_e [M_e + L2_{e,c} K_e] wp_c = sum_e M_e f_c,
// M_e = (A/12)(1 + delta_ab), K_e = A grad N_a . grad N_b, f the local
// right-hand side.  L2_{e,c} = L_ij^2 from the element averages of the nodal
// k and eps, with C_xi,ij = 1 + 1.3 n_i n_j and n the outward normal of the
// no-slip wall edge closest to the element's centroid; L2 = 0 where eps <= 0.
// Rows of nodes on no-slip walls hold the Dirichlet values; the conjugate
// gradients run on the other rows (the search directions vanish on the wall
// rows).  Each solve assembles the CSR values of the mass matrix and of the
// four L2 classes row by row (every master node gathers the elements around
// it, no atomics); the iteration vectors are node-major ([nn][9]) so that a
// column's nine components are one contiguous read; the dot products are
// block sums added with atomics.  With the multigrid the iteration runs on
// compact vectors of the free rows ([n0][9]): the residual of the warm start
// (with the wall columns' Dirichlet values) is formed on the full rows once,
// gathered, and the solution scattered back at the end.
#include <hip/hip_runtime.h>

#include "pdf_solvers.h"

namespace pdfk {

namespace {

constexpr int NB = 256;

// L2 class of component c = 3i+j: C_xi = 1 + 1.3 n_i n_j with n_3 = 0
__device__ __forceinline__ int ell_class(int c) {
  const int i = c / 3, j = c % 3;
  if (i == 2 || j == 2) return 3;
  return i + j;  // (0,0) -> 0, (0,1),(1,0) -> 1, (1,1) -> 2
}

__device__ __forceinline__ double k_of(const double *S, int nn, int q, double k_floor) {
  const double k = 0.5 * (S[5 * nn + q] + S[6 * nn + q] + S[7 * nn + q]);
  return k > k_floor ? k : k_floor;
}

// closest no-slip wall edge to each element's centroid (lowest index on ties)
__global__ __launch_bounds__(NB) void k_ell_normals(MeshDev m, int32_t nw, const double4 *wall, double2 *nrm) {
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.ne) return;
  const ElemGeo g = m.geo[e];
  const double cx = (g.x[0] + g.x[1] + g.x[2]) / 3.0, cy = (g.y[0] + g.y[1] + g.y[2]) / 3.0;
  double best = -1.0;
  int32_t bj = -1;
  for (int32_t j = 0; j < nw; ++j) {
    const double4 w = wall[j];
    const double dx = w.z - w.x, dy = w.w - w.y;
    double t = ((cx - w.x) * dx + (cy - w.y) * dy) / (dx * dx + dy * dy);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    const double ex = cx - (w.x + t * dx), ey = cy - (w.y + t * dy);
    const double d2 = ex * ex + ey * ey;
    if (bj < 0 || d2 < best) {
      best = d2;
      bj = j;
    }
  }
  double2 n = make_double2(0.0, 0.0);
  if (bj >= 0) {
    const double4 w = wall[bj];
    const double dx = w.z - w.x, dy = w.w - w.y, len = sqrt(dx * dx + dy * dy);
    n = make_double2(dy / len, -dx / len);  // the domain lies on the edge's left
  }
  nrm[e] = n;
}

// per element: L_ij^2 for the four C_xi classes
__global__ __launch_bounds__(NB) void k_ell_elem(MeshDev m, ModelDev md, const double *S, const double2 *nrm,
                                                 double4 *L2) {
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.ne) return;
  const int nn = m.nn;
  const int q0 = m.mnode[3 * e], q1 = m.mnode[3 * e + 1], q2 = m.mnode[3 * e + 2];
  double R[3];
  for (int f = 0; f < 3; ++f) R[f] = (S[(5 + f) * nn + q0] + S[(5 + f) * nn + q1] + S[(5 + f) * nn + q2]) / 3.0;
  double k = 0.5 * (R[0] + R[1] + R[2]);
  if (!(k > md.k_floor)) k = md.k_floor;
  const double Om = (S[3 * nn + q0] + S[3 * nn + q1] + S[3 * nn + q2]) / 3.0;
  const double eps = Om * (k + md.nu * md.CT * md.CT * Om);
  double4 out = make_double4(0.0, 0.0, 0.0, 0.0);
  if (eps > 0.0) {
    const double2 n = nrm[e];
    const double kolm = md.Ceta * pow(md.nu * md.nu * md.nu / eps, 0.25);
    const double turb = k * sqrt(k) / eps;
    const double cx[4] = {1.0 + 1.3 * n.x * n.x, 1.0 + 1.3 * n.x * n.y, 1.0 + 1.3 * n.y * n.y, 1.0};
    double l2[4];
    for (int c = 0; c < 4; ++c) {
      const double t = cx[c] * turb;
      const double L = md.CL * (t > kolm ? t : kolm);
      l2[c] = L * L;
    }
    out = make_double4(l2[0], l2[1], l2[2], l2[3]);
  }
  L2[e] = out;
}

// element mass (A/12)(1 + delta) and stiffness A grad N_a . grad N_b
__device__ __forceinline__ double elem_area(const ElemGeo &g) {
  return 0.5 * ((g.x[1] - g.x[0]) * (g.y[2] - g.y[0]) - (g.x[2] - g.x[0]) * (g.y[1] - g.y[0]));
}

// class value of a double4 row; only with a class known at compile time (the
// unrolled per-row loops below), see cls_at for lane-varying classes
__device__ __forceinline__ double l2_of(const double4 &v, int cls) {
  return cls == 0 ? v.x : (cls == 1 ? v.y : (cls == 2 ? v.z : v.w));
}

// the CSR values of row a (a master node): the mass matrix and, for the four
// L2 classes, M + L2 K, gathered from the elements around a (the row is this
// thread's alone, so no atomics)
__global__ __launch_bounds__(NB) void k_ell_assemble(MeshDev m, const double4 *L2, const int32_t *row_off,
                                                     const int32_t *cols, double *mv, double4 *av) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_masters) return;
  const int32_t a = m.masters[t];
  const int32_t j0 = row_off[a], j1 = row_off[a + 1];
  for (int32_t j = j0; j < j1; ++j) {
    mv[j] = 0.0;
    av[j] = make_double4(0.0, 0.0, 0.0, 0.0);
  }
  for (int32_t i = m.m2e_off[a]; i < m.m2e_off[a + 1]; ++i) {
    const int32_t e = m.m2e[i];
    const ElemGeo g = m.geo[e];
    const double A = elem_area(g);
    const double *d = m.dN + 6 * (size_t)e;
    const double4 l2 = L2[e];
    const int32_t qk[3] = {m.mnode[3 * e], m.mnode[3 * e + 1], m.mnode[3 * e + 2]};
    for (int la = 0; la < 3; ++la) {
      if (qk[la] != a) continue;
      for (int lb = 0; lb < 3; ++lb) {
        int32_t j = j0;
        while (j + 1 < j1 && cols[j] != qk[lb]) ++j;  // the column is in the row by construction
        const double M = A / 12.0 * (la == lb ? 2.0 : 1.0);
        const double K = A * (d[la] * d[lb] + d[3 + la] * d[3 + lb]);
        mv[j] += M;
        double4 v = av[j];
        v.x += M + l2.x * K;
        v.y += M + l2.y * K;
        v.z += M + l2.z * K;
        v.w += M + l2.w * K;
        av[j] = v;
      }
    }
  }
}

__device__ __forceinline__ void block_add9(const double v[9], double *dst) {
  __shared__ double red[NB / 64][9];
  for (int c = 0; c < 9; ++c) {
    double s = v[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = s;
  }
  __syncthreads();
  if (threadIdx.x < 9) {
    double s = 0.0;
    for (int w = 0; w < NB / 64; ++w) s += red[w][threadIdx.x];
    atomicAdd(&dst[threadIdx.x], s);
  }
}

// the vectors of the iteration are node-major, [nn][9]
// wall rows: the Dirichlet values in x, zero residual and direction, unit
// diagonal
__global__ __launch_bounds__(NB) void k_ell_start(MeshDev m, ModelDev md, const double *S, const int8_t *dir,
                                                  const double2 *dnv, double *x, double *r, double *z, double *p,
                                                  double *diag) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_masters) return;
  const int nn = m.nn;
  const int32_t a = m.masters[t];
  if (dir[a] == 0) return;
  const double k = k_of(S, nn, a, md.k_floor);
  const double Om = S[3 * nn + a];
  const double eps = Om * (k + md.nu * md.CT * md.CT * Om);
  const double n[3] = {dnv[a].x, dnv[a].y, 0.0};
  for (int c = 0; c < 9; ++c) {
    const size_t o = 9 * (size_t)a + c;
    x[o] = -4.5 * eps * n[c / 3] * n[c % 3];
    r[o] = z[o] = p[o] = 0.0;
    diag[o] = 1.0;
  }
}

// b = M f, r = b - A x, z = r / diag, p = z on the free rows (every x, wall
// rows included, in place); rz0 += r.z, bb += b.(b / diag)
__global__ __launch_bounds__(NB) void k_ell_resid(MeshDev m, const double *f, const int8_t *dir,
                                                  const int32_t *row_off, const int32_t *cols, const double *mv,
                                                  const double4 *av, const double *x, double *r, double *z,
                                                  double *p, double *diag, double *rz0, double *bb) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  double part[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, pb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (t < m.n_masters) {
    const int nn = m.nn;
    const int32_t a = m.masters[t];
    if (dir[a] == 0) {
      double b[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ax[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, dg[9];
      for (int32_t j = row_off[a]; j < row_off[a + 1]; ++j) {
        const int32_t q = cols[j];
        const double M = mv[j];
        const double4 v = av[j];
        const double *xq = x + 9 * (size_t)q;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const double A = l2_of(v, ell_class(c));
          b[c] += M * f[(size_t)c * nn + q];
          ax[c] += A * xq[c];
          if (q == a) dg[c] = A;
        }
      }
      for (int c = 0; c < 9; ++c) {
        const size_t o = 9 * (size_t)a + c;
        const double rr = b[c] - ax[c];
        const double zz = rr / dg[c];
        r[o] = rr;
        z[o] = zz;
        p[o] = zz;
        diag[o] = dg[c];
        part[c] = rr * zz;
        pb[c] = b[c] * b[c] / dg[c];
      }
    }
  }
  block_add9(part, rz0);
  __syncthreads();
  block_add9(pb, bb);
}

// q = A p on the free rows; pq += p.q
__global__ __launch_bounds__(NB) void k_ell_apply(MeshDev m, const int8_t *dir, const int32_t *row_off,
                                                  const int32_t *cols, const double4 *av, const double *p, double *q,
                                                  double *pq, const int *stop) {
  if (*stop) return;
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  double part[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (t < m.n_masters) {
    const int32_t a = m.masters[t];
    double y[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (dir[a] == 0) {
      for (int32_t j = row_off[a]; j < row_off[a + 1]; ++j) {
        const double4 v = av[j];
        const double *pq_ = p + 9 * (size_t)cols[j];
        const double cl[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int c = 0; c < 9; ++c) y[c] += cl[ell_class(c)] * pq_[c];
      }
      for (int c = 0; c < 9; ++c) part[c] = p[9 * (size_t)a + c] * y[c];
    }
    for (int c = 0; c < 9; ++c) q[9 * (size_t)a + c] = y[c];
  }
  block_add9(part, pq);
}

// x += alpha p, r -= alpha q, z = r / diag; rz_next += r.z.  Over the vector
// entries (node-major: entry i is node i / 9, component i % 9) with a grid-
// stride loop whose block size and stride are multiples of 9, so that a thread
// keeps one component, every access is coalesced, and each block adds nine
// sums; only the free rows (role 0) change
constexpr int NB9 = 252;

__global__ __launch_bounds__(NB9) void k_ell_update(int64_t n9, const int8_t *role, const double *p, const double *q,
                                                    const double *diag, double *x, double *r, double *z,
                                                    const double *rz, const double *pq, double *rz_next,
                                                    const int *stop) {
  if (*stop) return;
  __shared__ double part[NB9];
  const int c = threadIdx.x % 9;
  const double alpha = (pq[c] != 0.0) ? rz[c] / pq[c] : 0.0;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NB9 + threadIdx.x; i < n9; i += (int64_t)gridDim.x * NB9) {
    if (role[i / 9] != 0) continue;
    x[i] += alpha * p[i];
    const double rr = r[i] - alpha * q[i];
    r[i] = rr;
    const double zz = rr / diag[i];
    z[i] = zz;
    acc += rr * zz;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < 9) {
    double sum = 0.0;
    for (int k = threadIdx.x; k < NB9; k += 9) sum += part[k];
    atomicAdd(&rz_next[threadIdx.x], sum);
  }
}

// p = z + beta p with beta = rz_next / rz, per entry
__global__ __launch_bounds__(NB) void k_ell_dir(int64_t n9, const int8_t *role, const double *z, double *p,
                                                const double *rz, const double *rz_next, const int *stop) {
  if (*stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n9 || role[i / 9] != 0) return;
  const int c = (int)(i % 9);
  const double beta = (rz[c] != 0.0) ? rz_next[c] / rz[c] : 0.0;
  p[i] = z[i] + beta * p[i];
}

// stop once every component's preconditioned residual r.D^-1 r is below tol^2
// times that of its right-hand side (or vanished); stop = iterations + 1
__global__ void k_ell_check(const double *bb, const double *rz, double tol2, int iters, int *stop) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || *stop) return;
  bool done = true;
  for (int c = 0; c < 9; ++c) done = done && !(rz[c] > tol2 * bb[c]);
  if (done) *stop = iters + 1;
}

// node-major x to the component-major wp, masters then their identified nodes
__global__ __launch_bounds__(NB) void k_ell_out(MeshDev m, const double *x, double *wp) {
  const int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= m.nn) return;
  const int32_t q = m.master[n];
  for (int c = 0; c < 9; ++c) wp[(size_t)c * m.nn + n] = x[9 * (size_t)q + c];
}

// component-major warm start to node-major (masters)
__global__ __launch_bounds__(NB) void k_ell_in(MeshDev m, const double *wp, double *x) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_masters) return;
  const int32_t a = m.masters[t];
  for (int c = 0; c < 9; ++c) x[9 * (size_t)a + c] = wp[(size_t)c * m.nn + a];
}

// ---- plain-aggregation multigrid preconditioner (EllMg) ----
// One thread per (row, component) on every level: consecutive threads read
// consecutive components of a row, so the [n][9] vectors are read coalesced.
//
// Kernels whose lanes take different components read a class value by its
// address, one 8-byte load at element k of the double4 row.  Selecting among
// the loaded members by a lane-varying class (a chain of conditionals) was
// compiled into branches that pick a load address, and lanes of class 3 kept
// the class-1 address: the wrong matrix value, found against a host product.
__device__ __forceinline__ double cls_at(const double4 *a, size_t i, int k) { return ((const double *)(a + i))[k]; }

// the next level's values: sums of this level's (the Galerkin product with the
// tentative prolongator)
__global__ __launch_bounds__(NB) void k_mg_vals(int32_t nnzc, const int32_t *g_off, const int32_t *g_idx,
                                                const double4 *vf, double4 *vc) {
  const int32_t J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= nnzc) return;
  double4 s = make_double4(0.0, 0.0, 0.0, 0.0);
  for (int32_t k = g_off[J]; k < g_off[J + 1]; ++k) {
    const double4 v = vf[g_idx[k]];
    s.x += v.x;
    s.y += v.y;
    s.z += v.z;
    s.w += v.w;
  }
  vc[J] = s;
}

// the smoother's diagonal per class: d_i = a_ii + (1/2) sum_{j != i} |a_ij|
// (l1-Jacobi with the off-diagonal sum halved).  For a symmetric matrix with
// a positive diagonal, 2 D - A then has the diagonal a_ii + sum_{j != i}
// |a_ij| and is diagonally dominant, so the smoothing step converges in the
// energy norm and the V-cycle stays symmetric positive definite, with no
// spectral estimate; with the full l1 sum (weight 1 instead of 1/2) the
// step is damped more and the conjugate gradients take 12-16 % more
// iterations (23.8 against 20.6 per solve on the 1M-triangle graded channel,
// 27 against 24 on a 5913-node channel).  A row without a positive diagonal
// entry keeps the full l1 sum.
__device__ __forceinline__ double half_l1(double diag, double l1) {
  return diag > 0.0 ? 0.5 * (diag + l1) : l1;
}
__global__ __launch_bounds__(NB) void k_mg_dinv(int32_t n, const int32_t *off, const int32_t *col, const double4 *val,
                                                double4 *dinv) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double4 s = make_double4(0.0, 0.0, 0.0, 0.0), dg = make_double4(0.0, 0.0, 0.0, 0.0);
  for (int32_t j = off[i]; j < off[i + 1]; ++j) {
    const double4 v = val[j];
    s.x += fabs(v.x);
    s.y += fabs(v.y);
    s.z += fabs(v.z);
    s.w += fabs(v.w);
    if (col[j] == i) dg = v;
  }
  dinv[i] = make_double4(1.0 / half_l1(dg.x, s.x), 1.0 / half_l1(dg.y, s.y), 1.0 / half_l1(dg.z, s.z),
                         1.0 / half_l1(dg.w, s.w));
}

// the pre-smoothing step from zero folded into the residual: r = b - A (D^-1 b)
__global__ __launch_bounds__(NB) void k_mg_pre(int32_t n, const int32_t *off, const int32_t *col,
                                               const double4 *val, const double4 *dinv, const double *b, double *r,
                                               const int *stop) {
  if (*stop) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * (int64_t)n) return;
  const int32_t i = (int32_t)(t / 9);
  const int c = (int)(t - 9 * (int64_t)i);
  const int k = ell_class(c);
  double s = 0.0;
  for (int32_t j = off[i]; j < off[i + 1]; ++j) {
    const int32_t q = col[j];
    s += cls_at(val, j, k) * (cls_at(dinv, q, k) * b[9 * (size_t)q + c]);
  }
  r[t] = b[t] - s;
}

// the coarse correction folded into the post-smoothing step:
// x = D^-1 b + T yc, y = x + D^-1 (b - A x)
__global__ __launch_bounds__(NB) void k_mg_post(int32_t n, const int32_t *off, const int32_t *col,
                                                const double4 *val, const double4 *dinv, const int32_t *agg,
                                                const double *yc, const double *b, double *y, const int *stop) {
  if (*stop) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * (int64_t)n) return;
  const int32_t i = (int32_t)(t / 9);
  const int c = (int)(t - 9 * (int64_t)i);
  const int k = ell_class(c);
  double s = 0.0;
  for (int32_t j = off[i]; j < off[i + 1]; ++j) {
    const int32_t q = col[j];
    s += cls_at(val, j, k) * (cls_at(dinv, q, k) * b[9 * (size_t)q + c] + yc[9 * (size_t)agg[q] + c]);
  }
  const double di = cls_at(dinv, i, k);
  const double x = di * b[t] + yc[9 * (size_t)agg[i] + c];
  y[t] = x + di * (b[t] - s);
}

// bc = T^T r: the sum over each aggregate's rows
__global__ __launch_bounds__(NB) void k_mg_restrict(int32_t nc, const int32_t *m_off, const int32_t *mem,
                                                    const double *r, double *bc, const int *stop) {
  if (*stop) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * (int64_t)nc) return;
  const int32_t I = (int32_t)(t / 9);
  const int c = (int)(t - 9 * (int64_t)I);
  double s = 0.0;
  for (int32_t m = m_off[I]; m < m_off[I + 1]; ++m) s += r[9 * (size_t)mem[m] + c];
  bc[t] = s;
}


// the last level: `sweeps` smoothing sweeps from zero, in one workgroup,
// the iterate in LDS (n <= ELL_COARSE_MAX)
constexpr int NBC = 1024;
constexpr int CQ = (9 * ELL_COARSE_MAX + NBC - 1) / NBC;
__global__ __launch_bounds__(NBC) void k_mg_coarse(int32_t n, const int32_t *off, const int32_t *col,
                                                   const double4 *val, const double4 *dinv, const double *b,
                                                   double *y, int sweeps, const int *stop) {
  if (*stop) return;
  __shared__ double xs[9 * ELL_COARSE_MAX];
  const int32_t n9 = 9 * n;
  double nx[CQ];
  for (int32_t t = threadIdx.x; t < n9; t += NBC) {
    const int32_t i = t / 9;
    xs[t] = cls_at(dinv, i, ell_class(t - 9 * i)) * b[t];
  }
  __syncthreads();
  for (int sw = 1; sw < sweeps; ++sw) {
#pragma unroll
    for (int q = 0; q < CQ; ++q) {
      const int32_t t = threadIdx.x + q * NBC;
      if (t < n9) {
        const int32_t i = t / 9;
        const int c = t - 9 * i;
        const int k = ell_class(c);
        double s = 0.0;
        for (int32_t j = off[i]; j < off[i + 1]; ++j) s += cls_at(val, j, k) * xs[9 * col[j] + c];
        nx[q] = xs[t] + cls_at(dinv, i, k) * (b[t] - s);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CQ; ++q) {
      const int32_t t = threadIdx.x + q * NBC;
      if (t < n9) xs[t] = nx[q];
    }
    __syncthreads();
  }
  for (int32_t t = threadIdx.x; t < n9; t += NBC) y[t] = xs[t];
}

inline unsigned g9(int32_t n) { return (unsigned)((9 * (int64_t)n + NB - 1) / NB); }

void mg_vcycle(hipStream_t s, const EllMg &g, int l, const int *stop) {
  const EllMgLevel &L = g.lv[l];
  if (l == g.nl - 1) {
    hipLaunchKernelGGL(k_mg_coarse, dim3(1), dim3(NBC), 0, s, L.n, L.off, L.col, L.val, L.dinv, L.b, L.y, g.sweeps,
                       stop);
    return;
  }
  const EllMgLevel &C = g.lv[l + 1];
  hipLaunchKernelGGL(k_mg_pre, dim3(g9(L.n)), dim3(NB), 0, s, L.n, L.off, L.col, L.val, L.dinv, L.b, L.r, stop);
  hipLaunchKernelGGL(k_mg_restrict, dim3(g9(C.n)), dim3(NB), 0, s, C.n, L.m_off, L.mem, L.r, C.b, stop);
  mg_vcycle(s, g, l + 1, stop);
  hipLaunchKernelGGL(k_mg_post, dim3(g9(L.n)), dim3(NB), 0, s, L.n, L.off, L.col, L.val, L.dinv, L.agg, C.y, L.b,
                     L.y, stop);
}

// ---- the conjugate gradients on compact free-row vectors ([n0][9]) ----
// level 0 is the free-free block of the matrix, its values gathered from the
// full matrix every solve; the CG kernels take one thread per (row,
// component) with block sizes and strides that are multiples of 9, so a
// thread keeps one component and the dot products add nine block sums

__global__ __launch_bounds__(NB) void k_c_vals0(int32_t nnz, const int32_t *g0, const double4 *av, double4 *val) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nnz) val[j] = av[g0[j]];
}

// compact residual, right-hand side and iterate from the full vectors
__global__ __launch_bounds__(NB) void k_c_gather(int32_t n0, const int32_t *fidx, const double *r, const double *q,
                                                 const double *x, double *cr, double *cb, double *cx) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * (int64_t)n0) return;
  const int32_t k = (int32_t)(t / 9);
  const size_t o = 9 * (size_t)fidx[k] + (size_t)(t - 9 * (int64_t)k);
  cr[t] = r[o];
  cb[t] = q[o];
  cx[t] = x[o];
}

__global__ __launch_bounds__(NB) void k_c_scatter(int32_t n0, const int32_t *fidx, const double *cx, double *x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * (int64_t)n0) return;
  const int32_t k = (int32_t)(t / 9);
  x[9 * (size_t)fidx[k] + (size_t)(t - 9 * (int64_t)k)] = cx[t];
}

// the nine per-component sums of a block of NB9 threads added to out
__device__ __forceinline__ void add9(double acc, double *out) {
  __shared__ double part[NB9];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < 9) {
    double sum = 0.0;
    for (int k = threadIdx.x; k < NB9; k += 9) sum += part[k];
    atomicAdd(&out[threadIdx.x], sum);
  }
}

// q = A p, pq += p.q
__global__ __launch_bounds__(NB9) void k_c_apply(int32_t n0, const int32_t *off, const int32_t *col,
                                                 const double4 *val, const double *p, double *q, double *pq,
                                                 const int *stop) {
  if (*stop) return;
  const int c = threadIdx.x % 9;
  const int k = ell_class(c);
  double acc = 0.0;
  const int64_t n9 = 9 * (int64_t)n0;
  for (int64_t t = (int64_t)blockIdx.x * NB9 + threadIdx.x; t < n9; t += (int64_t)gridDim.x * NB9) {
    const int32_t i = (int32_t)(t / 9);
    double y = 0.0;
    for (int32_t j = off[i]; j < off[i + 1]; ++j) y += cls_at(val, j, k) * p[9 * (size_t)col[j] + c];
    q[t] = y;
    acc += p[t] * y;
  }
  add9(acc, pq);
}

// x += alpha p, r -= alpha q
__global__ __launch_bounds__(NB9) void k_c_update(int64_t n9, const double *p, const double *q, double *x, double *r,
                                                  const double *rz, const double *pq, const int *stop) {
  if (*stop) return;
  const int c = threadIdx.x % 9;
  const double alpha = (pq[c] != 0.0) ? rz[c] / pq[c] : 0.0;
  for (int64_t t = (int64_t)blockIdx.x * NB9 + threadIdx.x; t < n9; t += (int64_t)gridDim.x * NB9) {
    x[t] += alpha * p[t];
    r[t] -= alpha * q[t];
  }
}

// p = z + beta p, beta = rzn / rz (rz null: p = z)
__global__ __launch_bounds__(NB9) void k_c_dir(int64_t n9, const double *z, double *p, const double *rz,
                                               const double *rzn, const int *stop) {
  if (*stop) return;
  const int c = threadIdx.x % 9;
  const double beta = (rz && rz[c] != 0.0) ? rzn[c] / rz[c] : 0.0;
  for (int64_t t = (int64_t)blockIdx.x * NB9 + threadIdx.x; t < n9; t += (int64_t)gridDim.x * NB9)
    p[t] = rz ? z[t] + beta * p[t] : z[t];
}

// level 0's post-smoothing with the coarse correction folded in (yc null: no
// coarser level) and the dot product: x = D^-1 b + T yc,
// y = x + D^-1 (b - A x), dot += b.y
__global__ __launch_bounds__(NB9) void k_c_post0(int32_t n0, const int32_t *off, const int32_t *col,
                                                 const double4 *val, const double4 *dinv, const int32_t *agg,
                                                 const double *yc, const double *b, double *y, double *dot,
                                                 const int *stop) {
  if (*stop) return;
  const int c = threadIdx.x % 9;
  const int k = ell_class(c);
  double acc = 0.0;
  const int64_t n9 = 9 * (int64_t)n0;
  for (int64_t t = (int64_t)blockIdx.x * NB9 + threadIdx.x; t < n9; t += (int64_t)gridDim.x * NB9) {
    const int32_t i = (int32_t)(t / 9);
    double s = 0.0;
    for (int32_t j = off[i]; j < off[i + 1]; ++j) {
      const int32_t q = col[j];
      const double xq = cls_at(dinv, q, k) * b[9 * (size_t)q + c] + (yc ? yc[9 * (size_t)agg[q] + c] : 0.0);
      s += cls_at(val, j, k) * xq;
    }
    const double di = cls_at(dinv, i, k);
    const double xa = di * b[t] + (yc ? yc[9 * (size_t)agg[i] + c] : 0.0);
    const double ya = xa + di * (b[t] - s);
    y[t] = ya;
    acc += b[t] * ya;
  }
  add9(acc, dot);
}

// z = V-cycle of r (compact), dot += r.z
void mg_apply(hipStream_t s, const EllMg &g, const double *r, double *z, double *dot, const int *stop) {
  const EllMgLevel &L0 = g.lv[0];
  const int64_t gp = (9 * (int64_t)L0.n + NB9 - 1) / NB9;
  const unsigned gpost = (unsigned)(gp < 2048 ? gp : 2048);
  if (g.nl > 1) {
    const EllMgLevel &C = g.lv[1];
    hipLaunchKernelGGL(k_mg_pre, dim3(g9(L0.n)), dim3(NB), 0, s, L0.n, L0.off, L0.col, L0.val, L0.dinv, r, L0.r,
                       stop);
    hipLaunchKernelGGL(k_mg_restrict, dim3(g9(C.n)), dim3(NB), 0, s, C.n, L0.m_off, L0.mem, L0.r, C.b, stop);
    mg_vcycle(s, g, 1, stop);
    hipLaunchKernelGGL(k_c_post0, dim3(gpost), dim3(NB9), 0, s, L0.n, L0.off, L0.col, L0.val, L0.dinv, L0.agg,
                       (const double *)C.y, r, z, dot, stop);
  } else {
    // a single level: two smoothing steps from zero
    hipLaunchKernelGGL(k_c_post0, dim3(gpost), dim3(NB9), 0, s, L0.n, L0.off, L0.col, L0.val, L0.dinv,
                       (const int32_t *)nullptr, (const double *)nullptr, r, z, dot, stop);
  }
}

// the hierarchy's values for this solve
void mg_values(hipStream_t s, const EllMg &g, const double4 *av) {
  const EllMgLevel &L0 = g.lv[0];
  hipLaunchKernelGGL(k_c_vals0, dim3((L0.nnz + NB - 1) / NB), dim3(NB), 0, s, L0.nnz, g.g0, av, L0.val);
  for (int l = 0; l < g.nl; ++l) {
    const EllMgLevel &L = g.lv[l];
    if (l + 1 < g.nl) {
      const EllMgLevel &C = g.lv[l + 1];
      hipLaunchKernelGGL(k_mg_vals, dim3((C.nnz + NB - 1) / NB), dim3(NB), 0, s, C.nnz, L.g_off, L.g_idx, L.val,
                         C.val);
    }
    hipLaunchKernelGGL(k_mg_dinv, dim3((L.n + NB - 1) / NB), dim3(NB), 0, s, L.n, L.off, L.col, L.val, L.dinv);
  }
}

// multigrid start: b of the free rows into q, r = b - A x (x holds the wall
// values), z and the other vectors zero elsewhere
__global__ __launch_bounds__(NB) void k_ell_resid_mg(MeshDev m, const double *f, const int8_t *dir,
                                                     const int32_t *row_off, const int32_t *cols, const double *mv,
                                                     const double4 *av, const double *x, double *r, double *q) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_masters) return;
  const int nn = m.nn;
  const int32_t a = m.masters[t];
  if (dir[a] != 0) return;
  double b[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ax[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int32_t j = row_off[a]; j < row_off[a + 1]; ++j) {
    const int32_t qn = cols[j];
    const double M = mv[j];
    const double4 v = av[j];
    const double *xq = x + 9 * (size_t)qn;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      b[c] += M * f[(size_t)c * nn + qn];
      ax[c] += l2_of(v, ell_class(c)) * xq[c];
    }
  }
  for (int c = 0; c < 9; ++c) {
    r[9 * (size_t)a + c] = b[c] - ax[c];
    q[9 * (size_t)a + c] = b[c];
  }
}




}  // namespace

void launch_ell_normals(hipStream_t s, const MeshDev &m, int32_t nw, const double4 *wall, double2 *nrm) {
  hipLaunchKernelGGL(k_ell_normals, dim3((m.ne + NB - 1) / NB), dim3(NB), 0, s, m, nw, wall, nrm);
}

int launch_ell_solve(hipStream_t s, const MeshDev &m, const ModelDev &md, const EllBuf &b, const double *S,
                     const double *f, double *wp, double tol, int maxit) {
  const unsigned gm = (unsigned)((m.n_masters + NB - 1) / NB);
  const unsigned ge = (unsigned)((m.ne + NB - 1) / NB);
  const unsigned gn = (unsigned)((m.nn + NB - 1) / NB);
  const int64_t n9 = 9 * (int64_t)m.nn;
  const unsigned gn9 = (unsigned)((n9 + NB - 1) / NB);
  const int64_t gu_ = (n9 + NB9 - 1) / NB9;
  const unsigned gu = (unsigned)(gu_ < 2048 ? gu_ : 2048);
  // scal: [0, 9) rz0, [9, 18) bb, then per iteration k: pq at 18 + 18k, the
  // next rz at 27 + 18k
  (void)hipMemsetAsync(b.scal, 0, (size_t)(18 * (maxit + 1)) * sizeof(double), s);
  (void)hipMemsetAsync(b.stop, 0, sizeof(int), s);
  hipLaunchKernelGGL(k_ell_elem, dim3(ge), dim3(NB), 0, s, m, md, S, b.nrm, b.L2);
  hipLaunchKernelGGL(k_ell_assemble, dim3(gm), dim3(NB), 0, s, m, b.L2, b.row_off, b.cols, b.mv, b.av);
  hipLaunchKernelGGL(k_ell_in, dim3(gm), dim3(NB), 0, s, m, wp, b.x);
  hipLaunchKernelGGL(k_ell_start, dim3(gm), dim3(NB), 0, s, m, md, S, b.dir, b.dnv, b.x, b.r, b.z, b.p, b.diag);
  const bool mg = b.mg.nl > 0;
  const double *rz0 = b.scal, *bb = b.scal + 9;
  const EllMg &g = b.mg;
  const int32_t n0 = mg ? g.lv[0].n : 0;
  const int64_t c9 = 9 * (int64_t)n0;
  const int64_t gc_ = (c9 + NB9 - 1) / NB9;
  const unsigned gc = (unsigned)(gc_ < 2048 ? (gc_ > 0 ? gc_ : 1) : 2048);
  if (mg) {
    // the stopping rule measures residuals in the preconditioner's norm:
    // r.M r against b.M b (M the V-cycle)
    mg_values(s, g, b.av);
    hipLaunchKernelGGL(k_ell_resid_mg, dim3(gm), dim3(NB), 0, s, m, f, b.dir, b.row_off, b.cols, b.mv, b.av, b.x,
                       b.r, b.q);
    hipLaunchKernelGGL(k_c_gather, dim3(g9(n0)), dim3(NB), 0, s, n0, g.fidx, b.r, b.q, b.x, g.cr, g.cb, g.cx);
    mg_apply(s, g, g.cb, g.cz, b.scal + 9, b.stop);
    mg_apply(s, g, g.cr, g.cz, b.scal, b.stop);
    hipLaunchKernelGGL(k_c_dir, dim3(gc), dim3(NB9), 0, s, c9, g.cz, g.cp, (const double *)nullptr,
                       (const double *)nullptr, b.stop);
  } else {
    hipLaunchKernelGGL(k_ell_resid, dim3(gm), dim3(NB), 0, s, m, f, b.dir, b.row_off, b.cols, b.mv, b.av, b.x, b.r,
                       b.z, b.p, b.diag, b.scal, b.scal + 9);
  }
  hipLaunchKernelGGL(k_ell_check, dim3(1), dim3(64), 0, s, bb, rz0, tol * tol, 0, b.stop);
  int it = 0;
  int stop_host = 0;
  while (it < maxit && !stop_host) {
    const int chunk = (maxit - it) < 8 ? (maxit - it) : 8;
    for (int j = 0; j < chunk; ++j, ++it) {
      const double *rz = it == 0 ? rz0 : b.scal + 27 + 18 * (it - 1);
      double *pq = b.scal + 18 + 18 * it;
      double *rzn = b.scal + 27 + 18 * it;
      if (mg) {
        const EllMgLevel &L0 = g.lv[0];
        hipLaunchKernelGGL(k_c_apply, dim3(gc), dim3(NB9), 0, s, n0, L0.off, L0.col, L0.val, g.cp, g.cq, pq, b.stop);
        hipLaunchKernelGGL(k_c_update, dim3(gc), dim3(NB9), 0, s, c9, g.cp, g.cq, g.cx, g.cr, rz, pq, b.stop);
        mg_apply(s, g, g.cr, g.cz, rzn, b.stop);
        hipLaunchKernelGGL(k_ell_check, dim3(1), dim3(64), 0, s, bb, rzn, tol * tol, it + 1, b.stop);
        hipLaunchKernelGGL(k_c_dir, dim3(gc), dim3(NB9), 0, s, c9, g.cz, g.cp, rz, rzn, b.stop);
      } else {
        hipLaunchKernelGGL(k_ell_apply, dim3(gm), dim3(NB), 0, s, m, b.dir, b.row_off, b.cols, b.av, b.p, b.q, pq,
                           b.stop);
        hipLaunchKernelGGL(k_ell_update, dim3(gu), dim3(NB9), 0, s, n9, b.dir, b.p, b.q, b.diag, b.x, b.r, b.z, rz,
                           pq, rzn, b.stop);
        hipLaunchKernelGGL(k_ell_check, dim3(1), dim3(64), 0, s, bb, rzn, tol * tol, it + 1, b.stop);
        hipLaunchKernelGGL(k_ell_dir, dim3(gn9), dim3(NB), 0, s, n9, b.dir, b.z, b.p, rz, rzn, b.stop);
      }
    }
    (void)hipMemcpyAsync(&stop_host, b.stop, sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
  }
  if (mg) hipLaunchKernelGGL(k_c_scatter, dim3(g9(n0)), dim3(NB), 0, s, n0, g.fidx, g.cx, b.x);
  hipLaunchKernelGGL(k_ell_out, dim3(gn), dim3(NB), 0, s, m, b.x, wp);
  return stop_host > 0 ? stop_host - 1 : it;
}

}  // namespace pdfk
