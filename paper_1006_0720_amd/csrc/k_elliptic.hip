// Elliptic relaxation for wp_ij on gfx950 (eq:elliptic-relaxation-Lagrangian
// with eq:L and eq:Cxi; wall condition wp_ij = -4.5 eps n_i n_j): linear
// finite elements on the triangles, all nine components at once, solved by
// Jacobi-preconditioned conjugate gradients warm-started from the previous
// solution (Ch.3, Sec. Solution of the Eulerian equations).
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
// block sums added with atomics.
#include <hip/hip_runtime.h>

#include "pdf_internal.h"

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
  const unsigned g9 = (unsigned)((n9 + NB - 1) / NB);
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
  hipLaunchKernelGGL(k_ell_resid, dim3(gm), dim3(NB), 0, s, m, f, b.dir, b.row_off, b.cols, b.mv, b.av, b.x, b.r,
                     b.z, b.p, b.diag, b.scal, b.scal + 9);
  const double *rz0 = b.scal, *bb = b.scal + 9;
  hipLaunchKernelGGL(k_ell_check, dim3(1), dim3(64), 0, s, bb, rz0, tol * tol, 0, b.stop);
  int it = 0;
  int stop_host = 0;
  while (it < maxit && !stop_host) {
    const int chunk = (maxit - it) < 8 ? (maxit - it) : 8;
    for (int j = 0; j < chunk; ++j, ++it) {
      const double *rz = it == 0 ? rz0 : b.scal + 27 + 18 * (it - 1);
      double *pq = b.scal + 18 + 18 * it;
      double *rzn = b.scal + 27 + 18 * it;
      hipLaunchKernelGGL(k_ell_apply, dim3(gm), dim3(NB), 0, s, m, b.dir, b.row_off, b.cols, b.av, b.p, b.q, pq,
                         b.stop);
      hipLaunchKernelGGL(k_ell_update, dim3(gu), dim3(NB9), 0, s, n9, b.dir, b.p, b.q, b.diag, b.x, b.r, b.z, rz,
                         pq, rzn, b.stop);
      hipLaunchKernelGGL(k_ell_check, dim3(1), dim3(64), 0, s, bb, rzn, tol * tol, it + 1, b.stop);
      hipLaunchKernelGGL(k_ell_dir, dim3(g9), dim3(NB), 0, s, n9, b.dir, b.z, b.p, rz, rzn, b.stop);
    }
    (void)hipMemcpyAsync(&stop_host, b.stop, sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
  }
  hipLaunchKernelGGL(k_ell_out, dim3(gn), dim3(NB), 0, s, m, b.x, wp);
  return stop_host > 0 ? stop_host - 1 : it;
}

}  // namespace pdfk
