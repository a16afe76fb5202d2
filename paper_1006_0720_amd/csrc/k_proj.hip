// Stabilized mean-pressure projection on gfx950 (Ch.3, Sec. Solution of the
// Eulerian equations: eq:pressure-projection-smooth, eq:velocity-correction).
//
// With rho = 1 and P = x.G + P' (G the imposed gradient, P' solved), per step
// after the velocity prediction and its estimate <U>*:
//   K dP = -(d + C_p K P') / dt + (C_p/dt) B(g^n - G.n) + B(g^{n+1} - g^n),
// d_a = sum_e (A_e / 3) div_e(<U>*), K the stiffness matrix over the master
// nodes (CSR, assembled once).  g is the wall datum of eq:wall-pressure-
// condition, dP/dn = nu lap<U_i> n_i - d<u_i u_j>/dx_j n_i (less <U_j>
// d<U_i>/dx_j n_i at wall-function edges), from the predicted statistics: the
// nodal Laplacians at an edge's ends and the element gradients of the nodal
// Reynolds stresses of its element; B(q)_a integrates N_a q over the wall
// edges (q linear along an edge); g^n is the datum P^n satisfies (G.n before
// the first step).  The right-hand side is made compatible by removing its
// mean and dP has zero mean over the masters.  Conjugate gradients from zero,
// preconditioned by one V-cycle of the smoothed-aggregation hierarchy
// (k_amg.hip) or, without one, by Jacobi as in the paper.  Then every particle's velocity changes by
// -dt grad(dP) of its element, the element means by the same amount (the
// central moments are unchanged), P' += dP, and the next prediction uses G
// plus the node average of the element gradients of P'.
#include <hip/hip_runtime.h>

#include "pdf_solvers.h"

#include <utility>

namespace pdfk {

namespace {

constexpr int NB = 256;

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[NB / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NB / 64; ++w) s += red[w];
  return s;  // valid in thread 0
}

__device__ __forceinline__ double elem_area(const ElemGeo &g) {
  return 0.5 * ((g.x[1] - g.x[0]) * (g.y[2] - g.y[0]) - (g.x[2] - g.x[0]) * (g.y[1] - g.y[0]));
}

// the wall data at both ends of every wall edge, integrated against the
// shape functions into Bnew (and G.n into BG); one thread per edge
__global__ __launch_bounds__(NB) void k_proj_wallflux(MeshDev m, int32_t nwe, const int4 *we, const double4 *wg,
                                                      const double *S, double nu, const double *gin, double *Bnew,
                                                      double *BG) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nwe) return;
  const int nn = m.nn;
  const int4 w = we[t];
  const double4 G4 = wg[t];
  const double nx = G4.x, ny = G4.y, L = G4.z;
  const int32_t e = w.z;
  const double *dN = m.dN + 6 * (size_t)e;
  const int32_t qk[3] = {m.mnode[3 * e], m.mnode[3 * e + 1], m.mnode[3 * e + 2]};
  // element gradients of the nodal Reynolds stresses R11, R22, R12
  double g5x = 0.0, g5y = 0.0, g6x = 0.0, g6y = 0.0, g8x = 0.0, g8y = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double r5 = S[5 * (size_t)nn + qk[k]], r6 = S[6 * (size_t)nn + qk[k]], r8 = S[8 * (size_t)nn + qk[k]];
    g5x += dN[k] * r5;
    g5y += dN[3 + k] * r5;
    g6x += dN[k] * r6;
    g6y += dN[3 + k] * r6;
    g8x += dN[k] * r8;
    g8y += dN[3 + k] * r8;
  }
  const double dRx = g5x + g8y, dRy = g8x + g6y;
  double ux = 0.0, uy = 0.0, vx = 0.0, vy = 0.0;
  if (w.w) {
    for (int k = 0; k < 3; ++k) {
      const double u = S[qk[k]], v = S[(size_t)nn + qk[k]];
      ux += dN[k] * u;
      uy += dN[3 + k] * u;
      vx += dN[k] * v;
      vy += dN[3 + k] * v;
    }
  }
  double g[2], gn[2];
  const int32_t q[2] = {w.x, w.y};
  for (int j = 0; j < 2; ++j) {
    double v = nu * (S[21 * (size_t)nn + q[j]] * nx + S[22 * (size_t)nn + q[j]] * ny) - (dRx * nx + dRy * ny);
    if (w.w) {
      const double U = S[q[j]], V = S[(size_t)nn + q[j]];
      v = v - ((U * ux + V * uy) * nx + (U * vx + V * vy) * ny);
    }
    g[j] = v;
    gn[j] = gin ? gin[q[j]] * nx + gin[(size_t)nn + q[j]] * ny : 0.0;
  }
  atomicAdd(&Bnew[q[0]], L * (2.0 * g[0] + g[1]) / 6.0);
  atomicAdd(&Bnew[q[1]], L * (g[0] + 2.0 * g[1]) / 6.0);
  atomicAdd(&BG[q[0]], L * (2.0 * gn[0] + gn[1]) / 6.0);
  atomicAdd(&BG[q[1]], L * (gn[0] + 2.0 * gn[1]) / 6.0);
}

// before the first step P' = 0 satisfies the imposed gradient's data
__global__ __launch_bounds__(NB) void k_proj_copy(int32_t n, const double *src, double *dst) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

// b_a = -(d_a + C_p (K P')_a) / dt + (C_p/dt) (Bprev - BG)_a + (Bnew - Bprev)_a; bsum += b
__global__ __launch_bounds__(NB) void k_proj_rhs(MeshDev m, const double *S, const int32_t *row_off,
                                                 const int32_t *cols, const double *kval, const double *P,
                                                 double Cp, double dt, const double *dtp, const double *Bnew,
                                                 const double *Bprev, const double *BG, double *b, double *bsum) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (t < m.n_masters) {
    const double dtv = dtp ? dtp[0] : dt;
    const int nn = m.nn;
    const int32_t a = m.masters[t];
    double d = 0.0;
    for (int32_t i = m.m2e_off[a]; i < m.m2e_off[a + 1]; ++i) {
      const int32_t e = m.m2e[i];
      const double *dN = m.dN + 6 * (size_t)e;
      const int32_t qk[3] = {m.mnode[3 * e], m.mnode[3 * e + 1], m.mnode[3 * e + 2]};
      double div = 0.0;
      for (int k = 0; k < 3; ++k) div += dN[k] * S[qk[k]] + dN[3 + k] * S[nn + qk[k]];
      const double w = elem_area(m.geo[e]) / 3.0 * div;
      for (int la = 0; la < 3; ++la)
        if (qk[la] == a) d += w;
    }
    double kp = 0.0;
    for (int32_t j = row_off[a]; j < row_off[a + 1]; ++j) kp += kval[j] * P[cols[j]];
    v = -(d + Cp * kp) / dtv;
    if (Bnew) v = v + ((Cp / dtv) * (Bprev[a] - BG[a]) + (Bnew[a] - Bprev[a]));
    b[a] = v;
  }
  const double s = block_sum(v);
  if (threadIdx.x == 0) atomicAdd(bsum, s);
}

// b -= mean(b); x = 0; r = b; with Jacobi (kdiag != null) also z = r / diag,
// p = z, rz0 += r.z and bb += r.z (the multigrid start is k_proj_pinit)
__global__ __launch_bounds__(NB) void k_proj_start(MeshDev m, const double *kdiag, const double *bsum, double *b,
                                                   double *x, double *r, double *z, double *p, double *rz0,
                                                   double *bb) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0, w = 0.0;
  if (t < m.n_masters) {
    const int32_t a = m.masters[t];
    const double bv = b[a] - bsum[0] / (double)m.n_masters;
    b[a] = bv;
    x[a] = 0.0;
    r[a] = bv;
    if (kdiag) {
      const double zz = bv / kdiag[a];
      z[a] = zz;
      p[a] = zz;
      v = bv * zz;
      w = v;
    }
  }
  if (!kdiag) return;
  const double s = block_sum(v);
  if (threadIdx.x == 0) atomicAdd(rz0, s);
  __syncthreads();
  const double s2 = block_sum(w);
  if (threadIdx.x == 0) atomicAdd(bb, s2);
}

// multigrid start: p = z (= M^-1 r); rz0 += r.z; bb += r.z
__global__ __launch_bounds__(NB) void k_proj_pinit(MeshDev m, const double *r, const double *z, double *p, double *rz0,
                                                   double *bb) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (t < m.n_masters) {
    const int32_t a = m.masters[t];
    p[a] = z[a];
    v = r[a] * z[a];
  }
  const double s = block_sum(v);
  if (threadIdx.x == 0) {
    atomicAdd(rz0, s);
    atomicAdd(bb, s);
  }
}

// rzn += r.z after the multigrid step
__global__ __launch_bounds__(NB) void k_proj_rz(MeshDev m, const double *r, const double *z, double *rzn,
                                                const int *stop) {
  if (*stop) return;
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (t < m.n_masters) {
    const int32_t a = m.masters[t];
    v = r[a] * z[a];
  }
  const double s = block_sum(v);
  if (threadIdx.x == 0) atomicAdd(rzn, s);
}

// q = K p, pq += p.q; GA lanes per row (consecutive entries, then a sum across
// the group)
constexpr int GA = 8;
__global__ __launch_bounds__(NB) void k_proj_apply(MeshDev m, const int32_t *row_off, const int32_t *cols,
                                                   const double *kval, const double *p, double *q, double *pq,
                                                   const int *stop) {
  if (*stop) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t k = (int32_t)(t / GA);
  const int g = (int)(t % GA);
  double v = 0.0;
  if (k < m.n_masters) {
    const int32_t a = m.masters[k];
    double y = 0.0;
    for (int32_t j = row_off[a] + g; j < row_off[a + 1]; j += GA) y += kval[j] * p[cols[j]];
#pragma unroll
    for (int o = GA / 2; o > 0; o >>= 1) y += __shfl_xor(y, o, GA);
    if (g == 0) {
      q[a] = y;
      v = p[a] * y;
    }
  }
  const double s = block_sum(v);
  if (threadIdx.x == 0) atomicAdd(pq, s);
}

__global__ __launch_bounds__(NB) void k_proj_update(MeshDev m, const double *kdiag, const double *p, const double *q,
                                                    double *x, double *r, double *z, const double *rz,
                                                    const double *pq, double *rzn, const int *stop) {
  if (*stop) return;
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (t < m.n_masters) {
    const int32_t a = m.masters[t];
    const double alpha = (pq[0] != 0.0) ? rz[0] / pq[0] : 0.0;
    x[a] += alpha * p[a];
    const double rr = r[a] - alpha * q[a];
    r[a] = rr;
    if (kdiag) {  // Jacobi; with the multigrid, z and r.z follow in their own kernels
      const double zz = rr / kdiag[a];
      z[a] = zz;
      v = rr * zz;
    }
  }
  if (!kdiag) return;
  const double s = block_sum(v);
  if (threadIdx.x == 0) atomicAdd(rzn, s);
}

__global__ __launch_bounds__(NB) void k_proj_dir(MeshDev m, const double *z, double *p, const double *rz,
                                                 const double *rzn, const int *stop) {
  if (*stop) return;
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_masters) return;
  const int32_t a = m.masters[t];
  const double beta = (rz[0] != 0.0) ? rzn[0] / rz[0] : 0.0;
  p[a] = z[a] + beta * p[a];
}

// after the iteration that produced rz: count it, stop (stop = iterations + 1)
// at the tolerance or at maxit, and clear the ring slot of the next iteration
// (its previous contents belong to the iteration 8 steps back, long consumed)
__global__ void k_proj_check(const double *bb, const double *rz, double tol2, int maxit, int *iter, int *stop,
                             double *next_slot) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || *stop) return;
  const int it = ++(*iter);
  if (!(rz[0] > tol2 * bb[0]) || it >= maxit) *stop = it + 1;
  next_slot[0] = 0.0;
  next_slot[1] = 0.0;
}

// before the first iteration: converged already (stop = 1)?
__global__ void k_proj_check0(const double *bb, const double *rz, double tol2, int *stop) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (!(rz[0] > tol2 * bb[0])) *stop = 1;
}

// xsum += x over the masters
__global__ __launch_bounds__(NB) void k_proj_xsum(MeshDev m, const double *x, double *xsum) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const double v = t < m.n_masters ? x[m.masters[t]] : 0.0;
  const double s = block_sum(v);
  if (threadIdx.x == 0) atomicAdd(xsum, s);
}

// dP = x - mean at every node (identified nodes from their master); P' += dP
__global__ __launch_bounds__(NB) void k_proj_accum(MeshDev m, const double *x, const double *xsum, double *dP,
                                                   double *P) {
  const int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= m.nn) return;
  const double v = x[m.master[n]] - xsum[0] / (double)m.n_masters;
  dP[n] = v;
  P[n] += v;
}

// element gradient of dP; the element means of u and v shift by -dt grad dP
__global__ __launch_bounds__(NB) void k_proj_egrad(MeshDev m, const double *dP, double dt, const double *dtp,
                                                   double2 *ge, double *emom) {
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.ne) return;
  const double dtv = dtp ? dtp[0] : dt;
  const double *dN = m.dN + 6 * (size_t)e;
  double gx = 0.0, gy = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double v = dP[m.mnode[3 * e + k]];
    gx += dN[k] * v;
    gy += dN[3 + k] * v;
  }
  ge[e] = make_double2(dtv * gx, dtv * gy);
  double *em = emom + (size_t)e * 16;
  if (em[0] > 0.0) {
    em[1] -= dtv * gx;
    em[2] -= dtv * gy;
  }
}

// eq:velocity-correction on the particles
template <typename T>
__global__ __launch_bounds__(NB) void k_proj_correct(PartDev<T> p, int64_t np, const double2 *ge) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const double2 g = ge[p.e[i]];
  p.u[i] = (T)((double)p.u[i] - g.x);
  p.v[i] = (T)((double)p.v[i] - g.y);
}

// the gradient of the next prediction: G (input, or zero) plus the average
// over the elements around each master of the element gradients of P'
__global__ __launch_bounds__(NB) void k_proj_gradp(MeshDev m, const double *P, const double *gin, double *gtot) {
  const int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= m.nn) return;
  const int32_t a = m.master[n];
  double gx = 0.0, gy = 0.0;
  int c = 0;
  for (int32_t i = m.m2e_off[a]; i < m.m2e_off[a + 1]; ++i) {
    const int32_t e = m.m2e[i];
    const double *dN = m.dN + 6 * (size_t)e;
    for (int k = 0; k < 3; ++k) {
      const double v = P[m.mnode[3 * e + k]];
      gx += dN[k] * v;
      gy += dN[3 + k] * v;
    }
    c++;
  }
  gtot[n] = (gin ? gin[n] : 0.0) + (c ? gx / c : 0.0);
  gtot[m.nn + n] = (gin ? gin[m.nn + n] : 0.0) + (c ? gy / c : 0.0);
}

}  // namespace

void launch_proj_gradp(hipStream_t s, const MeshDev &m, const ProjBuf &b, const double *gin) {
  hipLaunchKernelGGL(k_proj_gradp, dim3((m.nn + NB - 1) / NB), dim3(NB), 0, s, m, b.P, gin, b.gtot);
}

// One conjugate-gradient iteration j (0..7) of a chunk: the scalars of
// iteration j live in ring slot j (pq, then r.z), the previous r.z in slot
// (j + 7) % 8, so the 8-iteration chunk is the same sequence of launches every
// time and is captured once as a HIP graph.
void proj_iteration(hipStream_t s, const MeshDev &m, const ProjBuf &b, int j, double tol2, int maxit) {
  const unsigned gm = (unsigned)((m.n_masters + NB - 1) / NB);
  const bool mg = b.amg.nl > 0;
  const double *kd = mg ? nullptr : b.kdiag;
  const double *rz = b.ring + 2 * ((j + 7) % 8) + 1;
  double *pq = b.ring + 2 * j, *rzn = b.ring + 2 * j + 1;
  const unsigned ga = (unsigned)(((int64_t)m.n_masters * GA + NB - 1) / NB);
  hipLaunchKernelGGL(k_proj_apply, dim3(ga), dim3(NB), 0, s, m, b.row_off, b.cols, b.kval, b.p, b.q, pq, b.stop);
  hipLaunchKernelGGL(k_proj_update, dim3(gm), dim3(NB), 0, s, m, kd, b.p, b.q, b.x, b.r, b.z, rz, pq, rzn, b.stop);
  if (mg) {
    launch_amg_apply(s, b.amg, m.masters, b.r, b.z, b.stop);
    hipLaunchKernelGGL(k_proj_rz, dim3(gm), dim3(NB), 0, s, m, b.r, b.z, rzn, b.stop);
  }
  hipLaunchKernelGGL(k_proj_check, dim3(1), dim3(64), 0, s, b.scal + 2, rzn, tol2, maxit, b.iter, b.stop,
                     b.ring + 2 * ((j + 1) % 8));
  hipLaunchKernelGGL(k_proj_dir, dim3(gm), dim3(NB), 0, s, m, b.z, b.p, rz, rzn, b.stop);
}

template <typename T>
int launch_proj_solve(hipStream_t s, const MeshDev &m, ProjBuf &b, const double *S, double Cp, double dt,
                      const double *dtp, double tol, int maxit, PartDev<T> p, int64_t np, double *emom,
                      double nu, const double *gin) {
  const unsigned gm = (unsigned)((m.n_masters + NB - 1) / NB);
  const double tol2 = tol * tol;
  // scal: [0] bsum, [1] unused, [2] bb, [3] xsum; ring: 8 slots of (pq, r.z),
  // slot 7's r.z holding the starting r.z
  (void)hipMemsetAsync(b.scal, 0, 4 * sizeof(double), s);
  (void)hipMemsetAsync(b.ring, 0, 16 * sizeof(double), s);
  (void)hipMemsetAsync(b.stop, 0, 2 * sizeof(int), s);  // stop and the iteration counter
  const bool walls = b.nwe > 0;
  if (walls) {
    (void)hipMemsetAsync(b.Bnew, 0, (size_t)m.nn * sizeof(double), s);
    (void)hipMemsetAsync(b.BG, 0, (size_t)m.nn * sizeof(double), s);
    hipLaunchKernelGGL(k_proj_wallflux, dim3((b.nwe + NB - 1) / NB), dim3(NB), 0, s, m, b.nwe, b.we, b.wgeom, S, nu,
                       gin, b.Bnew, b.BG);
    if (!b.wall_started) {
      hipLaunchKernelGGL(k_proj_copy, dim3((m.nn + NB - 1) / NB), dim3(NB), 0, s, m.nn, b.BG, b.Bprev);
      b.wall_started = true;
    }
  }
  hipLaunchKernelGGL(k_proj_rhs, dim3(gm), dim3(NB), 0, s, m, S, b.row_off, b.cols, b.kval, b.P, Cp, dt, dtp,
                     walls ? b.Bnew : nullptr, b.Bprev, b.BG, b.b, b.scal);
  if (walls) std::swap(b.Bnew, b.Bprev);  // the new data is what P' satisfies from now on
  const bool mg = b.amg.nl > 0;
  const double *kd = mg ? nullptr : b.kdiag;
  hipLaunchKernelGGL(k_proj_start, dim3(gm), dim3(NB), 0, s, m, kd, b.scal, b.b, b.x, b.r, b.z, b.p, b.ring + 15,
                     b.scal + 2);
  if (mg) {
    launch_amg_apply(s, b.amg, m.masters, b.r, b.z, b.stop);
    hipLaunchKernelGGL(k_proj_pinit, dim3(gm), dim3(NB), 0, s, m, b.r, b.z, b.p, b.ring + 15, b.scal + 2);
  }
  hipLaunchKernelGGL(k_proj_check0, dim3(1), dim3(64), 0, s, b.scal + 2, b.ring + 15, tol2, b.stop);
  // the chunk of 8 iterations: captured on the private capture stream the
  // first time, then replayed on s
  if (!b.chunk && b.cap) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      for (int j = 0; j < 8; ++j) proj_iteration(b.cap, m, b, j, tol2, maxit);
      if (hipStreamEndCapture(b.cap, &g) == hipSuccess && g) {
        hipGraphExec_t e = nullptr;
        if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) == hipSuccess) b.chunk = e;
        (void)hipGraphDestroy(g);
      }
    }
  }
  int stop_host = 0, launched = 0;
  while (launched < maxit && !stop_host) {
    if (b.chunk) {
      (void)hipGraphLaunch(b.chunk, s);
    } else {
      for (int j = 0; j < 8; ++j) proj_iteration(s, m, b, j, tol2, maxit);
    }
    launched += 8;
    (void)hipMemcpyAsync(&stop_host, b.stop, sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
  }
  hipLaunchKernelGGL(k_proj_xsum, dim3(gm), dim3(NB), 0, s, m, b.x, b.scal + 3);
  hipLaunchKernelGGL(k_proj_accum, dim3((m.nn + NB - 1) / NB), dim3(NB), 0, s, m, b.x, b.scal + 3, b.dP, b.P);
  hipLaunchKernelGGL(k_proj_egrad, dim3((m.ne + NB - 1) / NB), dim3(NB), 0, s, m, b.dP, dt, dtp, b.ge, emom);
  if (np > 0)
    hipLaunchKernelGGL(k_proj_correct<T>, dim3((unsigned)((np + NB - 1) / NB)), dim3(NB), 0, s, p, np, b.ge);
  return stop_host > 0 ? stop_host - 1 : maxit;
}

template int launch_proj_solve<float>(hipStream_t, const MeshDev &, ProjBuf &, const double *, double, double,
                                      const double *, double, int, PartDev<float>, int64_t, double *, double,
                                      const double *);
template int launch_proj_solve<double>(hipStream_t, const MeshDev &, ProjBuf &, const double *, double, double,
                                       const double *, double, int, PartDev<double>, int64_t, double *, double,
                                       const double *);

}  // namespace pdfk
