// Statistics kernels for gfx950: the two-pass particle-in-cell estimator
// (Ch.3, Sec. Estimation of Eulerian statistics), FEM derivatives (Sec.
// Derivatives), the local elliptic-relaxation tensor, the time step of
// eq:CFL, and the counting-sort reorder of particles by host element.
//
// Every nodal kernel is a gather over the linked list "elements surrounding
// master node" (no atomics), so nodal results do not depend on launch order.
#include <hip/hip_runtime.h>

#include "pdf_internal.h"

namespace pdfk {

// element means and central second moments (1/N) from the shifted sums:
// 16 lanes per element, lane f producing output f, so that every load and
// store of a wave covers whole 128-byte element rows
template <typename T>
__global__ __launch_bounds__(256) void k_elem_moments(int32_t ne, const double *sums, const T *rec,
                                                      double *emom) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t e = (int32_t)(t >> 4);
  const int f = (int)(t & 15);
  if (e >= ne) return;
  const double *s = sums + (size_t)e * NSUM;
  const double N = s[0];
  double v;
  if (f == 0) {
    v = N;
  } else if (!(N > 0.0)) {
    v = 0.0;
  } else if (f < 6) {
    v = (double)rec[(size_t)e * NREC + (f - 1)] + s[f] / N;
  } else {
    const int c = f - 6;
    const int a = c < 3 ? c : (c < 5 ? 0 : (c == 5 ? 1 : (c == 6 ? 4 : c - 7)));
    const int b = c < 3 ? c : (c == 3 ? 1 : (c == 4 ? 2 : (c == 5 ? 2 : 4)));
    v = s[f] / N - (s[1 + a] / N) * (s[1 + b] / N);
  }
  emom[(size_t)e * 16 + f] = v;
}

template <typename T>
void launch_elem_moments(hipStream_t s, int32_t ne, const double *sums, const T *rec, double *emom) {
  hipLaunchKernelGGL(k_elem_moments<T>, dim3((unsigned)(((int64_t)ne * 16 + 255) / 256)), dim3(256), 0, s, ne,
                     sums, rec, emom);
}

// pass 2: node value = average over the surrounding elements holding particles;
// nodes with none keep their previous value
__global__ __launch_bounds__(256) void k_node_stats(MeshDev m, const double *emom, const double *prev,
                                                    double *out, unsigned long long *cnt) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  int empty = 0;
  if (t < m.n_masters) {
    const int32_t n = m.masters[t];
    const int nn = m.nn;
    double acc[15];
    for (int f = 0; f < 15; ++f) acc[f] = 0.0;
    double sup = 0.0;
    int c = 0;
    // two elements per step, each row loaded whole before it is tested, so
    // that the dependent loads of a node overlap; summed in list order
    const int32_t i0 = ldg(m.m2e_off, n), i1 = ldg(m.m2e_off, n + 1);
    for (int32_t i = i0; i < i1; i += 2) {
      const bool two = i + 1 < i1;
      const int32_t ea = ldg(m.m2e, i), eb = two ? ldg(m.m2e, i + 1) : ea;
      double ra[16], rb[16];
#pragma unroll
      for (int f = 0; f < 16; f += 2) {
        const double2 a = ldg((const double2 *)(emom + (size_t)ea * 16), f / 2);
        const double2 b = ldg((const double2 *)(emom + (size_t)eb * 16), f / 2);
        ra[f] = a.x;
        ra[f + 1] = a.y;
        rb[f] = b.x;
        rb[f + 1] = b.y;
      }
      if (ra[0] > 0.0) {
        c++;
        sup += ra[0];
        for (int f = 0; f < 15; ++f) acc[f] += ra[1 + f];
      }
      if (two && rb[0] > 0.0) {
        c++;
        sup += rb[0];
        for (int f = 0; f < 15; ++f) acc[f] += rb[1 + f];
      }
    }
    if (c > 0) {
      for (int f = 0; f < 15; ++f) out[f * nn + n] = acc[f] / (double)c;
    } else {
      for (int f = 0; f < 15; ++f) out[f * nn + n] = prev[f * nn + n];
      empty = 1;
    }
    out[24 * nn + n] = sup;
  }
  if (__ballot(empty) != 0) {
    int v = empty;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&cnt[PDF_CNT_EMPTY_NODE], (unsigned long long)v);
  }
}

void launch_node_stats(hipStream_t s, const MeshDev &m, const double *emom, const double *prev,
                       double *out, unsigned long long *cnt) {
  hipLaunchKernelGGL(k_node_stats, dim3((m.n_masters + 255) / 256), dim3(256), 0, s, m, emom, prev,
                     out, cnt);
}

// SHAPE node values: weighted means and central moments from the node's sums
// (weight W, 5 weighted first and 10 weighted second moments shifted by the
// node's reference ref, as rounded to T in the records); nodes with W = 0
// keep their previous values.  ref == nullptr: zero reference.
template <typename T>
__global__ __launch_bounds__(256) void k_node_stats_shape(MeshDev m, const double *nsums, const double *ref,
                                                          const double *prev, double *out,
                                                          unsigned long long *cnt) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  int empty = 0;
  if (t < m.n_masters) {
    const int32_t n = m.masters[t];
    const int nn = m.nn;
    const double *s = nsums + (size_t)n * NSUM;
    const double W = s[0];
    if (W > 0.0) {
      double d[5];
      for (int f = 0; f < 5; ++f) d[f] = s[1 + f] / W;
      const int ca[10] = {0, 1, 2, 0, 0, 1, 4, 0, 1, 2};
      const int cb[10] = {0, 1, 2, 1, 2, 2, 4, 4, 4, 4};
      double mom[10];
      for (int c = 0; c < 10; ++c) mom[c] = s[6 + c] / W - d[ca[c]] * d[cb[c]];
      for (int f = 0; f < 5; ++f) {
        const double r = ref ? (double)(T)ref[f * nn + n] : 0.0;
        out[f * nn + n] = r + d[f];
      }
      for (int c = 0; c < 10; ++c) out[(5 + c) * nn + n] = mom[c];
    } else {
      for (int f = 0; f < 15; ++f) out[f * nn + n] = prev[f * nn + n];
      empty = 1;
    }
    out[24 * nn + n] = W;
  }
  if (__ballot(empty) != 0) {
    int v = empty;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&cnt[PDF_CNT_EMPTY_NODE], (unsigned long long)v);
  }
}

template <typename T>
void launch_node_stats_shape(hipStream_t s, const MeshDev &m, const double *nsums, const double *ref,
                             const double *prev, double *out, unsigned long long *cnt) {
  hipLaunchKernelGGL(k_node_stats_shape<T>, dim3((m.n_masters + 255) / 256), dim3(256), 0, s, m, nsums, ref,
                     prev, out, cnt);
}

// The averaged element gradient at a master q, (1/c) sum over the c elements
// around q of sum_k dN_e,k f(node k), is linear in the values at q and at
// its ring: weights w_j = (1/c) sum over (e, k) with node k of e = j of
// dN_e,k, formed once per mesh.  gw[q] holds q's own weight, gw[nn + i] the
// weight of ring entry i.  A ring entry that the elements do not reach
// (none, by the ring's construction) is counted in bad.
__global__ void k_grad_weights(MeshDev m, const int32_t *p2p_off, const int32_t *p2p, double2 *gw,
                               unsigned long long *bad) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m.nn) return;
  const int32_t rb = p2p_off[q], re = p2p_off[q + 1];
  double2 self = make_double2(0.0, 0.0);
  for (int32_t i = rb; i < re; ++i) gw[m.nn + i] = make_double2(0.0, 0.0);
  if (m.master[q] != q) {
    gw[q] = self;
    return;
  }
  const int32_t eb = m.m2e_off[q], ee = m.m2e_off[q + 1];
  for (int32_t i = eb; i < ee; ++i) {
    const int32_t e = m.m2e[i];
    for (int k = 0; k < 3; ++k) {
      const int32_t j = m.mnode[3 * e + k];
      const double wx = m.dN[6 * (size_t)e + k], wy = m.dN[6 * (size_t)e + 3 + k];
      if (j == q) {
        self.x += wx;
        self.y += wy;
        continue;
      }
      int32_t pos = -1;
      for (int32_t r = rb; r < re; ++r)
        if (p2p[r] == j) pos = r;
      if (pos < 0) {
        atomicAdd(bad, 1ull);
        continue;
      }
      gw[m.nn + pos].x += wx;
      gw[m.nn + pos].y += wy;
    }
  }
  const double ic = ee > eb ? 1.0 / (double)(ee - eb) : 0.0;
  gw[q] = make_double2(self.x * ic, self.y * ic);
  for (int32_t i = rb; i < re; ++i) gw[m.nn + i] = make_double2(gw[m.nn + i].x * ic, gw[m.nn + i].y * ic);
}

void launch_grad_weights(hipStream_t s, const MeshDev &m, const int32_t *p2p_off, const int32_t *p2p, double2 *gw,
                         unsigned long long *bad) {
  hipLaunchKernelGGL(k_grad_weights, dim3((unsigned)((m.nn + 255) / 256)), dim3(256), 0, s, m, p2p_off, p2p, gw,
                     bad);
}

// first derivatives: eq:gradient in every surrounding element, averaged
__global__ __launch_bounds__(256) void k_node_grad(MeshDev m, double *S) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_masters) return;
  const int32_t n = m.masters[t];
  const int nn = m.nn;
  // the average of the element gradients is a weighted sum over the master
  // and its ring (weights formed once per mesh); ring entries four at a time
  const double2 w0 = ldg(m.gw, n);
  double g[6];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const double v = ldg(S, (size_t)f * nn + n);
    g[2 * f] = w0.x * v;
    g[2 * f + 1] = w0.y * v;
  }
  const int32_t rb = ldg(m.ring_off, n), re = ldg(m.ring_off, n + 1);
  for (int32_t i = rb; i < re; i += 4) {
    int32_t j[4];
    double2 w[4];
    double v[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t k = min(i + u, re - 1);
      j[u] = ldg(m.ring, k);
      w[u] = ldg(m.gw, (size_t)nn + k);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int f = 0; f < 3; ++f) v[u][f] = ldg(S, (size_t)f * nn + j[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u < re)
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          g[2 * f] += w[u].x * v[u][f];
          g[2 * f + 1] += w[u].y * v[u][f];
        }
  }
  for (int f = 0; f < 6; ++f) S[(15 + f) * nn + n] = g[f];
}

// second derivatives: eq:gradient applied to the nodal first derivatives,
// through the same ring weights
__global__ __launch_bounds__(256) void k_node_lap(MeshDev m, double *S) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_masters) return;
  const int32_t n = m.masters[t];
  const int nn = m.nn;
  const double2 w0 = ldg(m.gw, n);
  double l[3];
#pragma unroll
  for (int f = 0; f < 3; ++f)
    l[f] = w0.x * ldg(S, (size_t)(15 + 2 * f) * nn + n) + w0.y * ldg(S, (size_t)(16 + 2 * f) * nn + n);
  const int32_t rb = ldg(m.ring_off, n), re = ldg(m.ring_off, n + 1);
  for (int32_t i = rb; i < re; i += 4) {
    int32_t j[4];
    double2 w[4];
    double gx[4][3], gy[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t k = min(i + u, re - 1);
      j[u] = ldg(m.ring, k);
      w[u] = ldg(m.gw, (size_t)nn + k);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        gx[u][f] = ldg(S, (size_t)(15 + 2 * f) * nn + j[u]);
        gy[u][f] = ldg(S, (size_t)(16 + 2 * f) * nn + j[u]);
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u < re)
#pragma unroll
        for (int f = 0; f < 3; ++f) l[f] += w[u].x * gx[u][f] + w[u].y * gy[u][f];
  }
  for (int f = 0; f < 3; ++f) S[(21 + f) * nn + n] = l[f];
}

__global__ void k_copy_slaves(MeshDev m, double *S, int nf) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_slaves) return;
  const int32_t n = m.slaves[t], q = m.slave_master[t];
  for (int f = 0; f < nf; ++f) S[f * m.nn + n] = S[f * m.nn + q];
}

void launch_node_derivs(hipStream_t s, const MeshDev &m, double *stats) {
  const unsigned g = (m.n_masters + 255) / 256;
  hipLaunchKernelGGL(k_node_grad, dim3(g), dim3(256), 0, s, m, stats);
  hipLaunchKernelGGL(k_node_lap, dim3(g), dim3(256), 0, s, m, stats);
  if (m.n_slaves > 0)
    hipLaunchKernelGGL(k_copy_slaves, dim3((m.n_slaves + 255) / 256), dim3(256), 0, s, m, stats,
                       PDF_NSTAT);
}

// ---- time step of eq:CFL ----
// dt = C_CFL * min over master nodes of sqrt(A_n) / |<U>_n|, A_n the mean
// area of the elements around the node and <U>_n the in-plane mean velocity;
// nodes at rest do not bound the step; capped at dt_max (also when every node
// is at rest).  The minimum runs over the bit patterns of the positive
// candidates (their order as unsigned integers is their order as numbers), so
// the result does not depend on the reduction order.  Products and sums are
// rounded one by one (no contraction), as written.
__global__ void k_cfl_begin(double *buf) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    buf[1] = 0.0;
    reinterpret_cast<unsigned long long *>(buf)[2] = ~0ull;
  }
}

__global__ __launch_bounds__(256) void k_cfl_min(int32_t nn, const double *len, const double *S, double *buf) {
#pragma clang fp contract(off)
  const int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long best = ~0ull;
  if (n < nn) {
    const double a = len[n];
    if (a >= 0.0) {
      const double u = S[n], v = S[nn + n];
      const double sp = sqrt(u * u + v * v);
      if (sp > 0.0) best = (unsigned long long)__double_as_longlong(a / sp);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(best, off, 64);
    best = o < best ? o : best;
  }
  if ((threadIdx.x & 63) == 0 && best != ~0ull)
    atomicMin(reinterpret_cast<unsigned long long *>(buf) + 2, best);
}

__global__ void k_cfl_final(double c_cfl, double dt_max, double *buf) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long *bits = reinterpret_cast<unsigned long long *>(buf) + 2;
  double dt = dt_max;
  if (*bits != ~0ull) {
    const double d = c_cfl * __longlong_as_double((long long)*bits);
    dt = d < dt_max ? d : dt_max;
  }
  buf[0] = dt;
  buf[1] = buf[1] + dt;
  *bits = ~0ull;  // ready for the next step
}

void launch_cfl_begin(hipStream_t s, double *buf) { hipLaunchKernelGGL(k_cfl_begin, dim3(1), dim3(64), 0, s, buf); }

void launch_cfl_dt(hipStream_t s, const MeshDev &m, const double *stats, double c_cfl, double dt_max,
                   double *buf) {
  hipLaunchKernelGGL(k_cfl_min, dim3((m.nn + 255) / 256), dim3(256), 0, s, m.nn, m.cfl_len, stats, buf);
  hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(64), 0, s, c_cfl, dt_max, buf);
}

// Local elliptic-relaxation tensor: the right-hand side of
// eq:elliptic-relaxation-Lagrangian (L -> 0) with H from eq:H, A_v and b_ij
// (eq:bij), from the nodal k, <omega>, Reynolds stress and mean-velocity gradient.
__global__ __launch_bounds__(256) void k_local_wp(MeshDev m, ModelDev md, const double *S, double *wp) {
  const int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= m.nn) return;
  const int nn = m.nn;
  const int32_t q = m.master[n];  // identified nodes use their master's statistics
  double R[6];
  for (int i = 0; i < 6; ++i) R[i] = S[(5 + i) * nn + q];
  double k = 0.5 * (R[0] + R[1] + R[2]);
  if (!(k > md.k_floor)) k = md.k_floor;
  const double om = S[3 * nn + q];
  const double Sg[3][3] = {{S[15 * nn + q], S[16 * nn + q], 0.0},
                           {S[17 * nn + q], S[18 * nn + q], 0.0},
                           {S[19 * nn + q], S[20 * nn + q], 0.0}};
  const double det = R[0] * (R[1] * R[2] - R[5] * R[5]) - R[3] * (R[3] * R[2] - R[5] * R[4]) +
                     R[4] * (R[3] * R[5] - R[1] * R[4]);
  const double k23 = 2.0 / 3.0 * k;
  double Av = md.Cv * det / (k23 * k23 * k23);
  if (Av > 1.0) Av = 1.0;
  const int sidx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  double b[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) b[i][j] = R[sidx[i][j]] / (2.0 * k) - ((i == j) ? 1.0 / 3.0 : 0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double h = (md.C2 * Av + md.gamma5 / 3.0) * Sg[i][j] - md.gamma5 / 3.0 * Sg[j][i];
      for (int l = 0; l < 3; ++l) h += md.gamma5 * b[i][l] * Sg[l][j] - md.gamma5 * b[i][l] * Sg[j][l];
      wp[(3 * i + j) * nn + n] = k * h + ((i == j) ? 0.5 * (1.0 - md.C1) * k * om : 0.0);
    }
}

void launch_local_wp(hipStream_t s, const MeshDev &m, const ModelDev &md, const double *stats,
                     double *wp) {
  hipLaunchKernelGGL(k_local_wp, dim3((m.nn + 255) / 256), dim3(256), 0, s, m, md, stats, wp);
}

// element statistics out of the AoS buffer into [16][ne]
__global__ void k_export_elem(int32_t ne, const double *emom, double *out) {
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  for (int f = 0; f < 16; ++f) out[(size_t)f * ne + e] = emom[(size_t)e * 16 + f];
}

void launch_export_elem(hipStream_t s, int32_t ne, const double *emom, double *out) {
  hipLaunchKernelGGL(k_export_elem, dim3((ne + 255) / 256), dim3(256), 0, s, ne, emom, out);
}

// ---------------------------------------------------------------------------
// Reorder: counting sort of the particle SoA by host element.  Counts are the
// element sums' particle counts of the last accumulation.
// ---------------------------------------------------------------------------
constexpr int SCAN_B = 1024;

__global__ __launch_bounds__(SCAN_B) void k_scan_blocks(int32_t ne, const double *sums, int32_t *offs,
                                                        int32_t *blocksums) {
  __shared__ int32_t sh[SCAN_B];
  const int32_t i = blockIdx.x * SCAN_B + threadIdx.x;
  const int32_t v = (i < ne) ? (int32_t)sums[(size_t)i * NSUM] : 0;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_B; off <<= 1) {
    const int32_t a = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += a;
    __syncthreads();
  }
  if (i < ne) offs[i] = sh[threadIdx.x] - v;  // exclusive within the block
  if (threadIdx.x == SCAN_B - 1) blocksums[blockIdx.x] = sh[threadIdx.x];
}

__global__ __launch_bounds__(SCAN_B) void k_scan_top(int32_t nblocks, int32_t *blocksums) {
  __shared__ int32_t sh[SCAN_B];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int32_t base = 0; base < nblocks; base += SCAN_B) {
    const int32_t i = base + threadIdx.x;
    const int32_t v = (i < nblocks) ? blocksums[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_B; off <<= 1) {
      const int32_t a = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < nblocks) blocksums[i] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == SCAN_B - 1) carry += sh[threadIdx.x];
    __syncthreads();
  }
}

__global__ void k_scan_add(int32_t ne, int32_t *offs, const int32_t *blocksums, int32_t *cursor) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  offs[i] += blocksums[i / SCAN_B];
  cursor[i] = 0;
}

// Scatter: each workgroup ranks its chunk's particles per element in an LDS
// table (local ranks from LDS atomics), reserves one range per element and
// workgroup with a single global atomic, then writes every particle to
// offs[e] + range base + local rank.  Elements that do not fit in the table
// fall back to one global atomic per particle.
constexpr int SC_WG = 256, SC_PPT = 16, SC_TAB = 512;

template <typename T>
__global__ __launch_bounds__(SC_WG) void k_scatter(int64_t np, const int32_t *offs, int32_t *cursor,
                                                   PartDev<T> src, PartDev<T> dst) {
  __shared__ int32_t key[SC_TAB];
  __shared__ int32_t cntl[SC_TAB];
  __shared__ int32_t basel[SC_TAB];
  for (int s = threadIdx.x; s < SC_TAB; s += SC_WG) {
    key[s] = -1;
    cntl[s] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * (SC_WG * SC_PPT);
  int slot[SC_PPT], rank[SC_PPT];
  int32_t el[SC_PPT];
  for (int j = 0; j < SC_PPT; ++j) {
    const int64_t i = base + (int64_t)j * SC_WG + threadIdx.x;
    slot[j] = -1;
    rank[j] = 0;
    el[j] = -1;
    if (i >= np) continue;
    const int32_t e = src.e[i];
    el[j] = e;
    uint32_t h = ((uint32_t)e * 2654435761u) >> 23;  // 9 bits
    for (int probe = 0; probe < 64; ++probe) {
      const int32_t k = __hip_atomic_load(&key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (k == e) {
        slot[j] = (int)h;
        break;
      }
      if (k == -1) {
        const int32_t old = atomicCAS(&key[h], -1, e);
        if (old == -1 || old == e) {
          slot[j] = (int)h;
          break;
        }
      }
      h = (h + 1u) & (uint32_t)(SC_TAB - 1);
    }
    if (slot[j] < 0) rank[j] = atomicAdd(&cursor[e], 1);  // global rank (overflow path)
  }
  // ranks within the table: the lanes of a wave holding the same element get
  // consecutive ranks in lane order (one LDS atomic per distinct element and
  // wave), so that neighbouring lanes write neighbouring destinations
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int j = 0; j < SC_PPT; ++j) {
    bool pending = slot[j] >= 0;
    while (__ballot(pending) != 0) {
      const uint64_t act = __ballot(pending);
      const int leader = __ffsll((unsigned long long)act) - 1;
      const int lkey = __shfl(slot[j], leader, 64);
      const uint64_t same = __ballot(pending && slot[j] == lkey);
      int base_r = 0;
      if (lane == leader) base_r = atomicAdd(&cntl[lkey], __popcll(same));
      base_r = __shfl(base_r, leader, 64);
      if (pending && slot[j] == lkey) {
        rank[j] = base_r + __popcll(same & below);
        pending = false;
      }
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < SC_TAB; s += SC_WG)
    if (key[s] >= 0) basel[s] = atomicAdd(&cursor[key[s]], cntl[s]);
  __syncthreads();
  // destinations first, then the moves in groups of four particles per thread
  // with every load of a group issued before its stores (the source and
  // destination buffers are distinct, which the compiler cannot assume)
  int64_t dd[SC_PPT];
  for (int j = 0; j < SC_PPT; ++j) {
    const int64_t i = base + (int64_t)j * SC_WG + threadIdx.x;
    dd[j] = (i < np) ? (int64_t)ldg(offs, el[j]) + (slot[j] >= 0 ? basel[slot[j]] + rank[j] : rank[j]) : -1;
  }
  constexpr int GRP = 4;
  static_assert(SC_PPT % GRP == 0, "groups of four");
  for (int j0 = 0; j0 < SC_PPT; j0 += GRP) {
    T vx[GRP], vy[GRP], vu[GRP], vv[GRP], vw[GRP], vo[GRP], vp[GRP];
    uint32_t vid[GRP];
#pragma unroll
    for (int q = 0; q < GRP; ++q) {
      const int64_t i = base + (int64_t)(j0 + q) * SC_WG + threadIdx.x;
      if (dd[j0 + q] < 0) continue;
      vx[q] = ldg(src.x, i);
      vy[q] = ldg(src.y, i);
      vu[q] = ldg(src.u, i);
      vv[q] = ldg(src.v, i);
      vw[q] = ldg(src.w, i);
      vo[q] = ldg(src.om, i);
      vp[q] = ldg(src.psi, i);
      vid[q] = ldg(src.id, i);
    }
#pragma unroll
    for (int q = 0; q < GRP; ++q) {
      const int64_t d = dd[j0 + q];
      if (d < 0) continue;
      dst.x[d] = vx[q];
      dst.y[d] = vy[q];
      dst.u[d] = vu[q];
      dst.v[d] = vv[q];
      dst.w[d] = vw[q];
      dst.om[d] = vo[q];
      dst.psi[d] = vp[q];
      dst.e[d] = el[j0 + q];
      dst.id[d] = vid[q];
    }
  }
}

template <typename T>
void launch_reorder(hipStream_t s, int32_t ne, int64_t np, const double *sums, int32_t *offs,
                    int32_t *cursor, int32_t *blocksums, PartDev<T> src, PartDev<T> dst) {
  const int32_t nb = (ne + SCAN_B - 1) / SCAN_B;
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(SCAN_B), 0, s, ne, sums, offs, blocksums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_B), 0, s, nb, blocksums);
  hipLaunchKernelGGL(k_scan_add, dim3((ne + 255) / 256), dim3(256), 0, s, ne, offs, blocksums, cursor);
  hipLaunchKernelGGL(k_scatter<T>, dim3((unsigned)((np + SC_WG * SC_PPT - 1) / (SC_WG * SC_PPT))),
                     dim3(SC_WG), 0, s, np, offs, cursor, src, dst);
}

// particle state <-> double [7][n]
template <typename T>
__global__ void k_pack(PartDev<T> p, int64_t np, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  out[0 * np + i] = (double)p.x[i];
  out[1 * np + i] = (double)p.y[i];
  out[2 * np + i] = (double)p.u[i];
  out[3 * np + i] = (double)p.v[i];
  out[4 * np + i] = (double)p.w[i];
  out[5 * np + i] = (double)p.om[i];
  out[6 * np + i] = (double)p.psi[i];
}

template <typename T>
__global__ void k_unpack(PartDev<T> p, int64_t np, const double *in) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  p.x[i] = (T)in[0 * np + i];
  p.y[i] = (T)in[1 * np + i];
  p.u[i] = (T)in[2 * np + i];
  p.v[i] = (T)in[3 * np + i];
  p.w[i] = (T)in[4 * np + i];
  p.om[i] = (T)in[5 * np + i];
  p.psi[i] = (T)in[6 * np + i];
}

template <typename T>
void launch_pack_state(hipStream_t s, PartDev<T> p, int64_t np, double *out) {
  hipLaunchKernelGGL(k_pack<T>, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, p, np, out);
}
template <typename T>
void launch_unpack_state(hipStream_t s, PartDev<T> p, int64_t np, const double *in) {
  hipLaunchKernelGGL(k_unpack<T>, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, p, np, in);
}

#define INST(T)                                                                                  \
  template void launch_node_stats_shape<T>(hipStream_t, const MeshDev &, const double *,            \
                                           const double *, const double *, double *,                \
                                           unsigned long long *);                                   \
  template void launch_elem_moments<T>(hipStream_t, int32_t, const double *, const T *, double *); \
  template void launch_reorder<T>(hipStream_t, int32_t, int64_t, const double *, int32_t *,         \
                                  int32_t *, int32_t *, PartDev<T>, PartDev<T>);                  \
  template void launch_pack_state<T>(hipStream_t, PartDev<T>, int64_t, double *);                  \
  template void launch_unpack_state<T>(hipStream_t, PartDev<T>, int64_t, const double *);
INST(float)
INST(double)
#undef INST

}  // namespace pdfk
