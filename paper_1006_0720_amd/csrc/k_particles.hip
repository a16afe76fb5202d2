// Particle kernels for gfx950: seeding, element records and the fused
// Euler-Maruyama step with tracking, boundary conditions and accumulation.
//
// Method: J. Bakosi, "PDF modeling of turbulent flows on unstructured grids"
// (2008).  Equations are cited by their labels; "Ch.3 ..." names a section.
//
// Precision: particle state in T (float or double).  Positions are advanced,
// reflected and located in binary64 and stored rounded to T, so the element
// decision is taken on the stored position.  The library is compiled with
// floating-point contraction off; fused multiply-adds are written explicitly
// only where the element decision does not depend on them.
#include <hip/hip_runtime.h>

#include "pdf_internal.h"
#include "rng.h"

#include <type_traits>

namespace pdfk {

template <typename T>
__device__ __forceinline__ double stor(double v) {
  return (double)(T)v;
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// Element test (eq:element-test): signed areas of the sub-triangles formed by
// the point and each edge, each edge evaluated from its lower to its higher
// global node number so that the two elements sharing an edge get the same
// magnitude with opposite signs.  lam[k] belongs to the edge opposite local
// node k.  The canonical start points and the oriented edge vectors are
// stored per element (WalkGeo), so the test is two subtractions, two products
// and a difference per edge.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void edge_lambdas(const WalkGeo &g, double px, double py, double lam[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) lam[k] = g.a[k][2] * (py - g.a[k][1]) - g.a[k][3] * (px - g.a[k][0]);
}

__device__ __forceinline__ bool contains(const WalkGeo &g, double px, double py) {
  double l[3];
  edge_lambdas(g, px, py, l);
  return l[0] >= 0.0 && l[1] >= 0.0 && l[2] >= 0.0;
}

// fall-back for concave corners (Fig. corner): elements surrounding the nodes of e
__device__ int32_t search_patch(const MeshDev &m, int32_t e, double px, double py) {
  const ElemGeo g = ldg(m.geo, e);
  for (int k = 0; k < 3; ++k) {
    const int32_t n = g.n[k];
    for (int32_t i = ldg(m.n2e_off, n); i < ldg(m.n2e_off, n + 1); ++i) {
      const int32_t c = ldg(m.n2e, i);
      if (contains(ldg(m.wgeo, c), px, py)) return c;
    }
  }
  return -1;
}

// The lowest-numbered element whose closed triangle contains the point (the
// plain brute-force answer), found among the elements listed for the point's
// cell of the bucket grid: every element containing the point has its
// bounding box, and so its cell list entry, there.
__device__ int32_t locate_brute(const MeshDev &m, double px, double py) {
  const double fx = (px - m.gx0) * m.gsx, fy = (py - m.gy0) * m.gsy;
  if (!(fx >= -1e-6 && fy >= -1e-6 && fx <= m.gnx + 1e-6 && fy <= m.gny + 1e-6)) return -1;
  int32_t i = (int32_t)floor(fx), j = (int32_t)floor(fy);
  i = i < 0 ? 0 : (i >= m.gnx ? m.gnx - 1 : i);
  j = j < 0 ? 0 : (j >= m.gny ? m.gny - 1 : j);
  const size_t c = (size_t)j * m.gnx + i;
  for (int32_t k = ldg(m.cell_off, c); k < ldg(m.cell_off, c + 1); ++k) {
    const int32_t e = ldg(m.cell_list, k);
    if (contains(ldg(m.wgeo, e), px, py)) return e;
  }
  return -1;
}

// a[k] for k in {0,1,2} without dynamic indexing (keeps the arrays in registers)
template <typename V>
__device__ __forceinline__ V sel3(const V (&a)[3], int k) {
  return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]);
}

// wave-wide sum of a per-lane count followed by one atomic per wave
__device__ __forceinline__ void wave_count(unsigned long long *dst, int v) {
  if (__ballot(v != 0) == 0) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(dst, (unsigned long long)v);
}

// ---------------------------------------------------------------------------
// Seeding (Ch.3, Sec. Particle-number control)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_seed(MeshDev m, ModelDev md, PartDev<T> p, int32_t ppe,
                                              uint32_t k0, uint32_t k1, int32_t psi_mode, double pa,
                                              double pb, double pc, const double *U0,
                                              const double *R0, const double *Om0, int64_t np,
                                              unsigned long long *cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int gfail = 0;
  if (i < np) {
    const int32_t e = (int32_t)(i / ppe);
    const uint32_t id = (uint32_t)i;
    const ElemGeo g = ldg(m.geo, e);
    const int nn = m.nn;
    const u32x4 r = philox10(id, 0xFFFFFFFFu, 0u, 0u, k0, k1);
    const u32x4 r2 = philox10(id, 0xFFFFFFFFu, 1u, 0u, k0, k1);
    double b1 = unif_d(r.a), b2 = unif_d(r.b);
    if (b1 + b2 > 1.0) {
      b1 = 1.0 - b1;
      b2 = 1.0 - b2;
    }
    double x = g.x[0] + b1 * (g.x[1] - g.x[0]) + b2 * (g.x[2] - g.x[0]);
    double y = g.y[0] + b1 * (g.y[1] - g.y[0]) + b2 * (g.y[2] - g.y[0]);
    const double wA = 1.0 - b1 - b2, wB = b1, wC = b2;
    double z0, z1, z2, z3;
    box_muller_d(r.c, r.d, z0, z1);
    box_muller_d(r2.a, r2.b, z2, z3);
    const int nA = g.n[0], nB = g.n[1], nC = g.n[2];
    double U[3], R[6];
    for (int f = 0; f < 3; ++f)
      U[f] = wA * U0[f * nn + nA] + wB * U0[f * nn + nB] + wC * U0[f * nn + nC];
    for (int f = 0; f < 6; ++f)
      R[f] = wA * R0[f * nn + nA] + wB * R0[f * nn + nB] + wC * R0[f * nn + nC];
    const double Om = wA * Om0[nA] + wB * Om0[nB] + wC * Om0[nC];
    // velocity = U + L z with L the Cholesky factor of the Reynolds stress
    const double L11 = sqrt(R[0] > 0.0 ? R[0] : 0.0);
    const double L21 = L11 > 0.0 ? R[3] / L11 : 0.0, L31 = L11 > 0.0 ? R[4] / L11 : 0.0;
    const double t22 = R[1] - L21 * L21;
    const double L22 = sqrt(t22 > 0.0 ? t22 : 0.0);
    const double L32 = L22 > 0.0 ? (R[5] - L31 * L21) / L22 : 0.0;
    const double t33 = R[2] - L31 * L31 - L32 * L32;
    const double L33 = sqrt(t33 > 0.0 ? t33 : 0.0);
    const double u = U[0] + L11 * z0;
    const double v = U[1] + L21 * z0 + L22 * z1;
    const double w = U[2] + L31 * z0 + L32 * z1 + L33 * z2;
    int fail = 0;
    const double om =
        (Om > 0.0) ? gamma_mt(1.0 / md.C4, md.C4 * Om, k0, k1, id, 0xFFFFFFFFu, 16u, &fail) : 0.0;
    gfail = fail;
    x = stor<T>(x);
    y = stor<T>(y);
    double psi = 0.0;
    if (psi_mode == PDF_PSI_STEP_X) psi = (x < pa) ? 1.0 : 0.0;
    else if (psi_mode == PDF_PSI_GAUSS_X) psi = exp(-(x - pa) * (x - pa) / (2.0 * pb * pb));
    else if (psi_mode == PDF_PSI_BERNOULLI) psi = (unif_d(r2.c) < 0.5) ? 1.0 : 0.0;
    else if (psi_mode == PDF_PSI_DISC) psi = ((x - pa) * (x - pa) + (y - pb) * (y - pb) <= pc * pc) ? 1.0 : 0.0;
    p.x[i] = (T)x;
    p.y[i] = (T)y;
    p.u[i] = (T)u;
    p.v[i] = (T)v;
    p.w[i] = (T)w;
    p.om[i] = (T)om;
    p.psi[i] = (T)psi;
    p.e[i] = e;
    p.id[i] = id;
  }
  wave_count(&cnt[PDF_CNT_GAMMA_FAIL], gfail);
}

template <typename T>
void launch_seed(hipStream_t s, const MeshDev &m, const ModelDev &md, PartDev<T> p, int32_t ppe,
                 uint64_t seed, int32_t psi_mode, double a, double b, double c, const double *U0,
                 const double *R0, const double *Om0, unsigned long long *cnt) {
  const int64_t np = (int64_t)m.ne * ppe;
  const unsigned grid = (unsigned)((np + 255) / 256);
  hipLaunchKernelGGL(k_seed<T>, dim3(grid), dim3(256), 0, s, m, md, p, ppe, (uint32_t)seed,
                     (uint32_t)(seed >> 32), psi_mode, a, b, c, U0, R0, Om0, np, cnt);
}

// ---------------------------------------------------------------------------
// Step coefficients from the statistics seen by a particle (loop (ii) of
// Table tab:loops): k, eps (eq:dissipation-from-frequency_wall), G_ij and C0
// (eq:wall-GandC or eq:GandC with the tensor W = wp_ij), production, S_omega
// (eq:frequency-source) and t_m, pre-multiplied by dt where the step uses them.
// (px, py) is the point where the source-aware t_m measures its distance.
// ---------------------------------------------------------------------------
template <typename T, typename C = double>
__device__ __forceinline__ void record_from(const ModelDev &md, const C U[3], C Om, C Phi, const C R[6],
                                            const C lap[3], const C gp[2], const C *W, const C dU[3][2],
                                            const C gs[2], C dt, C px, C py, T *r) {
  const C k_floor = (C)md.k_floor, nu = (C)md.nu, CT = (C)md.CT, C0m = (C)md.C0, C3 = (C)md.C3, C4 = (C)md.C4,
          Cw1 = (C)md.Cw1, Cw2 = (C)md.Cw2, Cphi = (C)md.Cphi, Cs = (C)md.Cs, Ct = (C)md.Ct, sx = (C)md.src_x,
          sy = (C)md.src_y, sr = (C)md.src_r;
  C k = C(0.5) * (R[0] + R[1] + R[2]);
  if (!(k > k_floor)) k = k_floor;
  const C eps = Om * (k + nu * CT * CT * Om);
  C G[3][3], C0;
  const int sidx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  if (md.model == PDF_MODEL_SLM) {
    C0 = C0m;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) G[i][j] = (i == j) ? -(C(0.5) + C(0.75) * C0m) * Om : C(0.0);
  } else {
    C wr = C(0.0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const C Wij = W[3 * i + j];
        G[i][j] = (Wij - ((i == j) ? C(0.5) * eps : C(0.0))) / k;
        wr += Wij * R[sidx[i][j]];
      }
    const C c0 = -C(2.0) * wr / (C(3.0) * k * eps);
    C0 = (c0 > C(0.0)) ? c0 : C(0.0);
  }
  C prod = C(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 2; ++j) prod -= R[sidx[i][j]] * dU[i][j];
  const C Sw = md.omega_source ? (Cw2 - Cw1 * prod / eps) : C(0.0);
  C inv_tm;
  if (md.tm_mode == PDF_TM_CPHI) {
    inv_tm = C(0.5) * Cphi * Om;
  } else {
    const C ta = k / eps, tb = CT * sqrt(nu / eps);
    C tm = ta > tb ? ta : tb;
    if (md.tm_mode == PDF_TM_SOURCE) {
      // eq:micromixing-timescale-canyon: the source term C_s (r0^2/eps)^(1/3)
      // + C_t d / U_c drops out where U_c = |<U>| = 0
      const C dx = px - sx, dy = py - sy;
      const C d = sqrt(dx * dx + dy * dy);
      const C uc = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
      if (uc > C(0.0)) {
        const C ts = Cs * cbrt(sr * sr / eps) + Ct * d / uc;
        if (ts < tm) tm = ts;
      }
    }
    inv_tm = C(1.0) / tm;
  }
  r[R_U] = (T)U[0];
  r[R_V] = (T)U[1];
  r[R_W] = (T)U[2];
  r[R_OM] = (T)Om;
  r[R_PHI] = (T)Phi;
  r[R_A0] = (T)((-gp[0] + C(2.0) * nu * lap[0]) * dt);
  r[R_A1] = (T)((-gp[1] + C(2.0) * nu * lap[1]) * dt);
  r[R_A2] = (T)((C(2.0) * nu * lap[2]) * dt);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r[R_G00 + 3 * i + j] = (T)(G[i][j] * dt);
  r[R_SC0] = (T)sqrt(C0 * eps * dt);
  const C sv = sqrt(C(2.0) * nu * dt);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 2; ++j) r[R_B00 + 2 * i + j] = (T)(sv * dU[i][j]);
  r[R_WA] = (T)(C3 * Om * dt);
  r[R_WB] = (T)(Sw * Om * dt);
  r[R_WC] = (T)sqrt(C(2.0) * C3 * C4 * Om * Om * dt);
  r[R_MIX] = (T)(dt * inv_tm);
  r[R_GSX] = (T)gs[0];
  r[R_GSY] = (T)gs[1];
}

// element FEM gradients (eq:gradient) of the nodal <U_i> and of sqrt(2k)
__device__ __forceinline__ void elem_gradients(const MeshDev &m, const double *S, int32_t e,
                                               const int qk[3], double dU[3][2], double gs[2]) {
  const int nn = m.nn;
  const double *d = m.dN + 6 * (size_t)e;
  for (int i = 0; i < 3; ++i) {
    double gx = 0.0, gy = 0.0;
    for (int k = 0; k < 3; ++k) {
      gx += d[k] * S[i * nn + qk[k]];
      gy += d[3 + k] * S[i * nn + qk[k]];
    }
    dU[i][0] = gx;
    dU[i][1] = gy;
  }
  gs[0] = gs[1] = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double kn = 0.5 * (S[5 * nn + qk[k]] + S[6 * nn + qk[k]] + S[7 * nn + qk[k]]);
    const double sq = sqrt(2.0 * (kn > 0.0 ? kn : 0.0));
    gs[0] += d[k] * sq;
    gs[1] += d[3 + k] * sq;
  }
}

// ELEM records: the statistics of the element's particles are the element
// average of its three nodal values (Fig. mesh-particles).
template <typename T>
__global__ __launch_bounds__(256) void k_elem_prep(MeshDev m, ModelDev md, const double *S,
                                                   const double *wp, const double *gradp, double dt,
                                                   const double *dtp, T *rec) {
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.ne) return;
  if (dtp) dt = dtp[0];  // time step chosen on the device this step
  const int nn = m.nn;
  const int q0 = m.mnode[3 * e], q1 = m.mnode[3 * e + 1], q2 = m.mnode[3 * e + 2];
  const int qk[3] = {q0, q1, q2};
#define AVG(arr, f) ((arr[(f) * nn + q0] + arr[(f) * nn + q1] + arr[(f) * nn + q2]) / 3.0)
  const double U[3] = {AVG(S, 0), AVG(S, 1), AVG(S, 2)};
  const double Om = AVG(S, 3), Phi = AVG(S, 4);
  double R[6];
  for (int i = 0; i < 6; ++i) R[i] = AVG(S, 5 + i);
  const double lap[3] = {AVG(S, 21), AVG(S, 22), AVG(S, 23)};
  const double gp[2] = {gradp ? AVG(gradp, 0) : 0.0, gradp ? AVG(gradp, 1) : 0.0};
  double W[9];
  if (md.model == PDF_MODEL_GLM)
    for (int f = 0; f < 9; ++f) W[f] = AVG(wp, f);
#undef AVG
  double dU[3][2], gs[2];
  elem_gradients(m, S, e, qk, dU, gs);
  // the element centroid locates the element for the source-aware t_m
  const ElemGeo &g = m.geo[e];
  const double cx = (g.x[0] + g.x[1] + g.x[2]) / 3.0, cy = (g.y[0] + g.y[1] + g.y[2]) / 3.0;
  // formed in registers, stored as whole 16-byte words (the record is
  // NREC * sizeof(T) = 128 or 256 bytes, aligned)
  T r[NREC];
  record_from<T>(md, U, Om, Phi, R, lap, gp, W, dU, gs, dt, cx, cy, r);
  r[30] = (T)0;
  r[31] = (T)0;
  using V4 = std::conditional_t<sizeof(T) == 4, float4, double2>;
  constexpr int PER = 16 / sizeof(T);
  V4 *dst = reinterpret_cast<V4 *>(rec + (size_t)e * NREC);
#pragma unroll
  for (int k = 0; k < NREC / PER; ++k) {
    V4 v;
    __builtin_memcpy(&v, &r[k * PER], 16);
    dst[k] = v;
  }
}

// SHAPE records: the raw statistics of the element's three nodes and the
// element-constant gradients; S == nullptr gives all-zero statistics.
template <typename T>
__global__ __launch_bounds__(256) void k_elem_prep_shape(MeshDev m, ModelDev md, const double *S,
                                                         const double *wp, const double *gradp, T *rec) {
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.ne) return;
  const int nn = m.nn;
  const int qk[3] = {m.mnode[3 * e], m.mnode[3 * e + 1], m.mnode[3 * e + 2]};
  T *r = rec + (size_t)e * NRECS;
  for (int k = 0; k < 3; ++k) {
    T *o = r + k * S_NODE;
    const int q = qk[k];
    for (int f = 0; f < 11; ++f) o[S_U + f] = S ? (T)S[f * nn + q] : (T)0;  // U, omega, phi, R_ij
    for (int f = 0; f < 3; ++f) o[S_L0 + f] = S ? (T)S[(21 + f) * nn + q] : (T)0;
    for (int f = 0; f < 2; ++f) o[S_GP0 + f] = gradp ? (T)gradp[f * nn + q] : (T)0;
    for (int f = 0; f < 9; ++f)
      o[S_WP00 + f] = (wp && md.model == PDF_MODEL_GLM) ? (T)wp[f * nn + q] : (T)0;
  }
  double dU[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}}, gs[2] = {0.0, 0.0};
  if (S) elem_gradients(m, S, e, qk, dU, gs);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 2; ++j) r[S_DU + 2 * i + j] = (T)dU[i][j];
  r[S_GS] = (T)gs[0];
  r[S_GS + 1] = (T)gs[1];
  for (int f = S_GS + 2; f < NRECS; ++f) r[f] = (T)0;
}

template <typename T>
void launch_elem_prep_shape(hipStream_t s, const MeshDev &m, const ModelDev &md, const double *stats,
                            const double *wp, const double *gradp, T *rec) {
  hipLaunchKernelGGL(k_elem_prep_shape<T>, dim3((m.ne + 255) / 256), dim3(256), 0, s, m, md, stats, wp,
                     gradp, rec);
}

// shape-function values N^j at (x, y) of eq:approximation: the signed areas
// of eq:element-test over their sum (the area coordinates)
__device__ __forceinline__ void shape_w(const double lam[3], double w[3]) {
  const double s = lam[0] + lam[1] + lam[2];
  w[0] = lam[0] / s;
  w[1] = lam[1] / s;
  w[2] = lam[2] / s;
}

// statistics of a SHAPE record interpolated with weights w (eq:approximation),
// then the step coefficients as for an element record
// FP32 state forms these per-particle coefficients in binary32 (the FP64
// state, and every element record, in binary64): they are rounded to the
// state's precision anyway, and in binary32 the divisions and square roots
// are single hardware-assisted sequences
template <typename T>
__device__ __forceinline__ void shape_record(const ModelDev &md, const T *rs, const double w[3], double dt,
                                             double px, double py, T *r) {
  using C = T;
  const C w0 = (C)w[0], w1 = (C)w[1], w2 = (C)w[2];
#define INTERP(f) (w0 * (C)rs[(f)] + w1 * (C)rs[S_NODE + (f)] + w2 * (C)rs[2 * S_NODE + (f)])
  const C U[3] = {INTERP(S_U), INTERP(S_V), INTERP(S_W)};
  const C Om = INTERP(S_OM), Phi = INTERP(S_PHI);
  C R[6];
  for (int i = 0; i < 6; ++i) R[i] = INTERP(S_R11 + i);
  const C lap[3] = {INTERP(S_L0), INTERP(S_L1), INTERP(S_L2)};
  const C gp[2] = {INTERP(S_GP0), INTERP(S_GP0 + 1)};
  C W[9];
  if (md.model == PDF_MODEL_GLM)
    for (int f = 0; f < 9; ++f) W[f] = INTERP(S_WP00 + f);
#undef INTERP
  C dU[3][2];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 2; ++j) dU[i][j] = (C)rs[S_DU + 2 * i + j];
  const C gs[2] = {(C)rs[S_GS], (C)rs[S_GS + 1]};
  record_from<T, C>(md, U, Om, Phi, R, lap, gp, W, dU, gs, (C)dt, (C)px, (C)py, r);
}

template <typename T>
void launch_elem_prep(hipStream_t s, const MeshDev &m, const ModelDev &md, const double *stats,
                      const double *wp, const double *gradp, double dt, const double *dtp, T *rec) {
  hipLaunchKernelGGL(k_elem_prep<T>, dim3((m.ne + 255) / 256), dim3(256), 0, s, m, md, stats, wp,
                     gradp, dt, dtp, rec);
}

// ---------------------------------------------------------------------------
// Accumulation of element sums about the element's reference means.
//
// Each workgroup owns a contiguous chunk of particles (sorted by host element
// at the last reorder) and accumulates their contributions in an LDS table
// keyed by element (open addressing).  The table is flushed to the global
// FP64 sums with one atomic per value per element and workgroup, so a
// particle costs LDS atomics instead of contended global atomics.  A full
// table (never expected at the chunk sizes used) falls back to global atomics.
// ---------------------------------------------------------------------------
#ifndef PDF_TAB_LOG2
#define PDF_TAB_LOG2 7
#endif
#ifndef PDF_TAB_COPIES
#define PDF_TAB_COPIES 3
#endif
#ifndef PDF_PPT
#define PDF_PPT 16
#endif
constexpr int TAB = 1 << PDF_TAB_LOG2;  // LDS table slots per workgroup (power of two)
constexpr int NCOPY = PDF_TAB_COPIES;    // accumulator copies (lane % NCOPY picks one)
constexpr int WG = 256;                  // threads per workgroup of the particle kernels
constexpr int PPT = PDF_PPT;             // most particles per thread: chunk of WG*ppt particles

// Particles per thread for np particles over ne elements: at most PPT, halved
// while a workgroup's chunk of WG*ppt particles (sorted by element) would hold
// more than about CHUNK_ELEMS elements' worth at the mean count per element
// (the LDS table keeps room for the elements its particles move into), and
// halved again while the grid has fewer than MIN_WGS workgroups (small
// problems then spread over more waves, which hides the latency of the
// per-particle dependent loads).  Large chunks amortise the table set-up and
// flush.
constexpr int64_t MIN_WGS = 2048;
constexpr int64_t CHUNK_ELEMS = 48;
inline int pick_ppt(int64_t np, int64_t ne, int64_t chunk_elems = CHUNK_ELEMS) {
  int ppt = PPT;
  while (ppt > 1 && (int64_t)WG * ppt * (ne > 0 ? ne : 1) > chunk_elems * np) ppt >>= 1;
  while (ppt > 1 && (np + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt) < MIN_WGS) ppt >>= 1;
  return ppt;
}

// One key array and NCOPY copies of the accumulators: lanes of a wave that add
// to the same element (typically the particles that stayed in their host)
// are spread over the copies, dividing the serialisation of same-address LDS
// atomics by NCOPY; the copies are summed when the table is flushed.  Rows are
// padded by one word (TPAD) so that the copies of a value fall in different
// LDS banks: unpadded, the copy stride is a multiple of the bank count and
// the copies would conflict on the bank instead of on the address.
//
// Two geometries: at many particles per element (the default) 2^PDF_TAB_LOG2
// slots with NCOPY copies; at few per element (below SPARSE_PPE) the lanes of
// a wave seldom share an element, so one copy of 256 slots serves a chunk of
// more elements in the same LDS, and the flush (one global atomic per value,
// slot and workgroup) is spread over more particles.
constexpr int TPAD = 1;
template <int LOG2, int COPIES>
struct SumTableT {
  static constexpr int SLOTS = 1 << LOG2, NC = COPIES;
  int32_t key[SLOTS];
  uint32_t n[COPIES][SLOTS + TPAD];
  double acc[COPIES][15][SLOTS + TPAD];
};
using SumTable = SumTableT<PDF_TAB_LOG2, NCOPY>;
using SumTableSparse = SumTableT<8, 1>;
#ifndef PDF_SPARSE_PPE
#define PDF_SPARSE_PPE 45
#endif
constexpr int64_t SPARSE_PPE = PDF_SPARSE_PPE;  // mean particles per element below which the sparse table is used
#ifndef PDF_CHUNK_SPARSE
#define PDF_CHUNK_SPARSE 120
#endif
constexpr int64_t CHUNK_ELEMS_SPARSE = PDF_CHUNK_SPARSE;  // elements' worth of particles per workgroup chunk with it

template <int LOG2, int COPIES>
__device__ __forceinline__ void table_init(SumTableT<LOG2, COPIES> &t) {
  for (int s = threadIdx.x; s < SumTableT<LOG2, COPIES>::SLOTS; s += blockDim.x) {
    t.key[s] = -1;
#pragma unroll
    for (int c = 0; c < COPIES; ++c) {
      t.n[c][s] = 0u;
#pragma unroll
      for (int f = 0; f < 15; ++f) t.acc[c][f][s] = 0.0;
    }
  }
}

template <int LOG2, int COPIES>
__device__ __forceinline__ int table_slot(SumTableT<LOG2, COPIES> &t, int32_t e) {
  constexpr int SL = SumTableT<LOG2, COPIES>::SLOTS;
  uint32_t h = ((uint32_t)e * 2654435761u) >> (32 - LOG2);
  for (int probe = 0; probe < SL; ++probe) {
    const int32_t k = __hip_atomic_load(&t.key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == e) return (int)h;
    if (k == -1) {
      const int32_t old = atomicCAS(&t.key[h], -1, e);
      if (old == -1 || old == e) return (int)h;
    }
    h = (h + 1u) & (uint32_t)(SL - 1);
  }
  return -1;
}

// one particle's contribution to element e, shifted by the element's
// reference means ref[0..4] (<U>, <V>, <W>, <omega>, <phi> of its record)
template <typename T, int LOG2, int COPIES>
__device__ __forceinline__ void table_add(SumTableT<LOG2, COPIES> &t, double *sums, const T ref[5], int32_t e,
                                          T u, T v, T w, T om, T psi) {
  const double q0 = (double)u - (double)ref[0], q1 = (double)v - (double)ref[1],
               q2 = (double)w - (double)ref[2], q3 = (double)om - (double)ref[3],
               q4 = (double)psi - (double)ref[4];
  const double val[15] = {q0,      q1,      q2,      q3,      q4,      q0 * q0, q1 * q1, q2 * q2,
                          q0 * q1, q0 * q2, q1 * q2, q4 * q4, q0 * q4, q1 * q4, q2 * q4};
  const int s = table_slot(t, e);
  if (s >= 0) {
    const int c = (int)(threadIdx.x % COPIES);
    atomicAdd(&t.n[c][s], 1u);
#pragma unroll
    for (int f = 0; f < 15; ++f) unsafeAtomicAdd(&t.acc[c][f][s], val[f]);
  } else {
    double *g = sums + (size_t)e * NSUM;
    unsafeAtomicAdd(&g[0], 1.0);
#pragma unroll
    for (int f = 0; f < 15; ++f) unsafeAtomicAdd(&g[1 + f], val[f]);
  }
}

template <int LOG2, int COPIES>
__device__ __forceinline__ void table_flush(SumTableT<LOG2, COPIES> &t, double *sums) {
  __syncthreads();
  // sixteen lanes to a slot, one per value: each atomic instruction of a wave
  // then covers four elements' lines instead of one line per lane
  for (int idx = threadIdx.x; idx < SumTableT<LOG2, COPIES>::SLOTS * 16; idx += blockDim.x) {
    const int s = idx >> 4, f = idx & 15;
    const int32_t e = t.key[s];
    if (e < 0) continue;
    double v = 0.0;
    if (f == 0) {
      uint32_t n = 0;
#pragma unroll
      for (int c = 0; c < COPIES; ++c) n += t.n[c][s];
      v = (double)n;
    } else {
#pragma unroll
      for (int c = 0; c < COPIES; ++c) v += t.acc[c][f - 1][s];
    }
    unsafeAtomicAdd(&sums[(size_t)e * NSUM + f], v);
  }
}

// Table of the SHAPE reading, keyed by (master) node: the sum of the node's
// shape-function weights and the 15 weighted shifted moments.
struct SumTableW {
  int32_t key[TAB];
  double acc[NCOPY][16][TAB + TPAD];
};

__device__ __forceinline__ void table_init(SumTableW &t) {
  for (int s = threadIdx.x; s < TAB; s += blockDim.x) {
    t.key[s] = -1;
#pragma unroll
    for (int c = 0; c < NCOPY; ++c)
#pragma unroll
      for (int f = 0; f < 16; ++f) t.acc[c][f][s] = 0.0;
  }
}

__device__ __forceinline__ int table_slot(SumTableW &t, int32_t e) {
  uint32_t h = ((uint32_t)e * 2654435761u) >> (32 - PDF_TAB_LOG2);
  for (int probe = 0; probe < TAB; ++probe) {
    const int32_t k = __hip_atomic_load(&t.key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == e) return (int)h;
    if (k == -1) {
      const int32_t old = atomicCAS(&t.key[h], -1, e);
      if (old == -1 || old == e) return (int)h;
    }
    h = (h + 1u) & (uint32_t)(TAB - 1);
  }
  return -1;
}

// one particle's contribution to node `node` with weight wt, shifted by the
// node's reference means ref[S_U .. S_PHI]
template <typename T>
__device__ __forceinline__ void table_add_w(SumTableW &t, double *nsums, int32_t node, double wt,
                                            const T *ref, T u, T v, T w, T om, T psi) {
  const double q0 = (double)u - (double)ref[S_U], q1 = (double)v - (double)ref[S_V],
               q2 = (double)w - (double)ref[S_W], q3 = (double)om - (double)ref[S_OM],
               q4 = (double)psi - (double)ref[S_PHI];
  const double val[16] = {wt,           wt * q0,      wt * q1,      wt * q2,      wt * q3,      wt * q4,
                          wt * q0 * q0, wt * q1 * q1, wt * q2 * q2, wt * q0 * q1, wt * q0 * q2, wt * q1 * q2,
                          wt * q4 * q4, wt * q0 * q4, wt * q1 * q4, wt * q2 * q4};
  const int s = table_slot(t, node);
  if (s >= 0) {
    const int c = (int)(threadIdx.x % NCOPY);
#pragma unroll
    for (int f = 0; f < 16; ++f) unsafeAtomicAdd(&t.acc[c][f][s], val[f]);
  } else {
    double *g = nsums + (size_t)node * NSUM;
#pragma unroll
    for (int f = 0; f < 16; ++f) unsafeAtomicAdd(&g[f], val[f]);
  }
}

__device__ __forceinline__ void table_flush(SumTableW &t, double *nsums) {
  __syncthreads();
  // sixteen lanes to a slot, one per value (as for the element table)
  for (int idx = threadIdx.x; idx < TAB * 16; idx += blockDim.x) {
    const int s = idx >> 4, f = idx & 15;
    const int32_t e = t.key[s];
    if (e < 0) continue;
    double a = 0.0;
#pragma unroll
    for (int c = 0; c < NCOPY; ++c) a += t.acc[c][f][s];
    unsafeAtomicAdd(&nsums[(size_t)e * NSUM + f], a);
  }
}

// scatter of one particle at (x, y) in element e to the element's three nodes
template <typename T>
__device__ __forceinline__ void scatter_shape(SumTableW &t, const MeshDev &m, double *nsums, const T *rec,
                                              int32_t e, double x, double y, T u, T v, T w, T om, T psi,
                                              double l0 = -1.0, double l1 = 0.0, double l2 = 0.0) {
  double lam[3] = {l0, l1, l2}, wt[3];
  if (l0 < 0.0) edge_lambdas(ldg(m.wgeo, e), x, y, lam);
  shape_w(lam, wt);
  const T *rs = rec + (size_t)e * NRECS;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    table_add_w<T>(t, nsums, m.mnode[3 * e + k], wt[k], rs + k * S_NODE, u, v, w, om, psi);
}

template <typename T>
__global__ __launch_bounds__(WG) void k_accumulate_shape(MeshDev m, PartDev<T> p, int64_t np, int ppt,
                                                         const T *rec, double *nsums) {
  __shared__ SumTableW tab;
  table_init(tab);
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * WG * ppt;
  for (int j = 0; j < ppt; ++j) {
    const int64_t i = base + (int64_t)j * WG + threadIdx.x;
    if (i < np)
      scatter_shape<T>(tab, m, nsums, rec, p.e[i], (double)p.x[i], (double)p.y[i], p.u[i], p.v[i], p.w[i],
                       p.om[i], p.psi[i]);
  }
  table_flush(tab, nsums);
}

template <typename T>
void launch_accumulate_shape(hipStream_t s, const MeshDev &m, PartDev<T> p, int64_t np, const T *rec,
                             double *nsums) {
  const int ppt = pick_ppt(np, m.ne);
  hipLaunchKernelGGL(k_accumulate_shape<T>,
                     dim3((unsigned)((np + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt))), dim3(WG), 0, s,
                     m, p, np, ppt, rec, nsums);
}

// particles per element (the histogram of the reorder), as doubles in the
// count slot of each element's sums
template <typename T>
__global__ void k_elem_count(PartDev<T> p, int64_t np, double *sums) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) unsafeAtomicAdd(&sums[(size_t)p.e[i] * NSUM], 1.0);
}

template <typename T>
void launch_elem_count(hipStream_t s, PartDev<T> p, int64_t np, double *sums) {
  hipLaunchKernelGGL(k_elem_count<T>, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, p, np, sums);
}

template <typename T>
__global__ __launch_bounds__(WG) void k_accumulate(PartDev<T> p, int64_t np, int ppt, const T *rec,
                                                   double *sums) {
  __shared__ SumTable tab;
  table_init(tab);
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * WG * ppt;
  for (int j = 0; j < ppt; ++j) {
    const int64_t i = base + (int64_t)j * WG + threadIdx.x;
    if (i < np) {
      const int32_t e = p.e[i];
      const T *r = rec + (size_t)e * NREC;
      const T ref[5] = {r[R_U], r[R_V], r[R_W], r[R_OM], r[R_PHI]};
      table_add<T>(tab, sums, ref, e, p.u[i], p.v[i], p.w[i], p.om[i], p.psi[i]);
    }
  }
  table_flush(tab, sums);
}

template <typename T>
void launch_accumulate(hipStream_t s, PartDev<T> p, int64_t np, int32_t ne, const T *rec, double *sums) {
  const int ppt = pick_ppt(np, ne);
  hipLaunchKernelGGL(k_accumulate<T>, dim3((unsigned)((np + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt))),
                     dim3(WG), 0, s, p, np, ppt, rec, sums);
}

// reference means from a first accumulation pass made with zero references
template <typename T>
__global__ void k_ref_from_sums(int32_t ne, const double *sums, T *rec) {
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double *s = sums + (size_t)e * NSUM;
  T *r = rec + (size_t)e * NREC;
  for (int f = 0; f < NREC; ++f) r[f] = (T)0;
  if (s[0] > 0.0)
    for (int f = 0; f < 5; ++f) r[f] = (T)(s[1 + f] / s[0]);
}

template <typename T>
void launch_ref_from_sums(hipStream_t s, int32_t ne, const double *sums, T *rec) {
  hipLaunchKernelGGL(k_ref_from_sums<T>, dim3((ne + 255) / 256), dim3(256), 0, s, ne, sums, rec);
}

// ---------------------------------------------------------------------------
// No-slip particle condition (Ch.3, Sec. No-slip wall-boundary conditions):
// U_i = 0 and a frequency drawn from the gamma distribution with mean
// (1/C_T) d sqrt(2k)/dn (inward) and variance C4 <omega>^2 (eq:frequency-wallstats)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void noslip(const ModelDev &md, const T *r, double nx, double ny,
                                       uint32_t k0, uint32_t k1, uint32_t id, uint32_t step, int hit,
                                       T &u, T &v, T &w, T &om, int &gfail) {
  u = (T)0;
  v = (T)0;
  w = (T)0;
  double omw = -((double)r[R_GSX] * nx + (double)r[R_GSY] * ny) / md.CT;
  if (!(omw > 0.0)) omw = (double)r[R_OM];
  if (omw > 0.0) {
    int fail = 0;
    om = (T)gamma_mt(1.0 / md.C4, md.C4 * omw, k0, k1, id, step, 16u + 32u * (uint32_t)hit, &fail);
    gfail += fail;
  }
}

// ---------------------------------------------------------------------------
// The fused particle step.  One thread per particle in storage order:
//   noise (Philox) -> eq:Lagrangian-position-exact / -wf -> eq:velocity-prediction
//   -> eq:frequency-model -> eq:IEM -> next-best-element walk with periodic,
//   slip and no-slip conditions -> trajectory (b) of eq:fw -> source
//   -> store -> element sums of the new host.
// ---------------------------------------------------------------------------
// event counters of one thread, packed 16 bits each in ca (walk steps, periodic
// crossings, reflections, trajectory-(b) conditions) and 8 bits each in cb
// (fall-backs, brute-force searches, lost, omega folds, gamma failures, non-finite,
// outflow relocations)
#define C_WALK(v) (ca += (uint64_t)(v))
#define C_PER(v) (ca += (uint64_t)(v) << 16)
#define C_REFL(v) (ca += (uint64_t)(v) << 32)
#define C_B(v) (ca += (uint64_t)(v) << 48)
#define C_FALL(v) (cb += (uint64_t)(v))
#define C_BRUTE(v) (cb += (uint64_t)(v) << 8)
#define C_LOST(v) (cb += (uint64_t)(v) << 16)
#define C_CLAMP(v) (cb += (uint64_t)(v) << 24)
#define C_GFAIL(v) (cb += (uint64_t)(v) << 32)
#define C_NAN(v) (cb += (uint64_t)(v) << 40)
#define C_OUT(v) (cb += (uint64_t)(v) << 48)

// Wall-function condition (eq:wall-normal-velocity, eq:particle-wallcondition-wf
// with eq:alpha, eq:hatu, eq:Ue and eq:friction-velocity; eq:wall-omega) for a
// particle reflected at the edge from (xa, ya) along (dx, dy), the domain on
// its left.  The first gridpoint from the wall is the element's vertex off the
// edge, at (xc, yc), with master node q; its nodal statistics S (and the mean-
// pressure gradient gp, may be null) are taken in the edge's frame.  Returns
// the reflected in-plane velocity and frequency; the spanwise velocity is kept.
__device__ __noinline__ double3 wall_function(const ModelDev &md, const double *S, const double *gp, int32_t nn,
                                              int32_t q, double xa, double ya, double dx, double dy, double xc,
                                              double yc, double u, double v, double om) {
  constexpr double Cmu_sqrt = 0.3, kappa = 0.41, E = 8.5;  // sqrt(0.09)
  const double len = sqrt(dx * dx + dy * dy);
  const double tx = dx / len, ty = dy / len, nx = -ty, ny = tx;
  const double yp = (xc - xa) * nx + (yc - ya) * ny;
  const double Up = S[q] * tx + S[nn + q] * ty;
  const double Om = S[3 * nn + q];
  const double R11 = S[5 * nn + q], R22 = S[6 * nn + q], R33 = S[7 * nn + q], R12 = S[8 * nn + q];
  const double vvp = R11 * nx * nx + 2.0 * R12 * nx * ny + R22 * ny * ny;
  const double uvp = R11 * tx * nx + R12 * (tx * ny + ty * nx) + R22 * ty * ny;
  const double kp = 0.5 * (R11 + R22 + R33);
  const double dPdx = gp ? gp[q] * tx + gp[nn + q] * ty : 0.0;
  const double uhat2 = Cmu_sqrt * (kp > 0.0 ? kp : 0.0);
  const double utau = sqrt(uhat2 + ((uvp * dPdx > 0.0) ? fabs(yp * dPdx) : 0.0));
  const double Ue = utau / kappa * log(E * yp * utau / md.nu_wall);
  const double alpha = (Ue > 0.0 && vvp > 0.0) ? 2.0 * uhat2 * Up * fabs(Up) / (vvp * Ue * Ue) : 0.0;
  const double UI = u * tx + v * ty, VI = u * nx + v * ny;
  const double UR = UI + alpha * VI, VR = -VI;
  const double beta = -2.0 / (0.5 + 0.75 * md.C0 + md.C3 + md.Cw2 - md.Cw1);
  const double omr = (Om > 0.0 && yp > 0.0) ? om * exp(beta * VI / (yp * Om)) : om;
  return make_double3(UR * tx + VR * nx, UR * ty + VR * ny, omr);
}

// Occupancy: the FP32 kernels are held to 3 waves per SIMD (at most 168
// VGPRs; the LDS table of 3 copies, 48.5 KB, with the geometry window lets 3
// workgroups share a CU), which hides more of the latency of the walk's
// dependent loads than the 2 waves their unconstrained register count would
// allow; the SHAPE kernel spills some registers for it and is still faster.
// The window takes the rest of the LDS that three workgroups may hold: 53760
// bytes each (measured on gfx950: a workgroup of 53888 bytes leaves room for
// two only, and the kernel then runs 23 % slower).
constexpr int GWIN = 41;  // elements of the workgroup's geometry window (5.1 KB of LDS)
constexpr size_t LDS_3WG = 53760;
static_assert(sizeof(SumTable) + GWIN * sizeof(WalkGeo) <= LDS_3WG &&
                  sizeof(SumTableSparse) + GWIN * sizeof(WalkGeo) <= LDS_3WG,
              "the particle kernel's LDS must leave room for three workgroups per CU");
template <typename T, bool SHAPE>
constexpr int advance_waves() { return sizeof(T) == 4 ? 3 : 1; }

template <typename T, bool VISC, bool WALLB, bool SHAPE, bool SPARSE, bool OUTF>
__global__ __launch_bounds__(WG, (advance_waves<T, SHAPE>())) void k_advance(const KArgs *__restrict__ ka, PartDev<T> p, int64_t np,
                                                int ppt, const T *__restrict__ rec, double *sums, uint32_t k0,
                                                uint32_t k1, uint32_t step, double dt, double sdt,
                                                const double *dtp, double s2nu, const T *__restrict__ cm,
                                                const double *S, const double *gradp, unsigned long long *cnt) {
  __shared__ std::conditional_t<SHAPE, SumTableW, std::conditional_t<SPARSE, SumTableSparse, SumTable>> tab;
  __shared__ WalkGeo gwin[SHAPE ? 1 : GWIN];
  const MeshDev &m = ka->m;
  const ModelDev &md = ka->md;
  if (dtp) {  // time step chosen on the device this step
    dt = dtp[0];
    sdt = sqrt(dt);
  }
  table_init(tab);
  // the geometry of GWIN consecutive elements from the host of the
  // workgroup's first particle, staged in LDS: after a reorder the
  // workgroup's particles sit in a few consecutive elements, and the walk's
  // first test then reads LDS instead of waiting on the cache
  int32_t e_lo = 0, n_win = 0;
  if constexpr (!SHAPE) {
    const int64_t b0 = (int64_t)blockIdx.x * WG * ppt;
    e_lo = b0 < np ? ldg(p.e, b0) : 0;
    n_win = m.ne - e_lo < GWIN ? m.ne - e_lo : GWIN;
    const uint4 *src = (const uint4 *)(m.wgeo + e_lo);
    uint4 *dst = (uint4 *)gwin;
    for (int k = threadIdx.x; k < n_win * (int)(sizeof(WalkGeo) / 16); k += WG) dst[k] = ldg(src, k);
  }
  __syncthreads();
  uint64_t ca = 0, cb = 0;
  const int64_t base = (int64_t)blockIdx.x * WG * ppt;
  // software pipeline: the state of the thread's next particle is loaded
  // while the current one is advanced
  int32_t n_e = 0;
  uint32_t n_id = 0;
  T n_x = (T)0, n_y = (T)0, n_u = (T)0, n_v = (T)0, n_w = (T)0, n_om = (T)0, n_psi = (T)0, n_cm = (T)0;
  {
    const int64_t i0 = base + threadIdx.x;
    if (i0 < np) {
      if (cm) n_cm = cm[i0];
      n_e = p.e[i0];
      n_id = p.id[i0];
      n_x = p.x[i0];
      n_y = p.y[i0];
      n_u = p.u[i0];
      n_v = p.v[i0];
      n_w = p.w[i0];
      n_om = p.om[i0];
      n_psi = p.psi[i0];
    }
  }
  for (int jj = 0; jj < ppt; ++jj) {
    const int64_t i = base + (int64_t)jj * WG + threadIdx.x;
    if (i >= np) break;
    const int32_t e0 = n_e;
    const uint32_t id = n_id;
    const double x0 = (double)n_x, y0 = (double)n_y;
    const T up0 = n_u, up1 = n_v, up2 = n_w, om = n_om, psi = n_psi, cmv = n_cm;
    const int64_t inx = i + WG;
    if (jj + 1 < ppt && inx < np) {
      if (cm) n_cm = cm[inx];
      n_e = p.e[inx];
      n_id = p.id[inx];
      n_x = p.x[inx];
      n_y = p.y[inx];
      n_u = p.u[inx];
      n_v = p.v[inx];
      n_w = p.w[inx];
      n_om = p.om[inx];
      n_psi = p.psi[inx];
    }
    // statistics seen by the particle: its element's record (ELEM), or the
    // nodal statistics interpolated at its position (SHAPE)
    T rl[SHAPE ? NREC : 1];
    const T *r = rec + (size_t)e0 * NREC;
    if constexpr (SHAPE) {
      const WalkGeo g0 = ldg(m.wgeo, e0);
      double lam0[3], w0[3];
      edge_lambdas(g0, x0, y0, lam0);
      shape_w(lam0, w0);
      shape_record<T>(md, rec + (size_t)e0 * NRECS, w0, dt, x0, y0, rl);
      r = rl;
    }

    // ---- noise: six standard normals and one uniform per particle-step ----
    const u32x4 q0 = philox10(id, step, 0u, 0u, k0, k1);
    const u32x4 q1 = philox10(id, step, 1u, 0u, k0, k1);
    // the position noise in binary64 for FP64 state, on the binary32
    // transcendental units for FP32 state (as the other four normals)
    double xi0 = 0.0, xi1 = 0.0;
    T xi2, xi3, xi4, xi5;
    if constexpr (sizeof(T) == 8) {
      if (VISC) box_muller_d(q0.a, q0.b, xi0, xi1);
    } else if (VISC) {
      float z0, z1;
      box_muller_f(q0.a, q0.b, z0, z1);
      xi0 = z0;
      xi1 = z1;
    }
    if constexpr (sizeof(T) == 8) {
      double a0, a1, a2, a3;
      box_muller_d(q0.c, q0.d, a0, a1);
      box_muller_d(q1.a, q1.b, a2, a3);
      xi2 = a0;
      xi3 = a1;
      xi4 = a2;
      xi5 = a3;
    } else {
      box_muller_f(q0.c, q0.d, xi2, xi3);
      box_muller_f(q1.a, q1.b, xi4, xi5);
    }
    const double eta = unif_d(q1.c);

    // ---- position (binary64, stored rounded to T) ----
    double x = x0 + (double)up0 * dt;
    double y = y0 + (double)up1 * dt;
    if (VISC) {
      x = x + s2nu * (sdt * xi0);
      y = y + s2nu * (sdt * xi1);
    }
    x = stor<T>(x);
    y = stor<T>(y);

    // ---- velocity: eq:velocity-prediction with G_ij and C0 of the record ----
    const T ref0[5] = {r[R_U], r[R_V], r[R_W], r[R_OM], r[R_PHI]};
    const T d0 = up0 - ref0[0], d1 = up1 - ref0[1], d2 = up2 - ref0[2];
    T un0 = up0 + r[R_A0], un1 = up1 + r[R_A1], un2 = up2 + r[R_A2];
    un0 = fmaT(r[R_G00], d0, fmaT(r[R_G01], d1, fmaT(r[R_G02], d2, un0)));
    un1 = fmaT(r[R_G10], d0, fmaT(r[R_G11], d1, fmaT(r[R_G12], d2, un1)));
    un2 = fmaT(r[R_G20], d0, fmaT(r[R_G21], d1, fmaT(r[R_G22], d2, un2)));
    if (VISC) {
      const T x0n = (T)xi0, x1n = (T)xi1;
      un0 = fmaT(r[R_B00], x0n, fmaT(r[R_B01], x1n, un0));
      un1 = fmaT(r[R_B10], x0n, fmaT(r[R_B11], x1n, un1));
      un2 = fmaT(r[R_B20], x0n, fmaT(r[R_B21], x1n, un2));
    }
    const T sc = r[R_SC0];
    un0 = fmaT(sc, xi2, un0);
    un1 = fmaT(sc, xi3, un1);
    un2 = fmaT(sc, xi4, un2);

    // ---- frequency: eq:frequency-model, negative excursions folded back ----
    const T omp = om > (T)0 ? om : (T)0;
    T omn = om - r[R_WA] * (om - ref0[3]) - r[R_WB] * om + r[R_WC] * sqrt(omp) * xi5;
    if (omn < (T)0) {
      omn = -omn;
      C_CLAMP(1);
    }
    // ---- scalar: eq:IEM, or eq:IECM with the conditioned mean <phi|V> ----
    T psin = psi - r[R_MIX] * (psi - (cm ? cmv : ref0[4]));

    // ---- tracking: next-best-element walk (Ch.3, Sec. Particle tracking) ----
    int32_t e = e0, found = -1, nrefl = 0;
    int32_t fwb = 0, fwn = -1;  // wall segments near the host found by the walk
    double shx = 0.0, shy = 0.0;
    double lf0 = -1.0, lf1 = 0.0, lf2 = 0.0;  // SHAPE: the host's area coordinates from the walk
    // a non-finite position cannot be located: the particle is lost at once
    const bool finite_pos = isfinite(x) && isfinite(y);
    for (int it = 0; it < 64 && finite_pos; ++it) {
      C_WALK(1);
      const WalkGeo g = (!SHAPE && (uint32_t)(e - e_lo) < (uint32_t)n_win) ? gwin[e - e_lo] : ldg(m.wgeo, e);
      double lam[3];
      edge_lambdas(g, x, y, lam);
      if (lam[0] >= 0.0 && lam[1] >= 0.0 && lam[2] >= 0.0) {
        found = e;
        fwb = g.wb;
        fwn = g.wn;
        if constexpr (SHAPE) {
          lf0 = lam[0];
          lf1 = lam[1];
          lf2 = lam[2];
        }
        break;
      }
      int k = 0;
      if (lam[1] < lam[k]) k = 1;
      if (lam[2] < lam[k]) k = 2;
      const int32_t nb = sel3(g.nb, k);
      if (nb >= 0) {
        e = nb;
        continue;
      }
      const int32_t b = -(nb + 1);
      const int32_t bt = ldg(m.btype, b);
      if (bt == PDF_BC_PERIODIC || (OUTF && bt == PDF_BC_OUTFLOW)) {
        // periodic, or an outflow edge: the same translation to the paired
        // (inflow) edge, and there the velocity of the incoming flow (Ch.6,
        // cylinder flow, Sec. Results: its boundary conditions), on which
        // any later wall condition of the walk then acts
        const double sx = ldg(m.bshift, 2 * b), sy = ldg(m.bshift, 2 * b + 1);
        x = stor<T>(x + sx);
        y = stor<T>(y + sy);
        shx += sx;
        shy += sy;
        e = ldg(m.belem, ldg(m.bpart, b));
        if (OUTF && bt == PDF_BC_OUTFLOW) {
          un0 = (T)md.inflow_u;
          un1 = (T)0;
          un2 = (T)0;
          C_OUT(1);
        } else {
          C_PER(1);
        }
        continue;
      }
      // a boundary edge: the element's vertices and node numbers
      const ElemGeo gb = ldg(m.geo, e);
      const int ia = (k + 1) % 3, ib = (k + 2) % 3;
      const double xa = sel3(gb.x, ia), ya = sel3(gb.y, ia);
      const double dx = sel3(gb.x, ib) - xa, dy = sel3(gb.y, ib) - ya;
      const double t = ((x - xa) * dx + (y - ya) * dy) / (dx * dx + dy * dy);
      bool refl = (t >= 0.0 && t <= 1.0);
      if (!refl) {
        // past the end node c of this wall segment: with the boundary walked
        // with the domain on its left, a left turn at c (convex or straight
        // corner) puts the point, behind this wall's line, outside the domain;
        // at a reflex corner it is outside only if also behind the other wall
        const int32_t cn = sel3(gb.n, t < 0.0 ? ia : ib);
        int32_t wdg = -1;
        for (int32_t j = ldg(m.nwall_off, cn); j < ldg(m.nwall_off, cn + 1); ++j)
          if (ldg(m.nwall, j) != b) {
            wdg = ldg(m.nwall, j);
            break;
          }
        if (wdg < 0) {
          refl = true;  // the wall ends at a periodic or open boundary
        } else {
          const ElemGeo gw = ldg(m.geo, ldg(m.belem, wdg));
          const int kw = ldg(m.blocal, wdg);
          const double wa = sel3(gw.x, (kw + 1) % 3), wya = sel3(gw.y, (kw + 1) % 3);
          const double wdx = sel3(gw.x, (kw + 2) % 3) - wa, wdy = sel3(gw.y, (kw + 2) % 3) - wya;
          const double turn = (t < 0.0) ? (wdx * dy - wdy * dx) : (dx * wdy - dy * wdx);
          const double behind_w = (x - wa) * wdy - (y - wya) * wdx;
          if (turn >= 0.0 || behind_w > 0.0) refl = true;
        }
      }
      if (!refl) {
        // in the domain beyond a concave corner: fall-back of Fig. corner
        int32_t f = search_patch(m, e0, x, y);
        if (f < 0) f = search_patch(m, e, x, y);
        if (f >= 0) {
          C_FALL(1);
          found = f;
          break;
        }
        C_BRUTE(1);
        f = locate_brute(m, x, y);
        if (f >= 0) {
          found = f;
          break;
        }
        refl = true;
      }
      if (nrefl >= 8) break;
      // perfect reflection across the wall line
      const double len = sqrt(dx * dx + dy * dy);
      const double nx = dy / len, ny = -dx / len;
      const double dist = (x - xa) * nx + (y - ya) * ny;
      x = stor<T>(x - 2.0 * dist * nx);
      y = stor<T>(y - 2.0 * dist * ny);
      C_REFL(1);
      if (bt == PDF_BC_SLIP) {
        const double vn = (double)un0 * nx + (double)un1 * ny;
        un0 = (T)((double)un0 - 2.0 * vn * nx);
        un1 = (T)((double)un1 - 2.0 * vn * ny);
      } else if (!VISC && bt == PDF_BC_WALLFN) {
        // wall functions go with the inviscid particle equations
        const double3 rw = wall_function(md, S, gradp, m.nn, ldg(m.master, sel3(gb.n, k)), xa, ya, dx, dy,
                                         sel3(gb.x, k), sel3(gb.y, k), (double)un0, (double)un1, (double)omn);
        un0 = (T)rw.x;
        un1 = (T)rw.y;
        omn = (T)rw.z;
      } else {
        { int gf = 0; noslip<T>(md, r, nx, ny, k0, k1, id, step, nrefl, un0, un1, un2, omn, gf); C_GFAIL(gf); }
      }
      nrefl++;
    }
    if (found < 0) {
      int32_t f = finite_pos ? search_patch(m, e0, x, y) : -1;
      if (f < 0 && finite_pos) {
        C_BRUTE(1);
        f = locate_brute(m, x, y);
      }
      if (f >= 0) {
        found = f;
      } else {
        C_LOST(1);
        x = x0;
        y = y0;
        found = e0;
      }
    }

    // ---- no-slip trajectory (b): eq:fw and eq:exp-wall-condition ----
    if (WALLB && nrefl == 0) {
      if (fwn < 0) {  // host found by a fall-back search
        fwb = ldg(m.wgeo, found).wb;
        fwn = ldg(m.wgeo, found).wn;
      }
      int32_t best = -1;
      double bd = 0.0;
      for (int32_t j = fwb; j < fwb + fwn; ++j) {
        const WallSeg ws = ldg(m.wseg, j);
        const double xa = ws.xa, ya = ws.ya;
        const double dx = ws.xb - xa, dy = ws.yb - ya;
        double t = ((x - xa) * dx + (y - ya) * dy) / (dx * dx + dy * dy);
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
        const double ex = x - (xa + t * dx), ey = y - (ya + t * dy);
        const double d2 = ex * ex + ey * ey;
        if (best < 0 || d2 < bd) {
          best = j;
          bd = d2;
        }
      }
      if (best >= 0) {
        const WallSeg ws = ldg(m.wseg, best);
        const double xa = ws.xa, ya = ws.ya;
        const double dx = ws.xb - xa, dy = ws.yb - ya;
        const double len = sqrt(dx * dx + dy * dy);
        const double nx = dy / len, ny = -dx / len;
        const double d1 = -((x - xa) * nx + (y - ya) * ny);
        const double dd0 = -((x0 + shx - xa) * nx + (y0 + shy - ya) * ny);
        if (dd0 > 0.0 && d1 >= 0.0) {
          const double fw = exp(-dd0 * d1 / (md.nu * dt));
          if (eta < fw) {
            C_B(1);
            { int gf = 0; noslip<T>(md, r, nx, ny, k0, k1, id, step, 8, un0, un1, un2, omn, gf); C_GFAIL(gf); }
          }
        }
      }
    }
    // ---- continuous scalar source ----
    if (md.src_r > 0.0) {
      const double ddx = x - md.src_x, ddy = y - md.src_y;
      if (ddx * ddx + ddy * ddy <= md.src_r * md.src_r) psin = (T)1;
    }
    if (!(isfinite((double)un0) && isfinite((double)un1) && isfinite((double)un2) &&
          isfinite((double)omn) && isfinite((double)psin)))
      C_NAN(1);

    p.x[i] = (T)x;
    p.y[i] = (T)y;
    p.u[i] = un0;
    p.v[i] = un1;
    p.w[i] = un2;
    p.om[i] = omn;
    p.psi[i] = psin;
    p.e[i] = found;
    if constexpr (SHAPE)
      scatter_shape<T>(tab, m, sums, rec, found, x, y, un0, un1, un2, omn, psin, lf0, lf1, lf2);
    else {
      // reloaded rather than kept from the start of the step: holding them
      // across the walk costs register spills
      const T *rf = rec + (size_t)found * NREC;
      const T ref[5] = {rf[R_U], rf[R_V], rf[R_W], rf[R_OM], rf[R_PHI]};
      table_add<T>(tab, sums, ref, found, un0, un1, un2, omn, psin);
    }
  }
  table_flush(tab, sums);
  wave_count(&cnt[PDF_CNT_WALK_STEPS], (int)(ca & 0xFFFF));
  wave_count(&cnt[PDF_CNT_PERIODIC], (int)((ca >> 16) & 0xFFFF));
  wave_count(&cnt[PDF_CNT_REFLECT], (int)((ca >> 32) & 0xFFFF));
  wave_count(&cnt[PDF_CNT_NOSLIP_B], (int)((ca >> 48) & 0xFFFF));
  wave_count(&cnt[PDF_CNT_FALLBACK], (int)(cb & 0xFF));
  wave_count(&cnt[PDF_CNT_BRUTE], (int)((cb >> 8) & 0xFF));
  wave_count(&cnt[PDF_CNT_LOST], (int)((cb >> 16) & 0xFF));
  wave_count(&cnt[PDF_CNT_OMEGA_CLAMP], (int)((cb >> 24) & 0xFF));
  wave_count(&cnt[PDF_CNT_GAMMA_FAIL], (int)((cb >> 32) & 0xFF));
  wave_count(&cnt[PDF_CNT_NONFINITE], (int)((cb >> 40) & 0xFF));
  if constexpr (OUTF) wave_count(&cnt[PDF_CNT_OUTFLOW], (int)((cb >> 48) & 0xFF));
}

template <typename T, bool SHAPE, bool SPARSE, bool OUTF>
void launch_advance_k(hipStream_t s, const KArgs *dka, const ModelDev &md, PartDev<T> p, int64_t np, int ppt,
                      const T *rec, double *sums, uint64_t seed, uint32_t step, double dt, const double *dtp,
                      const T *cm, const double *S, const double *gradp, unsigned long long *cnt) {
  const unsigned grid = (unsigned)((np + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt));
  const bool visc = md.nu > 0.0;
  const bool wallb = visc && md.wall_b;
  const double sdt = sqrt(dt), s2nu = sqrt(2.0 * md.nu);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  if (visc && wallb)
    hipLaunchKernelGGL((k_advance<T, true, true, SHAPE, SPARSE, OUTF>), dim3(grid), dim3(WG), 0, s, dka, p, np, ppt,
                       rec, sums, k0, k1, step, dt, sdt, dtp, s2nu, cm, S, gradp, cnt);
  else if (visc)
    hipLaunchKernelGGL((k_advance<T, true, false, SHAPE, SPARSE, OUTF>), dim3(grid), dim3(WG), 0, s, dka, p, np, ppt,
                       rec, sums, k0, k1, step, dt, sdt, dtp, s2nu, cm, S, gradp, cnt);
  else
    hipLaunchKernelGGL((k_advance<T, false, false, SHAPE, SPARSE, OUTF>), dim3(grid), dim3(WG), 0, s, dka, p, np, ppt,
                       rec, sums, k0, k1, step, dt, sdt, dtp, s2nu, cm, S, gradp, cnt);
}

template <typename T, bool SHAPE>
void launch_advance_m(hipStream_t s, const KArgs *dka, const ModelDev &md, PartDev<T> p, int64_t np,
                      int32_t ne, const T *rec, double *sums, uint64_t seed, uint32_t step, double dt,
                      const double *dtp, const T *cm, const double *S, const double *gradp,
                      unsigned long long *cnt) {
  if constexpr (!SHAPE) {
    if (np < SPARSE_PPE * (int64_t)ne) {  // few particles per element: the sparse table
      if (md.outflow)
        launch_advance_k<T, false, true, true>(s, dka, md, p, np, pick_ppt(np, ne, CHUNK_ELEMS_SPARSE), rec, sums,
                                               seed, step, dt, dtp, cm, S, gradp, cnt);
      else
        launch_advance_k<T, false, true, false>(s, dka, md, p, np, pick_ppt(np, ne, CHUNK_ELEMS_SPARSE), rec, sums,
                                                seed, step, dt, dtp, cm, S, gradp, cnt);
      return;
    }
  }
  // the outflow relocation lives in its own kernel variant: its code in the
  // walk changes the register allocation of the whole kernel (8 more bytes
  // of spills, 1.5 % slower), which meshes without outflow edges do not pay
  if (md.outflow)
    launch_advance_k<T, SHAPE, false, true>(s, dka, md, p, np, pick_ppt(np, ne), rec, sums, seed, step, dt, dtp, cm,
                                            S, gradp, cnt);
  else
    launch_advance_k<T, SHAPE, false, false>(s, dka, md, p, np, pick_ppt(np, ne), rec, sums, seed, step, dt, dtp,
                                             cm, S, gradp, cnt);
}

template <typename T>
void launch_advance(hipStream_t s, const KArgs *dka, const ModelDev &md, PartDev<T> p, int64_t np,
                    int32_t ne, const T *rec, double *sums, uint64_t seed, uint32_t step, double dt,
                    const double *dtp, const T *cm, const double *S, const double *gradp,
                    unsigned long long *cnt) {
  if (md.stats_mode == PDF_STATS_SHAPE)
    launch_advance_m<T, true>(s, dka, md, p, np, ne, rec, sums, seed, step, dt, dtp, cm, S, gradp, cnt);
  else
    launch_advance_m<T, false>(s, dka, md, p, np, ne, rec, sums, seed, step, dt, dtp, cm, S, gradp, cnt);
}

#define INST(T)                                                                                  \
  template void launch_seed<T>(hipStream_t, const MeshDev &, const ModelDev &, PartDev<T>, int32_t, \
                               uint64_t, int32_t, double, double, double, const double *,         \
                               const double *, const double *, unsigned long long *);            \
  template void launch_elem_prep<T>(hipStream_t, const MeshDev &, const ModelDev &, const double *, \
                                    const double *, const double *, double, const double *, T *); \
  template void launch_advance<T>(hipStream_t, const KArgs *, const ModelDev &, PartDev<T>, int64_t, \
                                  int32_t, const T *, double *, uint64_t, uint32_t, double,                 \
                                  const double *, const T *, const double *, const double *,       \
                                  unsigned long long *);                                         \
  template void launch_accumulate<T>(hipStream_t, PartDev<T>, int64_t, int32_t, const T *, double *);        \
  template void launch_elem_prep_shape<T>(hipStream_t, const MeshDev &, const ModelDev &,           \
                                          const double *, const double *, const double *, T *);    \
  template void launch_accumulate_shape<T>(hipStream_t, const MeshDev &, PartDev<T>, int64_t,       \
                                           const T *, double *);                                    \
  template void launch_elem_count<T>(hipStream_t, PartDev<T>, int64_t, double *);                   \
  template void launch_ref_from_sums<T>(hipStream_t, int32_t, const double *, T *);
INST(float)
INST(double)
#undef INST

}  // namespace pdfk
