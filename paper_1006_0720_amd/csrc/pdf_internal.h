// Internal declarations shared by the host side of the C ABI (capi.hip) and
// the kernel translation units (k_particles.hip, k_stats.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pdf.h"

namespace pdfk {

// Element geometry for the walk: node coordinates, global node ids,
// neighbours (>= 0 element, < 0 boundary edge -(b+1)) and the range
// [wb, wb + wn) of the element's nearby no-slip wall segments.  80 bytes.
struct ElemGeo {
  double x[3], y[3];
  int32_t n[3];
  int32_t nb[3];
  int32_t wb, wn;
};

// Element geometry in the form the element test evaluates (eq:element-test):
// for the edge opposite local node k, its start point in the canonical
// direction (from the lower to the higher global node number) and the edge
// vector from there, negated where that direction runs against the element's
// counter-clockwise order.  The signed area of point P at edge k is then
//   lam_k = ex_k (P_y - ay_k) - ey_k (P_x - ax_k),
// bit-identical to the canonical cross product with its sign flipped as
// needed (negation is exact), with no selections left to the walk.  Plus the
// neighbours and the element's range of nearby no-slip wall segments.
// 128 bytes.
struct WalkGeo {
  double a[3][4];  // per edge k: ax, ay, ex, ey
  int32_t nb[3];
  int32_t wb, wn;
  int32_t pad[3];
};

// A no-slip wall edge near an element: its end points (local nodes k+1 and
// k+2 of its boundary element, in that order).
struct WallSeg {
  double xa, ya, xb, yb;
};

// Element record: element-average statistics and the pre-multiplied
// coefficients of one Euler-Maruyama step (rebuilt every step).
enum RecField {
  R_U = 0, R_V, R_W, R_OM, R_PHI,       // reference means (element average of nodal means)
  R_A0, R_A1, R_A2,                     // (-dP/dx_i/rho + 2 nu lap U_i) dt
  R_G00, R_G01, R_G02, R_G10, R_G11, R_G12, R_G20, R_G21, R_G22,  // G_ij dt
  R_SC0,                                // sqrt(C0 eps dt)
  R_B00, R_B01, R_B10, R_B11, R_B20, R_B21,  // sqrt(2 nu dt) dU_i/dx_j
  R_WA, R_WB, R_WC,                     // C3<om>dt, S_om<om>dt, sqrt(2 C3 C4 <om>^2 dt)
  R_MIX,                                // dt / t_m
  R_GSX, R_GSY,                         // gradient of sqrt(2k) (wall frequency)
  R_N                                   // = 30
};
constexpr int NREC = 32;

// Record of the SHAPE reading: the statistics of the element's three nodes
// (raw nodal values, interpolated at each particle) and the element-constant
// FEM gradients.  Per node: <U_i> (3), <omega>, <phi>, R_ij (6), Laplacian of
// <U_i> (3), mean-pressure gradient (2), wp_ij (9).
enum ShapeRecField {
  S_U = 0, S_V, S_W, S_OM, S_PHI, S_R11, S_R22, S_R33, S_R12, S_R13, S_R23,
  S_L0, S_L1, S_L2, S_GP0, S_GP1, S_WP00,  // S_WP00 .. S_WP00 + 8
  S_NODE = 25                              // values per node
};
constexpr int S_DU = 3 * S_NODE;  // dU_i/dx_j (6): i = U,V,W; j = x,y
constexpr int S_GS = S_DU + 6;    // gradient of sqrt(2k) (2)
constexpr int NRECS = 88;         // padded record length

// Element sums: count, 5 shifted first moments, 10 shifted second moments.
constexpr int NSUM = 16;

struct MeshDev {
  int32_t ne, nn, nb;
  const ElemGeo *geo;
  const WalkGeo *wgeo;      // [ne] the element test's form of the geometry
  const int32_t *mnode;     // [3*ne] master node of each element node
  const double *dN;         // [6*ne] dN_k/dx (k=0..2), dN_k/dy (k=0..2)
  const int32_t *btype, *bpart, *belem, *blocal;
  const double *bshift;     // [2*nb]
  const int32_t *n2e_off, *n2e;  // node -> elements
  const int32_t *m2e_off, *m2e;  // master node -> elements (statistics)
  const int32_t *w_off, *w_list; // element -> nearby no-slip wall edges
  const WallSeg *wseg;            // [w_off[ne]]: geometry of each w_list entry
  const double *cfl_len;          // [nn]: sqrt of the mean area of the elements around a master node, -1 elsewhere
  const int32_t *nwall_off, *nwall; // node -> wall (slip/no-slip) edges ending at it
  const int32_t *master;    // [nn] periodic identification
  const int32_t *masters;   // list of master nodes
  int32_t n_masters;
  const int32_t *slaves;    // list of identified (non-master) nodes
  const int32_t *slave_master;
  int32_t n_slaves;
  // uniform grid over the mesh bounding box for the last-resort point location:
  // cell (i, j) lists, in ascending order, every element whose bounding box
  // (padded by a millionth of a cell) meets the cell
  int32_t gnx, gny;
  double gx0, gy0, gsx, gsy;      // origin and cells per unit length
  const int32_t *cell_off, *cell_list;
  // each master's ring (the other masters it shares an element with,
  // ascending; empty for identified nodes) and the weights that give the
  // average over its elements of their gradients from the values at it and
  // at its ring: gw[q] its own, gw[nn + i] that of ring entry i
  const int32_t *ring_off, *ring;
  const double2 *gw;
};

template <typename T>
struct PartDev {
  T *x, *y, *u, *v, *w, *om, *psi;
  int32_t *e;
  uint32_t *id;
};

struct ModelDev {
  int32_t model, wp_source, omega_source, tm_mode, wall_b, stats_mode;
  int32_t mix_model, cond_nu, cond_nv, cond_nw, cond_min;
  int32_t outflow;  // 1: the mesh has PDF_BC_OUTFLOW edges (the particle kernel's variant with them)
  double C0, C1, C2, C3, C4, CT, Cv, gamma5, Cw1, Cw2, Cphi, nu, k_floor;
  double src_x, src_y, src_r, Cs, Ct, nu_wall;
  double inflow_u;  // velocity of particles relocated at the inflow (PDF_BC_OUTFLOW)
  double CL, Ceta;  // eq:L
};

// p[i] for p pointing into device memory, loaded through a global-segment
// pointer so that it compiles to a global rather than a flat instruction (flat
// loads also count against the LDS wait counter, which makes every LDS wait
// drain them).  The host pass only parses this device function.
template <typename T>
__device__ __forceinline__ T ldg(const T *p, size_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(1))) T *)p)[i];
#else
  return p[i];
#endif
}

// Mesh and model parameters of the particle kernel, kept in device memory and
// passed by pointer (uniform loads through the scalar cache instead of ~120
// kernel-argument registers).
struct KArgs {
  MeshDev m;
  ModelDev md;
};

// ---- launchers (defined in the kernel translation units) ----
template <typename T>
void launch_seed(hipStream_t s, const MeshDev &m, const ModelDev &md, PartDev<T> p, int32_t ppe,
                 uint64_t seed, int32_t psi_mode, double a, double b, double c, const double *U0,
                 const double *R0, const double *Om0, unsigned long long *cnt);
template <typename T>
void launch_elem_prep(hipStream_t s, const MeshDev &m, const ModelDev &md, const double *stats,
                      const double *wp, const double *gradp, double dt, const double *dtp, T *rec);
template <typename T>
void launch_elem_prep_shape(hipStream_t s, const MeshDev &m, const ModelDev &md, const double *stats,
                            const double *wp, const double *gradp, T *rec);
// ELEM: rec has NREC values per element, sums NSUM per element;
// SHAPE: rec has NRECS values per element, sums NSUM per node.
// dtp (record and particle kernels): when non-null, the step's time step is
// read from dtp[0] on the device and the dt argument is ignored.  cm (particle
// kernel): when non-null, each particle's velocity-conditioned scalar mean
// (storage order), used by eq:IECM in place of the element's <phi>.  S, gradp:
// the current nodal statistics and mean-pressure gradient (gradp may be null),
// read at wall-function edges
template <typename T>
void launch_advance(hipStream_t s, const KArgs *dka, const ModelDev &md, PartDev<T> p, int64_t np,
                    int32_t ne, const T *rec, double *sums, uint64_t seed, uint32_t step, double dt,
                    const double *dtp, const T *cm, const double *S, const double *gradp,
                    unsigned long long *cnt);
template <typename T>
void launch_accumulate_shape(hipStream_t s, const MeshDev &m, PartDev<T> p, int64_t np, const T *rec,
                             double *nsums);
template <typename T>
void launch_node_stats_shape(hipStream_t s, const MeshDev &m, const double *nsums, const double *ref,
                             const double *prev, double *out, unsigned long long *cnt);
template <typename T>
void launch_elem_count(hipStream_t s, PartDev<T> p, int64_t np, double *sums);
template <typename T>
void launch_accumulate(hipStream_t s, PartDev<T> p, int64_t np, int32_t ne, const T *rec, double *sums);
template <typename T>
void launch_ref_from_sums(hipStream_t s, int32_t ne, const double *sums, T *rec);
template <typename T>
void launch_elem_moments(hipStream_t s, int32_t ne, const double *sums, const T *rec, double *emom);
void launch_node_stats(hipStream_t s, const MeshDev &m, const double *emom, const double *prev,
                       double *out, unsigned long long *cnt);
void launch_node_derivs(hipStream_t s, const MeshDev &m, double *stats);
// time step of eq:CFL on the device.  buf: [0] the step's dt, [1] the time
// advanced since launch_cfl_begin, [2] scratch (the running minimum's bits)
void launch_cfl_begin(hipStream_t s, double *buf);
void launch_cfl_dt(hipStream_t s, const MeshDev &m, const double *stats, double c_cfl, double dt_max,
                   double *buf);
void launch_local_wp(hipStream_t s, const MeshDev &m, const ModelDev &md, const double *stats,
                     double *wp);
void launch_export_elem(hipStream_t s, int32_t ne, const double *emom, double *out);
template <typename T>
void launch_reorder(hipStream_t s, int32_t ne, int64_t np, const double *sums, int32_t *offs,
                    int32_t *cursor, int32_t *blocksums, PartDev<T> src, PartDev<T> dst);
template <typename T>
void launch_pack_state(hipStream_t s, PartDev<T> p, int64_t np, double *out);
template <typename T>
void launch_unpack_state(hipStream_t s, PartDev<T> p, int64_t np, const double *in);

}  // namespace pdfk

namespace pdfk {
// ---- denoiser kernels (k_denoise.hip) ----
void launch_gemm_bf16(hipStream_t s, int M, int N, int K, const uint16_t *A, int lda, int ta,
                      const uint16_t *B, int ldb, int tb, float *C, int ldc, float beta);
void launch_bias_act(hipStream_t s, int M, int N, float *Z, const float *b, uint16_t *H, int act);
void launch_dgelu(hipStream_t s, int64_t n, float *dH, const float *Z, uint16_t *dZb);
void launch_colsum(hipStream_t s, int M, int N, const float *G, float *out);
int launch_mse(hipStream_t s, int M, int nout, int ldy, float *Y, const float *T, uint16_t *dYb,
               float *part);
void launch_adam(hipStream_t s, int64_t n, float *w, const float *g, float *m, float *v, uint16_t *wb,
                 float lr, float b1, float b2, float eps, float c1, float c2);
void launch_to_bf16(hipStream_t s, int64_t n, const float *x, uint16_t *y);
// fused inference of the whole MLP (hidden width 48 .. 128) from the
// transposed weight copy; false: not applicable
size_t mlp_transposed_elems(int H);
void launch_transpose_weights(hipStream_t s, int H, const uint16_t *W1, const uint16_t *W2, const uint16_t *W3,
                              const uint16_t *W4, uint16_t *Wt);
bool launch_mlp_forward(hipStream_t s, int64_t n, int H, const float *x, const uint16_t *Wt_all, const float *b1,
                        const float *b2, const float *b3, const float *b4, float *y);
void launch_features(hipStream_t s, const MeshDev &m, const int32_t *p2p_off, const int32_t *p2p,
                     const double2 *gw, const double *S, const float *mu, const float *sig, float *F,
                     uint16_t *Fb);
void launch_grad_weights(hipStream_t s, const MeshDev &m, const int32_t *p2p_off, const int32_t *p2p, double2 *gw,
                         unsigned long long *bad);
void launch_merge(hipStream_t s, int nn, const int32_t *master, const double *S, const float *R, int ldr,
                  const float *scale, double tau, double C4, double *out, unsigned long long *nfall);
// the same over the nodes n0 .. n0 + cnt - 1 only, with row r of F and R
// belonging to node n0 + r
void launch_features_range(hipStream_t s, const MeshDev &m, const int32_t *p2p_off, const int32_t *p2p,
                           const double2 *gw, const double *S, const float *mu, const float *sig, int32_t n0,
                           int32_t cnt, float *F, uint16_t *Fb);
void launch_merge_range(hipStream_t s, int nn, const int32_t *master, const double *S, int32_t n0, int32_t cnt,
                        const float *R, int ldr, const float *scale, double tau, double C4, double *out,
                        unsigned long long *nfall);
}  // namespace pdfk
