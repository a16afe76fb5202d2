// Internal declarations of the solvers around the particle step: the
// particle redistribution, the velocity-conditioned scalar means, the
// elliptic relaxation and the pressure projection with their multigrid
// hierarchies.  Kept apart from pdf_internal.h, which the particle kernel
// compiles against, so that the particle kernel's sources change only with
// what it uses.
#pragma once

#include "pdf_internal.h"

namespace pdfk {

// Buffers of the particle redistribution (k_redist.hip)
struct RedistBuf {
  int32_t ne = 0;
  int64_t np = 0;
  int32_t *cnt = nullptr, *iota = nullptr, *skey = nullptr, *sval = nullptr, *role = nullptr;
  int4 *plan = nullptr;
  int32_t *psize = nullptr, *poff = nullptr, *fill = nullptr, *list = nullptr, *npairs = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0;
};
bool redist_alloc(RedistBuf &b, int32_t ne, int64_t np, void *(*alloc)(size_t, void *), void *user);

// elliptic relaxation for wp_ij: per-element L^2 classes and wall normals,
// Dirichlet flags and normals per node, conjugate-gradient vectors ([9][nn])
// and scalars
// Plain-aggregation hierarchy of the elliptic relaxation (k_amg.hip builds
// the chain on the host from the stiffness matrix over the free masters;
// k_elliptic.hip forms each level's values every solve).  Level l has n rows
// (vectors [n][9]) and a CSR pattern; its values, four L2 classes per entry,
// are sums of the finer level's values (the Galerkin product with the
// tentative prolongator, whose entries are all 1): coarse entry J sums the
// fine entries g_idx[g_off[J] .. g_off[J+1]).  Level 0 takes its values from
// the full matrix's entries g0 and its rows from the free masters fidx.
struct AggHostLevel {
  int32_t n = 0;
  std::vector<int32_t> off, col;     // pattern of this level
  std::vector<int32_t> agg;          // row -> aggregate (the next level's row); empty on the last
  std::vector<int32_t> m_off, mem;   // rows of each aggregate
  std::vector<int32_t> g_off, g_idx; // next level's entries as sums of this level's
};
// false if no coarsening is possible; the last level has at most max_last rows
bool agg_chain(int32_t n, const std::vector<int32_t> &off, const std::vector<int32_t> &col,
               const std::vector<double> &val, int32_t max_last, std::vector<AggHostLevel> &lv);
constexpr int ELL_MAXL = 16;
constexpr int32_t ELL_COARSE_MAX = 128;  // rows of the last level (its sweeps run in one workgroup's LDS)
struct EllMgLevel {
  int32_t n = 0, nnz = 0;
  const int32_t *off = nullptr, *col = nullptr;
  double4 *val = nullptr, *dinv = nullptr;  // values; inverse smoother diagonal per class
  double *b = nullptr, *x = nullptr, *r = nullptr, *y = nullptr;  // [n][9]
  const int32_t *agg = nullptr, *m_off = nullptr, *mem = nullptr, *g_off = nullptr, *g_idx = nullptr;
};
// With the multigrid the conjugate gradients run on compact vectors of the
// free rows ([n0][9], fidx maps them to nodes), and level 0 is the free-free
// block of the matrix: its pattern over the free rows is built once, its
// values are the full matrix's entries g0 of every solve.
struct EllMg {
  int nl = 0;  // 0: Jacobi preconditioning
  int sweeps = 8;  // smoothing sweeps on the last level
  const int32_t *fidx = nullptr, *g0 = nullptr;
  double *cx = nullptr, *cr = nullptr, *cz = nullptr, *cp = nullptr, *cq = nullptr, *cb = nullptr;
  EllMgLevel lv[ELL_MAXL];
};

struct EllBuf {
  EllMg mg;
  double4 *L2 = nullptr;
  double2 *nrm = nullptr, *dnv = nullptr;
  int8_t *dir = nullptr;                        // row role: 0 free master, 1 wall master, 2 not a master
  int32_t *row_off = nullptr, *cols = nullptr;  // CSR over master nodes (rows of other nodes empty)
  double *mv = nullptr;                         // mass matrix values
  double4 *av = nullptr;                        // M + L2 K for the four L2 classes
  double *f = nullptr;                          // local right-hand side, [9][nn]
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *diag = nullptr;  // [nn][9]
  double *scal = nullptr;
  int *stop = nullptr;
};
void launch_ell_normals(hipStream_t s, const MeshDev &m, int32_t nw, const double4 *wall, double2 *nrm);
// solves into wp ([9][nn], also the warm start), from the right-hand side f
// ([9][nn]); returns the iterations taken (the host checks convergence every
// 8 iterations, so the call waits for the stream)
int launch_ell_solve(hipStream_t s, const MeshDev &m, const ModelDev &md, const EllBuf &b, const double *S,
                     const double *f, double *wp, double tol, int maxit);

// stabilized pressure projection: stiffness matrix (CSR over the masters),
// the solved pressure P', the increment, CG vectors (nn), element gradients
// (dt grad dP), the gradient of the next prediction ([2][nn]) and scalars
// Smoothed-aggregation multigrid hierarchy of the projection's stiffness
// matrix (k_amg.hip): built on the host, applied as one V-cycle per
// conjugate-gradient step.  Level l holds A (CSR), D^-1, the damping omega and
// the prolongator P to level l+1 with its transpose; the last level is solved
// by a dense inverse.
constexpr int AMG_MAXL = 12;
struct AmgHostLevel {
  int32_t n = 0;
  double omega = 0.0;
  std::vector<int32_t> a_off, a_col, p_off, p_col, r_off, r_col;
  std::vector<double> a_val, dinv, p_val, r_val;
};
struct AmgHost {
  std::vector<AmgHostLevel> lv;
  std::vector<double> cinv;  // coarsest level, n x n row-major
};
// false if the hierarchy could not be built (the caller keeps Jacobi)
bool amg_build(int32_t n, const std::vector<int32_t> &off, const std::vector<int32_t> &col,
               const std::vector<double> &val, AmgHost &h);
struct AmgDevLevel {
  int32_t n = 0;
  int ga = 1, gp = 1, gr = 1;  // lanes per row of the products with A, P and P^T
  double omega = 0.0;
  const int32_t *a_off = nullptr, *a_col = nullptr, *p_off = nullptr, *p_col = nullptr, *r_off = nullptr,
                *r_col = nullptr;
  const double *a_val = nullptr, *dinv = nullptr, *p_val = nullptr, *r_val = nullptr;
  double *b = nullptr, *x = nullptr, *r = nullptr, *y = nullptr;
};
struct AmgDev {
  int nl = 0;
  AmgDevLevel lv[AMG_MAXL];
  const double *cinv = nullptr;
};
// zout[masters[k]] = (V-cycle applied to rin gathered at masters[k]), k < lv[0].n
void launch_amg_apply(hipStream_t s, const AmgDev &a, const int32_t *masters, const double *rin, double *zout,
                      const int *stop);

struct ProjBuf {
  AmgDev amg;  // nl == 0: Jacobi preconditioning
  int32_t *row_off = nullptr, *cols = nullptr;
  double *kval = nullptr, *kdiag = nullptr;
  double *P = nullptr, *dP = nullptr, *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr,
         *q = nullptr;
  double2 *ge = nullptr;
  double *gtot = nullptr;
  double *scal = nullptr;
  double *ring = nullptr;  // 8 x (p.q, r.z) of the conjugate-gradient iterations
  int *stop = nullptr;     // stop flag; the iteration counter follows it (iter = stop + 1)
  int *iter = nullptr;
  hipStream_t cap = nullptr;       // private stream on which the iteration chunk is captured
  hipGraphExec_t chunk = nullptr;  // 8 iterations as one graph (null: launched one by one)
  // wall edges of eq:wall-pressure-condition: (master a, master b, element,
  // wall-function edge) and (outward normal x, y, length, 0); the boundary
  // vectors B of the new data, of the data P' satisfies and of G.n
  int32_t nwe = 0;
  const int4 *we = nullptr;
  const double4 *wgeom = nullptr;
  double *Bnew = nullptr, *Bprev = nullptr, *BG = nullptr;
  bool wall_started = false;
};
void launch_proj_gradp(hipStream_t s, const MeshDev &m, const ProjBuf &b, const double *gin);
// from the predicted statistics S: dP, P' += dP, the particle correction and
// the shift of the element means (emom); returns the iterations taken (waits
// for the stream every 8 iterations; the 8 are one captured graph)
template <typename T>
int launch_proj_solve(hipStream_t s, const MeshDev &m, ProjBuf &b, const double *S, double Cp, double dt,
                      const double *dtp, double tol, int maxit, PartDev<T> p, int64_t np, double *emom,
                      double nu, const double *gin);

// velocity-conditioned scalar means (eq:IECM): per-element particle lists and
// the result cm (T[np], storage order)
struct CondBuf {
  int32_t ne = 0;
  int64_t np = 0;
  int32_t *cnt = nullptr, *off = nullptr, *cursor = nullptr, *big = nullptr, *mid = nullptr, *nbig = nullptr;
  int32_t *list = nullptr, *list2 = nullptr;
  void *cm = nullptr, *temp = nullptr;
  size_t temp_bytes = 0;
};
bool cond_alloc(CondBuf &b, int32_t ne, int64_t np, size_t tsize, void *(*alloc)(size_t, void *), void *user);
// elem_sums: the element sums of the last accumulation when their count slot
// holds the current particles per element (else null: counted afresh)
template <typename T>
hipError_t launch_cond_means(hipStream_t s, const ModelDev &md, const CondBuf &b, PartDev<T> p,
                             const double *elem_sums);
template <typename T>
hipError_t launch_redistribute(hipStream_t s, const KArgs *dka, const RedistBuf &b, const double *sums, int stride,
                               PartDev<T> p, int32_t min_ppe, uint64_t seed, uint32_t step,
                               unsigned long long *cnt);


}  // namespace pdfk
