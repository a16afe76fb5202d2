// Host side of the C ABI declared in include/pdf.h.
//
// Owns the device memory of a context, validates and uploads the mesh, builds
// the linked lists the method needs (Ch.3, Sec. Estimation of Eulerian
// statistics and Sec. Particle tracking: elements surrounding elements,
// elements surrounding nodes) and enqueues the per-step kernel pipeline on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "pdf_solvers.h"

using namespace pdfk;

struct pdf_ctx {
  int32_t prec = PDF_FP64;
  int32_t device = -1;        // the HIP device current at pdf_init_mesh
  hipStream_t stream = nullptr;
  pdf_allocator alloc{};
  bool has_alloc = false;
  std::string err;
  pdf_model_params params{};
  MeshDev md{};
  ModelDev model{};
  std::vector<void *> owned;
  // nodal fields
  double *stats_a = nullptr, *stats_b = nullptr, *stats_cur = nullptr, *stats_est = nullptr,
         *latest = nullptr;
  double *wp = nullptr, *gradp = nullptr;
  bool wp_set = false, gradp_set = false;
  // element data
  void *rec = nullptr;        // element records (NREC, or NRECS in the SHAPE mode, values each)
  double *sums = nullptr, *emom = nullptr;
  double *cfl = nullptr;      // time step of eq:CFL: dt, time advanced, running minimum
  double *nsums = nullptr;    // SHAPE: per-node weighted sums
  RedistBuf rb;               // particle redistribution (min_ppe > 0)
  CondBuf cb;                 // velocity-conditioned scalar means (IECM)
  EllBuf ell;                 // elliptic relaxation (PDF_WP_ELLIPTIC)
  ProjBuf pb;                 // pressure projection (params.proj)
  uint64_t proj_iters = 0;    // its conjugate-gradient iterations since the last counter reset
  uint64_t ell_iters = 0;     // conjugate-gradient iterations since the last counter reset
  int32_t *offs = nullptr, *cursor = nullptr, *blocksums = nullptr;
  // particles (two buffers for the reorder)
  void *pbuf[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t np = 0;
  int32_t ppe = 0;
  uint64_t seed = 0;
  uint32_t step = 0;
  bool seeded = false;
  unsigned long long *cnt = nullptr;
  KArgs *dka = nullptr;  // device copy of the mesh and model parameters
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_phase;
  double phase_ms[4] = {0, 0, 0, 0};
};

// ---------------------------------------------------------------------------
// Scratch of pdf_denoise_stats_noalloc: the features and network outputs of
// one chunk of nodes.  Each GPU the library runs on holds its own copy until
// the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (scratch_dev), never through the
// array's name.
// ---------------------------------------------------------------------------
namespace {
constexpr int32_t NOALLOC_CHUNK = 32768;  // nodes per chunk
constexpr size_t NOALLOC_BYTES = (size_t)NOALLOC_CHUNK * (PDF_DN_NIN + PDF_DN_NOUT) * sizeof(float);
constexpr int NOALLOC_MAX_DEV = 64;
void *scratch_dev[NOALLOC_MAX_DEV] = {nullptr};
std::mutex scratch_mu;
}  // namespace
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
// once per device, with that device current (called by pdf_init_mesh)
hipError_t scratch_setup(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_dev[dev]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  scratch_dev[dev] = ptr;
  return hipSuccess;
}

__global__ void k_clear_u64(unsigned long long *p) {
  if (threadIdx.x == 0) *p = 0ull;
}
}  // namespace

namespace {

pdf_status fail(pdf_ctx *c, pdf_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, call)                                                                       \
  do {                                                                                          \
    hipError_t _e = (call);                                                                     \
    if (_e != hipSuccess)                                                                       \
      return fail(ctx, PDF_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(_e));        \
  } while (0)

void *dalloc(pdf_ctx *c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~(size_t)255;
  void *p = nullptr;
  if (c->has_alloc) {
    p = c->alloc.alloc(bytes, c->alloc.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) c->owned.push_back(p);
  return p;
}

void dfree(pdf_ctx *c, void *p) {
  if (!p) return;
  auto it = std::find(c->owned.begin(), c->owned.end(), p);
  if (it != c->owned.end()) c->owned.erase(it);
  if (c->has_alloc)
    c->alloc.free(p, c->alloc.user);
  else
    (void)hipFree(p);
}

template <typename V>
bool upload(pdf_ctx *c, const std::vector<V> &h, const V **out) {
  V *d = (V *)dalloc(c, h.size() * sizeof(V));
  if (!d) return false;
  if (!h.empty() && hipMemcpyAsync(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return false;
  *out = d;
  return true;
}

size_t tsize(const pdf_ctx *c) { return c->prec == PDF_FP32 ? 4 : 8; }

template <typename T>
PartDev<T> part_view(pdf_ctx *c, int which) {
  char *b = (char *)c->pbuf[which];
  const int64_t n = c->np;
  PartDev<T> p;
  T *t = (T *)b;
  p.x = t;
  p.y = t + n;
  p.u = t + 2 * n;
  p.v = t + 3 * n;
  p.w = t + 4 * n;
  p.om = t + 5 * n;
  p.psi = t + 6 * n;
  char *ip = b + ((7 * n * sizeof(T) + 255) & ~(size_t)255);
  p.e = (int32_t *)ip;
  p.id = (uint32_t *)(ip + ((n * 4 + 255) & ~(size_t)255));
  return p;
}

size_t part_bytes(size_t tsz, int64_t n) {
  return ((7 * n * tsz + 255) & ~(size_t)255) + 2 * ((n * 4 + 255) & ~(size_t)255);
}

void mark(pdf_ctx *c, int phase) {
  if (!c->timing) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, c->stream);
  c->ev.push_back(e);
  c->ev_phase.push_back(phase);
}

// estimate the statistics of the current particle state from scratch:
// a first pass with zero references gives the element means, which become the
// references of a second, shifted pass (prev = nodal values kept for empty nodes)
template <typename T>
pdf_status estimate_from_scratch(pdf_ctx *c, const double *prev) {
  const int32_t ne = c->md.ne;
  T *rec = (T *)c->rec;
  if (c->model.stats_mode == PDF_STATS_SHAPE) {
    // two passes: weighted means about a zero reference, then all moments
    // about those means; nodes without weight keep prev
    const size_t nsb = (size_t)c->md.nn * NSUM * sizeof(double);
    launch_elem_prep_shape<T>(c->stream, c->md, c->model, nullptr, nullptr, nullptr, rec);
    HIPCHK(c, hipMemsetAsync(c->nsums, 0, nsb, c->stream));
    launch_accumulate_shape<T>(c->stream, c->md, part_view<T>(c, c->cur), c->np, rec, c->nsums);
    launch_node_stats_shape<T>(c->stream, c->md, c->nsums, nullptr, prev, c->stats_est, c->cnt);
    launch_elem_prep_shape<T>(c->stream, c->md, c->model, c->stats_est, nullptr, nullptr, rec);
    HIPCHK(c, hipMemsetAsync(c->nsums, 0, nsb, c->stream));
    launch_accumulate_shape<T>(c->stream, c->md, part_view<T>(c, c->cur), c->np, rec, c->nsums);
    launch_node_stats_shape<T>(c->stream, c->md, c->nsums, c->stats_est, prev, c->stats_est, c->cnt);
    launch_node_derivs(c->stream, c->md, c->stats_est);
    HIPCHK(c, hipGetLastError());
    std::swap(c->stats_cur, c->stats_est);
    c->latest = c->stats_cur;
    return PDF_OK;
  }
  HIPCHK(c, hipMemsetAsync(rec, 0, (size_t)ne * NREC * sizeof(T), c->stream));
  HIPCHK(c, hipMemsetAsync(c->sums, 0, (size_t)ne * NSUM * sizeof(double), c->stream));
  launch_accumulate<T>(c->stream, part_view<T>(c, c->cur), c->np, c->md.ne, rec, c->sums);
  launch_ref_from_sums<T>(c->stream, ne, c->sums, rec);
  HIPCHK(c, hipMemsetAsync(c->sums, 0, (size_t)ne * NSUM * sizeof(double), c->stream));
  launch_accumulate<T>(c->stream, part_view<T>(c, c->cur), c->np, c->md.ne, rec, c->sums);
  launch_elem_moments<T>(c->stream, ne, c->sums, rec, c->emom);
  launch_node_stats(c->stream, c->md, c->emom, prev, c->stats_est, c->cnt);
  launch_node_derivs(c->stream, c->md, c->stats_est);
  HIPCHK(c, hipGetLastError());
  // the estimate becomes the current statistics
  std::swap(c->stats_cur, c->stats_est);
  c->latest = c->stats_cur;
  return PDF_OK;
}

void *rb_alloc(size_t n, void *u) { return dalloc((pdf_ctx *)u, n); }

bool redist_reserve(pdf_ctx *c) {
  if (c->rb.cnt && c->rb.np == c->np) return true;
  RedistBuf &b = c->rb;
  void *old[] = {b.cnt, b.iota, b.skey, b.sval, b.role, b.plan, b.psize, b.poff, b.fill, b.list, b.npairs, b.temp};
  for (void *q : old) dfree(c, q);
  b = RedistBuf();
  return redist_alloc(b, c->md.ne, c->np, rb_alloc, c);
}

bool cond_reserve(pdf_ctx *c) {
  if (c->cb.cnt && c->cb.np == c->np) return true;
  CondBuf &b = c->cb;
  void *old[] = {b.cnt, b.off, b.cursor, b.big, b.mid, b.nbig, b.list, b.list2, b.cm, b.temp};
  for (void *q : old) dfree(c, q);
  b = CondBuf();
  if (!cond_alloc(b, c->md.ne, c->np, tsize(c), rb_alloc, c)) return false;
  // valid particle indices from the start, whatever a list position holds
  return hipMemsetAsync(b.list, 0, (size_t)(c->np > 0 ? c->np : 1) * 4, c->stream) == hipSuccess;
}

// CSR sparsity over the master nodes: row a holds the masters of the
// elements around a (sorted); rows of identified nodes are empty
void master_csr(const pdf_mesh_desc *mesh, std::vector<int32_t> &row_off, std::vector<int32_t> &cols) {
  const int32_t nn = mesh->n_nodes, ne = mesh->n_elems;
  const int32_t *en = mesh->elem_nodes, *master = mesh->node_master;
  std::vector<std::vector<int32_t>> adj((size_t)nn);
  for (int32_t e = 0; e < ne; ++e)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) adj[master[en[3 * e + i]]].push_back(master[en[3 * e + j]]);
  row_off.assign((size_t)nn + 1, 0);
  cols.clear();
  for (int32_t n = 0; n < nn; ++n) {
    std::vector<int32_t> &r = adj[n];
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    row_off[n + 1] = row_off[n] + (int32_t)r.size();
    cols.insert(cols.end(), r.begin(), r.end());
  }
}

// pressure projection: the stiffness matrix (assembled once on the host, the
// element entries A grad N_a . grad N_b added into the masters' rows) and the
// buffers
// the stiffness matrix over the masters on the pattern of master_csr: the
// element entries A grad N_a . grad N_b added into the masters' rows
void stiffness_values(const pdf_mesh_desc *mesh, const std::vector<int32_t> &row_off,
                      const std::vector<int32_t> &cols, std::vector<double> &kval) {
  const int32_t ne = mesh->n_elems;
  const double *xy = mesh->node_xy;
  const int32_t *en = mesh->elem_nodes, *master = mesh->node_master;
  kval.assign(cols.size(), 0.0);
  for (int32_t e = 0; e < ne; ++e) {
    const int32_t n0 = en[3 * e], n1 = en[3 * e + 1], n2 = en[3 * e + 2];
    const double xBA = xy[2 * n1] - xy[2 * n0], yBA = xy[2 * n1 + 1] - xy[2 * n0 + 1];
    const double xCA = xy[2 * n2] - xy[2 * n0], yCA = xy[2 * n2 + 1] - xy[2 * n0 + 1];
    const double twoA = xBA * yCA - xCA * yBA, A = 0.5 * twoA;
    const double dx[3] = {(yBA - yCA) / twoA, yCA / twoA, -yBA / twoA};
    const double dy[3] = {(xCA - xBA) / twoA, -xCA / twoA, xBA / twoA};
    for (int i = 0; i < 3; ++i) {
      const int32_t qa = master[en[3 * e + i]];
      for (int j = 0; j < 3; ++j) {
        const int32_t qb = master[en[3 * e + j]];
        const int32_t *r0 = cols.data() + row_off[qa], *r1 = cols.data() + row_off[qa + 1];
        const int32_t pos = (int32_t)(std::lower_bound(r0, r1, qb) - cols.data());
        kval[pos] += A * (dx[i] * dx[j] + dy[i] * dy[j]);
      }
    }
  }
}

pdf_status proj_setup(pdf_ctx *c, const pdf_mesh_desc *mesh) {
  const int32_t nn = c->md.nn, ne = c->md.ne;
  ProjBuf &b = c->pb;
  std::vector<int32_t> row_off, cols;
  master_csr(mesh, row_off, cols);
  std::vector<double> kval, kdiag((size_t)nn, 1.0);
  stiffness_values(mesh, row_off, cols, kval);
  const double *xy = mesh->node_xy;
  const int32_t *en = mesh->elem_nodes, *master = mesh->node_master;
  for (int32_t n = 0; n < nn; ++n)
    for (int32_t j = row_off[n]; j < row_off[n + 1]; ++j)
      if (cols[j] == n) kdiag[n] = kval[j] > 0.0 ? kval[j] : 1.0;
  const size_t vn = (size_t)nn * sizeof(double);
  bool ok = upload(c, row_off, (const int32_t **)&b.row_off) && upload(c, cols, (const int32_t **)&b.cols) &&
            upload(c, kval, (const double **)&b.kval) && upload(c, kdiag, (const double **)&b.kdiag);
  b.P = (double *)dalloc(c, vn);
  b.dP = (double *)dalloc(c, vn);
  b.b = (double *)dalloc(c, vn);
  b.x = (double *)dalloc(c, vn);
  b.r = (double *)dalloc(c, vn);
  b.z = (double *)dalloc(c, vn);
  b.p = (double *)dalloc(c, vn);
  b.q = (double *)dalloc(c, vn);
  b.ge = (double2 *)dalloc(c, (size_t)ne * sizeof(double2));
  b.gtot = (double *)dalloc(c, 2 * vn);
  b.scal = (double *)dalloc(c, 4 * sizeof(double));
  b.ring = (double *)dalloc(c, 16 * sizeof(double));
  b.stop = (int *)dalloc(c, 256);
  b.iter = b.stop ? b.stop + 1 : nullptr;
  ok = ok && b.P && b.dP && b.b && b.x && b.r && b.z && b.p && b.q && b.ge && b.gtot && b.scal && b.ring && b.stop;
  if (!ok) return fail(c, PDF_E_OOM, "pressure projection buffers");
  // the wall edges of eq:wall-pressure-condition: every non-periodic boundary
  // edge, from local node k+1 to k+2 of its element (the domain on its left),
  // its outward unit normal and length
  {
    std::vector<int4> we;
    std::vector<double4> wg;
    for (int32_t bi = 0; bi < mesh->n_bedges; ++bi) {
      if (mesh->bedge_type[bi] == PDF_BC_PERIODIC || mesh->bedge_type[bi] == PDF_BC_OUTFLOW) continue;
      const int32_t e = mesh->bedge_elem[bi], k = mesh->bedge_local[bi];
      const int32_t na = en[3 * e + (k + 1) % 3], nb = en[3 * e + (k + 2) % 3];
      const double dx = xy[2 * nb] - xy[2 * na], dy = xy[2 * nb + 1] - xy[2 * na + 1];
      const double L = std::sqrt(dx * dx + dy * dy);
      we.push_back(make_int4(master[na], master[nb], e, mesh->bedge_type[bi] == PDF_BC_WALLFN ? 1 : 0));
      wg.push_back(make_double4(dy / L, -dx / L, L, 0.0));
    }
    b.nwe = (int32_t)we.size();
    if (b.nwe > 0) {
      ok = upload(c, we, &b.we) && upload(c, wg, &b.wgeom);
      b.Bnew = (double *)dalloc(c, vn);
      b.Bprev = (double *)dalloc(c, vn);
      b.BG = (double *)dalloc(c, vn);
      if (!ok || !b.Bnew || !b.Bprev || !b.BG) return fail(c, PDF_E_OOM, "pressure projection wall buffers");
      HIPCHK(c, hipStreamSynchronize(c->stream));  // the host arrays end with this block
    }
    b.wall_started = false;
  }
  // the conjugate-gradient iterations are captured on a stream of the
  // library's own (capture is not possible on the legacy default stream);
  // without it they are launched one by one
  if (hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking) != hipSuccess) b.cap = nullptr;
  AmgHost h;  // kept until the uploads below have completed
  if (c->params.proj_precond == 1) {
    // K over the masters in their compact order (the k-th master is the k-th
    // node that is its own master, as in the device list of masters)
    std::vector<int32_t> cidx((size_t)nn, -1);
    int32_t nm = 0;
    for (int32_t n = 0; n < nn; ++n)
      if (master[n] == n) cidx[n] = nm++;
    std::vector<int32_t> aoff((size_t)nm + 1, 0), acol;
    std::vector<double> aval;
    for (int32_t n = 0; n < nn; ++n) {
      if (master[n] != n) continue;
      for (int32_t j = row_off[n]; j < row_off[n + 1]; ++j) {
        acol.push_back(cidx[cols[j]]);
        aval.push_back(kval[j]);
      }
      aoff[cidx[n] + 1] = (int32_t)acol.size();
    }
    if (!amg_build(nm, aoff, acol, aval, h))
      return fail(c, PDF_E_NUMERIC, "the multigrid hierarchy of the projection could not be built");
    AmgDev &a = b.amg;
    a.nl = (int)h.lv.size();
    for (int l = 0; l < a.nl; ++l) {
      const AmgHostLevel &H = h.lv[l];
      AmgDevLevel &D = a.lv[l];
      D.n = H.n;
      D.omega = H.omega;
      // lanes per row: the power of two at or above the mean row length, at most 64
      auto lanes = [](const std::vector<int32_t> &off) {
        const int32_t rows = (int32_t)off.size() - 1;
        const double mean = rows > 0 ? (double)off.back() / rows : 1.0;
        int g = 1;
        while (g < 64 && g < mean) g *= 2;
        return g;
      };
      if (l + 1 < a.nl) {
        D.ga = lanes(H.a_off);
        D.gp = lanes(H.p_off);
        D.gr = lanes(H.r_off);
      }
      const size_t vb = (size_t)H.n * sizeof(double);
      D.b = (double *)dalloc(c, vb);
      D.y = (double *)dalloc(c, vb);
      ok = ok && D.b && D.y;
      if (l + 1 < a.nl) {
        D.x = (double *)dalloc(c, vb);
        D.r = (double *)dalloc(c, vb);
        ok = ok && D.x && D.r && upload(c, H.a_off, &D.a_off) && upload(c, H.a_col, &D.a_col) &&
             upload(c, H.a_val, &D.a_val) && upload(c, H.dinv, &D.dinv) && upload(c, H.p_off, &D.p_off) &&
             upload(c, H.p_col, &D.p_col) && upload(c, H.p_val, &D.p_val) && upload(c, H.r_off, &D.r_off) &&
             upload(c, H.r_col, &D.r_col) && upload(c, H.r_val, &D.r_val);
      }
    }
    ok = ok && upload(c, h.cinv, &a.cinv);
    if (!ok) return fail(c, PDF_E_OOM, "multigrid hierarchy of the projection");
  }
  HIPCHK(c, hipMemsetAsync(b.P, 0, vn, c->stream));
  HIPCHK(c, hipMemsetAsync(b.dP, 0, vn, c->stream));
  HIPCHK(c, hipMemsetAsync(b.gtot, 0, 2 * vn, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PDF_OK;
}

// elliptic relaxation: buffers, the nodes of no-slip edges (Dirichlet rows)
// with the normalised sum of their edges' outward unit normals, and each
// element's closest no-slip wall normal (computed once, on the device)
pdf_status ell_setup(pdf_ctx *c, const pdf_mesh_desc *mesh) {
  const int32_t nn = c->md.nn, ne = c->md.ne, nb = mesh->n_bedges;
  EllBuf &b = c->ell;
  const size_t v9 = 9 * (size_t)nn * sizeof(double);
  b.L2 = (double4 *)dalloc(c, (size_t)ne * sizeof(double4));
  b.nrm = (double2 *)dalloc(c, (size_t)ne * sizeof(double2));
  b.dnv = (double2 *)dalloc(c, (size_t)nn * sizeof(double2));
  b.dir = (int8_t *)dalloc(c, (size_t)nn);
  b.f = (double *)dalloc(c, v9);
  b.x = (double *)dalloc(c, v9);
  b.r = (double *)dalloc(c, v9);
  b.z = (double *)dalloc(c, v9);
  b.p = (double *)dalloc(c, v9);
  b.q = (double *)dalloc(c, v9);
  b.diag = (double *)dalloc(c, v9);
  b.scal = (double *)dalloc(c, (size_t)(18 * (c->params.ell_maxit + 1)) * sizeof(double));
  b.stop = (int *)dalloc(c, 256);
  if (!b.L2 || !b.nrm || !b.dnv || !b.dir || !b.f || !b.x || !b.r || !b.z || !b.p || !b.q || !b.diag || !b.scal ||
      !b.stop)
    return fail(c, PDF_E_OOM, "elliptic relaxation buffers");
  const double *xy = mesh->node_xy;
  const int32_t *en = mesh->elem_nodes, *master = mesh->node_master;
  std::vector<int32_t> row_off, cols;
  master_csr(mesh, row_off, cols);
  const size_t nnz = cols.size();
  b.mv = (double *)dalloc(c, (nnz + 1) * sizeof(double));
  b.av = (double4 *)dalloc(c, (nnz + 1) * sizeof(double4));
  if (!b.mv || !b.av || !upload(c, row_off, (const int32_t **)&b.row_off) ||
      !upload(c, cols, (const int32_t **)&b.cols))
    return fail(c, PDF_E_OOM, "elliptic relaxation matrix");
  std::vector<double4> wall;
  std::vector<double2> dn((size_t)nn, make_double2(0.0, 0.0));
  std::vector<int8_t> dir((size_t)nn, 0);
  for (int32_t e = 0; e < nb; ++e) {
    if (mesh->bedge_type[e] != PDF_BC_NOSLIP) continue;
    const int32_t el = mesh->bedge_elem[e], k = mesh->bedge_local[e];
    const int32_t na = en[3 * el + (k + 1) % 3], nc = en[3 * el + (k + 2) % 3];
    const double xa = xy[2 * na], ya = xy[2 * na + 1], xb = xy[2 * nc], yb = xy[2 * nc + 1];
    wall.push_back(make_double4(xa, ya, xb, yb));
    const double dx = xb - xa, dy = yb - ya, len = std::sqrt(dx * dx + dy * dy);
    for (const int32_t n : {master[na], master[nc]}) {
      dn[n].x += dy / len;
      dn[n].y += -dx / len;
      dir[n] = 1;
    }
  }
  for (int32_t n = 0; n < nn; ++n)
    if (dir[n]) {
      const double l = std::sqrt(dn[n].x * dn[n].x + dn[n].y * dn[n].y);
      dn[n].x /= l;
      dn[n].y /= l;
    }
  // row roles: 0 a free master row, 1 a wall (Dirichlet) master row, 2 no row
  for (int32_t n = 0; n < nn; ++n)
    if (master[n] != n) dir[n] = 2;
  hipStream_t s = c->stream;
  HIPCHK(c, hipMemcpyAsync(b.dnv, dn.data(), dn.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(b.dir, dir.data(), dir.size(), hipMemcpyHostToDevice, s));
  double4 *wd = (double4 *)dalloc(c, (wall.size() + 1) * sizeof(double4));
  if (!wd) return fail(c, PDF_E_OOM, "elliptic relaxation wall list");
  if (!wall.empty())
    HIPCHK(c, hipMemcpyAsync(wd, wall.data(), wall.size() * sizeof(double4), hipMemcpyHostToDevice, s));
  launch_ell_normals(s, c->md, (int32_t)wall.size(), wd, b.nrm);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  dfree(c, wd);
  if (c->params.ell_precond == 1) {
    // the multigrid hierarchy over the free masters (row role 0), in node
    // order; its aggregates come from the stiffness matrix
    std::vector<double> kval;
    stiffness_values(mesh, row_off, cols, kval);
    std::vector<int32_t> fidx, lidx((size_t)nn, -1);
    for (int32_t n = 0; n < nn; ++n)
      if (dir[n] == 0) {
        lidx[n] = (int32_t)fidx.size();
        fidx.push_back(n);
      }
    const int32_t n0 = (int32_t)fidx.size();
    if (n0 > 0) {
      std::vector<int32_t> off0((size_t)n0 + 1, 0), col0, g0;
      std::vector<double> val0;
      for (int32_t k = 0; k < n0; ++k) {
        const int32_t a = fidx[k];
        for (int32_t j = row_off[a]; j < row_off[a + 1]; ++j)
          if (lidx[cols[j]] >= 0) {
            col0.push_back(lidx[cols[j]]);
            g0.push_back(j);
            val0.push_back(kval[j]);
          }
        off0[k + 1] = (int32_t)col0.size();
      }
      std::vector<AggHostLevel> lv;
      if (!agg_chain(n0, off0, col0, val0, ELL_COARSE_MAX, lv))
        return fail(c, PDF_E_NUMERIC, "the multigrid hierarchy of the elliptic relaxation could not be built");
      EllMg &g = b.mg;
      const size_t c9b = 9 * (size_t)n0 * sizeof(double);
      g.cx = (double *)dalloc(c, c9b);
      g.cr = (double *)dalloc(c, c9b);
      g.cz = (double *)dalloc(c, c9b);
      g.cp = (double *)dalloc(c, c9b);
      g.cq = (double *)dalloc(c, c9b);
      g.cb = (double *)dalloc(c, c9b);
      bool ok = g.cx && g.cr && g.cz && g.cp && g.cq && g.cb && upload(c, fidx, &g.fidx) && upload(c, g0, &g.g0);
      for (size_t l = 0; l < lv.size() && ok; ++l) {
        const AggHostLevel &H = lv[l];
        EllMgLevel &D = g.lv[l];
        D.n = H.n;
        D.nnz = (int32_t)H.col.size();
        const size_t v9b = 9 * (size_t)H.n * sizeof(double);
        D.val = (double4 *)dalloc(c, ((size_t)D.nnz + 1) * sizeof(double4));
        D.dinv = (double4 *)dalloc(c, (size_t)H.n * sizeof(double4));
        D.r = (double *)dalloc(c, v9b);
        ok = D.val && D.dinv && D.r && upload(c, H.off, &D.off) && upload(c, H.col, &D.col);
        if (ok && l > 0) {  // level 0 takes its input and output vectors from the caller
          D.b = (double *)dalloc(c, v9b);
          D.y = (double *)dalloc(c, v9b);
          ok = D.b && D.y;
        }
        if (ok && l + 1 < lv.size())
          ok = upload(c, H.agg, &D.agg) && upload(c, H.m_off, &D.m_off) && upload(c, H.mem, &D.mem) &&
               upload(c, H.g_off, &D.g_off) && upload(c, H.g_idx, &D.g_idx);
      }
      if (!ok) return fail(c, PDF_E_OOM, "multigrid hierarchy of the elliptic relaxation");
      g.nl = (int)lv.size();
      g.sweeps = 8;
      HIPCHK(c, hipStreamSynchronize(s));  // the host arrays end with this block
    }
  }
  return PDF_OK;
}

template <typename T>
pdf_status advance_impl(pdf_ctx *c, int32_t nsteps, double dt, const double *cfl) {
  const int32_t ne = c->md.ne;
  T *rec = (T *)c->rec;
  if (c->params.min_ppe > 0 && !redist_reserve(c)) return fail(c, PDF_E_OOM, "redistribution buffers");
  const bool iecm = c->params.mix_model == PDF_MIX_IECM;
  if (iecm && !cond_reserve(c)) return fail(c, PDF_E_OOM, "conditioned-mean buffers");
  // cfl = {C_CFL, dt_max}: each step's dt is formed on the device from the
  // current statistics and read there by the record and particle kernels
  const double *dtp = cfl ? c->cfl : nullptr;
  if (cfl) launch_cfl_begin(c->stream, c->cfl);
  for (int32_t s = 0; s < nsteps; ++s) {
    mark(c, 4);
    if (cfl) launch_cfl_dt(c->stream, c->md, c->stats_cur, cfl[0], cfl[1], c->cfl);
    if (c->params.min_ppe > 0) {
      // particle counts per element: the count slot of the element sums (the
      // last accumulation, ELEM) or a fresh count (SHAPE)
      if (c->model.stats_mode == PDF_STATS_SHAPE) {
        HIPCHK(c, hipMemsetAsync(c->sums, 0, (size_t)ne * NSUM * sizeof(double), c->stream));
        launch_elem_count<T>(c->stream, part_view<T>(c, c->cur), c->np, c->sums);
      }
      HIPCHK(c, launch_redistribute<T>(c->stream, c->dka, c->rb, c->sums, NSUM, part_view<T>(c, c->cur),
                                       c->params.min_ppe, c->seed, c->step, c->cnt));
    }
    // eq:IECM: <phi|V> of every particle from the state at the start of the step
    const T *cm = nullptr;
    if (iecm) {
      // ELEM statistics without redistribution: the last accumulation's count
      // slot holds the particles per element
      const bool sums_valid = c->model.stats_mode == PDF_STATS_ELEM && c->params.min_ppe == 0;
      HIPCHK(c, launch_cond_means<T>(c->stream, c->model, c->cb, part_view<T>(c, c->cur),
                                     sums_valid ? c->sums : nullptr));
      cm = (const T *)c->cb.cm;
    }
    mark(c, 0);
    if (c->params.model == PDF_MODEL_GLM && c->params.wp_source == PDF_WP_LOCAL)
      launch_local_wp(c->stream, c->md, c->model, c->stats_cur, c->wp);
    if (c->params.model == PDF_MODEL_GLM && c->params.wp_source == PDF_WP_ELLIPTIC) {
      // the local right-hand side, then the solve from the previous wp
      launch_local_wp(c->stream, c->md, c->model, c->stats_cur, c->ell.f);
      c->ell_iters += (uint64_t)launch_ell_solve(c->stream, c->md, c->model, c->ell, c->stats_cur, c->ell.f, c->wp,
                                                 c->params.ell_tol, c->params.ell_maxit);
      HIPCHK(c, hipGetLastError());
    }
    const bool shape = c->model.stats_mode == PDF_STATS_SHAPE;
    const bool proj = c->params.proj != 0;
    // the mean-pressure gradient of the prediction: the input, plus grad P'
    // with the projection
    if (proj) launch_proj_gradp(c->stream, c->md, c->pb, c->gradp_set ? c->gradp : nullptr);
    const double *gp = proj ? c->pb.gtot : (c->gradp_set ? c->gradp : nullptr);
    if (shape) {
      launch_elem_prep_shape<T>(c->stream, c->md, c->model, c->stats_cur,
                                c->params.model == PDF_MODEL_GLM ? c->wp : nullptr,
                                c->gradp_set ? c->gradp : nullptr, rec);
      HIPCHK(c, hipMemsetAsync(c->nsums, 0, (size_t)c->md.nn * NSUM * sizeof(double), c->stream));
    } else {
      launch_elem_prep<T>(c->stream, c->md, c->model, c->stats_cur,
                          c->params.model == PDF_MODEL_GLM ? c->wp : nullptr, gp, dt, dtp, rec);
      HIPCHK(c, hipMemsetAsync(c->sums, 0, (size_t)ne * NSUM * sizeof(double), c->stream));
    }
    mark(c, 1);
    launch_advance<T>(c->stream, c->dka, c->model, part_view<T>(c, c->cur), c->np, c->md.ne, rec,
                      shape ? c->nsums : c->sums, c->seed, c->step, dt, dtp, cm, c->stats_cur,
                      c->gradp_set ? c->gradp : nullptr, c->cnt);
    mark(c, 2);
    if (shape) {
      launch_node_stats_shape<T>(c->stream, c->md, c->nsums, c->stats_cur, c->stats_cur, c->stats_est,
                                 c->cnt);
    } else {
      launch_elem_moments<T>(c->stream, ne, c->sums, rec, c->emom);
      launch_node_stats(c->stream, c->md, c->emom, c->stats_cur, c->stats_est, c->cnt);
    }
    launch_node_derivs(c->stream, c->md, c->stats_est);
    if (proj) {
      // eq:pressure-projection-smooth from the predicted statistics, the
      // correction of the particles and element means, then the statistics
      // of the corrected particles
      c->proj_iters += (uint64_t)launch_proj_solve<T>(c->stream, c->md, c->pb, c->stats_est, c->params.Cp, dt, dtp,
                                                      c->params.proj_tol, c->params.proj_maxit,
                                                      part_view<T>(c, c->cur), c->np, c->emom, c->params.nu,
                                                      c->gradp_set ? c->gradp : nullptr);
      launch_node_stats(c->stream, c->md, c->emom, c->stats_cur, c->stats_est, c->cnt);
      launch_node_derivs(c->stream, c->md, c->stats_est);
      HIPCHK(c, hipGetLastError());
    }
    if (!c->params.frozen) {
      std::swap(c->stats_cur, c->stats_est);
      c->latest = c->stats_cur;
    } else {
      c->latest = c->stats_est;
    }
    c->step++;
    mark(c, 3);
    if (c->params.reorder_every > 0 && (c->step % (uint32_t)c->params.reorder_every) == 0) {
      if (shape) {  // the sort needs the particles per element
        HIPCHK(c, hipMemsetAsync(c->sums, 0, (size_t)ne * NSUM * sizeof(double), c->stream));
        launch_elem_count<T>(c->stream, part_view<T>(c, c->cur), c->np, c->sums);
      }
      launch_reorder<T>(c->stream, ne, c->np, c->sums, c->offs, c->cursor, c->blocksums,
                        part_view<T>(c, c->cur), part_view<T>(c, 1 - c->cur));
      c->cur = 1 - c->cur;
    }
    mark(c, 5);
    HIPCHK(c, hipGetLastError());
  }
  return PDF_OK;
}

}  // namespace

extern "C" {

const char *pdf_last_error(const pdf_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void pdf_destroy(pdf_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto e : ctx->ev) (void)hipEventDestroy(e);
  if (ctx->pb.chunk) (void)hipGraphExecDestroy(ctx->pb.chunk);
  if (ctx->pb.cap) (void)hipStreamDestroy(ctx->pb.cap);
  std::vector<void *> own = ctx->owned;
  for (void *p : own) dfree(ctx, p);
  delete ctx;
}

pdf_status pdf_init_mesh(const pdf_mesh_desc *mesh, const pdf_model_params *params, int32_t precision,
                         const pdf_allocator *alloc, void *hip_stream, pdf_ctx **out) {
  if (!out) return PDF_E_INVALID_ARG;
  *out = nullptr;
  if (!mesh || !params || (precision != PDF_FP32 && precision != PDF_FP64)) return PDF_E_INVALID_ARG;
  if (mesh->n_nodes <= 0 || mesh->n_elems <= 0 || mesh->n_bedges < 0 || !mesh->node_xy ||
      !mesh->elem_nodes || !mesh->elem_nbr || !mesh->node_master ||
      (mesh->n_bedges > 0 && (!mesh->bedge_elem || !mesh->bedge_local || !mesh->bedge_type ||
                              !mesh->bedge_partner || !mesh->bedge_shift)))
    return PDF_E_INVALID_ARG;
  if (params->model != PDF_MODEL_SLM && params->model != PDF_MODEL_GLM) return PDF_E_INVALID_ARG;
  if (params->stats_mode != PDF_STATS_ELEM && params->stats_mode != PDF_STATS_SHAPE) return PDF_E_INVALID_ARG;
  if (params->min_ppe < 0 || params->min_ppe > 64) return PDF_E_INVALID_ARG;
  if (params->tm_mode < PDF_TM_CPHI || params->tm_mode > PDF_TM_SOURCE) return PDF_E_INVALID_ARG;
  if (params->wp_source < PDF_WP_INPUT || params->wp_source > PDF_WP_ELLIPTIC) return PDF_E_INVALID_ARG;
  if (params->proj != 0 && params->proj != 1) return PDF_E_INVALID_ARG;
  if (params->proj &&
      (params->stats_mode != PDF_STATS_ELEM || params->frozen || !(params->Cp >= 0.0) || !std::isfinite(params->Cp) ||
       params->proj_maxit < 1 || params->proj_maxit > 100000 || !(params->proj_tol > 0.0) ||
       !std::isfinite(params->proj_tol) || (params->proj_precond != 0 && params->proj_precond != 1)))
    return PDF_E_INVALID_ARG;
  if (params->model == PDF_MODEL_GLM && params->wp_source == PDF_WP_ELLIPTIC &&
      (params->ell_maxit < 1 || params->ell_maxit > 100000 || !(params->ell_tol > 0.0) ||
       !std::isfinite(params->ell_tol) || (params->ell_precond != 0 && params->ell_precond != 1)))
    return PDF_E_INVALID_ARG;
  // wall functions replace the viscous terms of the particle equations and
  // need the viscosity of the log law
  bool has_wallfn = false;
  for (int32_t b = 0; b < mesh->n_bedges; ++b) has_wallfn |= mesh->bedge_type[b] == PDF_BC_WALLFN;
  if (!std::isfinite(params->inflow_u)) return PDF_E_INVALID_ARG;
  if (has_wallfn && (params->nu != 0.0 || !(params->nu_wall > 0.0) || !std::isfinite(params->nu_wall)))
    return PDF_E_INVALID_ARG;
  if (params->mix_model != PDF_MIX_IEM && params->mix_model != PDF_MIX_IECM) return PDF_E_INVALID_ARG;
  if (params->cond_nu < 1 || params->cond_nu > 16 || params->cond_nv < 1 || params->cond_nv > 16 ||
      params->cond_nw < 1 || params->cond_nw > 16 || params->cond_min < 1 || params->cond_min > 64)
    return PDF_E_INVALID_ARG;
  if (!(params->C4 > 0.0 && params->C4 <= 1.0) || params->nu < 0.0 || params->reorder_every < 0)
    return PDF_E_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return PDF_E_DEVICE;
  pdf_ctx *c = new pdf_ctx();
  c->prec = precision;
  c->device = dev;
  c->stream = (hipStream_t)hip_stream;
  if (scratch_setup(dev) != hipSuccess) {
    c->err = "hipGetSymbolAddress of the allocation-free scratch failed on device " + std::to_string(dev);
    *out = c;  // the caller can read the message, then destroy
    return PDF_E_DEVICE;
  }
  c->params = *params;
  if (alloc && alloc->alloc && alloc->free) {
    c->alloc = *alloc;
    c->has_alloc = true;
  }
  const int32_t nn = mesh->n_nodes, ne = mesh->n_elems, nb = mesh->n_bedges;
  const double *xy = mesh->node_xy;
  const int32_t *en = mesh->elem_nodes, *nbr = mesh->elem_nbr, *master = mesh->node_master;
  // ---- validation ----
  auto bad = [&](const std::string &m) {
    c->err = m;
    *out = c;  // the caller can read the message, then destroy
    return PDF_E_BAD_MESH;
  };
  for (int32_t n = 0; n < nn; ++n) {
    if (master[n] < 0 || master[n] >= nn || master[master[n]] != master[n])
      return bad("node_master is not a projection at node " + std::to_string(n));
  }
  std::vector<ElemGeo> geo(ne);
  std::vector<double> dN(6 * (size_t)ne), area(ne);
  std::vector<int32_t> mnode(3 * (size_t)ne);
  for (int32_t e = 0; e < ne; ++e) {
    ElemGeo &g = geo[e];
    for (int k = 0; k < 3; ++k) {
      const int32_t n = en[3 * e + k];
      if (n < 0 || n >= nn) return bad("element node out of range in element " + std::to_string(e));
      g.n[k] = n;
      g.x[k] = xy[2 * n];
      g.y[k] = xy[2 * n + 1];
      g.nb[k] = nbr[3 * e + k];
      mnode[3 * e + k] = master[n];
    }
    // shape-function derivatives of the linear triangle (Ch.3, Sec. Derivatives)
    const double xBA = g.x[1] - g.x[0], yBA = g.y[1] - g.y[0];
    const double xCA = g.x[2] - g.x[0], yCA = g.y[2] - g.y[0];
    const double twoA = xBA * yCA - xCA * yBA;
    if (!(twoA > 0.0)) return bad("non-positive area or clockwise element " + std::to_string(e));
    area[e] = 0.5 * twoA;
    dN[6 * e + 0] = (yBA - yCA) / twoA;
    dN[6 * e + 1] = yCA / twoA;
    dN[6 * e + 2] = -yBA / twoA;
    dN[6 * e + 3] = (xCA - xBA) / twoA;
    dN[6 * e + 4] = -xCA / twoA;
    dN[6 * e + 5] = xBA / twoA;
  }
  for (int32_t e = 0; e < ne; ++e)
    for (int k = 0; k < 3; ++k) {
      const int32_t o = nbr[3 * e + k];
      if (o >= 0) {
        if (o >= ne) return bad("neighbour out of range in element " + std::to_string(e));
        const int32_t a = en[3 * e + (k + 1) % 3], b = en[3 * e + (k + 2) % 3];
        bool ok = false;
        for (int j = 0; j < 3; ++j)
          if (nbr[3 * o + j] == e && en[3 * o + (j + 1) % 3] == b && en[3 * o + (j + 2) % 3] == a) ok = true;
        if (!ok) return bad("neighbour table not symmetric at element " + std::to_string(e));
      } else {
        const int32_t b = -(o + 1);
        if (b >= nb || mesh->bedge_elem[b] != e || mesh->bedge_local[b] != k)
          return bad("boundary edge table inconsistent at element " + std::to_string(e));
      }
    }
  for (int32_t b = 0; b < nb; ++b) {
    const int32_t t = mesh->bedge_type[b];
    if (t != PDF_BC_PERIODIC && t != PDF_BC_SLIP && t != PDF_BC_NOSLIP && t != PDF_BC_WALLFN &&
        t != PDF_BC_OUTFLOW)
      return bad("unknown boundary type at edge " + std::to_string(b));
    const int32_t e = mesh->bedge_elem[b], k = mesh->bedge_local[b];
    if (e < 0 || e >= ne || k < 0 || k > 2 || nbr[3 * e + k] != -(b + 1))
      return bad("boundary edge " + std::to_string(b) + " does not match elem_nbr");
    if (t == PDF_BC_PERIODIC || t == PDF_BC_OUTFLOW) {
      // a periodic edge pairs with a periodic or an outflow edge, an outflow
      // edge with a periodic (inflow) edge
      const int32_t p = mesh->bedge_partner[b];
      if (p < 0 || p >= nb || mesh->bedge_partner[p] != b ||
          !(mesh->bedge_type[p] == PDF_BC_PERIODIC || (t == PDF_BC_PERIODIC && mesh->bedge_type[p] == PDF_BC_OUTFLOW)))
        return bad("periodic partner not mutual at edge " + std::to_string(b));
    }
  }
  // ---- linked lists ----
  // elements surrounding nodes (ascending element index)
  std::vector<int32_t> n2e_off(nn + 1, 0), n2e(3 * (size_t)ne);
  for (int32_t i = 0; i < 3 * ne; ++i) n2e_off[en[i] + 1]++;
  for (int32_t n = 0; n < nn; ++n) n2e_off[n + 1] += n2e_off[n];
  {
    std::vector<int32_t> fill(n2e_off.begin(), n2e_off.end() - 1);
    for (int32_t e = 0; e < ne; ++e)
      for (int k = 0; k < 3; ++k) n2e[fill[en[3 * e + k]]++] = e;
  }
  // elements surrounding each master node (an element once per distinct master)
  std::vector<int32_t> m2e_off(nn + 1, 0);
  std::vector<int32_t> m2e;
  {
    std::vector<std::vector<int32_t>> lists(nn);
    for (int32_t e = 0; e < ne; ++e) {
      const int32_t q[3] = {mnode[3 * e], mnode[3 * e + 1], mnode[3 * e + 2]};
      for (int k = 0; k < 3; ++k) {
        bool dup = false;
        for (int j = 0; j < k; ++j) dup |= (q[j] == q[k]);
        if (!dup) lists[q[k]].push_back(e);
      }
    }
    for (int32_t n = 0; n < nn; ++n) m2e_off[n + 1] = m2e_off[n] + (int32_t)lists[n].size();
    m2e.reserve(m2e_off[nn]);
    for (int32_t n = 0; n < nn; ++n) m2e.insert(m2e.end(), lists[n].begin(), lists[n].end());
  }
  // length scale of eq:CFL per master node: sqrt of the mean area of the
  // elements around it (ascending element order), -1 where none
  std::vector<double> cfl_len(nn, -1.0);
  for (int32_t n = 0; n < nn; ++n) {
    if (master[n] != n || m2e_off[n + 1] <= m2e_off[n]) continue;
    double a = 0.0;
    for (int32_t i = m2e_off[n]; i < m2e_off[n + 1]; ++i) a += area[m2e[i]];
    cfl_len[n] = std::sqrt(a / (double)(m2e_off[n + 1] - m2e_off[n]));
  }
  // element -> no-slip wall edges sharing a node with the element (ascending)
  std::vector<int32_t> w_off(ne + 1, 0), w_list;
  {
    std::vector<std::vector<int32_t>> nw(nn);
    for (int32_t b = 0; b < nb; ++b) {
      if (mesh->bedge_type[b] != PDF_BC_NOSLIP) continue;
      const int32_t e = mesh->bedge_elem[b], k = mesh->bedge_local[b];
      nw[en[3 * e + (k + 1) % 3]].push_back(b);
      nw[en[3 * e + (k + 2) % 3]].push_back(b);
    }
    for (int32_t e = 0; e < ne; ++e) {
      std::vector<int32_t> l;
      for (int k = 0; k < 3; ++k)
        for (int32_t b : nw[en[3 * e + k]])
          if (std::find(l.begin(), l.end(), b) == l.end()) l.push_back(b);
      std::sort(l.begin(), l.end());
      w_list.insert(w_list.end(), l.begin(), l.end());
      w_off[e + 1] = (int32_t)w_list.size();
      geo[e].wb = w_off[e];
      geo[e].wn = w_off[e + 1] - w_off[e];
    }
  }
  // the element test's form of the geometry (the canonical edge directions)
  std::vector<WalkGeo> wgeo(ne);
  for (int32_t e = 0; e < ne; ++e) {
    const ElemGeo &g = geo[e];
    WalkGeo &w = wgeo[e];
    std::memset(&w, 0, sizeof(w));
    for (int k = 0; k < 3; ++k) {
      const int a = (k + 1) % 3, b = (k + 2) % 3;
      const bool fwd = g.n[a] < g.n[b];
      const int p = fwd ? a : b, q = fwd ? b : a;
      const double dx = g.x[q] - g.x[p], dy = g.y[q] - g.y[p];
      w.a[k][0] = g.x[p];
      w.a[k][1] = g.y[p];
      w.a[k][2] = fwd ? dx : -dx;
      w.a[k][3] = fwd ? dy : -dy;
      w.nb[k] = g.nb[k];
    }
    w.wb = g.wb;
    w.wn = g.wn;
  }
  std::vector<WallSeg> wseg(w_list.size());
  for (size_t j = 0; j < w_list.size(); ++j) {
    const int32_t b = w_list[j], e = mesh->bedge_elem[b], k = mesh->bedge_local[b];
    const int32_t a = en[3 * e + (k + 1) % 3], c = en[3 * e + (k + 2) % 3];
    wseg[j] = {xy[2 * a], xy[2 * a + 1], xy[2 * c], xy[2 * c + 1]};
  }
  // node -> wall edges (slip and no-slip) ending at the node (ascending)
  std::vector<int32_t> nwall_off(nn + 1, 0), nwall;
  {
    std::vector<std::vector<int32_t>> l(nn);
    for (int32_t b = 0; b < nb; ++b) {
      if (mesh->bedge_type[b] == PDF_BC_PERIODIC || mesh->bedge_type[b] == PDF_BC_OUTFLOW) continue;
      const int32_t e = mesh->bedge_elem[b], k = mesh->bedge_local[b];
      l[en[3 * e + (k + 1) % 3]].push_back(b);
      l[en[3 * e + (k + 2) % 3]].push_back(b);
    }
    for (int32_t n = 0; n < nn; ++n) {
      nwall.insert(nwall.end(), l[n].begin(), l[n].end());
      nwall_off[n + 1] = (int32_t)nwall.size();
    }
  }
  std::vector<int32_t> masters, slaves, slave_master;
  for (int32_t n = 0; n < nn; ++n) {
    if (master[n] == n)
      masters.push_back(n);
    else {
      slaves.push_back(n);
      slave_master.push_back(master[n]);
    }
  }
  std::vector<int32_t> btype(mesh->bedge_type, mesh->bedge_type + nb);
  std::vector<int32_t> bpart(mesh->bedge_partner, mesh->bedge_partner + nb);
  std::vector<int32_t> belem(mesh->bedge_elem, mesh->bedge_elem + nb);
  std::vector<int32_t> blocal(mesh->bedge_local, mesh->bedge_local + nb);
  std::vector<double> bshift(mesh->bedge_shift, mesh->bedge_shift + 2 * (size_t)nb);
  std::vector<int32_t> vmaster(master, master + nn);
  // ---- bucket grid for the last-resort point location ----
  double bx0 = xy[0], bx1 = xy[0], by0 = xy[1], by1 = xy[1];
  for (int32_t n = 0; n < nn; ++n) {
    bx0 = std::min(bx0, xy[2 * n]);
    bx1 = std::max(bx1, xy[2 * n]);
    by0 = std::min(by0, xy[2 * n + 1]);
    by1 = std::max(by1, xy[2 * n + 1]);
  }
  const double wx = std::max(bx1 - bx0, 1e-300), wy = std::max(by1 - by0, 1e-300);
  // about two elements per cell, cells roughly square
  const double cells = std::max(1.0, 0.5 * ne);
  int32_t gnx = (int32_t)std::max(1.0, std::floor(std::sqrt(cells * wx / wy)));
  int32_t gny = (int32_t)std::max(1.0, std::floor(cells / gnx));
  gnx = std::min(gnx, 1 << 14);
  gny = std::min(gny, 1 << 14);
  const double gsx = gnx / wx, gsy = gny / wy;
  std::vector<int32_t> cell_off((size_t)gnx * gny + 1, 0), cell_list;
  {
    auto crange = [](double lo, double hi, double o, double sc, int32_t nmax, int32_t &a, int32_t &b) {
      a = (int32_t)std::floor((lo - o) * sc - 1e-6);
      b = (int32_t)std::floor((hi - o) * sc + 1e-6);
      a = std::max(a, 0);
      b = std::min(b, nmax - 1);
    };
    std::vector<int32_t> ia(ne), ib(ne), ja(ne), jb(ne);
    for (int32_t e = 0; e < ne; ++e) {
      const ElemGeo &g = geo[e];
      crange(std::min({g.x[0], g.x[1], g.x[2]}), std::max({g.x[0], g.x[1], g.x[2]}), bx0, gsx, gnx, ia[e], ib[e]);
      crange(std::min({g.y[0], g.y[1], g.y[2]}), std::max({g.y[0], g.y[1], g.y[2]}), by0, gsy, gny, ja[e], jb[e]);
      for (int32_t j = ja[e]; j <= jb[e]; ++j)
        for (int32_t i = ia[e]; i <= ib[e]; ++i) cell_off[(size_t)j * gnx + i + 1]++;
    }
    for (size_t k = 0; k < (size_t)gnx * gny; ++k) cell_off[k + 1] += cell_off[k];
    cell_list.resize(cell_off.back());
    std::vector<int32_t> fill(cell_off.begin(), cell_off.end() - 1);
    for (int32_t e = 0; e < ne; ++e)  // ascending element order within every cell
      for (int32_t j = ja[e]; j <= jb[e]; ++j)
        for (int32_t i = ia[e]; i <= ib[e]; ++i) cell_list[fill[(size_t)j * gnx + i]++] = e;
  }
  // rings of the masters: the masters of the nodes of the elements around each
  std::vector<int32_t> ring_off(nn + 1, 0), ring;
  for (int32_t n = 0; n < nn; ++n) {
    std::vector<int32_t> l;
    if (vmaster[n] == n)
      for (int32_t i = m2e_off[n]; i < m2e_off[n + 1]; ++i)
        for (int k = 0; k < 3; ++k) {
          const int32_t q = mnode[3 * (size_t)m2e[i] + k];
          if (q != n && std::find(l.begin(), l.end(), q) == l.end()) l.push_back(q);
        }
    std::sort(l.begin(), l.end());
    ring.insert(ring.end(), l.begin(), l.end());
    ring_off[n + 1] = (int32_t)ring.size();
  }
  const size_t n_gw = (size_t)nn + ring.size();
  if (ring.empty()) ring.push_back(0);  // never read: every ring is empty
  // ---- upload ----
  MeshDev &m = c->md;
  m.gnx = gnx;
  m.gny = gny;
  m.gx0 = bx0;
  m.gy0 = by0;
  m.gsx = gsx;
  m.gsy = gsy;
  m.ne = ne;
  m.nn = nn;
  m.nb = nb;
  m.n_masters = (int32_t)masters.size();
  m.n_slaves = (int32_t)slaves.size();
  bool ok = upload(c, geo, &m.geo) && upload(c, wgeo, &m.wgeo) && upload(c, mnode, &m.mnode) && upload(c, dN, &m.dN) &&
            upload(c, btype, &m.btype) && upload(c, bpart, &m.bpart) && upload(c, belem, &m.belem) &&
            upload(c, blocal, &m.blocal) && upload(c, bshift, &m.bshift) &&
            upload(c, n2e_off, &m.n2e_off) && upload(c, n2e, &m.n2e) &&
            upload(c, m2e_off, &m.m2e_off) && upload(c, m2e, &m.m2e) && upload(c, w_off, &m.w_off) && upload(c, wseg, &m.wseg) &&
            upload(c, w_list, &m.w_list) && upload(c, vmaster, &m.master) &&
            upload(c, nwall_off, &m.nwall_off) && upload(c, nwall, &m.nwall) &&
            upload(c, masters, &m.masters) && upload(c, slaves, &m.slaves) &&
            upload(c, slave_master, &m.slave_master) && upload(c, cell_off, &m.cell_off) &&
            upload(c, cell_list, &m.cell_list) && upload(c, cfl_len, &m.cfl_len) &&
            upload(c, ring_off, &m.ring_off) && upload(c, ring, &m.ring);
  double2 *gw = (double2 *)dalloc(c, n_gw * sizeof(double2));
  unsigned long long *gw_bad = (unsigned long long *)dalloc(c, sizeof(unsigned long long));
  m.gw = gw;
  ok = ok && gw && gw_bad;
  const size_t ts = tsize(c);
  c->stats_a = (double *)dalloc(c, (size_t)PDF_NSTAT * nn * sizeof(double));
  c->stats_b = (double *)dalloc(c, (size_t)PDF_NSTAT * nn * sizeof(double));
  c->wp = (double *)dalloc(c, 9 * (size_t)nn * sizeof(double));
  c->gradp = (double *)dalloc(c, 2 * (size_t)nn * sizeof(double));
  const int nrec = params->stats_mode == PDF_STATS_SHAPE ? NRECS : NREC;
  c->rec = dalloc(c, (size_t)ne * nrec * ts);
  if (params->stats_mode == PDF_STATS_SHAPE) {
    c->nsums = (double *)dalloc(c, (size_t)nn * NSUM * sizeof(double));
    ok = ok && c->nsums;
  }
  c->sums = (double *)dalloc(c, (size_t)ne * NSUM * sizeof(double));
  c->emom = (double *)dalloc(c, (size_t)ne * 16 * sizeof(double));
  c->offs = (int32_t *)dalloc(c, ((size_t)ne + 1) * sizeof(int32_t));
  c->cursor = (int32_t *)dalloc(c, ((size_t)ne + 1) * sizeof(int32_t));
  c->blocksums = (int32_t *)dalloc(c, ((size_t)ne / 1024 + 2) * sizeof(int32_t));
  c->cnt = (unsigned long long *)dalloc(c, PDF_NCOUNTERS * sizeof(unsigned long long));
  c->cfl = (double *)dalloc(c, 4 * sizeof(double));
  if (!ok || !c->stats_a || !c->stats_b || !c->wp || !c->gradp || !c->rec || !c->sums || !c->emom ||
      !c->offs || !c->cursor || !c->blocksums || !c->cnt || !c->cfl) {
    c->err = "device allocation or upload failed";
    *out = c;  // the caller reads the message, then destroys
    return PDF_E_OOM;
  }
  c->stats_cur = c->stats_a;
  c->stats_est = c->stats_b;
  c->latest = c->stats_cur;
  hipStream_t s = c->stream;
  if (hipMemsetAsync(c->stats_a, 0, (size_t)PDF_NSTAT * nn * sizeof(double), s) != hipSuccess ||
      hipMemsetAsync(c->stats_b, 0, (size_t)PDF_NSTAT * nn * sizeof(double), s) != hipSuccess ||
      hipMemsetAsync(c->wp, 0, 9 * (size_t)nn * sizeof(double), s) != hipSuccess ||
      hipMemsetAsync(c->gradp, 0, 2 * (size_t)nn * sizeof(double), s) != hipSuccess ||
      hipMemsetAsync(c->rec, 0, (size_t)ne * nrec * ts, s) != hipSuccess ||
      hipMemsetAsync(c->emom, 0, (size_t)ne * 16 * sizeof(double), s) != hipSuccess ||
      hipMemsetAsync(c->cnt, 0, PDF_NCOUNTERS * sizeof(unsigned long long), s) != hipSuccess ||
      hipMemsetAsync(gw_bad, 0, sizeof(unsigned long long), s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    c->err = "device initialisation failed";
    *out = c;  // the caller reads the message, then destroys
    return PDF_E_DEVICE;
  }
  {  // the gradient weights over the rings
    unsigned long long bad = 0;
    launch_grad_weights(s, m, m.ring_off, m.ring, gw, gw_bad);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&bad, gw_bad, sizeof(bad), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess || bad) {
      c->err = bad ? "mesh set-up: an element node outside its master's ring" : "mesh set-up: gradient weights failed";
      *out = c;  // the caller reads the message, then destroys
      return PDF_E_DEVICE;
    }
  }
  ModelDev &md = c->model;
  md.model = params->model;
  md.wp_source = params->wp_source;
  md.omega_source = params->omega_source;
  md.tm_mode = params->tm_mode;
  md.wall_b = params->wall_b;
  md.stats_mode = params->stats_mode;
  md.C0 = params->C0;
  md.C1 = params->C1;
  md.C2 = params->C2;
  md.C3 = params->C3;
  md.C4 = params->C4;
  md.CT = params->CT;
  md.Cv = params->Cv;
  md.gamma5 = params->gamma5;
  md.Cw1 = params->Cw1;
  md.Cw2 = params->Cw2;
  md.Cphi = params->Cphi;
  md.nu = params->nu;
  md.k_floor = params->k_floor;
  md.src_x = params->src_x;
  md.src_y = params->src_y;
  md.src_r = params->src_r;
  md.Cs = params->Cs;
  md.Ct = params->Ct;
  md.mix_model = params->mix_model;
  md.cond_nu = params->cond_nu;
  md.cond_nv = params->cond_nv;
  md.cond_nw = params->cond_nw;
  md.cond_min = params->cond_min;
  md.outflow = 0;
  for (int32_t b = 0; b < nb; ++b) md.outflow |= mesh->bedge_type[b] == PDF_BC_OUTFLOW ? 1 : 0;
  md.nu_wall = params->nu_wall;
  md.inflow_u = params->inflow_u;
  md.CL = params->CL;
  md.Ceta = params->Ceta;
  if (params->model == PDF_MODEL_GLM && params->wp_source == PDF_WP_ELLIPTIC) {
    const pdf_status es = ell_setup(c, mesh);
    if (es != PDF_OK) {
      *out = c;  // the caller reads the message, then destroys
      return es;
    }
  }
  if (params->proj) {
    const pdf_status ps = proj_setup(c, mesh);
    if (ps != PDF_OK) {
      *out = c;  // the caller reads the message, then destroys
      return ps;
    }
  }
  KArgs hka;
  hka.m = c->md;
  hka.md = c->model;
  c->dka = (KArgs *)dalloc(c, sizeof(KArgs));
  if (!c->dka || hipMemcpyAsync(c->dka, &hka, sizeof(KArgs), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    c->err = "device allocation or upload failed";
    *out = c;  // the caller reads the message, then destroys
    return PDF_E_OOM;
  }
  *out = c;
  return PDF_OK;
}

pdf_status pdf_set_nodal_field(pdf_ctx *c, int32_t field, const double *data, int32_t on_device) {
  if (!c || !data) return PDF_E_INVALID_ARG;
  const size_t nn = (size_t)c->md.nn;
  double *dst;
  size_t nf;
  if (field == PDF_FIELD_STATS) {
    dst = c->stats_cur;
    nf = PDF_NSTAT;
  } else if (field == PDF_FIELD_WP) {
    dst = c->wp;
    nf = 9;
    c->wp_set = true;
  } else if (field == PDF_FIELD_GRADP) {
    dst = c->gradp;
    nf = 2;
    c->gradp_set = true;
  } else {
    return fail(c, PDF_E_INVALID_ARG, "unknown field id");
  }
  HIPCHK(c, hipMemcpyAsync(dst, data, nf * nn * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
  if (field == PDF_FIELD_STATS) c->latest = c->stats_cur;
  return PDF_OK;
}

pdf_status pdf_seed_particles(pdf_ctx *c, const pdf_seed_desc *sd) {
  if (!c || !sd || sd->ppe <= 0 || !sd->U0 || !sd->R0 || !sd->Om0) return PDF_E_INVALID_ARG;
  if (sd->psi_mode < PDF_PSI_ZERO || sd->psi_mode > PDF_PSI_DISC) return PDF_E_INVALID_ARG;
  const int64_t np = (int64_t)c->md.ne * sd->ppe;
  if (np > (int64_t)0x7FFFFFFF) return fail(c, PDF_E_INVALID_ARG, "too many particles for 32-bit ids");
  const size_t nn = (size_t)c->md.nn;
  for (int i = 0; i < 2; ++i) {
    dfree(c, c->pbuf[i]);
    c->pbuf[i] = nullptr;
  }
  c->np = np;
  c->ppe = sd->ppe;
  c->seed = sd->seed;
  c->step = 0;
  c->cur = 0;
  const size_t pb = part_bytes(tsize(c), np);
  c->pbuf[0] = dalloc(c, pb);
  if (c->params.reorder_every > 0) c->pbuf[1] = dalloc(c, pb);
  double *tmp = (double *)dalloc(c, 10 * nn * sizeof(double));
  if (!c->pbuf[0] || (c->params.reorder_every > 0 && !c->pbuf[1]) || !tmp)
    return fail(c, PDF_E_OOM, "particle allocation failed");
  HIPCHK(c, hipMemcpyAsync(tmp, sd->U0, 3 * nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(tmp + 3 * nn, sd->R0, 6 * nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(tmp + 9 * nn, sd->Om0, nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync(c->stats_cur, 0, PDF_NSTAT * nn * sizeof(double), c->stream));
  pdf_status st;
  if (c->prec == PDF_FP32) {
    launch_seed<float>(c->stream, c->md, c->model, part_view<float>(c, 0), sd->ppe, sd->seed,
                       sd->psi_mode, sd->a, sd->b, sd->c, tmp, tmp + 3 * nn, tmp + 9 * nn, c->cnt);
    st = estimate_from_scratch<float>(c, c->stats_cur);
  } else {
    launch_seed<double>(c->stream, c->md, c->model, part_view<double>(c, 0), sd->ppe, sd->seed,
                        sd->psi_mode, sd->a, sd->b, sd->c, tmp, tmp + 3 * nn, tmp + 9 * nn, c->cnt);
    st = estimate_from_scratch<double>(c, c->stats_cur);
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  dfree(c, tmp);
  if (st != PDF_OK) return st;
  c->seeded = true;
  return PDF_OK;
}

namespace {
pdf_status advance_checks(pdf_ctx *c) {
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_advance before pdf_seed_particles");
  if (c->params.model == PDF_MODEL_GLM && c->params.wp_source == PDF_WP_INPUT && !c->wp_set)
    return fail(c, PDF_E_STATE, "GLM with PDF_WP_INPUT needs the PDF_FIELD_WP field");
  if (c->timing) {
    for (auto e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    c->ev_phase.clear();
  }
  return PDF_OK;
}
}  // namespace

pdf_status pdf_advance(pdf_ctx *c, int32_t nsteps, double dt) {
  if (!c || nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return PDF_E_INVALID_ARG;
  const pdf_status st = advance_checks(c);
  if (st != PDF_OK) return st;
  return c->prec == PDF_FP32 ? advance_impl<float>(c, nsteps, dt, nullptr)
                             : advance_impl<double>(c, nsteps, dt, nullptr);
}

pdf_status pdf_advance_cfl(pdf_ctx *c, int32_t nsteps, double c_cfl, double dt_max, double *t_advanced) {
  if (!c || nsteps < 0 || !(c_cfl > 0.0) || !std::isfinite(c_cfl) || !(dt_max > 0.0) || !std::isfinite(dt_max))
    return PDF_E_INVALID_ARG;
  pdf_status st = advance_checks(c);
  if (st != PDF_OK) return st;
  const double cfl[2] = {c_cfl, dt_max};
  st = c->prec == PDF_FP32 ? advance_impl<float>(c, nsteps, dt_max, cfl)
                           : advance_impl<double>(c, nsteps, dt_max, cfl);
  if (st != PDF_OK || !t_advanced) return st;
  if (nsteps == 0) {
    *t_advanced = 0.0;
    return PDF_OK;
  }
  HIPCHK(c, hipMemcpyAsync(t_advanced, c->cfl + 1, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PDF_OK;
}

pdf_status pdf_get_nodal_field(pdf_ctx *c, int32_t field, double *data, int32_t on_device) {
  if (!c || !data) return PDF_E_INVALID_ARG;
  const size_t nn = (size_t)c->md.nn;
  const double *src;
  size_t nf;
  if (field == PDF_FIELD_STATS) {
    src = c->latest;
    nf = PDF_NSTAT;
  } else if (field == PDF_FIELD_WP) {
    src = c->wp;
    nf = 9;
  } else if (field == PDF_FIELD_GRADP) {
    if (c->params.proj) launch_proj_gradp(c->stream, c->md, c->pb, c->gradp_set ? c->gradp : nullptr);
    src = c->params.proj ? c->pb.gtot : c->gradp;
    nf = 2;
  } else if (field == PDF_FIELD_PRESSURE && c->params.proj) {
    src = c->pb.P;
    nf = 1;
  } else {
    return fail(c, PDF_E_INVALID_ARG, "unknown field id");
  }
  HIPCHK(c, hipMemcpyAsync(data, src, nf * nn * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
  return PDF_OK;
}

pdf_status pdf_estimate_stats(pdf_ctx *c, double *nodal, double *elem, int32_t on_device) {
  if (!c || (!nodal && !elem)) return PDF_E_INVALID_ARG;
  if (!c->seeded) return fail(c, PDF_E_STATE, "no particles");
  if (elem && c->model.stats_mode == PDF_STATS_SHAPE)
    return fail(c, PDF_E_STATE, "the SHAPE statistics mode forms no element statistics");
  const size_t nn = (size_t)c->md.nn, ne = (size_t)c->md.ne;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (nodal) HIPCHK(c, hipMemcpyAsync(nodal, c->latest, PDF_NSTAT * nn * sizeof(double), kind, c->stream));
  if (elem) {
    double *tmp = on_device ? elem : (double *)dalloc(c, 16 * ne * sizeof(double));
    if (!tmp) return fail(c, PDF_E_OOM, "temporary allocation failed");
    launch_export_elem(c->stream, (int32_t)ne, c->emom, tmp);
    HIPCHK(c, hipGetLastError());
    if (!on_device) {
      HIPCHK(c, hipMemcpyAsync(elem, tmp, 16 * ne * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      dfree(c, tmp);
    }
  }
  if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
  return PDF_OK;
}

pdf_status pdf_num_particles(pdf_ctx *c, int64_t *n) {
  if (!c || !n) return PDF_E_INVALID_ARG;
  *n = c->np;
  return PDF_OK;
}

pdf_status pdf_get_particles(pdf_ctx *c, double *state, int32_t *elem, uint32_t *id) {
  if (!c) return PDF_E_INVALID_ARG;
  if (!c->seeded) return fail(c, PDF_E_STATE, "no particles");
  const int64_t np = c->np;
  if (state) {
    double *tmp = (double *)dalloc(c, 7 * (size_t)np * sizeof(double));
    if (!tmp) return fail(c, PDF_E_OOM, "temporary allocation failed");
    if (c->prec == PDF_FP32)
      launch_pack_state<float>(c->stream, part_view<float>(c, c->cur), np, tmp);
    else
      launch_pack_state<double>(c->stream, part_view<double>(c, c->cur), np, tmp);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(state, tmp, 7 * (size_t)np * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, tmp);
  }
  if (elem) {
    int32_t *e = c->prec == PDF_FP32 ? part_view<float>(c, c->cur).e : part_view<double>(c, c->cur).e;
    HIPCHK(c, hipMemcpyAsync(elem, e, (size_t)np * 4, hipMemcpyDeviceToHost, c->stream));
  }
  if (id) {
    uint32_t *d = c->prec == PDF_FP32 ? part_view<float>(c, c->cur).id : part_view<double>(c, c->cur).id;
    HIPCHK(c, hipMemcpyAsync(id, d, (size_t)np * 4, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PDF_OK;
}

pdf_status pdf_set_particles(pdf_ctx *c, int64_t n, const double *state, const int32_t *elem,
                             const uint32_t *id) {
  if (!c || n <= 0 || !state || !elem || !id) return PDF_E_INVALID_ARG;
  const int32_t ne = c->md.ne;
  for (int64_t i = 0; i < n; ++i)
    if (elem[i] < 0 || elem[i] >= ne) return fail(c, PDF_E_INVALID_ARG, "element index out of range");
  if (n != c->np || !c->pbuf[0]) {
    for (int i = 0; i < 2; ++i) {
      dfree(c, c->pbuf[i]);
      c->pbuf[i] = nullptr;
    }
    c->np = n;
    c->cur = 0;
    const size_t pb = part_bytes(tsize(c), n);
    c->pbuf[0] = dalloc(c, pb);
    if (c->params.reorder_every > 0) c->pbuf[1] = dalloc(c, pb);
    if (!c->pbuf[0] || (c->params.reorder_every > 0 && !c->pbuf[1]))
      return fail(c, PDF_E_OOM, "particle allocation failed");
  }
  double *tmp = (double *)dalloc(c, 7 * (size_t)n * sizeof(double));
  if (!tmp) return fail(c, PDF_E_OOM, "temporary allocation failed");
  HIPCHK(c, hipMemcpyAsync(tmp, state, 7 * (size_t)n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  pdf_status st;
  if (c->prec == PDF_FP32) {
    PartDev<float> p = part_view<float>(c, c->cur);
    launch_unpack_state<float>(c->stream, p, n, tmp);
    HIPCHK(c, hipMemcpyAsync(p.e, elem, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(p.id, id, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
    st = estimate_from_scratch<float>(c, c->stats_cur);
  } else {
    PartDev<double> p = part_view<double>(c, c->cur);
    launch_unpack_state<double>(c->stream, p, n, tmp);
    HIPCHK(c, hipMemcpyAsync(p.e, elem, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(p.id, id, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
    st = estimate_from_scratch<double>(c, c->stats_cur);
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  dfree(c, tmp);
  if (st != PDF_OK) return st;
  c->seeded = true;
  return PDF_OK;
}

pdf_status pdf_get_counters(pdf_ctx *c, uint64_t *out, int32_t n, int32_t reset) {
  if (!c || !out || n < 0 || n > PDF_NCOUNTERS) return PDF_E_INVALID_ARG;
  unsigned long long h[PDF_NCOUNTERS];
  HIPCHK(c, hipMemcpyAsync(h, c->cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  h[PDF_CNT_STEPS] = c->step;
  h[PDF_CNT_ELL_ITERS] = c->ell_iters;
  h[PDF_CNT_PROJ_ITERS] = c->proj_iters;
  if (reset) c->ell_iters = c->proj_iters = 0;
  for (int i = 0; i < n; ++i) out[i] = h[i];
  if (reset) {
    HIPCHK(c, hipMemsetAsync(c->cnt, 0, sizeof(h), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return PDF_OK;
}

pdf_status pdf_enable_timing(pdf_ctx *c, int32_t on) {
  if (!c) return PDF_E_INVALID_ARG;
  c->timing = on != 0;
  return PDF_OK;
}

pdf_status pdf_get_timing(pdf_ctx *c, double *out_ms, int32_t n) {
  if (!c || !out_ms || n < 0) return PDF_E_INVALID_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double acc[5] = {0, 0, 0, 0, 0};
  for (size_t i = 0; i + 1 < c->ev.size(); ++i) {
    const int ph = c->ev_phase[i];
    if (ph > 4) continue;  // phase 5 marks the end of a step
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
    acc[ph] += ms;
  }
  for (int i = 0; i < n && i < 5; ++i) out_ms[i] = acc[i];
  return PDF_OK;
}

}  // extern "C"

// ===========================================================================
// Learned denoiser (host orchestration of the kernels in k_denoise.hip)
// ===========================================================================
struct pdf_denoiser {
  pdf_ctx *ctx = nullptr;
  int32_t H = 128;
  int64_t np = 0;
  int64_t off[8] = {0};  // W1 b1 W2 b2 W3 b3 W4 b4
  float *P = nullptr, *G = nullptr, *Mom = nullptr, *Vel = nullptr;
  uint16_t *Pb = nullptr;  // bf16 copy of the parameters (weights used by the GEMMs)
  uint16_t *Wt = nullptr;  // transposed, padded bf16 weights of the fused inference
  bool wt_stale = true;    // Wt must be rebuilt from Pb before the next inference
  float *R = nullptr;      // network outputs of pdf_denoise_stats [n_nodes][8]
  double *res = nullptr;   // denoised statistics staging [PDF_NSTAT][n_nodes]
  float *mu = nullptr, *sig = nullptr, *scale = nullptr;
  bool norm_set = false;
  int64_t adam_t = 0;
  // point-surrounding-point lists over master nodes
  const int32_t *p2p_off = nullptr, *p2p = nullptr;  // the mesh's rings (not owned)
  const double2 *gw = nullptr;                       // and gradient weights (not owned)
  // batch buffers
  int32_t cap = 0;
  uint16_t *Xb = nullptr, *H1 = nullptr, *H2 = nullptr, *H3 = nullptr, *dYb = nullptr, *dZb = nullptr;
  float *Z1 = nullptr, *Z2 = nullptr, *Z3 = nullptr, *Y = nullptr, *dH = nullptr, *part = nullptr;
  float *feat = nullptr;
  unsigned long long *nfall = nullptr;
};

namespace {

bool dn_reserve(pdf_denoiser *d, int32_t B) {
  if (B <= d->cap) return true;
  pdf_ctx *c = d->ctx;
  void *old[12] = {d->Xb, d->H1, d->H2, d->H3, d->dYb, d->dZb, d->Z1, d->Z2, d->Z3, d->Y, d->dH, d->part};
  for (void *p : old) dfree(c, p);
  const size_t H = (size_t)d->H, b = (size_t)B;
  d->Xb = (uint16_t *)dalloc(c, b * PDF_DN_NIN * 2);
  d->H1 = (uint16_t *)dalloc(c, b * H * 2);
  d->H2 = (uint16_t *)dalloc(c, b * H * 2);
  d->H3 = (uint16_t *)dalloc(c, b * H * 2);
  d->dYb = (uint16_t *)dalloc(c, b * PDF_DN_NOUT * 2);
  d->dZb = (uint16_t *)dalloc(c, b * H * 2);
  d->Z1 = (float *)dalloc(c, b * H * 4);
  d->Z2 = (float *)dalloc(c, b * H * 4);
  d->Z3 = (float *)dalloc(c, b * H * 4);
  d->Y = (float *)dalloc(c, b * PDF_DN_NOUT * 4);
  d->dH = (float *)dalloc(c, b * H * 4);
  d->part = (float *)dalloc(c, (b * PDF_DN_NOUT / 256 + 2) * 4);
  d->cap = B;
  return d->Xb && d->H1 && d->H2 && d->H3 && d->dYb && d->dZb && d->Z1 && d->Z2 && d->Z3 && d->Y &&
         d->dH && d->part;
}

// forward pass of B rows of standardised features (fp32 x), keeping Z and H
pdf_status dn_forward(pdf_denoiser *d, const float *x, int32_t B) {
  pdf_ctx *c = d->ctx;
  hipStream_t s = c->stream;
  const int H = d->H;
  const uint16_t *W1 = d->Pb + d->off[0], *W2 = d->Pb + d->off[2], *W3 = d->Pb + d->off[4],
                 *W4 = d->Pb + d->off[6];
  const float *b1 = d->P + d->off[1], *b2 = d->P + d->off[3], *b3 = d->P + d->off[5],
              *b4 = d->P + d->off[7];
  launch_to_bf16(s, (int64_t)B * PDF_DN_NIN, x, d->Xb);
  launch_gemm_bf16(s, B, H, PDF_DN_NIN, d->Xb, PDF_DN_NIN, 0, W1, H, 0, d->Z1, H, 0.f);
  launch_bias_act(s, B, H, d->Z1, b1, d->H1, 1);
  launch_gemm_bf16(s, B, H, H, d->H1, H, 0, W2, H, 0, d->Z2, H, 0.f);
  launch_bias_act(s, B, H, d->Z2, b2, d->H2, 1);
  launch_gemm_bf16(s, B, H, H, d->H2, H, 0, W3, H, 0, d->Z3, H, 0.f);
  launch_bias_act(s, B, H, d->Z3, b3, d->H3, 1);
  launch_gemm_bf16(s, B, PDF_DN_NOUT, H, d->H3, H, 0, W4, PDF_DN_NOUT, 0, d->Y, PDF_DN_NOUT, 0.f);
  launch_bias_act(s, B, PDF_DN_NOUT, d->Y, b4, nullptr, 0);
  HIPCHK(c, hipGetLastError());
  return PDF_OK;
}

}  // namespace

extern "C" {

pdf_status pdf_denoiser_create(pdf_ctx *c, int32_t hidden, uint64_t seed, pdf_denoiser **out) {
  if (!c || !out || hidden < 16 || hidden > 1024 || hidden % 16) return PDF_E_INVALID_ARG;
  pdf_denoiser *d = new pdf_denoiser();
  d->ctx = c;
  d->H = hidden;
  const int64_t H = hidden;
  const int64_t sizes[8] = {PDF_DN_NIN * H, H, H * H, H, H * H, H, H * PDF_DN_NOUT, PDF_DN_NOUT};
  int64_t o = 0;
  for (int i = 0; i < 8; ++i) {
    d->off[i] = o;
    o += sizes[i];
  }
  d->np = o;
  d->P = (float *)dalloc(c, o * 4);
  d->G = (float *)dalloc(c, o * 4);
  d->Mom = (float *)dalloc(c, o * 4);
  d->Vel = (float *)dalloc(c, o * 4);
  d->Pb = (uint16_t *)dalloc(c, o * 2);
  if (hidden >= 48 && hidden <= 128) d->Wt = (uint16_t *)dalloc(c, mlp_transposed_elems(hidden) * 2);
  d->mu = (float *)dalloc(c, 64 * 4);
  d->sig = (float *)dalloc(c, 64 * 4);
  d->scale = (float *)dalloc(c, 16 * 4);
  d->nfall = (unsigned long long *)dalloc(c, 8);
  const int32_t nn = c->md.nn;
  d->feat = (float *)dalloc(c, (size_t)nn * PDF_DN_NIN * 4);
  // the rings and gradient weights of the mesh
  d->p2p_off = c->md.ring_off;
  d->p2p = c->md.ring;
  d->gw = c->md.gw;
  const bool ok = d->P && d->G && d->Mom && d->Vel && d->Pb && d->mu && d->sig && d->scale && d->nfall && d->feat;
  if (!ok) {
    pdf_denoiser_destroy(d);
    return fail(c, PDF_E_OOM, "denoiser allocation failed");
  }
  // initial parameters: uniform in +-1/sqrt(fan_in) (splitmix64 stream), zero biases
  std::vector<float> h(o, 0.f);
  uint64_t st = seed ^ 0x9E3779B97F4A7C15ull;
  auto next = [&]() {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  const int64_t fan[4] = {PDF_DN_NIN, H, H, H};
  for (int l = 0; l < 4; ++l) {
    const double a = 1.0 / std::sqrt((double)fan[l]);
    for (int64_t i = 0; i < sizes[2 * l]; ++i) h[d->off[2 * l] + i] = (float)((2.0 * next() - 1.0) * a);
  }
  std::vector<float> one(64, 1.f), zero(64, 0.f);
  if (pdf_denoiser_params(d, h.data(), o, 1) != PDF_OK ||
      hipMemcpy(d->mu, zero.data(), 64 * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d->sig, one.data(), 64 * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d->scale, one.data(), 16 * 4, hipMemcpyHostToDevice) != hipSuccess) {
    pdf_denoiser_destroy(d);
    return fail(c, PDF_E_DEVICE, "denoiser initialisation failed");
  }
  *out = d;
  return PDF_OK;
}

void pdf_denoiser_destroy(pdf_denoiser *d) {
  if (!d) return;
  pdf_ctx *c = d->ctx;
  (void)hipStreamSynchronize(c->stream);
  void *ps[] = {d->P, d->G, d->Mom, d->Vel, d->Pb, d->mu, d->sig, d->scale, d->Xb,
                d->H1, d->H2, d->H3, d->dYb, d->dZb, d->Z1, d->Z2, d->Z3, d->Y, d->dH, d->part, d->feat,
                d->nfall, d->Wt, d->R, d->res};
  for (void *p : ps) dfree(c, p);
  delete d;
}

pdf_status pdf_denoiser_params(pdf_denoiser *d, float *host, int64_t n, int32_t set) {
  if (!d || !host || n != d->np) return PDF_E_INVALID_ARG;
  pdf_ctx *c = d->ctx;
  if (set) {
    HIPCHK(c, hipMemcpyAsync(d->P, host, n * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(d->Mom, 0, n * 4, c->stream));
    HIPCHK(c, hipMemsetAsync(d->Vel, 0, n * 4, c->stream));
    launch_to_bf16(c->stream, n, d->P, d->Pb);
    d->wt_stale = true;
    d->adam_t = 0;
  } else {
    HIPCHK(c, hipMemcpyAsync(host, d->P, n * 4, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PDF_OK;
}

pdf_status pdf_denoiser_set_norm(pdf_denoiser *d, const float *mu48, const float *sig48, const float *scale8) {
  if (!d || !mu48 || !sig48 || !scale8) return PDF_E_INVALID_ARG;
  for (int i = 0; i < PDF_DN_NIN; ++i)
    if (!(sig48[i] > 0.f)) return fail(d->ctx, PDF_E_INVALID_ARG, "feature scale must be positive");
  pdf_ctx *c = d->ctx;
  HIPCHK(c, hipMemcpyAsync(d->mu, mu48, PDF_DN_NIN * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d->sig, sig48, PDF_DN_NIN * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d->scale, scale8, PDF_DN_NOUT * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  d->norm_set = true;
  return PDF_OK;
}

pdf_status pdf_denoiser_set_fallback(pdf_denoiser *d, const float *kappa8) {
  if (!d || !kappa8) return PDF_E_INVALID_ARG;
  for (int i = 0; i < PDF_DN_NOUT; ++i)
    if (!(kappa8[i] > 0.f) || !std::isfinite(kappa8[i]))
      return fail(d->ctx, PDF_E_INVALID_ARG, "fallback factors must be positive and finite");
  pdf_ctx *c = d->ctx;
  HIPCHK(c, hipMemcpyAsync(d->scale + PDF_DN_NOUT, kappa8, PDF_DN_NOUT * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PDF_OK;
}

pdf_status pdf_denoiser_io(pdf_denoiser *d, int32_t save, const char *path) {
  if (!d || !path) return PDF_E_INVALID_ARG;
  pdf_ctx *c = d->ctx;
  static const char TAG[8] = {'p', 'd', 'f', 'd', 'n', '0', '0', '1'};
  const size_t np = (size_t)d->np;
  std::vector<float> P(np), norm(2 * PDF_DN_NIN + 2 * PDF_DN_NOUT);  // mu, sig, scales, fallback factors
  if (save) {
    HIPCHK(c, hipMemcpyAsync(P.data(), d->P, np * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(norm.data(), d->mu, PDF_DN_NIN * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(norm.data() + PDF_DN_NIN, d->sig, PDF_DN_NIN * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(norm.data() + 2 * PDF_DN_NIN, d->scale, 2 * PDF_DN_NOUT * 4, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    FILE *f = fopen(path, "wb");
    if (!f) return fail(c, PDF_E_INVALID_ARG, std::string("cannot open for writing: ") + path);
    const int32_t hdr[2] = {d->H, d->norm_set ? 1 : 0};
    const int64_t n64 = d->np;
    bool ok = fwrite(TAG, 1, 8, f) == 8 && fwrite(hdr, 4, 2, f) == 2 && fwrite(&n64, 8, 1, f) == 1 &&
              fwrite(P.data(), 4, np, f) == np && fwrite(norm.data(), 4, norm.size(), f) == norm.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) return fail(c, PDF_E_INVALID_ARG, std::string("write failed: ") + path);
    return PDF_OK;
  }
  FILE *f = fopen(path, "rb");
  if (!f) return fail(c, PDF_E_INVALID_ARG, std::string("cannot open for reading: ") + path);
  char tag[8];
  int32_t hdr[2];
  int64_t n64 = -1;
  bool ok = fread(tag, 1, 8, f) == 8 && memcmp(tag, TAG, 8) == 0;
  if (!ok) {
    fclose(f);
    return fail(c, PDF_E_INVALID_ARG, std::string("not a denoiser file: ") + path);
  }
  ok = fread(hdr, 4, 2, f) == 2 && fread(&n64, 8, 1, f) == 1;
  if (!ok || hdr[0] != d->H || n64 != d->np) {
    fclose(f);
    return fail(c, PDF_E_INVALID_ARG, "the file's hidden width or parameter count differs from this denoiser's");
  }
  ok = fread(P.data(), 4, np, f) == np && fread(norm.data(), 4, norm.size(), f) == norm.size();
  char extra;
  ok = ok && fread(&extra, 1, 1, f) == 0;  // nothing after the last field
  fclose(f);
  if (!ok) return fail(c, PDF_E_INVALID_ARG, std::string("truncated or oversized denoiser file: ") + path);
  for (int i = 0; i < PDF_DN_NIN; ++i)
    if (!(norm[PDF_DN_NIN + i] > 0.f)) return fail(c, PDF_E_INVALID_ARG, "feature scale must be positive");
  for (int i = 0; i < PDF_DN_NOUT; ++i) {
    const float k = norm[2 * PDF_DN_NIN + PDF_DN_NOUT + i];
    if (!(k > 0.f) || !std::isfinite(k)) return fail(c, PDF_E_INVALID_ARG, "fallback factors must be positive and finite");
  }
  const pdf_status st = pdf_denoiser_params(d, P.data(), d->np, 1);
  if (st != PDF_OK) return st;
  HIPCHK(c, hipMemcpyAsync(d->mu, norm.data(), PDF_DN_NIN * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d->sig, norm.data() + PDF_DN_NIN, PDF_DN_NIN * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d->scale, norm.data() + 2 * PDF_DN_NIN, 2 * PDF_DN_NOUT * 4, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  d->norm_set = hdr[1] != 0;
  return PDF_OK;
}

pdf_status pdf_denoiser_features(pdf_denoiser *d, const double *nodal, float *feat, int32_t standardized) {
  if (!d || !feat) return PDF_E_INVALID_ARG;
  pdf_ctx *c = d->ctx;
  if (!nodal && !c->seeded) return fail(c, PDF_E_STATE, "no statistics");
  launch_features(c->stream, c->md, d->p2p_off, d->p2p, d->gw, nodal ? nodal : c->latest,
                  standardized ? d->mu : nullptr, d->sig, feat, nullptr);
  HIPCHK(c, hipGetLastError());
  return PDF_OK;
}

pdf_status pdf_denoiser_forward(pdf_denoiser *d, const float *x, int32_t n, float *y) {
  if (!d || !x || !y || n < 0) return PDF_E_INVALID_ARG;
  pdf_ctx *c = d->ctx;
  if (n == 0) return PDF_OK;
  // the fused kernel keeps every activation in LDS (hidden widths up to 128)
  if (d->Wt) {
    if (d->wt_stale) {
      launch_transpose_weights(c->stream, d->H, d->Pb + d->off[0], d->Pb + d->off[2], d->Pb + d->off[4],
                               d->Pb + d->off[6], d->Wt);
      d->wt_stale = false;
    }
    if (launch_mlp_forward(c->stream, n, d->H, x, d->Wt, d->P + d->off[1], d->P + d->off[3], d->P + d->off[5],
                           d->P + d->off[7], y)) {
      HIPCHK(c, hipGetLastError());
      return PDF_OK;
    }
  }
  const int32_t chunk = 65536;
  if (!dn_reserve(d, n < chunk ? n : chunk)) return fail(c, PDF_E_OOM, "denoiser buffers");
  for (int32_t r0 = 0; r0 < n; r0 += chunk) {
    const int32_t b = (n - r0) < chunk ? (n - r0) : chunk;
    pdf_status st = dn_forward(d, x + (size_t)r0 * PDF_DN_NIN, b);
    if (st != PDF_OK) return st;
    HIPCHK(c, hipMemcpyAsync(y + (size_t)r0 * PDF_DN_NOUT, d->Y, (size_t)b * PDF_DN_NOUT * 4,
                             hipMemcpyDeviceToDevice, c->stream));
  }
  return PDF_OK;
}

pdf_status pdf_denoiser_train_step(pdf_denoiser *d, const float *x, const float *target, int32_t B,
                                   float lr, float *loss, float *grad_host) {
  if (!d || !x || !target || B <= 0 || lr < 0.f) return PDF_E_INVALID_ARG;
  pdf_ctx *c = d->ctx;
  hipStream_t s = c->stream;
  if (!dn_reserve(d, B)) return fail(c, PDF_E_OOM, "denoiser buffers");
  pdf_status st = dn_forward(d, x, B);
  if (st != PDF_OK) return st;
  const int H = d->H, O = PDF_DN_NOUT;
  const uint16_t *W2 = d->Pb + d->off[2], *W3 = d->Pb + d->off[4], *W4 = d->Pb + d->off[6];
  float *g = d->G;
  // dL/dY (mean squared error) into Y (fp32) and dYb (bf16)
  const int nb = launch_mse(s, B, O, O, d->Y, target, d->dYb, d->part);
  // layer 4
  launch_gemm_bf16(s, H, O, B, d->H3, H, 1, d->dYb, O, 0, g + d->off[6], O, 0.f);
  launch_colsum(s, B, O, d->Y, g + d->off[7]);
  launch_gemm_bf16(s, B, H, O, d->dYb, O, 0, W4, O, 1, d->dH, H, 0.f);
  launch_dgelu(s, (int64_t)B * H, d->dH, d->Z3, d->dZb);
  // layer 3
  launch_gemm_bf16(s, H, H, B, d->H2, H, 1, d->dZb, H, 0, g + d->off[4], H, 0.f);
  launch_colsum(s, B, H, d->dH, g + d->off[5]);
  launch_gemm_bf16(s, B, H, H, d->dZb, H, 0, W3, H, 1, d->dH, H, 0.f);
  launch_dgelu(s, (int64_t)B * H, d->dH, d->Z2, d->dZb);
  // layer 2
  launch_gemm_bf16(s, H, H, B, d->H1, H, 1, d->dZb, H, 0, g + d->off[2], H, 0.f);
  launch_colsum(s, B, H, d->dH, g + d->off[3]);
  launch_gemm_bf16(s, B, H, H, d->dZb, H, 0, W2, H, 1, d->dH, H, 0.f);
  launch_dgelu(s, (int64_t)B * H, d->dH, d->Z1, d->dZb);
  // layer 1
  launch_gemm_bf16(s, PDF_DN_NIN, H, B, d->Xb, PDF_DN_NIN, 1, d->dZb, H, 0, g + d->off[0], H, 0.f);
  launch_colsum(s, B, H, d->dH, g + d->off[1]);
  HIPCHK(c, hipGetLastError());
  if (lr > 0.f) {
    d->adam_t++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - (float)std::pow((double)b1, (double)d->adam_t);
    const float c2 = 1.f - (float)std::pow((double)b2, (double)d->adam_t);
    launch_adam(s, d->np, d->P, g, d->Mom, d->Vel, d->Pb, lr, b1, b2, 1e-8f, c1, c2);
    d->wt_stale = true;
    HIPCHK(c, hipGetLastError());
  }
  if (loss) {
    std::vector<float> hp(nb);
    HIPCHK(c, hipMemcpyAsync(hp.data(), d->part, nb * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    double acc = 0.0;
    for (float v : hp) acc += v;
    *loss = (float)(acc / ((double)B * O));
  }
  if (grad_host) {
    HIPCHK(c, hipMemcpyAsync(grad_host, g, d->np * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  return PDF_OK;
}

pdf_status pdf_denoise_stats(pdf_denoiser *d, double tau, double *out, int32_t on_device,
                             uint64_t *n_fallback) {
  if (!d || !out || !(tau >= 0.0)) return PDF_E_INVALID_ARG;
  pdf_ctx *c = d->ctx;
  if (!c->seeded) return fail(c, PDF_E_STATE, "no statistics");
  hipStream_t s = c->stream;
  const int32_t nn = c->md.nn;
  launch_features(s, c->md, d->p2p_off, d->p2p, d->gw, c->latest, d->mu, d->sig, d->feat, nullptr);
  if (!d->R) d->R = (float *)dalloc(c, (size_t)nn * PDF_DN_NOUT * 4);
  if (!on_device && !d->res) d->res = (double *)dalloc(c, (size_t)PDF_NSTAT * nn * 8);
  float *R = d->R;
  double *res = on_device ? out : d->res;
  if (!R || !res) return fail(c, PDF_E_OOM, "denoiser output buffers");
  pdf_status st = pdf_denoiser_forward(d, d->feat, nn, R);
  if (st != PDF_OK) return st;
  HIPCHK(c, hipMemsetAsync(d->nfall, 0, 8, s));
  launch_merge(s, nn, c->md.master, c->latest, R, PDF_DN_NOUT, d->scale, tau, c->params.C4, res, d->nfall);
  HIPCHK(c, hipGetLastError());
  if (on_device && !n_fallback) return PDF_OK;  // nothing for the host to wait for
  unsigned long long nf = 0;
  HIPCHK(c, hipMemcpyAsync(&nf, d->nfall, 8, hipMemcpyDeviceToHost, s));
  if (!on_device)
    HIPCHK(c, hipMemcpyAsync(out, res, (size_t)PDF_NSTAT * nn * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (n_fallback) *n_fallback = nf;
  return PDF_OK;
}

pdf_status pdf_denoise_stats_noalloc(pdf_denoiser *d, double tau, double *out, uint64_t *n_fallback_dev) {
  if (!d || !out || !(tau >= 0.0)) return PDF_E_INVALID_ARG;
  pdf_ctx *c = d->ctx;
  if (!c->seeded) return fail(c, PDF_E_STATE, "no statistics");
  if (!d->Wt)
    return fail(c, PDF_E_INVALID_ARG,
                "pdf_denoise_stats_noalloc needs the fused inference (hidden width 48..128, a multiple of 16)");
  void *base = (c->device >= 0 && c->device < NOALLOC_MAX_DEV) ? scratch_dev[c->device] : nullptr;
  if (!base) return fail(c, PDF_E_STATE, "the allocation-free scratch is not set up on this device");
  hipStream_t s = c->stream;
  float *F = (float *)base;                          // [chunk][48] features
  float *R = F + (size_t)NOALLOC_CHUNK * PDF_DN_NIN;  // [chunk][8] network outputs
  if (d->wt_stale) {
    launch_transpose_weights(s, d->H, d->Pb + d->off[0], d->Pb + d->off[2], d->Pb + d->off[4], d->Pb + d->off[6],
                             d->Wt);
    d->wt_stale = false;
  }
  // the caller's counter is cleared by a kernel, not a memset, so that the
  // call can be captured in a graph
  auto *nfall = reinterpret_cast<unsigned long long *>(n_fallback_dev);
  if (nfall) hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(64), 0, s, nfall);
  const int32_t nn = c->md.nn;
  for (int32_t n0 = 0; n0 < nn; n0 += NOALLOC_CHUNK) {
    const int32_t cnt = (nn - n0) < NOALLOC_CHUNK ? (nn - n0) : NOALLOC_CHUNK;
    launch_features_range(s, c->md, d->p2p_off, d->p2p, d->gw, c->latest, d->mu, d->sig, n0, cnt, F, nullptr);
    if (!launch_mlp_forward(s, cnt, d->H, F, d->Wt, d->P + d->off[1], d->P + d->off[3], d->P + d->off[5],
                            d->P + d->off[7], R))
      return fail(c, PDF_E_DEVICE, "fused inference launch failed");
    launch_merge_range(s, nn, c->md.master, c->latest, n0, cnt, R, PDF_DN_NOUT, d->scale, tau, c->params.C4, out,
                       nfall);
  }
  HIPCHK(c, hipGetLastError());
  return PDF_OK;
}

}  // extern "C"
