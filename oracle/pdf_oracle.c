/*
 * Oracle for the particle hot path (TEST INFRASTRUCTURE ONLY; see pdf_oracle.h).
 *
 * Built with -O2 -ffp-contract=off and no fast-math: every floating-point
 * operation is a plain IEEE binary64 operation in the order written here.
 *
 * Sources (Bakosi, "PDF modeling of turbulent flows on unstructured grids"):
 *   particle SDEs ............ Ch.2: eq:Lagrangian-position-exact, eq:Lagrangian-model,
 *                              eq:GandC, eq:wall-GandC, eq:frequency-model,
 *                              eq:frequency-source, eq:dissipation-from-frequency_wall, eq:IEM
 *   time integration ......... Ch.3, Sec. Timestepping (explicit Euler-Maruyama),
 *                              eq:velocity-prediction (particle part)
 *   statistics ............... Ch.3, Sec. Estimation of Eulerian statistics (two-pass
 *                              element -> node estimator, Fig. mesh-particles)
 *   derivatives .............. Ch.3, Sec. Derivatives: eq:shapefunctions, eq:gradient,
 *                              the two-pass second derivatives
 *   tracking ................. Ch.3, Sec. Particle tracking: eq:element-test, the
 *                              "next best element" rule and the concave-corner fallback
 *   no-slip walls ............ Ch.3, Sec. No-slip wall-boundary conditions: eq:fw,
 *                              eq:exp-wall-condition, eq:frequency-wallstats
 *   initial conditions ....... Ch.3, Sec. Particle-number control (uniform positions per
 *                              element, Gaussian velocities, gamma frequencies)
 *   random numbers ........... Philox4x32-10 of Salmon, Moraes, Dror & Shaw, "Parallel
 *                              random numbers: as easy as 1, 2, 3" (SC'11), replacing the
 *                              per-step random tables of Ch.3, Sec. Parallel random numbers;
 *                              gamma variates by Marsaglia & Tsang (ACM TOMS 26, 2000);
 *                              normals by the Box-Muller transform.
 */
#include "pdf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011): 10 rounds of the 4x32 Philox S-box,  */
/* multipliers 0xD2511F53 / 0xCD9E8D57, key schedule Weyl increments        */
/* 0x9E3779B9 / 0xBB67AE85 applied between rounds.                          */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

static void draw(uint64_t seed, uint32_t id, uint32_t step, uint32_t sub, uint32_t out[4]) {
  uint32_t ctr[4] = {id, step, sub, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  or_philox4x32_10(ctr, key, out);
}

/* uniform on (0,1): the top 23 bits, centred in their cell; (2k+1) 2^-24 with
 * k < 2^23 is exact in binary32 as well as binary64 */
double or_uniform(uint32_t r) { return ((double)(r >> 9) + 0.5) * (1.0 / 8388608.0); }

/* Box-Muller transform */
void or_box_muller(double u1, double u2, double *z0, double *z1) {
  double rad = sqrt(-2.0 * log(u1));
  double ang = 6.283185307179586 * u2;
  *z0 = rad * cos(ang);
  *z1 = rad * sin(ang);
}

/* Marsaglia & Tsang gamma variate, shape >= 1; attempt a uses Philox
 * sub-stream subbase + a; after 32 rejections the mean is returned. */
double or_gamma(double shape, double scale, uint64_t seed, uint32_t id, uint32_t step,
                uint32_t subbase, int32_t *fail) {
  double d = shape - 1.0 / 3.0;
  double c = 1.0 / sqrt(9.0 * d);
  for (uint32_t a = 0; a < 32; ++a) {
    uint32_t r[4];
    draw(seed, id, step, subbase + a, r);
    double z, z1;
    or_box_muller(or_uniform(r[0]), or_uniform(r[1]), &z, &z1);
    double v = 1.0 + c * z;
    if (v <= 0.0) continue;
    v = v * v * v;
    double u = or_uniform(r[2]);
    if (log(u) < 0.5 * z * z + d - d * v + d * log(v)) return d * v * scale;
  }
  if (fail) *fail = 1;
  return shape * scale;
}

/* ------------------------------------------------------------------------ */
/* Mesh                                                                      */
/* ------------------------------------------------------------------------ */
struct or_mesh {
  int32_t nn, ne, nb;
  double *xy;
  int32_t *en, *nbr, *be, *bl, *bt, *bp;
  double *bs;
  int32_t *master;
  double *area, *dNdx, *dNdy;
  int32_t *n2e_off, *n2e; /* node -> elements */
  int32_t *m2e_off, *m2e; /* master node -> elements touching any node identified with it */
  int32_t *w_off, *w_list; /* element -> no-slip wall edges sharing a node with it */
  int32_t *nwall_off, *nwall; /* node -> wall (slip or no-slip) edges ending at it */
};

static void *dup(const void *p, size_t n) {
  void *q = malloc(n ? n : 1);
  if (n) memcpy(q, p, n);
  return q;
}

static void build_csr(int32_t nkeys, int64_t nitems, const int32_t *key, const int32_t *val,
                      int32_t **off_out, int32_t **list_out) {
  int32_t *off = (int32_t *)calloc((size_t)nkeys + 1, sizeof(int32_t));
  for (int64_t i = 0; i < nitems; ++i) off[key[i] + 1]++;
  for (int32_t k = 0; k < nkeys; ++k) off[k + 1] += off[k];
  int32_t *fill = (int32_t *)dup(off, sizeof(int32_t) * (size_t)nkeys);
  int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nitems ? nitems : 1));
  for (int64_t i = 0; i < nitems; ++i) list[fill[key[i]]++] = val[i];
  free(fill);
  *off_out = off;
  *list_out = list;
}

or_mesh *or_mesh_new(int32_t nn, int32_t ne, int32_t nb, const double *xy, const int32_t *en,
                     const int32_t *nbr, const int32_t *be, const int32_t *bl, const int32_t *bt,
                     const int32_t *bp, const double *bs, const int32_t *master) {
  or_mesh *m = (or_mesh *)calloc(1, sizeof(or_mesh));
  m->nn = nn;
  m->ne = ne;
  m->nb = nb;
  m->xy = (double *)dup(xy, sizeof(double) * 2 * (size_t)nn);
  m->en = (int32_t *)dup(en, sizeof(int32_t) * 3 * (size_t)ne);
  m->nbr = (int32_t *)dup(nbr, sizeof(int32_t) * 3 * (size_t)ne);
  m->be = (int32_t *)dup(be, sizeof(int32_t) * (size_t)nb);
  m->bl = (int32_t *)dup(bl, sizeof(int32_t) * (size_t)nb);
  m->bt = (int32_t *)dup(bt, sizeof(int32_t) * (size_t)nb);
  m->bp = (int32_t *)dup(bp, sizeof(int32_t) * (size_t)nb);
  m->bs = (double *)dup(bs, sizeof(double) * 2 * (size_t)nb);
  m->master = (int32_t *)dup(master, sizeof(int32_t) * (size_t)nn);
  m->area = (double *)malloc(sizeof(double) * (size_t)ne);
  m->dNdx = (double *)malloc(sizeof(double) * 3 * (size_t)ne);
  m->dNdy = (double *)malloc(sizeof(double) * 3 * (size_t)ne);
  /* element area and shape-function derivatives (Sec. Derivatives) */
  for (int32_t e = 0; e < ne; ++e) {
    const double *A = &xy[2 * en[3 * e + 0]], *B = &xy[2 * en[3 * e + 1]], *C = &xy[2 * en[3 * e + 2]];
    double xBA = B[0] - A[0], yBA = B[1] - A[1], xCA = C[0] - A[0], yCA = C[1] - A[1];
    double twoA = xBA * yCA - xCA * yBA;
    m->area[e] = 0.5 * twoA;
    m->dNdx[3 * e + 0] = (-yCA + yBA) / twoA;
    m->dNdx[3 * e + 1] = yCA / twoA;
    m->dNdx[3 * e + 2] = -yBA / twoA;
    m->dNdy[3 * e + 0] = (xCA - xBA) / twoA;
    m->dNdy[3 * e + 1] = -xCA / twoA;
    m->dNdy[3 * e + 2] = xBA / twoA;
  }
  /* linked lists: elements surrounding points, by node and by master node */
  int32_t *key = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)ne);
  int32_t *val = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)ne);
  for (int32_t e = 0; e < ne; ++e)
    for (int k = 0; k < 3; ++k) {
      key[3 * e + k] = en[3 * e + k];
      val[3 * e + k] = e;
    }
  build_csr(nn, 3 * (int64_t)ne, key, val, &m->n2e_off, &m->n2e);
  int64_t cnt = 0;
  for (int32_t e = 0; e < ne; ++e) {
    /* an element appears once per distinct master among its nodes */
    int32_t mk[3] = {master[en[3 * e]], master[en[3 * e + 1]], master[en[3 * e + 2]]};
    for (int k = 0; k < 3; ++k) {
      int dupe = 0;
      for (int j = 0; j < k; ++j) dupe |= (mk[j] == mk[k]);
      if (dupe) continue;
      key[cnt] = mk[k];
      val[cnt] = e;
      cnt++;
    }
  }
  build_csr(nn, cnt, key, val, &m->m2e_off, &m->m2e);
  free(key);
  free(val);
  /* element -> no-slip wall edges that share a node with the element */
  int32_t *nw_off = (int32_t *)calloc((size_t)nn + 1, sizeof(int32_t));
  for (int32_t b = 0; b < nb; ++b) {
    if (bt[b] != OR_BC_NOSLIP) continue;
    int32_t e = be[b], k = bl[b];
    nw_off[en[3 * e + (k + 1) % 3] + 1]++;
    nw_off[en[3 * e + (k + 2) % 3] + 1]++;
  }
  for (int32_t n = 0; n < nn; ++n) nw_off[n + 1] += nw_off[n];
  int32_t *nw = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nw_off[nn] + 1));
  int32_t *fill = (int32_t *)dup(nw_off, sizeof(int32_t) * (size_t)nn);
  for (int32_t b = 0; b < nb; ++b) {
    if (bt[b] != OR_BC_NOSLIP) continue;
    int32_t e = be[b], k = bl[b];
    nw[fill[en[3 * e + (k + 1) % 3]]++] = b;
    nw[fill[en[3 * e + (k + 2) % 3]]++] = b;
  }
  free(fill);
  m->w_off = (int32_t *)calloc((size_t)ne + 1, sizeof(int32_t));
  int32_t cap = 16 * ne + 16, used = 0;
  m->w_list = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
  for (int32_t e = 0; e < ne; ++e) {
    int32_t tmp[64];
    int nt = 0;
    for (int k = 0; k < 3; ++k) {
      int32_t n = en[3 * e + k];
      for (int32_t i = nw_off[n]; i < nw_off[n + 1]; ++i) {
        int32_t b = nw[i], seen = 0;
        for (int j = 0; j < nt; ++j) seen |= (tmp[j] == b);
        if (!seen && nt < 64) tmp[nt++] = b;
      }
    }
    /* ascending edge index */
    for (int i = 1; i < nt; ++i)
      for (int j = i; j > 0 && tmp[j - 1] > tmp[j]; --j) {
        int32_t t = tmp[j];
        tmp[j] = tmp[j - 1];
        tmp[j - 1] = t;
      }
    if (used + nt > cap) {
      cap = 2 * cap + nt;
      m->w_list = (int32_t *)realloc(m->w_list, sizeof(int32_t) * (size_t)cap);
    }
    for (int i = 0; i < nt; ++i) m->w_list[used++] = tmp[i];
    m->w_off[e + 1] = used;
  }
  free(nw_off);
  free(nw);
  /* node -> wall edges (slip and no-slip) ending at the node, ascending */
  m->nwall_off = (int32_t *)calloc((size_t)nn + 1, sizeof(int32_t));
  for (int32_t b = 0; b < nb; ++b) {
    if (bt[b] == OR_BC_PERIODIC || bt[b] == OR_BC_OUTFLOW) continue;
    int32_t e = be[b], k = bl[b];
    m->nwall_off[en[3 * e + (k + 1) % 3] + 1]++;
    m->nwall_off[en[3 * e + (k + 2) % 3] + 1]++;
  }
  for (int32_t n = 0; n < nn; ++n) m->nwall_off[n + 1] += m->nwall_off[n];
  m->nwall = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m->nwall_off[nn] + 1));
  fill = (int32_t *)dup(m->nwall_off, sizeof(int32_t) * (size_t)nn);
  for (int32_t b = 0; b < nb; ++b) {
    if (bt[b] == OR_BC_PERIODIC || bt[b] == OR_BC_OUTFLOW) continue;
    int32_t e = be[b], k = bl[b];
    m->nwall[fill[en[3 * e + (k + 1) % 3]]++] = b;
    m->nwall[fill[en[3 * e + (k + 2) % 3]]++] = b;
  }
  free(fill);
  return m;
}

void or_mesh_free(or_mesh *m) {
  if (!m) return;
  free(m->xy); free(m->en); free(m->nbr); free(m->be); free(m->bl); free(m->bt); free(m->bp);
  free(m->bs); free(m->master); free(m->area); free(m->dNdx); free(m->dNdy);
  free(m->n2e_off); free(m->n2e); free(m->m2e_off); free(m->m2e); free(m->w_off); free(m->w_list);
  free(m->nwall_off); free(m->nwall);
  free(m);
}

/* ------------------------------------------------------------------------ */
/* Element test (eq:element-test).  The three signed areas of the triangles */
/* formed by the point and each edge are evaluated directly as 2-D cross    */
/* products, each edge in one canonical direction (from its lower to its    */
/* higher node number) so that both elements sharing an edge obtain the     */
/* same magnitude with opposite sign.  lam[k] belongs to the edge opposite   */
/* local node k and equals twice the area coordinate of node k.              */
/* ------------------------------------------------------------------------ */
void or_lambdas(const or_mesh *m, int32_t e, double x, double y, double lam[3]) {
  for (int k = 0; k < 3; ++k) {
    int32_t a = m->en[3 * e + (k + 1) % 3], b = m->en[3 * e + (k + 2) % 3];
    int32_t p = a < b ? a : b, q = a < b ? b : a;
    double xp = m->xy[2 * p], yp = m->xy[2 * p + 1], xq = m->xy[2 * q], yq = m->xy[2 * q + 1];
    double cr = (xq - xp) * (y - yp) - (yq - yp) * (x - xp);
    lam[k] = a < b ? cr : -cr;
  }
}

static int inside(const or_mesh *m, int32_t e, double x, double y) {
  double l[3];
  or_lambdas(m, e, x, y, l);
  return l[0] >= 0.0 && l[1] >= 0.0 && l[2] >= 0.0;
}

int32_t or_locate_brute(const or_mesh *m, double x, double y) {
  for (int32_t e = 0; e < m->ne; ++e)
    if (inside(m, e, x, y)) return e;
  return -1;
}

/* fall-back of Fig. corner: the elements surrounding the nodes of element e */
static int32_t search_patch(const or_mesh *m, int32_t e, double x, double y) {
  for (int k = 0; k < 3; ++k) {
    int32_t n = m->en[3 * e + k];
    for (int32_t i = m->n2e_off[n]; i < m->n2e_off[n + 1]; ++i)
      if (inside(m, m->n2e[i], x, y)) return m->n2e[i];
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Element-average statistics (loop (ii) of Table tab:loops): the average of */
/* the nodal values of the element's three nodes, plus the element's own     */
/* FEM gradient of the nodal mean velocity (eq:gradient).                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  double U[3], Om, Phi, R[6], k, eps, G[3][3], C0, dU[3][2], lap[3], gp[2], Sw, inv_tm, gsk[2];
} orec;

#define S(f, n) stats[(size_t)(f) * (size_t)nn + (size_t)(n)]

static double sym(const double R[6], int i, int j) {
  static const int idx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  return R[idx[i][j]];
}

/* Value over element e of a nodal field f (values a[f*nn + node]): with w ==
 * NULL the element average of its three nodal values (Fig. mesh-particles);
 * otherwise the shape-function combination sum_j N^j q_j of eq:approximation
 * with N^j = w[j]. */
static double nodal_at(const double *a, int32_t nn, int f, const int32_t mk[3], const double *w) {
  const double *q = a + (size_t)f * (size_t)nn;
  if (!w) return (q[mk[0]] + q[mk[1]] + q[mk[2]]) / 3.0;
  return w[0] * q[mk[0]] + w[1] * q[mk[1]] + w[2] * q[mk[2]];
}

/* Shape-function values N^j of point (x, y) in element e: the area
 * coordinates, i.e. each signed area of eq:element-test over their sum. */
static void shape_values(const or_mesh *m, int32_t e, double x, double y, double w[3]) {
  double lam[3];
  or_lambdas(m, e, x, y, lam);
  double s = lam[0] + lam[1] + lam[2];
  for (int k = 0; k < 3; ++k) w[k] = lam[k] / s;
}

/* Statistics and coefficients for the particles of element e: from the
 * element average of the nodal values (w == NULL, the paper's reading) or
 * from their shape-function values at one particle position (w = N^j). */
static void elem_record(const or_mesh *m, const or_params *p, const double *stats, const double *wp,
                        const double *gradp, int32_t e, const double *w, const double *pt, orec *r) {
  int32_t nn = m->nn;
  int32_t mk[3];
  for (int k = 0; k < 3; ++k) mk[k] = m->master[m->en[3 * e + k]];
  memset(r, 0, sizeof(*r));
  for (int i = 0; i < 3; ++i) r->U[i] = nodal_at(stats, nn, i, mk, w);
  r->Om = nodal_at(stats, nn, 3, mk, w);
  r->Phi = nodal_at(stats, nn, 4, mk, w);
  for (int i = 0; i < 6; ++i) r->R[i] = nodal_at(stats, nn, 5 + i, mk, w);
  for (int i = 0; i < 3; ++i) r->lap[i] = nodal_at(stats, nn, 21 + i, mk, w);
  for (int i = 0; i < 2; ++i) r->gp[i] = gradp ? nodal_at(gradp, nn, i, mk, w) : 0.0;
  /* eq:gradient with the precomputed shape-function derivatives */
  for (int i = 0; i < 3; ++i) {
    double gx = 0.0, gy = 0.0;
    for (int k = 0; k < 3; ++k) {
      gx += m->dNdx[3 * e + k] * S(i, mk[k]);
      gy += m->dNdy[3 * e + k] * S(i, mk[k]);
    }
    r->dU[i][0] = gx;
    r->dU[i][1] = gy;
  }
  /* gradient of sqrt(2k) for the wall frequency of eq:frequency-wallstats */
  r->gsk[0] = r->gsk[1] = 0.0;
  for (int k = 0; k < 3; ++k) {
    double kn = 0.5 * (S(5, mk[k]) + S(6, mk[k]) + S(7, mk[k]));
    double s = sqrt(2.0 * (kn > 0.0 ? kn : 0.0));
    r->gsk[0] += m->dNdx[3 * e + k] * s;
    r->gsk[1] += m->dNdy[3 * e + k] * s;
  }
  /* k = <u_i u_i>/2 and eq:dissipation-from-frequency_wall */
  double k = 0.5 * (r->R[0] + r->R[1] + r->R[2]);
  if (!(k > p->k_floor)) k = p->k_floor;
  r->k = k;
  r->eps = r->Om * (k + p->nu * p->CT * p->CT * r->Om);
  if (p->model == 0) {
    /* eq:wall-GandC: simplified Langevin model */
    r->C0 = p->C0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) r->G[i][j] = (i == j) ? -(0.5 + 0.75 * p->C0) * r->Om : 0.0;
  } else {
    /* eq:GandC with the element average of the nodal tensor wp_ij */
    double W[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) W[i][j] = nodal_at(wp, nn, 3 * i + j, mk, w);
    double wr = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        r->G[i][j] = (W[i][j] - ((i == j) ? 0.5 * r->eps : 0.0)) / k;
        wr += W[i][j] * sym(r->R, i, j);
      }
    double c0 = -2.0 * wr / (3.0 * k * r->eps);
    r->C0 = (c0 > 0.0) ? c0 : 0.0; /* realizability: C0 >= 0 */
  }
  /* production P = -<u_i u_j> dU_i/dx_j (two in-plane directions) and eq:frequency-source */
  double prod = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 2; ++j) prod -= sym(r->R, i, j) * r->dU[i][j];
  r->Sw = p->omega_source ? (p->Cw2 - p->Cw1 * prod / r->eps) : 0.0;
  /* micromixing time scale */
  if (p->tm_mode == 0) {
    r->inv_tm = 0.5 * p->Cphi * r->Om;
  } else {
    double a = k / r->eps, b = p->CT * sqrt(p->nu / r->eps);
    double tm = a > b ? a : b;
    if (p->tm_mode == 2) {
      /* eq:micromixing-timescale-canyon at the point pt: the source term
       * C_s (r0^2/eps)^(1/3) + C_t d / U_c, with d the distance from the
       * source centre and U_c the magnitude of the mean velocity; it drops
       * out where U_c = 0 */
      double dx = pt[0] - p->src_x, dy = pt[1] - p->src_y;
      double d = sqrt(dx * dx + dy * dy);
      double uc = sqrt(r->U[0] * r->U[0] + r->U[1] * r->U[1] + r->U[2] * r->U[2]);
      if (uc > 0.0) {
        double ts = p->Cs * cbrt(p->src_r * p->src_r / r->eps) + p->Ct * d / uc;
        if (ts < tm) tm = ts;
      }
    }
    r->inv_tm = 1.0 / tm;
  }
}

/* the point at which the source-aware time scale is evaluated for element e
 * in the ELEM reading: the centroid */
static void centroid(const or_mesh *m, int32_t e, double pt[2]) {
  const double *A = &m->xy[2 * m->en[3 * e]], *B = &m->xy[2 * m->en[3 * e + 1]],
               *C = &m->xy[2 * m->en[3 * e + 2]];
  pt[0] = (A[0] + B[0] + C[0]) / 3.0;
  pt[1] = (A[1] + B[1] + C[1]) / 3.0;
}

/* ------------------------------------------------------------------------ */
/* Local form of the elliptic relaxation (eq:elliptic-relaxation-Lagrangian  */
/* with L -> 0): wp_ij = (1-C1)/2 k<omega> delta_ij + k H_ijkl dU_k/dx_l,     */
/* H from eq:H, A_v, and b_ij from eq:bij; evaluated from nodal statistics.  */
/* ------------------------------------------------------------------------ */
void or_local_wp(const or_mesh *m, const or_params *p, const double *stats, double *wp) {
  int32_t nn = m->nn;
  for (int32_t n = 0; n < nn; ++n) {
    int32_t q = m->master[n];
    double R[6];
    for (int i = 0; i < 6; ++i) R[i] = S(5 + i, q);
    double k = 0.5 * (R[0] + R[1] + R[2]);
    if (!(k > p->k_floor)) k = p->k_floor;
    double om = S(3, q);
    double Sg[3][3] = {{S(15, q), S(16, q), 0.0}, {S(17, q), S(18, q), 0.0}, {S(19, q), S(20, q), 0.0}};
    double det = R[0] * (R[1] * R[2] - R[5] * R[5]) - R[3] * (R[3] * R[2] - R[5] * R[4]) +
                 R[4] * (R[3] * R[5] - R[1] * R[4]);
    double k23 = 2.0 / 3.0 * k;
    double Av = p->Cv * det / (k23 * k23 * k23);
    if (Av > 1.0) Av = 1.0;
    double b[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) b[i][j] = sym(R, i, j) / (2.0 * k) - ((i == j) ? 1.0 / 3.0 : 0.0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        /* H_ijkl S_kl, term by term of eq:H */
        double h = (p->C2 * Av + p->gamma5 / 3.0) * Sg[i][j] - p->gamma5 / 3.0 * Sg[j][i];
        for (int l = 0; l < 3; ++l) h += p->gamma5 * b[i][l] * Sg[l][j] - p->gamma5 * b[i][l] * Sg[j][l];
        double v = k * h + ((i == j) ? 0.5 * (1.0 - p->C1) * k * om : 0.0);
        wp[(size_t)(3 * i + j) * nn + n] = v;
      }
  }
}


/* First and second derivatives of the nodal mean velocity (Sec. Derivatives):
 * eq:gradient over every element, averaged to the nodes; the same procedure
 * applied to the nodal first derivatives gives the second derivatives, whose
 * in-plane trace is the Laplacian.  Reads fields 0-2, writes 15-23. */
void or_derivatives(const or_mesh *m, double *stats) {
  int32_t nn = m->nn;
  /* first derivatives: element gradient of nodal means, averaged to nodes */
  for (int32_t n = 0; n < nn; ++n) {
    if (m->master[n] != n) continue;
    double g[6] = {0};
    int32_t c = 0;
    for (int32_t i = m->m2e_off[n]; i < m->m2e_off[n + 1]; ++i) {
      int32_t e = m->m2e[i];
      c++;
      for (int f = 0; f < 3; ++f)
        for (int k = 0; k < 3; ++k) {
          int32_t mk = m->master[m->en[3 * e + k]];
          g[2 * f] += m->dNdx[3 * e + k] * S(f, mk);
          g[2 * f + 1] += m->dNdy[3 * e + k] * S(f, mk);
        }
    }
    for (int f = 0; f < 6; ++f) S(15 + f, n) = c ? g[f] / (double)c : 0.0;
  }
  /* second derivatives: element gradient of the nodal first derivatives */
  for (int32_t n = 0; n < nn; ++n) {
    if (m->master[n] != n) continue;
    double l[3] = {0};
    int32_t c = 0;
    for (int32_t i = m->m2e_off[n]; i < m->m2e_off[n + 1]; ++i) {
      int32_t e = m->m2e[i];
      c++;
      for (int f = 0; f < 3; ++f)
        for (int k = 0; k < 3; ++k) {
          int32_t mk = m->master[m->en[3 * e + k]];
          l[f] += m->dNdx[3 * e + k] * S(15 + 2 * f, mk) + m->dNdy[3 * e + k] * S(16 + 2 * f, mk);
        }
    }
    for (int f = 0; f < 3; ++f) S(21 + f, n) = c ? l[f] / (double)c : 0.0;
  }
  /* identified (periodic) nodes carry their master's values */
  for (int32_t n = 0; n < nn; ++n) {
    int32_t q0 = m->master[n];
    if (q0 != n)
      for (int f = 0; f < OR_NSTAT; ++f) S(f, n) = S(f, q0);
  }
}

/* ------------------------------------------------------------------------ */
/* Statistics: the two-pass particle-in-cell estimator.  Element means and   */
/* central second moments (1/N) from the particles residing in each element; */
/* nodal values as the average over the surrounding elements that hold       */
/* particles; first and second derivatives by eq:gradient and the two-pass   */
/* node averaging.                                                           */
/* Nodal fields: 0-2 <U_i>, 3 <omega>, 4 <phi>, 5-10 <u_i u_j> (11,22,33,12,  */
/* 13,23), 11 <phi'^2>, 12-14 <u_i phi'>, 15-20 d<U_i>/dx, d<U_i>/dy (i =    */
/* U,V,W), 21-23 laplacian of <U_i>, 24 number of particles in the non-empty  */
/* surrounding elements.                                                     */
/* ------------------------------------------------------------------------ */
void or_estimate(const or_mesh *m, const or_params *p, int64_t np, const double *state,
                 const int32_t *elem, const double *prev, double *stats, double *elem_out,
                 uint64_t *cnt) {
  int32_t ne = m->ne, nn = m->nn;
  const double *q[5] = {state + 2 * np, state + 3 * np, state + 4 * np, state + 5 * np, state + 6 * np};
  double *N = (double *)calloc((size_t)ne, sizeof(double));
  double *mean = (double *)calloc((size_t)ne * 5, sizeof(double));
  double *cov = (double *)calloc((size_t)ne * 10, sizeof(double));
  static const int ca[10] = {0, 1, 2, 0, 0, 1, 4, 0, 1, 2};
  static const int cb[10] = {0, 1, 2, 1, 2, 2, 4, 4, 4, 4};
  for (int64_t i = 0; i < np; ++i) {
    int32_t e = elem[i];
    N[e] += 1.0;
    for (int f = 0; f < 5; ++f) mean[5 * e + f] += q[f][i];
  }
  for (int32_t e = 0; e < ne; ++e)
    if (N[e] > 0.0)
      for (int f = 0; f < 5; ++f) mean[5 * e + f] /= N[e];
  for (int64_t i = 0; i < np; ++i) {
    int32_t e = elem[i];
    for (int c = 0; c < 10; ++c)
      cov[10 * e + c] += (q[ca[c]][i] - mean[5 * e + ca[c]]) * (q[cb[c]][i] - mean[5 * e + cb[c]]);
  }
  for (int32_t e = 0; e < ne; ++e)
    if (N[e] > 0.0)
      for (int c = 0; c < 10; ++c) cov[10 * e + c] /= N[e];
  if (elem_out) {
    for (int32_t e = 0; e < ne; ++e) {
      elem_out[e] = N[e];
      for (int f = 0; f < 5; ++f) elem_out[(size_t)(1 + f) * ne + e] = mean[5 * e + f];
      for (int c = 0; c < 10; ++c) elem_out[(size_t)(6 + c) * ne + e] = cov[10 * e + c];
    }
  }
  if (p && p->stats_mode == 1) {
    /* SHAPE: node n gathers every particle of the elements around it, each
     * with weight N^n at the particle's position (eq:approximation used as a
     * scatter): weighted means, then weighted central second moments. */
    double *W = (double *)calloc((size_t)nn, sizeof(double));
    double *M = (double *)calloc((size_t)nn * 5, sizeof(double));
    double *CV = (double *)calloc((size_t)nn * 10, sizeof(double));
    for (int64_t i = 0; i < np; ++i) {
      double w[3];
      shape_values(m, elem[i], state[i], state[np + i], w);
      for (int k = 0; k < 3; ++k) {
        int32_t n = m->master[m->en[3 * elem[i] + k]];
        W[n] += w[k];
        for (int f = 0; f < 5; ++f) M[5 * n + f] += w[k] * q[f][i];
      }
    }
    for (int32_t n = 0; n < nn; ++n)
      if (W[n] > 0.0)
        for (int f = 0; f < 5; ++f) M[5 * n + f] /= W[n];
    for (int64_t i = 0; i < np; ++i) {
      double w[3];
      shape_values(m, elem[i], state[i], state[np + i], w);
      for (int k = 0; k < 3; ++k) {
        int32_t n = m->master[m->en[3 * elem[i] + k]];
        for (int c = 0; c < 10; ++c)
          CV[10 * n + c] += w[k] * (q[ca[c]][i] - M[5 * n + ca[c]]) * (q[cb[c]][i] - M[5 * n + cb[c]]);
      }
    }
    for (int32_t n = 0; n < nn; ++n) {
      if (m->master[n] != n) continue;
      if (W[n] > 0.0) {
        for (int f = 0; f < 5; ++f) S(f, n) = M[5 * n + f];
        for (int c = 0; c < 10; ++c) S(5 + c, n) = CV[10 * n + c] / W[n];
      } else {
        for (int f = 0; f < 15; ++f) S(f, n) = prev ? prev[(size_t)f * nn + n] : 0.0;
        if (cnt) cnt[OR_CNT_EMPTY_NODE]++;
      }
      S(24, n) = W[n];
    }
    free(W);
    free(M);
    free(CV);
    or_derivatives(m, stats);
    free(N);
    free(mean);
    free(cov);
    return;
  }
  /* pass 2: element -> node averages over non-empty surrounding elements */
  for (int32_t n = 0; n < nn; ++n) {
    if (m->master[n] != n) continue;
    double acc[15] = {0}, sup = 0.0;
    int32_t cntE = 0;
    for (int32_t i = m->m2e_off[n]; i < m->m2e_off[n + 1]; ++i) {
      int32_t e = m->m2e[i];
      if (!(N[e] > 0.0)) continue;
      cntE++;
      sup += N[e];
      for (int f = 0; f < 5; ++f) acc[f] += mean[5 * e + f];
      for (int c = 0; c < 10; ++c) acc[5 + c] += cov[10 * e + c];
    }
    if (cntE > 0) {
      for (int f = 0; f < 15; ++f) S(f, n) = acc[f] / (double)cntE;
    } else {
      for (int f = 0; f < 15; ++f) S(f, n) = prev ? prev[(size_t)f * nn + n] : 0.0;
      if (cnt) cnt[OR_CNT_EMPTY_NODE]++;
    }
    S(24, n) = sup;
  }
  or_derivatives(m, stats);
  free(N);
  free(mean);
  free(cov);
}

/* ------------------------------------------------------------------------ */
/* Initial particle state (Sec. Particle-number control): ppe particles per  */
/* element, uniform positions, Gaussian velocities with the prescribed mean  */
/* and Reynolds stress, gamma frequencies with mean Om0 and variance        */
/* C4 Om0^2, scalar from the chosen initial condition.                       */
/* ------------------------------------------------------------------------ */
static double st(const or_params *p, double v) { return p->store_fp32 ? (double)(float)v : v; }

void or_seed(const or_mesh *m, const or_params *p, const or_seedspec *s, double *state,
             int32_t *elem, uint32_t *id) {
  int64_t np = (int64_t)m->ne * s->ppe;
  int32_t nn = m->nn;
  for (int32_t e = 0; e < m->ne; ++e) {
    int32_t nA = m->en[3 * e], nB = m->en[3 * e + 1], nC = m->en[3 * e + 2];
    const double *A = &m->xy[2 * nA], *B = &m->xy[2 * nB], *C = &m->xy[2 * nC];
    for (int32_t j = 0; j < s->ppe; ++j) {
      int64_t i = (int64_t)e * s->ppe + j;
      uint32_t pid = (uint32_t)i;
      uint32_t r[4], r2[4];
      draw(s->seed, pid, 0xFFFFFFFFu, 0, r);
      draw(s->seed, pid, 0xFFFFFFFFu, 1, r2);
      double r1 = or_uniform(r[0]), rr2 = or_uniform(r[1]);
      if (r1 + rr2 > 1.0) {
        r1 = 1.0 - r1;
        rr2 = 1.0 - rr2;
      }
      double x = A[0] + r1 * (B[0] - A[0]) + rr2 * (C[0] - A[0]);
      double y = A[1] + r1 * (B[1] - A[1]) + rr2 * (C[1] - A[1]);
      double wA = 1.0 - r1 - rr2, wB = r1, wC = rr2;
      double z[4];
      or_box_muller(or_uniform(r[2]), or_uniform(r[3]), &z[0], &z[1]);
      or_box_muller(or_uniform(r2[0]), or_uniform(r2[1]), &z[2], &z[3]);
      double U[3], R[6], Om;
      for (int f = 0; f < 3; ++f)
        U[f] = wA * s->U0[(size_t)f * nn + nA] + wB * s->U0[(size_t)f * nn + nB] + wC * s->U0[(size_t)f * nn + nC];
      for (int f = 0; f < 6; ++f)
        R[f] = wA * s->R0[(size_t)f * nn + nA] + wB * s->R0[(size_t)f * nn + nB] + wC * s->R0[(size_t)f * nn + nC];
      Om = wA * s->Om0[nA] + wB * s->Om0[nB] + wC * s->Om0[nC];
      /* Cholesky factor of the Reynolds stress (11,22,33,12,13,23) */
      double L11 = sqrt(R[0] > 0.0 ? R[0] : 0.0);
      double L21 = L11 > 0.0 ? R[3] / L11 : 0.0, L31 = L11 > 0.0 ? R[4] / L11 : 0.0;
      double t22 = R[1] - L21 * L21;
      double L22 = sqrt(t22 > 0.0 ? t22 : 0.0);
      double L32 = L22 > 0.0 ? (R[5] - L31 * L21) / L22 : 0.0;
      double t33 = R[2] - L31 * L31 - L32 * L32;
      double L33 = sqrt(t33 > 0.0 ? t33 : 0.0);
      double u = U[0] + L11 * z[0];
      double v = U[1] + L21 * z[0] + L22 * z[1];
      double w = U[2] + L31 * z[0] + L32 * z[1] + L33 * z[2];
      int32_t fail = 0;
      double om = (Om > 0.0) ? or_gamma(1.0 / p->C4, p->C4 * Om, s->seed, pid, 0xFFFFFFFFu, 16, &fail) : 0.0;
      x = st(p, x);
      y = st(p, y);
      double psi = 0.0;
      switch (s->psi_mode) {
        case 1: psi = (x < s->a) ? 1.0 : 0.0; break;
        case 2: psi = exp(-(x - s->a) * (x - s->a) / (2.0 * s->b * s->b)); break;
        case 3: psi = (or_uniform(r2[2]) < 0.5) ? 1.0 : 0.0; break;
        case 4: psi = ((x - s->a) * (x - s->a) + (y - s->b) * (y - s->b) <= s->c * s->c) ? 1.0 : 0.0; break;
        default: psi = 0.0;
      }
      state[0 * np + i] = x;
      state[1 * np + i] = y;
      state[2 * np + i] = st(p, u);
      state[3 * np + i] = st(p, v);
      state[4 * np + i] = st(p, w);
      state[5 * np + i] = st(p, om);
      state[6 * np + i] = st(p, psi);
      elem[i] = e;
      id[i] = pid;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* eq:CFL: the time step from the smallest characteristic time of the grid   */
/* nodes, sqrt of the average surrounding element area over the length of    */
/* the in-plane mean velocity.                                               */
/* ------------------------------------------------------------------------ */
double or_cfl_dt(const or_mesh *m, const double *stats, double c_cfl, double dt_max) {
  const int32_t nn = m->nn;
  double best = -1.0;
  for (int32_t n = 0; n < nn; ++n) {
    if (m->master[n] != n) continue;
    const int32_t a = m->m2e_off[n], b = m->m2e_off[n + 1];
    if (b <= a) continue;
    double area = 0.0;
    for (int32_t i = a; i < b; ++i) area += m->area[m->m2e[i]];
    const double sa = sqrt(area / (double)(b - a));
    const double u = S(0, n), v = S(1, n);
    const double sp = sqrt(u * u + v * v);
    if (!(sp > 0.0)) continue;
    const double t = sa / sp;
    if (best < 0.0 || t < best) best = t;
  }
  if (best < 0.0) return dt_max;
  const double dt = c_cfl * best;
  return dt < dt_max ? dt : dt_max;
}

/* ------------------------------------------------------------------------ */
/* Particle redistribution (App. D, improved algorithm).                     */
/* The elements are ordered by increasing particle count (ties: increasing   */
/* element number).  The k-th element of that order with fewer than         */
/* min_ppe particles receives particles from the k-th element from the top:  */
/* m = min(min_ppe - N_receiver, N_donor - min_ppe) of the donor's particles */
/* (its first ones by increasing id) move, each taking the whole state of a   */
/* receiver resident (its residents by increasing id, cycled).  An empty     */
/* receiver gets a uniform position in the element instead (uniforms from    */
/* sub-stream 3 of the particle's step counter), the rest of the moving      */
/* particle's state kept.  Donors never fall below min_ppe; a donor at or    */
/* below its receiver's place in the order ends the pass.                    */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t n, e; } or_ne;
static int cmp_ne(const void *a, const void *b) {
  const or_ne *x = (const or_ne *)a, *y = (const or_ne *)b;
  if (x->n != y->n) return x->n < y->n ? -1 : 1;
  return x->e < y->e ? -1 : (x->e > y->e ? 1 : 0);
}
typedef struct { uint32_t id; int64_t i; } or_idx;
static int cmp_idx(const void *a, const void *b) {
  const or_idx *x = (const or_idx *)a, *y = (const or_idx *)b;
  return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}
/* the particles of element e in increasing id order */
static int64_t members(int64_t np, const int32_t *elem, const uint32_t *id, int32_t e, or_idx *out) {
  int64_t c = 0;
  for (int64_t i = 0; i < np; ++i)
    if (elem[i] == e) {
      out[c].id = id[i];
      out[c].i = i;
      c++;
    }
  qsort(out, (size_t)c, sizeof(or_idx), cmp_idx);
  return c;
}

int64_t or_redistribute(const or_mesh *m, const or_params *p, int64_t np, double *state, int32_t *elem,
                        const uint32_t *id, uint64_t seed, uint32_t step) {
  const int32_t ne = m->ne, mn = p->min_ppe;
  if (mn <= 0) return 0;
  or_ne *ord = (or_ne *)malloc(sizeof(or_ne) * (size_t)ne);
  for (int32_t e = 0; e < ne; ++e) {
    ord[e].n = 0;
    ord[e].e = e;
  }
  for (int64_t i = 0; i < np; ++i) ord[elem[i]].n++;
  qsort(ord, (size_t)ne, sizeof(or_ne), cmp_ne);
  or_idx *don = (or_idx *)malloc(sizeof(or_idx) * (size_t)(np + 1));
  or_idx *rec = (or_idx *)malloc(sizeof(or_idx) * (size_t)(np + 1));
  /* the moves are decided on the counts and residents before any move */
  int32_t *e0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np + 1));
  double *s0 = (double *)malloc(sizeof(double) * 7 * (size_t)(np + 1));
  memcpy(e0, elem, sizeof(int32_t) * (size_t)np);
  memcpy(s0, state, sizeof(double) * 7 * (size_t)np);
  int64_t moved = 0;
  for (int32_t k = 0; k < ne && ord[k].n < mn; ++k) {
    const int32_t kd = ne - 1 - k;
    if (kd <= k) break;
    const int32_t c = ord[k].e, d = ord[kd].e, nc = ord[k].n, nd = ord[kd].n;
    int32_t mv = mn - nc;
    if (nd - mn < mv) mv = nd - mn;
    if (mv <= 0) continue;
    int64_t cd = members(np, e0, id, d, don);
    int64_t cr = members(np, e0, id, c, rec);
    (void)cd;
    for (int32_t q = 0; q < mv; ++q) {
      const int64_t P = don[q].i;
      if (cr > 0) {
        const int64_t T = rec[q % cr].i;
        for (int f = 0; f < 7; ++f) state[(size_t)f * np + P] = s0[(size_t)f * np + T];
      } else {
        uint32_t r[4];
        draw(seed, id[P], step, 3, r);
        double r1 = or_uniform(r[0]), r2 = or_uniform(r[1]);
        if (r1 + r2 > 1.0) {
          r1 = 1.0 - r1;
          r2 = 1.0 - r2;
        }
        const double *A = &m->xy[2 * m->en[3 * c]], *B = &m->xy[2 * m->en[3 * c + 1]],
                     *C = &m->xy[2 * m->en[3 * c + 2]];
        state[P] = st(p, A[0] + r1 * (B[0] - A[0]) + r2 * (C[0] - A[0]));
        state[(size_t)np + P] = st(p, A[1] + r1 * (B[1] - A[1]) + r2 * (C[1] - A[1]));
      }
      elem[P] = c;
      moved++;
    }
  }
  free(ord);
  free(don);
  free(rec);
  free(e0);
  free(s0);
  return moved;
}

/* ------------------------------------------------------------------------ */
/* One explicit Euler-Maruyama step for every particle (mask: optional       */
/* subset), with tracking and boundary conditions.                           */
/* ------------------------------------------------------------------------ */
static void edge_geom(const or_mesh *m, int32_t e, int k, double *xa, double *ya, double *xb, double *yb) {
  int32_t a = m->en[3 * e + (k + 1) % 3], b = m->en[3 * e + (k + 2) % 3];
  *xa = m->xy[2 * a];
  *ya = m->xy[2 * a + 1];
  *xb = m->xy[2 * b];
  *yb = m->xy[2 * b + 1];
}

/* ------------------------------------------------------------------------ */
/* Wall functions (the wall treatment for complex geometries reported in    */
/* Ch.2): a particle reflected at a wall-function edge keeps its spanwise    */
/* velocity; in the edge's frame (tangent t along the edge, normal n into    */
/* the domain) its normal velocity reverses (eq:wall-normal-velocity) and its */
/* tangential velocity changes by alpha times the incident normal velocity   */
/* (eq:particle-wallcondition-wf), with alpha from the statistics at the      */
/* first gridpoint off the wall (eq:alpha, eq:hatu, eq:Ue and                */
/* eq:friction-velocity, all in the edge's frame); its frequency is scaled   */
/* by eq:wall-omega.  Constants: C_mu = 0.09, kappa = 0.41, E = 8.5.         */
/* ------------------------------------------------------------------------ */
void or_wall_function(const or_params *p, int32_t nn, const double *stats, const double *gradp, int32_t node,
                      double xa, double ya, double xb, double yb, double xc, double yc, double *u, double *v,
                      double *w, double *om) {
  const double Cmu = 0.09, kappa = 0.41, E = 8.5;
  (void)w; /* the spanwise component is not changed */
  double dx = xb - xa, dy = yb - ya, len = sqrt(dx * dx + dy * dy);
  double tx = dx / len, ty = dy / len; /* tangent */
  double nx = -ty, ny = tx;             /* normal into the domain */
  double yp = (xc - xa) * nx + (yc - ya) * ny;
  /* statistics at y_p in the edge's frame */
  double U = S(0, node), V = S(1, node), Om = S(3, node);
  double R11 = S(5, node), R22 = S(6, node), R33 = S(7, node), R12 = S(8, node);
  double Up = U * tx + V * ty;
  double vvp = R11 * nx * nx + 2.0 * R12 * nx * ny + R22 * ny * ny;
  double uvp = R11 * tx * nx + R12 * (tx * ny + ty * nx) + R22 * ty * ny;
  double kp = 0.5 * (R11 + R22 + R33);
  double dPdx = gradp ? gradp[node] * tx + gradp[(size_t)nn + node] * ty : 0.0;
  /* eq:hatu */
  double uhat2 = sqrt(Cmu) * (kp > 0.0 ? kp : 0.0);
  /* eq:friction-velocity */
  double gam = (uvp * dPdx > 0.0) ? 1.0 : 0.0;
  double utau = sqrt(uhat2 + gam * fabs(yp * dPdx));
  /* eq:Ue */
  double Ue = utau / kappa * log(E * yp * utau / p->nu_wall);
  /* eq:alpha; no transfer where the log law gives no positive U_e */
  double alpha = (Ue > 0.0 && vvp > 0.0) ? 2.0 * uhat2 * Up * fabs(Up) / (vvp * Ue * Ue) : 0.0;
  /* incident components, eq:wall-normal-velocity and eq:particle-wallcondition-wf */
  double UI = *u * tx + *v * ty, VI = *u * nx + *v * ny;
  double UR = UI + alpha * VI, VR = -VI;
  *u = UR * tx + VR * nx;
  *v = UR * ty + VR * ny;
  /* eq:wall-omega */
  double beta = -2.0 / (0.5 + 0.75 * p->C0 + p->C3 + p->Cw2 - p->Cw1);
  if (Om > 0.0 && yp > 0.0) *om = *om * exp(beta * VI / (yp * Om));
}

/* the condition at a wall-function edge of element e: its vertex c off the
 * edge is the first gridpoint from the wall (statistics of its master node) */
static void wall_fn_at(const or_params *p, const or_mesh *m, const double *stats, const double *gradp, int32_t c,
                       double xa, double ya, double xb, double yb, double *u, double *v, double *w, double *om) {
  or_wall_function(p, m->nn, stats, gradp, m->master[c], xa, ya, xb, yb, m->xy[2 * c], m->xy[2 * c + 1], u, v, w,
                   om);
}

/* no-slip particle condition: U_i = 0 and a gamma frequency with the mean and
 * variance of eq:frequency-wallstats (mean from the inward derivative of
 * sqrt(2k)); sub-stream block 16 + 32*hit */
static void noslip(const or_params *p, const orec *r, double nx, double ny, uint64_t seed,
                   uint32_t id, uint32_t step, int hit, double *u, double *v, double *w, double *om,
                   uint64_t *cnt) {
  *u = 0.0;
  *v = 0.0;
  *w = 0.0;
  double omw = -(r->gsk[0] * nx + r->gsk[1] * ny) / p->CT;
  if (!(omw > 0.0)) omw = r->Om;
  if (omw > 0.0) {
    int32_t fail = 0;
    *om = or_gamma(1.0 / p->C4, p->C4 * omw, seed, id, step, 16u + 32u * (uint32_t)hit, &fail);
    if (fail && cnt) cnt[OR_CNT_GAMMA_FAIL]++;
  }
}

/* ------------------------------------------------------------------------ */
/* Velocity-conditioned scalar mean (Sec. Estimation of the velocity-        */
/* conditioned scalar mean; App. B).  In every element the particles are     */
/* sorted by their U velocity and divided into n_u groups; each group is     */
/* sorted by V and divided into n_v; each of those by W into n_w.  A level   */
/* is taken only while every subgroup keeps at least cond_min particles (the */
/* adaptive stop); the groups taken last are the bins.  Group boundaries    */
/* follow the bin index of App. B at every level: with P groups over the n  */
/* particles of the element, the particle at position j of the order belongs */
/* to group P*j/n (integer division).  The particles start in increasing id */
/* order, and ties in a velocity component are ordered by id; a direction   */
/* with a single interval is not sorted.  <phi|V> of a particle is the mean  */
/* scalar of its bin, summed in the order of the final positions.            */
/* ------------------------------------------------------------------------ */
typedef struct { double k; uint32_t id; int64_t i; } or_ck;
static int cmp_ck(const void *a, const void *b) {
  const or_ck *x = (const or_ck *)a, *y = (const or_ck *)b;
  if (x->k != y->k) return x->k < y->k ? -1 : 1;
  return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

void or_cond_means(const or_mesh *m, const or_params *p, int64_t np, const double *state,
                   const int32_t *elem, const uint32_t *id, double *cm) {
  const int32_t ne = m->ne;
  const int32_t f[3] = {p->cond_nu, p->cond_nv, p->cond_nw};
  const int32_t cmin = p->cond_min > 1 ? p->cond_min : 1;
  /* the particles of every element (storage order; the sorts fix the order) */
  int64_t *off = (int64_t *)calloc((size_t)ne + 1, sizeof(int64_t));
  for (int64_t i = 0; i < np; ++i) off[elem[i] + 1]++;
  for (int32_t e = 0; e < ne; ++e) off[e + 1] += off[e];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)ne + 1));
  memcpy(fill, off, sizeof(int64_t) * ((size_t)ne + 1));
  or_ck *all = (or_ck *)malloc(sizeof(or_ck) * (size_t)(np + 1));
  for (int64_t i = 0; i < np; ++i) {
    or_ck *c = &all[fill[elem[i]]++];
    c->id = id[i];
    c->i = i;
  }
  for (int32_t e = 0; e < ne; ++e) {
    or_ck *b = all + off[e];
    const int64_t n = off[e + 1] - off[e];
    if (n == 0) continue;
    /* the starting order: increasing id */
    for (int64_t j = 0; j < n; ++j) b[j].k = 0.0;
    qsort(b, (size_t)n, sizeof(or_ck), cmp_ck);
    /* levels: a direction with one interval divides nothing and is skipped;
     * nc groups after the levels taken */
    int64_t nc = 1;
    for (int l = 0; l < 3; ++l) {
      if (f[l] <= 1) continue;
      const int64_t next = nc * f[l];
      if (n / next < cmin) break; /* the adaptive stop */
      /* sort each group of the previous level by velocity component l */
      for (int64_t j = 0; j < n; ++j) b[j].k = state[(size_t)(2 + l) * np + b[j].i];
      for (int64_t g = 0; g < nc; ++g) {
        const int64_t s0 = (g * n + nc - 1) / nc, s1 = ((g + 1) * n + nc - 1) / nc;
        qsort(b + s0, (size_t)(s1 - s0), sizeof(or_ck), cmp_ck);
      }
      nc = next;
    }
    /* App. B: bin index, particle count and scalar sum per bin, bin means */
    double *sum = (double *)calloc((size_t)nc, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
    for (int64_t j = 0; j < n; ++j) {
      const int64_t bin = nc * j / n;
      cnt[bin]++;
      sum[bin] += state[(size_t)6 * np + b[j].i];
    }
    for (int64_t j = 0; j < n; ++j) {
      const int64_t bin = nc * j / n;
      cm[b[j].i] = sum[bin] / (double)cnt[bin];
    }
    free(sum);
    free(cnt);
  }
  free(off);
  free(fill);
  free(all);
}

int32_t or_step(const or_mesh *m, const or_params *p, const double *stats, const double *wp,
                const double *gradp, int64_t np, double *state, int32_t *elem, const uint32_t *id,
                uint64_t seed, uint32_t step, double dt, const uint8_t *mask, uint64_t *cnt) {
  int32_t ne = m->ne;
  const int shape = (p->stats_mode == 1);
  orec *rec = (orec *)malloc(sizeof(orec) * (size_t)ne);
  if (!shape)
    for (int32_t e = 0; e < ne; ++e) {
      double pt[2];
      centroid(m, e, pt);
      elem_record(m, p, stats, wp, gradp, e, NULL, pt, &rec[e]);
    }
  orec rl;
  double *X = state, *Y = state + np, *Uu = state + 2 * np, *Vv = state + 3 * np,
         *Ww = state + 4 * np, *OM = state + 5 * np, *PS = state + 6 * np;
  int32_t lost = 0;
  /* eq:IECM: the conditioned means from the particles at the start of the step */
  double *cm = NULL;
  if (p->mix_model == 1) {
    cm = (double *)malloc(sizeof(double) * (size_t)(np + 1));
    or_cond_means(m, p, np, state, elem, id, cm);
    for (int64_t i = 0; i < np; ++i) cm[i] = st(p, cm[i]);
  }
  double sdt = sqrt(dt), s2nu = sqrt(2.0 * p->nu);
  for (int64_t i = 0; i < np; ++i) {
    if (mask && !mask[i]) continue;
    int32_t e0 = elem[i];
    const orec *r = &rec[e0];
    if (shape) {
      /* statistics at the particle's position at the start of the step */
      double w[3];
      shape_values(m, e0, X[i], Y[i], w);
      const double pt[2] = {X[i], Y[i]};
      elem_record(m, p, stats, wp, gradp, e0, w, pt, &rl);
      r = &rl;
    }
    uint32_t pid = id[i];
    uint32_t q0[4], q1[4];
    draw(seed, pid, step, 0, q0);
    draw(seed, pid, step, 1, q1);
    double xi[6];
    or_box_muller(or_uniform(q0[0]), or_uniform(q0[1]), &xi[0], &xi[1]);
    or_box_muller(or_uniform(q0[2]), or_uniform(q0[3]), &xi[2], &xi[3]);
    or_box_muller(or_uniform(q1[0]), or_uniform(q1[1]), &xi[4], &xi[5]);
    double eta = or_uniform(q1[2]);
    double dW[2] = {sdt * xi[0], sdt * xi[1]};
    double dWp[3] = {sdt * xi[2], sdt * xi[3], sdt * xi[4]};
    double dWo = sdt * xi[5];
    double x0 = X[i], y0 = Y[i];
    double up[3] = {Uu[i], Vv[i], Ww[i]};
    double om = OM[i], psi = PS[i];
    /* eq:Lagrangian-position-exact (nu > 0) / eq:Lagrangian-position-wf (nu = 0) */
    double x = x0 + up[0] * dt + s2nu * dW[0];
    double y = y0 + up[1] * dt + s2nu * dW[1];
    x = st(p, x);
    y = st(p, y);
    /* eq:velocity-prediction / eq:Lagrangian-model */
    double un[3];
    for (int a = 0; a < 3; ++a) {
      double gpa = (a < 2) ? r->gp[a] : 0.0;
      double v = up[a] - gpa * dt + 2.0 * p->nu * r->lap[a] * dt;
      v += s2nu * (r->dU[a][0] * dW[0] + r->dU[a][1] * dW[1]);
      for (int b = 0; b < 3; ++b) v += r->G[a][b] * (up[b] - r->U[b]) * dt;
      v += sqrt(r->C0 * r->eps) * dWp[a];
      un[a] = v;
    }
    /* eq:frequency-model; negative excursions of the explicit step are folded back */
    double omp = om > 0.0 ? om : 0.0;
    double omn = om - p->C3 * r->Om * (om - r->Om) * dt - r->Sw * r->Om * om * dt +
                 sqrt(2.0 * p->C3 * p->C4 * r->Om * r->Om * omp) * dWo;
    if (omn < 0.0) {
      omn = -omn;
      if (cnt) cnt[OR_CNT_OMEGA_CLAMP]++;
    }
    /* eq:IEM, or eq:IECM with the particle's velocity-conditioned mean */
    double psin = psi - dt * r->inv_tm * (psi - (cm ? cm[i] : r->Phi));
    /* tracking: next best element walk with boundary conditions */
    int32_t e = e0, found = -1, nrefl = 0;
    double shx = 0.0, shy = 0.0;
    /* a non-finite position cannot be located: the particle is lost at once */
    int finite_pos = isfinite(x) && isfinite(y);
    for (int it = 0; it < 64 && found < 0 && finite_pos; ++it) {
      if (cnt) cnt[OR_CNT_WALK_STEPS]++;
      double lam[3];
      or_lambdas(m, e, x, y, lam);
      if (lam[0] >= 0.0 && lam[1] >= 0.0 && lam[2] >= 0.0) {
        found = e;
        break;
      }
      int k = 0;
      if (lam[1] < lam[k]) k = 1;
      if (lam[2] < lam[k]) k = 2;
      int32_t nb = m->nbr[3 * e + k];
      if (nb >= 0) {
        e = nb;
        continue;
      }
      int32_t b = -(nb + 1);
      if (m->bt[b] == OR_BC_PERIODIC || m->bt[b] == OR_BC_OUTFLOW) {
        x = st(p, x + m->bs[2 * b]);
        y = st(p, y + m->bs[2 * b + 1]);
        shx += m->bs[2 * b];
        shy += m->bs[2 * b + 1];
        e = m->be[m->bp[b]];
        if (m->bt[b] == OR_BC_OUTFLOW) {
          /* relocated at the inflow with the velocity of the incoming flow;
           * a later wall condition of the same walk acts on it */
          un[0] = p->inflow_u;
          un[1] = 0.0;
          un[2] = 0.0;
          if (cnt) cnt[OR_CNT_OUTFLOW]++;
        } else if (cnt) {
          cnt[OR_CNT_PERIODIC]++;
        }
        continue;
      }
      double xa, ya, xb, yb;
      edge_geom(m, e, k, &xa, &ya, &xb, &yb);
      double dx = xb - xa, dy = yb - ya;
      double t = ((x - xa) * dx + (y - ya) * dy) / (dx * dx + dy * dy);
      int reflect = (t >= 0.0 && t <= 1.0);
      if (!reflect) {
        /* past the end node c of this wall segment.  With the boundary walked
         * with the domain on its left, the corner at c is convex (or straight)
         * when the boundary turns left there: the point, being behind this
         * wall's line, is then outside the domain.  At a reflex corner it is
         * outside only if it is also behind the other wall ending at c. */
        int32_t c = m->en[3 * e + (t < 0.0 ? (k + 1) % 3 : (k + 2) % 3)];
        int32_t w = -1;
        for (int32_t j = m->nwall_off[c]; j < m->nwall_off[c + 1]; ++j)
          if (m->nwall[j] != b) {
            w = m->nwall[j];
            break;
          }
        if (w < 0) {
          reflect = 1; /* the wall ends at a periodic or open boundary */
        } else {
          double wa, wya, wb, wyb;
          edge_geom(m, m->be[w], m->bl[w], &wa, &wya, &wb, &wyb);
          double wdx = wb - wa, wdy = wyb - wya;
          /* incoming and outgoing boundary directions at c */
          double turn = (t < 0.0) ? (wdx * dy - wdy * dx) : (dx * wdy - dy * wdx);
          double behind_w = (x - wa) * wdy - (y - wya) * wdx;
          if (turn >= 0.0 || behind_w > 0.0) reflect = 1;
        }
      }
      if (!reflect) {
        /* in the domain beyond a concave corner: fall-back of Fig. corner */
        int32_t f = search_patch(m, e0, x, y);
        if (f < 0) f = search_patch(m, e, x, y);
        if (f >= 0) {
          if (cnt) cnt[OR_CNT_FALLBACK]++;
          found = f;
          break;
        }
        if (cnt) cnt[OR_CNT_BRUTE]++;
        f = or_locate_brute(m, x, y);
        if (f >= 0) {
          found = f;
          break;
        }
        reflect = 1;
      }
      if (!reflect || nrefl >= 8) break;
      /* perfect reflection across the wall line */
      double len = sqrt(dx * dx + dy * dy);
      double nx = dy / len, ny = -dx / len;
      double dist = (x - xa) * nx + (y - ya) * ny;
      x = st(p, x - 2.0 * dist * nx);
      y = st(p, y - 2.0 * dist * ny);
      if (cnt) cnt[OR_CNT_REFLECT]++;
      if (m->bt[b] == OR_BC_SLIP) {
        double un_n = un[0] * nx + un[1] * ny;
        un[0] = un[0] - 2.0 * un_n * nx;
        un[1] = un[1] - 2.0 * un_n * ny;
      } else if (m->bt[b] == OR_BC_WALLFN) {
        /* the element's vertex off the edge is the first gridpoint from the wall */
        const int32_t c = m->en[3 * e + k];
        wall_fn_at(p, m, stats, gradp, c, xa, ya, xb, yb, &un[0], &un[1], &un[2], &omn);
      } else {
        noslip(p, r, nx, ny, seed, pid, step, nrefl, &un[0], &un[1], &un[2], &omn, cnt);
      }
      nrefl++;
    }
    if (found < 0) {
      int32_t f = finite_pos ? search_patch(m, e0, x, y) : -1;
      if (f < 0 && finite_pos) {
        if (cnt) cnt[OR_CNT_BRUTE]++;
        f = or_locate_brute(m, x, y);
      }
      if (f >= 0) {
        found = f;
      } else {
        /* lost: the particle keeps its old position and host */
        if (cnt) cnt[OR_CNT_LOST]++;
        lost++;
        x = x0;
        y = y0;
        found = e0;
      }
    }
    /* no-slip trajectory (b): eq:fw and eq:exp-wall-condition */
    if (p->wall_b && p->nu > 0.0 && nrefl == 0) {
      int32_t best = -1;
      double bd = 0.0;
      for (int32_t j = m->w_off[found]; j < m->w_off[found + 1]; ++j) {
        int32_t b = m->w_list[j];
        double xa, ya, xb, yb;
        edge_geom(m, m->be[b], m->bl[b], &xa, &ya, &xb, &yb);
        double dx = xb - xa, dy = yb - ya;
        double t = ((x - xa) * dx + (y - ya) * dy) / (dx * dx + dy * dy);
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
        double ex = x - (xa + t * dx), ey = y - (ya + t * dy);
        double d2 = ex * ex + ey * ey;
        if (best < 0 || d2 < bd) {
          best = b;
          bd = d2;
        }
      }
      if (best >= 0) {
        double xa, ya, xb, yb;
        edge_geom(m, m->be[best], m->bl[best], &xa, &ya, &xb, &yb);
        double dx = xb - xa, dy = yb - ya;
        double len = sqrt(dx * dx + dy * dy);
        double nx = dy / len, ny = -dx / len;
        double d1 = -((x - xa) * nx + (y - ya) * ny);
        double d0 = -((x0 + shx - xa) * nx + (y0 + shy - ya) * ny);
        if (d0 > 0.0 && d1 >= 0.0) {
          double fw = exp(-d0 * d1 / (p->nu * dt));
          if (eta < fw) {
            if (cnt) cnt[OR_CNT_NOSLIP_B]++;
            noslip(p, r, nx, ny, seed, pid, step, 8, &un[0], &un[1], &un[2], &omn, cnt);
          }
        }
      }
    }
    /* continuous scalar source */
    if (p->src_r > 0.0) {
      double ddx = x - p->src_x, ddy = y - p->src_y;
      if (ddx * ddx + ddy * ddy <= p->src_r * p->src_r) psin = 1.0;
    }
    X[i] = x;
    Y[i] = y;
    Uu[i] = st(p, un[0]);
    Vv[i] = st(p, un[1]);
    Ww[i] = st(p, un[2]);
    OM[i] = st(p, omn);
    PS[i] = st(p, psin);
    elem[i] = found;
  }
  free(rec);
  free(cm);
  return lost;
}
