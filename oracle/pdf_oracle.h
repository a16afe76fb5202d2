/*
 * Plain, slow, single-threaded FP64 reference ("oracle") for the particle hot
 * path of the stand-alone PDF method on triangle grids (Bakosi 2008).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this library; it exists so that tests, the smoke check and the CPU
 * timing leg of the benchmark can compare the GPU results against a direct
 * transcription of the method.  It shares no source with the GPU library.
 *
 * Every routine follows the paper's equations in the paper's order; the
 * citations are by chapter/section and equation label.  Parity status of each
 * routine is listed in the pin table of the tests (tests/test_oracle_*.py).
 */
#ifndef PDF_ORACLE_H
#define PDF_ORACLE_H
#include <stdint.h>

#define OR_NSTAT 25 /* nodal statistics per node, see or_estimate() */

/* boundary types */
#define OR_BC_PERIODIC 1
#define OR_BC_SLIP 2
#define OR_BC_NOSLIP 3
#define OR_BC_WALLFN 4 /* wall treated by the wall functions of eq:wall-normal-velocity to eq:wall-omega */
/* outflow edge, paired with an inflow edge (of type OR_BC_PERIODIC): a
 * particle leaving through it is relocated at the inflow with its
 * cross-stream position kept (the pair's translation) and its velocity set to
 * (inflow_u, 0, 0) (Ch.6, cylinder flow, Sec. Results: its boundary
 * conditions) when it crosses, so that a wall condition later in the same
 * walk acts on that velocity; the other properties are kept.  Leaving through
 * the inflow edge is periodic. */
#define OR_BC_OUTFLOW 5

typedef struct or_params {
  int32_t model;        /* 0 = simplified Langevin (eq:wall-GandC), 1 = generalized Langevin (eq:GandC) */
  int32_t wp_source;    /* GLM: 0 = nodal field given, 1 = local right-hand side of eq:elliptic-relaxation-Lagrangian */
  int32_t omega_source; /* 1 = S_omega of eq:frequency-source, 0 = S_omega = 0 */
  int32_t tm_mode;      /* 0: 1/t_m = C_phi <omega>/2 ; 1: t_m = max(k/eps, C_T sqrt(nu/eps));
                           2: eq:micromixing-timescale-canyon (source-aware) */
  int32_t frozen;       /* 1: statistics are not fed back (fixed nodal fields) */
  int32_t wall_b;       /* 1: apply the no-slip trajectory (b) test of eq:fw */
  int32_t store_fp32;   /* 1: particle state is rounded to binary32 wherever the GPU stores it */
  int32_t stats_mode;   /* 0 ELEM: element average of nodal values at particles, element -> node
                           averages; 1 SHAPE: shape-function (eq:approximation) values at the
                           particle, N_j-weighted particle sums at the nodes */
  int32_t min_ppe;      /* particle redistribution (App. D): minimum particles per element; 0 = off */
  int32_t mix_model;    /* 0 IEM (eq:IEM), 1 IECM (eq:IECM) */
  int32_t cond_nu, cond_nv, cond_nw; /* IECM binning structure (n_u x n_v x n_w) */
  int32_t cond_min;     /* IECM: fewest particles a subgroup may keep (the adaptive stop) */
  double C0, C1, C2, C3, C4, CT, CL, Ceta, Cv, gamma5, Cw1, Cw2, Cphi, nu, k_floor;
  double src_x, src_y, src_r;
  double Cs, Ct;        /* constants of eq:micromixing-timescale-canyon */
  double nu_wall;       /* kinematic viscosity of the log law eq:Ue (wall-function walls) */
  double inflow_u;      /* streamwise velocity given to particles relocated at the inflow */
} or_params;

typedef struct or_seedspec {
  int32_t ppe;
  int32_t psi_mode; /* 0 zero, 1 step (psi=1 for x<a), 2 gaussian in x (a, b=sigma), 3 bernoulli(1/2), 4 disc (a,b,c=r) */
  uint64_t seed;
  double a, b, c;
  const double *U0;  /* [3][nn] */
  const double *R0;  /* [6][nn]  11,22,33,12,13,23 */
  const double *Om0; /* [nn] */
} or_seedspec;

typedef struct or_mesh or_mesh;

/* counters (index) */
enum { OR_CNT_WALK_STEPS = 0, OR_CNT_FALLBACK, OR_CNT_BRUTE, OR_CNT_LOST, OR_CNT_REFLECT,
       OR_CNT_PERIODIC, OR_CNT_NOSLIP_B, OR_CNT_OMEGA_CLAMP, OR_CNT_GAMMA_FAIL, OR_CNT_EMPTY_NODE,
       OR_CNT_REDIST, OR_CNT_OUTFLOW, OR_CNT_N };

#ifdef __cplusplus
extern "C" {
#endif
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_uniform(uint32_t r);
void or_box_muller(double u1, double u2, double *z0, double *z1);
double or_gamma(double shape, double scale, uint64_t seed, uint32_t id, uint32_t step,
                uint32_t subbase, int32_t *fail);

or_mesh *or_mesh_new(int32_t nn, int32_t ne, int32_t nb, const double *xy, const int32_t *en,
                     const int32_t *nbr, const int32_t *be, const int32_t *bl, const int32_t *bt,
                     const int32_t *bp, const double *bs, const int32_t *master);
void or_mesh_free(or_mesh *m);
int32_t or_locate_brute(const or_mesh *m, double x, double y);
void or_lambdas(const or_mesh *m, int32_t e, double x, double y, double lam[3]);

void or_seed(const or_mesh *m, const or_params *p, const or_seedspec *s, double *state /*[7][np]*/,
             int32_t *elem, uint32_t *id);

void or_estimate(const or_mesh *m, const or_params *p, int64_t np, const double *state,
                 const int32_t *elem, const double *prev, double *stats /*[OR_NSTAT][nn]*/,
                 double *elem_out /*[16][ne] or NULL*/, uint64_t *cnt);

void or_derivatives(const or_mesh *m, double *stats /*[OR_NSTAT][nn]*/);
void or_local_wp(const or_mesh *m, const or_params *p, const double *stats, double *wp /*[9][nn]*/);

/* Time step of eq:CFL from the nodal mean velocity: c_cfl times the smallest,
 * over master nodes with a non-zero in-plane mean velocity, of sqrt(A_n) /
 * |(<U>, <V>)| with A_n the average area of the elements around node n;
 * dt_max when that is larger or no node moves. */
double or_cfl_dt(const or_mesh *m, const double *stats, double c_cfl, double dt_max);

/* Wall-function condition on a particle reflected at a wall-function edge
 * (eq:wall-normal-velocity, eq:particle-wallcondition-wf with eq:alpha,
 * eq:hatu, eq:Ue, eq:friction-velocity, and eq:wall-omega).  The edge runs
 * from (xa, ya) to (xb, yb) with the domain on its left; the statistics at y_p
 * are the nodal statistics stats[f*nn + node] (and gradp[f*nn + node], may be
 * NULL) at `node`, the element's vertex off the edge, at (xc, yc).  u, v, w,
 * om: the incident velocity and frequency, replaced by the reflected ones. */
void or_wall_function(const or_params *p, int32_t nn, const double *stats, const double *gradp, int32_t node,
                      double xa, double ya, double xb, double yb, double xc, double yc, double *u, double *v,
                      double *w, double *om);

/* Velocity-conditioned scalar mean <phi|V> of every particle (Sec. Estimation
 * of the velocity-conditioned scalar mean, App. B): the mean scalar of its
 * subgroup in its host element after the sort-and-divide binning. */
void or_cond_means(const or_mesh *m, const or_params *p, int64_t np, const double *state,
                   const int32_t *elem, const uint32_t *id, double *cm /*[np]*/);

/* Particle redistribution (App. D, the improved algorithm) before step `step`:
 * elements below p->min_ppe particles receive particles from the most
 * populated ones; returns the number of particles moved. */
int64_t or_redistribute(const or_mesh *m, const or_params *p, int64_t np, double *state, int32_t *elem,
                        const uint32_t *id, uint64_t seed, uint32_t step);

int32_t or_step(const or_mesh *m, const or_params *p, const double *stats, const double *wp,
                const double *gradp, int64_t np, double *state, int32_t *elem, const uint32_t *id,
                uint64_t seed, uint32_t step, double dt, const uint8_t *mask, uint64_t *cnt);
#ifdef __cplusplus
}
#endif
#endif
