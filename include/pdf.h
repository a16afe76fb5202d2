/*
 * pdf.h -- C ABI of the MI355X (gfx950) particle hot path of the stand-alone
 * PDF method for turbulent velocity, frequency and passive-scalar transport on
 * unstructured triangle grids (J. Bakosi, "PDF modeling of turbulent flows on
 * unstructured grids", 2008).
 *
 * The problem, as the dissertation states it (Ch.3, Introduction):
 *   given an unstructured triangle grid, model constants, the nodal Eulerian
 *   inputs of the particle equations and an initial particle population,
 *   advance the particle SDEs by explicit Euler-Maruyama steps while tracking
 *   every particle through the grid, and estimate Eulerian statistics at the
 *   grid nodes from the particles.
 *
 * Conventions shared by every entry point
 *   - Every function returns pdf_status; PDF_OK == 0.  No C++ exception and no
 *     abort crosses this interface.  pdf_last_error() returns the context's
 *     last message.
 *   - Host arrays passed in are borrowed for the duration of the call and
 *     copied; the library never keeps a caller pointer.
 *   - All device work is enqueued on the hipStream_t given to pdf_init_mesh().
 *     Calls that return data into host memory synchronize that stream; all
 *     others are asynchronous.  A context belongs to one host thread.
 *   - Arrays are field-major ("structure of arrays"): field f of item i is at
 *     [f * n_items + i].
 *   - Particle identifiers are id = e * ppe + j for the j-th particle seeded in
 *     element e (caller numbering); the counter-based random numbers are a pure
 *     function of (seed, id, step), so results do not depend on launch shape or
 *     particle storage order.
 */
#ifndef PDF_H
#define PDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdf_ctx pdf_ctx;

typedef enum pdf_status {
  PDF_OK = 0,
  PDF_E_INVALID_ARG = 1,   /* a pointer, size or enum is out of range */
  PDF_E_BAD_MESH = 2,      /* the mesh fails a consistency check (orientation, neighbours, periodic pairs) */
  PDF_E_OOM = 3,           /* a device allocation failed */
  PDF_E_DEVICE = 4,        /* a HIP call failed (message in pdf_last_error) */
  PDF_E_STATE = 5,         /* wrong call order (e.g. advance before seeding) */
  PDF_E_LOST_PARTICLE = 6, /* a particle was found by neither the walk, the fall-back nor brute force */
  PDF_E_NUMERIC = 7        /* non-finite particle state detected */
} pdf_status;

enum { PDF_FP64 = 0, PDF_FP32 = 1 };                          /* particle-state precision */
/* boundary-edge types.  PDF_BC_OUTFLOW: an outflow edge paired (bedge_partner,
 * bedge_shift) with an inflow edge of type PDF_BC_PERIODIC; a particle leaving
 * through it is relocated at the inflow with its cross-stream position kept
 * (the pair's translation) and its velocity set to (inflow_u, 0, 0) (Ch.6,
 * cylinder flow, Sec. Results: its boundary conditions) as it crosses, so
 * that a wall condition later in the same step's walk acts on that velocity;
 * its frequency and scalar are kept, and leaving through the inflow edge is
 * periodic.  The
 * nodes of the pair stay identified through node_master. */
enum { PDF_BC_PERIODIC = 1, PDF_BC_SLIP = 2, PDF_BC_NOSLIP = 3, PDF_BC_WALLFN = 4, PDF_BC_OUTFLOW = 5 };
enum { PDF_MODEL_SLM = 0, PDF_MODEL_GLM = 1 };                /* eq:wall-GandC / eq:GandC */
enum { PDF_WP_INPUT = 0, PDF_WP_LOCAL = 1, PDF_WP_ELLIPTIC = 2 };                  /* source of the tensor wp_ij (GLM) */
enum { PDF_TM_CPHI = 0, PDF_TM_KEPS = 1, PDF_TM_SOURCE = 2 }; /* micromixing time scale */
enum { PDF_MIX_IEM = 0, PDF_MIX_IECM = 1 };                  /* micromixing model */
enum { PDF_PSI_ZERO = 0, PDF_PSI_STEP_X = 1, PDF_PSI_GAUSS_X = 2, PDF_PSI_BERNOULLI = 3,
       PDF_PSI_DISC = 4 };                                    /* scalar initial conditions */
enum { PDF_FIELD_STATS = 0, PDF_FIELD_WP = 1, PDF_FIELD_GRADP = 2, PDF_FIELD_PRESSURE = 3 }; /* nodal field ids */
enum { PDF_STATS_ELEM = 0, PDF_STATS_SHAPE = 1 };             /* statistics at particles and nodes */

#define PDF_NSTAT 25     /* nodal statistics per node, see pdf_estimate_stats */
#define PDF_NELEMSTAT 16 /* element statistics per element */
#define PDF_NCOUNTERS 16

/* counter indices (pdf_get_counters) */
enum {
  PDF_CNT_WALK_STEPS = 0, PDF_CNT_FALLBACK = 1, PDF_CNT_BRUTE = 2, PDF_CNT_LOST = 3,
  PDF_CNT_REFLECT = 4, PDF_CNT_PERIODIC = 5, PDF_CNT_NOSLIP_B = 6, PDF_CNT_OMEGA_CLAMP = 7,
  PDF_CNT_GAMMA_FAIL = 8, PDF_CNT_EMPTY_NODE = 9, PDF_CNT_NONFINITE = 10, PDF_CNT_STEPS = 11,
  PDF_CNT_REDIST = 12, /* particles moved by the redistribution */
  PDF_CNT_ELL_ITERS = 13, /* conjugate-gradient iterations of the elliptic relaxation */
  PDF_CNT_PROJ_ITERS = 14, /* conjugate-gradient iterations of the pressure projection */
  PDF_CNT_OUTFLOW = 15     /* particles relocated at the inflow (PDF_BC_OUTFLOW) */
};

/* Device allocator hook.  alloc returns device memory of at least `bytes`
 * bytes (256-byte aligned) or NULL; free releases it.  Passing NULL to
 * pdf_init_mesh selects hipMalloc/hipFree. */
typedef struct pdf_allocator {
  void *(*alloc)(size_t bytes, void *user);
  void (*free)(void *ptr, void *user);
  void *user;
} pdf_allocator;

/* Unstructured triangle grid (Ch.3, Sec. Particle tracking and Sec. Estimation
 * of Eulerian statistics: elements, the elements surrounding each element with
 * tagged boundary neighbours, and the grid nodes).  Host pointers.
 *   node_xy       2*n_nodes doubles, interleaved (x0,y0,x1,y1,...)
 *   elem_nodes    3*n_elems node indices per element, counter-clockwise
 *   elem_nbr      3*n_elems: element across the edge opposite local node k, or
 *                 -(b+1) for boundary edge b
 *   bedge_elem/local  element and local edge index of boundary edge b
 *   bedge_type    PDF_BC_* per boundary edge (PDF_BC_WALLFN: a wall with the
 *                 wall-function particle condition, see pdf_model_params.nu_wall)
 *   bedge_partner periodic partner edge, or -1
 *   bedge_shift   2*n_bedges: translation added to a particle crossing edge b
 *                 (periodic edges only)
 *   node_master   periodic identification: statistics of node n are those of
 *                 node node_master[n] (n itself when not periodic)
 * Errors: PDF_E_BAD_MESH if an element has non-positive area, elem_nbr is not
 * symmetric, a periodic partner is not mutual or a master is not its own master. */
typedef struct pdf_mesh_desc {
  int32_t n_nodes, n_elems, n_bedges, pad;
  const double *node_xy;
  const int32_t *elem_nodes;
  const int32_t *elem_nbr;
  const int32_t *bedge_elem;
  const int32_t *bedge_local;
  const int32_t *bedge_type;
  const int32_t *bedge_partner;
  const double *bedge_shift;
  const int32_t *node_master;
} pdf_mesh_desc;

/* Model constants and switches.  Constants as in the paper's tables
 * (Ch.4 tab:fd-constants, Ch.5 tab:constants); nu is the kinematic viscosity
 * (nu = 0 selects the inviscid position equation eq:Lagrangian-position-wf).
 *   model        PDF_MODEL_SLM: G_ij = -(1/2 + 3/4 C0)<omega> delta_ij, C0 constant
 *                PDF_MODEL_GLM: G_ij and C0 from wp_ij by eq:GandC
 *   wp_source    GLM only: PDF_WP_INPUT (nodal field set by pdf_set_nodal_field)
 *                or PDF_WP_LOCAL (right-hand side of eq:elliptic-relaxation-Lagrangian
 *                evaluated at the nodes from the estimated statistics)
 *                or PDF_WP_ELLIPTIC: eq:elliptic-relaxation-Lagrangian solved every step
 *                with linear finite elements (Ch.3, Sec. Solution of the Eulerian
 *                equations): per component (M + L_ij^2 K) wp = M f with M the consistent
 *                mass and K the stiffness matrix, f the local right-hand side, L_ij from
 *                eq:L (element averages of k and eps; C_xi,ij = 1 + 1.3 n_i n_j of eq:Cxi
 *                with n the outward normal of the no-slip wall edge closest to the
 *                element), wp_ij = -4.5 eps n_i n_j at no-slip wall nodes; conjugate
 *                gradients from the previous solution (preconditioner: ell_precond) until
 *                the preconditioned residual of every component is below ell_tol times
 *                that of its right-hand side, at most ell_maxit iterations (the call then
 *                waits for the stream every 8 iterations)
 *   omega_source 1: S_omega of eq:frequency-source; 0: S_omega = 0
 *   tm_mode      PDF_TM_CPHI: 1/t_m = C_phi <omega>/2; PDF_TM_KEPS: t_m = max(k/eps, C_T sqrt(nu/eps));
 *                PDF_TM_SOURCE: eq:micromixing-timescale-canyon, t_m = min(C_s (r0^2/eps)^(1/3)
 *                + C_t d/U_c, max(k/eps, C_T sqrt(nu/eps))) with r0 = src_r, d the distance
 *                from (src_x, src_y) to the element centroid (PDF_STATS_ELEM) or the
 *                particle (PDF_STATS_SHAPE) and U_c = |<U>| there (the first argument
 *                drops out where U_c = 0)
 *   frozen       1: element records always come from the PDF_FIELD_STATS field;
 *                the estimator still runs but is not fed back
 *   wall_b       1: apply the no-slip trajectory (b) condition of eq:fw (nu > 0)
 *   reorder_every  particles are re-sorted by host element every R steps (0: never)
 *   stats_mode   PDF_STATS_ELEM: a particle sees the element average of the nodal
 *                statistics of its host, and node values are averages of element
 *                means and central moments over the surrounding elements (Ch.3,
 *                Fig. mesh-particles); PDF_STATS_SHAPE: a particle sees the nodal
 *                statistics interpolated at its position by the shape functions of
 *                eq:approximation, and node j's values are the N^j(x_p)-weighted
 *                means and central moments of the particles in the elements around j
 *   min_ppe      particle redistribution (App. D, improved algorithm) at the start of
 *                every step: elements with fewer than min_ppe particles (0: off; at
 *                most 64) receive particles from the most populated ones, as copies
 *                of their residents
 *   mix_model    PDF_MIX_IEM: psi relaxes toward <phi> (eq:IEM); PDF_MIX_IECM: toward the
 *                velocity-conditioned mean <phi|V> (eq:IECM), estimated at the start of
 *                each step in every element by the sort-and-divide binning of Ch.3,
 *                Sec. Estimation of the velocity-conditioned scalar mean and App. B:
 *                the element's particles (from increasing id) are sorted by U and
 *                divided into cond_nu groups, each by V into cond_nv, each by W into
 *                cond_nw (ties by id; group g of P over n particles holds the positions
 *                j with P*j/n = g; a direction with one interval is skipped); a level is
 *                taken only while every subgroup keeps at least cond_min particles;
 *                <phi|V> is the mean psi of the particle's final subgroup
 *   cond_nu, cond_nv, cond_nw  binning structure, each 1..16 (the paper: 5 x 5 x 5)
 *   cond_min     fewest particles per subgroup, 1..64 (the paper's example: 2)
 *   src_x,src_y,src_r  continuous scalar source disc: psi = 1 inside (r <= 0: none)
 *   Cs, Ct       constants of eq:micromixing-timescale-canyon (tab:constants: 0.02, 0.7)
 *   proj         1: the stabilized mean-pressure projection every step (Ch.3, Sec. Solution
 *                of the Eulerian equations; PDF_STATS_ELEM, statistics fed back): with
 *                P = x.G + P' (G the PDF_FIELD_GRADP input, zero if unset), after the
 *                velocity prediction and its estimate <U>*, K dP = -(d + Cp K P')/dt
 *                (eq:pressure-projection-smooth in weak form: K the linear-element
 *                stiffness matrix over the master nodes, d_a = sum_e A_e/3 div_e <U>*,
 *                the right-hand side's mean removed, dP of zero mean; at walls the
 *                Neumann datum g of eq:wall-pressure-condition, nu lap<U_i> n_i -
 *                d<u_i u_j>/dx_j n_i, less <U_j> d<U_i>/dx_j n_i at PDF_BC_WALLFN
 *                edges, from the predicted statistics, enters as the boundary
 *                integrals (Cp/dt) B(g_old - G.n) + B(g_new - g_old), B(q)_a the
 *                integral of N_a q over the wall edges and g_old the datum P
 *                satisfies, G.n before the first step), solved by preconditioned conjugate gradients to proj_tol
 *                (preconditioned residual against the right-hand side's) in at most
 *                proj_maxit iterations (the call waits for the stream every 8);
 *                then every particle's velocity changes by -dt grad dP of its element
 *                (eq:velocity-correction), P' += dP, and the next prediction uses G plus
 *                the node average of the element gradients of P' (PDF_FIELD_GRADP then
 *                returns that sum, PDF_FIELD_PRESSURE returns P')
 *   proj_precond preconditioner of the projection: 0 Jacobi (the paper's), 1 one V-cycle of
 *                a smoothed-aggregation multigrid hierarchy of K (built once by
 *                pdf_init_mesh on the host; Jacobi smoothing, Galerkin coarse levels,
 *                a dense coarsest solve; PDF_E_NUMERIC if it cannot be built)
 *   ell_precond  preconditioner of the elliptic relaxation: 0 Jacobi (the paper's), 1 one
 *                V-cycle of a plain-aggregation multigrid hierarchy (aggregates built once by
 *                pdf_init_mesh from the stiffness matrix over the free master nodes; every
 *                solve sums the matrix entries over pairs of aggregates for the coarser
 *                levels, one Jacobi step on the diagonal a_ii + (1/2) sum_{j!=i} |a_ij|
 *                before and after each coarse correction, 8 such sweeps on the last level
 *                of at most 128 rows; PDF_E_NUMERIC if it cannot be built)
 *   Cp           stabilization constant of eq:pressure-projection-smooth (the paper: 1e-3)
 *   nu_wall      kinematic viscosity of the log law eq:Ue at PDF_BC_WALLFN edges (> 0 when
 *                the mesh has such edges).  A particle reflected at such an edge gets the
 *                wall-function condition: in the edge's frame (tangent along the edge,
 *                normal into the domain) V_R = -V_I (eq:wall-normal-velocity),
 *                U_R = U_I + alpha V_I (eq:particle-wallcondition-wf, alpha from eq:alpha,
 *                eq:hatu, eq:Ue, eq:friction-velocity with C_mu = 0.09, kappa = 0.41,
 *                E = 8.5; alpha = 0 where U_e <= 0), omega_R by eq:wall-omega (unchanged where
 *                <omega> <= 0), the spanwise velocity kept.  The statistics at y_p are the
 *                current nodal statistics at the wall element's vertex off the edge; y_p is
 *                that vertex's distance to the edge's line.  Wall functions replace the
 *                viscous terms of the particle equations (eq:Lagrangian-position-wf,
 *                eq:Lagrangian-model-wf): a mesh with PDF_BC_WALLFN edges needs nu = 0
 *                (PDF_E_INVALID_ARG otherwise).
 *   inflow_u     streamwise velocity given to particles relocated at the inflow when they
 *                leave through a PDF_BC_OUTFLOW edge (finite; PDF_E_INVALID_ARG otherwise;
 *                unused without such edges) */
typedef struct pdf_model_params {
  int32_t model, wp_source, omega_source, tm_mode, frozen, wall_b, reorder_every, stats_mode;
  int32_t min_ppe, mix_model, cond_nu, cond_nv, cond_nw, cond_min, ell_maxit, proj, proj_maxit, proj_precond;
  int32_t ell_precond;
  double C0, C1, C2, C3, C4, CT, CL, Ceta, Cv, gamma5, Cw1, Cw2, Cphi, nu, k_floor;
  double src_x, src_y, src_r, Cs, Ct, nu_wall, ell_tol, Cp, proj_tol;
  double inflow_u;  /* streamwise velocity of particles relocated at the inflow (PDF_BC_OUTFLOW) */
} pdf_model_params;

/* Initial particle population (Ch.3, Sec. Particle-number control): ppe
 * particles uniformly distributed in every element; velocity Gaussian with the
 * nodal mean U0 and Reynolds stress R0 interpolated linearly at the particle;
 * frequency Gamma(1/C4, C4*Om0); scalar by psi_mode with parameters a, b, c
 * (STEP_X: psi = [x < a]; GAUSS_X: exp(-(x-a)^2/(2 b^2)); BERNOULLI: 0/1 with
 * probability 1/2; DISC: psi = [|x-(a,b)| <= c]).  Host pointers:
 *   U0 [3][n_nodes], R0 [6][n_nodes] (11,22,33,12,13,23), Om0 [n_nodes]. */
typedef struct pdf_seed_desc {
  int32_t ppe, psi_mode;
  uint64_t seed;
  double a, b, c;
  const double *U0, *R0, *Om0;
} pdf_seed_desc;

/* Create a context: validate and upload the mesh, derive the linked lists
 * (elements surrounding nodes, wall edges near each element, the ring of
 * masters around each master) and shape-function derivatives (Ch.3, Sec.
 * Derivatives), with the weights that apply the average over a master's
 * elements of their gradients as a sum over its ring (formed on the device;
 * PDF_E_DEVICE if that fails).  precision is PDF_FP64 or PDF_FP32;
 * hip_stream is a hipStream_t (NULL: the null stream); alloc may be NULL.
 * On success *out owns all device memory until pdf_destroy.  On failure *out
 * is NULL when no context was formed (invalid arguments, no current device);
 * otherwise it holds the failed context so that pdf_last_error gives the
 * reason, and the caller destroys it. */
pdf_status pdf_init_mesh(const pdf_mesh_desc *mesh, const pdf_model_params *params,
                         int32_t precision, const pdf_allocator *alloc, void *hip_stream,
                         pdf_ctx **out);

/* Set a nodal input field from host (on_device = 0) or device (1) memory:
 *   PDF_FIELD_STATS [PDF_NSTAT][n_nodes]  nodal statistics (frozen mode, restart)
 *   PDF_FIELD_WP    [9][n_nodes]          wp_ij row-major (GLM with PDF_WP_INPUT)
 *   PDF_FIELD_GRADP [2][n_nodes]          mean-pressure gradient / rho
 *                                         (eq:velocity-prediction; default 0) */
pdf_status pdf_set_nodal_field(pdf_ctx *ctx, int32_t field, const double *data, int32_t on_device);

/* Copy a nodal field out, same ids and layouts: PDF_FIELD_STATS the latest
 * statistics, PDF_FIELD_WP the tensor wp_ij the last step used (the solution
 * of the elliptic relaxation with PDF_WP_ELLIPTIC), PDF_FIELD_GRADP the
 * mean-pressure gradient (with the projection: the one the next step uses),
 * PDF_FIELD_PRESSURE [1][n_nodes] the solved pressure P' (projection only).  on_device = 0: host memory (synchronizes); 1:
 * device memory (asynchronous). */
pdf_status pdf_get_nodal_field(pdf_ctx *ctx, int32_t field, double *data, int32_t on_device);

/* Seed n_elems*ppe particles (ids e*ppe+j) and estimate the initial statistics. */
pdf_status pdf_seed_particles(pdf_ctx *ctx, const pdf_seed_desc *seed);

/* Advance nsteps explicit Euler-Maruyama steps of size dt (Ch.3, Sec.
 * Timestepping).  Each step: element-average statistics from the nodal fields
 * (loop (ii) of Table tab:loops), one fused particle kernel (noise, SDEs
 * eq:Lagrangian-position-exact/-wf, eq:Lagrangian-model, eq:frequency-model,
 * eq:IEM, tracking eq:element-test with boundary conditions, accumulation of
 * element sums), then the two-pass nodal estimator and its derivatives.
 * Asynchronous; lost particles are reported through the counters. */
pdf_status pdf_advance(pdf_ctx *ctx, int32_t nsteps, double dt);

/* As pdf_advance, with each step's size chosen by the condition eq:CFL from
 * the statistics current at the start of that step (Ch.3, Sec.
 * Timestepping):
 *   dt = min(dt_max, c_cfl * min_n sqrt(A_n) / |<U>_n|),
 * n over the master nodes, A_n the mean area of the elements around node n,
 * |<U>_n| the magnitude of the in-plane mean velocity (<U>,<V>); nodes where
 * it is zero (or not a number) do not bound the step, and with none left
 * dt = dt_max.  The step size is formed and consumed on the device (no host
 * round trip per step).  c_cfl > 0 and dt_max > 0, both finite
 * (PDF_E_INVALID_ARG otherwise).  t_advanced (host, may be NULL) receives the
 * sum of the nsteps step sizes; when it is given the call waits for the
 * stream, otherwise it is asynchronous. */
pdf_status pdf_advance_cfl(pdf_ctx *ctx, int32_t nsteps, double c_cfl, double dt_max, double *t_advanced);

/* Copy the latest nodal statistics (and optionally element statistics) out.
 * nodal [PDF_NSTAT][n_nodes]: 0-2 <U>,<V>,<W>; 3 <omega>; 4 <phi>; 5-10 <u_i u_j>
 * (11,22,33,12,13,23); 11 <phi'^2>; 12-14 <u_i phi'>; 15-20 d<U_i>/dx, d<U_i>/dy
 * for i = U,V,W; 21-23 Laplacian of <U_i>; 24 particles in the non-empty
 * surrounding elements (PDF_STATS_SHAPE: the sum of the node's shape-function
 * weights over those particles).
 * elem [PDF_NELEMSTAT][n_elems] or NULL: count, 5 means (u,v,w,omega,psi),
 * 10 central moments (uu,vv,ww,uv,uw,vw,psipsi,upsi,vpsi,wpsi), 1/N normalised;
 * PDF_STATS_ELEM only (PDF_E_STATE in PDF_STATS_SHAPE, which forms no element
 * statistics).
 * on_device = 0: host buffers (synchronizes); 1: device buffers (asynchronous). */
pdf_status pdf_estimate_stats(pdf_ctx *ctx, double *nodal, double *elem, int32_t on_device);

/* Number of particles currently held. */
pdf_status pdf_num_particles(pdf_ctx *ctx, int64_t *n);

/* Copy the particle state to host memory in storage order:
 * state [7][n] = x, y, u, v, w, omega, psi (as double), elem [n], id [n]. */
pdf_status pdf_get_particles(pdf_ctx *ctx, double *state, int32_t *elem, uint32_t *id);

/* Replace the particle state from host memory (same layout; n particles).
 * Values are rounded to the context precision.  Statistics are re-estimated.
 * PDF_E_INVALID_ARG for n < 1 (a context always holds particles once seeded)
 * or an element index outside [0, n_elems); the state is then unchanged. */
pdf_status pdf_set_particles(pdf_ctx *ctx, int64_t n, const double *state, const int32_t *elem,
                             const uint32_t *id);

/* Read (and optionally reset) the device counters PDF_CNT_*; synchronizes. */
pdf_status pdf_get_counters(pdf_ctx *ctx, uint64_t *out, int32_t n, int32_t reset);

/* Per-kernel timing of the last pdf_advance call, measured with HIP events on
 * the context stream: out[0] element records, out[1] particle kernel,
 * out[2] estimator, out[3] reorder, out[4] the work at the start of a step
 * (time step of eq:CFL, redistribution, conditioned means) (milliseconds,
 * summed over its steps; n <= 5 values are written).
 * Timing is recorded only while enabled (pdf_enable_timing). */
pdf_status pdf_enable_timing(pdf_ctx *ctx, int32_t on);
pdf_status pdf_get_timing(pdf_ctx *ctx, double *out_ms, int32_t n);

const char *pdf_last_error(const pdf_ctx *ctx);
void pdf_destroy(pdf_ctx *ctx);

/* ------------------------------------------------------------------------
 * Learned denoiser of the nodal statistics (not part of the dissertation's
 * method: it addresses the statistical noise that makes the method need 80-500
 * particles per element, Ch.4 particle-number study).  A 4-layer perceptron
 * 48 -> H -> H -> H -> 8 with GELU activations, BF16 weights and activations
 * and FP32 accumulation on the matrix cores, predicts a correction of 8 nodal
 * statistics (<U>, <V>, <phi>, <uu>, <vv>, <uv>, <phi'^2>, <omega>) from 48
 * features of the plain estimate (for each statistic: node value, mean, std,
 * min and max over the node and its neighbours, gradient magnitude).  The
 * plain estimator stays as the fallback: a correction larger than tau times
 * the plain standard error at the node (times a per-statistic calibration,
 * pdf_denoiser_set_fallback) is rejected.
 *
 * Parameter vector (float32, PDF_DN_NPARAM(H) values): W1 [48][H], b1 [H],
 * W2 [H][H], b2 [H], W3 [H][H], b3 [H], W4 [H][8], b4 [8]; y = x W + b.
 * ------------------------------------------------------------------------ */
typedef struct pdf_denoiser pdf_denoiser;
#define PDF_DN_NIN 48
#define PDF_DN_NOUT 8
#define PDF_DN_NPARAM(H) (48 * (H) + (H) + 2 * ((H) * (H) + (H)) + (H) * 8 + 8)

/* Create a denoiser for the mesh of ctx (borrowed; must outlive the denoiser).
 * hidden: H (multiple of 16, <= 1024); weights initialised uniform in
 * +-1/sqrt(fan_in) from seed, biases 0; feature standardisation identity. */
pdf_status pdf_denoiser_create(pdf_ctx *ctx, int32_t hidden, uint64_t seed, pdf_denoiser **out);
void pdf_denoiser_destroy(pdf_denoiser *dn);

/* Read (set = 0) or write (set = 1) the host parameter vector (n values). */
pdf_status pdf_denoiser_params(pdf_denoiser *dn, float *host, int64_t n, int32_t set);

/* Feature standardisation (48 means and standard deviations) and the output
 * scales of the 8 statistics (correction = scale_q * network output q). */
pdf_status pdf_denoiser_set_norm(pdf_denoiser *dn, const float *mu48, const float *sig48,
                                 const float *scale8);

/* The fallback test's calibration: a correction of statistic q is rejected
 * where it exceeds tau * kappa8[q] times the plain standard error at the node
 * (pdf_denoise_stats).  kappa_q = 1 (the default) judges corrections against
 * the estimator's noise alone; a larger kappa_q against its actual error,
 * noise and bias, e.g. tau * kappa_q set to a high quantile of the ratio
 * |error| / standard error that the plain estimator shows on calibration runs.
 * Each factor positive and finite (PDF_E_INVALID_ARG otherwise). */
pdf_status pdf_denoiser_set_fallback(pdf_denoiser *dn, const float *kappa8);

/* Save (save != 0) or load (save = 0) a trained denoiser at path, so that a
 * network trained once (on pairs of low- and high-count runs) can serve later
 * runs on a mesh.  The file holds an 8-byte tag "pdfdn001", the hidden width
 * and a flag for a set standardisation (int32 each), the parameter count
 * (int64), the float32 parameter vector (layout above), the 48 feature means,
 * the 48 feature scales, the 8 output scales and the 8 fallback factors
 * (float32), in the host's byte order.  The optimiser state is not kept: a
 * load resets it, as pdf_denoiser_params does.  Loading needs a denoiser of
 * the same hidden width (on any mesh) and rejects a file with another tag,
 * width or parameter count, a short or oversized file, non-positive feature
 * scales and non-positive or non-finite fallback factors; these and a file
 * that cannot be opened, read or written are PDF_E_INVALID_ARG with the
 * reason in pdf_last_error.  The denoiser is unchanged by a failed load.
 * Waits for the context's stream. */
pdf_status pdf_denoiser_io(pdf_denoiser *dn, int32_t save, const char *path);

/* Features of nodal statistics [PDF_NSTAT][n_nodes] (device pointer; NULL: the
 * context's latest estimate) into feat [n_nodes][48] (device, float32),
 * standardised when standardized != 0. */
pdf_status pdf_denoiser_features(pdf_denoiser *dn, const double *nodal, float *feat, int32_t standardized);

/* Network output y [n][8] (device, float32) for standardised inputs x [n][48]
 * (device, float32). */
pdf_status pdf_denoiser_forward(pdf_denoiser *dn, const float *x, int32_t n, float *y);

/* One training step on a batch (device pointers x [B][48], target [B][8]):
 * forward, mean-squared error, backward, Adam (lr, beta1 0.9, beta2 0.999,
 * eps 1e-8) on the float32 master parameters.  *loss (host) receives the
 * batch loss before the update.  With lr = 0 the parameters are unchanged and
 * grad_host (may be NULL) receives the gradient vector. */
pdf_status pdf_denoiser_train_step(pdf_denoiser *dn, const float *x, const float *target, int32_t B,
                                   float lr, float *loss, float *grad_host);

/* Denoised nodal statistics of the context's latest estimate into out
 * [PDF_NSTAT][n_nodes] (host or device): the plain statistics with the 8
 * corrected fields; *n_fallback (may be NULL) counts rejected corrections.
 * tau >= 0; tau = +inf (HUGE_VAL) takes every finite correction, also at
 * nodes where the standard error is zero; a non-finite correction is always
 * rejected.  With out on the device and n_fallback NULL the call only queues
 * the work on the context's stream and returns; otherwise it waits for it. */
pdf_status pdf_denoise_stats(pdf_denoiser *dn, double tau, double *out, int32_t on_device,
                             uint64_t *n_fallback);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as pdf_denoise_stats with out on the device, computed without any
 * allocation.  The work runs over chunks of 32768 nodes through a fixed
 * scratch area of 7 MiB (the features and network outputs of one chunk) that
 * the library holds in device memory on every GPU it runs on, until the
 * process ends; pdf_init_mesh sets it up on the current device.
 *   out            device [PDF_NSTAT][n_nodes]: the plain statistics with the 8
 *                  corrected fields
 *   n_fallback_dev device, 8-byte aligned, or NULL: receives the number of
 *                  rejected corrections (cleared by the call)
 * Asynchronous on the context's stream: no host synchronisation, no memset and
 * no allocation, so the call can be captured in a graph.  Needs the fused
 * inference: PDF_E_INVALID_ARG for a hidden width outside 48..128 (its
 * activations would not fit the scratch), as for a negative tau or a NULL out;
 * PDF_E_STATE before seeding.  All calls on one GPU share its scratch: calls
 * that overlap in time on one GPU (other streams or threads) race and give
 * undefined results. */
pdf_status pdf_denoise_stats_noalloc(pdf_denoiser *dn, double tau, double *out, uint64_t *n_fallback_dev);

#ifdef __cplusplus
}
#endif
#endif
