"""Seeded synthetic workloads shaped like the dissertation's test cases.

A workload bundles a mesh, the model constants, the initial-condition recipe
(nodal mean velocity, Reynolds stress and mean frequency, plus the scalar
initial condition), optional nodal input fields (mean-pressure gradient and
the elliptic-relaxation tensor), a time step and a step count.  These are
inputs only: no step of the particle method is computed here.

Model constants are those of the paper's constant tables (Ch.4 tab:fd-constants,
Ch.5 tab:constants); the workload-specific values (meshes, particle counts,
time steps, sources) are stated in each workload's constructor below.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

from . import meshes as M

# Ch.4 / Ch.5 constant tables
PAPER_CONSTANTS = dict(C1=1.85, C2=0.63, C3=5.0, C4=0.25, CT=6.0, CL=0.134, Ceta=72.0, Cv=1.4,
                       gamma5=0.1, Cw1=0.5, Cw2=0.73, Cs=0.02, Ct=0.7)

MODEL_SLM, MODEL_GLM = 0, 1
WP_INPUT, WP_LOCAL, WP_ELLIPTIC = 0, 1, 2
TM_CPHI, TM_KEPS, TM_SOURCE = 0, 1, 2
MIX_IEM, MIX_IECM = 0, 1
PSI_ZERO, PSI_STEP_X, PSI_GAUSS_X, PSI_BERNOULLI, PSI_DISC = 0, 1, 2, 3, 4
STATS_ELEM, STATS_SHAPE = 0, 1


def params(**kw):
    p = dict(model=MODEL_SLM, wp_source=WP_LOCAL, omega_source=0, tm_mode=TM_CPHI, frozen=0,
             wall_b=0, stats_mode=STATS_ELEM, min_ppe=0, mix_model=MIX_IEM, cond_nu=5, cond_nv=5,
             cond_nw=5, cond_min=2, nu_wall=0.0, C0=2.1, Cphi=2.0, nu=0.0, k_floor=1e-10, src_x=0.0, src_y=0.0, src_r=0.0)
    p.update(PAPER_CONSTANTS)
    p.update(kw)
    return p


@dataclass
class Workload:
    name: str
    mesh: M.Mesh
    params: dict
    seed: dict                  # ppe, seed, psi_mode, a, b, c, U0 (3,nn), R0 (6,nn), Om0 (nn)
    dt: float
    steps: int
    precision: str              # "f64" or "f32"
    gradp: np.ndarray | None = None   # (2, nn) nodal mean-pressure gradient / rho
    wp: np.ndarray | None = None      # (9, nn) nodal elliptic-relaxation tensor (WP_INPUT)
    meta: dict = field(default_factory=dict)

    @property
    def n_particles(self):
        return self.mesh.n_elems * int(self.seed["ppe"])


def _iso(nn, U=(0.0, 0.0, 0.0), var=2.0 / 3.0, Om=1.0):
    U0 = np.zeros((3, nn))
    for i in range(3):
        U0[i] = U[i]
    R0 = np.zeros((6, nn))
    R0[0:3] = var
    return U0, R0, np.full(nn, Om)


# ----------------------------------------------------------------------------
# Workload 1: periodic unit square, simplified Langevin model, FP64
# ----------------------------------------------------------------------------

def periodic_square(n=32, ppe=50, seed=0, steps=100, dt=0.01, psi_mode=PSI_STEP_X, frozen=0,
                    U=(1.0, 0.0, 0.0), var=0.01, Om=1.0, precision="f64", **pkw):
    """Unit square, n x n squares split into 2 triangles, periodic on all sides;
    uniform mean velocity (1,0), velocities N(0, 0.1^2) about it, gamma
    frequencies (mean 1, C4 = 0.25), simplified Langevin C0 = 2.1, C3 = 1,
    S_omega = 0, IEM with C_phi = 2, scalar step phi = 1 for x < 0.5."""
    mesh = M.periodic_square(n)
    nn = mesh.n_nodes
    U0, R0, Om0 = _iso(nn, U, var, Om)
    p = params(model=MODEL_SLM, C0=2.1, C3=1.0, C4=0.25, omega_source=0, tm_mode=TM_CPHI,
               Cphi=2.0, nu=0.0, frozen=frozen)
    p.update(pkw)
    sd = dict(ppe=ppe, seed=seed, psi_mode=psi_mode, a=0.5, b=0.0, c=0.0, U0=U0, R0=R0, Om0=Om0)
    return Workload(f"periodic_square_{n}_ppe{ppe}_{precision}", mesh, p, sd, dt, steps, precision)


def frozen_stats_for(mesh, U=(1.0, 0.0, 0.0), R_diag=(2.0 / 3.0,) * 3, Om=1.0, Phi=0.5):
    """Nodal statistics for the frozen-statistics test mode (uniform fields)."""
    st = np.zeros((25, mesh.n_nodes))
    st[0:3] = np.asarray(U)[:, None]
    st[3] = Om
    st[4] = Phi
    st[5:8] = np.asarray(R_diag)[:, None]
    return st


# ----------------------------------------------------------------------------
# Wall-bounded flows: analytic near-wall fields
# ----------------------------------------------------------------------------

KAPPA, E_WALL = 0.41, 8.5  # law of the wall constants (Ch.2, eq:Ue)


def _loglaw(dplus):
    """Mean streamwise velocity in wall units: y+ below 11, log law above."""
    return np.where(dplus < 11.0, dplus, np.log(E_WALL * np.maximum(dplus, 1e-30)) / KAPPA)


def _wall_fields(d, dmax, nu, utau=1.0):
    """Synthetic near-wall statistics as functions of wall distance d:
    log-law mean velocity, Reynolds stresses damped toward the wall (with a
    floor of 0.2 u_tau^2 per component) and mean frequency
    ~ u_tau / (sqrt(C_mu) kappa d), capped within 50 viscous lengths of the wall
    so that the explicit scheme stays within its stability limit."""
    dplus = d * utau / nu
    U = utau * _loglaw(dplus)
    f = 1.0 - np.exp(-dplus / 10.0)
    eta = np.clip(d / dmax, 0.0, 1.0)
    r11 = (2.0 * utau * f) ** 2 * (1.0 - 0.5 * eta) + 0.2 * utau ** 2
    r22 = (0.8 * utau * f) ** 2 * (1.0 - 0.3 * eta) + 0.2 * utau ** 2
    r33 = (1.2 * utau * f) ** 2 * (1.0 - 0.4 * eta) + 0.2 * utau ** 2
    r12 = -0.8 * (1.0 - eta) * np.sqrt(r11 * r22) * f
    Om = utau / (0.3 * KAPPA * (d + 50.0 * nu))
    R = np.stack([r11, r22, r33, r12, np.zeros_like(d), np.zeros_like(d)])
    return U, R, Om


def _box_wall_distance(xy, mesh):
    """Distance from each node to the nearest no-slip boundary edge, from a
    KD-tree over points sampled densely along the wall edges (8 per edge), so
    the error is at most 1/16 of a wall edge length."""
    from scipy.spatial import cKDTree

    sel = np.nonzero(mesh.bedge_type == M.BC_NOSLIP)[0]
    e = mesh.bedge_elem[sel]
    k = mesh.bedge_local[sel]
    a = mesh.node_xy[mesh.elem_nodes[e, (k + 1) % 3]]
    b = mesh.node_xy[mesh.elem_nodes[e, (k + 2) % 3]]
    t = np.linspace(0.0, 1.0, 9)
    pts = (a[:, None, :] + t[None, :, None] * (b - a)[:, None, :]).reshape(-1, 2)
    d, _ = cKDTree(pts).query(xy)
    return d


def cfl_dt(mesh, U0, c_cfl=0.7):
    """Time step from eq:CFL on the initial mean field: C_CFL min_n sqrt(A_n)/|U_n|."""
    A = mesh.areas()
    nn = mesh.n_nodes
    s = np.zeros(nn)
    c = np.zeros(nn)
    for k in range(3):
        np.add.at(s, mesh.elem_nodes[:, k], A)
        np.add.at(c, mesh.elem_nodes[:, k], 1.0)
    An = s / np.maximum(c, 1)
    speed = np.sqrt((U0[:2] ** 2).sum(0))
    ok = speed > 1e-12
    return float(c_cfl * np.min(np.sqrt(An[ok]) / speed[ok]))


def channel(nx=100, n_half=50, ppe=100, seed=0, steps=500, dt=1e-3, precision="f32",
            re_tau=392.0, wp_source=WP_LOCAL):
    """Plane channel [0,6]x[0,2], ~20k triangles refined toward the walls,
    Re_tau = 392 (u_tau = 1, h = 1, nu = 1/392); full generalized Langevin model;
    no-slip walls with the trajectory (b) test; streamwise periodic; unit mean
    pressure gradient; scalar from a Gaussian line source at x = 0.5 (sigma 0.02)."""
    mesh = M.graded_channel(nx, n_half, 6.0, 1.0, 0.15, seed)
    nu = 1.0 / re_tau
    xy = mesh.node_xy
    d = np.minimum(xy[:, 1], 2.0 - xy[:, 1])
    U, R, Om = _wall_fields(d, 1.0, nu)
    U0 = np.stack([U, np.zeros_like(U), np.zeros_like(U)])
    gradp = np.stack([np.full(mesh.n_nodes, -1.0), np.zeros(mesh.n_nodes)])
    p = params(model=MODEL_GLM, wp_source=wp_source, omega_source=1, tm_mode=TM_KEPS, nu=nu,
               wall_b=1)
    sd = dict(ppe=ppe, seed=seed, psi_mode=PSI_GAUSS_X, a=0.5, b=0.02, c=0.0, U0=U0, R0=R,
              Om0=Om)
    return Workload(f"channel_{mesh.n_elems}_ppe{ppe}_{precision}", mesh, p, sd, dt, steps,
                    precision, gradp=gradp)


def channel_wallfn(nx=40, n_half=10, ppe=50, seed=0, steps=200, dt=2e-3, precision="f64", re_tau=392.0):
    """Plane channel [0,6]x[0,2] with wall functions at both walls (the
    coarse-wall variant of Ch.2): a uniform grid whose first gridpoints sit at
    y+ ~ 40; the simplified Langevin model with C0 = 3.5 (eq:wall-GandC), no
    viscous terms in the particle equations (nu = 0), nu = 1/Re_tau only in
    the log law eq:Ue; unit mean pressure gradient; gamma frequency, IEM."""
    mesh = M.uniform_channel(nx, 2 * n_half, 6.0, 1.0, 0.15, seed)
    nu = 1.0 / re_tau
    xy = mesh.node_xy
    d = np.minimum(xy[:, 1], 2.0 - xy[:, 1])
    U, R, Om = _wall_fields(np.maximum(d, 2.0 / (2 * n_half)), 1.0, nu)
    U0 = np.stack([U, np.zeros_like(U), np.zeros_like(U)])
    gradp = np.stack([np.full(mesh.n_nodes, -1.0), np.zeros(mesh.n_nodes)])
    p = params(model=MODEL_SLM, C0=3.5, omega_source=1, tm_mode=TM_KEPS, nu=0.0, nu_wall=nu)
    sd = dict(ppe=ppe, seed=seed, psi_mode=PSI_GAUSS_X, a=0.5, b=0.05, c=0.0, U0=U0, R0=R, Om0=Om)
    return Workload(f"channel_wallfn_{mesh.n_elems}_ppe{ppe}_{precision}", mesh, p, sd, dt, steps,
                    precision, gradp=gradp)


def canyon(target_elems=200_000, ppe=50, seed=0, steps=1000, precision="f32", src=(10.0, 0.5, 0.1),
           mesh=None):
    """Street-canyon-like box [0,20]x[0,10] with two 2x3 blocks, ~200k triangles
    graded 5:1 toward walls; generalized Langevin + gamma frequency + IEM;
    log-profile initial mean velocity; continuous disc scalar source between
    the blocks; time step from C_CFL = 0.7 on the initial field."""
    mesh = mesh if mesh is not None else M.canyon(target_elems, 0.15, seed)
    nu = 3.5 / 600.0
    xy = mesh.node_xy
    d = _box_wall_distance(xy, mesh)
    U, R, Om = _wall_fields(d, 3.5, nu)
    U0 = np.stack([U, np.zeros_like(U), np.zeros_like(U)])
    gradp = np.stack([np.full(mesh.n_nodes, -1.0 / 7.0), np.zeros(mesh.n_nodes)])
    p = params(model=MODEL_GLM, wp_source=WP_LOCAL, omega_source=1, tm_mode=TM_KEPS, nu=nu,
               wall_b=1, src_x=src[0], src_y=src[1], src_r=src[2])
    sd = dict(ppe=ppe, seed=seed, psi_mode=PSI_ZERO, a=0.0, b=0.0, c=0.0, U0=U0, R0=R, Om0=Om)
    dt = cfl_dt(mesh, U0, 0.7)
    return Workload(f"canyon_{mesh.n_elems}_ppe{ppe}_{precision}", mesh, p, sd, dt, steps,
                    precision, gradp=gradp, meta={"nu": nu})


def channel_block(target_elems=1_000_000, ppe=100, seed=0, steps=200, precision="f32", mesh=None):
    """Graded channel [0,30]x[0,2] with a 1x0.5 floor block at x in [5,6],
    ~1M triangles; generalized Langevin + gamma frequency + IEM; Re_tau = 392;
    scalar from a Gaussian line at x = 2 (sigma 0.05)."""
    mesh = mesh if mesh is not None else M.channel_block(target_elems, 0.15, seed)
    nu = 1.0 / 392.0
    xy = mesh.node_xy
    d = _box_wall_distance(xy, mesh)
    U, R, Om = _wall_fields(d, 1.0, nu)
    U0 = np.stack([U, np.zeros_like(U), np.zeros_like(U)])
    gradp = np.stack([np.full(mesh.n_nodes, -1.0), np.zeros(mesh.n_nodes)])
    p = params(model=MODEL_GLM, wp_source=WP_LOCAL, omega_source=1, tm_mode=TM_KEPS, nu=nu,
               wall_b=1)
    sd = dict(ppe=ppe, seed=seed, psi_mode=PSI_GAUSS_X, a=2.0, b=0.05, c=0.0, U0=U0, R0=R, Om0=Om)
    dt = cfl_dt(mesh, U0, 0.7)
    return Workload(f"channel_block_{mesh.n_elems}_ppe{ppe}_{precision}", mesh, p, sd, dt, steps,
                    precision, gradp=gradp)
