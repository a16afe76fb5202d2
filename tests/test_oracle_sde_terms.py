"""Pins for the viscous and mean-pressure terms of the particle equations
(eq:Lagrangian-position-exact and eq:Lagrangian-model, Ch.2) in the oracle.

One explicit Euler-Maruyama step from a known particle state with frozen
statistics.  With dW the position noise (shared by the velocity's viscous
term) and dW' the velocity noise,

  dx_i = u_i dt + sqrt(2 nu) dW_i
  du_i = (-d<P>/dx_i + 2 nu lap<U_i>) dt + sqrt(2 nu) d<U_i>/dx_j dW_j
         + G_ij (u_j - <U_j>) dt + sqrt(C0 eps) dW'_i,

so that, over many particles and with r_i the velocity increment less its
drift:
  * E[r_i] = 0 (the drift, with the sign of the pressure gradient, the factor
    2 nu of the Laplacian and the return term G (u - <U>)),
  * E[r_1 (dx_2 - u_2 dt)] = 2 nu d<U_1>/dy dt (the shared dW, its sign and
    its factor sqrt(2 nu) twice), while E[r_1 (dx_1 - u_1 dt)] = 0,
  * Var(dx_i) = 2 nu dt, Var(r_2) = C0 eps dt.
The tolerances are 5 standard errors of each estimate; every alternative
reading (a flipped sign, a dropped factor 2, dW' in place of dW) moves the
estimate by more than 10.
"""
import numpy as np

import oracle as O
from synth import configs as CF
from synth import meshes as M

NU, DT, OM, RDIAG, C0 = 0.01, 0.01, 0.5, 0.02, 2.1


def _particles_in(mesh, n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    om = O.OracleMesh(mesh)
    x = rng.uniform(lo, hi, n)
    y = rng.uniform(lo, hi, n)
    e = np.array([om.locate_brute(a, b) for a, b in zip(x, y)], np.int32)
    assert (e >= 0).all()
    return x, y, e


def _one_step(mesh, stats, gradp, x, y, e, u):
    p = CF.params(frozen=1, nu=NU, C0=C0, omega_source=0, wall_b=0)
    o = O.Oracle(mesh, p, gradp=gradp)
    U0, R0, Om0 = CF._iso(mesh.n_nodes)
    o.seed(dict(ppe=1, seed=11, psi_mode=0, U0=U0, R0=R0, Om0=Om0))
    n = x.size
    o.state = np.zeros((7, n))
    o.state[0], o.state[1] = x, y
    o.state[2:5] = np.asarray(u)[:, None]
    o.state[5] = OM
    o.elem = e.copy()
    o.id = np.arange(n, dtype=np.uint32)
    o.set_stats(stats)
    s0 = o.state.copy()
    assert o.step(DT) == 0
    assert o.counter_dict()["reflect"] == 0 and o.counter_dict()["periodic"] == 0
    return s0, o.state.copy()


def _coeffs():
    k = 0.5 * 3 * RDIAG
    eps = OM * (k + NU * CF.PAPER_CONSTANTS["CT"] ** 2 * OM)  # eq:dissipation-from-frequency_wall
    G = -(0.5 + 0.75 * C0) * OM                                # eq:wall-GandC
    return k, eps, G


def _z(est, expect, se):
    return abs(est - expect) / se


def test_viscous_pressure_terms_linear_shear():
    """<U_1> = 0.2 + S y (a linear field, so the element gradient is exactly
    S), an input Laplacian field (constant) and a uniform mean-pressure
    gradient; one step of 2e5 particles in the middle of a jittered box."""
    mesh = M.box(16, 16, jitter=0.15, seed=1, bc=M.BC_SLIP)
    S, L = 2.0, np.array([20.0, -15.0, 10.0])
    gp = np.array([0.5, -0.3])
    st = CF.frozen_stats_for(mesh, U=(0, 0, 0), R_diag=(RDIAG,) * 3, Om=OM, Phi=0.0)
    st[0] = 0.2 + S * mesh.node_xy[:, 1]
    st[21:24] = L[:, None]
    gradp = np.tile(gp[:, None], (1, mesh.n_nodes))
    n = 200_000
    x, y, e = _particles_in(mesh, n, 0.25, 0.75, seed=5)
    u = np.array([0.3, -0.2, 0.1])
    s0, s1 = _one_step(mesh, st, gradp, x, y, e, u)
    k, eps, G = _coeffs()
    # the element average of the linear nodal field is its value at the centroid
    yc = mesh.node_xy[mesh.elem_nodes[e], 1].mean(axis=1)
    Ue = np.stack([0.2 + S * yc, np.zeros(n), np.zeros(n)])
    drift = np.stack([(-gp[0] + 2 * NU * L[0]) * DT + G * (u[0] - Ue[0]) * DT,
                      (-gp[1] + 2 * NU * L[1]) * DT + G * (u[1] - Ue[1]) * DT,
                      (2 * NU * L[2]) * DT + G * (u[2] - Ue[2]) * DT])
    r = (s1[2:5] - s0[2:5]) - drift
    dxp = s1[0] - s0[0] - u[0] * DT
    dyp = s1[1] - s0[1] - u[1] * DT
    # drift: every component's residual has zero mean
    for a in range(3):
        se = r[a].std() / np.sqrt(n)
        assert _z(r[a].mean(), 0.0, se) < 5, (a, r[a].mean(), se)
        # the alternatives are far outside: a flipped pressure gradient, the
        # Laplacian without its factor 2, the return term with its sign flipped
        alt = [2 * gp[a] * DT if a < 2 else 0.0, NU * L[a] * DT, 2 * G * (u[a] - Ue[a]).mean() * DT]
        assert max(abs(v) for v in alt) / se > 10
    # position noise: zero mean, variance 2 nu dt
    for d in (dxp, dyp):
        assert _z(d.mean(), 0.0, d.std() / np.sqrt(n)) < 5
        assert abs(d.var() / (2 * NU * DT) - 1) < 5 * np.sqrt(2 / n)
    # the shared dW: E[r_1 dy'] = 2 nu S dt, and no x-gradient term
    c1y, c1x, c2y = r[0] * dyp, r[0] * dxp, r[1] * dyp
    se = c1y.std() / np.sqrt(n)
    assert _z(c1y.mean(), 2 * NU * S * DT, se) < 5, (c1y.mean(), 2 * NU * S * DT, se)
    assert 2 * NU * S * DT / se > 100
    assert _z(c1x.mean(), 0.0, c1x.std() / np.sqrt(n)) < 5
    assert _z(c2y.mean(), 0.0, c2y.std() / np.sqrt(n)) < 5
    # velocity noise: Var(r_2) = C0 eps dt, Var(r_1) = (2 nu S^2 + C0 eps) dt
    assert abs(r[1].var() / (C0 * eps * DT) - 1) < 5 * np.sqrt(2 / n)
    assert abs(r[0].var() / ((2 * NU * S * S + C0 * eps) * DT) - 1) < 5 * np.sqrt(2 / n)


def test_laplacian_drift_from_quadratic_mean():
    """<U_1> = a (y - 1/2)^2 on a uniform structured box; its nodal Laplacian
    from the estimator's two-pass derivatives is 2a at interior nodes (a
    closed form, checked first), and the particles' mean velocity change is
    2 nu (2a) dt plus the return term toward the element average."""
    mesh = M.box(16, 16, jitter=0.0, bc=M.BC_SLIP)
    a = 10.0
    st = CF.frozen_stats_for(mesh, U=(0, 0, 0), R_diag=(RDIAG,) * 3, Om=OM, Phi=0.0)
    st[0] = a * (mesh.node_xy[:, 1] - 0.5) ** 2
    st = O.OracleMesh(mesh).derivatives(st)
    n = 200_000
    x, y, e = _particles_in(mesh, n, 0.3, 0.7, seed=6)
    nodes = mesh.elem_nodes[e]
    assert np.abs(st[21, nodes] - 2 * a).max() < 1e-9  # the closed-form Laplacian
    assert np.abs(st[22:24, nodes]).max() < 1e-9
    u = np.array([0.1, 0.0, 0.0])
    s0, s1 = _one_step(mesh, st, None, x, y, e, u)
    k, eps, G = _coeffs()
    Ue = st[0, nodes].mean(axis=1)  # element average of the three nodal values
    r = (s1[2] - s0[2]) - (2 * NU * 2 * a * DT + G * (u[0] - Ue) * DT)
    se = r.std() / np.sqrt(n)
    assert _z(r.mean(), 0.0, se) < 5, (r.mean(), se)
    assert NU * 2 * a * DT / se > 10  # the Laplacian drift without its factor 2 is far outside
