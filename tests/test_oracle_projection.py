"""Pins for the oracle's stabilized pressure projection (eq:pressure-
projection-smooth, eq:velocity-correction):

- a gradient field u* = grad(phi) on the doubly periodic square is removed:
  dt dP converges to phi at second order, so the corrected velocity
  u* - dt grad(dP) vanishes;
- a field that varies only across itself (u* = (cos 2 pi y, 0)) has zero
  element divergence and is left untouched;
- the stabilizing term alone (no divergence) gives dP = -C_p (P' - mean P')
  exactly;
- in a step, every particle's velocity changes by exactly -dt grad(dP) of its
  element after the move, positions unchanged, and the gradient of the next
  step is the imposed one plus the nodal gradient of P'."""
import math

import numpy as np

import oracle as O
from oracle import projection as PR
from synth import configs as CF
from synth import meshes as M


def _gradient_case(n, dt=0.01):
    mesh = M.periodic_square(n)
    x, y = mesh.node_xy.T
    phi = np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) / (2 * np.pi)
    U = np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y)
    V = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    dP = PR.solve_dp(mesh, U, V, np.zeros(mesh.n_nodes), dt, 0.0)
    return np.abs(dt * dP - (phi - phi.mean())).max()


def test_gradient_field_is_removed_second_order():
    e1, e2 = _gradient_case(16), _gradient_case(32)
    assert e2 < 2e-3 and 1.8 < math.log2(e1 / e2) < 2.3


def test_divergence_free_field_untouched():
    mesh = M.periodic_square(16)
    y = mesh.node_xy[:, 1]
    dP = PR.solve_dp(mesh, np.cos(2 * np.pi * y), np.zeros(mesh.n_nodes), np.zeros(mesh.n_nodes), 0.01, 0.0)
    assert np.abs(dP).max() < 1e-12


def test_stabilizing_term():
    mesh = M.periodic_square(12)
    x, y = mesh.node_xy.T
    P = np.sin(2 * np.pi * x) + 0.3 * np.cos(4 * np.pi * y) + 5.0
    Cp, dt = 1e-3, 0.01
    dP = PR.solve_dp(mesh, np.ones(mesh.n_nodes), np.zeros(mesh.n_nodes), P, dt, Cp)
    masters = np.unique(mesh.node_master)
    Pm = P - P[masters].mean()
    np.testing.assert_allclose(dP * dt, -Cp * Pm, rtol=0, atol=1e-12)


def test_step_corrects_particle_velocities():
    w = CF.periodic_square(n=8, ppe=30, seed=1)
    w.params = dict(w.params, model=CF.MODEL_SLM, nu=0.0)
    base = O.Oracle(w.mesh, w.params)
    base.seed(w.seed)
    proj = O.Oracle(w.mesh, dict(w.params, proj=1, Cp=1e-3))
    proj.seed(w.seed)
    base.step(w.dt)
    proj.step(w.dt)
    assert np.array_equal(base.elem, proj.elem)
    assert np.array_equal(base.state[[0, 1, 4, 5, 6]], proj.state[[0, 1, 4, 5, 6]])
    g = PR.elem_gradient(w.mesh, proj.last_dp)
    np.testing.assert_allclose(proj.state[2], base.state[2] - w.dt * g[base.elem, 0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(proj.state[3], base.state[3] - w.dt * g[base.elem, 1], rtol=0, atol=1e-15)
    assert np.abs(proj.last_dp).max() > 0
    np.testing.assert_allclose(proj.gradp, PR.node_gradient(w.mesh, proj.Pp), rtol=0, atol=1e-15)


# ---- walls: the Neumann condition of eq:wall-pressure-condition ----

def _wall_case(n, with_flux, dt=0.01):
    """u* = dt grad(phi) on a box with walls: dP = phi when the walls carry
    dP/dn = dphi/dn (here phi has non-zero normal derivatives on every side)."""
    mesh = M.box(n, n, 1.0, 1.0, bc=M.BC_NOSLIP)
    x, y = mesh.node_xy.T
    phi = np.cos(1.3 * x + 0.4) * np.sin(2.1 * y + 0.7) + 0.5 * x * x
    U = dt * (-1.3 * np.sin(1.3 * x + 0.4) * np.sin(2.1 * y + 0.7) + x)
    V = dt * (2.1 * np.cos(1.3 * x + 0.4) * np.cos(2.1 * y + 0.7))
    W = PR.wall_edges(mesh)
    g = []
    for end in ("a", "b"):
        q = W[end]
        gx = -1.3 * np.sin(1.3 * x[q] + 0.4) * np.sin(2.1 * y[q] + 0.7) + x[q]
        gy = 2.1 * np.cos(1.3 * x[q] + 0.4) * np.cos(2.1 * y[q] + 0.7)
        g.append(gx * W["n"][:, 0] + gy * W["n"][:, 1])
    flux = PR.boundary_vector(mesh, np.array(g)) if with_flux else None
    dP = PR.solve_dp(mesh, U, V, np.zeros(mesh.n_nodes), dt, 0.0, flux=flux)
    return np.abs(dP - (phi - phi.mean())).max()


def test_wall_neumann_condition_second_order():
    # the maximum nodal error approaches second order from below (1.48, 1.63,
    # 1.70 over 8 -> 16 -> 32 -> 64 cells a side)
    e1, e2 = _wall_case(32, True), _wall_case(64, True)
    assert e2 < 1e-3 and 1.6 < math.log2(e1 / e2) < 2.4
    # natural (zero-flux) conditions miss it by O(1)
    assert _wall_case(32, False) > 100 * e2


def test_wall_edges_and_boundary_vector():
    mesh = M.box(6, 4, 3.0, 2.0, bc=M.BC_SLIP)
    W = PR.wall_edges(mesh)
    # the outward normals of the rectangle's four sides; the lengths add up
    assert np.isclose(W["L"].sum(), 2 * (3.0 + 2.0))
    mid = 0.5 * (mesh.node_xy[W["a"]] + mesh.node_xy[W["b"]])
    out = np.where(np.isclose(mid[:, 0], 0)[:, None], [-1, 0], 0) + np.where(np.isclose(mid[:, 0], 3)[:, None], [1, 0], 0) \
        + np.where(np.isclose(mid[:, 1], 0)[:, None], [0, -1], 0) + np.where(np.isclose(mid[:, 1], 2)[:, None], [0, 1], 0)
    np.testing.assert_allclose(W["n"], out, atol=1e-15)
    # B of a constant integrates it over the boundary; of a linear q, exactly
    B1 = PR.boundary_vector(mesh, np.ones((2, W["L"].size)))
    assert np.isclose(B1.sum(), 10.0)
    xa, xb = mesh.node_xy[W["a"], 0], mesh.node_xy[W["b"], 0]
    Bx = PR.boundary_vector(mesh, np.array([xa, xb]))
    # the integral of x over the boundary: two horizontal sides (3^2/2 each) + the right side (3 * 2)
    assert np.isclose(Bx.sum(), 9.0 + 6.0)


def test_neumann_data_closed_form():
    """Linear Reynolds stresses (their element gradients exact) and given
    nodal Laplacians: g = nu lap<U>.n - div<uu>.n at every wall edge end."""
    mesh = M.box(5, 5, 1.0, 1.0, jitter=0.2, seed=3, bc=M.BC_NOSLIP)
    x, y = mesh.node_xy.T
    st = np.zeros((25, mesh.n_nodes))
    st[5] = 0.3 + 0.5 * x - 0.2 * y      # R11
    st[6] = 0.1 - 0.4 * x + 0.7 * y      # R22
    st[8] = -0.05 + 0.9 * x + 0.3 * y    # R12
    st[21] = 1.0 + 2.0 * x               # lap <U>
    st[22] = -3.0 + y                    # lap <V>
    nu = 0.02
    g = PR.neumann_data(mesh, st, nu)
    W = PR.wall_edges(mesh)
    divR = np.array([0.5 + 0.3, 0.9 + 0.7])
    for j, end in enumerate(("a", "b")):
        q = W[end]
        ref = nu * (st[21][q] * W["n"][:, 0] + st[22][q] * W["n"][:, 1]) - (divR[0] * W["n"][:, 0] + divR[1] * W["n"][:, 1])
        np.testing.assert_allclose(g[j], ref, rtol=0, atol=1e-13)


def test_step_flux_bookkeeping():
    """In a step, the boundary term is (C_p/dt) B(g^n - G.n) + B(g^{n+1} - g^n)
    with g^n the previous step's data (G.n before the first step)."""
    w = CF.channel(nx=8, n_half=4, ppe=20, precision="f64")
    w.params = dict(w.params, proj=1, Cp=1e-4)
    o = O.Oracle(w.mesh, w.params, gradp=w.gradp)
    o.seed(w.seed)
    BG = PR.boundary_vector(w.mesh, PR.imposed_normal(w.mesh, o.gradp_in))
    o.step(w.dt)
    B1 = o.B_prev
    assert np.abs(B1).max() > 0
    # the flux of the first step: (Cp/dt) * 0 + (B1 - BG)
    est = o.est
    o2 = O.Oracle(w.mesh, w.params, gradp=w.gradp)
    o2.seed(w.seed)
    o2.step(w.dt)
    assert np.array_equal(o2.B_prev, B1)
    P0 = np.zeros(w.mesh.n_nodes)
    # recompute the first solve by hand from the predicted statistics of a third run
    o3 = O.Oracle(w.mesh, dict(w.params, proj=0), gradp=w.gradp)
    o3.seed(w.seed)
    o3.step(w.dt)
    pred = o3.est
    Bp = PR.boundary_vector(w.mesh, PR.neumann_data(w.mesh, pred, w.params["nu"]))
    np.testing.assert_allclose(Bp, B1, rtol=0, atol=1e-14)
    dP = PR.solve_dp(w.mesh, pred[0], pred[1], P0, w.dt, 1e-4, flux=Bp - BG)
    np.testing.assert_allclose(dP, o.last_dp, rtol=0, atol=1e-12 * np.abs(dP).max())
    assert est is not None


def test_canyon_with_projection_stays_finite_200_steps():
    """The street canyon (floor blocks with reflex corners, slip top,
    streamwise periodic) with the projection and the wall datum, C_p = 0.1 dt
    and the redistribution keeping 3 per element: 200 steps stay finite, lose
    no particle and keep the RMS speed within 25 % of its start."""
    w = CF.canyon(target_elems=4000, ppe=12, precision="f64")
    w.params = dict(w.params, proj=1, Cp=0.1 * w.dt, min_ppe=3)
    o = O.Oracle(w.mesh, w.params, gradp=w.gradp)
    o.seed(w.seed)
    rms0 = np.sqrt((o.state[2] ** 2 + o.state[3] ** 2).mean())
    for _ in range(4):
        o.run(w.dt, 50)
        rms = np.sqrt((o.state[2] ** 2 + o.state[3] ** 2).mean())
        assert np.isfinite(o.state).all() and np.isfinite(o.Pp).all()
        assert 0.75 * rms0 <= rms <= 1.25 * rms0, (rms, rms0)
    assert o.counter_dict()["lost"] == 0
