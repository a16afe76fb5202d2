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
