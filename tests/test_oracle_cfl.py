"""Pins for the oracle's time step of eq:CFL: a closed form on a uniform grid
with uniform flow, a NumPy evaluation of the definition on a jittered grid
with a varying flow, the cap and the no-flow case."""
import numpy as np

import oracle as O
from synth import configs as CF
from synth import meshes as M


def _oracle(mesh, U, V):
    o = O.Oracle(mesh, CF.params())
    st = np.zeros((25, mesh.n_nodes))
    st[0], st[1] = U, V
    o.set_stats(st)
    return o


def test_uniform_grid_uniform_flow_closed_form():
    n = 16
    mesh = M.periodic_square(n)
    o = _oracle(mesh, 2.0, 0.0)
    # every element is a right triangle of area h^2/2 with h = 1/n
    assert abs(o.cfl_dt(0.7, 1.0) - 0.7 * np.sqrt(0.5 / n ** 2) / 2.0) < 1e-15


def test_definition_on_jittered_grid():
    mesh = M.box(9, 7, 2.0, 1.0, jitter=0.25, seed=3)
    rng = np.random.default_rng(1)
    U = rng.normal(size=mesh.n_nodes)
    V = rng.normal(size=mesh.n_nodes)
    U[5] = V[5] = 0.0  # a node at rest does not limit the step
    o = _oracle(mesh, U, V)
    P = mesh.node_xy[mesh.elem_nodes]
    A = 0.5 * np.abs((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                     - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1]))
    s = np.zeros(mesh.n_nodes)
    c = np.zeros(mesh.n_nodes)
    for k in range(3):
        np.add.at(s, mesh.elem_nodes[:, k], A)
        np.add.at(c, mesh.elem_nodes[:, k], 1.0)
    sp = np.hypot(U, V)
    ok = sp > 0
    expect = 0.5 * np.min(np.sqrt(s[ok] / c[ok]) / sp[ok])
    assert abs(o.cfl_dt(0.5, 10.0) - expect) <= 1e-14 * expect
    assert o.cfl_dt(0.5, 0.1 * expect) == 0.1 * expect  # capped


def test_no_flow_gives_the_cap():
    mesh = M.box(3, 3, 1.0, 1.0)
    assert _oracle(mesh, 0.0, 0.0).cfl_dt(0.7, 0.25) == 0.25
