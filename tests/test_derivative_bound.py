"""The derivative bound of tests/parity.py against the oracle's own FEM
derivative operator: the nodal means are perturbed by a known amount and the
oracle recomputes fields 15-23 on both; every discrepancy must lie within the
bound, and the bound must not be vacuous (within a few orders of the worst
discrepancy).  Meshes: a box stretched toward its wall (element sizes 1e-3 to
6e-2) and a jittered channel periodic in x (identified nodes carry their
master's values)."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from synth import meshes as M
from tests.parity import derivative_bounds


def _stretched():
    m = M.box(16, 32, 1.0, 1.0, jitter=0.0, seed=0, bc=M.BC_SLIP)
    xy = m.node_xy.copy()
    xy[:, 1] = xy[:, 1] ** 2.0
    return dataclasses.replace(m, node_xy=xy)


@pytest.mark.parametrize("make", [_stretched, lambda: M.uniform_channel(24, 12, 2.0, 1.0, jitter=0.2, seed=3)])
@pytest.mark.parametrize("rel", [1e-12, 1e-6])
def test_derivative_bound_holds_and_is_tight(make, rel):
    mesh = make()
    om = O.OracleMesh(mesh)
    rng = np.random.default_rng(7)
    x, y = mesh.node_xy[:, 0], mesh.node_xy[:, 1]
    S = np.zeros((25, mesh.n_nodes))
    S[0] = np.sin(2 * np.pi * x) * np.cos(np.pi * y) + 0.3
    S[1] = x * y
    S[2] = np.exp(-((x - 0.5) ** 2 + (y - 0.3) ** 2) / 0.05)
    S = np.ascontiguousarray(S[:, mesh.node_master])  # identified nodes carry their master's values
    ref = om.derivatives(S)
    P = S.copy()
    P[0:3] += rel * rng.uniform(-1.0, 1.0, (3, mesh.n_nodes))
    P = np.ascontiguousarray(P[:, mesh.node_master])
    pert = om.derivatives(P)
    tol1, tol2 = derivative_bounds(mesh, pert, ref)
    r1 = (np.abs(pert[15:21] - ref[15:21]) / tol1).max()
    r2 = (np.abs(pert[21:24] - ref[21:24]) / tol2).max()
    assert r1 <= 1.0 and r2 <= 1.0, (r1, r2)
    assert r1 > 1e-3 and r2 > 1e-4, (r1, r2)
