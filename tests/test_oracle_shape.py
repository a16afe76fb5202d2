"""Pins for the oracle's SHAPE reading of the statistics at particles and
nodes: the finite-element approximation of eq:approximation used to gather
nodal statistics at a particle's position and, weighted by the same shape
functions N^j, to scatter particle values to the nodes.

- The node estimator against a NumPy evaluation of its definition, with the
  shape functions from the local coordinates of eq:shapefunctions (a 2x2
  solve), not from the signed areas the oracle uses.
- Partition of unity: the node weights sum to the particle count.
- A constant property is reproduced; particles on a vertex feed that node only.
- The gather reproduces a linear nodal field exactly at the particle (one IEM
  step toward a linear mean scalar has a closed form), which the element
  average of the ELEM reading does not.
"""
import numpy as np

import oracle as O
from synth import configs as CF
from synth import meshes as M


def _random_particles(mesh, n, rng):
    elem = rng.integers(0, mesh.n_elems, n)
    r1, r2 = rng.random(n), rng.random(n)
    flip = r1 + r2 > 1.0
    r1[flip], r2[flip] = 1.0 - r1[flip], 1.0 - r2[flip]
    P = mesh.node_xy[mesh.elem_nodes[elem]]
    xy = P[:, 0] + r1[:, None] * (P[:, 1] - P[:, 0]) + r2[:, None] * (P[:, 2] - P[:, 0])
    state = np.empty((7, n))
    state[0:2] = xy.T
    state[2:7] = rng.normal(size=(5, n)) * np.array([1.0, 0.5, 0.3, 0.4, 2.0])[:, None] + 0.7
    return state, elem


def _oracle(mesh, state, elem, **kw):
    o = O.Oracle(mesh, CF.params(stats_mode=CF.STATS_SHAPE, **kw))
    o.state = np.ascontiguousarray(state, np.float64)
    o.elem = np.ascontiguousarray(elem, np.int32)
    o.id = np.arange(state.shape[1], dtype=np.uint32)
    return o


def _local_shape(mesh, elem, xy):
    """(1 - xi - eta, xi, eta) from x = A + xi (B - A) + eta (C - A)."""
    P = mesh.node_xy[mesh.elem_nodes[elem]]
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=2)  # columns B-A, C-A
    xe = np.linalg.solve(J, (xy - P[:, 0])[..., None])[..., 0]
    return np.stack([1.0 - xe[:, 0] - xe[:, 1], xe[:, 0], xe[:, 1]], axis=1)


def test_node_estimator_matches_definition():
    mesh = M.box(5, 4, 2.0, 1.0, jitter=0.2, seed=3)
    rng = np.random.default_rng(1)
    state, elem = _random_particles(mesh, 3000, rng)
    o = _oracle(mesh, state, elem)
    S = o.estimate()
    N = _local_shape(mesh, elem, state[0:2].T)
    node = mesh.elem_nodes[elem]
    nn = mesh.n_nodes
    W = np.zeros(nn)
    np.add.at(W, node.ravel(), N.ravel())
    q = state[2:7]
    mean = np.zeros((5, nn))
    for f in range(5):
        np.add.at(mean[f], node.ravel(), (N * q[f][:, None]).ravel())
    mean /= W
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2), (4, 4), (0, 4), (1, 4), (2, 4)]
    assert np.allclose(S[24], W, rtol=1e-12, atol=1e-12)
    assert np.allclose(S[0:5], mean, rtol=1e-12, atol=1e-12)
    for c, (a, b) in enumerate(pairs):
        cov = np.zeros(nn)
        da = q[a][:, None] - mean[a][node]
        db = q[b][:, None] - mean[b][node]
        np.add.at(cov, node.ravel(), (N * da * db).ravel())
        assert np.allclose(S[5 + c], cov / W, rtol=1e-10, atol=1e-12), c


def test_partition_of_unity_and_periodic_identification():
    mesh = M.periodic_square(8)
    rng = np.random.default_rng(2)
    state, elem = _random_particles(mesh, 5000, rng)
    S = _oracle(mesh, state, elem).estimate()
    masters = np.unique(mesh.node_master)
    assert abs(S[24][masters].sum() - 5000) < 1e-9
    # identified nodes carry their master's values
    assert np.array_equal(S[:, np.arange(mesh.n_nodes)], S[:, mesh.node_master])


def test_constant_property_and_vertex_particles():
    mesh = M.box(4, 4, 1.0, 1.0, jitter=0.1, seed=5)
    rng = np.random.default_rng(3)
    state, elem = _random_particles(mesh, 2000, rng)
    state[2:7] = np.array([1.25, -0.5, 3.0, 0.75, 0.125])[:, None]
    S = _oracle(mesh, state, elem).estimate()
    assert np.allclose(S[0:5], np.array([1.25, -0.5, 3.0, 0.75, 0.125])[:, None], rtol=1e-14, atol=0)
    assert np.abs(S[5:15]).max() < 1e-14
    # every particle on one vertex of its element: only those vertices gain weight
    e = np.array([0, 0, 7, 7, 7])
    k = np.array([0, 0, 2, 2, 2])
    v = mesh.elem_nodes[e, k]
    st = np.zeros((7, 5))
    st[0:2] = mesh.node_xy[v].T
    st[2] = [1.0, 3.0, 5.0, 6.0, 7.0]
    o = _oracle(mesh, st, e)
    prev = np.full((25, mesh.n_nodes), -9.0)
    o.stats = prev
    S = o.estimate()
    for vv, vals in ((v[0], [1.0, 3.0]), (v[2], [5.0, 6.0, 7.0])):
        assert S[24][vv] == len(vals)
        assert abs(S[0][vv] - np.mean(vals)) < 1e-14
        assert abs(S[5][vv] - np.var(vals)) < 1e-13
    others = np.setdiff1d(np.arange(mesh.n_nodes), v)
    assert np.all(S[24][others] == 0.0)
    assert np.all(S[0:15][:, others] == -9.0)  # no support: previous values kept
    assert o.counter_dict()["empty_node"] == len(others)


def test_gather_reproduces_linear_mean_scalar_in_iem_step():
    """Frozen statistics with <phi> = a + b x + c y and constant <omega>: one
    IEM step (1/t_m = C_phi <omega>/2) gives psi - dt/t_m (psi - <phi>(x_p))
    with x_p the particle's position at the start of the step."""
    mesh = M.box(6, 5, 1.5, 1.0, jitter=0.2, seed=7)
    nn = mesh.n_nodes
    a, b, c, Om, Cphi, dt = 0.3, 1.7, -0.9, 1.3, 2.0, 0.01
    F = CF.frozen_stats_for(mesh, U=(0.0, 0.0, 0.0), R_diag=(0.1, 0.1, 0.1), Om=Om)
    F[4] = a + b * mesh.node_xy[:, 0] + c * mesh.node_xy[:, 1]
    for mode, expect_exact in ((CF.STATS_SHAPE, True), (CF.STATS_ELEM, False)):
        p = CF.params(frozen=1, Cphi=Cphi, stats_mode=mode)
        o = O.Oracle(mesh, p)
        w = CF.Workload("t", mesh, p, dict(ppe=20, seed=11, psi_mode=CF.PSI_BERNOULLI, a=0, b=0, c=0,
                                           U0=F[0:3], R0=F[5:11], Om0=np.full(nn, Om)), dt, 1, "f64")
        o.seed(w.seed)
        o.set_stats(F)
        x0, y0, psi0 = o.state[0].copy(), o.state[1].copy(), o.state[6].copy()
        o.step(dt)
        phi_p = a + b * x0 + c * y0
        expect = psi0 - dt * (0.5 * Cphi * Om) * (psi0 - phi_p)
        err = np.abs(o.state[6] - expect).max()
        if expect_exact:
            assert err < 1e-14
        else:
            assert err > 1e-6  # the element average is the centroid value, not phi(x_p)
