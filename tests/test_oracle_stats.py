"""Pins for the oracle's statistics (Ch.3, Sec. Estimation of Eulerian
statistics; Sec. Derivatives): exact element means against NumPy group sums,
constant fields, empty elements, linear fields (exact gradients, zero
Laplacian), a quadratic field's Laplacian, and periodic node identification."""
import numpy as np

import oracle as O
from synth import configs as CF
from synth import meshes as M


def _oracle_with_state(mesh, state, elem):
    o = O.Oracle(mesh, CF.params())
    o.state = np.ascontiguousarray(state, np.float64)
    o.elem = np.ascontiguousarray(elem, np.int32)
    o.id = np.arange(state.shape[1], dtype=np.uint32)
    return o


def test_element_moments_match_group_sums():
    mesh = M.graded_channel(6, 4, 6.0, 1.0, 0.1, 0)
    rng = np.random.default_rng(0)
    n = 20000
    elem = rng.integers(0, mesh.n_elems, n)
    state = rng.normal(size=(7, n)) * np.array([1, 1, 2, 3, 4, 0.5, 0.1])[:, None] + 1.5
    o = _oracle_with_state(mesh, state, elem)
    o.estimate()
    N = np.bincount(elem, minlength=mesh.n_elems).astype(float)
    assert np.array_equal(o.elem_stats[0], N)
    means = np.stack([np.bincount(elem, weights=state[f], minlength=mesh.n_elems) for f in range(2, 7)]) / N
    assert np.allclose(o.elem_stats[1:6], means, rtol=1e-13, atol=1e-13)
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2), (4, 4), (0, 4), (1, 4), (2, 4)]
    q = state[2:7]
    for c, (a, b) in enumerate(pairs):
        # E[q_a q_b] - E[q_a]E[q_b] with 1/N normalisation
        cov = np.bincount(elem, weights=q[a] * q[b], minlength=mesh.n_elems) / N - means[a] * means[b]
        assert np.allclose(o.elem_stats[6 + c], cov, rtol=1e-9, atol=1e-12)


def test_constant_property_gives_exact_nodal_values_and_zero_moments():
    mesh = M.canyon(4000, 0.15, 1)
    rng = np.random.default_rng(1)
    n = 30 * mesh.n_elems
    elem = np.repeat(np.arange(mesh.n_elems), 30)
    state = np.zeros((7, n))
    state[0:2] = rng.uniform(size=(2, n))
    state[2:7] = np.array([0.25, -1.5, 2.0, 0.75, 0.5])[:, None]
    o = _oracle_with_state(mesh, state, elem)
    st = o.estimate()
    for f, v in enumerate([0.25, -1.5, 2.0, 0.75, 0.5]):
        assert np.abs(st[f] - v).max() <= 4e-16 * max(1.0, abs(v))
    assert np.abs(st[5:15]).max() == 0.0
    assert np.abs(st[15:24]).max() < 1e-9
    assert np.array_equal(st[24] > 0, np.ones(mesh.n_nodes, bool))


def test_empty_elements_keep_previous_nodal_values():
    mesh = M.box(8, 8, 1.0, 1.0)
    xy = mesh.node_xy
    cent = xy[mesh.elem_nodes].mean(axis=1)
    full = np.nonzero(cent[:, 0] < 0.5)[0]
    elem = np.repeat(full, 5)
    state = np.ones((7, elem.shape[0]))
    o = _oracle_with_state(mesh, state, elem)
    prev = np.full((O.NSTAT, mesh.n_nodes), -7.0)
    o.stats = prev.copy()
    st = o.estimate()
    # nodes touching no populated element keep the previous value (-7); others see 1
    touched = np.zeros(mesh.n_nodes, bool)
    touched[mesh.elem_nodes[full].ravel()] = True
    assert (st[0][touched] == 1.0).all()
    assert (st[0][~touched] == -7.0).all()
    assert (st[24][~touched] == 0).all()


def test_linear_fields_have_exact_gradients_and_zero_laplacian():
    """eq:gradient reproduces the gradient of a linear nodal field exactly in every
    element, hence at every node after averaging; the second pass then sees a
    constant field and returns a zero Laplacian."""
    mesh = M.box(12, 9, 2.0, 1.5, 0.25, 3, M.BC_SLIP, "delaunay")
    om = O.OracleMesh(mesh)
    xy = mesh.node_xy
    st = np.zeros((O.NSTAT, mesh.n_nodes))
    coef = np.array([[0.5, 2.0, -1.0], [1.0, -0.5, 3.0], [-2.0, 0.25, 0.75]])
    for i in range(3):
        st[i] = coef[i, 0] + coef[i, 1] * xy[:, 0] + coef[i, 2] * xy[:, 1]
    out = om.derivatives(st)
    for i in range(3):
        assert np.abs(out[15 + 2 * i] - coef[i, 1]).max() < 1e-12
        assert np.abs(out[16 + 2 * i] - coef[i, 2]).max() < 1e-12
        assert np.abs(out[21 + i]).max() < 1e-9


def test_periodic_linear_in_y_field_on_channel():
    mesh = M.graded_channel(10, 6, 6.0, 1.0, 0.15, 4)
    om = O.OracleMesh(mesh)
    y = mesh.node_xy[:, 1]
    st = np.zeros((O.NSTAT, mesh.n_nodes))
    st[0] = 3.0 * y - 1.0
    out = om.derivatives(st)
    assert np.abs(out[15]).max() < 1e-12
    assert np.abs(out[16] - 3.0).max() < 1e-12
    # identified nodes carry identical values
    m = mesh.node_master
    assert np.array_equal(out[:, m], out)


def test_quadratic_field_laplacian_interior_nodes():
    """Second derivatives by the two-pass procedure on a uniform mesh: for
    q = x^2 + 3 y^2 (Laplacian 8) interior nodes two rings from the boundary
    are exact to rounding."""
    n = 16
    mesh = M.box(n, n, 1.0, 1.0)
    om = O.OracleMesh(mesh)
    xy = mesh.node_xy
    st = np.zeros((O.NSTAT, mesh.n_nodes))
    st[0] = xy[:, 0] ** 2 + 3.0 * xy[:, 1] ** 2
    out = om.derivatives(st)
    h = 1.0 / n
    inner = ((xy[:, 0] > 2.5 * h) & (xy[:, 0] < 1 - 2.5 * h) & (xy[:, 1] > 2.5 * h) & (xy[:, 1] < 1 - 2.5 * h))
    assert inner.sum() > 100
    assert np.abs(out[21][inner] - 8.0).max() < 1e-9
    # first derivatives at interior nodes are the exact ones (symmetric patches)
    inner1 = ((xy[:, 0] > 1.5 * h) & (xy[:, 0] < 1 - 1.5 * h) & (xy[:, 1] > 1.5 * h) & (xy[:, 1] < 1 - 1.5 * h))
    assert np.abs(out[15][inner1] - 2.0 * xy[inner1, 0]).max() < 1e-12
    assert np.abs(out[16][inner1] - 6.0 * xy[inner1, 1]).max() < 1e-12
