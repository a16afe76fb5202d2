"""Pins for the oracle's initial particle state (Ch.3, Sec. Particle-number
control): equal counts per element, uniform positions, Gaussian velocities with
the prescribed covariance, gamma frequencies, and the scalar initial
conditions.  Independent checks use NumPy/SciPy, not the oracle's formulas."""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from synth import configs as CF
from synth import meshes as M


def _bary(mesh, elem, x, y):
    """Area coordinates by solving the 2x2 affine system (numpy.linalg)."""
    p = mesh.node_xy[mesh.elem_nodes[elem]]
    T = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]], axis=2)  # (n,2,2) columns B-A, C-A
    rhs = np.stack([x, y], 1) - p[:, 0]
    lb = np.linalg.solve(T, rhs[..., None])[..., 0]
    return np.stack([1.0 - lb[:, 0] - lb[:, 1], lb[:, 0], lb[:, 1]], 1)


def _seed(mesh, U0, R0, Om0, ppe=40, psi_mode=0, a=0.0, b=0.0, c=0.0, seed=3, **pk):
    o = O.Oracle(mesh, CF.params(**pk))
    o.seed(dict(ppe=ppe, seed=seed, psi_mode=psi_mode, a=a, b=b, c=c, U0=U0, R0=R0, Om0=Om0))
    return o


def test_counts_ids_and_uniform_positions():
    mesh = M.graded_channel(12, 6, 6.0, 1.0, 0.15, 1)
    nn = mesh.n_nodes
    U0, R0, Om0 = CF._iso(nn)
    o = _seed(mesh, U0, R0, Om0, ppe=60)
    ne = mesh.n_elems
    assert np.array_equal(np.bincount(o.elem, minlength=ne), np.full(ne, 60))
    assert np.array_equal(o.id, np.arange(ne * 60, dtype=np.uint32))
    assert np.array_equal(o.elem, np.repeat(np.arange(ne), 60))
    lam = _bary(mesh, o.elem, o.state[0], o.state[1])
    assert lam.min() > -1e-12
    # uniform in a triangle <=> each area coordinate ~ Beta(1, 2)
    for k in range(3):
        assert stats.kstest(lam[:, k], stats.beta(1, 2).cdf).pvalue > 1e-3


def test_velocity_covariance_and_gaussianity():
    mesh = M.periodic_square(8)
    nn = mesh.n_nodes
    R = np.array([[1.0, 0.5, 0.2], [0.5, 2.0, 0.3], [0.2, 0.3, 1.5]])
    U0 = np.zeros((3, nn))
    U0[0] = 2.0
    R0 = np.zeros((6, nn))
    for f, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        R0[f] = R[i, j]
    o = _seed(mesh, U0, R0, np.ones(nn), ppe=400)
    u = o.state[2:5]
    n = u.shape[1]
    assert np.allclose(u.mean(1), [2.0, 0.0, 0.0], atol=5 * np.sqrt(2.0 / n))
    C = np.cov(u)
    assert np.allclose(C, R, atol=6 * np.sqrt(2.0 * 4.0 / n))
    # standardised components are N(0,1)
    L = np.linalg.cholesky(R)
    z = np.linalg.solve(L, u - np.array([[2.0], [0.0], [0.0]]))
    for k in range(3):
        assert stats.kstest(z[k], "norm").pvalue > 1e-3


def test_linear_mean_velocity_is_reproduced_exactly():
    """Shape functions reproduce linear fields (eq:approximation): with zero
    Reynolds stress the seeded velocity equals the linear field at the point."""
    mesh = M.graded_channel(10, 5, 6.0, 1.0, 0.15, 2)
    xy = mesh.node_xy
    U0 = np.stack([1.0 + 2.0 * xy[:, 0] - 0.5 * xy[:, 1], 3.0 * xy[:, 1], -xy[:, 0] + 0.25])
    o = _seed(mesh, U0, np.zeros((6, mesh.n_nodes)), np.ones(mesh.n_nodes), ppe=20)
    x, y = o.state[0], o.state[1]
    ref = np.stack([1.0 + 2.0 * x - 0.5 * y, 3.0 * y, -x + 0.25])
    assert np.abs(o.state[2:5] - ref).max() < 1e-13


def test_frequency_is_gamma_with_mean_om_and_variance_c4_om2():
    mesh = M.periodic_square(8)
    nn = mesh.n_nodes
    U0, R0, _ = CF._iso(nn)
    o = _seed(mesh, U0, R0, np.full(nn, 2.0), ppe=300, C4=0.25)
    om = o.state[5]
    # Gamma(shape 1/C4, scale C4*Om): mean Om, variance C4 Om^2 (Sec. Particle-number control)
    assert stats.kstest(om, stats.gamma(4.0, scale=0.5).cdf).pvalue > 1e-3


def test_scalar_initial_conditions():
    mesh = M.periodic_square(8)
    nn = mesh.n_nodes
    U0, R0, Om0 = CF._iso(nn)
    o = _seed(mesh, U0, R0, Om0, ppe=50, psi_mode=CF.PSI_STEP_X, a=0.5)
    assert np.array_equal(o.state[6], (o.state[0] < 0.5).astype(float))
    o = _seed(mesh, U0, R0, Om0, ppe=50, psi_mode=CF.PSI_GAUSS_X, a=0.5, b=0.1)
    assert np.allclose(o.state[6], np.exp(-(o.state[0] - 0.5) ** 2 / 0.02), rtol=1e-14)
    o = _seed(mesh, U0, R0, Om0, ppe=200, psi_mode=CF.PSI_BERNOULLI)
    n = o.state.shape[1]
    assert set(np.unique(o.state[6])) == {0.0, 1.0}
    assert abs(o.state[6].mean() - 0.5) < 5 * 0.5 / np.sqrt(n)


def test_fp32_storage_mode_rounds_state():
    mesh = M.periodic_square(8)
    nn = mesh.n_nodes
    U0, R0, Om0 = CF._iso(nn, (1.0, 0.0, 0.0), 0.01)
    o64 = _seed(mesh, U0, R0, Om0, ppe=10)
    o32 = O.Oracle(mesh, CF.params(), store_fp32=True)
    o32.seed(dict(ppe=10, seed=3, psi_mode=0, U0=U0, R0=R0, Om0=Om0))
    assert np.array_equal(o32.state, o32.state.astype(np.float32).astype(np.float64))
    assert np.array_equal(o32.state, o64.state.astype(np.float32).astype(np.float64))
