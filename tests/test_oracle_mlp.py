"""Pins for the FP64 reference of the denoiser network: analytic gradients
against central finite differences, bfloat16 rounding against exact binary
values, GELU identities, and the nodal features on constant and linear fields."""
import numpy as np
import pytest
from scipy.special import erf

import oracle.mlp as M
from synth import meshes as MS


def _rand(h, B, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=48 * h + h + 2 * (h * h + h) + h * 8 + 8) * 0.3
    return p, rng.normal(size=(B, 48)), rng.normal(size=(B, 8))


@pytest.mark.parametrize("h", [16, 32])
def test_gradient_matches_finite_differences(h):
    p, x, t = _rand(h, 7)
    loss, g = M.loss_and_grad(p, h, x, t)
    rng = np.random.default_rng(1)
    idx = rng.choice(p.size, 40, replace=False)
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (M.loss_and_grad(pp, h, x, t)[0] - M.loss_and_grad(pm, h, x, t)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * (abs(g[i]) + 1e-3)


def test_loss_is_mean_squared_error():
    h = 16
    p, x, t = _rand(h, 5)
    Y, _ = M.forward(p, h, x)
    assert abs(M.loss_and_grad(p, h, x, t)[0] - ((Y - t) ** 2).mean()) < 1e-15


def test_bf16_rounding():
    assert M.bf16(1.0) == 1.0
    assert M.bf16(1.0 + 2.0 ** -8) == 1.0           # tie -> even
    assert M.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie -> even (up)
    assert M.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert M.bf16(-3.0) == -3.0
    x = np.random.default_rng(0).normal(size=1000)
    r = M.bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))  # half an ulp of an 8-bit significand


def test_gelu_identities():
    z = np.linspace(-6, 6, 101)
    assert M.gelu(0.0) == 0.0
    assert np.allclose(M.gelu(z) - M.gelu(-z), z)             # gelu(x) - gelu(-x) = x
    assert np.allclose(M.gelu(z), 0.5 * z * (1 + erf(z / np.sqrt(2))))
    fd = (M.gelu(z + 1e-6) - M.gelu(z - 1e-6)) / 2e-6
    assert np.allclose(M.dgelu(z), fd, atol=1e-8)


def test_features_constant_and_linear_fields():
    mesh = MS.box(6, 5, 1.0, 1.0, 0.2, 3, MS.BC_SLIP, "delaunay")
    st = np.zeros((25, mesh.n_nodes))
    for a, fld in enumerate(M.QUANT):
        st[fld] = 0.5 + a
    F = M.features(mesh, st)
    for a in range(8):
        v = 0.5 + a
        assert np.allclose(F[:, 6 * a + 0], v) and np.allclose(F[:, 6 * a + 1], v)
        assert np.allclose(F[:, 6 * a + 2], 0) and np.allclose(F[:, 6 * a + 3], v)
        assert np.allclose(F[:, 6 * a + 4], v) and np.allclose(F[:, 6 * a + 5], 0)
    xy = mesh.node_xy
    st[0] = 3.0 * xy[:, 0] - 4.0 * xy[:, 1]
    F = M.features(mesh, st)
    assert np.allclose(F[:, 5], 5.0)  # |grad| of a linear field is exact
