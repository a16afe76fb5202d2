"""Pins for the oracle's elliptic relaxation solve (eq:elliptic-relaxation-
Lagrangian with eq:L, eq:Cxi and the wall condition wp_ij = -4.5 eps n_i n_j):

- a channel between two no-slip walls with uniform statistics: every
  component solves wp - L^2 wp'' = f with constant L and f, whose exact
  solution f + (g - f) cosh((y - 1)/L) / cosh(1/L) the linear elements match
  to second order in the mesh size; L differs between wp_22 (C_xi = 2.3 next
  to walls along x) and the other components (C_xi = 1);
- a doubly periodic square with f = sin(2 pi x) cos(2 pi y) and constant L:
  wp = f / (1 + 8 pi^2 L^2), again to second order;
- L = 0 returns f exactly;
- a step of the generalized Langevin model with the solved wp runs on the
  channel with no-slip walls."""
import math

import numpy as np

import oracle as O
from oracle import elliptic as EL
from synth import configs as CF
from synth import meshes as M


def _uniform_stats(nn, k=1.0, Om=0.5):
    st = np.zeros((O.NSTAT, nn))
    st[3] = Om
    st[5] = st[6] = st[7] = 2.0 * k / 3.0
    return st


def _L(params, k, Om, cxi):
    eps = Om * (k + params["nu"] * params["CT"] ** 2 * Om)
    return params["CL"] * max(cxi * k ** 1.5 / eps, params["Ceta"] * (params["nu"] ** 3 / eps) ** 0.25), eps


def _channel_error(ny):
    mesh = M.uniform_channel(ny // 2, ny, 1.0, 1.0, jitter=0.0, seed=0, wall=M.BC_NOSLIP)  # square cells
    p = CF.params(model=CF.MODEL_GLM, nu=1e-3)
    st = _uniform_stats(mesh.n_nodes)
    f = O.Oracle(mesh, p).local_wp(st)
    wp = EL.solve(mesh, p, st, f)
    y = mesh.node_xy[:, 1]
    errs = {}
    for c, cxi in ((0, 1.0), (4, 2.3), (8, 1.0)):
        L, eps = _L(p, 1.0, 0.5, cxi)  # L = 0.27 and 0.61: resolved by the grids
        g = -4.5 * eps if c == 4 else 0.0
        fc = f[c][0]
        exact = fc + (g - fc) * np.cosh((y - 1.0) / L) / math.cosh(1.0 / L)
        errs[c] = np.abs(wp[c] - exact).max() / abs(g - fc)
    assert np.abs(wp[1]).max() < 1e-14 and np.abs(wp[3]).max() < 1e-14  # f and g vanish off the diagonal
    return errs


def test_channel_cosh_profile_second_order():
    e1, e2 = _channel_error(32), _channel_error(64)
    for c in (0, 4, 8):
        assert e2[c] < 2e-3, (c, e2[c])
        rate = math.log2(e1[c] / e2[c])
        assert 1.7 < rate < 2.3, (c, rate)


def _periodic_error(n, L2=None):
    mesh = M.periodic_square(n)
    p = CF.params(model=CF.MODEL_GLM, nu=1e-3)
    st = _uniform_stats(mesh.n_nodes)
    x, y = mesh.node_xy.T
    shape = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    f = np.stack([(i + 1) * shape for i in range(9)])
    L2e = EL.element_L2(mesh, p, st) if L2 is None else L2
    wp = EL.solve(mesh, p, st, f, L2=L2e)
    L2v = L2e[0, 0, 0]
    return np.abs(wp - f / (1.0 + 8 * np.pi ** 2 * L2v)).max() / 9.0, wp, f


def test_periodic_manufactured_second_order():
    e1, _, _ = _periodic_error(16)
    e2, _, _ = _periodic_error(32)
    assert e2 < 5e-3 and 1.8 < math.log2(e1 / e2) < 2.3


def test_zero_length_scale_returns_f():
    mesh = M.periodic_square(8)
    _, wp, f = _periodic_error(8, L2=np.zeros((mesh.n_elems, 3, 3)))
    np.testing.assert_allclose(wp, f, rtol=0, atol=1e-13)


def test_step_with_solved_wp():
    w = CF.channel(nx=12, n_half=5, ppe=20, precision="f64")
    w.params = dict(w.params, wp_source=CF.WP_ELLIPTIC)
    o = O.Oracle(w.mesh, w.params, gradp=w.gradp)
    o.seed(w.seed)
    f = o.local_wp()
    wp = EL.solve(w.mesh, w.params, o.stats, f)
    assert np.all(np.isfinite(wp)) and not np.allclose(wp, f)
    o.run(w.dt, 3)
    assert np.all(np.isfinite(o.state)) and o.counter_dict()["lost"] == 0
