"""Pins for the oracle's wall-function particle condition (eq:wall-normal-
velocity, eq:particle-wallcondition-wf, eq:alpha, eq:hatu, eq:Ue,
eq:friction-velocity, eq:wall-omega):

- an equilibrium worked example: with <U>_p equal to the log-law U_e, a
  friction velocity of 1 and <v^2>_p = 2, alpha is 1, the value that makes the
  reflected particles carry the wall shear u_tau^2 = alpha <v^2>_p / 2;
- the frequency factor exp(-beta) at V_I = -y_p <omega> with the paper's
  constants (C0 = 3.5, C3 = 5, C_w1 = 0.5, C_w2 = 0.73);
- limits: no mean velocity gives a plain specular reflection; the change of
  the tangential velocity scales with <U>_p |<U>_p| and 1 / <v^2>_p; the
  pressure-gradient term of u_tau enters only when <uv> dP/dx > 0;
- invariances: a rotation of the whole configuration rotates the result;
  a mirror image (edge reversed) gives the mirrored result; the normal
  velocity reverses exactly and the spanwise one is kept;
- in a step, a particle crossing a wall-function edge gets this condition."""
import ctypes as C
import math

import numpy as np
import pytest

import oracle as O
from synth import configs as CF
from synth import meshes as M

KAPPA, E_ROUGH, CMU = 0.41, 8.5, 0.09


def _stats(U=(10.0, 0.0), R=(8.0 / 3.0, 2.0, 2.0, 0.0), Om=5.0, nn=1):
    st = np.zeros((O.NSTAT, nn))
    st[0], st[1], st[3] = U[0], U[1], Om
    st[5], st[6], st[7], st[8] = R
    return st


def _apply(p, st, gp, xa, ya, xb, yb, xc, yc, u, v, w, om):
    u_, v_, w_, om_ = (C.c_double(x) for x in (u, v, w, om))
    st = np.ascontiguousarray(st, np.float64)
    gpp = None if gp is None else O._p(np.ascontiguousarray(gp, np.float64), C.c_double)
    O.lib().or_wall_function(C.byref(p), st.shape[1], O._p(st, C.c_double), gpp, 0, xa, ya, xb, yb, xc, yc,
                             C.byref(u_), C.byref(v_), C.byref(w_), C.byref(om_))
    return np.array([u_.value, v_.value, w_.value, om_.value])


def _params(nu_wall, **kw):
    return O._params(CF.params(C0=3.5, nu_wall=nu_wall, **kw), False)


def test_equilibrium_worked_example():
    """Wall along x from (0,0) to (1,0) (domain above), first gridpoint at
    y_p = 0.1.  k_p = 1/0.3 so that u_hat^2 = sqrt(0.09) k_p = 1 and, with no
    pressure gradient, u_tau = 1; nu is chosen so that E y_p u_tau / nu =
    exp(4.1), hence U_e = 4.1 / 0.41 = 10 = <U>_p; <v^2>_p = 2.  Then alpha =
    2 * 1 * 10 * 10 / (2 * 100) = 1: an incident (7, -3) leaves as (4, 3)."""
    yp = 0.1
    nu = E_ROUGH * yp / math.exp(4.1)
    st = _stats(U=(10.0, 0.0), R=(8.0 / 3.0, 2.0, 2.0, 0.0))
    out = _apply(_params(nu), st, None, 0.0, 0.0, 1.0, 0.0, 0.5, yp, 7.0, -3.0, 0.7, 1.0)
    np.testing.assert_allclose(out[:3], [4.0, 3.0, 0.7], rtol=1e-13, atol=1e-13)


def test_frequency_factor():
    yp, Om = 0.1, 5.0
    st = _stats(U=(0.0, 0.0), Om=Om)
    beta = -2.0 / (0.5 + 0.75 * 3.5 + 5.0 + 0.73 - 0.5)  # -2 / 8.355
    out = _apply(_params(1e-3), st, None, 0.0, 0.0, 1.0, 0.0, 0.3, yp, 1.0, -yp * Om, 0.0, 2.0)
    assert out[3] == pytest.approx(2.0 * math.exp(-beta), rel=1e-14)
    assert out[3] == pytest.approx(2.0 * 1.2704582, rel=1e-6)  # exp(2 / 8.355)


def test_limits():
    p = _params(1e-3)
    # no mean velocity: specular reflection
    out = _apply(p, _stats(U=(0.0, 0.0)), None, 0.0, 0.0, 1.0, 0.0, 0.5, 0.1, 2.0, -1.5, 0.3, 1.0)
    np.testing.assert_allclose(out[:3], [2.0, 1.5, 0.3], rtol=0, atol=1e-15)
    # the tangential change scales with <U>|<U>| at fixed U_e (k, <v^2>, y_p fixed)
    d = []
    for U in (3.0, 6.0, -3.0):
        o = _apply(p, _stats(U=(U, 0.0)), None, 0.0, 0.0, 1.0, 0.0, 0.5, 0.1, 2.0, -1.5, 0.0, 1.0)
        d.append(o[0] - 2.0)
        assert o[1] == pytest.approx(1.5, abs=1e-15)
    assert d[0] < 0 and d[1] == pytest.approx(4 * d[0], rel=1e-12) and d[2] == pytest.approx(-d[0], rel=1e-12)
    # ... and with 1 / <v^2>_p (k kept)
    o1 = _apply(p, _stats(U=(3.0, 0.0), R=(3.0, 1.0, 2.0, 0.0)), None, 0, 0, 1, 0, 0.5, 0.1, 2.0, -1.5, 0, 1)
    o2 = _apply(p, _stats(U=(3.0, 0.0), R=(2.0, 2.0, 2.0, 0.0)), None, 0, 0, 1, 0, 0.5, 0.1, 2.0, -1.5, 0, 1)
    assert (o1[0] - 2.0) == pytest.approx(2.0 * (o2[0] - 2.0), rel=1e-12)


def test_pressure_gradient_term_only_when_uv_dpdx_positive():
    p = _params(1e-3)
    base = dict(xa=0.0, ya=0.0, xb=1.0, yb=0.0, xc=0.5, yc=0.1, u=2.0, v=-1.5, w=0.0, om=1.0)
    def run(R12, dPdx):
        st = _stats(U=(5.0, 0.0), R=(2.0, 1.0, 1.5, R12))
        gp = np.array([[dPdx], [0.0]])
        return _apply(p, st, gp, *base.values())
    ref = run(-0.4, 0.0)
    np.testing.assert_array_equal(run(-0.4, 2.0), ref)  # <uv> dP/dx < 0: gamma_tau = 0
    assert not np.array_equal(run(-0.4, -2.0), ref)      # <uv> dP/dx > 0: the term enters


def _rot(th, x, y):
    c, s = math.cos(th), math.sin(th)
    return c * x - s * y, s * x + c * y


def test_rotation_and_mirror_invariance():
    p = _params(2e-3)
    U, R, gpv = (6.0, 0.4), (2.0, 1.0, 1.5, -0.3), (-0.8, 0.2)
    inc = (3.0, -2.0)
    ref = _apply(p, _stats(U=U, R=R), np.array([[gpv[0]], [gpv[1]]]), 0.0, 0.0, 1.0, 0.0, 0.4, 0.15,
                 inc[0], inc[1], 0.5, 1.3)
    for th in (0.3, 1.7, -2.4):
        Ur = _rot(th, *U)
        Rm = np.array([[R[0], R[3]], [R[3], R[1]]])
        Q = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        Rr = Q @ Rm @ Q.T
        gr = _rot(th, *gpv)
        a, b, c_ = _rot(th, 0.0, 0.0), _rot(th, 1.0, 0.0), _rot(th, 0.4, 0.15)
        ir = _rot(th, *inc)
        out = _apply(p, _stats(U=Ur, R=(Rr[0, 0], Rr[1, 1], R[2], Rr[0, 1])), np.array([[gr[0]], [gr[1]]]),
                     *a, *b, *c_, ir[0], ir[1], 0.5, 1.3)
        np.testing.assert_allclose(out[:2], _rot(th, ref[0], ref[1]), rtol=1e-12, atol=1e-12)
        assert out[2] == 0.5 and out[3] == pytest.approx(ref[3], rel=1e-12)
    # mirror x -> -x: the edge is reversed so that the domain stays on its left
    out = _apply(p, _stats(U=(-U[0], U[1]), R=(R[0], R[1], R[2], -R[3])), np.array([[-gpv[0]], [gpv[1]]]),
                 -1.0, 0.0, 0.0, 0.0, -0.4, 0.15, -inc[0], inc[1], 0.5, 1.3)
    np.testing.assert_allclose(out, [-ref[0], ref[1], ref[2], ref[3]], rtol=1e-12, atol=1e-12)
    # the normal velocity reverses exactly
    assert ref[1] == -inc[1]


def test_step_applies_the_condition_at_wall_function_edges():
    """A channel whose walls use wall functions, 20 steps: particles reflect
    at the walls and none is lost; the trajectory (b) test of no-slip walls
    does not apply; the mean velocity near the walls stays positive."""
    w = CF.channel_wallfn(nx=12, n_half=5, ppe=40)
    o = O.Oracle(w.mesh, w.params, gradp=w.gradp)
    o.seed(w.seed)
    o.run(w.dt, 20)
    c = o.counter_dict()
    assert c["reflect"] > 0 and c["lost"] == 0 and c["noslip_b"] == 0
    assert np.all(np.isfinite(o.state))
    near = np.minimum(o.state[1], 2.0 - o.state[1]) < 0.2
    assert o.state[2][near].mean() > 0.0
