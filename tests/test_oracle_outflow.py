"""Oracle pin of the outflow relocation (Ch.6, cylinder flow, Sec. Results:
its boundary conditions): a particle leaving through an outflow edge is put
back at the inflow with its cross-stream position kept and its velocity set
to (U0, 0, 0); nothing else about the step changes.

The pin compares two oracle runs from the same particles and noise: on a
streamwise-periodic channel, and on the same channel with the periodic edges
at the largest x turned into outflow edges.  Positions, elements, frequencies
and scalars must agree bit for bit (the relocation is the periodic
translation), the particle that left through the outflow must carry exactly
(U0, 0, 0), every other velocity must agree, and a particle leaving upstream
through the inflow edge is treated periodically in both runs."""
import numpy as np

import oracle as O
from synth import configs as CF
from synth import meshes as M


def _particles(mesh, Lx):
    pts = [(Lx - 0.01, 1.0, 2.0),    # leaves through the outflow within the step
           (0.01, 0.9, -2.0),        # leaves upstream through the inflow
           (3.0, 1.1, 1.0)]          # stays inside
    om = O.OracleMesh(mesh)
    n = len(pts)
    state = np.zeros((7, n))
    for j, (x, y, u) in enumerate(pts):
        state[:, j] = (x, y, u, 0.0, 0.0, 1.3, 0.4)
    elem = np.array([om.locate_brute(x, y) for x, y, _ in pts], np.int32)
    assert (elem >= 0).all()
    return state, elem, np.arange(n, dtype=np.uint32)


def _step(mesh, params, state, elem, pid, dt):
    o = O.Oracle(mesh, params)
    o.state, o.elem, o.id = state.copy(), elem.copy(), pid.copy()
    o.seed_value = 7
    o.step_index = 3
    o.set_stats(CF.frozen_stats_for(mesh, U=(1.0, 0.0, 0.0), R_diag=(0.5, 0.4, 0.3), Om=1.0, Phi=0.5))
    o.step(dt)
    return o


def test_outflow_relocation_is_the_periodic_step_with_the_inflow_velocity():
    Lx, U0, dt = 6.0, 7.5, 0.01
    per = M.graded_channel(nx=20, n_half=8, Lx=Lx)
    out = M.with_outflow(per)
    params = CF.params(frozen=1, inflow_u=U0)
    state, elem, pid = _particles(per, Lx)
    a = _step(per, params, state, elem, pid, dt)
    b = _step(out, params, state, elem, pid, dt)
    assert np.array_equal(a.elem, b.elem)
    for f in (0, 1, 5, 6):  # x, y, omega, psi
        assert np.array_equal(a.state[f], b.state[f]), f
    # particle 0 left through the outflow: back at the inflow, y kept
    assert b.state[0, 0] == (state[0, 0] + state[2, 0] * dt) - Lx
    assert b.state[1, 0] == state[1, 0]
    assert (b.state[2:5, 0] == (U0, 0.0, 0.0)).all()
    assert not np.allclose(a.state[2:5, 0], (U0, 0.0, 0.0))
    # the others keep the velocities of the periodic run
    assert np.array_equal(a.state[2:5, 1:], b.state[2:5, 1:])
    # particle 1 left upstream: periodic in both runs, to the outflow side
    assert b.state[0, 1] > Lx - 0.05
    ca, cb = a.counter_dict(), b.counter_dict()
    assert ca["periodic"] == 2 and ca["outflow"] == 0
    assert cb["periodic"] == 1 and cb["outflow"] == 1
