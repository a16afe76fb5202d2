"""GPU parity of the particle redistribution (App. D) against the oracle,
through the C ABI: on a grid stretched toward a slip wall, elements drain and
are refilled every step (copies of residents, uniform positions in empty
elements).  Element indices bit-exact, FP64 state and statistics within
1e-12, the number of particles moved equal."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from synth import configs as CF
from synth import meshes as M
from tests.parity import compare_derivatives, compare_elements, compare_state, compare_stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_0720_amd import _lib
    return _lib


def _workload(power=2.5, ppe=20, min_ppe=4, precision="f64", stats_mode=CF.STATS_ELEM, frozen=1):
    m = M.box(16, 32, 1.0, 1.0, jitter=0.0, seed=0, bc=M.BC_SLIP)
    xy = m.node_xy.copy()
    xy[:, 1] = xy[:, 1] ** power
    mesh = dataclasses.replace(m, node_xy=xy)
    fz = CF.frozen_stats_for(mesh, U=(0.3, 0.0, 0.0), R_diag=(0.5, 0.4, 0.3), Om=1.0)
    p = CF.params(frozen=frozen, min_ppe=min_ppe, stats_mode=stats_mode)
    seed = dict(ppe=ppe, seed=4, psi_mode=CF.PSI_STEP_X, a=0.5, b=0, c=0, U0=fz[0:3], R0=fz[5:11], Om0=fz[3])
    return CF.Workload(f"stretched_box_redist_{precision}", mesh, p, seed, 0.01, 1, precision), fz


def _pair(w, fz, reorder_every=0):
    from paper_1006_0720_amd import _lib
    from paper_1006_0720_amd.runner import workload_context

    print(f"[redist] {w.name} np={w.n_particles} min_ppe={w.params['min_ppe']}", flush=True)
    ctx = workload_context(w, reorder_every=reorder_every)
    o = O.Oracle(w.mesh, w.params, store_fp32=(w.precision == "f32"))
    o.seed(w.seed)
    if w.params["frozen"]:
        ctx.set_nodal_field(_lib.FIELD_STATS, fz)
        o.set_stats(fz)
    return ctx, o


def _check(ctx, o, w, rtol, what, stats=True):
    st, el, pid = ctx.particles()
    assert np.array_equal(pid, o.id)
    assert np.array_equal(el, o.elem), f"{what}: {(el != o.elem).sum()} element mismatches"
    compare_state(st, o.state, w.mesh, rtol, what, elem=o.elem)
    if stats:
        compare_stats(ctx.stats(), o.est if w.params["frozen"] else o.stats, rtol, what=what)


@pytest.mark.parametrize("reorder", [0, 4])
def test_redistribution_trajectory_fp64(L, reorder):
    w, fz = _workload()
    ctx, o = _pair(w, fz, reorder)
    for chunk in range(3):
        ctx.advance(10, w.dt)
        o.run(w.dt, 10)
        _check(ctx, o, w, 1e-12, f"redistribution step {10 * (chunk + 1)}")
    c, oc = ctx.counters(), o.counter_dict()
    assert oc["redist"] > 100 and c["redist"] == oc["redist"], (c["redist"], oc["redist"])
    assert c["lost"] == oc["lost"] == 0
    ctx.close()


def test_redistribution_fed_back_shape_fp64(L):
    """Fed-back SHAPE statistics with redistribution.  The estimated moments
    (fields 0-14, 24) are held to 1e-12; their FEM first and second
    derivatives (15-23) to the bound that the measured discrepancy of the
    nodal means implies through the derivative operator on this grid (element
    sizes from 1e-3 to 6e-2 amplify it by up to P/(2A) per derivative), see
    tests/parity.derivative_bounds."""
    w, fz = _workload(power=2.0, ppe=16, min_ppe=5, stats_mode=CF.STATS_SHAPE, frozen=0)
    ctx, o = _pair(w, fz)
    ctx.advance(15, w.dt)
    o.run(w.dt, 15)
    _check(ctx, o, w, 1e-12, "redistribution, SHAPE, fed back", stats=False)
    g = ctx.stats()
    compare_stats(g, o.stats, 1e-12, fields=list(range(15)) + [24], what="SHAPE fed back, moments")
    r1, r2 = compare_derivatives(w.mesh, g, o.stats, what="SHAPE fed back, derivatives")
    print(f"[redist] derivative discrepancy / bound: first {r1:.3g}, Laplacian {r2:.3g}", flush=True)
    assert ctx.counters()["redist"] == o.counter_dict()["redist"] > 0
    ctx.close()


def test_redistribution_kernel_fp32(L):
    """FP32 state: 20 steps on the oracle to drain elements, then the GPU is
    given that state and both take one step with redistribution."""
    w, fz = _workload(precision="f32", min_ppe=0)
    o = O.Oracle(w.mesh, w.params, store_fp32=True)
    o.seed(w.seed)
    o.set_stats(fz)
    o.run(w.dt, 20)
    from paper_1006_0720_amd.runner import workload_context

    w.params = dict(w.params, min_ppe=6)
    ctx = workload_context(w)
    ctx.set_particles(o.state, o.elem, o.id)
    ctx.set_nodal_field(L.FIELD_STATS, fz)
    ctx.advance(20, w.dt)  # advances the GPU step counter to the oracle's
    ctx.set_particles(o.state, o.elem, o.id)
    ctx.set_nodal_field(L.FIELD_STATS, fz)
    ctx.counters(reset=True)
    o2 = O.Oracle(w.mesh, w.params, store_fp32=True)
    o2.state, o2.elem, o2.id = o.state.copy(), o.elem.copy(), o.id.copy()
    o2.seed_value, o2.step_index = o.seed_value, o.step_index
    o2.set_stats(fz)
    assert o2.step_index == 20
    ctx.advance(1, w.dt)
    o2.step(w.dt)
    st, el, pid = ctx.particles()
    compare_elements(el, st, o2.elem, o2.state, w.mesh, "redistribution fp32 step", fp32=True)
    compare_state(st, o2.state, w.mesh, 1e-5, "redistribution fp32 step", elem=o2.elem)
    assert ctx.counters()["redist"] == o2.counter_dict()["redist"] > 0
    ctx.close()
