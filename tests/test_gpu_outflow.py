"""GPU parity of the outflow relocation (PDF_BC_OUTFLOW; Ch.6, cylinder
flow, Sec. Results: its boundary conditions) through the C ABI against the
oracle: the GLM channel with walls whose periodic edges at x = 6 are outflow
edges, particles leaving there relocated at the inflow with the velocity
(inflow_u, 0, 0).  FP64 trajectories: element indices bit-exact, state and
nodal statistics within 1e-12, equal event counts with relocations
happening; one FP32 step within 1e-5; parameter checks."""
import numpy as np
import pytest

import oracle as O
from synth import configs as CF
from synth import meshes as M
from tests.parity import compare_elements, compare_state, compare_stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_0720_amd import _lib
    return _lib


def _workload(precision):
    w = CF.channel(nx=20, n_half=8, ppe=30, steps=20, precision=precision)
    w.mesh = M.with_outflow(w.mesh)
    w.params = dict(w.params, inflow_u=15.0)
    return w


def _pair(w):
    from paper_1006_0720_amd.runner import workload_context

    print(f"[outflow] {w.mesh.name} np={w.n_particles} prec={w.precision}", flush=True)
    ctx = workload_context(w)
    o = O.Oracle(w.mesh, w.params, store_fp32=(w.precision == "f32"), gradp=w.gradp, wp=w.wp)
    o.seed(w.seed)
    return ctx, o


def test_outflow_trajectory_fp64(L):
    w = _workload("f64")
    ctx, o = _pair(w)
    for chunk in range(2):
        ctx.advance(10, w.dt)
        o.run(w.dt, 10)
        st, el, pid = ctx.particles()
        assert np.array_equal(pid, o.id)
        assert np.array_equal(el, o.elem), f"step {10 * (chunk + 1)}: {(el != o.elem).sum()} element mismatches"
        compare_state(st, o.state, w.mesh, 1e-12, f"outflow step {10 * (chunk + 1)}", elem=o.elem)
        compare_stats(ctx.stats(), o.stats, 1e-12, what=f"outflow step {10 * (chunk + 1)}")
    c, oc = ctx.counters(), o.counter_dict()
    print(f"[outflow] relocated {c['outflow']}, periodic {c['periodic']}", flush=True)
    for k in ("walk_steps", "reflect", "noslip_b", "periodic", "outflow", "lost"):
        assert c[k] == oc[k], (k, c[k], oc[k])
    assert oc["outflow"] > 0
    # relocated particles sit near the inflow carrying the inflow velocity
    # unless a wall condition or later steps changed it: at least one does
    st, el, pid = ctx.particles()
    assert np.any((st[0] < 0.5) & (st[2] == 15.0) & (st[3] == 0.0) & (st[4] == 0.0))
    ctx.close()


def test_outflow_kernel_fp32(L):
    w = _workload("f32")
    ctx, o = _pair(w)
    ctx.advance(5, w.dt)
    st0, el0, pid0 = ctx.particles()
    stats0 = ctx.stats()
    ctx.advance(1, w.dt)
    st1, el1, pid1 = ctx.particles()
    o.state, o.elem, o.id = st0, el0, pid0
    o.step_index = 5
    o.set_stats(stats0)
    o.step(w.dt)
    nd = compare_elements(el1, st1, o.elem, o.state, w.mesh, "outflow fp32 step", fp32=True)
    compare_state(st1, o.state, w.mesh, 1e-5, "outflow fp32 step", elem=o.elem)
    assert ctx.counters()["outflow"] > 0
    ctx.close()


def test_outflow_parameter_and_mesh_checks(L):
    w = _workload("f64")
    with pytest.raises(L.PdfError) as ei:
        L.Context(w.mesh, dict(w.params, inflow_u=float("nan")))
    assert ei.value.status == 1
    # an outflow edge paired with another outflow edge is refused
    import dataclasses
    bt = w.mesh.bedge_type.copy()
    bt[bt == M.BC_PERIODIC] = M.BC_OUTFLOW
    bad = dataclasses.replace(w.mesh, bedge_type=bt)
    with pytest.raises(L.PdfError) as ei:
        L.Context(bad, w.params)
    assert ei.value.status == 2 and "partner" in str(ei.value)
