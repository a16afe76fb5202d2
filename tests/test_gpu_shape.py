"""GPU parity of the SHAPE statistics mode (nodal statistics interpolated at
the particle by the shape functions of eq:approximation; node values as
N^j-weighted particle moments) against the FP64 oracle, through the C ABI.
Same bars as the ELEM mode: element indices bit-exact, FP64 state and nodal
statistics within 1e-12, FP32 one step within 1e-5."""
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


def _shape(w):
    w.params = dict(w.params, stats_mode=CF.STATS_SHAPE)
    return w


def _pair(w, reorder_every=0):
    from paper_1006_0720_amd.runner import workload_context

    print(f"[shape] {w.name} np={w.n_particles} prec={w.precision}", flush=True)
    ctx = workload_context(w, reorder_every=reorder_every)
    o = O.Oracle(w.mesh, w.params, store_fp32=(w.precision == "f32"), gradp=w.gradp, wp=w.wp)
    o.seed(w.seed)
    return ctx, o


def _check(ctx, o, w, rtol, what):
    st, el, pid = ctx.particles()
    assert np.array_equal(pid, o.id)
    assert np.array_equal(el, o.elem), f"{what}: {(el != o.elem).sum()} element mismatches"
    compare_state(st, o.state, w.mesh, rtol, what, elem=o.elem)
    compare_stats(ctx.stats(), o.stats, rtol, what=what)


@pytest.mark.parametrize("reorder", [0, 4])
def test_shape_trajectory_fp64_periodic_square(L, reorder):
    w = _shape(CF.periodic_square())
    ctx, o = _pair(w, reorder)
    _check(ctx, o, w, 1e-12, "shape seed")
    for chunk in range(2):
        ctx.advance(20, w.dt)
        o.run(w.dt, 20)
        _check(ctx, o, w, 1e-12, f"shape step {20 * (chunk + 1)}")
    c, oc = ctx.counters(), o.counter_dict()
    for k in ("walk_steps", "periodic", "omega_clamp", "empty_node", "lost"):
        assert c[k] == oc[k], (k, c[k], oc[k])
    ctx.close()


def test_shape_trajectory_fp64_channel_glm_walls(L):
    w = _shape(CF.channel(nx=20, n_half=8, ppe=30, steps=20, precision="f64"))
    ctx, o = _pair(w)
    for chunk in range(2):
        ctx.advance(10, w.dt)
        o.run(w.dt, 10)
        _check(ctx, o, w, 1e-12, f"shape channel step {10 * (chunk + 1)}")
    c, oc = ctx.counters(), o.counter_dict()
    for k in ("walk_steps", "reflect", "noslip_b", "periodic", "gamma_fail", "lost"):
        assert c[k] == oc[k], (k, c[k], oc[k])
    assert oc["reflect"] > 0
    ctx.close()


def test_shape_trajectory_fp64_canyon_corners(L):
    mesh = M.canyon(3000, 0.15, 2)
    w = _shape(CF.canyon(mesh=mesh, ppe=20, precision="f64", steps=20))
    ctx, o = _pair(w, 4)
    for chunk in range(2):
        ctx.advance(10, w.dt)
        o.run(w.dt, 10)
        _check(ctx, o, w, 1e-12, f"shape canyon step {10 * (chunk + 1)}")
    ctx.close()


def test_shape_kernel_fp32_channel(L):
    w = _shape(CF.channel(nx=30, n_half=10, ppe=60, steps=1, precision="f32"))
    ctx, o = _pair(w)
    st, el, _ = ctx.particles()
    assert np.array_equal(el, o.elem)
    compare_stats(ctx.stats(), o.stats, 1e-5, what="shape fp32 seed stats")
    ctx.advance(1, w.dt)
    o.step(w.dt)
    st, el, _ = ctx.particles()
    compare_elements(el, st, o.elem, o.state, w.mesh, "shape fp32 step", fp32=True)
    compare_state(st, o.state, w.mesh, 1e-5, "shape fp32 step", elem=o.elem)
    compare_stats(ctx.stats(), o.stats, 1e-5, what="shape fp32 step stats")
    ctx.close()


def test_shape_mode_has_no_element_statistics(L):
    w = _shape(CF.periodic_square(n=8, ppe=10))
    ctx, _ = _pair(w)
    with pytest.raises(L.PdfError):
        ctx.stats(elem=True)
    ctx.close()
