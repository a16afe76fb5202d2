"""GPU parity of the wall-function particle condition (eq:wall-normal-velocity
to eq:wall-omega) at PDF_BC_WALLFN edges, through the C ABI, against the
oracle: a streamwise-periodic channel on a uniform grid with wall functions at
both walls, the simplified Langevin model with C0 = 3.5 and the inviscid
particle equations.  FP64 trajectories: element indices bit-exact, state and
statistics within 1e-12, equal reflection counts; one FP32 step (1e-5); the
parameter checks of such meshes."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from synth import configs as CF
from tests.parity import compare_elements, compare_state, compare_stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_0720_amd import _lib
    return _lib


def _pair(w):
    from paper_1006_0720_amd.runner import workload_context

    print(f"[wallfn] {w.name} np={w.n_particles} prec={w.precision} frozen={w.params['frozen']}", flush=True)
    ctx = workload_context(w)
    o = O.Oracle(w.mesh, w.params, store_fp32=(w.precision == "f32"), gradp=w.gradp, wp=w.wp)
    o.seed(w.seed)
    return ctx, o


@pytest.mark.parametrize("frozen", [0, 1])
def test_wallfn_channel_trajectory_fp64(L, frozen):
    w = CF.channel_wallfn(nx=20, n_half=6, ppe=30)
    w.params = dict(w.params, frozen=frozen)
    ctx, o = _pair(w)
    for c in range(2):
        ctx.advance(10, w.dt)
        o.run(w.dt, 10)
        st, el, pid = ctx.particles()
        assert np.array_equal(pid, o.id)
        assert np.array_equal(el, o.elem), f"chunk {c}: {(el != o.elem).sum()} element mismatches"
        compare_state(st, o.state, w.mesh, 1e-12, f"wall functions, chunk {c}", elem=o.elem)
        compare_stats(ctx.stats(), o.est if frozen else o.stats, 1e-12, what=f"wall functions, chunk {c}")
    g, oc = ctx.counters(), o.counter_dict()
    for k in ("walk_steps", "reflect", "periodic", "lost", "noslip_b"):
        assert g[k] == oc[k], (k, g[k], oc[k])
    assert oc["reflect"] > 50 and oc["noslip_b"] == 0
    ctx.close()


def test_wallfn_fp32_one_step(L):
    w = CF.channel_wallfn(nx=20, n_half=6, ppe=60, precision="f32")
    ctx, o = _pair(w)
    ctx.advance(1, w.dt)
    o.step(w.dt)
    st, el, _ = ctx.particles()
    compare_elements(el, st, o.elem, o.state, w.mesh, "wall functions fp32 step", fp32=True)
    compare_state(st, o.state, w.mesh, 1e-5, "wall functions fp32 step", elem=o.elem)
    assert ctx.counters()["reflect"] == o.counter_dict()["reflect"] > 0
    ctx.close()


def test_wallfn_parameter_checks(L):
    w = CF.channel_wallfn(nx=8, n_half=3, ppe=4)
    for bad in (dict(nu=1e-3), dict(nu_wall=0.0), dict(nu_wall=float("nan"))):
        with pytest.raises(L.PdfError) as ei:
            L.Context(w.mesh, dict(w.params, **bad))
        assert ei.value.status == 1, bad
    # the same mesh with no-slip walls needs neither
    from synth import meshes as M

    bt = np.where(w.mesh.bedge_type == M.BC_WALLFN, M.BC_NOSLIP, w.mesh.bedge_type).astype(np.int32)
    L.Context(dataclasses.replace(w.mesh, bedge_type=bt), dict(w.params, nu=1e-3, nu_wall=0.0)).close()
