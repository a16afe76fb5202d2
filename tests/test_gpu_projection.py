"""GPU parity of the stabilized mean-pressure projection (eq:pressure-
projection-smooth, eq:velocity-correction on the particles) through the C
ABI, against the oracle's exact sparse solve.

The solve is iterative: with the conjugate gradients stopped at 1e-14 of the
right-hand side, FP64 trajectories are held to 1e-11 (element indices
bit-exact) and the solved pressure P' to 1e-9 of its largest magnitude; one
FP32 step to 1e-5.  Both preconditioners are covered: the multigrid V-cycle
(the default; on the smallest meshes its hierarchy is a single dense level)
and Jacobi."""
import numpy as np
import pytest

import oracle as O
from synth import configs as CF
from tests.parity import compare_elements, compare_state, compare_stats

pytestmark = pytest.mark.gpu

PROJ = dict(proj=1, Cp=1e-3, proj_tol=1e-14, proj_maxit=5000)


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_0720_amd import _lib
    return _lib


def _pair(w):
    from paper_1006_0720_amd.runner import workload_context

    print(f"[projection] {w.name} np={w.n_particles} prec={w.precision}", flush=True)
    ctx = workload_context(w)
    o = O.Oracle(w.mesh, w.params, store_fp32=(w.precision == "f32"), gradp=w.gradp, wp=w.wp)
    o.seed(w.seed)
    return ctx, o


def _square(precision="f64"):
    w = CF.periodic_square(n=12, ppe=40, seed=3)
    w.params = dict(w.params, **PROJ)
    w.precision = precision
    return w


def _channel():
    w = CF.channel(nx=20, n_half=8, ppe=30, precision="f64")
    w.params = dict(w.params, **PROJ)
    return w


@pytest.mark.parametrize("precond", [1, 0], ids=["multigrid", "jacobi"])
@pytest.mark.parametrize("make", [_square, _channel], ids=["periodic_square", "channel_glm_walls"])
def test_projection_trajectory_fp64(L, make, precond):
    w = make()
    w.params = dict(w.params, proj_precond=precond)
    ctx, o = _pair(w)
    for c in range(2):
        ctx.advance(5, w.dt)
        o.run(w.dt, 5)
        st, el, pid = ctx.particles()
        assert np.array_equal(pid, o.id)
        assert np.array_equal(el, o.elem), f"chunk {c}: {(el != o.elem).sum()} element mismatches"
        compare_state(st, o.state, w.mesh, 1e-11, f"projection chunk {c}", elem=o.elem)
        compare_stats(ctx.stats(), o.stats, 1e-11, what=f"projection chunk {c}")
        P = ctx.nodal_field(L.FIELD_PRESSURE)[0]
        scale = np.abs(o.Pp).max()
        assert scale > 0 and np.abs(P - o.Pp).max() <= 1e-9 * scale
        gp = ctx.nodal_field(L.FIELD_GRADP)
        assert np.abs(gp - o.gradp).max() <= 1e-9 * max(1.0, np.abs(o.gradp).max())
    assert ctx.counters()["proj_iters"] > 0
    ctx.close()


@pytest.mark.parametrize("precond", [1, 0], ids=["multigrid", "jacobi"])
def test_projection_canyon_corners_fp64(L, precond):
    """A small street canyon (floor blocks: reflex corners and the patch
    search) with the GLM, slip top, periodic streamwise: 5 projected steps.
    Its ~2000 masters give the multigrid hierarchy more than one level."""
    w = CF.canyon(target_elems=4000, ppe=12, precision="f64")
    w.params = dict(w.params, proj_precond=precond, **PROJ)
    ctx, o = _pair(w)
    ctx.advance(5, w.dt)
    o.run(w.dt, 5)
    st, el, pid = ctx.particles()
    assert np.array_equal(el, o.elem), f"{(el != o.elem).sum()} element mismatches"
    compare_state(st, o.state, w.mesh, 1e-11, "projection canyon", elem=o.elem)
    P = ctx.nodal_field(L.FIELD_PRESSURE)[0]
    assert np.abs(P - o.Pp).max() <= 1e-9 * np.abs(o.Pp).max()
    its = ctx.counters()["proj_iters"]
    print(f"[projection] canyon, preconditioner {precond}: {its} iterations in 5 solves", flush=True)
    if precond == 1:
        assert its <= 5 * 40
    ctx.close()


def test_projection_multigrid_iterations(L):
    """On the same canyon the V-cycle needs several times fewer iterations
    than Jacobi for the same stopping rule, and the solved pressures agree."""
    from paper_1006_0720_amd.runner import workload_context

    out = {}
    for precond in (0, 1):
        w = CF.canyon(target_elems=20000, ppe=2, precision="f64")
        w.params = dict(w.params, proj_precond=precond, **PROJ)
        ctx = workload_context(w)
        ctx.advance(2, w.dt)
        out[precond] = (ctx.counters()["proj_iters"], ctx.nodal_field(L.FIELD_PRESSURE)[0])
        ctx.close()
    (ij, pj), (im, pm) = out[0], out[1]
    print(f"[projection] canyon 20k: jacobi {ij}, multigrid {im} iterations", flush=True)
    assert im * 5 <= ij
    assert np.abs(pm - pj).max() <= 1e-9 * np.abs(pj).max()


def test_projection_fp32_one_step(L):
    w = _square("f32")
    ctx, o = _pair(w)
    ctx.advance(1, w.dt)
    o.step(w.dt)
    st, el, _ = ctx.particles()
    compare_elements(el, st, o.elem, o.state, w.mesh, "projection fp32 step", fp32=True)
    compare_state(st, o.state, w.mesh, 1e-5, "projection fp32 step", elem=o.elem)
    ctx.close()


def test_projection_parameter_checks(L):
    w = _square()
    for bad in (dict(stats_mode=CF.STATS_SHAPE), dict(frozen=1), dict(Cp=-1.0), dict(proj_maxit=0),
                dict(proj_tol=0.0), dict(proj=2), dict(proj_precond=2)):
        with pytest.raises(L.PdfError) as ei:
            L.Context(w.mesh, dict(w.params, **bad))
        assert ei.value.status == 1, bad


def test_projection_canyon_200_steps(L):
    """The street canyon with the projection and the wall datum over 200
    steps (C_p = 0.1 dt, redistribution keeping 3 per element): the GPU run
    stays with the oracle's (element indices bit-exact, FP64 state within
    1e-10, the solved P' within 1e-9 of its largest magnitude), both finite
    and without lost particles."""
    w = CF.canyon(target_elems=4000, ppe=12, precision="f64")
    w.params = dict(w.params, proj=1, Cp=0.1 * w.dt, min_ppe=3, proj_tol=1e-14, proj_maxit=5000)
    ctx, o = _pair(w)
    for chunk in range(4):
        ctx.advance(50, w.dt)
        o.run(w.dt, 50)
        st, el, _ = ctx.particles()
        what = f"canyon projection step {50 * (chunk + 1)}"
        assert np.array_equal(el, o.elem), f"{what}: {(el != o.elem).sum()} element mismatches"
        compare_state(st, o.state, w.mesh, 1e-10, what, elem=o.elem)
        P = ctx.nodal_field(L.FIELD_PRESSURE)[0]
        assert np.abs(P - o.Pp).max() <= 1e-9 * np.abs(o.Pp).max(), what
    c, oc = ctx.counters(), o.counter_dict()
    assert c["lost"] == oc["lost"] == 0 and c["nonfinite"] == 0
    assert c["redist"] == oc["redist"] > 0
    ctx.close()


def test_projection_canyon_20k_stable(L):
    """At 20k triangles and 20 particles per element (the bench's projected
    canyon, C_p = 0.1 dt, solved to 1e-6) 200 projected steps stay finite,
    lose no particle and keep the RMS speed within 25 % of its start."""
    from paper_1006_0720_amd.runner import workload_context

    w = CF.canyon(target_elems=20000, ppe=20, precision="f64")
    w.params = dict(w.params, proj=1, Cp=0.1 * w.dt, min_ppe=3, proj_tol=1e-6, proj_maxit=2000)
    ctx = workload_context(w)
    st, _, _ = ctx.particles()
    rms0 = np.sqrt((st[2] ** 2 + st[3] ** 2).mean())
    for k in range(4):
        ctx.advance(50, w.dt)
        st, _, _ = ctx.particles()
        rms = np.sqrt((st[2] ** 2 + st[3] ** 2).mean())
        P = ctx.nodal_field(L.FIELD_PRESSURE)[0]
        print(f"[projection] canyon 20k step {50 * (k + 1)}: rms speed {rms:.4g} (start {rms0:.4g}), "
              f"P' {P.min():.4g}..{P.max():.4g}", flush=True)
        assert np.isfinite(st).all() and np.isfinite(P).all()
        assert 0.75 * rms0 <= rms <= 1.25 * rms0
    c = ctx.counters()
    assert c["lost"] == 0 and c["nonfinite"] == 0
    ctx.close()
