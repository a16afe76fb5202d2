"""GPU parity of IECM mixing (eq:IECM) with the velocity-conditioned scalar
mean (App. B binning) and of the source-aware micromixing time scale
(eq:micromixing-timescale-canyon), through the C ABI, against the oracle.

FP64 trajectories: element indices bit-exact, state and statistics within
1e-12.  The cases cover the three element paths (at most 128 particles: one
wave with the particles in LDS; 129-512: a 256-thread workgroup with the
particles in LDS; more than 512: a 256-thread workgroup keeping the order in
global memory), the adaptive stop at low counts, ties from the copies the
particle redistribution makes, SHAPE statistics, and FP32 steps (1e-5)."""
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


def _square(n, ppe, **kw):
    w = CF.periodic_square(n=n, ppe=ppe, seed=2)
    w.params = dict(w.params, **{"mix_model": CF.MIX_IECM, **kw})
    w.seed = dict(w.seed, psi_mode=CF.PSI_GAUSS_X, a=0.5, b=0.15)
    return w


def _pair(w, reorder_every=0):
    from paper_1006_0720_amd.runner import workload_context

    print(f"[iecm] {w.name} np={w.n_particles} prec={w.precision} "
          f"bins=({w.params.get('cond_nu')},{w.params.get('cond_nv')},{w.params.get('cond_nw')}) "
          f"min={w.params.get('cond_min')} tm={w.params.get('tm_mode')}", flush=True)
    ctx = workload_context(w, reorder_every=reorder_every)
    o = O.Oracle(w.mesh, w.params, store_fp32=(w.precision == "f32"), gradp=w.gradp, wp=w.wp)
    o.seed(w.seed)
    return ctx, o


def _run_and_check(ctx, o, w, chunks, steps, what):
    for c in range(chunks):
        ctx.advance(steps, w.dt)
        o.run(w.dt, steps)
        st, el, pid = ctx.particles()
        assert np.array_equal(pid, o.id)
        assert np.array_equal(el, o.elem), f"{what} {c}: {(el != o.elem).sum()} element mismatches"
        compare_state(st, o.state, w.mesh, 1e-12, f"{what} {c}", elem=o.elem)
        compare_stats(ctx.stats(), o.stats, 1e-12, what=f"{what} {c}")


@pytest.mark.parametrize("ppe,reorder", [(60, 0), (60, 4), (250, 0), (510, 0), (1500, 4)])
def test_iecm_trajectory_fp64(L, ppe, reorder):
    """5 x 5 x 5 bins, at least 2 per subgroup: 60 per element takes two
    levels (60 // 25 = 2) on the one-wave path; 250 takes three on the
    129-512 path; at 510 the counts spread to either side of 512, so elements
    run on both the 129-512 and the large-element path; 1500 runs every
    element on the large-element path."""
    # (on a 2 x 2 periodic square every averaged nodal gradient is zero by
    # symmetry, leaving only rounding to compare: 3 x 3 is the smallest useful)
    w = _square(3 if ppe > 400 else (4 if ppe > 200 else 8), ppe)
    ctx, o = _pair(w, reorder)
    cm = o.cond_means()
    assert np.unique(cm).size > 10 * w.mesh.n_elems  # conditioning is active
    _run_and_check(ctx, o, w, 2, 10, f"iecm ppe {ppe}")
    ctx.close()


def test_iecm_adaptive_stop_and_odd_bins(L):
    """Few particles and (3 x 2 x 4) bins with at least 3 per subgroup: the
    counts spread over about 5-25 per element, so elements stop after zero
    (n < 9), one or two (n >= 18) levels."""
    w = _square(8, 15, cond_nu=3, cond_nv=2, cond_nw=4, cond_min=3)
    ctx, o = _pair(w)
    _run_and_check(ctx, o, w, 2, 10, "iecm adaptive stop")
    ctx.close()


def test_iecm_with_redistribution_copies(L):
    """Redistribution copies whole particle states, so exact ties in all three
    velocity components occur; they are ordered by id on both sides."""
    from synth import meshes as M
    import dataclasses

    m = M.box(12, 24, 1.0, 1.0, jitter=0.0, seed=0, bc=M.BC_SLIP)
    xy = m.node_xy.copy()
    xy[:, 1] = xy[:, 1] ** 2.5
    mesh = dataclasses.replace(m, node_xy=xy)
    fz = CF.frozen_stats_for(mesh, U=(0.3, 0.0, 0.0), R_diag=(0.5, 0.4, 0.3), Om=1.0)
    p = CF.params(frozen=1, min_ppe=6, mix_model=CF.MIX_IECM, cond_nu=2, cond_nv=2, cond_nw=2, cond_min=1)
    seed = dict(ppe=16, seed=4, psi_mode=CF.PSI_GAUSS_X, a=0.5, b=0.2, c=0, U0=fz[0:3], R0=fz[5:11], Om0=fz[3])
    w = CF.Workload("stretched_box_iecm_redist", mesh, p, seed, 0.01, 1, "f64")
    ctx, o = _pair(w)
    ctx.set_nodal_field(L.FIELD_STATS, fz)
    o.set_stats(fz)
    for c in range(2):
        ctx.advance(10, w.dt)
        o.run(w.dt, 10)
        st, el, _ = ctx.particles()
        assert np.array_equal(el, o.elem), f"{(el != o.elem).sum()} element mismatches"
        compare_state(st, o.state, w.mesh, 1e-12, f"iecm redistribution {c}", elem=o.elem)
    assert ctx.counters()["redist"] == o.counter_dict()["redist"] > 0
    ctx.close()


def test_iecm_source_timescale_channel_fp64(L):
    """Channel, GLM, no-slip walls, a disc source, IECM with the source-aware
    t_m of eq:micromixing-timescale-canyon (C_s = 0.02, C_t = 0.7)."""
    w = CF.channel(nx=20, n_half=8, ppe=30, precision="f64")
    w.params = dict(w.params, mix_model=CF.MIX_IECM, tm_mode=CF.TM_SOURCE, src_x=1.0, src_y=0.5,
                    src_r=0.1)
    ctx, o = _pair(w)
    _run_and_check(ctx, o, w, 2, 10, "iecm channel source t_m")
    ctx.close()


@pytest.mark.parametrize("mix", [CF.MIX_IEM, CF.MIX_IECM])
def test_source_timescale_shape_fp64(L, mix):
    w = _square(8, 40, stats_mode=CF.STATS_SHAPE, tm_mode=CF.TM_SOURCE, nu=1e-3, src_x=0.3, src_y=0.6,
                src_r=0.08, mix_model=mix)
    ctx, o = _pair(w)
    _run_and_check(ctx, o, w, 2, 10, "shape source t_m")
    ctx.close()


@pytest.mark.parametrize("n,ppe", [(8, 120), (3, 700)])
def test_iecm_fp32_one_step(L, n, ppe):
    """FP32: one step from the common seeded state (the oracle rounds the
    conditioned means to binary32 as the GPU stores them); 700 per element
    runs on the large-element path."""
    w = _square(n, ppe)
    w.precision = "f32"
    ctx, o = _pair(w)
    ctx.advance(1, w.dt)
    o.step(w.dt)
    st, el, _ = ctx.particles()
    compare_elements(el, st, o.elem, o.state, w.mesh, "iecm fp32 step", fp32=True)
    compare_state(st, o.state, w.mesh, 1e-5, "iecm fp32 step", elem=o.elem)
    ctx.close()


def test_iecm_fp32_velocity_ties(L):
    """FP32 one step with exact ties planted in every element: U copied from
    one particle to the next (ties broken by id), a whole velocity copied, U
    of -0 and +0 side by side (equal keys), with a strong mixing rate so that
    a particle put in a wrong bin shows in its scalar.  About 100 per element
    runs the first division by velocity buckets on the one-wave path."""
    w = _square(8, 100, Cphi=10.0)
    w.precision = "f32"
    ctx, o = _pair(w)
    st, el, pid = ctx.particles()
    st = np.array(st, dtype=np.float64, order="C")
    order = np.argsort(el, kind="stable")
    first = np.flatnonzero(np.r_[True, np.diff(el[order]) != 0])
    assert np.diff(np.r_[first, el.size]).min() >= 8

    def at(k):  # the k-th particle of every element
        return order[first + k]

    st[2, at(1)] = st[2, at(0)]
    st[2:5, at(3)] = st[2:5, at(2)]
    st[2, at(4)] = -0.0
    st[2, at(5)] = 0.0
    st[2, at(6)] = -0.0
    ctx.set_particles(st, el, pid)
    st0, el0, pid0 = ctx.particles()
    assert np.array_equal(pid0, pid)
    assert np.signbit(st0[2, at(4)]).all() and not np.signbit(st0[2, at(5)]).any()
    o.state, o.elem, o.id = st0, el0, pid0
    o.set_stats(ctx.stats())
    ctx.advance(1, w.dt)
    o.step(w.dt)
    st1, el1, _ = ctx.particles()
    assert np.abs(st1[6] - st0[6]).max() > 1e-3  # mixing moved the scalar
    compare_elements(el1, st1, o.elem, o.state, w.mesh, "iecm fp32 ties", fp32=True)
    compare_state(st1, o.state, w.mesh, 1e-5, "iecm fp32 ties", elem=o.elem)
    ctx.close()


def test_iecm_invalid_parameters(L):
    from synth import meshes as M

    m = M.box(2, 2, 1.0, 1.0)
    for bad in (dict(mix_model=2), dict(cond_nu=0), dict(cond_nw=17), dict(cond_min=0), dict(cond_min=65),
                dict(tm_mode=3)):
        with pytest.raises(L.PdfError) as ei:
            L.Context(m, CF.params(**bad))
        assert ei.value.status == 1, bad
