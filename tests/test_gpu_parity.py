"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.

FP64 runs are compared as whole trajectories: element indices bit-exact,
particle state and nodal statistics within 1e-12 (relative with the per-
quantity scale of tests/parity.py).  FP32 runs are compared one step at a
time from the common seeded state (the oracle stores the state rounded to
binary32 exactly where the GPU does): element indices bit-exact, floats
within 1e-5.
"""
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


def _pair(L, w, reorder_every=0):
    from paper_1006_0720_amd.runner import workload_context

    print(f"[parity] {w.name} np={w.n_particles} prec={w.precision}", flush=True)
    ctx = workload_context(w, reorder_every=reorder_every)
    o = O.Oracle(w.mesh, w.params, store_fp32=(w.precision == "f32"), gradp=w.gradp, wp=w.wp)
    o.seed(w.seed)
    return ctx, o


def _check(ctx, o, w, rtol, what, stats_rtol=None):
    st, el, pid = ctx.particles()
    assert np.array_equal(pid, o.id)
    assert np.array_equal(el, o.elem), f"{what}: {(el != o.elem).sum()} element mismatches"
    errs = compare_state(st, o.state, w.mesh, rtol, what, elem=o.elem)
    g = ctx.stats()
    serr = compare_stats(g, o.stats, stats_rtol or rtol, what=what)
    return errs, serr


def test_seed_parity_fp64(L):
    w = CF.periodic_square()
    ctx, o = _pair(L, w)
    st, el, pid = ctx.particles()
    # positions are computed with identical IEEE operations: bit-exact
    assert np.array_equal(st[0], o.state[0]) and np.array_equal(st[1], o.state[1])
    assert np.array_equal(st[6], o.state[6])
    _check(ctx, o, w, 1e-12, "seed")
    ctx.close()


@pytest.mark.parametrize("reorder", [0, 4])
def test_trajectory_parity_fp64_periodic_square(L, reorder):
    """Workload 1 at full size: 2048 elements, 102400 particles, 100 steps;
    nodal statistics and the exported element moments."""
    w = CF.periodic_square()
    ctx, o = _pair(L, w, reorder_every=reorder)
    for chunk in range(4):
        ctx.advance(25, w.dt)
        o.run(w.dt, 25)
        _check(ctx, o, w, 1e-12, f"step {25 * (chunk + 1)}")
        # element moments of the last accumulation (formed on demand after a
        # step that gathered the node values straight from the sums; the last
        # chunk ends on a reorder step when reorder = 4)
        _, el = ctx.stats(elem=True)
        assert np.array_equal(el[0], o.elem_stats[0])
        compare_stats(el, o.elem_stats, 1e-12, fields=range(1, 16), what=f"element moments, step {25 * (chunk + 1)}")
    c = ctx.counters()
    oc = o.counter_dict()
    assert c["lost"] == 0 and oc["lost"] == 0
    for k in ("walk_steps", "periodic", "omega_clamp"):
        assert c[k] == oc[k], (k, c[k], oc[k])
    ctx.close()


def _small_channel(precision="f64", ppe=30, steps=30, nx=20, nh=8, seed=0):
    w = CF.channel(nx=nx, n_half=nh, ppe=ppe, steps=steps, precision=precision, seed=seed)
    return w


def test_trajectory_parity_fp64_channel_glm_walls(L):
    """Generalized Langevin model with the local elliptic-relaxation tensor,
    nu > 0, no-slip walls with trajectory (b) and gamma wall frequencies."""
    w = _small_channel("f64")
    ctx, o = _pair(L, w)
    for chunk in range(3):
        ctx.advance(10, w.dt)
        o.run(w.dt, 10)
        _check(ctx, o, w, 1e-12, f"channel step {10 * (chunk + 1)}")
    c, oc = ctx.counters(), o.counter_dict()
    for k in ("walk_steps", "reflect", "noslip_b", "periodic", "gamma_fail", "lost"):
        assert c[k] == oc[k], (k, c[k], oc[k])
    assert oc["reflect"] > 0 and oc["noslip_b"] > 0
    ctx.close()


def test_trajectory_parity_fp64_canyon_corners(L):
    """Canyon geometry: block corners (fall-back searches), slip top, no-slip
    floor and blocks, continuous scalar source."""
    mesh = M.canyon(3000, 0.15, 2)
    w = CF.canyon(mesh=mesh, ppe=20, precision="f64", steps=30)
    ctx, o = _pair(L, w)
    for chunk in range(3):
        ctx.advance(10, w.dt)
        o.run(w.dt, 10)
        _check(ctx, o, w, 1e-12, f"canyon step {10 * (chunk + 1)}")
    c, oc = ctx.counters(), o.counter_dict()
    for k in ("walk_steps", "reflect", "fallback", "brute", "noslip_b", "lost"):
        assert c[k] == oc[k], (k, c[k], oc[k])
    ctx.close()


def test_frozen_glm_input_wp_fp64(L):
    """Frozen statistics and an input wp field (PDF_WP_INPUT)."""
    w = _small_channel("f64", ppe=20)
    nn = w.mesh.n_nodes
    rng = np.random.default_rng(0)
    wp = np.zeros((9, nn))
    wp[0] = wp[4] = wp[8] = -0.4 + 0.05 * rng.standard_normal(nn)
    wp[1] = wp[3] = 0.02 * rng.standard_normal(nn)
    w.params = dict(w.params, wp_source=CF.WP_INPUT, frozen=1)
    w.wp = wp
    ctx, o = _pair(L, w)
    fz = CF.frozen_stats_for(w.mesh, U=(5.0, 0.0, 0.0), R_diag=(1.0, 0.5, 0.7), Om=3.0, Phi=0.2)
    ctx.set_nodal_field(L.FIELD_STATS, fz)
    o.set_stats(fz)
    ctx.advance(10, w.dt)
    o.run(w.dt, 10)
    st, el, pid = ctx.particles()
    assert np.array_equal(el, o.elem)
    compare_state(st, o.state, w.mesh, 1e-12, "frozen GLM", elem=o.elem)
    compare_stats(ctx.stats(), o.est, 1e-12, what="frozen GLM estimate")
    ctx.close()


def test_kernel_parity_fp32_channel(L):
    """FP32 state: one step from the common seeded state."""
    w = _small_channel("f32", ppe=60, nx=30, nh=10)
    ctx, o = _pair(L, w)
    st, el, pid = ctx.particles()
    assert np.array_equal(el, o.elem)
    compare_state(st, o.state, w.mesh, 1e-6, "fp32 seed", elem=o.elem)
    compare_stats(ctx.stats(), o.stats, 1e-5, what="fp32 seed stats")
    ctx.advance(1, w.dt)
    o.step(w.dt)
    st, el, pid = ctx.particles()
    compare_elements(el, st, o.elem, o.state, w.mesh, "fp32 step", fp32=True)
    compare_state(st, o.state, w.mesh, 1e-5, "fp32 step", elem=o.elem)
    compare_stats(ctx.stats(), o.stats, 1e-5, what="fp32 step stats")
    ctx.close()


def test_kernel_parity_fp32_canyon_full_size_sampled(L):
    """Street-canyon workload at full size (~200k elements, 50 per element,
    ~10M particles): seeded state and nodal statistics compared in full, one
    step compared on a 1% particle sample advanced by the oracle from the
    same state and statistics."""
    w = CF.canyon()
    ctx, o = _pair(L, w)
    st, el, pid = ctx.particles()
    assert np.array_equal(el, o.elem)
    compare_state(st, o.state, w.mesh, 1e-6, "canyon fp32 seed", elem=o.elem)
    compare_stats(ctx.stats(), o.stats, 1e-5, what="canyon fp32 seed stats")
    ctx.advance(1, w.dt)
    mask = np.zeros(o.state.shape[1], np.uint8)
    mask[np.random.default_rng(0).choice(mask.size, mask.size // 100, replace=False)] = 1
    o.step(w.dt, mask=mask)
    st, el, pid = ctx.particles()
    sel = mask.astype(bool)
    nd = compare_elements(el[sel], st[:, sel], o.elem[sel], o.state[:, sel], w.mesh, "canyon fp32 step", fp32=True)
    print(f"[canyon] {sel.sum()} sampled particles, {nd} with positions one ulp apart", flush=True)
    compare_state(st[:, sel], o.state[:, sel], w.mesh, 1e-5, "canyon fp32 step (sample)", elem=o.elem[sel])
    c = ctx.counters()
    assert c["lost"] == 0 and c["nonfinite"] == 0
    # particle count conservation: element counts add up to N_p
    _, elst = ctx.stats(elem=True)
    assert elst[0].sum() == w.n_particles
    ctx.close()


def test_gpu_ou_stationary_variance(L):
    """The closed-form OU limit on the GPU (frozen simplified Langevin model)."""
    mesh = M.periodic_square(16)
    w = CF.periodic_square(n=16, ppe=200, frozen=1)
    from paper_1006_0720_amd.runner import workload_context
    ctx = workload_context(w)
    fz = CF.frozen_stats_for(mesh, U=(1.0, 0.0, 0.0), R_diag=(2 / 3,) * 3, Om=1.0, Phi=0.5)
    ctx.set_nodal_field(L.FIELD_STATS, fz)
    dt = 0.01
    ctx.advance(200, dt)
    v = []
    for _ in range(5):
        ctx.advance(50, dt)
        st, _, _ = ctx.particles(sort_by_id=False)
        v.append(st[2:5].var(axis=1).mean())
    G = -(0.5 + 0.75 * 2.1)
    expect = 2.1 / (-2 * G - G * G * dt)
    assert abs(np.mean(v) - expect) / expect < 0.004
    ctx.close()


def test_brute_force_location_matches_oracle(L):
    """Particles handed wrong host elements: the walk (64 steps) and the
    patch search fail, and the last-resort location (a bucket grid on the GPU,
    the plain scan over all elements in the oracle) must return the same,
    lowest-numbered, containing element."""
    from paper_1006_0720_amd.runner import workload_context

    mesh = M.box(48, 40, 1.2, 1.0, jitter=0.2, seed=4, bc=M.BC_SLIP)
    p = CF.params(frozen=1)
    fz = CF.frozen_stats_for(mesh, U=(0.0, 0.0, 0.0), R_diag=(0.01,) * 3, Om=1.0)
    w = CF.Workload("box_brute", mesh, p, dict(ppe=4, seed=5, psi_mode=CF.PSI_ZERO, a=0, b=0, c=0,
                                               U0=fz[0:3], R0=fz[5:11], Om0=fz[3]), 1e-3, 1, "f64")
    ctx = workload_context(w)
    o = O.Oracle(mesh, p)
    o.seed(w.seed)
    rng = np.random.default_rng(9)
    perm = rng.permutation(mesh.n_elems)
    elem = perm[o.elem].astype(np.int32)  # hosts far from the particles
    ctx.set_particles(o.state, elem, o.id)
    o.elem = elem.copy()
    ctx.set_nodal_field(L.FIELD_STATS, fz)
    o.set_stats(fz)
    ctx.counters(reset=True)
    o.counters[:] = 0
    ctx.advance(1, w.dt)
    o.step(w.dt)
    st, el, pid = ctx.particles()
    assert np.array_equal(pid, o.id)
    assert np.array_equal(el, o.elem), f"{(el != o.elem).sum()} element mismatches"
    compare_state(st, o.state, mesh, 1e-12, "brute force", elem=o.elem)
    c, oc = ctx.counters(), o.counter_dict()
    # a particle that stepped outside the box and whose walk ran out before
    # reaching the wall is lost (restored) on both sides alike
    assert oc["brute"] > 100 and c["brute"] == oc["brute"] and c["lost"] == oc["lost"]
    ctx.close()


def test_kernel_parity_fp32_channel_block_full_size_sampled(L):
    """The benchmark workload at full size in the benchmark's launch
    configuration (~1M triangles, 100 per element, ~100M particles, FP32,
    reorder every 8 steps).  After 9 GPU steps, one more step is compared on a
    1% particle sample advanced by the oracle from the GPU's state and
    statistics; the nodal statistics after that step are compared with the
    oracle's estimate from the GPU's particles; particle count is conserved.
    Particles are compared in storage order, which the 10th step keeps (the
    reorder runs after steps 8, 16, ...)."""
    import time

    from paper_1006_0720_amd.runner import workload_context

    t0 = time.time()

    def say(msg):
        print(f"[parity c5] {time.time() - t0:6.1f}s {msg}", flush=True)

    w = CF.channel_block()
    say(f"{w.name} np={w.n_particles}")
    ctx = workload_context(w, reorder_every=8)
    ctx.advance(9, w.dt)
    st0, el0, pid0 = ctx.particles(sort_by_id=False)
    stats0 = ctx.stats()
    say("state after 9 steps copied")
    ctx.advance(1, w.dt)
    st1, el1, pid1 = ctx.particles(sort_by_id=False)
    g1 = ctx.stats()
    c = ctx.counters()
    _, elst = ctx.stats(elem=True)
    ctx.close()
    say("state after 10 steps copied")
    assert np.array_equal(pid0, pid1)
    assert c["lost"] == 0 and c["nonfinite"] == 0
    assert elst[0].sum() == w.n_particles
    o = O.Oracle(w.mesh, w.params, store_fp32=True, gradp=w.gradp)
    o.state, o.elem, o.id = st0, el0.copy(), pid0
    o.seed_value = int(w.seed["seed"])
    o.step_index = 9
    o.set_stats(stats0)
    mask = np.zeros(st0.shape[1], np.uint8)
    mask[np.random.default_rng(1).choice(mask.size, mask.size // 100, replace=False)] = 1
    o.step(w.dt, mask=mask)
    say("oracle step on the 1% sample done")
    sel = mask.astype(bool)
    nd = compare_elements(el1[sel], st1[:, sel], o.elem[sel], o.state[:, sel], w.mesh, "channel_block step 10",
                          fp32=True)
    say(f"{sel.sum()} sampled particles, {nd} with positions one ulp apart")
    es = compare_state(st1[:, sel], o.state[:, sel], w.mesh, 1e-5, "channel_block fp32 step (sample)", elem=o.elem[sel])
    say("state error vs the FP64 oracle (max relative): " + ", ".join(f"{k} {v:.2e}" for k, v in es.items()))
    # nodal statistics: the oracle's estimate from the GPU's particles after the step
    o.state, o.elem = st1, el1
    o.stats = stats0
    est = o.estimate()
    say("oracle estimate done")
    en = compare_stats(g1, est, 1e-9, what="channel_block statistics")
    say("nodal statistics error vs the FP64 oracle (max relative, field: error): " +
        ", ".join(f"{f}: {v:.1e}" for f, v in en.items()))


def test_kernel_parity_fp32_channel_block_driven_200_steps(L):
    """The benchmark workload over 200 steps in the benchmark's launch
    configuration, compared with the FP64 oracle in driven mode: at steps 20,
    40, ..., 200 the oracle advances a fresh 1% particle sample one step from
    the GPU's state and statistics, and that step's elements must match
    bit-exactly and the state within 1e-5 (the comparison re-synchronises each
    time, so FP32 rounding does not accumulate into it).  At the end the nodal
    statistics equal the oracle's estimate from the GPU's particles (1e-9)."""
    import time

    from paper_1006_0720_amd.runner import workload_context

    t0 = time.time()

    def say(msg):
        print(f"[driven c5] {time.time() - t0:6.1f}s {msg}", flush=True)

    w = CF.channel_block()
    say(f"{w.name} np={w.n_particles}")
    ctx = workload_context(w, reorder_every=8)
    rng = np.random.default_rng(7)
    worst = {}
    done = 0
    for k in range(1, 11):
        ctx.advance(20 * k - done, w.dt)  # to step 20k (the reorder follows steps 8, 16, ...)
        done = 20 * k
        st0, el0, pid0 = ctx.particles(sort_by_id=False)
        stats0 = ctx.stats()
        ctx.advance(1, w.dt)  # step 20k + 1 is odd: no reorder, storage order kept
        done += 1
        st1, el1, pid1 = ctx.particles(sort_by_id=False)
        assert np.array_equal(pid0, pid1)
        o = O.Oracle(w.mesh, w.params, store_fp32=True, gradp=w.gradp)
        o.state, o.elem, o.id = st0, el0.copy(), pid0
        o.seed_value = int(w.seed["seed"])
        o.step_index = 20 * k
        o.set_stats(stats0)
        mask = np.zeros(st0.shape[1], np.uint8)
        mask[rng.choice(mask.size, mask.size // 100, replace=False)] = 1
        o.step(w.dt, mask=mask)
        sel = mask.astype(bool)
        nd = compare_elements(el1[sel], st1[:, sel], o.elem[sel], o.state[:, sel], w.mesh, f"step {20 * k + 1}",
                              fp32=True)
        es = compare_state(st1[:, sel], o.state[:, sel], w.mesh, 1e-5, f"channel_block step {20 * k + 1} (sample)", elem=o.elem[sel])
        worst = {n: max(worst.get(n, 0.0), e) for n, e in es.items()}
        say(f"step {20 * k + 1}: " + ", ".join(f"{n} {e:.1e}" for n, e in es.items()) +
            f"; {nd} positions one ulp apart")
    c = ctx.counters()
    assert c["lost"] == 0 and c["nonfinite"] == 0
    g1 = ctx.stats()
    _, elst = ctx.stats(elem=True)
    ctx.close()
    assert elst[0].sum() == w.n_particles
    o.state, o.elem = st1, el1
    o.stats = stats0
    en = compare_stats(g1, o.estimate(), 1e-9, what="channel_block statistics after 201 steps")
    say("worst state error over the 10 driven steps: " + ", ".join(f"{n} {e:.1e}" for n, e in worst.items()))
    say("nodal statistics error after 201 steps (max over fields): %.1e" % max(en.values()))
