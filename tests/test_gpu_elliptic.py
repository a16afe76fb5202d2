"""GPU parity of the elliptic relaxation for wp_ij (PDF_WP_ELLIPTIC: linear
finite elements, conjugate gradients on the device preconditioned by the
plain-aggregation multigrid V-cycle or by Jacobi) against the oracle's exact
sparse solve, through the C ABI.

The solve is iterative, so the bar follows from its stopping rule: with the
preconditioned residual of every component below 1e-13 of its right-hand
side, the solution is compared within 1e-9 of its largest magnitude.  The
trajectories that use it are held to 1e-10 (element indices bit-exact): wp
enters the velocity through G_ij dt, which scales such differences down."""
import numpy as np
import pytest

import oracle as O
from oracle import elliptic as EL
from synth import configs as CF
from tests.parity import compare_state

pytestmark = pytest.mark.gpu

ELL = dict(wp_source=CF.WP_ELLIPTIC, ell_tol=1e-13, ell_maxit=4000)


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_0720_amd import _lib
    return _lib


def _pair(w):
    from paper_1006_0720_amd.runner import workload_context

    print(f"[elliptic] {w.name} np={w.n_particles} prec={w.precision}", flush=True)
    ctx = workload_context(w)
    o = O.Oracle(w.mesh, w.params, store_fp32=(w.precision == "f32"), gradp=w.gradp, wp=w.wp)
    o.seed(w.seed)
    return ctx, o


def _channel():
    w = CF.channel(nx=20, n_half=8, ppe=30, precision="f64")
    w.params = dict(w.params, **ELL)
    return w


def _square():
    w = CF.periodic_square(n=12, ppe=20)
    w.params = dict(w.params, model=CF.MODEL_GLM, nu=1e-3, **ELL)
    return w


@pytest.mark.parametrize("precond", [1, 0], ids=["multigrid", "jacobi"])
@pytest.mark.parametrize("make", [_channel, _square], ids=["channel_walls", "periodic_square"])
def test_solve_matches_oracle(L, make, precond):
    w = make()
    w.params = dict(w.params, ell_precond=precond)
    ctx, o = _pair(w)
    st0 = o.stats.copy()
    ctx.advance(1, w.dt)
    wp = ctx.nodal_field(L.FIELD_WP)
    ref = EL.solve(w.mesh, w.params, st0, o.local_wp(st0))
    scale = np.abs(ref).max()
    err = np.abs(wp - ref).max() / scale
    print(f"[elliptic] max |gpu - exact| / max|wp| = {err:.2e}, iterations {ctx.counters()['ell_iters']}")
    assert err < 1e-9
    assert ctx.counters()["ell_iters"] > 0
    ctx.close()


@pytest.mark.parametrize("precond", [1, 0], ids=["multigrid", "jacobi"])
def test_trajectory_and_warm_start(L, precond):
    """Ten steps with the solve every step.  The second solve starts from the
    first's solution: with Jacobi it needs fewer iterations; the V-cycle
    converges in a few iterations from either start on this small mesh (no
    more from the warm one)."""
    w = _channel()
    w.params = dict(w.params, ell_precond=precond)
    ctx, o = _pair(w)
    ctx.advance(1, w.dt)
    it1 = ctx.counters(reset=True)["ell_iters"]
    ctx.advance(1, w.dt)
    it2 = ctx.counters()["ell_iters"]
    print(f"[elliptic] preconditioner {precond}: {it1} iterations cold, {it2} warm", flush=True)
    assert 0 < it2 <= it1
    if precond == 0:
        assert it2 < it1  # started from the previous solution
    o.run(w.dt, 2)
    ctx.advance(8, w.dt)
    o.run(w.dt, 8)
    st, el, pid = ctx.particles()
    assert np.array_equal(pid, o.id)
    assert np.array_equal(el, o.elem), f"{(el != o.elem).sum()} element mismatches"
    compare_state(st, o.state, w.mesh, 1e-10, "GLM with the elliptic relaxation", elem=o.elem)
    ctx.close()


def test_multigrid_levels_match_oracle_in_fewer_iterations(L):
    """A channel of ~5900 nodes (a hierarchy of several levels): both
    preconditioners reach the oracle's solution within 1e-9, the V-cycle in
    at most half the iterations of Jacobi."""
    from paper_1006_0720_amd.runner import workload_context

    w = CF.channel(nx=80, n_half=36, ppe=4, precision="f64")
    w.params = dict(w.params, **ELL)
    o = O.Oracle(w.mesh, w.params, gradp=w.gradp, wp=w.wp)
    o.seed(w.seed)
    st0 = o.stats.copy()
    ref = EL.solve(w.mesh, w.params, st0, o.local_wp(st0))
    scale = np.abs(ref).max()
    its = {}
    for precond in (0, 1):
        w.params = dict(w.params, ell_precond=precond)
        ctx = workload_context(w)
        ctx.advance(1, w.dt)
        wp = ctx.nodal_field(L.FIELD_WP)
        its[precond] = ctx.counters()["ell_iters"]
        err = np.abs(wp - ref).max() / scale
        print(f"[elliptic] {w.mesh.n_nodes} nodes, preconditioner {precond}: {its[precond]} iterations, "
              f"max |gpu - exact| / max|wp| = {err:.2e}", flush=True)
        assert err < 1e-9
        ctx.close()
    assert 0 < 2 * its[1] <= its[0]


def test_parameter_checks(L):
    w = _channel()
    for bad in (dict(ell_maxit=0), dict(ell_tol=0.0), dict(ell_tol=float("nan")), dict(wp_source=3),
                dict(ell_precond=2)):
        with pytest.raises(L.PdfError) as ei:
            L.Context(w.mesh, dict(w.params, **bad))
        assert ei.value.status == 1, bad
