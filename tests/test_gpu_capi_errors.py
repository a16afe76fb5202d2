"""The C ABI's error behaviour and degenerate inputs on the GPU: malformed
meshes (PDF_E_BAD_MESH with a message), out-of-range parameters and sizes
(PDF_E_INVALID_ARG), calls in the wrong order (PDF_E_STATE); and the smallest
problems against the oracle: a two-triangle mesh with one particle per
element, zero steps, and a zero mean frequency (no gamma draws)."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from synth import configs as CF
from synth import meshes as M
from tests.parity import compare_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_0720_amd import _lib
    return _lib


def _status(L, fn):
    with pytest.raises(L.PdfError) as ei:
        fn()
    return ei.value.status, str(ei.value)


def test_malformed_meshes(L):
    m = M.box(3, 3, 1.0, 1.0)
    p = CF.params()
    # a clockwise element
    en = m.elem_nodes.copy()
    en[4] = en[4][::-1]
    st, msg = _status(L, lambda: L.Context(dataclasses.replace(m, elem_nodes=en), p))
    assert st == 2 and "element" in msg
    # a neighbour table that is not symmetric
    nb = m.elem_nbr.copy()
    i = np.argwhere(nb >= 0)[0]
    nb[i[0], i[1]] = (nb[i[0], i[1]] + 1) % m.n_elems
    st, msg = _status(L, lambda: L.Context(dataclasses.replace(m, elem_nbr=nb), p))
    assert st == 2 and "neighbour" in msg
    # a periodic partner that is not mutual
    q = M.periodic_square(4)
    bp = q.bedge_partner.copy()
    bp[0] = bp[1]
    st, _ = _status(L, lambda: L.Context(dataclasses.replace(q, bedge_partner=bp), p))
    assert st == 2


def test_invalid_parameters_and_sizes(L):
    m = M.box(2, 2, 1.0, 1.0)
    for bad in (dict(model=5), dict(min_ppe=65), dict(min_ppe=-1), dict(C4=0.0), dict(nu=-1.0),
                dict(stats_mode=2)):
        st, _ = _status(L, lambda: L.Context(m, CF.params(**bad)))
        assert st == 1, bad
    w = CF.periodic_square(n=4, ppe=2)
    from paper_1006_0720_amd.runner import workload_context

    ctx = workload_context(w, seed=False)
    st, msg = _status(L, lambda: ctx.advance(1, 0.01))
    assert st == 5 and "seed" in msg  # advance before seeding
    st, _ = _status(L, lambda: ctx.seed(dict(w.seed, ppe=0)))
    assert st == 1
    ctx.seed(w.seed)
    for dt in (0.0, -1.0, float("nan")):
        st, _ = _status(L, lambda: ctx.advance(1, dt))
        assert st == 1
    st, _ = _status(L, lambda: ctx.advance(-1, 0.01))
    assert st == 1
    state, elem, pid = ctx.particles()
    bad_elem = elem.copy()
    bad_elem[0] = w.mesh.n_elems
    st, msg = _status(L, lambda: ctx.set_particles(state, bad_elem, pid))
    assert st == 1 and "element" in msg
    # an empty particle set is refused and the context keeps its particles
    st, _ = _status(L, lambda: ctx.set_particles(state[:, :0], elem[:0], pid[:0]))
    assert st == 1
    assert ctx.num_particles() == elem.size
    assert np.array_equal(ctx.particles()[0], state)
    st, _ = _status(L, lambda: L.Denoiser(ctx, hidden=40))
    assert st == 1
    ctx.close()
    # generalized Langevin model with an input wp that was never given
    w2 = CF.periodic_square(n=4, ppe=2)
    w2.params = dict(w2.params, model=CF.MODEL_GLM, wp_source=CF.WP_INPUT)
    ctx = workload_context(w2)
    st, msg = _status(L, lambda: ctx.advance(1, 0.01))
    assert st == 5 and "WP" in msg
    ctx.close()


def test_two_triangles_one_particle_each(L):
    """The smallest mesh: 2 triangles, slip walls, 1 particle per element,
    20 steps (one partly filled workgroup; reflections every step)."""
    from paper_1006_0720_amd.runner import workload_context

    mesh = M.box(1, 1, 1.0, 1.0, bc=M.BC_SLIP)
    assert mesh.n_elems == 2
    fz = CF.frozen_stats_for(mesh, U=(3.0, 1.0, 0.0), R_diag=(1.0, 1.0, 1.0), Om=1.0)
    p = CF.params()
    spec = dict(ppe=1, seed=9, psi_mode=CF.PSI_STEP_X, a=0.5, b=0, c=0, U0=fz[0:3], R0=fz[5:11], Om0=fz[3])
    w = CF.Workload("two_triangles", mesh, p, spec, 0.05, 20, "f64")
    ctx = workload_context(w)
    o = O.Oracle(mesh, p)
    o.seed(spec)
    st_a, el_a, _ = ctx.particles()
    ctx.advance(0, w.dt)  # zero steps: nothing changes
    st_b, el_b, _ = ctx.particles()
    assert np.array_equal(st_a, st_b) and np.array_equal(el_a, el_b)
    compare_state(st_a, o.state, mesh, 1e-12, "two triangles, seeded", elem=o.elem)
    ctx.advance(20, w.dt)
    o.run(w.dt, 20)
    st, el, pid = ctx.particles()
    assert np.array_equal(el, o.elem)
    compare_state(st, o.state, mesh, 1e-12, "two triangles", elem=o.elem)
    assert ctx.counters()["reflect"] == o.counter_dict()["reflect"] > 0
    ctx.close()


def test_zero_mean_frequency(L):
    """<omega> = 0 everywhere: particle frequencies start at 0 (no gamma draw),
    the frequency equation keeps them at 0 and the step stays finite."""
    from paper_1006_0720_amd.runner import workload_context

    w = CF.periodic_square(n=8, ppe=10)
    w.seed = dict(w.seed, Om0=np.zeros(w.mesh.n_nodes))
    ctx = workload_context(w)
    o = O.Oracle(w.mesh, w.params)
    o.seed(w.seed)
    assert np.all(o.state[5] == 0.0)
    ctx.advance(5, w.dt)
    o.run(w.dt, 5)
    st, el, _ = ctx.particles()
    assert np.array_equal(el, o.elem) and np.all(np.isfinite(st)) and np.all(st[5] == 0.0)
    compare_state(st, o.state, w.mesh, 1e-12, "zero frequency", elem=o.elem)
    ctx.close()


def test_context_as_the_first_gpu_action_of_a_process(L):
    """A fresh process whose first GPU action is creating a context (the
    binding imported before torch has touched the GPU): the library must
    share torch's HIP runtime, or its first HIP call fails."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_1006_0720_amd.runner import workload_context\n"
            "from synth import configs as CF\n"
            "ctx = workload_context(CF.periodic_square(n=4, ppe=2))\n"
            "print('particles', ctx.num_particles())\n"
            "ctx.close()\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "particles 64" in r.stdout
