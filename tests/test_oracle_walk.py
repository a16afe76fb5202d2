"""Pins for the oracle's particle tracking and boundary conditions (Ch.3, Sec.
Particle tracking; Sec. No-slip wall-boundary conditions): the element found
by the neighbour walk contains the particle (checked against an independent
point-in-triangle test and against brute force), points on edges and vertices
and one ulp off them, periodic wrap, perfect reflection, the slip and no-slip
velocity conditions, and particle-count conservation."""
import numpy as np
import pytest

import oracle as O
from synth import configs as CF
from synth import meshes as M


def _contains(mesh, elem, x, y, tol=1e-12):
    """Independent closed containment test (numpy.linalg barycentric solve)."""
    p = mesh.node_xy[mesh.elem_nodes[elem]]
    T = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]], axis=2)
    lb = np.linalg.solve(T, (np.stack([x, y], 1) - p[:, 0])[..., None])[..., 0]
    lam = np.stack([1.0 - lb[:, 0] - lb[:, 1], lb[:, 0], lb[:, 1]], 1)
    return lam.min(axis=1) >= -tol


def _frozen_oracle(mesh, nu=0.0, **pk):
    o = O.Oracle(mesh, CF.params(frozen=1, nu=nu, **pk))
    U0, R0, Om0 = CF._iso(mesh.n_nodes)
    o.seed(dict(ppe=4, seed=1, psi_mode=0, U0=U0, R0=R0, Om0=Om0))
    o.set_stats(CF.frozen_stats_for(mesh, U=(0, 0, 0)))
    return o


def _place(o, elem, x, y, u, v):
    n = len(x)
    o.state = np.zeros((7, n))
    o.state[0], o.state[1], o.state[2], o.state[3] = x, y, u, v
    o.state[5] = 1.0
    o.elem = np.ascontiguousarray(elem, np.int32)
    o.id = np.arange(n, dtype=np.uint32)


def test_walk_random_jumps_periodic_square():
    mesh = M.periodic_square(8)
    o = _frozen_oracle(mesh)
    rng = np.random.default_rng(0)
    n = 20000
    e0 = rng.integers(0, mesh.n_elems, n)
    c = mesh.node_xy[mesh.elem_nodes[e0]].mean(axis=1)
    u = rng.uniform(-30, 30, n)
    v = rng.uniform(-30, 30, n)  # jumps of up to ~2.4 elements per step
    _place(o, e0, c[:, 0], c[:, 1], u, v)
    dt = 0.01
    assert o.step(dt) == 0
    x, y = o.state[0], o.state[1]
    assert (x >= 0).all() and (x <= 1).all() and (y >= 0).all() and (y <= 1).all()
    # periodic wrap of the straight-line move
    assert np.abs((c[:, 0] + u * dt) % 1.0 - x).max() < 1e-14 or \
        np.abs(((c[:, 0] + u * dt - x + 0.5) % 1.0) - 0.5).max() < 1e-14
    assert _contains(mesh, o.elem, x, y).all()
    cnt = o.counter_dict()
    assert cnt["lost"] == 0 and cnt["brute"] == 0


@pytest.mark.parametrize("meshname", ["square", "channel", "canyon"])
def test_walk_edges_vertices_and_ulps(meshname):
    mesh = {"square": lambda: M.periodic_square(6),
            "channel": lambda: M.graded_channel(8, 4, 6.0, 1.0, 0.15, 3),
            "canyon": lambda: M.canyon(3000, 0.15, 4)}[meshname]()
    om = O.OracleMesh(mesh)
    rng = np.random.default_rng(1)
    pts = []
    xy = mesh.node_xy
    # vertices, edge midpoints and points one ulp to either side
    for e in rng.integers(0, mesh.n_elems, 60):
        a, b, c = xy[mesh.elem_nodes[e]]
        for p in (a, b, 0.5 * (a + b), 0.5 * (b + c), (a + b + c) / 3.0):
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    px = np.nextafter(p[0], np.inf * dx) if dx else p[0]
                    py = np.nextafter(p[1], np.inf * dy) if dy else p[1]
                    pts.append((px, py))
    pts = np.array(pts)
    # keep points that lie in the closed domain according to brute force
    br = np.array([om.locate_brute(px, py) for px, py in pts])
    pts = pts[br >= 0]
    br = br[br >= 0]
    o = _frozen_oracle(mesh)
    n = pts.shape[0]
    # start the walk in the brute-force element's neighbour (or itself)
    nb = mesh.elem_nbr[br, rng.integers(0, 3, n)]
    start = np.where(nb >= 0, nb, br)
    _place(o, start, pts[:, 0], pts[:, 1], np.zeros(n), np.zeros(n))
    assert o.step(1e-3) == 0
    # points in the closed domain do not move; points one ulp outside a wall or a
    # periodic side are reflected or wrapped (by at most a few ulps of the box)
    lo, hi = mesh.node_xy.min(axis=0), mesh.node_xy.max(axis=0)
    indom = ((pts[:, 0] >= lo[0]) & (pts[:, 0] <= hi[0]) & (pts[:, 1] >= lo[1]) & (pts[:, 1] <= hi[1]))
    for (x0, x1, y1) in mesh.meta.get("blocks", []):
        indom &= ~((pts[:, 0] > x0) & (pts[:, 0] < x1) & (pts[:, 1] < y1))
    assert indom.sum() > 0.8 * n
    assert np.array_equal(o.state[0][indom], pts[indom, 0])
    assert np.array_equal(o.state[1][indom], pts[indom, 1])
    pts = np.stack([o.state[0], o.state[1]], 1)
    # the walk's element contains the point under the oracle's own closed test
    for e, (px, py) in zip(o.elem, pts):
        assert om.lambdas(e, px, py).min() >= 0.0
    assert _contains(mesh, o.elem, pts[:, 0], pts[:, 1]).all()
    br = np.where(indom, br, -1)
    # where brute force finds a unique element, the walk finds the same one
    interior = np.array([b >= 0 and om.lambdas(b, px, py).min() > 0 for b, (px, py) in zip(br, pts)])
    assert np.array_equal(o.elem[interior], br[interior])


def test_noslip_reflection_flat_wall():
    mesh = M.graded_channel(8, 6, 6.0, 1.0, 0.0, 0)
    o = _frozen_oracle(mesh)
    rng = np.random.default_rng(2)
    n = 2000
    # particles just above the lower wall moving down through it
    x = rng.uniform(0.5, 5.5, n)
    y = rng.uniform(1e-4, 5e-3, n)
    br = np.array([O.OracleMesh(mesh).locate_brute(a, b) for a, b in zip(x, y)])
    v = -rng.uniform(1.0, 3.0, n)
    dt = 0.01
    _place(o, br, x, y, rng.uniform(-1, 1, n), v)
    assert o.step(dt) == 0
    ystar = y + v * dt
    crossed = ystar < 0
    assert crossed.sum() > 100
    # perfect reflection and U_i = 0 (Sec. No-slip wall-boundary conditions)
    assert np.abs(o.state[1][crossed] + ystar[crossed]).max() < 1e-15
    assert (o.state[2:5, crossed] == 0).all()
    assert (o.state[5, crossed] > 0).all()
    assert _contains(mesh, o.elem, o.state[0], o.state[1]).all()


def test_slip_reflection_mirrors_positions():
    mesh = M.box(10, 10, 1.0, 1.0, 0.2, 5, M.BC_SLIP, "delaunay")
    o = _frozen_oracle(mesh)
    rng = np.random.default_rng(3)
    n = 5000
    e0 = rng.integers(0, mesh.n_elems, n)
    c = mesh.node_xy[mesh.elem_nodes[e0]].mean(axis=1)
    u = rng.uniform(-20, 20, n)
    v = rng.uniform(-20, 20, n)
    _place(o, e0, c[:, 0], c[:, 1], u, v)
    dt = 0.01
    assert o.step(dt) == 0
    x, y = o.state[0], o.state[1]
    xs, ys = c[:, 0] + u * dt, c[:, 1] + v * dt
    # mirror image of the straight move across the box walls (single reflections)
    single = (np.abs(xs - 0.5) < 1.5) & (np.abs(ys - 0.5) < 1.5)
    ex = np.where(xs < 0, -xs, np.where(xs > 1, 2 - xs, xs))
    ey = np.where(ys < 0, -ys, np.where(ys > 1, 2 - ys, ys))
    assert np.abs(x[single] - ex[single]).max() < 1e-14
    assert np.abs(y[single] - ey[single]).max() < 1e-14
    assert ((x >= 0) & (x <= 1) & (y >= 0) & (y <= 1)).all()
    assert _contains(mesh, o.elem, x, y).all()


def test_slip_velocity_reversal_exact_with_zero_model_terms():
    """With G = 0 and C0 = 0 (SLM with C0 = -2/3 makes G = 0) the velocity update is
    the identity, so the reflected velocity is exactly the mirrored one."""
    mesh = M.box(6, 6, 1.0, 1.0, 0.0, 0, M.BC_SLIP)
    o = O.Oracle(mesh, CF.params(frozen=1, C0=-2.0 / 3.0))
    U0, R0, Om0 = CF._iso(mesh.n_nodes)
    o.seed(dict(ppe=2, seed=1, psi_mode=0, U0=U0, R0=R0, Om0=Om0))
    o.set_stats(CF.frozen_stats_for(mesh, U=(0, 0, 0)))
    o.cp.C0 = -2.0 / 3.0
    rng = np.random.default_rng(4)
    n = 3000
    e0 = rng.integers(0, mesh.n_elems, n)
    c = mesh.node_xy[mesh.elem_nodes[e0]].mean(axis=1)
    u, v = rng.uniform(-10, 10, n), rng.uniform(-10, 10, n)
    _place(o, e0, c[:, 0], c[:, 1], u, v)
    # sqrt(C0 eps) of a negative C0 is NaN; C0 eps enters only as sqrt(C0*eps)*dW, so
    # use eps = 0 through Om = 0 instead
    o.set_stats(CF.frozen_stats_for(mesh, U=(0, 0, 0), Om=0.0))
    assert o.step(0.02) == 0
    xs, ys = c[:, 0] + u * 0.02, c[:, 1] + v * 0.02
    flipx = (xs < 0) | (xs > 1)
    flipy = (ys < 0) | (ys > 1)
    assert np.array_equal(o.state[2], np.where(flipx, -u, u))
    assert np.array_equal(o.state[3], np.where(flipy, -v, v))


def test_canyon_corners_no_particle_lost_or_inside_blocks():
    mesh = M.canyon(6000, 0.15, 7)
    o = _frozen_oracle(mesh)
    rng = np.random.default_rng(5)
    n = 30000
    # start near the block corners with fast random velocities
    corners = np.array([[7, 3], [9, 3], [11, 3], [13, 3], [7, 0], [9, 0], [11, 0], [13, 0]], float)
    k = rng.integers(0, len(corners), n)
    p = corners[k] + rng.uniform(-0.4, 0.4, (n, 2))
    om = O.OracleMesh(mesh)
    br = np.array([om.locate_brute(a, b) for a, b in p])
    ok = br >= 0
    p, br = p[ok], br[ok]
    n = p.shape[0]
    u = rng.uniform(-40, 40, (n, 2))
    _place(o, br, p[:, 0], p[:, 1], u[:, 0], u[:, 1])
    o.step(0.01)
    cnt = o.counter_dict()
    assert cnt["lost"] == 0
    x, y = o.state[0], o.state[1]
    assert _contains(mesh, o.elem, x, y).all()
    for (x0, x1, y1) in mesh.meta["blocks"]:
        assert not ((x > x0 + 1e-12) & (x < x1 - 1e-12) & (y < y1 - 1e-12)).any()
    assert cnt["reflect"] > 0 and cnt["fallback"] + cnt["brute"] > 0


def test_count_conservation_over_a_run():
    w = CF.periodic_square(n=8, ppe=30, steps=20)
    o = O.Oracle(w.mesh, w.params)
    o.seed(w.seed)
    npart = o.state.shape[1]
    for _ in range(20):
        assert o.step(w.dt) == 0
        assert o.elem_stats[0].sum() == npart
        assert np.array_equal(np.bincount(o.elem, minlength=w.mesh.n_elems), o.elem_stats[0])
