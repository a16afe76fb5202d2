"""Pins for the oracle's IECM mixing (eq:IECM) with the velocity-conditioned
scalar mean (Sec. Estimation of the velocity-conditioned scalar mean, App. B)
and the source-aware micromixing time scale (eq:micromixing-timescale-canyon):

- hand-worked bins of the sort-and-divide procedure, with odd counts and the
  adaptive stop;
- with one conditioning direction the bins are the equal-count quantile
  groups of that velocity component (NumPy's lexsort);
- invariants: the result does not depend on the storage order, exact copies
  are ordered by id, a constant scalar is returned exactly, the bin means
  conserve each element's scalar sum;
- one IECM step relaxes each particle toward the conditioned mean of the
  start of the step and conserves the total scalar when t_m is uniform;
- the source-aware time scale against its closed form at element centroids
  (ELEM) and particle positions (SHAPE)."""
import numpy as np
import pytest

import oracle as O
from synth import configs as CF
from synth import meshes as M


def _oracle(mesh, u, v, w, psi, elem, ids, **kw):
    o = O.Oracle(mesh, CF.params(mix_model=CF.MIX_IECM, **kw))
    n = len(u)
    st = np.zeros((7, n))
    cen = mesh.node_xy[mesh.elem_nodes].mean(1)
    st[0:2] = cen[np.asarray(elem, np.int64)].T
    st[2], st[3], st[4], st[5], st[6] = u, v, w, 1.0, psi
    o.state = st
    o.elem = np.asarray(elem, np.int32)
    o.id = np.asarray(ids, np.uint32)
    return o


# eight particles of one element: id, u, v, psi
_HAND = np.array([[0, 0.1, 0.9, 1.0], [1, 0.2, 0.1, 2.0], [2, 0.3, 0.5, 3.0], [3, 0.4, 0.3, 4.0],
                  [4, 0.5, 0.2, 5.0], [5, 0.6, 0.8, 6.0], [6, 0.7, 0.4, 7.0], [7, 0.8, 0.6, 8.0]])


def _hand(nparts, bins, cmin, perm_seed=0):
    mesh = M.box(1, 1, 1.0, 1.0)
    rows = _HAND[:nparts][np.random.default_rng(perm_seed).permutation(nparts)]
    w = np.random.default_rng(9).normal(size=nparts)
    o = _oracle(mesh, rows[:, 1], rows[:, 2], w, rows[:, 3], np.zeros(nparts), rows[:, 0],
                cond_nu=bins[0], cond_nv=bins[1], cond_nw=bins[2], cond_min=cmin)
    cm = o.cond_means()
    return dict(zip(o.id.tolist(), cm.tolist()))


def test_hand_worked_bins():
    """(2 x 2 x 1) bins.  Sorted by u the ids are 0..7; the halves {0,1,2,3}
    and {4,5,6,7} sorted by v give 1,3,2,0 and 4,6,7,5, so the bins are
    {1,3}, {2,0}, {4,6}, {7,5} with scalar means 3, 2, 6, 7."""
    assert _hand(8, (2, 2, 1), 1) == {0: 2.0, 1: 3.0, 2: 2.0, 3: 3.0, 4: 6.0, 5: 7.0, 6: 6.0, 7: 7.0}
    # the same for any storage order
    assert _hand(8, (2, 2, 1), 1, perm_seed=5) == _hand(8, (2, 2, 1), 1)
    # (2 x 2 x 2): a third division leaves one particle per bin
    assert _hand(8, (2, 2, 2), 1) == {i: float(i + 1) for i in range(8)}


def test_hand_worked_odd_count_and_adaptive_stop():
    """Seven particles.  Level 1 splits the u order at 7/2: positions 0-3
    (ids 0-3) and 4-6 (ids 4-6).  Level 2 (four bins) splits the positions at
    0, 2, 4, 6: by v the first group is 1,3 | 2,0 and the second 4,6 | 5, so
    the means are 3, 2, 6 and 6.  With at least 2 per subgroup only the first
    level is taken (7 // 4 = 1 < 2): means 2.5 and 6.  With at least 4 none is
    (7 // 2 = 3 < 4): the element mean 4."""
    assert _hand(7, (2, 2, 1), 1) == {0: 2.0, 1: 3.0, 2: 2.0, 3: 3.0, 4: 6.0, 5: 6.0, 6: 6.0}
    assert _hand(7, (2, 2, 1), 2) == {0: 2.5, 1: 2.5, 2: 2.5, 3: 2.5, 4: 6.0, 5: 6.0, 6: 6.0}
    assert _hand(7, (2, 2, 1), 4) == {i: 4.0 for i in range(7)}


def _random_state(seed=0, nx=6, ny=5, ppe_max=90):
    mesh = M.box(nx, ny, 1.0, 1.0, jitter=0.2, seed=seed)
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, ppe_max, mesh.n_elems)
    counts[0], counts[1] = 0, 1  # an empty element and a single particle
    elem = np.repeat(np.arange(mesh.n_elems), counts)
    n = elem.size
    ids = rng.permutation(n).astype(np.uint32)
    u, v, w = rng.normal(size=(3, n))
    psi = rng.uniform(size=n)
    return mesh, u, v, w, psi, elem, ids


@pytest.mark.parametrize("nu", [1, 3, 5])
def test_one_direction_is_quantile_groups(nu):
    """(n_u x 1 x 1): the bins are the groups 0..n_u-1 of the u order (ties
    by id) with boundaries at the App. B index n_u j / n."""
    mesh, u, v, w, psi, elem, ids = _random_state(1)
    o = _oracle(mesh, u, v, w, psi, elem, ids, cond_nu=nu, cond_nv=1, cond_nw=1, cond_min=1)
    cm = o.cond_means()
    for e in range(mesh.n_elems):
        idx = np.nonzero(elem == e)[0]
        if idx.size == 0:
            continue
        # one interval: no sort, the starting order of increasing id
        order = idx[np.lexsort((ids[idx], u[idx]))] if nu > 1 else idx[np.argsort(ids[idx])]
        n = idx.size
        nb = nu if n // nu >= 1 else 1  # the adaptive stop with at least 1 per group
        grp = nb * np.arange(n) // n
        sums = np.zeros(nb)
        for j in range(n):  # App. B: in the order of the final positions
            sums[grp[j]] += psi[order[j]]
        means = sums / np.bincount(grp, minlength=nb)
        assert np.array_equal(cm[order], means[grp]), e


def test_invariants():
    mesh, u, v, w, psi, elem, ids = _random_state(2)
    # exact copies (redistribution makes them): same velocity and scalar
    u[5:9], v[5:9], w[5:9], psi[5:9] = u[4], v[4], w[4], psi[4]
    kw = dict(cond_nu=5, cond_nv=5, cond_nw=5, cond_min=2)
    o = _oracle(mesh, u, v, w, psi, elem, ids, **kw)
    cm = o.cond_means()
    assert np.all(np.isfinite(cm))
    # storage order does not matter
    p = np.random.default_rng(7).permutation(u.size)
    o2 = _oracle(mesh, u[p], v[p], w[p], psi[p], elem[p], ids[p], **kw)
    assert np.array_equal(o2.cond_means(), cm[p])
    # bin means conserve each element's scalar sum
    for e in range(mesh.n_elems):
        sel = elem == e
        if sel.any():
            assert abs(cm[sel].sum() - psi[sel].sum()) <= 1e-12 * max(1.0, psi[sel].sum())
    # a constant (dyadic) scalar comes back exactly
    o3 = _oracle(mesh, u, v, w, np.full(u.size, 0.375), elem, ids, **kw)
    assert np.all(o3.cond_means() == 0.375)
    # a single particle is its own mean
    one = np.nonzero(elem == 1)[0]
    assert np.array_equal(cm[one], psi[one])


def test_bins_have_the_equal_count_sizes():
    """Every bin of an element holds floor(n/N_c) or ceil(n/N_c) particles,
    N_c = the product of the levels taken; at least cond_min each."""
    mesh, u, v, w, psi, elem, ids = _random_state(3, ppe_max=300)
    psi = np.random.default_rng(11).uniform(size=u.size)  # bin means distinct (almost surely)
    o = _oracle(mesh, u, v, w, psi, elem, ids, cond_nu=5, cond_nv=5, cond_nw=5, cond_min=2)
    cm = o.cond_means()
    for e in range(mesh.n_elems):
        sel = np.nonzero(elem == e)[0]
        n = sel.size
        if n == 0:
            continue
        nc = 1
        for f in (5, 5, 5):
            if n // (nc * f) < 2:
                break
            nc *= f
        _, sizes = np.unique(cm[sel], return_counts=True)
        assert sizes.size == nc, (e, n, nc, sizes.size)
        assert set(sizes.tolist()) <= {n // nc, -(-n // nc)} and sizes.min() >= min(2, n)


def _iecm_step(stats_mode=CF.STATS_ELEM):
    w = CF.periodic_square(n=8, ppe=60, seed=3)
    w.params = dict(w.params, frozen=1, mix_model=CF.MIX_IECM, cond_nu=3, cond_nv=3, cond_nw=2,
                    cond_min=2, stats_mode=stats_mode)
    fz = CF.frozen_stats_for(w.mesh, U=(0.2, 0.1, 0.0), R_diag=(0.5, 0.4, 0.3), Om=1.0)
    o = O.Oracle(w.mesh, w.params)
    o.seed(dict(w.seed, psi_mode=CF.PSI_GAUSS_X, a=0.5, b=0.2))
    o.state[6] += 0.3 * o.state[2]  # scalar correlated with velocity
    o.set_stats(fz)
    return o, w


def test_iecm_step_relaxes_toward_start_of_step_conditioned_mean():
    o, w = _iecm_step()
    cm = o.cond_means()
    psi0, ids0 = o.state[6].copy(), o.id.copy()
    a = w.dt * 0.5 * w.params["Cphi"] * 1.0  # dt / t_m with 1/t_m = C_phi <omega> / 2
    o.step(w.dt)
    assert np.array_equal(o.id, ids0)
    assert np.allclose(o.state[6], psi0 - a * (psi0 - cm), rtol=0, atol=1e-15)
    # t_m uniform: the bin means conserve the total scalar
    assert abs(o.state[6].sum() - psi0.sum()) < 1e-11


@pytest.mark.parametrize("stats_mode", [CF.STATS_ELEM, CF.STATS_SHAPE])
def test_source_aware_timescale_closed_form(stats_mode):
    """IEM with eq:micromixing-timescale-canyon and frozen uniform statistics:
    each particle's scalar relaxes toward <phi> at 1/t_m with t_m = min(C_s
    (r0^2/eps)^(1/3) + C_t d/U_c, max(k/eps, C_T sqrt(nu/eps))), d measured
    from the element centroid (ELEM) or the particle (SHAPE)."""
    mesh = M.box(10, 10, 1.0, 1.0, jitter=0.2, seed=4, bc=M.BC_SLIP)
    nu, U, Om, Phi = 1e-3, (0.3, 0.1, 0.05), 1.2, 0.5
    src = (0.4, 0.6, 0.05)
    p = CF.params(frozen=1, tm_mode=CF.TM_SOURCE, nu=nu, stats_mode=stats_mode, src_x=src[0],
                  src_y=src[1], src_r=src[2])
    fz = CF.frozen_stats_for(mesh, U=U, R_diag=(0.7, 0.6, 0.5), Om=Om, Phi=Phi)
    o = O.Oracle(mesh, p)
    o.seed(dict(ppe=20, seed=5, psi_mode=CF.PSI_BERNOULLI, a=0, b=0, c=0, U0=fz[0:3], R0=fz[5:11],
                Om0=fz[3]))
    o.set_stats(fz)
    x0, y0, e0, psi0 = o.state[0].copy(), o.state[1].copy(), o.elem.copy(), o.state[6].copy()
    dt = 0.01
    o.step(dt)
    k = 0.5 * (0.7 + 0.6 + 0.5)
    eps = Om * (k + nu * p["CT"] ** 2 * Om)
    if stats_mode == CF.STATS_ELEM:
        pt = mesh.node_xy[mesh.elem_nodes[e0]].sum(1) / 3.0
    else:
        pt = np.stack([x0, y0], 1)
    d = np.hypot(pt[:, 0] - src[0], pt[:, 1] - src[1])
    ts = p["Cs"] * np.cbrt(src[2] ** 2 / eps) + p["Ct"] * d / np.sqrt(sum(c * c for c in U))
    tm = np.minimum(ts, max(k / eps, p["CT"] * np.sqrt(nu / eps)))
    assert (ts <= tm).any() and (ts > tm).any()  # both branches occur
    expect = psi0 - dt / tm * (psi0 - Phi)
    outside = np.hypot(o.state[0] - src[0], o.state[1] - src[1]) > src[2]  # the source resets psi
    assert outside.sum() > 0.9 * outside.size
    np.testing.assert_allclose(o.state[6][outside], expect[outside], rtol=1e-13, atol=1e-15)
