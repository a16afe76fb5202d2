"""Pins for two parts of the oracle that uniform fields cannot tell apart.

* The ELEM node value (Ch.3, Sec. Estimation of Eulerian statistics, Fig.
  mesh-particles): the plain average of the element means and 1/N central
  moments over the surrounding elements that hold particles, every element
  counting once whatever its particle count; field 24 is the number of
  particles in those elements; a node with none keeps its previous values.
  Checked against a NumPy group-by on particles spread unevenly (0 to 40 per
  element, element-dependent means), where a count-weighted average differs by
  far more than the tolerance.  Periodic nodes gather the elements on both
  sides of the seam.
* The local elliptic-relaxation tensor (eq:elliptic-relaxation-Lagrangian with
  L -> 0): wp_ij = (1 - C1)/2 k <omega> delta_ij + k H_ijkl d<U_k>/dx_l with
  the fourth-order tensor of eq:H built explicitly from Kronecker deltas and
  b_ij of eq:bij, A_v = min(1, C_v det<u_i u_j> / (2k/3)^3), contracted with
  einsum, for anisotropic Reynolds stresses and full in-plane gradients.
"""
import numpy as np
import pytest

import oracle as O
from synth import configs as CF
from synth import meshes as M

PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2), (4, 4), (0, 4), (1, 4), (2, 4)]


def _uneven_particles(mesh, seed):
    rng = np.random.default_rng(seed)
    ne = mesh.n_elems
    counts = rng.choice([0, 0, 1, 2, 3, 7, 18, 40], size=ne)
    elem = np.repeat(np.arange(ne), counts).astype(np.int32)
    n = elem.size
    # element-dependent means so that a count-weighted node average differs
    off = rng.normal(size=(5, ne)) * np.array([1.0, 0.7, 0.4, 0.3, 0.5])[:, None]
    state = np.zeros((7, n))
    state[0:2] = 0.0  # positions play no part in ELEM statistics
    state[2:7] = off[:, elem] + rng.normal(size=(5, n)) * np.array([0.3, 0.2, 0.1, 0.2, 0.25])[:, None]
    state[5] = np.abs(state[5]) + 0.1
    return counts, elem, state


def _groupby_nodes(mesh, counts, elem, state, prev):
    """The definition with NumPy: element group-by, then per master node the
    unweighted average over its non-empty surrounding elements."""
    ne, nn = mesh.n_elems, mesh.n_nodes
    N = np.bincount(elem, minlength=ne).astype(float)
    q = state[2:7]
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.stack([np.bincount(elem, weights=q[f], minlength=ne) for f in range(5)]) / N
        cov = np.stack([np.bincount(elem, weights=(q[a] - mean[a, elem]) * (q[b] - mean[b, elem]),
                                    minlength=ne) for a, b in PAIRS]) / N
    ev = np.vstack([mean, cov])  # (15, ne)
    master = mesh.node_master
    # element e surrounds master node m if one of its nodes maps to m (once)
    inc = {}
    for e in range(ne):
        for m in set(master[mesh.elem_nodes[e]].tolist()):
            inc.setdefault(m, []).append(e)
    out = prev.copy()
    out_w = prev.copy()
    sup = np.zeros(nn)
    for m, es in inc.items():
        es = np.array(es)
        es = es[N[es] > 0]
        sup[m] = N[es].sum()
        if es.size:
            out[:15, m] = ev[:, es].mean(axis=1)
            out_w[:15, m] = (ev[:, es] * N[es]).sum(axis=1) / N[es].sum()
    out[:, master != np.arange(nn)] = out[:, master[master != np.arange(nn)]]
    return out, out_w, sup, inc


@pytest.mark.parametrize("which", ["canyon", "periodic"])
def test_elem_node_average_unweighted_over_nonempty(which):
    mesh = M.canyon(3000, 0.15, 2) if which == "canyon" else M.periodic_square(6)
    counts, elem, state = _uneven_particles(mesh, seed=4)
    nn = mesh.n_nodes
    prev = np.random.default_rng(9).normal(size=(25, nn))
    o = O.Oracle(mesh, CF.params())
    o.state, o.elem = state, elem
    o.id = np.arange(elem.size, dtype=np.uint32)
    o.stats = prev.copy()
    st = o.estimate()
    ref, ref_w, sup, inc = _groupby_nodes(mesh, counts, elem, state, prev)
    masters = np.flatnonzero(mesh.node_master == np.arange(nn))
    scale = np.sqrt((ref[:15, masters] ** 2).mean(axis=1))[:, None]
    err = np.abs(st[:15, masters] - ref[:15, masters]) / scale
    assert err.max() < 1e-13, err.max()
    assert np.array_equal(st[24, masters], sup[masters])
    # the data tell the readings apart: count weighting is far off
    dw = np.abs(ref_w[:15, masters] - ref[:15, masters]) / scale
    assert dw.max() > 0.05
    # nodes whose surrounding elements are all empty keep the previous values
    empty = [m for m in masters if counts[inc[m]].sum() == 0]
    if which == "canyon":
        assert len(empty) > 0
    for m in empty:
        assert np.array_equal(st[:15, m], prev[:15, m])
    # identified nodes carry their master's values
    sl = np.flatnonzero(mesh.node_master != np.arange(nn))
    if which == "periodic":
        assert sl.size > 0
    assert np.array_equal(st[:15, sl], st[:15, mesh.node_master[sl]])


def _H_tensor(R, C2, g5, Cv):
    """eq:H from Kronecker deltas and eq:bij."""
    d = np.eye(3)
    k = 0.5 * np.trace(R)
    b = R / np.trace(R) - d / 3.0
    Av = min(1.0, Cv * np.linalg.det(R) / (2.0 * k / 3.0) ** 3)
    H = ((C2 * Av + g5 / 3.0) * np.einsum("ik,jl->ijkl", d, d)
         - g5 / 3.0 * np.einsum("il,jk->ijkl", d, d)
         + g5 * np.einsum("ik,jl->ijkl", b, d)
         - g5 * np.einsum("il,jk->ijkl", b, d))
    return H, k, Av


def test_local_wp_matches_explicit_H_tensor():
    mesh = M.box(6, 6)
    nn = mesh.n_nodes
    rng = np.random.default_rng(7)
    st = np.zeros((25, nn))
    Rs = []
    for n in range(nn):
        if n % 5 == 0:  # isotropic: A_v = min(1, C_v) = 1, clipped
            R = np.eye(3) * rng.uniform(0.2, 2.0)
        else:  # anisotropic, symmetric positive definite
            A = rng.normal(size=(3, 3))
            R = A @ A.T + 0.05 * np.eye(3)
        Rs.append(R)
        st[5:11, n] = [R[0, 0], R[1, 1], R[2, 2], R[0, 1], R[0, 2], R[1, 2]]
    st[3] = rng.uniform(0.3, 3.0, nn)
    st[15:21] = rng.normal(size=(6, nn))  # d<U_i>/dx, d<U_i>/dy for i = U, V, W
    p = CF.params(model=CF.MODEL_GLM)
    wp = O.Oracle(mesh, p).local_wp(st)
    C1, C2, g5, Cv = p["C1"], p["C2"], p["gamma5"], p["Cv"]
    clipped = unclipped = 0
    for n in range(nn):
        H, k, Av = _H_tensor(Rs[n], C2, g5, Cv)
        clipped += Av == 1.0
        unclipped += Av < 1.0
        grad = np.zeros((3, 3))  # d<U_k>/dx_l, no z-derivatives
        grad[:, 0] = st[[15, 17, 19], n]
        grad[:, 1] = st[[16, 18, 20], n]
        ref = 0.5 * (1.0 - C1) * k * st[3, n] * np.eye(3) + k * np.einsum("ijkl,kl->ij", H, grad)
        got = wp[:, n].reshape(3, 3)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (n, got, ref)
        # the anisotropic terms matter at this node (b_ij != 0 there)
        if not np.allclose(Rs[n], Rs[n][0, 0] * np.eye(3)):
            Hiso, _, _ = _H_tensor(np.eye(3) * np.trace(Rs[n]) / 3, C2, g5, Cv)
            iso = 0.5 * (1.0 - C1) * k * st[3, n] * np.eye(3) + k * np.einsum("ijkl,kl->ij", Hiso, grad)
            assert np.abs(iso - ref).max() > 1e-6 * np.abs(ref).max()
    assert clipped > 0 and unclipped > 0
