"""Comparison helpers for GPU-versus-oracle parity (shared by the GPU tests).

Tolerance definition: |a - b| <= rtol * (|b| + s_q) with a per-quantity scale
s_q: velocity -> RMS speed of the reference state, omega -> mean omega,
psi -> 1; nodal statistics -> RMS of the field.

Positions are compared against the size of the particle's host element,
h_e = sqrt(2 A_e) (the leg of a right triangle of that area):
|a - b| <= rtol * h_e + 2 u_T |b|, where u_T is the unit roundoff of the
stored precision (2^-53 for binary64, 2^-24 for binary32).  A coordinate's
magnitude depends only on where the origin is, so it does not scale the
tolerance; the second term allows the storage rounding of the coordinate
itself (one unit in the last place).
"""
import numpy as np


def elem_size(mesh):
    """h_e = sqrt(2 A_e) of every element."""
    return np.sqrt(2.0 * np.abs(mesh.areas()))


def state_scales(ref_state):
    u_rms = float(np.sqrt((ref_state[2:5] ** 2).sum(0).mean()))
    om = float(np.abs(ref_state[5]).mean())
    return np.array([0.0, 0.0, u_rms, u_rms, u_rms, om, 1.0])


def max_rel_err(a, b, scale):
    """Largest |a - b| / (|b| + scale); identical values count as 0 (also
    when both and the scale are zero)."""
    if not a.size:
        return 0.0
    d = np.abs(a - b)
    den = np.abs(b) + scale
    r = np.where(d == 0.0, 0.0, d / np.where(den > 0.0, den, 1e-300))
    return float(r.max())


def position_err(a, b, h, unit_roundoff):
    """Largest (|a - b| - 2 u_T |b|) / h_e, at least 0."""
    if not a.size:
        return 0.0
    d = np.abs(a - b) - 2.0 * unit_roundoff * np.abs(b)
    return float(np.max(np.maximum(d, 0.0) / h))


def compare_state(gpu_state, ref_state, mesh, rtol, what="", *, elem, fp32=None):
    """Compare (7, n) particle states.  elem: the reference host elements (n,)
    that set the position scale.  fp32: whether the state is stored in
    binary32 (default: inferred from rtol > 1e-9)."""
    elem = np.asarray(elem)
    assert elem.shape == (ref_state.shape[1],)
    if fp32 is None:
        fp32 = rtol > 1e-9
    u = 2.0 ** -24 if fp32 else 2.0 ** -53
    h = elem_size(mesh)[elem]
    s = state_scales(ref_state)
    errs = [position_err(gpu_state[f], ref_state[f], h, u) for f in range(2)]
    errs += [max_rel_err(gpu_state[f], ref_state[f], s[f]) for f in range(2, 7)]
    names = ["x", "y", "u", "v", "w", "omega", "psi"]
    bad = [(n, e) for n, e in zip(names, errs) if not e <= rtol]
    assert not bad, f"{what} state mismatch (rtol {rtol}): {bad}"
    return dict(zip(names, errs))


def compare_stats(gpu, ref, rtol, fields=range(25), what=""):
    out = {}
    for f in fields:
        s = float(np.sqrt((ref[f] ** 2).mean())) + 1e-300
        out[f] = max_rel_err(gpu[f], ref[f], s)
    bad = {f: e for f, e in out.items() if not e <= rtol}
    assert not bad, f"{what} statistics mismatch (rtol {rtol}): {bad}"
    return out


def compare_elements(gpu_el, gpu_state, ref_el, ref_state, mesh, what="", fp32=False):
    """Host elements.  FP64 state: bit-exact.  FP32 state: the position noise
    is drawn on the binary32 transcendental units on the GPU and in binary64
    by the oracle, so a stored coordinate may differ by one unit in the last
    place; where both coordinates are bit-identical the elements must be too,
    and where they differ the GPU's element must contain the GPU's position
    (closed element test in binary64; a point within an ulp of an edge lies in
    either neighbour).  Returns the number of particles whose positions
    differ."""
    gpu_el = np.asarray(gpu_el)
    ref_el = np.asarray(ref_el)
    if not fp32:
        assert np.array_equal(gpu_el, ref_el), f"{what}: {(gpu_el != ref_el).sum()} element mismatches"
        return 0
    same = (gpu_state[0] == ref_state[0]) & (gpu_state[1] == ref_state[1])
    bad = same & (gpu_el != ref_el)
    assert not bad.any(), f"{what}: {bad.sum()} element mismatches at bit-identical positions"
    idx = np.flatnonzero(~same)
    if idx.size:
        import oracle as O
        om = O.OracleMesh(mesh)
        for i in idx:
            lam = om.lambdas(int(gpu_el[i]), float(gpu_state[0, i]), float(gpu_state[1, i]))
            assert (lam >= 0.0).all(), f"{what}: particle {i} is outside its GPU host element"
    return int(idx.size)


def derivative_bounds(mesh, gpu, ref):
    """Per-node bounds (tol1, tol2) on the discrepancy of the FEM derivative
    fields, first derivatives 15-20 and Laplacians 21-23, that follows from
    the discrepancy of the nodal means 0-2 they are formed from (eq:gradient
    with the two-pass node averaging).

    A nodal first derivative averages, over the c elements of the node's ring,
    the element gradient sum_k m_k grad N_k.  For a linear triangle
    |grad N_k| = L_k / (2A), L_k the edge opposite vertex k, so a change of
    at most d in every mean moves each component by at most a1 d, with
    r_e = P_e / (2A_e) (P_e the perimeter) and a1 = max of r_e over the ring.
    The Laplacians apply the same operator to the first derivatives: their
    change is at most max over the ring of r_e times the largest tol1 at the
    element's nodes.  Each side also rounds its own sums, at most 6c
    operations (forming ring weights, then applying them) on terms of size at
    most a M, M the largest magnitude of the operator's input: gamma a M with
    gamma = 12 c_max 2^-53 covers both sides.  d is the measured largest
    discrepancy of fields 0-2."""
    xy = np.asarray(mesh.node_xy, np.float64)
    en = np.asarray(mesh.elem_nodes)
    mst = np.asarray(mesh.node_master)
    nn = xy.shape[0]
    p = xy[en]  # (ne, 3, 2)
    edges = np.roll(p, -1, axis=1) - p
    perim = np.sqrt((edges ** 2).sum(-1)).sum(1)
    area2 = np.abs(edges[:, 0, 0] * edges[:, 1, 1] - edges[:, 0, 1] * edges[:, 1, 0])
    r = perim / area2
    q = mst[en]  # masters of each element's nodes
    a1 = np.zeros(nn)
    cnt = np.zeros(nn, np.int64)
    for k in range(3):
        np.maximum.at(a1, q[:, k], r)
        np.add.at(cnt, q[:, k], 1)
    s = r * a1[q].max(1)
    a2 = np.zeros(nn)
    for k in range(3):
        np.maximum.at(a2, q[:, k], s)
    gamma = 12.0 * int(cnt.max()) * 2.0 ** -53
    d0 = float(np.abs(np.asarray(gpu)[0:3] - np.asarray(ref)[0:3]).max())
    M0 = float(np.abs(np.asarray(ref)[0:3]).max())
    M1 = float(np.abs(np.asarray(ref)[15:21]).max())
    e0 = d0 + gamma * M0
    tol1 = (a1 * e0)[mst]
    tol2 = (a2 * e0 + gamma * a1 * M1)[mst]
    return tol1, tol2


def compare_derivatives(mesh, gpu, ref, what=""):
    """Fields 15-23 within derivative_bounds; returns the largest ratio of
    discrepancy to bound for the first derivatives and the Laplacians."""
    tol1, tol2 = derivative_bounds(mesh, gpu, ref)
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    r1 = float((np.abs(gpu[15:21] - ref[15:21]) / np.maximum(tol1, 1e-300)).max())
    r2 = float((np.abs(gpu[21:24] - ref[21:24]) / np.maximum(tol2, 1e-300)).max())
    assert r1 <= 1.0 and r2 <= 1.0, f"{what}: derivative discrepancy over its bound ({r1:.3g}, {r2:.3g})"
    return r1, r2
