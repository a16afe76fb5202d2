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
    assert not bad, f"{what} nodal statistics mismatch (rtol {rtol}): {bad}"
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
