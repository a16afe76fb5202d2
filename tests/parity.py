"""Comparison helpers for GPU-versus-oracle parity (shared by the GPU tests).

Tolerance definition: |a - b| <= rtol * (|b| + s_q) with a per-quantity scale
s_q: velocity -> RMS speed of the reference state, omega -> mean omega,
psi -> 1, position -> the domain extent; nodal statistics -> RMS of the field.
"""
import numpy as np


def state_scales(ref_state, mesh):
    ext = float(np.ptp(mesh.node_xy, axis=0).max())
    u_rms = float(np.sqrt((ref_state[2:5] ** 2).sum(0).mean()))
    om = float(np.abs(ref_state[5]).mean())
    return np.array([ext, ext, u_rms, u_rms, u_rms, om, 1.0])


def max_rel_err(a, b, scale):
    """Largest |a - b| / (|b| + scale); identical values count as 0 (also
    when both and the scale are zero)."""
    if not a.size:
        return 0.0
    d = np.abs(a - b)
    den = np.abs(b) + scale
    r = np.where(d == 0.0, 0.0, d / np.where(den > 0.0, den, 1e-300))
    return float(r.max())


def compare_state(gpu_state, ref_state, mesh, rtol, what=""):
    s = state_scales(ref_state, mesh)
    errs = [max_rel_err(gpu_state[f], ref_state[f], s[f]) for f in range(7)]
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
