"""Convenience: build a seeded Context from a workload description.

A workload is any object with the attributes mesh, params (dict), seed (dict
for pdf_seed_desc), precision ("f32"/"f64"), gradp and wp (optional nodal
arrays) -- e.g. the synthetic workloads in synth/configs.py.
"""
from __future__ import annotations

from . import _lib


def workload_context(w, device=0, reorder_every=None, seed=True, stream=None):
    ctx = _lib.Context(w.mesh, w.params, w.precision, device=device, stream=stream,
                       reorder_every=reorder_every)
    if getattr(w, "gradp", None) is not None:
        ctx.set_nodal_field(_lib.FIELD_GRADP, w.gradp)
    if getattr(w, "wp", None) is not None:
        ctx.set_nodal_field(_lib.FIELD_WP, w.wp)
    if seed:
        ctx.seed(w.seed)
    return ctx
