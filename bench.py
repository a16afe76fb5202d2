#!/usr/bin/env python3
"""Throughput benchmark of the particle hot path on one MI355X.

One step = one pass of the whole hot path over the synthetic workload:
element records, the fused particle kernel (noise, SDEs, tracking and
boundary conditions, element sums) and the two-pass nodal estimator with its
derivatives (plus the periodic reorder).  Inputs are resident in HBM before the
timed region; the timed region is exactly K calls' worth of steps bracketed by
device synchronisation.

Prints one JSON line.  Its roofline object prices the dominant kernel,
k_advance: algorithmic bytes per launch (68 B per particle and 384 B per
element in FP32) over the launch time measured with HIP events on the
context's stream, against the 8 TB/s HBM peak, with the HBM traffic of the
committed rocprofv3 counters when the kernel source and configuration match
the ones they were taken at.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s + %HBM peak; learned-vs-plain cost at equal stat error"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (constructor, description)
    "channel_block": ("channel_block", "graded channel with a floor block, ~1M triangles, "
                      "100 particles/element (~100M), FP32, GLM + gamma frequency + IEM"),
    "canyon": ("canyon", "street-canyon box with two blocks, ~200k triangles, 50 particles/element "
               "(~10M), FP32, GLM + gamma frequency + IEM, disc source"),
    "channel": ("channel", "plane channel, 20k triangles, 100 particles/element (2M), FP32, GLM"),
    "periodic_square": ("periodic_square", "periodic unit square, 2048 triangles, 50 particles/"
                        "element (102400), FP64, simplified Langevin"),
}


def kernel_bytes(w, tsize, shape=False):
    """Algorithmic HBM bytes of one launch of the fused particle kernel:
    per particle the state is read (7 values + element + id) and written
    (7 values + element); per element its record (32 values; 88 for the
    shape-function mode) is read once; the 16 FP64 sums of every element
    (every node in the shape-function mode) are read and written once."""
    n_p, n_e, n_n = w.n_particles, w.mesh.n_elems, w.mesh.n_nodes
    per_particle = (7 * tsize + 4 + 4) + (7 * tsize + 4)
    if shape:
        per_element = 88 * tsize + 2 * 16 * 8 * n_n / n_e
    else:
        per_element = 32 * tsize + 2 * 16 * 8
    return int(n_p * per_particle + n_e * per_element), per_particle, round(per_element, 1)


def copy_bandwidth(mib=2048, reps=5):
    """Best read-plus-write rate (GB/s) of a plain device-to-device copy of
    mib MiB, timed with events on the current stream."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * n * 4 / best / 1e9


def source_hash():
    h = hashlib.sha256()
    for f in ("k_particles.hip", "rng.h", "pdf_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1006_0720_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def profile_counters(workload, cfg):
    """Committed rocprofv3 counter summary of the particle kernel for this
    workload, or None when none exists, the kernel source changed since, or
    this run's configuration (particle count, kernel variant) is not the one
    the counters were taken at."""
    path = os.path.join(ROOT, "profiles", f"k_advance_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != source_hash():
        return None
    if any(cfg.get(k) != v for k, v in d.get("bench_config", {}).items()):
        return None
    return d


# plain (non-packed) VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def host_cpu():
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    try:
        lines = open("/proc/cpuinfo").read().splitlines()
    except OSError:
        return None
    names = [ln.split(":", 1)[1].strip() for ln in lines if ln.startswith("model name")]
    return f"{names[0]} ({len(names)} logical CPUs)" if names else None


def cpu_baseline(wname, w):
    """The FP64 oracle (single thread) on a bounded sample of the workload:
    the full mesh at a reduced particle count, a few steps."""
    import numpy as np

    import oracle as O

    target = 10_000_000
    ppe = max(10, min(int(w.seed["ppe"]), target // w.mesh.n_elems))
    steps = 2 if w.mesh.n_elems * ppe > 4_000_000 else 5
    seed = dict(w.seed, ppe=ppe)
    o = O.Oracle(w.mesh, w.params, store_fp32=(w.precision == "f32"), gradp=w.gradp, wp=w.wp)
    o.seed(seed)
    t0 = time.perf_counter()
    for _ in range(steps):
        o.step(w.dt)
    dt = time.perf_counter() - t0
    n = w.mesh.n_elems * ppe
    return {"value": n * steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"same mesh ({w.mesh.n_elems} elements) at {ppe} particles/element "
                      f"({n} particles), {steps} steps, FP64 oracle, 1 thread, includes the "
                      f"statistics estimate of each step",
            "host_cpu": host_cpu()}


def denoise_timing(ctx, calls):
    """Wall time of one pdf_denoise_stats call on the context's latest
    statistics (the call ends with a stream synchronisation)."""
    import numpy as np
    import torch

    from paper_1006_0720_amd import _lib

    dn = _lib.Denoiser(ctx, hidden=128, seed=1)
    dn.set_norm(np.zeros(48, np.float32), np.ones(48, np.float32), np.ones(8, np.float32))
    for _ in range(3):
        dn.denoise(3.0, device=True)
    ts = []
    for _ in range(calls):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dn.denoise(3.0, device=True)
        ts.append(time.perf_counter() - t0)
    dn.close()
    return {"n_nodes": ctx.n_nodes, "hidden": 128, "calls": calls, "ms_per_call_median": 1e3 * float(np.median(ts)),
            "weights": "seeded, untrained"}


def denoise_study(mode, out_path=""):
    """Learned-vs-plain cost at equal nodal-statistics error (the protocol of
    paper_1006_0720_amd/denoise_study.py: held-out source positions scored
    against the ensemble mean of independent high-count runs).
      bench     the default line's bounded study: the street-canyon mesh
                (~200k triangles), statistics fed back with the particle
                redistribution keeping 3 per element, 10 vs 200 particles per
                element, 16 training pairs, 16000 Adam steps, 4 held-out
                sources x 4 reference runs, plain runs at 20, 40, 80 and 160
                per element
      full      the same with 64 training pairs (4 x 4 = 16 held-out runs)
      quick     a 20k-triangle canyon, for tests
      c5        the 1M-triangle channel with a floor block, 10 vs 100 per
                element, fed back with redistribution, the scalar line at a
                different x in each run; 32 training pairs, 16000 Adam
                steps, plain runs at 20, 40, 80, 160, 200 and 240 per element
    A '-frozen' suffix freezes the model coefficients instead of feeding the
    statistics back."""
    import numpy as np

    from paper_1006_0720_amd.denoise_study import study
    from synth import configs as CF
    from synth import meshes as M

    frozen = mode.endswith("-frozen")
    mode = mode[:-7] if frozen else mode
    base = dict(frozen=frozen, min_ppe=0 if frozen else 3)
    if mode == "c5":
        mesh = M.channel_block(1_000_000, 0.15, 0)
        kw = dict(n_train=32, n_test=3, n_ref=3, steps_spin=100, n_snap=5, every=10, train_steps=16000,
                  batch=8192, ppe_low=10, ppe_high=100, eval_ppes=(20, 40, 80, 160, 200, 240),
                  source_box=(1.0, 4.0, 0.5, 1.5, 0.05))

        def make(ppe, seed, src):
            w = CF.channel_block(mesh=mesh, ppe=ppe, seed=seed)
            w.seed = dict(w.seed, a=src[0])  # the Gaussian scalar line at x = src[0]
            return w
    else:
        if mode == "quick":
            mesh = M.canyon(20_000, 0.15, 0)
            kw = dict(n_train=8, n_test=2, n_ref=3, steps_spin=40, n_snap=4, every=10, train_steps=1500,
                      batch=4096, eval_ppes=(20, 40))
        else:
            mesh = M.canyon(200_000, 0.15, 0)
            kw = dict(n_train=64 if mode == "full" else 16, n_test=4, n_ref=4, steps_spin=100, n_snap=5,
                      every=10, train_steps=16000, batch=8192, eval_ppes=(20, 40, 80, 160))

        def make(ppe, seed, src):
            return CF.canyon(mesh=mesh, ppe=ppe, seed=seed, src=src)

    kw.update(base)
    res, params, norm = study(make, log=lambda m: print(m, file=sys.stderr, flush=True), **kw)
    res["mesh_elements"] = mesh.n_elems
    res["mode"] = mode + ("-frozen" if frozen else "")
    lv = res["learned"]
    res["summary"] = {k: {"E": round(lv[k]["E"], 4), "ppe_eq": round(lv[k]["ppe_eq"], 1),
                          "cost_ratio": round(lv[k]["cost_ratio"], 3)}
                      for k in ("tau3_noise", "tau3_calibrated", "no_fallback")}
    res["target_cost_ratio"] = 4.0
    res["target_met_with_fallback"] = bool(lv["tau3_calibrated"]["cost_ratio"] >= 4.0)
    if out_path:
        base_p = os.path.splitext(out_path)[0]
        json.dump(res, open(base_p + ".json", "w"), indent=1)
        np.savez(base_p + ".npz", params=params, mu=norm[0], sig=norm[1], scale=norm[2])
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 24 timed steps after 8 warm-up steps hold exactly three of the reorders
    # that run every 8 steps: the timed steps carry the reorder's amortized
    # share, neither more nor less
    ap.add_argument("--steps", type=int, default=24)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--workload", default="channel_block", choices=sorted(WORKLOADS))
    ap.add_argument("--reorder-every", type=int, default=8)
    ap.add_argument("--ppe", type=int, default=0,
                    help="particles per element at seeding (0: the workload's own count)")
    ap.add_argument("--min-ppe", type=int, default=0,
                    help="particle redistribution: minimum particles per element (0: off)")
    ap.add_argument("--stats-mode", default="elem", choices=["elem", "shape"],
                    help="statistics at particles and nodes: element averages (the paper's) or "
                         "shape-function interpolation and weighting")
    ap.add_argument("--mix", default="iem", choices=["iem", "iecm"],
                    help="micromixing: IEM (eq:IEM) or IECM with the velocity-conditioned mean "
                         "(eq:IECM, 5 x 5 x 5 bins, at least 2 per subgroup)")
    ap.add_argument("--wp", default="local", choices=["local", "elliptic"],
                    help="tensor wp_ij of the generalized Langevin model: the local right-hand side of the "
                         "elliptic relaxation, or its finite-element solve every step")
    ap.add_argument("--ell-precond", default="multigrid", choices=["multigrid", "jacobi"],
                    help="preconditioner of the elliptic relaxation's conjugate gradients")
    ap.add_argument("--proj", action="store_true",
                    help="the stabilized mean-pressure projection every step (statistics fed back)")
    ap.add_argument("--proj-precond", default="multigrid", choices=["multigrid", "jacobi"],
                    help="preconditioner of the projection's conjugate gradients")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--denoise-study", default="bench",
                    help="the learned-vs-plain study added to the line as learned_vs_plain: 'bench' (the "
                         "default, bounded: street canyon, fed back, 16 training pairs, 4 held-out sources x 4 "
                         "reference runs), 'full' (64 training pairs), 'quick', 'c5' (the 1M-triangle channel, "
                         "10 vs 100 per element), each with an optional '-frozen' suffix; 'none' to skip")
    ap.add_argument("--denoise-calls", type=int, default=0,
                    help="also time this many pdf_denoise_stats calls (features, fused MLP, merge; H = 128, "
                         "seeded untrained weights) on the workload's nodal statistics")
    ap.add_argument("--study-out", default="", help="write the study result and weights here (.json/.npz)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the particle hot path is built and measured on a "
              "single MI355X; multi-GPU sharding (spatial domain decomposition) is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1006_0720_amd.runner import workload_context
    from synth import configs as CF

    ctor, desc = WORKLOADS[args.workload]
    w = getattr(CF, ctor)(**({"ppe": args.ppe} if args.ppe > 0 else {}))
    shape = args.stats_mode == "shape"
    if shape:
        w.params = dict(w.params, stats_mode=CF.STATS_SHAPE)
    if args.min_ppe > 0:
        w.params = dict(w.params, min_ppe=args.min_ppe)
    if args.wp == "elliptic":
        # solved to 1e-6 of the right-hand side, far below the statistical noise of its input
        w.params = dict(w.params, wp_source=CF.WP_ELLIPTIC, ell_tol=1e-6, ell_maxit=500,
                        ell_precond=1 if args.ell_precond == "multigrid" else 0)
    if args.proj:
        # solved to 1e-6 of the right-hand side, below the statistical noise of its input;
        # C_p = 0.1 dt: the stabilizing term multiplies P' by (1 - C_p/dt) every step
        w.params = dict(w.params, proj=1, Cp=0.1 * w.dt, proj_tol=1e-6, proj_maxit=2000, frozen=0,
                        proj_precond=1 if args.proj_precond == "multigrid" else 0)
    if args.mix == "iecm":
        w.params = dict(w.params, mix_model=CF.MIX_IECM, cond_nu=5, cond_nv=5, cond_nw=5, cond_min=2)
    tsize = 4 if w.precision == "f32" else 8
    ctx = workload_context(w, device=0, reorder_every=args.reorder_every)
    stream = torch.cuda.current_stream()

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    copy_gbs = copy_bandwidth()
    ctx.advance(args.warmup, w.dt)
    torch.cuda.synchronize()
    ctx.counters(reset=True)
    ctx.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advance(args.steps, w.dt)
    stream.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    tm = ctx.timing()
    cnt = ctx.counters()
    n_p = w.n_particles
    value = n_p * args.steps / wall

    bytes_alg, per_p, per_e = kernel_bytes(w, tsize, shape)
    adv_ms = tm["advance"] / args.steps
    achieved = bytes_alg / (adv_ms * 1e-3) / 1e9
    prof = None if shape else profile_counters(
        args.workload, {"n_particles": n_p, "n_elements": w.mesh.n_elems, "stats_mode": args.stats_mode,
                        "min_ppe": args.min_ppe, "mix": args.mix, "wp": args.wp, "proj": bool(args.proj)})
    traffic = prof["traffic_bytes_per_launch"] if prof else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_advance", "kernel_ms": round(adv_ms, 4),
            "bytes_per_launch": bytes_alg, "bytes_per_particle": per_p,
            "bytes_per_element": per_e,
            # what a plain device copy reaches on this GPU (read + write bytes)
            "copy_achievable": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}
    if prof:
        # the second roof: measured VALU instructions per particle-step (SQ_INSTS_VALU)
        ipp = prof["sq"]["valu_instructions_per_particle"]
        ach = ipp * w.n_particles / (adv_ms * 1e-3)
        roof["valu"] = {"instructions_per_particle": ipp, "achieved": round(ach / 1e12, 2),
                        "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2), "unit": "Tlane-op/s",
                        "frac": round(ach / VALU_PEAK_LANE_OPS, 4)}
    step_ms = wall * 1e3 / args.steps
    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if w.precision == "f32" else "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "n_particles": n_p,
                   "n_elements": w.mesh.n_elems, "n_nodes": w.mesh.n_nodes,
                   "particles_per_element": int(w.seed["ppe"]), "dt": w.dt,
                   "reorder_every": args.reorder_every, "stats_mode": args.stats_mode,
                   "min_ppe": args.min_ppe, "mix": args.mix, "wp": args.wp, "proj": bool(args.proj)} |
                  ({"ell_precond": args.ell_precond} if args.wp == "elliptic" else {}) |
                  ({"proj_precond": args.proj_precond, "Cp": w.params["Cp"],
                    "proj_tol": w.params["proj_tol"]} if args.proj else {}),
        "roofline": roof,
        "phase_ms_per_step": {k: round(v / args.steps, 4) for k, v in tm.items()},
        "counters": {k: cnt[k] for k in ("lost", "brute", "fallback", "nonfinite", "empty_node", "redist",
                                         "ell_iters", "proj_iters")},
    }
    if args.denoise_calls > 0:
        out["denoise_inference"] = denoise_timing(ctx, args.denoise_calls)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, w)
    ctx.close()
    if args.denoise_study and args.denoise_study != "none":
        out["learned_vs_plain"] = denoise_study(args.denoise_study, args.study_out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
