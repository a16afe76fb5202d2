"""Training and evaluation of the learned denoiser, all on the GPU.

Data: runs of one workload at a low particle count (the network's input) and
at a high count (its target), sharing the initial fields and the scalar
source position but not the particle seeds.  After a spin-up, snapshots of
the nodal statistics are taken every few steps.  The network learns the
correction (high - low) of 8 nodal statistics from 48 features of the
low-count estimate; the plain estimator stays the fallback.

With frozen=True the model coefficients of every run come from one fixed
field (the high-count estimate of the seeded initial state), so low- and
high-count runs sample the same particle process.  With frozen=False the
statistics are fed back, which at low counts needs the particle
redistribution (min_ppe > 0).

Fallback: a correction of statistic q at node n is rejected where it exceeds
tau * kappa_q * SE_q(n), SE_q the plain estimator's standard error from its
own second moments and support.  kappa_q = 1 judges corrections against the
noise alone.  The calibrated kappa_q judges them against the plain
estimator's actual error, bias included: over the training runs, the ratio
|q_high - q_low| / SE_q(n) of the high-count target's departure from the
low-count estimate to the standard error is collected at every node whose
standard error is at least the 5th percentile of the positive ones (a node
with almost no spread would give an unbounded ratio), and tau * kappa_q is
set to its quantile `coverage` (0.999): only a correction larger than
almost every departure the plain estimator actually shows is rejected.  The
held-out runs play no part in it.

Evaluation on held-out source positions.  For each, the reference is the
ensemble mean of n_ref independent high-count runs at the same snapshot.  The
error of an estimate is
  E = RMS over the nodes with particles and the 8 statistics of
      (q_est - q_ref) / s_q,   s_q = RMS of q_ref over the nodes.
E_plain is measured at the low count and at eval_ppes; ppe_eq, the count at
which the plain estimator reaches E_learned, is interpolated in log-log
between the measured counts, and beyond the largest measured count taken
from E(ppe) = b/ppe + s/sqrt(ppe) (a bias and a noise term) through the two
largest.  The cost ratio is T_plain(ppe_eq) / (T_plain(low) + T_denoise) with
the measured time per step (piecewise linear in the count) and the measured
time of one denoiser call, both amortized over back-to-back launches (the
steps over 10-step stretches, the calls over 20 queued calls with no host
wait or rejection count per call; T_denoise_sync_s keeps the single call's
time with its host wait and count readback).
"""
from __future__ import annotations

import time

import numpy as np

from . import _lib
from .runner import workload_context

QUANT = [0, 1, 4, 5, 6, 8, 11, 3]
NAMES = ["U", "V", "phi", "uu", "vv", "uv", "phi'^2", "omega"]
TAU_SWEEP = (1.0, 3.0, 10.0, 30.0, 100.0)


def _run(make_workload, ppe, seed, src, steps_spin, n_snap, every, frozen_field=None, reorder_every=4,
         min_ppe=0):
    """Advance one run; returns the context, the workload, the snapshots of
    nodal statistics (torch, device) and the measured time per step."""
    import torch

    w = make_workload(ppe=ppe, seed=seed, src=src)
    if frozen_field is not None:
        w.params = dict(w.params, frozen=1)
    if min_ppe > 0:
        w.params = dict(w.params, min_ppe=min_ppe)
    ctx = workload_context(w, reorder_every=reorder_every)
    if frozen_field is not None:
        ctx.set_nodal_field(_lib.FIELD_STATS, frozen_field)
    ctx.advance(steps_spin, w.dt)
    snaps = []
    t_adv = 0.0
    for _ in range(n_snap):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.advance(every, w.dt)
        torch.cuda.synchronize()
        t_adv += time.perf_counter() - t0
        snaps.append(ctx.stats_device())
    return ctx, w, snaps, t_adv / (n_snap * every)


def _sources(rng, n, box):
    x0, x1, y0, y1, r = box
    return [(float(rng.uniform(x0, x1)), float(rng.uniform(y0, y1)), r) for _ in range(n)]


def std_error(S, C4):
    """The plain estimator's standard error of the 8 statistics at every node
    (as the merge rule forms it), from nodal statistics S [25, nn]."""
    N = S[24]
    iN = np.where(N > 0, 1.0 / np.where(N > 0, N, 1.0), 1.0)
    uu, vv, uv, pp, om = np.abs(S[5]), np.abs(S[6]), S[8], np.abs(S[11]), np.abs(S[3])
    return np.stack([np.sqrt(uu * iN), np.sqrt(vv * iN), np.sqrt(pp * iN), uu * np.sqrt(2 * iN),
                     vv * np.sqrt(2 * iN), np.sqrt((uu * vv + uv * uv) * iN), pp * np.sqrt(2 * iN),
                     om * np.sqrt(C4 * iN)])


def ppe_at_error(E, ppes, errs):
    """Particles per element at which the plain estimator's error is E: log-log
    interpolation between the measured counts; past the largest, the model
    E = b/ppe + s/sqrt(ppe) through the two largest measured counts (a
    power law through them if either coefficient comes out negative)."""
    ppes = np.asarray(ppes, float)
    errs = np.asarray(errs, float)
    o = np.argsort(ppes)
    ppes, errs = ppes[o], errs[o]
    if E >= errs[0]:
        return float(ppes[0])
    # measured errors fall with the count; the first measured count at or below E
    for k in range(1, len(ppes)):
        if errs[k] <= E:
            la, lb = np.log(ppes[k - 1]), np.log(ppes[k])
            ea, eb = np.log(errs[k - 1]), np.log(errs[k])
            return float(np.exp(la + (np.log(E) - ea) * (lb - la) / (eb - ea)))
    p1, p2, e1, e2 = ppes[-2], ppes[-1], errs[-2], errs[-1]
    A = np.array([[1 / p1, 1 / np.sqrt(p1)], [1 / p2, 1 / np.sqrt(p2)]])
    b, s = np.linalg.solve(A, [e1, e2])
    if b >= 0 and s >= 0:
        if s == 0:
            return float(b / E)
        # b x^2 + s x - E = 0 with x = 1/sqrt(ppe)
        x = (-s + np.sqrt(s * s + 4 * b * E)) / (2 * b) if b > 0 else E / s
        return float(1.0 / (x * x))
    slope = (np.log(e2) - np.log(e1)) / (np.log(p2) - np.log(p1))
    if slope >= 0:
        return float("inf")
    return float(p2 * np.exp((np.log(E) - np.log(e2)) / slope))


def study(make_workload, n_train=16, n_test=4, n_ref=4, ppe_low=10, ppe_high=200, eval_ppes=(20, 40, 80),
          steps_spin=100, n_snap=5, every=10, hidden=128, train_steps=4000, batch=8192, lr=1e-3,
          tau=3.0, seed=0, source_box=(4.0, 16.0, 3.5, 6.5, 0.3), frozen=True, min_ppe=0, coverage=0.999,
          log=print):
    """make_workload(ppe=, seed=, src=(x, y, r)) -> workload (see runner);
    source_box = (x0, x1, y0, y1, r): disc sources uniform in the box.
    n_train training pairs; n_test held-out source positions, each with one
    low-count run, n_ref high-count runs (the ensemble reference) and one
    plain run at every count of eval_ppes."""
    import torch

    t_start = time.perf_counter()
    rng = np.random.default_rng(seed)
    srcs = _sources(rng, n_train + n_test, source_box)
    F = None
    if frozen:
        c_ref = workload_context(make_workload(ppe=ppe_high, seed=seed + 77, src=srcs[0]))
        F = c_ref.stats_device()
        c_ref.close()
    feats, targs, cal_ratio = [], [], []
    dn = ctx_keep = None
    t_low, t_high = [], []
    C4 = None
    for r in range(n_train):
        c_lo, w, s_lo, tl = _run(make_workload, ppe_low, 1000 + r, srcs[r], steps_spin, n_snap, every, F,
                                 min_ppe=min_ppe)
        c_hi, _, s_hi, th = _run(make_workload, ppe_high, 5000 + r, srcs[r], steps_spin, n_snap, every, F,
                                 min_ppe=min_ppe)
        c_hi.close()
        t_low.append(tl)
        t_high.append(th)
        C4 = float(w.params["C4"])
        if dn is None:
            dn = _lib.Denoiser(c_lo, hidden=hidden, seed=seed)
            ctx_keep = c_lo
        for a, b in zip(s_lo, s_hi):
            feats.append(dn.features(a))  # raw features of the low-count estimate
            targs.append((b[QUANT] - a[QUANT]).T.float())
            A = a.cpu().numpy()
            Bn = b.cpu().numpy()
            se = std_error(A, C4)
            keep = A[24] > 0
            keep[1::4] = keep[2::4] = keep[3::4] = False  # every fourth node
            cal_ratio.append((np.abs(A[QUANT][:, keep] - Bn[QUANT][:, keep]), se[:, keep]))
        if c_lo is not ctx_keep:
            c_lo.close()
        log(f"[denoise] training run {r + 1}/{n_train} (low-count step {tl * 1e3:.3f} ms)")
    dev = np.concatenate([c[0] for c in cal_ratio], axis=1)
    sev = np.concatenate([c[1] for c in cal_ratio], axis=1)
    kappa = np.ones(8)
    for j in range(8):
        pos = sev[j] > 0
        if pos.any():
            ok = sev[j] >= np.percentile(sev[j][pos], 5.0)
            kappa[j] = max(np.quantile(dev[j][ok] / sev[j][ok], coverage) / tau, 1e-3)
    X = torch.cat(feats)
    T = torch.cat(targs)
    mu = X.mean(0)
    sig = X.std(0).clamp_min(1e-12)
    scale = T.std(0).clamp_min(1e-12)
    dn.set_norm(mu.cpu().numpy(), sig.cpu().numpy(), scale.cpu().numpy())
    Xs = ((X - mu) / sig).contiguous()
    Ts = (T / scale).contiguous()
    n = Xs.shape[0]
    gen = torch.Generator(device=Xs.device)
    gen.manual_seed(seed)
    t0 = time.perf_counter()
    losses = []
    for it in range(train_steps):
        idx = torch.randint(0, n, (batch,), device=Xs.device, generator=gen)
        losses.append(dn.train_step(Xs[idx], Ts[idx], lr * (0.1 ** (it / max(1, train_steps)))))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"[denoise] trained {train_steps} steps in {t_train:.1f} s, loss {losses[0]:.4f} -> "
        f"{np.mean(losses[-50:]):.4f}; fallback calibration kappa = {np.round(kappa, 2).tolist()}")

    # ---- held-out source positions: ensemble references, low-count estimates ----
    def err(est, ref, valid, sq):
        # per-statistic RMS over nodes of (est - ref) / s_q
        return np.array([np.sqrt(np.mean(((est[f] - ref[f])[valid] / sq[j]) ** 2)) for j, f in enumerate(QUANT)])

    E_plain_runs = {p: [] for p in (ppe_low, *eval_ppes)}
    T_plain = {p: [] for p in (ppe_low, *eval_ppes)}
    T_plain[ppe_low] = list(t_low)
    variants = {"tau3_noise": (tau, np.ones(8)), "tau3_calibrated": (tau, kappa),
                "no_fallback": (float("inf"), np.ones(8))}
    variants.update({f"tau{t:g}_noise": (t, np.ones(8)) for t in TAU_SWEEP})
    E_var = {k: [] for k in variants}
    rejected = {k: [] for k in variants}
    t_den = []
    for r in range(n_train, n_train + n_test):
        # the ensemble reference: n_ref independent high-count runs
        refs = None
        for k in range(n_ref):
            c_hi, _, s_hi, th = _run(make_workload, ppe_high, 7000 + 50 * r + k, srcs[r], steps_spin, n_snap,
                                     every, F, min_ppe=min_ppe)
            c_hi.close()
            t_high.append(th)
            hs = [b.cpu().numpy() for b in s_hi]
            refs = hs if refs is None else [x + y for x, y in zip(refs, hs)]
        refs = [x / n_ref for x in refs]
        sq = [np.sqrt(np.mean(x[QUANT] ** 2, axis=1)) + 1e-300 for x in refs]
        for ppe in (ppe_low, *eval_ppes):
            c, _, s, tstep = _run(make_workload, ppe, 9000 + 50 * r + ppe, srcs[r], steps_spin, n_snap, every, F,
                                  min_ppe=min_ppe)
            if ppe != ppe_low:
                T_plain[ppe].append(tstep)
            for j, a in enumerate(s):
                A = a.cpu().numpy()
                valid = A[24] > 0
                E_plain_runs[ppe].append(err(A, refs[j], valid, sq[j]))
                if ppe != ppe_low:
                    continue
                # the learned estimate of this snapshot through the C ABI
                ctx_keep.set_nodal_field(_lib.FIELD_STATS, a)
                for name, (tv, kv) in variants.items():
                    dn.set_fallback(kv)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    den, nf = dn.denoise(tv, device=True)
                    t_den.append(time.perf_counter() - t1)
                    D = den.cpu().numpy()
                    E_var[name].append(err(D, refs[j], valid, sq[j]))
                    rejected[name].append(nf / (8.0 * ctx_keep.n_nodes))
            c.close()
        log(f"[denoise] held-out source {r - n_train + 1}/{n_test} done")
    dn.set_fallback(np.ones(8))

    def total(es):  # RMS over the 8 statistics of the per-statistic RMS errors
        return float(np.sqrt(np.mean(np.mean(np.square(es), axis=0))))

    ppes = sorted(E_plain_runs)
    E_plain = {p: total(E_plain_runs[p]) for p in ppes}
    T_mean = {p: float(np.mean(v)) for p, v in T_plain.items()}
    T_mean[ppe_high] = float(np.mean(t_high))
    pt = np.array(sorted(T_mean), float)
    tt = np.array([T_mean[p] for p in sorted(T_mean)])

    def t_at(pe):
        if not np.isfinite(pe):
            return float("inf")
        if pe > pt[-1]:  # beyond the last point: its segment's slope
            return float(tt[-1] + (pe - pt[-1]) * (tt[-1] - tt[-2]) / (pt[-1] - pt[-2]))
        return float(np.interp(pe, pt, tt))

    # the denoiser's cost per call as a step loop pays it: calls queued back to
    # back on the stream, with no host wait or rejection count per call (the
    # time per step of the plain runs is amortized the same way)
    dn.set_fallback(kappa)
    buf = torch.empty((_lib.NSTAT, ctx_keep.n_nodes), dtype=torch.float64, device=ctx_keep.device)
    dn.denoise_into(buf, tau)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(20):
        dn.denoise_into(buf, tau)
    torch.cuda.synchronize()
    t_dn = (time.perf_counter() - t1) / 20
    t_dn_sync = float(np.median(t_den))
    dn.set_fallback(np.ones(8))
    out_var = {}
    for name, es in E_var.items():
        E = total(es)
        pe = ppe_at_error(E, ppes, [E_plain[p] for p in ppes])
        out_var[name] = {"E": E, "ppe_eq": pe, "cost_ratio": t_at(pe) / (T_mean[ppe_low] + t_dn),
                         "rejected_fraction": float(np.mean(rejected[name])),
                         "per_statistic_over_plain": (np.sqrt(np.mean(np.square(es), axis=0)) /
                                                      np.sqrt(np.mean(np.square(E_plain_runs[ppe_low]), axis=0))
                                                      ).tolist()}
    out = {"E_plain": E_plain, "E_plain_per_statistic": {p: np.sqrt(np.mean(np.square(E_plain_runs[p]), axis=0)).tolist()
                                                         for p in ppes},
           "learned": out_var, "T_plain_s": T_mean, "T_denoise_s": t_dn, "T_denoise_sync_s": t_dn_sync,
           "kappa": kappa.tolist(),
           "statistics": NAMES, "train_loss_first": float(losses[0]),
           "train_loss_last": float(np.mean(losses[-50:])), "train_seconds": t_train,
           "n_train_samples": int(n), "hidden": hidden, "n_train_runs": n_train, "n_test_sources": n_test,
           "n_ref_runs": n_ref, "ppe_low": ppe_low, "ppe_high": ppe_high, "eval_ppes": list(eval_ppes),
           "frozen_coefficients": bool(frozen), "min_ppe": min_ppe, "steps_spin": steps_spin,
           "n_snap": n_snap, "every": every, "tau": tau, "coverage": coverage,
           "wall_seconds": time.perf_counter() - t_start}
    params = dn.params()
    norm_arrays = dn.norm
    dn.close()
    ctx_keep.close()
    return out, params, norm_arrays
