#!/usr/bin/env python3
"""Benchmark: weighted-ensemble SSA on one MI355X.

One step = one full WE iteration over every run of the workload: propagate
every walker through tau (Gillespie direct method), recycle walkers that
reached the target, bin, split/merge per bin, accumulate the histogram.

Headline workload: the seeded stand-in for the 354-species / 3680-reaction
model of Sec. III.D -- 50 bins of width 20 on its binned species, 81 walkers
per bin (4050 slots), tau = 0.1, with the 5-species joint histogram -- on the
wave-per-walker kernels.  It starts from x0 and is burnt in (untimed) until
live walkers and events per step have settled; the `burn_in` key says how
many steps that took.  Then K steps are run with HIP events around every
kernel (per-kernel times, the roofline) and K more without them, timed as a
whole: `value` is SSA events/s over that second window.  Inputs are
synthetic; the ensemble is resident in HBM for the whole timed region.

Extra keys: `schlogl_lane`, the same measurement for 2048 Schloegl replicas
(Sec. III.B, recycling X >= 563 -> 82) on the lane-per-walker kernel;
`toggle_mfpt`, GPU-seconds until 16 replicas' MFPT estimates of the toggle
stay within 5% of the brute-force reference, plain species-difference bins
against learned-committor bins.  `cpu_baseline` is the CPU oracle on every
host core (at most 16) on a bounded sample of the headline workload.
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "SSA events/s; GPU-seconds to MFPT rel-err 5%, learned vs plain bins"

# MI355X: 256 CUs, 64 lanes each, 2.4 GHz; one VALU operation per lane per clock
# (FP64 FMA at this rate gives the published 78.6 TFLOP/s).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12
# LDS: 128 bytes per clock per CU
PEAK_LDS = 256 * 128 * 2.4e9


def alg_ops_per_event(net) -> float:
    """Arithmetic of one direct-method event with full propensity recompute,
    counted per operation of the algorithm (each a single lane operation; a
    log or a divide counts as one):
      Philox4x32-10: 10 rounds x (2 32x32->64 products, 4 xor); the key
        schedule does not depend on the counter and is not counted       = 60
      two 53-bit uniforms: 2 x (2 shifts, 1 or, 1 convert, 1 scale)      = 10
      waiting time: 1 - u1, log, divide by a0, t + dt, compare to tau     = 5
      selection target u2*a0, time update                                 = 2
      per reaction: reactant factor (C(x,2): 3, C(x,3): 6, two species: 1)
        + convert + multiply by c + add to a0 + running sum + compare     = 5 + f_j
      state update: one add per changed species + 2 bound checks.
    """
    per_rxn = 0.0
    for j in range(net.R):
        f = 0
        lo, hi = net.reac_ptr[j], net.reac_ptr[j + 1]
        for p in range(lo, hi):
            nu = int(net.reac_mult[p])
            f += {1: 0, 2: 3, 3: 6}[nu]
        if hi - lo == 2:
            f += 1
        per_rxn += 5 + f
    nchg = np.diff(net.chg_ptr).mean()
    return 60 + 10 + 5 + 2 + per_rxn + nchg + 2


def alg_ops_per_event_wave(net) -> float:
    """Arithmetic of one event of the chunked direct method on one wave, per
    the same operation model as alg_ops_per_event:
      random numbers, waiting time, target, time update     = 77
      chunk-sum scan over K = ceil(R/64) chunks             = K adds + ballot (1)
      the chosen chunk: 64 propensity evaluations (5 + f each, the mean f
        over reactions) and a 64-lane scan (63 adds) + ballot (1)
      dependents of the fired reaction (mean list length d): propensity
        before and after (2 x (4 + f)), their difference, and the segmented
        fold into the chunk sums (one add)                  = d x (2 (4 + f) + 2)
      state update: changed species + 2 bound checks."""
    fs = []
    users = [[] for _ in range(net.S)]
    for j in range(net.R):
        lo, hi = net.reac_ptr[j], net.reac_ptr[j + 1]
        f = sum({1: 0, 2: 3, 3: 6}[int(net.reac_mult[p])] for p in range(lo, hi)) + (1 if hi - lo == 2 else 0)
        fs.append(f)
        for p in range(lo, hi):
            users[int(net.reac_species[p])].append(j)
    fbar = float(np.mean(fs))
    deps = []
    for j in range(net.R):
        d = set()
        for p in range(net.chg_ptr[j], net.chg_ptr[j + 1]):
            d.update(users[int(net.chg_species[p])])
        deps.append(len(d))
    dbar = float(np.mean(deps))
    K = (net.R + 63) // 64
    nchg = float(np.diff(net.chg_ptr).mean())
    return 77 + K + 1 + 64 * (5 + fbar) + 63 + 1 + dbar * (2 * (4 + fbar) + 2) + nchg + 2


def _code_only(text: str) -> str:
    """C++ source without comments and blank space, so that the digest tracks
    the code a kernel is compiled from, not its commentary."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_tag: str, digest: str):
    """HBM bytes per launch measured by rocprofv3 counters, if the committed
    measurement was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_digest") != digest:
        return None
    return rec.get("bytes_per_launch")


def _rel_err_curve(flux, tau, burn, ref):
    """Running MFPT of every run (tau / mean recycled weight over iterations
    [burn, t]) and the RMS relative error against ref, for every t > burn."""
    f = np.asarray(flux, np.float64)[:, burn:]
    csum = np.cumsum(f, axis=1)
    n = np.arange(1, f.shape[1] + 1)
    mean = csum / n
    with np.errstate(divide="ignore"):
        mfpt = np.where(mean > 0, tau / mean, np.inf)
    err = np.sqrt(np.mean((mfpt / ref - 1.0) ** 2, axis=0))
    return err


def _time_to(err, times, thr):
    """First time after which the error stays at or below thr."""
    ok = err <= thr
    if not ok[-1]:
        return None
    bad = np.flatnonzero(~ok)
    first = 0 if bad.size == 0 else bad[-1] + 1
    return float(times[first])


def experiment_toggle_mfpt(args):
    """GPU-seconds until 16 replicas' MFPT estimates stay within a relative
    error of the reference, plain Delta bins vs learned committor bins, on
    the synthetic toggle.  The learned time includes its plain-bin record
    phase and the training."""
    import dataclasses

    import torch
    from paper_1303_5986_amd import we, workloads as wl

    chunk = 10
    total = args.exp_iters
    burn = 100
    base = wl.toggle_config(n_runs=16, n_iters=total)
    if args.plain_coord == "total1":
        # a single product coordinate: all protein of gene 1, P1 + 2 D1
        coef = np.array([0, 0, 0, 0, 1, 0, 2, 0], np.float64)
        base = dataclasses.replace(base, bin_coef=coef,
                                   edges=wl.uniform_edges(-0.5, 48.0, base.n_bins))
        base.a_thr = -base.tgt_thr
    if args.toggle_rule:
        base = dataclasses.replace(base, resample_rule=args.toggle_rule)
    tau = base.tau

    # reference: brute force = one bin, 1024 walkers per run x 64 runs, recycling
    ref_iters = args.ref_iters
    bf = dataclasses.replace(base, edges=np.array([-1e9, 1e9]), m_targ=1024,
                             seeds=np.arange(1001, 1065, dtype=np.uint64))
    # each sim on the kernel the autotuner picks for its shape (the same for
    # plain and learned bins)
    kb = we.autotune(bf)
    kern = we.autotune(base)
    simb = we.sim_from_config(bf, kernel=kb[0], walkers_per_wave=kb[1], max_iters=ref_iters)
    simb.graph_capture(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    simb.graph_replay(ref_iters // 20)
    simb.synchronize()
    t_ref = time.perf_counter() - t0
    ref_mfpt, ref_flux, ref_sem = simb.mfpt(200)
    ev_ref = simb.counters()[0]

    def run(learned: bool, edge_mode: int = 0, record_iters: int = 150, train_steps: int = 600,
            extra: int = 0, group: int = 0):
        """edge_mode 0/1: the trainer's edges (equal-count quantiles / equal
        logit widths over the data); 2: equal logit widths from the A state's
        logit to extra / 2 (a half-unit upper logit); 3: equal logit widths
        first, then, after `extra` iterations of measuring every learned bin's
        mean weight, inner edges at equal quantiles of
        y(z) = int sqrt(rho(z) q(z) (1 - q(z))) dz (rho: weight per unit logit,
        piecewise constant over the bins), which equalizes the bins' terms
        w_b * Var_b(q) of the split/merge variance for a discrepancy
        function proportional to q."""
        cfg = base if group == 0 else dataclasses.replace(
            base, seeds=base.seeds + np.uint64(group * base.seeds.size))
        sim = we.sim_from_config(cfg, kernel=kern[0], walkers_per_wave=kern[1], max_iters=total,
                                 record_iters=record_iters if learned else 0)
        times, iters = [], []
        gpu = 0.0
        done = 0
        train_s = 0.0
        if learned:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(record_iters)
            sim.synchronize()
            gpu += time.perf_counter() - t0
            done = record_iters
            times.append(gpu)
            iters.append(done)
            t0 = time.perf_counter()
            loss, n = sim.train_committor(np.array([0, 0, 0, 0, 1, -1, 2, -2.0]), -base.tgt_thr,
                                          steps=train_steps,
                                          batch=1024, lr=2e-3, seed=7, edge_mode=min(edge_mode, 1))
            sim.use_committor_bins(True)
            if edge_mode == 2:
                qa = float(sim.committor(cfg.x_rec[None, :])[0])
                za, zhi = float(np.log(qa / (1.0 - qa))), 0.5 * extra
                e = za + (zhi - za) * np.arange(cfg.n_bins + 1) / cfg.n_bins
                e[0], e[-1] = za - 50.0, zhi + 50.0
                sim.set_learned_bins(e)
            sim.synchronize()
            train_s = time.perf_counter() - t0
            gpu += train_s
            _, _, edges = sim.committor_state()
            if edge_mode == 3:
                nb, wsum, cnt = cfg.n_bins, np.zeros(cfg.n_bins), 0
                for i in range(extra):
                    t0 = time.perf_counter()
                    sim.step(1)
                    sim.synchronize()
                    gpu += time.perf_counter() - t0
                    done += 1
                    for r in range(cfg.seeds.size):
                        _, w, b, _ = sim.walkers(r)
                        wsum += np.bincount(b, weights=w, minlength=nb)[:nb]
                    cnt += cfg.seeds.size
                    if done % chunk == 0:
                        times.append(gpu)
                        iters.append(done)
                edges = _weighted_logit_edges(edges, wsum / cnt)
                sim.set_learned_bins(edges)
                while done % chunk:
                    t0 = time.perf_counter()
                    sim.step(1)
                    sim.synchronize()
                    gpu += time.perf_counter() - t0
                    done += 1
        sim.graph_capture(chunk)
        while done + chunk <= total:
            t0 = time.perf_counter()
            sim.graph_replay(1)
            sim.synchronize()
            gpu += time.perf_counter() - t0
            done += chunk
            times.append(gpu)
            iters.append(done)
        flux = np.stack([sim.flux(r, 0, done) for r in range(cfg.seeds.size)])
        err = _rel_err_curve(flux, tau, burn, ref_mfpt)
        at = np.array(iters) - burn - 1
        keep = at >= 0
        err_at = err[at[keep]]
        tt = np.array(times)[keep]
        res = {"gpu_s_total": gpu, "iterations": done, "train_s": train_s,
               "final_rel_err": float(err_at[-1]),
               "mfpt_mean": float(np.mean(tau / flux[:, burn:].mean(axis=1))),
               "mfpt_runs_rel": [round(float(v), 3) for v in
                                 (tau / flux[:, burn:].mean(axis=1)) / ref_mfpt]}
        if learned:
            res.update(edge_mode=edge_mode, record_iters=record_iters, train_steps=train_steps, extra=extra,
                       train_states=n, loss_first=float(loss[:10].mean()),
                       loss_last=float(loss[-50:].mean()),
                       edges=[round(float(v), 2) for v in edges[1:-1:8]])
            occ = []
            for r in range(2):
                _, _, b, _ = sim.walkers(r)
                occ.append(int(len(set(b.tolist()))))
            res["occupied_bins"] = occ
        for thr in (0.05, 0.1, 0.2):
            res[f"gpu_s_to_{int(thr * 100)}pct"] = _time_to(err_at, tt, thr)
        return res

    plain = run(False)
    variants = []
    specs = [tuple(int(v) for v in spec.split(":")) for spec in args.variants.split(",")]
    specs = [sp + (0,) * (4 - len(sp)) for sp in specs]
    for sp in specs:
        variants.append(run(True, *sp))
    learned = variants[0]
    # further independent groups of 16 replicas (seeds shifted by 16 per
    # group): the time to 5% of one group is itself a noisy statistic
    groups = {"plain": [plain["gpu_s_to_5pct"]], "learned": [learned["gpu_s_to_5pct"]],
              "plain_final": [plain["final_rel_err"]], "learned_final": [learned["final_rel_err"]]}
    per_variant = [{"spec": ":".join(str(v) for v in sp), "to_5pct": [r["gpu_s_to_5pct"]],
                    "final": [r["final_rel_err"]]} for sp, r in zip(specs, variants)]
    for g in range(1, args.toggle_groups):
        pg = run(False, group=g)
        groups["plain"].append(pg["gpu_s_to_5pct"])
        groups["plain_final"].append(pg["final_rel_err"])
        for k, sp in enumerate(specs if args.toggle_groups_all else specs[:1]):
            lg = run(True, *sp, group=g)
            if k == 0:
                groups["learned"].append(lg["gpu_s_to_5pct"])
                groups["learned_final"].append(lg["final_rel_err"])
            per_variant[k]["to_5pct"].append(lg["gpu_s_to_5pct"])
            per_variant[k]["final"].append(lg["final_rel_err"])
    groups["variants"] = per_variant
    return {"metric": "GPU-seconds to MFPT rel-err 5%, learned vs plain bins",
           "workload": "toggle (seed 101), 16 replicas x 64 bins x 16 walkers, tau 0.7",
           "resample_rule": base.resample_rule, "groups": groups,
           "kernel": {"we_iterations": list(kern), "reference": list(kb)},
           "plain_coordinate": args.plain_coord,
           "reference": {"mfpt": ref_mfpt, "sem_rel": ref_sem / ref_flux, "kind":
                         "GPU brute force: 64 runs x 1024 walkers in one bin, recycling",
                         "iterations": ref_iters, "gpu_s": t_ref, "events": ev_ref},
           "burn_in_iterations": burn, "plain": plain, "learned": learned,
           "learned_variants": variants[1:]}


def _weighted_logit_edges(edges, wbar, floor=0.02):
    """Inner logit edges at equal quantiles of y(z) = int sqrt(rho q (1-q)) dz,
    rho the mean weight per unit logit of each inner bin (wbar[b] / width),
    q = 1 / (1 + exp(-z)) at the bin's centre; the first and last inner
    edges stay.  Each inner bin's increment is kept at or above `floor`
    times the mean, so the edges stay strictly increasing."""
    e = np.asarray(edges, np.float64)
    nb = len(e) - 1
    z = e[1:-1]
    dz = np.diff(z)
    zc = 0.5 * (z[:-1] + z[1:])
    q = 1.0 / (1.0 + np.exp(-zc))
    dy = np.sqrt(np.maximum(np.asarray(wbar, np.float64)[1:-1], 0.0) * dz * q * (1.0 - q))
    dy = np.maximum(dy, floor * max(dy.mean(), 1e-300))
    y = np.concatenate([[0.0], np.cumsum(dy)])
    out = e.copy()
    out[1:-1] = np.interp(np.linspace(0.0, y[-1], nb - 1), y, z)
    return out


def schlogl_mfpt_exact(a: int = 82, b: int = 563, top: int = 1500) -> float:
    """Mean first passage time a -> b of the Schloegl birth-death chain
    (combinatorial mass action, constants of Sec. III.B): with the chain's
    stationary law pi, T = sum_{k=a}^{b-1} P(X <= k) / (lambda_k pi_k)."""
    from paper_1303_5986_amd import workloads as wl
    p = wl.SCHLOGL_K
    x = np.arange(top + 1, dtype=np.float64)
    lam = p["k1"] * p["A"] * x * (x - 1) / 2.0 + p["k3"] * p["B"]
    mu = p["k2"] * x * (x - 1) * (x - 2) / 6.0 + p["k4"] * x
    logpi = np.zeros(top + 1)
    for k in range(1, top + 1):
        logpi[k] = logpi[k - 1] + np.log(lam[k - 1]) - np.log(mu[k])
    pi = np.exp(logpi - logpi.max())
    pi /= pi.sum()
    cum = np.cumsum(pi)
    return float(sum(cum[k] / (lam[k] * pi[k]) for k in range(a, b)))


def _half_window_err(flux, tau, ref):
    """RMS relative error over runs of the MFPT estimate tau / mean(flux) with
    the mean over iterations [t // 2, t], for every t."""
    f = np.asarray(flux, np.float64)
    csum = np.concatenate([np.zeros((f.shape[0], 1)), np.cumsum(f, axis=1)], axis=1)
    t = np.arange(1, f.shape[1] + 1)
    lo = t // 2
    mean = (csum[:, t] - csum[:, lo]) / (t - lo)
    with np.errstate(divide="ignore"):
        mfpt = np.where(mean > 0, tau / mean, np.inf)
    return np.sqrt(np.mean((mfpt / ref - 1.0) ** 2, axis=0))


def _pooled_err(flux, tau, ref):
    """Relative error of the MFPT estimate from all runs together: tau / the
    mean recycled weight over runs and iterations [t // 2, t], for every t."""
    f = np.asarray(flux, np.float64).mean(axis=0, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.abs(_half_window_err(f, tau, ref))


def experiment_schlogl_rw(args):
    """The Schloegl flux experiment of Sec. III.B at its published size (80
    bins of width 10, 32 walkers per bin, tau = 0.1, recycling X >= 563 ->
    X = 82), with steady-state reweighting every 100, 5 or 2 iterations or
    none: GPU-seconds (and iterations) until the replicas' MFPT estimates stay
    within a relative error of the exact MFPT."""
    import dataclasses

    import torch
    from paper_1303_5986_amd import we, workloads as wl

    total, chunk = args.exp_iters, 10
    runs = args.rw_runs
    base = dataclasses.replace(wl.schlogl_config(n_runs=runs, seed0=301, n_iters=total),
                               edges=wl.uniform_edges(0.0, 800.0, 80), m_targ=32, tau=0.1)
    exact = schlogl_mfpt_exact()
    out = {"metric": "GPU-seconds to MFPT rel-err 5%, steady-state reweighting periods",
           "workload": f"Schloegl, 80 bins x 32 walkers, tau 0.1, {runs} replicas, X>=563 -> X=82",
           "exact_mfpt": exact, "estimator": "tau / mean recycled weight over iterations [t/2, t], "
           "RMS relative error over replicas", "variants": []}
    for period, reset in ((0, False), (100, False), (5, False), (2, False), (100, True), (5, True),
                          (2, True)):
        sim = we.sim_from_config(base, kernel=we.WE_KERNEL_LANE, max_iters=total, rw_period=period,
                                 rw_reset=reset)
        sim.graph_capture(chunk)
        torch.cuda.synchronize()
        gpu, done, times = 0.0, 0, []
        while done + chunk <= total:
            t0 = time.perf_counter()
            sim.graph_replay(1)
            sim.synchronize()
            gpu += time.perf_counter() - t0
            done += chunk
            times.append(gpu)
        flux = np.stack([sim.flux(r, 0, done) for r in range(runs)])
        at = np.arange(chunk, done + 1, chunk) - 1
        res = {"rw_period": period, "rw_reset": reset, "iterations": done, "gpu_s_total": gpu,
               "events": sim.counters()[0]}
        if period:
            ap = [sim.rw_counts(r) for r in range(runs)]
            res["events_applied"] = int(sum(a for a, _ in ap))
            res["events_skipped"] = int(sum(b for _, b in ap))
        for name, err in (("pooled", _pooled_err(flux, base.tau, exact)),
                          ("per_replica_rms", _half_window_err(flux, base.tau, exact))):
            r = {"final_rel_err": float(err[-1]),
                 "rel_err_at": {str(i + 1): round(float(err[i]), 4)
                                for i in (29, 49, 99, 199, 499, done - 1) if i < done}}
            for thr in (0.05, 0.1, 0.2):
                r[f"gpu_s_to_{int(thr * 100)}pct"] = _time_to(err[at], np.array(times), thr)
                ok = err <= thr
                r[f"iters_to_{int(thr * 100)}pct"] = (None if not ok[-1] else
                                                     int(np.flatnonzero(~ok)[-1] + 2 if (~ok).any() else 1))
            res[name] = r
        out["variants"].append(res)
        print(json.dumps({"rw_period": period, "rw_reset": reset,
                          "pooled_iters_to_5pct": res["pooled"]["iters_to_5pct"],
                          "pooled_gpu_s_to_5pct": res["pooled"]["gpu_s_to_5pct"]}),
              file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def experiment_switch_mfpt(args):
    """The epigenetic switch of Sec. III.C at the paper's WE settings (15 x 31
    bins, 16 walkers per bin, tau = 0.1, 500 iterations, reweighting every
    100, first 100 iterations discarded): the combined MFPT of the replicas
    against the exact value, the paper's six-run estimate, and E_50% (the MFPT
    over the brute-force-equivalent dynamics, segments x tau, propagated
    until a replica's running estimate first comes within 50%)."""
    import torch
    from paper_1303_5986_amd import we, workloads as wl
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import closed_form as cf

    runs, total, chunk = args.switch_runs, 500, 50
    cfg = wl.switch_config(n_runs=runs, n_iters=total)
    exact = cf.switch_mfpt()
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=total, rw_period=100)
    sim.graph_capture(chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.graph_replay(total // chunk)
    sim.synchronize()
    gpu = time.perf_counter() - t0
    flux = np.stack([sim.flux(r, 0, total) for r in range(runs)])
    per_run = flux[:, 100:].mean(axis=1) / cfg.tau
    mfpt = 1.0 / per_run.mean()
    sem_rel = per_run.std(ddof=1) / np.sqrt(runs) / per_run.mean()
    six = per_run[:6]
    e50 = []
    for r in range(runs):
        run_mean = np.cumsum(flux[r]) / np.arange(1, total + 1) / cfg.tau
        with np.errstate(divide="ignore"):
            est = np.where(run_mean > 0, 1.0 / run_mean, np.inf)
        ok = np.flatnonzero(np.abs(est / exact - 1.0) <= 0.5)
        e50.append(int(ok[0]) + 1 if ok.size else None)
    ev, seg_total, _ = sim.counters()
    out = {"metric": "MFPT of the epigenetic switch, WE with reweighting every 100 iterations",
           "workload": f"switch (Sec. III.C), 15x31 bins x 16 walkers, tau 0.1, {runs} replicas x {total} iterations",
           "exact_mfpt": exact, "mfpt": mfpt, "rel_err": mfpt / exact - 1.0, "sem_rel": sem_rel,
           "replica_rel_sd": float(per_run.std(ddof=1) / per_run.mean()),
           "first_six": {"mfpt": float(1.0 / six.mean()),
                         "sem": float(six.std(ddof=1) / np.sqrt(6) / six.mean() / six.mean())},
           "iterations_to_50pct": e50[:6], "median_iterations_to_50pct": float(np.median([v for v in e50 if v])),
           "segments_per_replica": seg_total / runs,
           "e50_approx": exact / (float(np.median([v for v in e50 if v])) * seg_total / runs / total * cfg.tau),
           "events": ev, "gpu_s": gpu,
           "ms_per_iteration": gpu * 1e3 / total}
    print(json.dumps(out), flush=True)


def experiment_tauleap(args):
    """The tau-leaping engine (Sec. IV proposes combining WE with it) against
    the exact direct method on two workloads: the default Schloegl benchmark
    (2048 replicas; leaps only pay in the upper well) and a high-copy
    birth-death chain (k = 1e4, gamma = 1, stationary law Poisson(1e4), 40
    bins of width 10 around the mean, 16 walkers per bin, tau = 0.1, 256
    replicas).  Time per WE iteration, reactions fired per second, and the
    accuracy of the weighted ensemble's mean and variance (birth-death) or of
    the flux (Schloegl)."""
    import dataclasses

    import torch
    from paper_1303_5986_amd import we, workloads as wl

    W, K = args.warmup, args.steps
    out = {"metric": "tau-leaping vs exact SSA, WE iteration time and accuracy", "leap_eps": 0.03,
           "workloads": {}}
    bd_net = wl.birth_death(k=1e4, gamma=1.0)
    bd = wl.WEConfig(name="birth_death_1e4", net=bd_net, x0=np.array([10000], np.int32),
                     bin_coef=np.array([1.0]), edges=wl.uniform_edges(9800.0, 10200.0, 40), m_targ=16,
                     tau=0.1, n_iters=W + K, seeds=np.arange(1, 257, dtype=np.uint64))
    sch = wl.schlogl_config(n_runs=args.runs, seed0=1, n_iters=W + K)
    for name, base in (("birth_death_1e4", bd), ("schlogl", sch)):
        res = {}
        for engine in ("ssa", "tauleap"):
            cfg = dataclasses.replace(base, engine=engine, leap_eps=0.03)
            sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=W + K)
            sim.step(W)
            sim.synchronize()
            ev0 = sim.counters()[0]
            sim.graph_capture(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.graph_replay(K // 2)
            sim.synchronize()
            dt = time.perf_counter() - t0
            ev = sim.counters()[0] - ev0
            r = {"ms_per_iteration": dt * 1e3 / K, "reactions_per_s": ev / dt, "reactions_per_iteration": ev / K}
            if name == "birth_death_1e4":
                m1 = m2 = 0.0
                for run in range(len(cfg.seeds)):
                    x, w, _, _ = sim.walkers(run)
                    m1 += float(np.dot(w, x[:, 0]))
                    m2 += float(np.dot(w, x[:, 0].astype(np.float64) ** 2))
                m1 /= len(cfg.seeds)
                m2 /= len(cfg.seeds)
                r.update(mean=m1, var=m2 - m1 * m1, mean_exact=1e4, var_exact=1e4)
            else:
                flux = np.stack([sim.flux(run, W, K) for run in range(len(cfg.seeds))])
                r["mean_flux_per_s"] = float(flux.mean() / cfg.tau)
            res[engine] = r
        res["speedup"] = res["ssa"]["ms_per_iteration"] / res["tauleap"]["ms_per_iteration"]
        out["workloads"][name] = res
        print(json.dumps({name: {"speedup": res["speedup"]}}), file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def experiment_batch(args):
    """64 independent WE runs on seeded networks of 8..3680 reactions and
    256..8192 walker slots: one batch (persistent propagation launches,
    autotuned lane/wave choice, HIP graph) against the same runs stepped as
    plain sequential launches, one run after another."""
    import torch
    from paper_1303_5986_amd import we, workloads as wl

    W, K = args.warmup, args.steps
    cfgs = wl.batch_configs(n_runs=args.batch_runs, n_iters=W + 2 * K)
    cache = os.path.join(ROOT, "profiles", "batch_autotune.json") if args.tune_cache else None
    t0 = time.perf_counter()
    b = we.Batch(cfgs, max_iters=W + 2 * K, autotune_iters=args.autotune_iters, cache_path=cache)
    tune_s = time.perf_counter() - t0
    b.step(W)
    b.synchronize()
    ev0 = sum(m.counters()[0] for m in b.members)
    b.graph_capture(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.graph_replay(K // 2)
    b.synchronize()
    tb = time.perf_counter() - t0
    evb = sum(m.counters()[0] for m in b.members) - ev0
    kernels = b.kernels().tolist()
    wpw = b.walkers_per_wave().tolist()

    # the same runs as independent sims, each launched on its own, in turn
    sims = [we.sim_from_config(c, kernel=int(k), walkers_per_wave=int(w) if int(k) == we.WE_KERNEL_GROUP else 0,
                               max_iters=W + 2 * K) for c, k, w in zip(cfgs, kernels, wpw)]
    for s in sims:
        s.step(W)
    for s in sims:
        s.synchronize()
    ev0 = sum(s.counters()[0] for s in sims)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        for s in sims:
            s.step(1)
    for s in sims:
        s.synchronize()
    ts = time.perf_counter() - t0
    evs = sum(s.counters()[0] for s in sims) - ev0
    out = {"metric": "SSA events/s, batched vs sequential launches", "runs": len(cfgs),
           "reactions": [cfgs[0].net.R, cfgs[-1].net.R],
           "walker_slots_total": int(sum(c.cap for c in cfgs)), "steps": K, "warmup": W,
           "batched": {"events_per_s": evb / tb, "we_iters_per_s": K / tb, "ms_per_step": tb * 1e3 / K},
           "sequential": {"events_per_s": evs / ts, "we_iters_per_s": K / ts, "ms_per_step": ts * 1e3 / K},
           "speedup": ts / tb, "events_equal": bool(evb == evs),
           "kernels": {"lane": kernels.count(1), "group": kernels.count(3), "wave": kernels.count(2)},
           "walkers_per_wave": wpw,
           "autotune_s": tune_s}
    print(json.dumps(out), flush=True)


def _rare_batch_configs(cfgs, we, wl, log):
    """Pilot runs of the uneven batch (one batch each, grid bins, no
    recycling): 40 intervals at tau 0.01 measure each run's events per
    walker, then 100 intervals at the calibrated tau relax the ensemble; its
    events re-calibrate tau and its weights give the recycling target
    (workloads.rare_target, tail 1e-4)."""
    import dataclasses
    b = we.Batch(cfgs, max_iters=40)
    b.step(20)
    b.synchronize()
    e0 = [m.counters() for m in b.members]
    b.step(20)
    b.synchronize()
    e1 = [m.counters() for m in b.members]
    b.close()
    taus = [wl.batch_tau((z1[0] - z0[0]) / max(1, z1[1] - z0[1])) for z0, z1 in zip(e0, e1)]
    relaxed = [dataclasses.replace(c, tau=t) for c, t in zip(cfgs, taus)]
    b = we.Batch(relaxed, max_iters=100)
    b.step(80)
    b.synchronize()
    e0 = [m.counters() for m in b.members]
    b.step(20)
    b.synchronize()
    out = []
    for c, m, t, z0 in zip(cfgs, b.members, taus, e0):
        z1 = m.counters()
        t2 = wl.batch_tau((z1[0] - z0[0]) / max(1, z1[1] - z0[1]), tau0=t)
        x, w, _, _ = m.walkers(0)
        sp, xa, thr = wl.rare_target(x, w)
        out.append(wl.rare_batch_config(c, t2, sp, xa, thr))
    b.close()
    log(f"rare batch: {len(out)} runs, tau {min(c.tau for c in out):.3g}..{max(c.tau for c in out):.3g}")
    return out


def _mfpt_curves(flux, taus, burn, ref, at):
    """Per-run MFPT estimates tau_k / (mean recycled weight over [burn, t))
    at every t in `at`, relative to ref_k: array [len(at), runs]."""
    out = []
    for t in at:
        m = np.array([f[burn:t].mean() for f in flux])
        with np.errstate(divide="ignore"):
            out.append(np.where(m > 0, np.asarray(taus) / m, np.inf) / ref)
    return np.array(out)


def experiment_rare_batch(args):
    """The batched rare-event workload: 64 runs of the uneven batch, each
    with a recycling target at its pilot's 1e-4 tail.  Compared: one batch
    (persistent launches, one HIP graph per chunk) binning every run on its
    own learned committor after a 150-interval plain-bin record phase, the
    same batch on plain bins, and the runs as sequential per-run launches on
    plain bins; each at the GPU-seconds after which the RMS over runs of the
    MFPT relative error stays within 5%.  Reference MFPT per run: a plain-bin
    batch with other seeds, 10x as many intervals.  Runs whose reference is
    not resolved (batch-means relative s.e. above 2%, first and second
    halves more than 5% apart, or the reference run's own estimate over the
    measured window more than 10% from its long-run value) are reported and
    left out of the RMS."""
    import torch
    from paper_1303_5986_amd import we, workloads as wl

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    T, chunk, burn, rec = args.exp_iters, 50, 200, 150
    base = wl.batch_configs(n_runs=args.batch_runs, n_iters=T)
    rcfg = _rare_batch_configs(base, we, wl, log)
    taus = [c.tau for c in rcfg]
    n = len(rcfg)

    # reference: plain bins, other seeds, 10x the intervals
    import dataclasses
    ref_iters = 10 * T
    refc = [dataclasses.replace(c, seeds=c.seeds + np.uint64(7919)) for c in rcfg]
    b = we.Batch(refc, max_iters=ref_iters)
    b.graph_capture(chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(ref_iters // chunk):
        b.graph_replay(1)
        if (i + 1) % 40 == 0:
            b.synchronize()
            log(f"reference {(i + 1) * chunk}/{ref_iters} intervals, {time.perf_counter() - t0:.1f} s")
    b.synchronize()
    t_ref = time.perf_counter() - t0
    rb = ref_iters // 10
    ref, resolved, ref_sem = np.zeros(n), np.zeros(n, bool), np.zeros(n)
    ref_window = np.zeros(n)
    for k, m in enumerate(b.members):
        full = m.flux(0)
        f = full[rb:]
        mean = f.mean()
        blocks = f[: len(f) // 20 * 20].reshape(20, -1).mean(axis=1)
        h1, h2 = f[: len(f) // 2].mean(), f[len(f) // 2:].mean()
        ref[k] = taus[k] / mean if mean > 0 else np.inf
        ref_sem[k] = blocks.std(ddof=1) / np.sqrt(20) / mean if mean > 0 else np.inf
        # the reference run itself over the measured window [burn, T): a run
        # that has not relaxed within the budget on its own is out of reach
        # of every method compared here
        wm = full[burn:T].mean()
        ref_window[k] = (taus[k] / wm) / ref[k] if (wm > 0 and mean > 0) else np.inf
        resolved[k] = (mean > 0 and ref_sem[k] <= 0.02 and h1 > 0 and abs(h2 / h1 - 1) <= 0.05
                       and abs(ref_window[k] - 1) <= 0.10)
    b.close()
    log(f"reference: {resolved.sum()} of {n} runs resolved, {t_ref:.1f} s")
    at = np.arange(burn + chunk, T + 1, chunk)

    def rms(curves):
        c = curves[:, resolved]
        return np.sqrt(np.mean((c - 1.0) ** 2, axis=1))

    # kernel choice per run: the autotuner's (lane, group with 32..2 walkers
    # per wave, or wave), timed once on pilot sims; every method below runs
    # each run on the same kernel
    t0 = time.perf_counter()
    tb = we.Batch(rcfg, max_iters=2, autotune_iters=args.autotune_iters)
    tune_s = time.perf_counter() - t0
    choice = [(int(k), int(w)) for k, w in zip(tb.kernels(), tb.walkers_per_wave())]
    tb.close()
    kernels = [(k, w if k == we.WE_KERNEL_GROUP else 0) for k, w in choice]
    log(f"autotune {tune_s:.1f} s: walkers per wave {[w for _, w in choice]}")

    def batch_run(learned: bool):
        b = we.Batch(rcfg, max_iters=T, record_iters=rec if learned else 0, kernels=kernels)
        gpu, times, done = 0.0, [], 0
        trained = 0
        if learned:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.step(rec)
            b.synchronize()
            for c, m in zip(rcfg, b.members):
                try:
                    m.train_committor(c.bin_coef, c.a_thr, steps=args.rare_train_steps, batch=512, lr=2e-3,
                                      seed=7, edge_mode=1)
                except we.WEError:
                    continue          # no resolved outcome yet: this run keeps plain bins
                m.use_committor_bins(True)
                trained += 1
            torch.cuda.synchronize()
            gpu += time.perf_counter() - t0
            done = rec
        b.graph_capture(chunk)
        while done + chunk <= T:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.graph_replay(1)
            b.synchronize()
            gpu += time.perf_counter() - t0
            done += chunk
            times.append((done, gpu))
            if done % (20 * chunk) == 0:
                log(f"{'learned' if learned else 'plain'} batch {done}/{T} intervals, {gpu:.1f} GPU-s")
        flux = [m.flux(0) for m in b.members]
        seg = float(sum(m.counters()[1] for m in b.members)) / T
        b.close()
        return flux, dict(times), trained, seg

    def sequential_run():
        sims = [we.sim_from_config(c, kernel=k, walkers_per_wave=w, max_iters=T) for c, (k, w) in zip(rcfg, kernels)]
        for s in sims:
            s.graph_capture(chunk)
        gpu, times, done = 0.0, [], 0
        while done + chunk <= T:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in sims:
                s.graph_replay(1)
            for s in sims:
                s.synchronize()
            gpu += time.perf_counter() - t0
            done += chunk
            times.append((done, gpu))
            if done % (20 * chunk) == 0:
                log(f"sequential {done}/{T} intervals, {gpu:.1f} GPU-s")
        flux = [s.flux(0) for s in sims]
        seg = float(sum(s.counters()[1] for s in sims)) / T
        return flux, dict(times), seg

    res = {}
    for name in ("learned_batched", "plain_batched", "plain_sequential"):
        if name == "plain_sequential":
            flux, tmap, seg = sequential_run()
            trained = 0
        else:
            flux, tmap, trained, seg = batch_run(name == "learned_batched")
        curves = _mfpt_curves(flux, taus, burn, ref, at)
        err = rms(curves)
        tt = np.array([tmap[int(t)] for t in at])
        res[name] = {"gpu_s_to_5pct": _time_to(err, tt, 0.05), "gpu_s_to_10pct": _time_to(err, tt, 0.10),
                     "final_rel_err": float(err[-1]), "gpu_s_total": float(tt[-1]),
                     "ms_per_interval": float((tt[-1] - tt[0]) / (at[-1] - at[0]) * 1e3),
                     "walkers_per_interval": seg,
                     "final_run_errors": [round(float(v), 3) for v in curves[-1] - 1.0]}
        if name == "learned_batched":
            res[name]["runs_on_learned_bins"] = trained
        log(f"{name}: final RMS rel-err {err[-1]:.3f}, to 5% {res[name]['gpu_s_to_5pct']}, "
            f"total {tt[-1]:.2f} GPU-s")
    out = {"metric": "GPU-seconds to MFPT rel-err 5% (RMS over resolved runs)",
           "workload": f"{n} runs of the uneven batch, 8-3680 reactions, 256-8192 walker slots, "
                       f"16 bins, recycling at the pilot's 1e-4 tail",
           "intervals": T, "burn_in_intervals": burn, "record_intervals": rec,
           "autotune_s": tune_s, "walkers_per_wave": [w for _, w in choice],
           "train_steps": args.rare_train_steps,
           "reference": {"intervals": ref_iters, "gpu_s": t_ref, "resolved_runs": int(resolved.sum()),
                         "resolved": [bool(v) for v in resolved],
                         "mfpt": [float(v) for v in ref], "rel_sem": [float(v) for v in ref_sem],
                         "window_over_long_run": [float(v) for v in ref_window]},
           "runs": [{"reactions": c.net.R, "species": c.net.S, "walker_slots": c.cap, "tau": c.tau,
                     "x_a": int(c.x0[np.flatnonzero(c.bin_coef)[0]]), "threshold": int(c.tgt_thr)}
                    for c in rcfg],
           **res}
    print(json.dumps(out), flush=True)


def experiment_paper_tails(args):
    """The paper's two rare-state sweeps at its own settings, timed: the
    Schloegl transient (Sec. III.B: 802 unit bins on X, 100 walkers per bin,
    tau 0.05, 100 intervals from X = 82, P(X >= 700, t = 5)) and the futile
    cycle (Sec. III.A: 101 unit bins on S1, 100 walkers per bin, tau 1, 100
    intervals from S1 = S2 = 50, P(S1 > 90, t = 100), weight-equalizing
    split/merge), each as `replicas` independent runs in one launch per
    interval.  Reports GPU seconds, segments and events per second, and the
    replicas' mean and standard error of the tail beside the values the
    paper prints (its CME and WE numbers; its own WE runs took "2-3 seconds"
    per futile-cycle run on a CPU, context only)."""
    import torch
    from paper_1303_5986_amd import we, workloads as wl
    paper = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))
    R = args.tail_replicas
    cases = [
        ("schlogl_t5", wl.WEConfig(name="schlogl_t5", net=wl.schlogl(), x0=np.array([82], np.int32),
                                   bin_coef=np.array([1.0]), edges=np.arange(0.0, 803.0), m_targ=100, tau=0.05,
                                   n_iters=100, seeds=np.arange(501, 501 + R, dtype=np.uint64)),
         0, 700, paper["schlogl_tail_t5"]["value"], paper["schlogl_tail_t5_we"]),
        ("futile_t100", wl.WEConfig(name="futile_t100", net=wl.futile_cycle(),
                                    x0=np.array([50, 50, 1, 1, 0, 0], np.int32),
                                    bin_coef=np.array([1.0, 0, 0, 0, 0, 0]), edges=np.arange(0.0, 102.0),
                                    m_targ=100, tau=1.0, n_iters=100,
                                    seeds=np.arange(601, 601 + R, dtype=np.uint64), resample_rule=1),
         0, 91, paper["futile_tail_t100"]["value"], paper.get("futile_tail_t100_we")),
    ]
    out = {"metric": "GPU seconds per paper-scale rare-state sweep", "replicas": R, "cases": {}}
    for name, cfg, sp, lo, exact, pw in cases:
        sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(100)
        sim.synchronize()
        el = time.perf_counter() - t0
        ev, seg, _ = sim.counters()
        est = []
        for r in range(R):
            x, w, _, _ = sim.walkers(r)
            est.append(float(w[x[:, sp] >= lo].sum()))
        est = np.array(est)
        out["cases"][name] = {
            "gpu_s": el, "gpu_s_per_replica": el / R, "segments": int(seg), "events": int(ev),
            "segments_per_s": seg / el, "events_per_s": ev / el,
            "tail_mean": float(est.mean()), "tail_sem": float(est.std(ddof=1) / np.sqrt(R)),
            "tail_median": float(np.median(est)), "paper_exact": exact,
            "paper_we": None if pw is None else {"value": pw["value"], "err": pw.get("err")}}
        print(f"{name}: {el:.2f} GPU-s for {R} replicas, {seg} segments, tail {est.mean():.3e} +- "
              f"{est.std(ddof=1) / np.sqrt(R):.1e} (paper exact {exact:.3e})", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def experiment_walkers_per_wave(args):
    """Events/s of every propagation kernel a network fits, across network
    sizes: the lane kernel (64 walkers per wave, up to 64 reactions), the
    group kernel with 32, 16, 8, 4 and 2 walkers per wave, and the wave
    kernel (one).  Seeded random networks of R reactions (S = max(8,
    R * 354 / 3680) species, counts log-uniform on [0, 20]), 32 runs x 16 bins
    x 16 walkers, tau chosen for about ten events per walker; 20 untimed
    intervals, then 40 timed with HIP events around the propagation launch
    (the kernel's own time, the work the autotuner's choice is about)."""
    import dataclasses
    import torch
    from paper_1303_5986_amd import we, workloads as wl
    rows = []
    for R in (16, 40, 100, 300, 1000, 3000):
        S = max(8, int(round(R * 354 / 3680)))
        net = wl.random_network(4000 + R, S, R)
        x0 = wl.log_uniform_counts(np.random.default_rng(4001 + R), S, hi=20)
        sp = int(np.argmax(x0))
        coef = np.zeros(S)
        coef[sp] = 1.0
        cfg = wl.WEConfig(name=f"wpw{R}", net=net, x0=x0, bin_coef=coef, edges=wl.uniform_edges(0.0, 32.0, 16),
                          m_targ=16, tau=0.01, n_iters=80, seeds=np.arange(1, 33, dtype=np.uint64))
        # calibrate tau to about ten events per walker on the wave kernel
        sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_WAVE, max_iters=20)
        sim.step(10)
        sim.synchronize()
        ev, sg, _ = sim.counters()
        cfg = dataclasses.replace(cfg, tau=wl.batch_tau(ev / max(sg, 1)))
        cands = []
        if S <= 32 and R <= 64:
            cands.append(("lane", we.WE_KERNEL_LANE, 0))
        for wpw in (32, 16, 8, 4, 2):
            if (wpw * S) <= 4096:
                cands.append((f"group{wpw}", we.WE_KERNEL_GROUP, wpw))
        cands.append(("wave", we.WE_KERNEL_WAVE, 0))
        row = {"reactions": R, "species": S, "tau": cfg.tau}
        for name, k, wpw in cands:
            sim = we.sim_from_config(cfg, kernel=k, walkers_per_wave=wpw, max_iters=80)
            sim.step(20)
            sim.synchronize()
            e0, _, _ = sim.counters()
            sim.profile(True)
            sim.step(40)
            sim.synchronize()
            ms_ssa, _, _, _ = sim.profile_read()
            e1, _, _ = sim.counters()
            row[name] = {"events_per_s": (e1 - e0) / (ms_ssa * 1e-3), "ms_per_launch": ms_ssa / 40,
                         "kernel": sim.propagation_kernel()}
        best = max((n for n, _, _ in cands), key=lambda n: row[n]["events_per_s"])
        row["fastest"] = best
        rows.append(row)
        print(f"R={R}: " + ", ".join(f"{n} {row[n]['events_per_s']:.2e}" for n, _, _ in cands) + f" -> {best}",
              file=sys.stderr, flush=True)
    print(json.dumps({"metric": "propagation events/s by walkers per wave", "runs": 32, "bins": 16,
                      "walkers_per_bin": 16, "rows": rows}), flush=True)


def _burn_in(sim, warmup: int, chunk: int = 25, min_iters: int = 100, cap: int = 1000) -> int:
    """Untimed steps until the workload is in its steady window: at least
    max(warmup, min_iters) steps, then until two successive chunks of `chunk`
    steps agree on live walkers per step within 2% and on events per step
    within 5% (or `cap` steps).  Returns the steps taken."""
    done, prev = 0, None
    while True:
        ev0, seg0, _ = sim.counters()
        sim.step(chunk)
        sim.synchronize()
        ev1, seg1, _ = sim.counters()
        done += chunk
        cur = ((seg1 - seg0) / chunk, (ev1 - ev0) / chunk)
        if prev is not None and done >= max(warmup, min_iters):
            if abs(cur[0] - prev[0]) <= 0.02 * prev[0] and abs(cur[1] - prev[1]) <= 0.05 * max(prev[1], 1.0):
                return done
        if done >= cap:
            return done
        prev = cur


def _measure(sim, K: int, W: int):
    """Steady-window measurement of one sim: burn in, then K steps with HIP
    events around every kernel (per-kernel times), then K more steps with no
    events recorded, timed as a whole (the headline rate)."""
    import torch
    burn = _burn_in(sim, W)
    ev0, seg0, _ = sim.counters()
    sim.profile(True)
    sim.step(K)
    sim.synchronize()
    ms_ssa, ms_res, ms_obs, _ = sim.profile_read()
    sim.profile(False)
    ev1, seg1, _ = sim.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(K)
    sim.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev2, seg2, _ = sim.counters()
    return {"burn_in": burn, "events_profiled": ev1 - ev0, "segments_profiled": seg1 - seg0,
            "ms_ssa": ms_ssa / K, "ms_res": ms_res / K, "ms_obs": ms_obs / K,
            "events": ev2 - ev1, "segments": seg2 - seg1, "elapsed": t1 - t0}


def lds_bytes_per_event_fact(net) -> float:
    """LDS bytes one event of the factored-table wave kernel moves, as built:
      the chosen chunk: 64 x (16 B descriptor + 8 B header + 2 x 4 B counts);
      the changed species: old count and incidence word (8 B), the store (4 B);
      each dependent (mean list length d, repeats included): 2 B id, 16 B
        descriptor, 2 x 4 B counts before and 2 x 4 B after the firing;
      the chunk sums: one LDS atomic add per dependent (8 B read, 8 B
        written), then the 64 chunk lanes reload their sums (512 B)."""
    users = [0] * net.S
    for j in range(net.R):
        for p in range(net.reac_ptr[j], net.reac_ptr[j + 1]):
            users[int(net.reac_species[p])] += 1
    dl = [sum(users[int(net.chg_species[p])] for p in range(net.chg_ptr[j], net.chg_ptr[j + 1]))
          for j in range(net.R)]
    d = float(np.mean(dl))
    nchg = float(np.diff(net.chg_ptr).mean())
    return 64 * (16 + 8 + 8) + nchg * 12 + d * (2 + 16 + 8 + 8) + d * 16 + 512


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_worker(job):
    """A bounded sample of the workload on the oracle, timed inside the
    worker: for the large network, `n` direct-method intervals of length tau
    from its initial state; for Schloegl, one WE run of `n` iterations."""
    kind, seed, tau, n = job
    from oracle import oracle as orc
    from paper_1303_5986_amd import workloads as wl
    t0 = time.perf_counter()
    ev = 0
    if kind == "large":
        cfg = wl.large_network_config()
        onet = orc.OracleNet(cfg.net)
        for k in range(n):
            _, e = orc.ssa_interval(onet, cfg.x0, tau, seed, k, 0)
            ev += e
    else:
        cfg = wl.schlogl_config(n_runs=1, seed0=seed, n_iters=n)
        o = orc.OracleWE(cfg, seed)
        o.step(n)
        ev = sum(o.events)
    return ev, time.perf_counter() - t0


def cpu_baseline_all_cores(kind: str, tau: float, n: int):
    """The oracle on every host core the process may use (at most 16, the
    box's share per GPU), one worker per core with its own seed; the value is
    all workers' events over the wall time."""
    import multiprocessing as mp
    cores = min(16, len(os.sched_getaffinity(0)))
    jobs = [(kind, 1000 + i, tau, n) for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_cpu_worker, jobs)
    wall = time.perf_counter() - t0
    ev = sum(e for e, _ in res)
    per_core = float(np.mean([e / t for e, t in res]))
    what = (f"{n} direct-method interval(s) of tau={tau:g} from the workload's initial state"
            if kind == "large" else f"one WE run of {n} iterations from the workload's initial ensemble")
    return {"value": ev / wall, "unit": "events/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(), "single_core_value": per_core,
            "sample": f"{cores} workers x {what}, each with its own seed ({ev} events, {wall:.1f} s wall)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=150)
    ap.add_argument("--runs", type=int, default=2048, help="Schloegl replicas in the lane-kernel line")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: skip the Schloegl lane-kernel line and the toggle experiment")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times "
                         "(reference kernel for scaling the HBM byte counters)")
    ap.add_argument("--experiment", default="",
                    choices=["", "toggle_mfpt", "batch", "schlogl_rw", "switch_mfpt", "tauleap", "rare_batch",
                             "paper_tails", "walkers_per_wave"])
    ap.add_argument("--switch-runs", type=int, default=64, help="replicas in the switch experiment")
    ap.add_argument("--rw-runs", type=int, default=32,
                    help="replicas in the reweighting experiment")
    ap.add_argument("--large-runs", type=int, default=1,
                    help="independent replicas of the large network (the configuration is 1; "
                         "more fill the chip and show the wave kernels' throughput ceiling)")
    ap.add_argument("--workload", default="large", choices=["schlogl", "large"],
                    help="headline workload. large (default): the 354-species / 3680-reaction "
                         "network, 50 bins x 81 walkers, tau 0.1, with its 5-species joint "
                         "histogram, wave kernel; schlogl: 2048 Schloegl replicas, lane kernel")
    ap.add_argument("--batch-runs", type=int, default=64)
    ap.add_argument("--tail-replicas", type=int, default=10,
                    help="independent runs per case in the paper-scale tail sweeps")
    ap.add_argument("--rare-train-steps", type=int, default=300,
                    help="Adam steps per run's committor in the rare batch experiment")
    ap.add_argument("--autotune-iters", type=int, default=3)
    ap.add_argument("--tune-cache", action="store_true")
    ap.add_argument("--exp-iters", type=int, default=4000)
    ap.add_argument("--ref-iters", type=int, default=4000)
    ap.add_argument("--plain-coord", default="delta", choices=["delta", "total1"],
                    help="hand-chosen bin coordinate: Delta = (P1+2D1)-(P2+2D2), or P1+2D1")
    ap.add_argument("--toggle-rule", type=int, default=0, choices=[0, 1],
                    help="split/merge rule of the toggle experiment (both binnings)")
    ap.add_argument("--toggle-groups", type=int, default=4,
                    help="independent 16-replica groups of the toggle experiment")
    ap.add_argument("--variants", default="1:400:1500",
                    help="learned-bin runs as edge_mode:record_iters:train_steps[:extra], comma "
                         "separated; the first is the reported one (edge modes 2 and 3 and their "
                         "extra parameter: see experiment_toggle_mfpt)")
    ap.add_argument("--toggle-groups-all", action="store_true",
                    help="run every learned variant in every group (default: the first only)")
    args = ap.parse_args()
    if args.experiment == "toggle_mfpt":
        print(json.dumps(experiment_toggle_mfpt(args)), flush=True)
        return
    if args.experiment == "batch":
        experiment_batch(args)
        return
    if args.experiment == "rare_batch":
        experiment_rare_batch(args)
        return
    if args.experiment == "paper_tails":
        experiment_paper_tails(args)
        return
    if args.experiment == "walkers_per_wave":
        experiment_walkers_per_wave(args)
        return
    if args.experiment == "schlogl_rw":
        experiment_schlogl_rw(args)
        return
    if args.experiment == "switch_mfpt":
        experiment_switch_mfpt(args)
        return
    if args.experiment == "tauleap":
        experiment_tauleap(args)
        return
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); "
              "the weighted-ensemble runs shard by run with no communication, "
              "so N GPUs would each run this same line on their own replicas.", file=sys.stderr)
        sys.exit(2)

    from paper_1303_5986_amd import we, workloads as wl

    K, W = args.steps, args.warmup
    max_iters = 1000 + 2 * K + 50

    def line_large():
        cfg = wl.large_network_config(n_iters=max_iters)
        if args.large_runs > 1:
            cfg = cfg.with_seeds(np.arange(2024, 2024 + args.large_runs, dtype=np.uint64))
        sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_WAVE, max_iters=max_iters, joint=True)
        m = _measure(sim, K, W)
        ops_ev = alg_ops_per_event_wave(cfg.net)
        lds_ev = lds_bytes_per_event_fact(cfg.net)
        kname = sim.propagation_kernel()
        ev_launch = m["events_profiled"] / K
        ssa_s = m["ms_ssa"] / 1e3
        achieved = ops_ev * ev_launch / ssa_s
        traffic = traffic_from_profiles(
            "ssa_wave_large", source_digest(["paper_1303_5986_amd/csrc/ssa_wave.hip",
                                             "paper_1303_5986_amd/csrc/ssa_wave_body.h",
                                             "paper_1303_5986_amd/csrc/ssa_wave_fact.h",
                                             "paper_1303_5986_amd/csrc/queue_first.h",
                                             "paper_1303_5986_amd/csrc/we_common.h"]))
        if args.large_runs != 1:
            traffic = None   # the committed counters were taken on the one-run configuration
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "Tops/s",
                "frac": achieved / PEAK_LANE_OPS, "traffic": traffic, "ops_per_event": ops_ev,
                "kernel": kname, "avg_launch_ms": m["ms_ssa"], "events_per_launch": ev_launch}
        if kname == "ssa_wave_fact_kernel":
            lds = lds_ev * ev_launch / ssa_s
            roof["lds"] = {"achieved": lds / 1e12, "peak": PEAK_LDS / 1e12, "unit": "TB/s",
                           "frac": lds / PEAK_LDS, "bytes_per_event": lds_ev}
        desc = {"workload": "large_network_354x3680", "runs": args.large_runs, "species": cfg.net.S,
                "reactions": cfg.net.R, "bins": cfg.n_bins, "walkers_per_bin": cfg.m_targ, "tau": cfg.tau,
                "joint_histogram_species": len(cfg.joint_species), "kernel": "ssa_wave",
                "walkers_per_step": m["segments"] / K}
        return m, roof, desc

    def line_schlogl(runs):
        cfg = wl.schlogl_config(n_runs=runs, seed0=1, n_iters=max_iters)
        sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=max_iters)
        m = _measure(sim, K, W)
        ops_ev = alg_ops_per_event(cfg.net)
        ev_launch = m["events_profiled"] / K
        ssa_s = m["ms_ssa"] / 1e3
        achieved = ops_ev * ev_launch / ssa_s
        traffic = traffic_from_profiles(
            "ssa_lane_schlogl", source_digest(["paper_1303_5986_amd/csrc/ssa_lane.hip",
                                               "paper_1303_5986_amd/csrc/ssa_lane_body.h",
                                               "paper_1303_5986_amd/csrc/we_common.h"]))
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "Tops/s",
                "frac": achieved / PEAK_LANE_OPS, "traffic": traffic, "ops_per_event": ops_ev,
                "kernel": sim.propagation_kernel(), "avg_launch_ms": m["ms_ssa"], "events_per_launch": ev_launch}
        desc = {"workload": "schlogl_steady_state_recycling", "runs": runs, "bins": cfg.n_bins,
                "walkers_per_bin": cfg.m_targ, "tau": cfg.tau, "target": "X>=563 -> X=82",
                "kernel": "ssa_lane", "walkers_per_step": m["segments"] / K}
        return m, roof, desc

    if args.workload == "large":
        m, roof, desc = line_large()
    else:
        m, roof, desc = line_schlogl(args.runs)
    out = {
        "metric": METRIC,
        "value": m["events"] / m["elapsed"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "burn_in": m["burn_in"],
        "ms_per_step": m["elapsed"] * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": desc,
        "we_iters_per_s": K / m["elapsed"],
        "events_per_segment": m["events"] / max(m["segments"], 1),
        "kernel_ms_per_step": {"ssa": m["ms_ssa"], "resample": m["ms_res"], "observe": m["ms_obs"]},
        "roofline": roof,
    }
    # the ceilings measured on this device, beside the published ones
    pk = we.measure_peaks()
    out["measured_peaks"] = pk

    def add_measured(r):
        r["peak_measured"] = pk["int32_tops"]
        r["frac_measured"] = r["achieved"] / pk["int32_tops"]
        if "lds" in r:
            r["lds"]["peak_measured"] = pk["lds_tbs"]
            r["lds"]["frac_measured"] = r["lds"]["achieved"] / pk["lds_tbs"]

    add_measured(roof)
    if not args.no_cpu:
        if args.workload == "large":
            out["cpu_baseline"] = cpu_baseline_all_cores("large", 0.1, 6)
        else:
            out["cpu_baseline"] = cpu_baseline_all_cores("schlogl", 0.05, 2000)
    if not args.no_extras:
        if args.workload == "large":
            ms, rs, ds = line_schlogl(args.runs)
            add_measured(rs)
            out["schlogl_lane"] = {"config": ds, "events_per_s": ms["events"] / ms["elapsed"],
                                   "ms_per_step": ms["elapsed"] * 1e3 / K, "burn_in": ms["burn_in"],
                                   "roofline": rs}
        tg = experiment_toggle_mfpt(args)
        out["toggle_mfpt"] = {
            "metric": "GPU-seconds to MFPT rel-err 5% (16 replicas, RMS over replicas)",
            "workload": tg["workload"], "reference_mfpt": tg["reference"]["mfpt"],
            "learned_variant": args.variants.split(",")[0],
            "plain_delta_bins_gpu_s": tg["plain"]["gpu_s_to_5pct"],
            "learned_bins_gpu_s": tg["learned"]["gpu_s_to_5pct"],
            "plain_final_rel_err": tg["plain"]["final_rel_err"],
            "learned_final_rel_err": tg["learned"]["final_rel_err"],
            "groups_of_16": tg["groups"], "kernel": tg["kernel"],
            "learned_includes": "plain-bin record phase and training"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
