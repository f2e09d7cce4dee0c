#!/usr/bin/env python3
"""Throughput of the HIP graded-bed DEM stepper on one MI355X.

Workload: 2,000,000 spheres, radius r(d) = 1.5 mm (1 + d / 20 mm) capped at
8 r0 (the paper's linear grading with gamma = 0.15), +-10 % jitter, 0.2 m
deep, periodic square side from the count model (2.12 m), floor wall, paper
material set (2200 kg/m^3, 1 GPa, 0.15, mu_t 0.3, mu_r 0.02), dt = 2e-6 s.
Seeded synthetic bed (raft deposition), then `--warmup` untimed steps, then
exactly `--steps` timed steps.  One JSON line on stdout.

A step is the whole pipeline: broad phase (cell binning, scans, owner-side
search, reverse lists) on rebuild steps, then the fused narrow phase +
contact law + accumulation + walls + integration kernel and the FP64 body
reduction.  `--rebuild-every 1` (default) rebuilds the broad phase every
step; `--rebuild-every k --skin s` uses candidate lists with a skin rebuilt
every k steps (the contact set found each step is the same).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s at 2M-sphere graded bed; batched & adjoint vs plain, same GPU"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle-step: x (24) + r (4) + v (12) + omega (12)
# read, x + v + omega (48) written, and per contact pair the history
# (xi_t, xi_r: 24 B) and partner id (4 B) read and written (56 B)
B_PARTICLE = 100.0
B_PAIR = 56.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def counter_record(n_particles):
    """The committed rocprofv3 counter record of the metric bed (HBM bytes per
    launch of every kernel, every-step search and skin lists), when it was
    taken on the current kernel code and the same bed size; else None."""
    from paper_2501_05300_amd.profile_summary import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "step_kernel_counters_metric_bed.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        c = json.load(f)
    if c.get("kernel_source_hash") != kernel_source_hash() or c.get("n") != n_particles:
        return None
    return c


def kernel_traffic(rec, mode, kernel):
    """FETCH_SIZE + WRITE_SIZE bytes per launch of one kernel from the record."""
    if rec is None or kernel not in rec.get(mode, {}):
        return None
    k = rec[mode][kernel]
    return k["fetch_bytes"] + k["write_bytes"]


# the kernel that does most of each timed phase (the phase's own name when it
# is one kernel)
PHASE_KERNEL = {"binning": "k_bin", "resort": "k_rs_scatter", "cell_lists": "k_scatter", "search": "k_search",
                "reverse_lists": "k_rev_scatter", "contact_step": "k_step<{block}>", "body_reduction": "k_advance"}


def host_cpu():
    """Host CPU as the GPU machine reports it: nproc, os.cpu_count(), lscpu model."""
    import subprocess
    out = {"nproc": None, "cpu_count": os.cpu_count(), "model": None}
    try:
        out["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
    except Exception:  # noqa: BLE001
        pass
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                out["model"] = line.split(":", 1)[1].strip()
            if line.startswith("CPU(s):"):
                out["lscpu_cpus"] = int(line.split(":", 1)[1].strip())
    except Exception:  # noqa: BLE001
        pass
    return out


def settle_beds(specs, steps, chunk=5000, max_steps=None, rel_change=0.01):
    """Relaxes deposited beds in place (positions only), all in one batch,
    with the paper's relaxation friction (mu_t 0.1, mu_r 0.01, frictionless
    walls), extra normal damping (gamma_n = 10 dt) and dt = 5e-6 s;
    velocities are then zeroed.  Untimed preparation of the input.

    Runs at least `steps` steps, then (when max_steps is given) goes on in
    chunks until the contacts per particle change by less than rel_change
    over a chunk of `chunk` steps, or max_steps is reached.  Returns
    (steps run, contacts per particle at the end, whether the criterion was
    met).

    The damping term is explicit: its rate c/m must stay below 2/dt.  For a
    1.35 mm sphere under a 24 mm one (overlap ~3e-5 m) gamma_n = 10 dt gives
    dt c/m ~ 0.6; 50 dt would exceed 2 and eject the fine spheres."""
    import numpy as np
    from paper_2501_05300_amd import beds
    from paper_2501_05300_amd.lprdem import Batch
    work = []
    for spec in specs:
        s = spec.copy()
        s.params = beds.settle_params(spec.params).replace(dt=5e-6, gamma_factor=10.0)
        for w in s.walls:
            w.mu_t, w.mu_r = 0.0, 0.0
        work.append(s)
    rmin = min(float(s.radius.min()) for s in specs)
    sb = Batch(work, rebuild_every=5, skin=0.25 * rmin)
    done = 0
    t0 = time.perf_counter()
    ntot = sum(s.n for s in specs)
    cbar = prev = None
    settled = False
    limit = max(steps, max_steps or 0)
    while done < limit:
        k = min(chunk, limit - done)
        sb.step(k)
        sb.sync()
        done += k
        st = sb.stats()
        prev, cbar = cbar, st["contacts"] / ntot
        log(f"settle {done}/{steps}: contacts/particle {cbar:.3f}, "
            f"skin trips {st['skin_trips']} ({time.perf_counter() - t0:.1f} s)")
        if done >= steps:
            if max_steps is None:
                break
            if prev is not None and cbar > 0 and abs(cbar - prev) < rel_change * cbar:
                settled = True
                break
    for q, spec in enumerate(specs):
        pos, _, _ = sb.state(bed=q)
        spec.pos = pos
        spec.vel = np.zeros_like(spec.vel)
        spec.omega = np.zeros_like(spec.omega)
    sb.close()
    return done, cbar, settled


def batch_leg(steps, warmup, settle, tune_steps):
    """The 36-bed family in one batch vs the same beds stepped one at a time
    with the plain stepper, plus the autotuned batch."""
    import torch
    from paper_2501_05300_amd import beds
    from paper_2501_05300_amd.lprdem import Batch, Bed, autotune
    specs = beds.batch_family(plate=False)
    N = sum(s.n for s in specs)
    log(f"batch family: {len(specs)} beds, {N} spheres")
    if settle > 0:
        settle_beds(specs, settle)
    specs = [beds.add_plate(s, diameter=0.1, speed=0.01) for s in specs]

    def timed(stepper):
        stepper.step(warmup)
        stepper.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stepper.step(steps)
        stepper.sync()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    b = Batch(specs)
    wall_b = timed(b)
    st = b.stats()
    b.close()
    log(f"batched: {steps} steps in {wall_b:.3f} s")
    best, trials = autotune(specs, trial_steps=tune_steps)
    log(f"autotuner: {best}")
    tb = Batch(specs, band_ratio=best["band_ratio"], cell_factor=best["cell_factor"], block=best["block"],
               persistent=best["persistent"], level_cell_factor=best["level_cell_factor"])
    wall_t = timed(tb)
    tb.close()
    log(f"batched, tuned: {steps} steps in {wall_t:.3f} s")
    wall_s = 0.0
    for s in specs:
        one = Bed(s)
        wall_s += timed(one)
        one.close()
    log(f"one bed at a time: {steps} steps each in {wall_s:.3f} s total")
    return {"beds": len(specs), "spheres": N, "steps": steps,
            "batched_particle_steps_per_s": N * steps / wall_b,
            "batched_tuned_particle_steps_per_s": N * steps / wall_t,
            "sequential_plain_particle_steps_per_s": N * steps / wall_s,
            "speedup_batched_vs_plain": wall_s / wall_b, "speedup_tuned_vs_plain": wall_s / wall_t,
            "contacts_per_particle": st["contacts"] / N, "tuning": best, "tuning_trials": trials,
            "graph": "steady cycle replayed as one captured HIP graph"}


def adjoint_leg(n, window, ckpt, settle, pre, seed=0):
    """Adjoint form on the 50k-sphere graded bed (r0 1.5 mm, L 20 mm, k 1,
    0.2 m deep) under a 0.1 m plate pushed at 0.01 m/s (`pre` steps first, so
    that the plate is loaded: 50,000 steps sink it 1 mm): one reverse-mode
    window of `window` steps with a checkpoint every `ckpt` steps, timed
    against the same steps run forward only from the same state."""
    import torch
    from paper_2501_05300_amd import beds
    from paper_2501_05300_amd.lprdem import Bed
    spec = beds.graded_bed(n, r0=1.5e-3, L=0.02, k=1.0, depth=0.2, seed=seed + 50)
    log(f"adjoint bed: {spec.n} spheres, side {spec.box[0]:.3f} m")
    if settle > 0:
        settle_beds([spec], settle)
    spec = beds.add_plate(spec, diameter=0.1, speed=0.01)
    body = spec.info["plate_body"]
    skin = 0.25 * float(spec.radius.min())
    bed = Bed(spec, rebuild_every=10, skin=skin)
    done = 0
    while done < pre:
        k = min(10_000, pre - done)
        bed.step(k)
        bed.sync()
        done += k
    log(f"adjoint bed: plate pushed {pre} steps")
    x, v, w = bed.state()
    keys, vals = bed.history()
    clock = bed.clock()

    def rewind(b):
        b.set_state(x, v, w)
        b.set_history(keys, vals)
        b.set_clock(clock)
        b.sync()

    def forward(b):
        rewind(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(window)
        b.sync()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    plain = Bed(spec)
    forward(plain)  # warm the captured graph
    t_plain = forward(plain)
    plain.close()
    forward(bed)
    t_skin = forward(bed)
    rewind(bed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, g = bed.adjoint_window(window, ckpt, body)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    st = bed.stats()
    bed.close()
    log(f"adjoint window {window} steps, checkpoints every {st['adjoint_interval']}: {t_adj:.3f} s; "
        f"forward {t_plain:.3f} s (every-step lists), {t_skin:.3f} s (skin lists); J {J:.4g} N, grad {g}")
    return {"spheres": spec.n, "window_steps": window, "checkpoint_every": int(st["adjoint_interval"]),
            "J_mean_plate_reaction_N": J, "grad_s_k_mu_t_mu_r": [float(q) for q in g],
            "adjoint_s": t_adj, "forward_every_step_s": t_plain, "forward_skin_s": t_skin,
            "adjoint_particle_steps_per_s": spec.n * window / t_adj,
            "adjoint_over_forward_every_step": t_adj / t_plain, "adjoint_over_forward_skin": t_adj / t_skin}


def calibration_leg(n, window, ckpt, settle, seed=0):
    """Bulk calibration with the adjoint on the adjoint leg's 50k graded bed:
    two plate experiments (a 0.1 m plate pushed at 0.01 and 0.005 m/s until
    it has sunk 1 mm, then a window of `window` steps each) whose targets
    are the GPU's own mean plate reactions at theta* = (1.25, 0.36, 0.02);
    (s_k, mu_t) are fitted from the bed's own (1.0, 0.3) by damped
    Gauss-Newton, every evaluation one adjoint window per experiment."""
    import numpy as np
    import torch
    from paper_2501_05300_amd import beds
    from paper_2501_05300_amd.calibrate import Experiment, calibrate
    from paper_2501_05300_amd.lprdem import Bed
    base = beds.graded_bed(n, r0=1.5e-3, L=0.02, k=1.0, depth=0.2, seed=seed + 50)
    if settle > 0:
        settle_beds([base], settle)
    skin = 0.25 * float(base.radius.min())
    exps = []
    for speed, pre in ((0.01, 50_000), (0.005, 100_000)):
        spec = beds.add_plate(base.copy(), diameter=0.1, speed=speed)
        bed = Bed(spec, rebuild_every=10, skin=skin)
        done = 0
        while done < pre:
            k = min(10_000, pre - done)
            bed.step(k)
            bed.sync()
            done += k
        exps.append(Experiment.from_bed(spec, bed, spec.info["plate_body"], window, ckpt,
                                        rebuild_every=10, skin=skin))
        bed.close()
    log(f"calibration: two plate experiments pushed to 1 mm, windows of {window} steps")
    theta_star = np.array([1.25, 0.36, 0.02])
    theta0 = np.array([exps[0].spec.params.s_k, exps[0].spec.params.mu_t, exps[0].spec.params.mu_r])
    targets = [e.response(theta_star)[0] for e in exps]
    calls = [0]
    responses = [e.response for e in exps]
    for e, f in zip(exps, responses):
        def counted(th, f=f):
            calls[0] += 1
            return f(th)
        e.response = counted
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, hist = calibrate(exps, targets, theta0, (True, True, False), iters=8)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    for e in exps:
        e.close()
    evals = calls[0] // len(exps)
    log(f"calibration: theta {theta} after {len(hist) - 1} iterates, {evals} evaluations, {t_fit:.2f} s; "
        f"residuals {[h['residual'] for h in hist]}")
    return {"spheres": base.n, "window_steps": window, "experiments": len(exps),
            "targets_N": [float(t) for t in targets], "theta_start": theta0.tolist(), "theta_true": theta_star.tolist(),
            "theta_fit": theta.tolist(), "max_rel_error": float(np.max(np.abs(theta - theta_star) / theta_star)),
            "residuals": [h["residual"] for h in hist], "evaluations": evals, "fit_s": t_fit,
            "s_per_evaluation": t_fit / max(evals, 1)}


def implicit_leg(spec, steps, warmup, n_iter):
    """The paper's time-implicit step (SPOOK with projected block-Jacobi
    sweeps) on the settled bed `spec` at the paper's dt = 0.1 ms with n_iter
    sweeps per step (its refined beds use 215-275, table
    tab:bed-configurations-refinement): particle-steps/s, simulated time per
    wall time against the explicit step's, and the sweep kernels' rate
    against HBM bandwidth."""
    import torch
    from paper_2501_05300_amd.lprdem import Bed
    s = spec.copy()
    s.params = s.params.replace(dt=1e-4)
    bed = Bed(s)
    bed.set_stepper("spook", n_iter)
    bed.step(warmup)
    bed.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prof = bed.step_profiled(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = bed.stats()
    bed.close()
    N = s.n
    c_bar = st["contacts"] / N
    solve_ms = prof["step"] / steps
    sweep_ms = solve_ms / (n_iter + 1)      # n_iter sweeps plus rows, first velocities and finish
    from paper_2501_05300_amd import profile_summary as PS
    b_sweep = PS.SWEEP_PARTICLE + PS.SWEEP_CONTACT * c_bar   # bytes per particle a sweep must move
    traffic = None
    rec_path = os.path.join(PS.PROFILES, "implicit_sweep_counters_metric_bed.json")
    if os.path.exists(rec_path):
        with open(rec_path) as f:
            rec = json.load(f)
        if rec.get("spook_source_hash") == PS.spook_source_hash() and rec.get("n") == N:
            traffic = rec["sweep_hbm_bytes"]
    log(f"implicit: {steps} steps x {n_iter} sweeps in {wall:.3f} s ({1e3 * wall / steps:.2f} ms/step); "
        f"contacts/particle {c_bar:.3f}; {prof}")
    return {"dt_s": 1e-4, "sweeps_per_step": n_iter, "steps": steps, "n": N,
            "ms_per_step": 1e3 * wall / steps, "particle_steps_per_s": N * steps / wall,
            "simulated_s_per_wall_s": 1e-4 * steps / wall,
            "contact_sweeps_per_s": st["contacts"] * n_iter * steps / (prof["step"] / 1e3),
            "kernel_ms_per_step": {k: v / steps for k, v in prof.items()},
            # bytes the sweep kernels are designed to move (their own per-contact
            # rows, owner sums and partner parts included), not a method minimum
            "sweep_traffic": {"bound": "hbm", "kernels": ["k_sp_contacts", "k_sp_vel"], "unit": "GB/s",
                              "design_GBs": N * b_sweep / (sweep_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                              "design_frac": N * b_sweep / (sweep_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                              "design_bytes_per_particle_sweep": b_sweep, "counter_bytes_per_sweep": traffic,
                              "counter_frac": (traffic / (sweep_ms / 1e3) / 1e9 / HBM_PEAK_GBS) if traffic else None}}


def emission_leg(seed=0):
    """Layer-by-layer emission of a refined bed shaped like the paper's
    (d_min 8.5 mm to d_max 30 mm in 6 layers, gamma 0.05, 0.6 m deep, 0.3 m
    periodic side): wall time, relaxation steps, and the diagnostics the paper
    reports (bulk density and its local variation, mixing between layers)."""
    from paper_2501_05300_amd import emission as E
    d_min, d_max, L, gamma = 8.5e-3, 30e-3, 6, 0.05
    r = (d_max / d_min) ** (1.0 / L)
    eta = (r - 1.0) / (r * gamma)
    bed = E.emit_bed(d_min, r, eta, L, 0.6, 0.3, seed=seed, log=log)
    dg = E.diagnostics(bed, rho=2200.0)
    log(f"emission: {dg['n']} spheres in {bed.seconds:.1f} s, {bed.steps} steps; density {dg['density_mean']:.0f} "
        f"kg/m^3 (rel std {dg['density_rel_std']:.3f}); mixing {[round(m, 4) for m in dg['mixing']]}")
    return {"d_min": d_min, "d_max": d_max, "ratio": r, "eta": eta, "gamma": E.gamma_of(r, eta), "layers": L,
            "height_m": 0.6, "side_m": 0.3, "emitted": bed.emitted, "kept": dg["n"], "steps": bed.steps,
            "seconds": bed.seconds, "diagnostics": dg}


def terramech_leg(seed=0, t_static=0.05, pull_speed=0.5, pull_distance=0.1):
    """The plate test at one third of the paper's scale: a 0.1 x 0.06 m plate
    with four 14.3 mm grousers under 5 kPa (below this plate's bearing
    capacity on this sand; the paper's 50 kPa is for a plate three times as
    large) on 0.2 m deep beds (0.3 x 0.15 m
    periodic), phase I for t_static, then a pull of pull_distance at
    pull_speed; a uniform 3 mm reference, a bed refined from 3 to 10 mm
    (gamma 0.05) and a uniform 10 mm control, with the paper's normalised
    errors against the reference."""
    from paper_2501_05300_amd import terramech as T
    plate = T.Plate()
    cases = (("uniform_3mm_reference", 3e-3, 3e-3, 0.0), ("refined_3_10mm_gamma_0.05", 3e-3, 10e-3, 0.05),
             ("uniform_10mm_control", 10e-3, 10e-3, 0.0))
    out = {}
    for name, dmin, dmax, gamma in cases:
        t0 = time.perf_counter()
        spec = T.linear_bed(dmin, dmax, gamma, 0.2, 0.3, 0.15, seed=seed)
        t1 = time.perf_counter()
        res = T.run_protocol(spec, plate, t_static, pull_speed, pull_distance, log=log)
        t2 = time.perf_counter()
        out[name] = {"n": spec.n, "prepare_s": t1 - t0, "protocol_s": t2 - t1, "steps": res["steps"],
                     "particle_steps_per_s": spec.n * res["steps"] / (t2 - t1),
                     **{k: res[k] for k in ("static_sinkage", "dynamic_sinkage", "peak_traction", "average_traction")}}
        log(f"{name}: {spec.n} spheres, protocol {t2 - t1:.1f} s")
    ref = out["uniform_3mm_reference"]
    for name in list(out):
        out[name]["errors"] = T.normalized_errors(out[name], ref, plate.h_grouser, plate.load, plate.load)
        out[name]["count_reduction"] = ref["n"] / out[name]["n"]
    return out


def configs_leg(steps_c2, steps_c3, warmup, settle):
    """Further workloads on the plain stepper (every-step search):
    a 200k graded bed under a 0.1 m plate pushed at 0.01 m/s, and the
    grousered ring (5 kPa dead weight, 0.5 rad/s) on a 2.0M uniform bed and
    on a 150k graded bed (k = 2, L = 0.105 m) in the same 0.4 m box, whose
    particle-count and per-step cost ratios are the refinement's saving."""
    import numpy as np
    import torch
    from paper_2501_05300_amd import beds
    from paper_2501_05300_amd.lprdem import Bed
    c2 = beds.graded_bed(200_000, seed=0)
    c3c = beds.uniform_bed(2_000_000, r=1.5e-3, depth=0.2805, side=0.4, seed=0)
    c3g = beds.graded_bed(150_000, r0=1.5e-3, L=0.105, k=2.0, cap=8.0, depth=0.2805, side=0.4, seed=0)
    settle_beds([c2, c3c, c3g], settle)
    beds.add_plate(c2, diameter=0.1, speed=0.01)
    beds.add_ring(c3c)
    beds.add_ring(c3g)
    out = {}
    for name, spec, steps in (("plate_200k_graded", c2, steps_c2), ("ring_2M_uniform_control", c3c, steps_c3),
                              ("ring_150k_graded", c3g, steps_c3)):
        body = spec.info["plate_body"]
        bed = Bed(spec)
        bed.step(warmup)
        bed.sync()
        z0 = float(bed.body(body)[0][2])
        bed.reaction_window(body, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prof = bed.step_profiled(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = bed.stats()
        sum6, nsum = bed.reaction_window(body)
        out[name] = {"n": spec.n, "steps": steps, "ms_per_step": 1e3 * wall / steps,
                     "particle_steps_per_s": spec.n * steps / wall,
                     "contacts_per_s": st["contacts"] * steps / wall,
                     "contacts_per_particle": st["contacts"] / spec.n,
                     "kernel_ms_per_step": {k: v / steps for k, v in prof.items()},
                     "mean_body_reaction_z_N": float(sum6[2]) / max(nsum, 1),
                     "body_sinkage_m": z0 - float(bed.body(body)[0][2])}
        log(f"{name}: {out[name]['ms_per_step']:.3f} ms/step, {out[name]['particle_steps_per_s']:.3e} particle-steps/s")
        bed.close()
    c, g = out["ring_2M_uniform_control"], out["ring_150k_graded"]
    out["ring_count_ratio_control_over_graded"] = c["n"] / g["n"]
    out["ring_step_cost_ratio_control_over_graded"] = c["ms_per_step"] / g["ms_per_step"]
    return out


def sort_leg(spec, steps, warmup, block):
    """What the storage-order sort buys: the metric bed stored in its
    (shuffled) input order, once kept frozen and once re-sorted on the
    device at the default cadence (every 16th rebuild), then `steps` steps of
    each with per-phase HIP events.  Same contacts and results; only where
    the particles sit in memory differs."""
    import torch
    from paper_2501_05300_amd.lprdem import Bed
    out = {}
    for name, every in (("input_order_frozen", -1), ("input_order_resorted", 0)):
        bed = Bed(spec, block=block, sort_every=every, input_order=True)
        bed.step(max(warmup, 64))
        bed.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bed.step(steps)
        bed.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = bed.step_phases(steps)
        st = bed.stats()
        bed.close()
        out[name] = {"ms_per_step": 1e3 * wall / steps, "sorts": st["sorts"],
                     "kernel_ms_per_step": {k: v / steps for k, v in prof.items()}}
        log(f"storage order {name}: {1e3 * wall / steps:.3f} ms/step; phases {out[name]['kernel_ms_per_step']}")
    f, r = out["input_order_frozen"], out["input_order_resorted"]
    out["speedup_resorted_over_frozen"] = f["ms_per_step"] / r["ms_per_step"]
    out["steps"] = steps
    return out


def cpu_configs_leg(settled_2k=None):
    """The FP64 oracle on the smaller workloads, single-threaded and on every
    allowed host thread, on bounded samples: the two-layer bed (2,000
    spheres, 500 steps from placement), the 200k graded bed (20 steps) and
    the adjoint's 2,000-sphere graded copy (a 200-step window of forward-mode
    derivatives under a full-width plate).  Particle-steps/s each."""
    from oracle import oracle as O
    from paper_2501_05300_amd import beds
    env = os.environ.get("OMP_NUM_THREADS")
    allt = int(env) if env and env.isdigit() and int(env) > 0 else (os.cpu_count() or 1)
    out = {"host": host_cpu()}
    c1 = beds.two_layer_bed(0)
    c2 = beds.graded_bed(200_000, seed=0)
    c5 = settled_2k if settled_2k is not None else beds.graded_bed(2000, side=0.0671, seed=7)
    c5 = beds.add_plate(c5.copy(), speed=0.01, full_width=True)
    for threads in (1, allt):
        used = O.set_threads(threads)
        row = {}
        for name, spec, steps in (("two_layer_2k_500_steps", c1, 500), ("graded_200k_20_steps", c2, 20)):
            ob = O.OracleBed(spec)
            t0 = time.perf_counter()
            ob.step(steps)
            dt = time.perf_counter() - t0
            row[name] = {"particle_steps_per_s": spec.n * steps / dt, "seconds": dt}
        ob = O.OracleBed(c5)
        t0 = time.perf_counter()
        ob.tangent_window(200, c5.info["plate_body"], 2)
        dt = time.perf_counter() - t0
        row["adjoint_2k_window_200"] = {"particle_steps_per_s": c5.n * 200 / dt, "seconds": dt}
        out[f"threads_{used}"] = row
        log(f"cpu configs, {used} thread(s): {row}")
    return out


def cpu_baseline(spec, pos, vel, omg, keys, vals, clock, steps):
    """The FP64 oracle, as it stands, on the same bed state (bounded sample:
    `steps` steps of the full bed), on every host thread this job may use:
    OMP_NUM_THREADS when the environment sets it (the GPU machine allots its CPU
    share that way), else every CPU the process sees."""
    from oracle import oracle as O
    env = os.environ.get("OMP_NUM_THREADS")
    threads = int(env) if env and env.isdigit() and int(env) > 0 else (os.cpu_count() or 1)
    used = O.set_threads(threads)
    ob = O.OracleBed(spec)
    ob.set_state(pos, vel, omg)
    ob.set_history(keys, vals)
    ob.set_clock(clock)
    t0 = time.perf_counter()
    ob.step(steps)
    dt = time.perf_counter() - t0
    return {"value": spec.n * steps / dt, "unit": "particle-steps/s", "cores": used, "kind": "oracle",
            "sample": f"{steps} FP64 oracle step(s) of the full {spec.n}-sphere bed from the GPU state after "
                      f"warm-up, {dt:.1f} s, {used} OpenMP threads",
            "host": host_cpu()}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--rebuild-every", type=int, default=1)
    ap.add_argument("--skin", type=float, default=0.0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=3,
                    help="oracle steps of the full bed for the CPU baseline, about 17 s on 16 cores (0: skip)")
    ap.add_argument("--secondary-every", type=int, default=50,
                    help="also time candidate lists with a skin rebuilt every k steps (0: skip)")
    ap.add_argument("--secondary-skin", type=float, default=0.05,
                    help="skin of the secondary run, as a fraction of the smallest radius")
    ap.add_argument("--batch-steps", type=int, default=300, help="timed steps of the 36-bed leg (0: skip)")
    ap.add_argument("--batch-settle", type=int, default=40000)
    ap.add_argument("--adjoint-window", type=int, default=2000, help="steps of the adjoint leg (0: skip)")
    ap.add_argument("--implicit-steps", type=int, default=10,
                    help="timed steps of the time-implicit leg on the same bed (0: skip)")
    ap.add_argument("--implicit-sweeps", type=int, default=250)
    ap.add_argument("--calibrate-window", type=int, default=2000,
                    help="steps per experiment of the calibration leg (0: skip)")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="also time the oracle on the two-layer, 200k graded and 2k adjoint workloads (minutes)")
    ap.add_argument("--emission", action="store_true",
                    help="also build a refined bed layer by layer and report its diagnostics")
    ap.add_argument("--terramech", action="store_true",
                    help="also run the plate test on reference, refined and control beds")
    ap.add_argument("--configs", action="store_true",
                    help="also time the plate (200k graded) and grousered-ring (2.0M uniform vs 150k graded) beds")
    ap.add_argument("--settle", type=int, default=40000,
                    help="least relaxation steps before the measurement (paper's reduced friction, damped, dt 5e-6)")
    ap.add_argument("--settle-max", type=int, default=200000,
                    help="relaxation goes on until contacts per particle settle, at most this many steps")
    ap.add_argument("--settle-tol", type=float, default=0.01,
                    help="settled: contacts per particle change by less than this fraction over 5000 steps")
    ap.add_argument("--sort-steps", type=int, default=200,
                    help="timed steps of the storage-order leg (scrambled order frozen vs re-sorted; 0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this stepper runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2501_05300_amd import beds
    from paper_2501_05300_amd.lprdem import Bed

    t0 = time.perf_counter()
    spec = beds.metric_bed(args.n, seed=args.seed)
    log(f"bed generated: n={spec.n} side={spec.box[0]:.4f} m in {time.perf_counter() - t0:.1f} s")
    settle = {"steps": 0, "contacts_per_particle": None, "criterion_met": False}
    if args.settle > 0:
        done, cbar_s, ok = settle_beds([spec], args.settle, max_steps=args.settle_max, rel_change=args.settle_tol)
        settle = {"steps": done, "contacts_per_particle": cbar_s, "criterion_met": ok,
                  "criterion": f"contacts per particle change < {args.settle_tol:g} relative over 5000 steps "
                               f"(at least {args.settle}, at most {args.settle_max} steps)"}
    bed = Bed(spec, rebuild_every=args.rebuild_every, skin=args.skin, block=args.block)
    log("bed created on the GPU")
    done = 0
    while done < args.warmup:
        k = min(500, args.warmup - done)
        bed.step(k)
        bed.sync()
        done += k
        log(f"warm-up {done}/{args.warmup}")
    # timed region: the steps as a user runs them (captured-graph cycles)
    bed.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bed.step(args.steps)
    bed.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = bed.stats()
    log(f"timed {args.steps} steps in {wall:.3f} s")
    # the same number of steps again with HIP events at every phase boundary
    # (direct launches) for the per-kernel durations
    prof = bed.step_phases(args.steps)
    log(f"phases over {args.steps} steps (ms): {prof}")
    N = spec.n
    pairs = st["contacts"]
    cbar = pairs / N
    value = N * args.steps / wall
    b_alg = B_PARTICLE + B_PAIR * cbar
    per_step = {k: v / args.steps for k, v in prof.items()}
    phases = {k: v for k, v in per_step.items() if k != "total"}
    dom = max(phases, key=phases.get)
    block = args.block or 64
    kname = PHASE_KERNEL[dom].format(block=block)
    rec = counter_record(N)
    mode = "every_step" if args.rebuild_every == 1 else "skin_lists"

    def roof(phase, kernel):
        t = per_step[phase] * 1e-3
        ach = N * b_alg / t / 1e9
        tr = kernel_traffic(rec, mode, kernel)
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": tr, "traffic_frac": (tr / t / 1e9 / HBM_PEAK_GBS) if tr else None, "kernel": kernel,
                "launch_ms": per_step[phase], "bytes_per_particle_step": b_alg,
                "algorithmic_bytes_per_launch": N * b_alg}

    step_bytes = None
    if rec is not None:
        step_bytes = rec.get("hbm_bytes_per_step" if mode == "every_step" else "hbm_bytes_per_step_skin_lists")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 law, f64 positions/geometry/reactions",
        "data": "synthetic",
        "config": {"workload": "graded bed, 2M spheres, r0 1.5 mm, L 20 mm, k 1, cap 8 r0, 0.2 m deep, "
                               "periodic, floor, dt 2e-6 s, settled",
                   "settle": settle,
                   "n": N, "side_m": spec.box[0], "rebuild_every": args.rebuild_every, "skin_m": args.skin,
                   "timed": "lpr_step (captured-graph cycles); per-phase durations from lpr_step_phases over "
                            "the same number of steps right after"},
        "contacts_per_s": pairs * args.steps / wall,
        "contacts_per_particle": cbar,
        "kernel_ms_per_step": per_step,
        # the step's algorithmic bytes over the largest phase's kernel time
        "roofline": roof(dom, kname),
        "roofline_step_kernel": roof("contact_step", PHASE_KERNEL["contact_step"].format(block=block)),
        "algorithmic_frac_whole_step": N * b_alg / (wall / args.steps) / 1e9 / HBM_PEAK_GBS,
        "counter_frac_whole_step": (step_bytes / (wall / args.steps) / 1e9 / HBM_PEAK_GBS) if step_bytes else None,
        "paper_context": {
            "absolute_throughput_reported": False,
            "relative": "refined beds ran 3.1x to 43.0x faster than the 305k-sphere uniform reference bed "
                        "(2.3x to 25x fewer particles, fewer Gauss-Seidel iterations); implicit CPU solver, "
                        "hardware and precision not stated (abstract; results on simulation speed)",
        },
    }
    if args.secondary_every > 1:
        bed.close()
        skin = args.secondary_skin * float(spec.radius.min())
        bed = Bed(spec, rebuild_every=args.secondary_every, skin=skin, block=args.block)
        bed.step(args.warmup)
        bed.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        bed.step(args.steps)
        bed.sync()
        torch.cuda.synchronize()
        wall2 = time.perf_counter() - t1
        st2 = bed.stats()
        prof2 = bed.step_phases(args.steps)
        log(f"skin lists (every {args.secondary_every}, skin {skin:.2e} m): {args.steps} steps in {wall2:.3f} s; "
            f"phases {prof2}; trips {st2['skin_trips']}")
        step2 = prof2["contact_step"] / args.steps
        b2 = B_PARTICLE + B_PAIR * st2["contacts"] / N
        tr2 = kernel_traffic(rec, "skin_lists", PHASE_KERNEL["contact_step"].format(block=block))
        sb2 = rec.get("hbm_bytes_per_step_skin_lists") if rec else None
        out["skin_lists"] = {
            "value": N * args.steps / wall2, "ms_per_step": 1e3 * wall2 / args.steps,
            "rebuild_every": args.secondary_every, "skin_m": skin, "skin_trips": st2["skin_trips"],
            "contacts_per_particle": st2["contacts"] / N, "candidates_per_particle": st2["candidates"] / N,
            "kernel_ms_per_step": {k: v / args.steps for k, v in prof2.items()},
            "step_kernel_achieved_GBs": N * b2 / (step2 * 1e-3) / 1e9,
            "step_kernel_frac": N * b2 / (step2 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "step_kernel_traffic": tr2,
            "step_kernel_traffic_frac": tr2 / (step2 * 1e-3) / 1e9 / HBM_PEAK_GBS if tr2 else None,
            "algorithmic_frac_whole_step": N * b2 / (wall2 / args.steps) / 1e9 / HBM_PEAK_GBS,
            "counter_frac_whole_step": (sb2 / (wall2 / args.steps) / 1e9 / HBM_PEAK_GBS) if sb2 else None,
        }
    if args.sort_steps > 0:
        out["storage_order"] = sort_leg(spec, args.sort_steps, args.warmup, args.block)
    if args.cpu_steps > 0:
        pos, vel, omg = bed.state()
        keys, vals = bed.history()
        clock = bed.clock()
        log("CPU baseline: oracle on the same state")
        out["cpu_baseline"] = cpu_baseline(spec, pos, vel.astype(np.float64), omg.astype(np.float64), keys,
                                           vals.astype(np.float64), clock, args.cpu_steps)
    bed.close()
    if args.implicit_steps > 0:
        out["implicit"] = implicit_leg(spec, args.implicit_steps, 4, args.implicit_sweeps)
        out["implicit"]["explicit_simulated_s_per_wall_s"] = spec.params.dt * args.steps / wall
    if args.batch_steps > 0:
        out["batched"] = batch_leg(args.batch_steps, 100, args.batch_settle, 10)
    if args.adjoint_window > 0:
        out["adjoint"] = adjoint_leg(50_000, args.adjoint_window, 100, args.settle, 50_000, args.seed)
    if args.calibrate_window > 0:
        out["calibration"] = calibration_leg(50_000, args.calibrate_window, 100, args.settle, args.seed)
    if args.cpu_configs:
        out["cpu_configs"] = cpu_configs_leg()
    if args.emission:
        out["emission"] = emission_leg(args.seed)
    if args.terramech:
        out["terramech"] = terramech_leg(args.seed)
    if args.configs:
        out["other_configs"] = configs_leg(20_000, 10_000, 200, args.settle)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
