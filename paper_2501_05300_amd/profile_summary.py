"""Turns rocprofv3 output of the profiling workload into the short text
summaries kept under profiles/, and the counter record bench.py reads.

Inputs (directories written by the commands listed in each summary):
  trace_every, trace_skin   rocprofv3 --kernel-trace --stats (csv)
  fetch_every, write_every  rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (csv)
  fetch_skin, write_skin    the same with candidate lists and a skin

HBM bytes per launch = FETCH_SIZE * fetch_scale + WRITE_SIZE * write_scale
(KiB per dispatch).  The scales come from the plain 1 GiB device copy the
workload runs first (a copy of B bytes reads B and writes B).

  python -m paper_2501_05300_amd.profile_summary <dir containing the above>
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
N_METRIC = 2_000_000
COPY_BYTES = 1 << 30
SKIN = 6.979699828661979e-05  # 0.05 r_min of the metric bed, the bench's skin-list run
SETTLE = "python3 -m paper_2501_05300_amd.profile_workload --settle-only --cache /tmp/m.npz"
WORK = "python3 -m paper_2501_05300_amd.profile_workload --cache /tmp/m.npz"
SKIN_ARGS = f"--rebuild-every 50 --skin {SKIN!r}"
# algorithmic bytes per particle-step: x (24) + r (4) + v (12) + omega (12)
# read, x + v + omega (48) written; per contact pair 24 B of history and a
# 4 B partner id, read and written
B_PARTICLE = 100.0
B_PAIR = 56.0


def _code_only(text: str) -> str:
    """Source text without comments and whitespace (string literals in these
    files hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return re.sub(r"\s+", "", text)


def kernel_source_hash() -> str:
    """Hash of the device code (comments and layout ignored); a counter
    record is valid only for it."""
    h = hashlib.sha256()
    for f in ("lpr_dev.h", "lpr_cells.h", "lpr_kernels.hip"):
        with open(os.path.join(ROOT, "paper_2501_05300_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def spook_source_hash() -> str:
    """Hash of the implicit step's device code (comments and layout ignored)."""
    with open(os.path.join(ROOT, "paper_2501_05300_amd", "csrc", "lpr_spook.hip"), encoding="utf-8") as fh:
        return hashlib.sha256(_code_only(fh.read()).encode()).hexdigest()[:16]


def short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace("lpr::", "")
    return n if len(n) <= 27 else n[:24] + "..."


def kernel_stats(d):
    out = []
    with open(os.path.join(d, "run_kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            out.append((short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6,
                        float(r["Percentage"])))
    return out


def counters(d):
    per = defaultdict(list)
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            per[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return per


def write_trace(src, name, title, args, steps, step_kernel="k_step"):
    rows = kernel_stats(src)
    # every step launches its step (or finish) kernel once, so its calls
    # count the traced steps (the timed ones and the workload's warm-up)
    traced = next(c for n, c, a, t, p in rows if n.startswith(step_kernel))
    lines = [f"# rocprofv3 kernel trace: {title}",
             "# commands:",
             f"#   {SETTLE}",
             f"#   rocprofv3 --kernel-trace --stats -d <dir> -o run --output-format csv -- {WORK} --steps {steps}{args}",
             f"# the trace holds {traced} steps ({steps} timed after the workload's warm-up); "
             f"ms/step = total / {traced}",
             f"{'kernel':<28}{'calls':>7}{'avg us':>10}{'total ms':>10}{'ms/step':>9}{'share %':>9}"]
    for n, c, a, t, p in rows:
        lines.append(f"{n:<28}{c:>7}{a:>10.1f}{t:>10.2f}{t / traced:>9.4f}{p:>9.2f}")
    with open(os.path.join(PROFILES, name), "w") as f:
        f.write("\n".join(lines) + "\n")
    return {n: a for n, c, a, t, p in rows}, {n: c / traced for n, c, a, t, p in rows}


def scales(fetch, write):
    copy_f = fetch["__amd_rocclr_copyBuffer"]
    copy_w = write["__amd_rocclr_copyBuffer"]
    big_f = max(copy_f) * 1024.0
    big_w = max(copy_w) * 1024.0
    return COPY_BYTES / big_f, COPY_BYTES / big_w, big_f, big_w


def write_traffic(fdir, wdir, avg_us, name, title, args, cbar, alg_line=None, steps=6):
    fetch, write = counters(fdir), counters(wdir)
    sf, sw, big_f, big_w = scales(fetch, write)
    lines = [f"# rocprofv3 HBM counters: {title}",
             "# commands:",
             f"#   {SETTLE}",
             f"#   rocprofv3 --pmc FETCH_SIZE -d <dir> -o run --output-format csv -- {WORK} --steps {steps}{args}",
             f"#   rocprofv3 --pmc WRITE_SIZE -d <dir> -o run --output-format csv -- {WORK} --steps {steps}{args}",
             f"# calibration: a {COPY_BYTES >> 20} MiB device copy reads FETCH_SIZE {big_f / 2**20:.1f} MiB and WRITE_SIZE "
             f"{big_w / 2**20:.1f} MiB, so fetch x{sf:.3f}, write x{sw:.3f}",
             alg_line or (f"# algorithmic bytes per particle-step B_alg = {B_PARTICLE:.0f} + {B_PAIR:.0f} c (c = {cbar:.3f} "
                          f"pairs per particle) = {B_PARTICLE + B_PAIR * cbar:.1f} B; {N_METRIC} particles"),
             f"{'kernel':<28}{'fetch MB':>10}{'write MB':>10}{'HBM MB':>10}{'avg us':>9}{'GB/s':>9}{'% of 8 TB/s':>12}"]
    rec = {}
    for k in sorted(fetch):
        if k.startswith("__amd") or k.startswith("at::") or k not in write:
            continue
        f_ = sum(fetch[k]) / len(fetch[k]) * 1024.0 * sf
        w_ = sum(write[k]) / len(write[k]) * 1024.0 * sw
        t = avg_us.get(k)
        gbs = (f_ + w_) / (t * 1e-6) / 1e9 if t else float("nan")
        lines.append(f"{k:<28}{f_ / 1e6:>10.1f}{w_ / 1e6:>10.1f}{(f_ + w_) / 1e6:>10.1f}{(t or 0):>9.1f}{gbs:>9.0f}"
                     f"{100 * gbs / 8000:>12.1f}")
        rec[k] = {"fetch_bytes": f_, "write_bytes": w_, "avg_us": t}
    with open(os.path.join(PROFILES, name), "w") as f:
        f.write("\n".join(lines) + "\n")
    return rec, sf, sw


def measured_cbar(src, name, default):
    """Contacts per particle the workload recorded for a mode (or default)."""
    path = os.path.join(src, name)
    if os.path.exists(path):
        with open(path) as f:
            return float(json.load(f)["contacts_per_particle"])
    return default


def main(src, cbar_every=2.42, cbar_skin=2.42):
    os.makedirs(PROFILES, exist_ok=True)
    cbar_every = measured_cbar(src, "stats_every.json", cbar_every)
    cbar_skin = measured_cbar(src, "stats_skin.json", cbar_skin)
    every, calls_e = write_trace(os.path.join(src, "trace_every"), "kernels_metric_bed_every_step.txt",
                                 "settled 2,000,000-sphere graded bed, cell search every step", "", 100)
    skin, calls_s = write_trace(os.path.join(src, "trace_skin"), "kernels_metric_bed_skin_lists.txt",
                       "settled 2,000,000-sphere graded bed, candidate lists with a skin rebuilt every 50 steps",
                       " " + SKIN_ARGS, 200)
    rec_e, sf, sw = write_traffic(os.path.join(src, "fetch_every"), os.path.join(src, "write_every"), every,
                                  "hbm_traffic_metric_bed_every_step.txt", "settled 2,000,000-sphere graded bed, every step",
                                  "", cbar_every)
    rec_s, _, _ = write_traffic(os.path.join(src, "fetch_skin"), os.path.join(src, "write_skin"), skin,
                                "hbm_traffic_metric_bed_skin_lists.txt",
                                "settled 2,000,000-sphere graded bed, skin lists", " " + SKIN_ARGS, cbar_skin)
    step = next(k for k in rec_e if k.startswith("k_step"))

    def per_step(rec, calls):
        # HBM bytes of every kernel of the step, weighted by launches per step
        return sum((r["fetch_bytes"] + r["write_bytes"]) * calls.get(k, 0.0) for k, r in rec.items())

    out = {"kernel_source_hash": kernel_source_hash(), "n": N_METRIC, "kernel": step,
           "hbm_bytes_per_launch": rec_e[step]["fetch_bytes"] + rec_e[step]["write_bytes"],
           "hbm_bytes_per_launch_skin_lists": rec_s[step]["fetch_bytes"] + rec_s[step]["write_bytes"],
           "hbm_bytes_per_step": per_step(rec_e, calls_e),
           "hbm_bytes_per_step_skin_lists": per_step(rec_s, calls_s),
           "fetch_scale": sf, "write_scale": sw,
           "every_step": rec_e, "skin_lists": rec_s,
           "source": "profiles/hbm_traffic_metric_bed_every_step.txt, profiles/hbm_traffic_metric_bed_skin_lists.txt"}
    with open(os.path.join(PROFILES, "step_kernel_counters_metric_bed.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k not in ("every_step", "skin_lists")}, indent=1))


# Bytes one block-Jacobi sweep of the implicit step is designed to move, per
# particle and per contact (owner slot or wall): the sweep's own buffers (its
# rows, owner-side sums and partner parts) included, so this is design
# traffic, not a minimum that the method fixes.  Contacts kernel: the particle's
# velocity record (64 B) and flags (4 B) read, its owner-side sum written
# (48 B); per contact the partner index (4 B), the partner's velocity record
# (64 B), rows (64 B) and impulses (64 B) read, impulses (64 B) and the
# partner part (48 B) written.  Velocity kernel: state (64 B), split inverse
# masses (16 B), owner-side sum (48 B) and list offsets (8 B) read, velocity
# record (64 B) written; per contact a reverse entry (4 B) and partner part
# (48 B) read.
SWEEP_PARTICLE = 64 + 4 + 48 + 64 + 16 + 48 + 8 + 64
SWEEP_CONTACT = 4 + 64 + 64 + 64 + 64 + 48 + 4 + 48


def main_implicit(src, cbar, sweeps=250):
    """Summaries of the implicit step (dt 0.1 ms, `sweeps` sweeps): kernel
    trace and HBM counters; returns the sweep kernels' record."""
    os.makedirs(PROFILES, exist_ok=True)
    args = f" --implicit {sweeps}"
    avg, calls = write_trace(os.path.join(src, "trace_implicit"), "kernels_metric_bed_implicit.txt",
                             f"settled 2,000,000-sphere graded bed, time-implicit step at dt 0.1 ms, {sweeps} sweeps",
                             args, 6, step_kernel="k_sp_finish")
    alg = SWEEP_PARTICLE + SWEEP_CONTACT * cbar
    line = (f"# design bytes per particle-sweep (contacts + velocity kernels) = {SWEEP_PARTICLE} + "
            f"{SWEEP_CONTACT} c (c = {cbar:.3f} contacts per particle) = {alg:.1f} B; {N_METRIC} particles")
    rec, sf, sw = write_traffic(os.path.join(src, "fetch_implicit"), os.path.join(src, "write_implicit"), avg,
                                "hbm_traffic_metric_bed_implicit.txt",
                                f"settled 2,000,000-sphere graded bed, time-implicit step, {sweeps} sweeps", args,
                                cbar, alg_line=line, steps=1)
    sweep = {k: rec[k] for k in ("k_sp_contacts", "k_sp_vel")}
    t = sum(r["avg_us"] for r in sweep.values())
    b = sum(r["fetch_bytes"] + r["write_bytes"] for r in sweep.values())
    out = {"spook_source_hash": spook_source_hash(), "n": N_METRIC, "sweeps": sweeps, "contacts_per_particle": cbar,
           "sweep_us": t, "sweep_hbm_bytes": b, "sweep_design_bytes": alg * N_METRIC,
           "sweep_counter_frac": b / (t * 1e-6) / 1e9 / 8000.0,
           "sweep_design_frac": alg * N_METRIC / (t * 1e-6) / 1e9 / 8000.0, "kernels": sweep}
    out["source"] = "profiles/hbm_traffic_metric_bed_implicit.txt, profiles/kernels_metric_bed_implicit.txt"
    with open(os.path.join(PROFILES, "implicit_sweep_counters_metric_bed.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
    return out


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--implicit":
        main_implicit(sys.argv[2], float(sys.argv[3]) if len(sys.argv) > 3 else 2.385)
    else:
        main(sys.argv[1])
