"""Profiling workload: the settled 2M-sphere graded bed stepped in one mode
(every-step search, skin lists, or the time-implicit step),
plus a plain device copy of known size (the reference for scaling HBM
counters).  Run it under rocprofv3; the settled state is cached in a file so
that counter passes need not settle again.

  python -m paper_2501_05300_amd.profile_workload --settle-only --cache /tmp/m.npz
  rocprofv3 --pmc FETCH_SIZE -- python -m paper_2501_05300_amd.profile_workload --cache /tmp/m.npz --steps 20
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(f"[profile] {msg}", file=sys.stderr, flush=True)


def settled_metric_bed(cache, settle):
    from paper_2501_05300_amd import beds
    spec = beds.metric_bed()
    if cache and os.path.exists(cache):
        spec.pos = np.load(cache)["pos"]
        log(f"loaded settled state from {cache}")
        return spec
    import bench
    done, cbar, ok = bench.settle_beds([spec], settle, max_steps=200_000)
    log(f"settled {done} steps, contacts per particle {cbar:.3f}, criterion met: {ok}")
    if cache:
        np.savez(cache, pos=spec.pos)
    return spec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cache", default="")
    ap.add_argument("--settle", type=int, default=40000)
    ap.add_argument("--settle-only", action="store_true")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--rebuild-every", type=int, default=1)
    ap.add_argument("--skin", type=float, default=0.0)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--stats-out", default="", help="write the bed's stats after the steps to this JSON file")
    ap.add_argument("--implicit", type=int, default=0,
                    help="> 0: the time-implicit step at dt 0.1 ms with this many iterations per step")
    args = ap.parse_args()
    import torch
    from paper_2501_05300_amd.lprdem import Bed
    spec = settled_metric_bed(args.cache, args.settle)
    if args.settle_only:
        return
    # plain copy of known size: args.copy_mib MiB read, the same written
    a = torch.empty(args.copy_mib * 1024 * 1024 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {args.copy_mib} MiB")
    del a, b
    if args.implicit > 0:
        spec.params = spec.params.replace(dt=1e-4)
    bed = Bed(spec, rebuild_every=args.rebuild_every, skin=args.skin)
    if args.implicit > 0:
        bed.set_stepper("spook", args.implicit)
    bed.step(max(2 * args.rebuild_every, 4))
    bed.sync()
    t0 = time.perf_counter()
    bed.step(args.steps)
    bed.sync()
    st = bed.stats()
    log(f"{args.steps} steps in {time.perf_counter() - t0:.3f} s; stats {st}")
    if args.stats_out:
        import json
        with open(args.stats_out, "w") as f:
            json.dump({**st, "n": spec.n, "contacts_per_particle": st["contacts"] / spec.n}, f)


if __name__ == "__main__":
    main()
