"""Pressure-sinkage and shear-displacement protocol on refined and control
beds, with the paper's accuracy metric (section "Simulations": the test with
a grousered plate; section "Results": sinkage, traction and the aggregate
error).

A rigid plate with grousers below it is lowered slowly onto the bed until
the particles carry its load, then left under a dead weight (a body free in
z).  Phase I holds it in place horizontally: the sinkage it reaches is the
static sinkage.  Phases II-III pull it horizontally at a
constant speed while the load stays: the pull force F_T = -R_x (R the
reaction of the particles on the plate) gives the tractive resistance
F_T / F_N, its early peak is the initial peak traction, its mean over the
pull the average traction, and the sinkage at the end of the pull the
dynamic sinkage.  Against a reference bed, each measure gives a normalised
error (sinkage difference over the grouser depth, traction difference as a
force over the maximum load) and the aggregate error is the mean of the
four magnitudes.  Every step runs in the HIP library.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict

import numpy as np

from . import beds, emission


@dataclasses.dataclass
class Plate:
    length: float = 0.10      # along the pull (x)
    width: float = 0.06
    n_grousers: int = 4
    h_grouser: float = 0.0143  # grouser depth below the plate face
    t_grouser: float = 0.004   # grouser thickness along x
    t_face: float = 0.005      # plate thickness above the grousers
    pressure: float = 5.0e3    # normal stress over the plate area (load F_N = pressure * area): below the
                               # bearing capacity of this plate on this sand (about gamma D N_q + gamma B N_gamma
                               # / 2, some 9 kPa with the face at grouser depth); the paper's 50 kPa holds
                               # only for its larger plate

    @property
    def load(self) -> float:
        return self.pressure * self.length * self.width


def add_grouser_plate(spec: beds.BedSpec, plate: Plate, g: float = 9.81, speed: float = 0.0,
                      origin_x: float = None, vz0: float = 0.0, z_free: bool = True) -> beds.BedSpec:
    """The plate as a body free in z with mass F_N / g (initial vertical
    speed vz0), or with its vertical motion prescribed at vz0 (z_free
    False), grouser tips on the surface under it, moving along x at `speed`:
    a face box over grouser boxes spanning the width."""
    Lx, Ly = spec.box[0], spec.box[1]
    cx, cy = 0.5 * Lx, 0.5 * Ly
    R = 0.5 * math.hypot(plate.length, plate.width)
    z0 = beds.surface_height(spec.pos, spec.radius, cx, cy, R, spec.box) + plate.h_grouser
    b = len(spec.bodies)
    spec.bodies.append(beds.Body(origin=(cx if origin_x is None else origin_x, cy, z0), lin_vel=(speed, 0.0, vz0),
                                 z_free=1 if z_free else 0, mass=plate.load / g))
    eye = (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0)
    spec.walls.append(beds.Wall(kind=beds.WALL_BOX, body=b, origin=(0.0, 0.0, 0.5 * plate.t_face), frame=eye,
                                dims=(0.5 * plate.length, 0.5 * plate.width, 0.5 * plate.t_face)))
    pitch = plate.length / plate.n_grousers
    for q in range(plate.n_grousers):
        x = -0.5 * plate.length + (q + 0.5) * pitch
        spec.walls.append(beds.Wall(kind=beds.WALL_BOX, body=b, origin=(x, 0.0, -0.5 * plate.h_grouser), frame=eye,
                                    dims=(0.5 * plate.t_grouser, 0.5 * plate.width, 0.5 * plate.h_grouser)))
    spec.info["plate_body"] = b
    return spec


def linear_bed(d_min: float, d_max: float, gamma: float, depth: float, Lx: float, Ly: float, seed=0,
               params=None) -> beds.BedSpec:
    """Bed refined by the paper's linear profile d(z) = d_min + gamma z up to
    d_max (gamma = 0: uniform at d_min), deposited at rest and relaxed with
    the paper's relaxation friction for at least 0.3 s, then until it is
    still."""
    rng = np.random.default_rng(seed)
    prm = params or beds.paper_params()
    prof = beds.linear_profile(d_min, gamma, d_max) if gamma > 0 else (
        lambda z: np.full(np.shape(z), 0.5 * d_min, dtype=np.float64))
    n = int(round(beds.count_per_area(prof, depth) * Lx * Ly))
    pos, rad = beds.profile_bed(n, prof, depth, Lx, Ly, rng)
    relax_prm = beds.settle_params(prm).replace(dt=5e-6, gamma_factor=10.0)
    z = np.zeros((n, 3), np.float32)
    pos, _, _, _ = emission.relax(pos, rad, z, z, (Lx, Ly), relax_prm, v_tol=0.02,
                                  min_steps=int(round(0.3 / relax_prm.dt)))
    return beds.BedSpec(pos=pos, radius=rad, vel=np.zeros((n, 3), np.float32), omega=np.zeros((n, 3), np.float32),
                        box=(Lx, Ly, 0.0), periodic=3, params=prm, walls=[beds.floor_wall()], bodies=[beds.Body()],
                        info={"workload": "linear-profile", "d_min": d_min, "d_max": d_max, "gamma": gamma})


def _phase_bed(spec, plate, state, history, clock, z_start, z, vz, speed, z_free, b_expect):
    """A bed at (state, history, clock) with the plate at height z (z_start
    the height its pose is measured from) moving along x at `speed`; its x
    pose stays where the previous phase left it (x(t) = origin_x + speed t)."""
    from .lprdem import Bed
    dt = spec.params.dt
    s = spec.copy()
    s.pos, s.vel, s.omega = state
    x0 = 0.5 * spec.box[0]
    if z_free:
        add_grouser_plate(s, plate, speed=speed, origin_x=x0 - speed * clock * dt)
        b = s.info["plate_body"]
        s.bodies[b].origin = (s.bodies[b].origin[0], s.bodies[b].origin[1], z_start)
    else:  # prescribed descent at vz from z at this clock
        add_grouser_plate(s, plate, speed=speed, origin_x=x0 - speed * clock * dt, vz0=vz, z_free=False)
        b = s.info["plate_body"]
        s.bodies[b].origin = (s.bodies[b].origin[0], s.bodies[b].origin[1], z - vz * clock * dt)
    assert b == b_expect
    bed = Bed(s)
    if history is not None:
        bed.set_history(*history)
    bed.set_clock(clock)
    if z_free:
        bed.set_body_state(b, z, vz)
    return bed


def run_protocol(spec: beds.BedSpec, plate: Plate, t_static: float, pull_speed: float, pull_distance: float,
                 samples: int = 60, lower_speed: float = 0.2, log=None) -> Dict:
    """Lowers the plate at lower_speed until the particles carry its load,
    then phase I for t_static seconds (free in z under the load, held in x),
    then phases II-III: a pull of pull_distance at pull_speed.  Returns the
    sinkage and traction series and the four measures; sinkage is measured
    from grouser tips resting on the highest sphere under the plate."""
    dt = spec.params.dt
    s0 = spec.copy()
    add_grouser_plate(s0, plate)
    b = s0.info["plate_body"]
    z_start = s0.bodies[b].origin[2]
    state = (spec.pos, spec.vel, spec.omega)
    # lowering: prescribed descent until the mean reaction over a chunk
    # reaches the load (at most three grouser depths)
    bed = _phase_bed(spec, plate, state, None, 0, z_start, z_start, -lower_speed, 0.0, False, b)
    chunk0 = max(1, int(round(0.05 * plate.h_grouser / lower_speed / dt)))
    bed.reaction_window(b, reset=True)
    done = 0
    while done * dt * lower_speed < 3.0 * plate.h_grouser:
        bed.step(chunk0)
        done += chunk0
        sum6, cnt = bed.reaction_window(b, reset=True)
        if sum6[2] / max(cnt, 1) >= plate.load:
            break
    o, _ = bed.body(b)
    z_low = float(o[2])
    state, history, clock = bed.state(), bed.history(), bed.clock()
    bed.close()
    if log:
        log(f"lowering: {done} steps to {(z_start - z_low) * 1e3:.2f} mm")
    # phase I: free in z under the load
    bed = _phase_bed(spec, plate, state, history, clock, z_start, z_low, 0.0, 0.0, True, b)
    n1 = int(round(t_static / dt))
    bed.step(n1)
    bed.sync()
    o, v = bed.body(b)
    static = z_start - float(o[2])
    state, history, clock = bed.state(), bed.history(), bed.clock()
    bed.close()
    if log:
        log(f"phase I: {n1} steps, static sinkage {static * 1e3:.3f} mm")
    # phases II-III: pulled along x under the same load
    bed = _phase_bed(spec, plate, state, history, clock, z_start, float(o[2]), float(v[2]), pull_speed, True, b)
    n2 = int(round(pull_distance / pull_speed / dt))
    chunk2 = max(1, n2 // samples)
    t, sink, trac = [], [], []
    bed.reaction_window(b, reset=True)
    done2 = 0
    while done2 < n2:
        k = min(chunk2, n2 - done2)
        bed.step(k)
        done2 += k
        sum6, cnt = bed.reaction_window(b, reset=True)
        o2, _ = bed.body(b)
        t.append(done2 * dt)
        sink.append(z_start - float(o2[2]))
        trac.append(-(sum6[0] / max(cnt, 1)) / plate.load)
    bed.sync()
    bed.close()
    trac = np.array(trac)
    k_peak = max(1, len(trac) // 3)
    out = {"static_sinkage": static, "dynamic_sinkage": sink[-1], "peak_traction": float(np.max(trac[:k_peak])),
           "average_traction": float(np.mean(trac)), "t": t, "sinkage": sink, "traction": trac.tolist(),
           "steps": done + n1 + n2, "lowering_steps": done}
    if log:
        log(f"phases II-III: {n2} steps, dynamic sinkage {out['dynamic_sinkage'] * 1e3:.2f} mm, peak traction "
            f"{out['peak_traction']:.3f}, average {out['average_traction']:.3f}")
    return out


def normalized_errors(m: Dict, ref: Dict, h_grouser: float, F_N_max: float, F_N: float) -> Dict:
    """Section "Aggregate error": sinkage errors (z - z_ref) / h_grouser for
    the static and dynamic sinkage, traction errors (F_T - F_T,ref) / F_N,max
    for the initial peak and the average (F_T = traction ratio x F_N), and
    the aggregate error, the mean of the four magnitudes."""
    e = {"static_sinkage": (m["static_sinkage"] - ref["static_sinkage"]) / h_grouser,
         "dynamic_sinkage": (m["dynamic_sinkage"] - ref["dynamic_sinkage"]) / h_grouser,
         "peak_traction": (m["peak_traction"] - ref["peak_traction"]) * F_N / F_N_max,
         "average_traction": (m["average_traction"] - ref["average_traction"]) * F_N / F_N_max}
    e["aggregate"] = float(np.mean([abs(v) for v in e.values()]))
    return e
