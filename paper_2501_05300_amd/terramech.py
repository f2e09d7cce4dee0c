"""Pressure-sinkage and shear-displacement protocol on refined and control
beds, with the paper's accuracy metric (section "Simulations": the test with
a grousered plate; section "Results": sinkage, traction and the aggregate
error).

A rigid plate with grousers below it rests on the bed under a dead weight
(a body free in z).  Phase I holds it in place horizontally: the sinkage it
reaches is the static sinkage.  Phases II-III pull it horizontally at a
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
    pressure: float = 5.0e4 / 3.0   # normal stress over the plate area (load F_N = pressure * area): the
                                    # paper's 50 kPa scaled with length (stresses under gravity scale with
                                    # size; this plate is a third of the paper's)

    @property
    def load(self) -> float:
        return self.pressure * self.length * self.width


def add_grouser_plate(spec: beds.BedSpec, plate: Plate, g: float = 9.81, speed: float = 0.0,
                      origin_x: float = None, vz0: float = 0.0) -> beds.BedSpec:
    """The plate as a body free in z with mass F_N / g (initial vertical
    speed vz0), grouser tips on the surface under it, moving along x at
    `speed`: a face box over grouser boxes spanning the width."""
    Lx, Ly = spec.box[0], spec.box[1]
    cx, cy = 0.5 * Lx, 0.5 * Ly
    R = 0.5 * math.hypot(plate.length, plate.width)
    z0 = beds.surface_height(spec.pos, spec.radius, cx, cy, R, spec.box) + plate.h_grouser
    b = len(spec.bodies)
    spec.bodies.append(beds.Body(origin=(cx if origin_x is None else origin_x, cy, z0), lin_vel=(speed, 0.0, vz0),
                                 z_free=1, mass=plate.load / g))
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
    d_max (gamma = 0: uniform at d_min), deposited and relaxed with the
    paper's relaxation friction."""
    rng = np.random.default_rng(seed)
    prm = params or beds.paper_params()
    prof = beds.linear_profile(d_min, gamma, d_max) if gamma > 0 else (
        lambda z: np.full(np.shape(z), 0.5 * d_min, dtype=np.float64))
    n = int(round(beds.count_per_area(prof, depth) * Lx * Ly))
    pos, rad = beds.profile_bed(n, prof, depth, Lx, Ly, rng)
    relax_prm = beds.settle_params(prm).replace(dt=5e-6, gamma_factor=10.0)
    z = np.zeros((n, 3), np.float32)
    pos, _, _, _ = emission.relax(pos, rad, z, z, (Lx, Ly), relax_prm, v_tol=0.02)
    return beds.BedSpec(pos=pos, radius=rad, vel=np.zeros((n, 3), np.float32), omega=np.zeros((n, 3), np.float32),
                        box=(Lx, Ly, 0.0), periodic=3, params=prm, walls=[beds.floor_wall()], bodies=[beds.Body()],
                        info={"workload": "linear-profile", "d_min": d_min, "d_max": d_max, "gamma": gamma})


def run_protocol(spec: beds.BedSpec, plate: Plate, t_static: float, pull_speed: float, pull_distance: float,
                 samples: int = 60, log=None) -> Dict:
    """Phase I for t_static seconds, then phases II-III: a pull of
    pull_distance at pull_speed.  The plate's horizontal motion is
    prescribed; its height follows the load.  Returns the sinkage and
    traction series and the four measures."""
    from .lprdem import Bed
    dt = spec.params.dt
    s1 = spec.copy()
    add_grouser_plate(s1, plate)
    b = s1.info["plate_body"]
    z_start = s1.bodies[b].origin[2]
    bed = Bed(s1)
    n1 = int(round(t_static / dt))
    chunk1 = max(1, n1 // samples)
    t, sink, trac = [], [], []
    done = 0
    while done < n1:
        k = min(chunk1, n1 - done)
        bed.step(k)
        done += k
    bed.sync()
    o, v = bed.body(b)
    static = z_start - float(o[2])
    x, vel, w = bed.state()
    keys, vals = bed.history()
    clock = bed.clock()
    bed.close()
    if log:
        log(f"phase I: {n1} steps, static sinkage {static * 1e3:.3f} mm")
    # phases II-III: the same state with the plate moving along x; its pose
    # stays continuous (x(t) = origin_x + speed t)
    s2 = spec.copy()
    s2.pos, s2.vel, s2.omega = x, vel, w
    add_grouser_plate(s2, plate, speed=pull_speed, origin_x=0.5 * spec.box[0] - pull_speed * clock * dt)
    s2.bodies[b].origin = (s2.bodies[b].origin[0], s2.bodies[b].origin[1], z_start)
    bed = Bed(s2)
    bed.set_history(keys, vals)
    bed.set_clock(clock)
    bed.set_body_state(b, float(o[2]), float(v[2]))
    n2 = int(round(pull_distance / pull_speed / dt))
    chunk2 = max(1, n2 // samples)
    bed.reaction_window(b, reset=True)
    done = 0
    while done < n2:
        k = min(chunk2, n2 - done)
        bed.step(k)
        done += k
        sum6, cnt = bed.reaction_window(b, reset=True)
        o2, _ = bed.body(b)
        t.append(done * dt)
        sink.append(z_start - float(o2[2]))
        trac.append(-(sum6[0] / max(cnt, 1)) / plate.load)
    bed.sync()
    bed.close()
    trac = np.array(trac)
    k_peak = max(1, len(trac) // 3)
    out = {"static_sinkage": static, "dynamic_sinkage": sink[-1], "peak_traction": float(np.max(trac[:k_peak])),
           "average_traction": float(np.mean(trac)), "t": t, "sinkage": sink, "traction": trac.tolist(),
           "steps": n1 + n2}
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
