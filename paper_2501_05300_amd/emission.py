"""Layer-by-layer emission of refined beds.

Section "Generation of soil samples": a bed with a refinement profile is
built from the bottom up in layers.  Layer n holds spheres of diameter d_n
(uniform in [0.9, 1.1] d_n) and is filled to a height eta d_n; then the
emitter pauses and every sphere above the layer is removed before the next
layer is emitted.  Emission and relaxation use reduced friction (mu_t 0.1,
mu_r 0.01, none at the container walls).  The layers follow the layer
construction of section "Local particle refinement and scaling
agressiveness": d_n = r^n d_min, thickness eta d_n, a uniform base of d_max
below the deepest layer, scaling aggressiveness gamma = (r - 1) / (r eta).

This module plans the layers, places each layer's spheres (sheets of a
jittered lattice above the current surface, never overlapping), trims, and
computes the diagnostics the paper checks: the size profile, mixing between
layers (percolation of finer spheres into coarser layers) and the bulk
density with its local variation.  Every step of the fall and relaxation
runs in the HIP library (lprdem).
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

import numpy as np

from . import beds

EU3 = (1.1 ** 4 - 0.9 ** 4) / (4 * 0.2)   # E[u^3] for u uniform in [0.9, 1.1]


@dataclasses.dataclass
class Layer:
    d: float      # nominal diameter
    z_lo: float   # bottom height above the floor
    z_hi: float   # top height above the floor


def gamma_of(r: float, eta: float) -> float:
    """Scaling aggressiveness of a layering with ratio r and thickness factor eta."""
    return (r - 1.0) / (r * eta)


def plan_layers(d_min: float, r: float, eta: float, n_layers: int, height: float) -> List[Layer]:
    """Layers from the floor up: a uniform base of d_max = r^n_layers d_min
    below z_max (depth of the deepest refined layer's bottom), then refined
    layers n = n_layers - 1, ..., 0 of diameter r^n d_min and thickness
    eta d_n, the finest at the surface (height `height`)."""
    d, zb = beds.layer_profile(d_min, r, eta, n_layers)   # diameters, depth of each layer's bottom
    z_max = float(zb[-1])
    if not (height > z_max):
        raise ValueError("the bed must be deeper than its refined layers")
    out = [Layer(d_min * r ** n_layers, 0.0, height - z_max)]
    for n in range(n_layers - 1, -1, -1):
        out.append(Layer(float(d[n]), height - float(zb[n]), height - float(zb[n]) + eta * float(d[n])))
    return out


def emission_count(layer: Layer, side: float, phi: float = 0.62, excess: float = 1.25) -> int:
    """Spheres to emit for a layer: `excess` times what fills it at packing
    fraction phi (the surplus is trimmed)."""
    vol = side * side * (layer.z_hi - layer.z_lo)
    return int(math.ceil(excess * phi * vol / ((math.pi / 6.0) * EU3 * layer.d ** 3)))


def emit(rng, layer: Layer, side: float, z_start: float, count: int):
    """`count` spheres of the layer's size in sheets of a square lattice above
    z_start.  Lattice spacing s >= 1.21 d and a jitter below 0.05 d keep
    every pair (also across the periodic sides) apart."""
    d = layer.d
    nx = max(1, int(math.floor(side / (1.21 * d))))
    s = side / nx
    per_sheet = nx * nx
    sheets = int(math.ceil(count / per_sheet))
    k = np.arange(sheets * per_sheet)[:count]
    ix, iy, iz = k % nx, (k // nx) % nx, k // per_sheet
    jit = 0.05 * d * rng.uniform(-1.0, 1.0, (count, 2))
    pos = np.stack([(ix + 0.5) * s + jit[:, 0], (iy + 0.5) * s + jit[:, 1], z_start + (iz + 0.5) * s], 1)
    rad = (0.5 * d * rng.uniform(0.9, 1.1, count)).astype(np.float32)
    return pos, rad


def relax_spec(pos, rad, vel, omg, side, params) -> "beds.BedSpec":
    """The bed a relaxation steps: the spheres in a box periodic in x and y
    (side `side`, or (Lx, Ly)) on a frictionless floor, with `params`."""
    n = len(rad)
    Lx, Ly = (side, side) if np.isscalar(side) else side
    return beds.BedSpec(pos=np.ascontiguousarray(pos, np.float64), radius=np.asarray(rad, np.float32),
                        vel=np.asarray(vel, np.float32).reshape(n, 3), omega=np.asarray(omg, np.float32).reshape(n, 3),
                        box=(Lx, Ly, 0.0), periodic=3, params=params, walls=[beds.floor_wall(0.0, 0.0)],
                        bodies=[beds.Body()], info={"workload": "emission"})


def relax_lists(spec) -> dict:
    """Broad-phase settings of a relaxation: candidate lists with a skin of a
    quarter of the smallest radius, rebuilt every 5 steps."""
    return {"rebuild_every": 5, "skin": 0.25 * float(np.min(spec.radius))}


def relax(pos, rad, vel, omg, side, params, v_tol=0.02, chunk=4000, max_steps=200_000, min_steps=0):
    """Steps the spheres on the GPU (periodic sides of length `side`, or
    (Lx, Ly), frictionless floor, the paper's relaxation friction) in chunks
    for at least min_steps and then until the fastest moves slower than
    v_tol (a packing deposited at rest starts slow: it needs the minimum to
    compact), at most max_steps (rounded up to whole chunks).  Returns
    positions, velocities, spins and the steps taken."""
    from .lprdem import Bed
    spec = relax_spec(pos, rad, vel, omg, side, params)
    bed = Bed(spec, **relax_lists(spec))
    steps = 0
    try:
        while True:
            bed.step(chunk)
            bed.sync()
            steps += chunk
            x, v, w = bed.state()
            if (steps >= min_steps and float(np.abs(v).max()) < v_tol) or steps >= max_steps:
                break
    finally:
        bed.close()
    return x, v, w, steps


@dataclasses.dataclass
class EmittedBed:
    pos: np.ndarray
    radius: np.ndarray
    layer: np.ndarray        # index into `layers` of each sphere's layer
    layers: List[Layer]
    side: float
    steps: int
    emitted: int
    seconds: float


def emit_bed(d_min, r, eta, n_layers, height, side, seed=0, params=None, v_tol=0.02, chunk=4000,
             max_steps=200_000, log=None) -> EmittedBed:
    """Builds a refined bed layer by layer (see the module docstring).
    `params` are the material parameters (the paper's set by default); the
    fall and relaxation use its reduced friction with dt 5e-6 s and extra
    normal damping (gamma_n = 10 dt)."""
    rng = np.random.default_rng(seed)
    base = params or beds.paper_params()
    relax_params = beds.settle_params(base).replace(dt=5e-6, gamma_factor=10.0)
    layers = plan_layers(d_min, r, eta, n_layers, height)
    pos = np.zeros((0, 3))
    rad = np.zeros(0, np.float32)
    lay = np.zeros(0, np.int32)
    vel = np.zeros((0, 3), np.float32)
    omg = np.zeros((0, 3), np.float32)
    steps = emitted = 0
    t0 = time.perf_counter()
    for q, L in enumerate(layers):
        top = float(np.max(pos[:, 2] + rad)) if len(rad) else 0.0
        cnt = emission_count(L, side)
        p_new, r_new = emit(rng, L, side, max(top, L.z_lo) + 0.1 * L.d, cnt)
        pos = np.concatenate([pos, p_new])
        rad = np.concatenate([rad, r_new])
        lay = np.concatenate([lay, np.full(cnt, q, np.int32)])
        vel = np.concatenate([vel, np.zeros((cnt, 3), np.float32)])
        omg = np.concatenate([omg, np.zeros((cnt, 3), np.float32)])
        emitted += cnt
        pos, vel, omg, k = relax(pos, rad, vel, omg, side, relax_params, v_tol, chunk, max_steps)
        steps += k
        keep = pos[:, 2] <= L.z_hi      # the surplus above the layer is removed
        pos, rad, lay, vel, omg = pos[keep], rad[keep], lay[keep], vel[keep], omg[keep]
        if log:
            log(f"layer {q} (d {L.d * 1e3:.2f} mm, {L.z_lo:.4f}-{L.z_hi:.4f} m): emitted {cnt}, kept "
                f"{int(np.sum(lay == q))}, {k} steps, {time.perf_counter() - t0:.1f} s")
    return EmittedBed(pos=pos, radius=rad, layer=lay, layers=layers, side=side, steps=steps, emitted=emitted,
                      seconds=time.perf_counter() - t0)


def mixing(pos, radius, layer, layers: List[Layer]) -> np.ndarray:
    """Per layer, the fraction of its spheres whose centre lies below the
    layer's bottom by more than half its diameter (spheres that percolated
    into a coarser layer)."""
    out = np.zeros(len(layers))
    for q, L in enumerate(layers):
        sel = layer == q
        if np.any(sel):
            out[q] = float(np.mean(pos[sel, 2] < L.z_lo - 0.5 * L.d))
    return out


def density_profile(pos, radius, rho, side, z_lo, z_hi, n_bins):
    """Bulk density in horizontal slabs between z_lo and z_hi: the volume of
    every sphere cut by each slab (exact spherical-cap integral) times rho,
    over the slab volume."""
    edges = np.linspace(z_lo, z_hi, n_bins + 1)
    r = np.asarray(radius, np.float64)
    z = np.asarray(pos)[:, 2]

    def below(h):   # volume of each sphere below height h
        t = np.clip(h - (z - r), 0.0, 2.0 * r)
        return math.pi * t * t * (3.0 * r - t) / 3.0

    vol = np.array([np.sum(below(edges[k + 1]) - below(edges[k])) for k in range(n_bins)])
    return rho * vol / (side * side * np.diff(edges)), edges


def diagnostics(bed: EmittedBed, rho: float, n_bins: Optional[int] = None) -> dict:
    """Size profile per layer, mixing, and the bulk density with its
    variation over slabs at least one coarse diameter thick, away from the
    floor and the surface by one coarse diameter."""
    d_max = bed.layers[0].d
    height = bed.layers[-1].z_hi
    lo, hi = d_max, height - bed.layers[-1].d
    nb = n_bins or max(1, int((hi - lo) / d_max))
    dens, _ = density_profile(bed.pos, bed.radius, rho, bed.side, lo, hi, nb)
    med = [float(np.median(2.0 * bed.radius[bed.layer == q])) if np.any(bed.layer == q) else float("nan")
           for q in range(len(bed.layers))]
    return {"layers": [{"d": L.d, "z_lo": L.z_lo, "z_hi": L.z_hi, "count": int(np.sum(bed.layer == q)),
                        "median_d": med[q]} for q, L in enumerate(bed.layers)],
            "mixing": mixing(bed.pos, bed.radius, bed.layer, bed.layers).tolist(),
            "density_mean": float(np.mean(dens)), "density_rel_std": float(np.std(dens) / np.mean(dens)),
            "density_max_rel_dev": float(np.max(np.abs(dens / np.mean(dens) - 1.0))),
            "top": float(np.max(bed.pos[:, 2])), "n": int(len(bed.radius))}
