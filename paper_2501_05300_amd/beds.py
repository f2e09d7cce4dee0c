"""Seeded synthetic graded beds (inputs only).

This module builds the inputs that both the HIP library and the CPU oracle
step: sphere positions and radii, the material/contact parameters, walls and
kinematic bodies.  It holds no contact mechanics.

Radius profile.  The paper grades particle size with depth below the soil
surface (section "Local particle refinement and scaling aggressiveness",
Eq. 1: d(z) = d_min + gamma z up to d_max).  The beds here use the power-law
generalisation r(d) = r0 (1 + d/L)^k, capped at 8 r0 (k = 1 is the paper's
linear profile with gamma = 2 r0 / L), and the discrete-layer form of the same
section (d_n = r d_{n-1}, layer thickness eta d_n).  Every radius is jittered
uniformly in [0.9, 1.1] times its mean (section "Generation of soil samples").

Counts.  A bed is specified by its particle count; its lateral periodic side
follows from a count model: solid fraction phi = 1400/2200 (the paper's bulk
density over its particle density) integrated over the radius profile.  With
the paper's container this model reproduces the particle counts of its
uniform-bed table.

Placement.  Spheres are laid out in horizontal rafts (periodic hexagonal
lattices whose spacing exceeds the largest diameter in the raft) and each
raft is dropped onto the bed below, every sphere coming to rest touching the
spheres under it or the floor, with no overlaps (csrc/bedgen.c).  The rafts
are deposited bottom-up; a raft's mean radius is the profile value at the
depth where the count model puts that raft.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import List, Optional, Sequence

import numpy as np

PHI = 1400.0 / 2200.0          # solid fraction from the paper's bulk density
JITTER = 0.1                   # +-10 % radius jitter
EU3 = ((1 + JITTER) ** 4 - (1 - JITTER) ** 4) / (4 * 2 * JITTER)  # E[u^3], u ~ U(0.9, 1.1)

WALL_PLANE, WALL_DISK, WALL_ANNULUS, WALL_BOX = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# Descriptions shared by both steppers.

@dataclasses.dataclass
class Params:
    rho: float = 2200.0          # particle density [kg/m^3]
    E: float = 1.0e9             # Young's modulus [Pa]
    nu: float = 0.15             # Poisson ratio
    mu_t: float = 0.3            # Coulomb friction
    mu_r: float = 0.02           # rolling resistance
    dt: float = 2.0e-6           # time step [s]
    gamma_factor: float = 4.5    # gamma_n = gamma_factor * dt
    e_H: float = 1.25            # gap exponent (5/4 Hertz, 1 linear)
    kappa_t: Optional[float] = None  # tangential/normal stiffness ratio (None: 2(1-nu)/(2-nu))
    s_k: float = 1.0             # stiffness multiplier
    g: tuple = (0.0, 0.0, -9.81)

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)

    def kappa(self) -> float:
        """The tangential stiffness ratio in effect: the value given, or the
        Mindlin ratio 2(1 - nu)/(2 - nu) of this parameter set's nu (so a
        replace(nu=...) moves it along)."""
        if self.kappa_t is not None:
            return float(self.kappa_t)
        return 2.0 * (1.0 - self.nu) / (2.0 - self.nu)

    def field(self, name: str) -> float:
        """A scalar field for marshalling, with kappa_t resolved."""
        return self.kappa() if name == "kappa_t" else float(getattr(self, name))


def paper_params(**kw) -> Params:
    """The paper's dry-sand set: 2200 kg/m^3, 1 GPa, 0.15, mu_t 0.3, mu_r 0.02."""
    return Params(**kw)


def settle_params(base: Params) -> Params:
    """The paper's reduced friction for bed relaxation (mu_t 0.1, mu_r 0.01)."""
    return base.replace(mu_t=0.1, mu_r=0.01)


@dataclasses.dataclass
class Wall:
    kind: int
    body: int = 0
    origin: tuple = (0.0, 0.0, 0.0)
    axis: tuple = (0.0, 0.0, 1.0)
    frame: tuple = (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0)
    dims: tuple = (0.0, 0.0, 0.0)
    mu_t: float = -1.0           # < 0: the bed's value
    mu_r: float = -1.0


@dataclasses.dataclass
class Body:
    origin: tuple = (0.0, 0.0, 0.0)
    lin_vel: tuple = (0.0, 0.0, 0.0)
    ang_vel: float = 0.0
    z_free: int = 0
    mass: float = 0.0


@dataclasses.dataclass
class BedSpec:
    pos: np.ndarray              # (n, 3) float64
    radius: np.ndarray           # (n,) float32
    vel: np.ndarray              # (n, 3) float32
    omega: np.ndarray            # (n, 3) float32
    box: tuple                   # (Lx, Ly, 0)
    periodic: int                # bit0 x, bit1 y
    params: Params
    walls: List[Wall]
    bodies: List[Body]
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.radius.shape[0])

    def copy(self) -> "BedSpec":
        return dataclasses.replace(
            self, pos=self.pos.copy(), radius=self.radius.copy(), vel=self.vel.copy(),
            omega=self.omega.copy(), walls=[dataclasses.replace(w) for w in self.walls],
            bodies=[dataclasses.replace(b) for b in self.bodies], info=dict(self.info))


# ---------------------------------------------------------------------------
# Profiles and the count model.

def graded_profile(r0: float, L: float, k: float, cap: float = 8.0):
    """Mean radius at depth d: r0 (1 + d/L)^k, capped at cap * r0."""
    def prof(d):
        d = np.maximum(np.asarray(d, dtype=np.float64), 0.0)
        return np.minimum(r0 * (1.0 + d / L) ** k, cap * r0)
    return prof


def linear_profile(d_min: float, gamma: float, d_max: float):
    """Eq. 1 of the paper as a radius profile: diameter d_min + gamma z up to d_max."""
    def prof(d):
        d = np.maximum(np.asarray(d, dtype=np.float64), 0.0)
        return 0.5 * np.minimum(d_min + gamma * d, d_max)
    return prof


def layer_profile(d0: float, ratio: float, eta: float, n_layers: int):
    """Discrete layers of the paper: d_n = ratio d_{n-1}, thickness eta d_n.

    Returns (d_n, z_n) with z_n the depth of the bottom of layer n, the
    geometric sum eta d0 (ratio^{n+1} - 1)/(ratio - 1)."""
    d = d0 * ratio ** np.arange(n_layers, dtype=np.float64)
    z = np.cumsum(eta * d)
    return d, z


def count_per_area(profile, depth: float, phi: float = PHI, samples: int = 20001) -> float:
    """Spheres per unit bed area between the surface and `depth`."""
    z = np.linspace(0.0, depth, samples)
    r = profile(z)
    dens = phi / ((4.0 / 3.0) * math.pi * EU3 * r ** 3)
    return float(np.trapezoid(dens, z))


def uniform_count(d: float, volume: float, phi: float = PHI) -> float:
    """Count of a uniform bed of mean diameter d filling `volume`."""
    return phi * volume / ((math.pi / 6.0) * EU3 * d ** 3)


def side_for_count(n: int, profile, depth: float) -> float:
    """Square periodic side that holds n spheres of the profile to `depth`."""
    return math.sqrt(n / count_per_area(profile, depth))


# ---------------------------------------------------------------------------
# Raft deposition.

_lib = None


def _bedgen():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "libbedgen.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        lib.bedgen_drop.restype = ctypes.c_int
        lib.bedgen_drop.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int32, ctypes.c_void_p]
        _lib = lib
    return _lib


class _Lattice:
    """Periodic hexagonal raft lattice with spacing >= 2 r_hi (1 + slack).

    Successive rafts on the same lattice alternate between the site set and
    the set of triangle centroids (ABAB stacking), so each sphere of a raft
    drops into a pocket of three spheres of the raft below; a new lattice
    (new spacing band) starts at a random offset."""

    def __init__(self, rng, Lx, Ly, r_hi, slack=0.05):
        a = 2.0 * r_hi * (1.0 + slack)
        self.nx = max(1, int(math.floor(Lx / a)))
        ny = int(math.floor(Ly / (a * math.sqrt(3.0) / 2.0)))
        ny -= ny % 2
        self.ny = max(ny, 1)
        self.ax, self.ay = Lx / self.nx, Ly / self.ny
        self.Lx, self.Ly = Lx, Ly
        self.r_hi = r_hi
        self.slack = slack
        self.ox, self.oy = rng.uniform(0, self.ax), rng.uniform(0, self.ay)
        self.parity = 0

    def raft(self, rng):
        ix, iy = np.meshgrid(np.arange(self.nx), np.arange(self.ny), indexing="xy")
        x = (ix + 0.5 * (iy % 2)) * self.ax + self.ox
        y = iy * self.ay + self.oy
        if self.parity:
            x = x + 0.5 * self.ax
            y = y + self.ay / 3.0
        self.parity ^= 1
        j = self.slack * self.r_hi / math.sqrt(2.0)
        x = np.mod(x.ravel() + rng.uniform(-j, j, x.size), self.Lx)
        y = np.mod(y.ravel() + rng.uniform(-j, j, y.size), self.Ly)
        return x, y


BAND = 1.1  # raft spacing is quantised to geometric bands of this ratio


def _band_radius(r_hi, r_base):
    b = math.floor(math.log(r_hi / r_base) / math.log(BAND) + 1e-9)
    return r_base * BAND ** (b + 1)


def deposit(rafts, Lx, Ly, rng, depth=4):
    """Drops rafts bottom-up.  rafts: list of (x, y, r) arrays."""
    x = np.concatenate([q[0] for q in rafts]).astype(np.float64)
    y = np.concatenate([q[1] for q in rafts]).astype(np.float64)
    r = np.concatenate([q[2] for q in rafts]).astype(np.float64)
    starts = np.zeros(len(rafts) + 1, dtype=np.int64)
    starts[1:] = np.cumsum([len(q[0]) for q in rafts])
    z = np.zeros_like(x)
    rc = _bedgen().bedgen_drop(len(x), x.ctypes.data, y.ctypes.data, r.ctypes.data, len(rafts),
                               starts.ctypes.data, Lx, Ly, depth, z.ctypes.data)
    if rc != 0:
        raise RuntimeError("bed deposition failed")
    return np.stack([x, y, z], axis=1)


def _raft_radii(rng, r_mean, count):
    return (r_mean * rng.uniform(1.0 - JITTER, 1.0 + JITTER, count)).astype(np.float32)


def _take(rng, x, y, count):
    if count >= len(x):
        return x, y
    idx = np.sort(rng.choice(len(x), size=count, replace=False))
    return x[idx], y[idx]


def layered_bed(layers, Lx, Ly, rng):
    """Bottom-up layers [(count, r_mean), ...] of rafts; returns (pos, radius)."""
    rafts = []
    for count, r_mean in layers:
        lat = _Lattice(rng, Lx, Ly, (1.0 + JITTER) * r_mean)
        left = count
        while left > 0:
            x, y = lat.raft(rng)
            x, y = _take(rng, x, y, left)
            rafts.append((x, y, _raft_radii(rng, r_mean, len(x))))
            left -= len(x)
    pos = deposit([(a, b, c.astype(np.float64)) for a, b, c in rafts], Lx, Ly, rng)
    radius = np.concatenate([q[2] for q in rafts]).astype(np.float32)
    return pos, radius


def profile_bed(n, profile, depth, Lx, Ly, rng):
    """n spheres graded by `profile` (mean radius vs depth), bottom-up rafts.
    A raft's depth is where the count model puts the spheres left to place."""
    area = Lx * Ly
    zs = np.linspace(0.0, depth * 1.5, 30001)
    r = profile(zs)
    dens = PHI / ((4.0 / 3.0) * math.pi * EU3 * r ** 3)
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(zs))]) * area
    r_base = float(np.min(r)) * (1.0 + JITTER) / BAND

    def depth_of(count_above):
        return float(np.interp(count_above, cum, zs))

    rafts = []
    placed = 0
    lat = None
    while placed < n:
        left = n - placed
        r_mean = float(profile(depth_of(left)))
        rb = _band_radius((1.0 + JITTER) * r_mean, r_base)
        if lat is None or abs(lat.r_hi - rb) > 1e-12 * rb:
            lat = _Lattice(rng, Lx, Ly, rb)
        per_raft = lat.nx * lat.ny
        r_mean = float(profile(depth_of(max(0.0, left - 0.5 * per_raft))))
        r_mean = min(r_mean, rb / (1.0 + JITTER))
        x, y = lat.raft(rng)
        x, y = _take(rng, x, y, left)
        rafts.append((x, y, _raft_radii(rng, r_mean, len(x))))
        placed += len(x)
    pos = deposit([(a, b, c.astype(np.float64)) for a, b, c in rafts], Lx, Ly, rng)
    radius = np.concatenate([q[2] for q in rafts]).astype(np.float32)
    return pos, radius


def _finish(pos, radius, box, periodic, params, walls, bodies, rng, shuffle, info):
    n = len(radius)
    if shuffle:
        perm = rng.permutation(n)
        pos, radius = pos[perm], radius[perm]
    return BedSpec(pos=np.ascontiguousarray(pos, dtype=np.float64),
                   radius=np.ascontiguousarray(radius, dtype=np.float32),
                   vel=np.zeros((n, 3), np.float32), omega=np.zeros((n, 3), np.float32),
                   box=tuple(box), periodic=periodic, params=params, walls=walls, bodies=bodies,
                   info=info)


# ---------------------------------------------------------------------------
# Walls and bodies.

def floor_wall(mu_t=-1.0, mu_r=-1.0) -> Wall:
    return Wall(kind=WALL_PLANE, body=0, origin=(0.0, 0.0, 0.0), axis=(0.0, 0.0, 1.0), mu_t=mu_t, mu_r=mu_r)


def surface_height(pos, radius, cx, cy, R, box):
    """Highest sphere top within horizontal distance R + r of (cx, cy)."""
    dx = pos[:, 0] - cx
    dy = pos[:, 1] - cy
    dx -= box[0] * np.round(dx / box[0])
    dy -= box[1] * np.round(dy / box[1])
    sel = np.hypot(dx, dy) < R + radius
    if not np.any(sel):
        return float(np.max(pos[:, 2] + radius))
    return float(np.max(pos[sel, 2] + radius[sel]))


def add_plate(spec: BedSpec, diameter=0.1, speed=0.01, full_width=False) -> BedSpec:
    """Flat rigid plate (one-sided disk facing down, or a full-width plane)
    starting at the highest sphere top under it, pushed down at `speed`."""
    Lx, Ly = spec.box[0], spec.box[1]
    cx, cy = 0.5 * Lx, 0.5 * Ly
    if full_width:
        z0 = float(np.max(spec.pos[:, 2] + spec.radius))
        wall = Wall(kind=WALL_PLANE, body=len(spec.bodies), origin=(0.0, 0.0, 0.0), axis=(0.0, 0.0, -1.0))
    else:
        z0 = surface_height(spec.pos, spec.radius, cx, cy, 0.5 * diameter, spec.box)
        wall = Wall(kind=WALL_DISK, body=len(spec.bodies), origin=(0.0, 0.0, 0.0), axis=(0.0, 0.0, -1.0),
                    dims=(0.5 * diameter, 0.0, 0.0))
    spec.bodies.append(Body(origin=(cx, cy, z0), lin_vel=(0.0, 0.0, -speed)))
    spec.walls.append(wall)
    spec.info["plate_body"] = len(spec.bodies) - 1
    return spec


def add_ring(spec: BedSpec, r_in=0.10, r_out=0.15, n_grousers=8, grouser_len=0.05,
             grouser_thick=0.009, grouser_depth=0.015, pressure=5.0e3, omega=0.5, g=9.81) -> BedSpec:
    """Grousered ring: annulus face plus radial grouser boxes below it, on a
    dead-weight body free in z, rotating at `omega` about +z."""
    Lx, Ly = spec.box[0], spec.box[1]
    cx, cy = 0.5 * Lx, 0.5 * Ly
    z0 = surface_height(spec.pos, spec.radius, cx, cy, r_out, spec.box) + grouser_depth
    mass = pressure * math.pi * (r_out ** 2 - r_in ** 2) / g
    b = len(spec.bodies)
    spec.bodies.append(Body(origin=(cx, cy, z0), ang_vel=omega, z_free=1, mass=mass))
    spec.walls.append(Wall(kind=WALL_ANNULUS, body=b, axis=(0.0, 0.0, -1.0), dims=(r_in, r_out, 0.0)))
    rm = 0.5 * (r_in + r_out)
    for q in range(n_grousers):
        phi = 2.0 * math.pi * q / n_grousers
        c, s = math.cos(phi), math.sin(phi)
        spec.walls.append(Wall(kind=WALL_BOX, body=b, origin=(rm * c, rm * s, -0.5 * grouser_depth),
                               frame=(c, s, 0.0, -s, c, 0.0, 0.0, 0.0, 1.0),
                               dims=(0.5 * grouser_len, 0.5 * grouser_thick, 0.5 * grouser_depth)))
    spec.info["plate_body"] = b
    return spec


# ---------------------------------------------------------------------------
# Workloads.

def two_layer_bed(seed=0, n_fine=1445, n_coarse=555, side=0.06, r_fine=1.5e-3, r_coarse=3.0e-3,
                  shuffle=True) -> BedSpec:
    """Two-layer bed: coarse spheres (3 mm) under a top layer of fine ones
    (1.5 mm), 0.06 m periodic square, floor wall; density 2600, mu_t 0.4."""
    rng = np.random.default_rng(seed)
    pos, radius = layered_bed([(n_coarse, r_coarse), (n_fine, r_fine)], side, side, rng)
    params = Params(rho=2600.0, mu_t=0.4, mu_r=0.02)
    return _finish(pos, radius, (side, side, 0.0), 3, params, [floor_wall()], [Body()], rng, shuffle,
                   {"workload": "two-layer", "seed": seed})


def graded_bed(n, r0=1.5e-3, L=0.02, k=1.0, cap=8.0, depth=0.2, side=None, seed=0, params=None,
               shuffle=True) -> BedSpec:
    """Graded bed of n spheres, r(d) = r0 (1 + d/L)^k capped at cap r0,
    depth `depth`; the periodic side follows from the count model unless given."""
    rng = np.random.default_rng(seed)
    prof = graded_profile(r0, L, k, cap)
    if side is None:
        side = side_for_count(n, prof, depth)
    pos, radius = profile_bed(n, prof, depth, side, side, rng)
    params = params if params is not None else paper_params()
    return _finish(pos, radius, (side, side, 0.0), 3, params, [floor_wall()], [Body()], rng, shuffle,
                   {"workload": "graded", "r0": r0, "L": L, "k": k, "cap": cap, "depth": depth,
                    "side": side, "seed": seed})


def uniform_bed(n, r=1.5e-3, depth=0.2, side=None, seed=0, params=None, shuffle=True) -> BedSpec:
    rng = np.random.default_rng(seed)
    prof = graded_profile(r, 1.0, 0.0, 1.0)
    if side is None:
        side = side_for_count(n, prof, depth)
    pos, radius = profile_bed(n, prof, depth, side, side, rng)
    params = params if params is not None else paper_params()
    return _finish(pos, radius, (side, side, 0.0), 3, params, [floor_wall()], [Body()], rng, shuffle,
                   {"workload": "uniform", "r": r, "depth": depth, "side": side, "seed": seed})


def jittered_lattice(n, r_mean, side, seed=0, params=None, shuffle=True) -> BedSpec:
    """Simple cubic lattice of spacing 2.2 r_mean with jitter, no overlaps."""
    rng = np.random.default_rng(seed)
    a = 2.0 * (1.0 + JITTER) * r_mean * 1.05
    m = max(1, int(side // a))
    layers = int(math.ceil(n / (m * m)))
    ix, iy, iz = np.meshgrid(np.arange(m), np.arange(m), np.arange(layers), indexing="ij")
    p = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], 1).astype(np.float64) * a
    order = np.lexsort((p[:, 0], p[:, 1], p[:, 2]))
    p = p[order][:n]
    j = 0.02 * r_mean
    p = p + rng.uniform(-j, j, p.shape)
    p[:, 0] = np.mod(p[:, 0] + 0.5 * a, side)
    p[:, 1] = np.mod(p[:, 1] + 0.5 * a, side)
    p[:, 2] += (1.0 + JITTER) * r_mean * 1.01
    radius = _raft_radii(rng, r_mean, n)
    params = params if params is not None else paper_params()
    return _finish(p, radius, (side, side, 0.0), 3, params, [floor_wall()], [Body()], rng, shuffle,
                   {"workload": "lattice", "seed": seed})


def random_cloud(n, side, height, r_min, r_max, seed=0, periodic=3, params=None, walls=None,
                 vel_scale=0.0, omega_scale=0.0, log_uniform=True) -> BedSpec:
    """Spheres at uniform random positions (overlaps allowed), radii spread
    between r_min and r_max: a stress input for contact detection."""
    rng = np.random.default_rng(seed)
    pos = np.stack([rng.uniform(0, side, n), rng.uniform(0, side, n), rng.uniform(0, height, n)], 1)
    if log_uniform:
        radius = np.exp(rng.uniform(math.log(r_min), math.log(r_max), n)).astype(np.float32)
    else:
        radius = rng.uniform(r_min, r_max, n).astype(np.float32)
    spec = BedSpec(pos=pos, radius=radius,
                   vel=(vel_scale * rng.standard_normal((n, 3))).astype(np.float32),
                   omega=(omega_scale * rng.standard_normal((n, 3))).astype(np.float32),
                   box=(side, side, 0.0), periodic=periodic,
                   params=params if params is not None else paper_params(),
                   walls=list(walls) if walls is not None else [], bodies=[Body()],
                   info={"workload": "cloud", "seed": seed})
    return spec


def metric_bed(n=2_000_000, seed=0) -> BedSpec:
    """The throughput workload: 2M spheres, r0 1.5 mm, L 20 mm, k = 1, cap
    8 r0, 0.2 m deep, periodic side from the count model, floor."""
    return graded_bed(n, r0=1.5e-3, L=0.02, k=1.0, cap=8.0, depth=0.2, seed=seed)


def batch_family(seed=0, depth=0.2, side=0.435, min_count=20_000, cap=8.0, plate=True):
    """The 36-bed family: full factorial r0 in {1.5, 2, 3} mm x L in {10, 20,
    40} mm x k in {0.5, 1, 1.5, 2}, depth 0.2 m, cap 8 r0, common periodic
    side 0.435 m; beds that would hold fewer than 20k spheres are widened to
    20k.  Each bed gets its own 0.1 m plate pushed at 0.01 m/s."""
    specs = []
    q = 0
    for r0 in (1.5e-3, 2.0e-3, 3.0e-3):
        for L in (0.01, 0.02, 0.04):
            for k in (0.5, 1.0, 1.5, 2.0):
                prof = graded_profile(r0, L, k, cap)
                n = int(round(side * side * count_per_area(prof, depth)))
                s = side
                if n < min_count:
                    n = min_count
                    s = side_for_count(n, prof, depth)
                spec = graded_bed(n, r0=r0, L=L, k=k, cap=cap, depth=depth, side=s, seed=seed * 1000 + q)
                if plate:
                    spec = add_plate(spec, diameter=0.1, speed=0.01)
                specs.append(spec)
                q += 1
    return specs
