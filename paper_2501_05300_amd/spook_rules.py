"""Guiding rules of the time-implicit step (section "Nonsmooth DEM and
multibody dynamics", eq:Nit, eq:timestep and eq:contact_network).

The projected iterations need more sweeps the longer the contact network in
the direction of the dominant stress, and the step is limited by the largest
acceleration a contact force can give a particle, not by the contact period.
These helpers turn a bed's sizes into an iteration count and a time step
(host logic; the step itself runs in the HIP library)."""
from __future__ import annotations

import math


def iterations(n_d: float, eps: float) -> int:
    """eq:Nit: N_it = 0.1 n_d / eps, rounded up; n_d is the contact-network
    length (particles along the dominant stress), eps the error tolerance."""
    return max(1, math.ceil(0.1 * n_d / eps))


def timestep(eps: float, d: float, sigma: float, rho: float) -> float:
    """eq:timestep: dt = (1/2) sqrt(eps d / a), with the largest acceleration
    estimated as a = sigma A / m = 3 sigma / (2 rho d) for a sphere of
    diameter d and density rho under normal stress sigma."""
    a = 3.0 * sigma / (2.0 * rho * d)
    return 0.5 * math.sqrt(eps * d / a)


def contact_network_uniform(h: float, d: float) -> float:
    """n_d = h / d for a uniform bed of height h."""
    return h / d


def contact_network_graded(d_min: float, d_max: float, r: float, eta: float, h: float) -> float:
    """eq:contact_network: n_d = eta log(d_max / d_min) / log r + (h - z_max) / d_max
    for a bed refined in layers of diameter d_n = r^n d_min and thickness
    eta d_n (section "Local particle refinement and scaling agressiveness"),
    uniform at d_max below z_max = eta d_min (r^L - 1) / (r - 1), where L =
    log(d_max / d_min) / log r is the number of refined layers."""
    L = math.log(d_max / d_min) / math.log(r)
    z_max = eta * d_min * (r ** L - 1.0) / (r - 1.0)
    return eta * L + (h - z_max) / d_max
