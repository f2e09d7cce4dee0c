"""The time-implicit step's guiding rules (eq:Nit, eq:timestep,
eq:contact_network) against the paper's own statements and tables (CPU)."""
import math

import numpy as np

from paper_2501_05300_amd import spook_rules as R


def test_general_timestep_reduces_to_the_uniform_rule():
    """With a = 3 sigma / (2 rho d), (1/2) sqrt(eps d / a) is the uniform-bed
    form d sqrt(eps rho / (6 sigma)) the paper states."""
    for eps, d, sigma, rho in ((0.02, 8.5e-3, 5e4, 2200.0), (0.005, 0.03, 1e3, 2600.0)):
        assert math.isclose(R.timestep(eps, d, sigma, rho), d * math.sqrt(eps * rho / (6 * sigma)), rel_tol=1e-14)


def test_uniform_table_fits_one_tolerance_and_stress():
    """Table tab:bed-configurations-uniform (d = 8.5, 15, 22.5, 30 mm; dt =
    0.10, 0.18, 0.25, 0.35 ms; N_it = 375, 225, 175, 125): one ratio eps/sigma
    reproduces every dt within 6 %, and with the 600 mm bed (n_d = h/d, the
    bed depth the discussion section uses) one eps reproduces every N_it
    within 15 %, the table's rounding."""
    d = np.array([8.5, 15.0, 22.5, 30.0]) * 1e-3
    dt = np.array([0.10, 0.18, 0.25, 0.35]) * 1e-3
    nit = np.array([375, 225, 175, 125])
    rho, h = 2200.0, 0.6
    ratio = np.median((dt / d) ** 2 * 6 / rho)           # eps / sigma
    eps = np.median(0.1 * (h / d) / nit)
    for k in range(4):
        sigma = eps / ratio
        assert abs(R.timestep(eps, d[k], sigma, rho) / dt[k] - 1) < 0.06
        assert abs(R.iterations(R.contact_network_uniform(h, d[k]), eps) / nit[k] - 1) < 0.15
    assert 0.01 < eps < 0.03


def test_graded_network_counts_the_layers():
    """eq:contact_network against a direct walk down the layer construction:
    layer n has diameter r^n d_min and thickness eta d_n, so it is eta
    particles high; below the last refined layer the bed is uniform at d_max."""
    for d_min, L, r, eta, h in ((8.5e-3, 5, 1.25, 2.0, 0.6), (8.5e-3, 6, 1.1, 1.5, 0.6), (1.5e-3, 3, 2.0, 3.0, 0.2)):
        d_max = d_min * r ** L
        z, n_d, dn = 0.0, 0.0, d_min
        for _ in range(L):
            z += eta * dn
            n_d += eta
            dn *= r
        n_d += (h - z) / d_max
        assert math.isclose(R.contact_network_graded(d_min, d_max, r, eta, h), n_d, rel_tol=1e-12)


def test_refined_beds_need_fewer_iterations():
    """The point of the rule for refined beds: a bed refined from d_min to
    d_max has a shorter contact network than a uniform bed of d_min, so
    fewer iterations (the paper's 215-275 against 375 at 8.5 mm)."""
    eps, h = 0.018, 0.6
    uni = R.iterations(R.contact_network_uniform(h, 8.5e-3), eps)
    for d_max in (15e-3, 22.5e-3, 30e-3):
        gr = R.iterations(R.contact_network_graded(8.5e-3, d_max, 1.2, 2.0, h), eps)
        assert gr < uni
