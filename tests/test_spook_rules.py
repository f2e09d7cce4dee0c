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


def test_block_jacobi_sweeps_track_the_iteration_rule():
    """eq:Nit (written for the paper's Gauss-Seidel sweeps) against the
    oracle's block-Jacobi sweeps: columns of n_d spheres at the Hertz
    equilibrium, started from zero impulses, reach 1 % error in the floor
    force within twice N_it = 0.1 n_d / 0.01, and need more sweeps as the
    column grows."""
    from oracle import oracle as O
    from paper_2501_05300_amd import beds
    from test_oracle_pins import make_spec
    prm = beds.Params(rho=2600.0, dt=1e-4)
    Estar = prm.E / (2 * (1 - prm.nu ** 2))
    r = float(np.float32(1.5e-3))
    m = prm.rho * 4 / 3 * math.pi * r ** 3
    needed = []
    for n in (4, 8, 16):
        load = m * 9.81 * np.arange(n, 0, -1)
        z = [r - (load[0] / (Estar * math.sqrt(2 * r) / 3)) ** (2 / 3)]
        for i in range(1, n):
            z.append(z[-1] + 2 * r - (load[i] / (Estar * math.sqrt(r) / 3)) ** (2 / 3))
        spec = make_spec([[0.01, 0.01, zz] for zz in z], [r] * n, params=prm, walls=[beds.floor_wall()],
                         box=(1, 1, 0))
        for N in (2 ** k for k in range(13)):
            b = O.OracleBed(spec)
            b.set_stepper("spook", N)
            b.step(1)
            if abs(-b.last_reaction(0)[2] - load[0]) < 0.01 * load[0]:
                break
        needed.append(N)
        assert N <= 2 * R.iterations(n, 0.01), (n, N)
    assert needed[0] < needed[1] < needed[2]
