"""Edge cases of the HIP stepper: a lone sphere, rejected descriptions, a
particle with more partners than slots and one with exactly as many, cells
too crowded for the search's row table, coincident spheres, and closed-form
motion on an incline and of a stuck contact (GPU)."""
import math

import numpy as np
import pytest

from paper_2501_05300_amd import beds
from parity_util import assert_parity, compare_one_step

pytestmark = pytest.mark.gpu


def spec_of(pos, radius, box=(0.1, 0.1, 0.0), periodic=3, params=None, walls=None, bodies=None):
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    n = pos.shape[0]
    return beds.BedSpec(pos=pos, radius=np.asarray(radius, np.float32).reshape(n), vel=np.zeros((n, 3), np.float32),
                        omega=np.zeros((n, 3), np.float32), box=box, periodic=periodic,
                        params=params if params is not None else beds.paper_params(), walls=walls or [],
                        bodies=bodies or [beds.Body()])


def test_lone_sphere_falls_freely():
    """No contacts: velocity-then-position Euler gives v_k = k dt g and
    z_k = z_0 + dt^2 g k (k + 1) / 2 (FP32 velocity, FP64 position)."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = spec_of([[0.05, 0.05, 0.5]], [2e-3])
    bed = Bed(spec)
    k = 1000
    bed.step(k)
    x, v, _ = bed.state()
    dt, g = spec.params.dt, spec.params.g[2]
    vz = k * dt * g
    dz = dt * dt * g * k * (k + 1) / 2
    assert abs(v[0, 2] - vz) <= 1e-4 * abs(vz)  # k FP32 additions
    assert abs((x[0, 2] - 0.5) - dz) <= 1e-4 * abs(dz)
    assert x[0, 0] == 0.05 and x[0, 1] == 0.05
    assert bed.contacts().shape[0] == 0


@pytest.mark.parametrize("case", ["empty", "negative_radius", "nan_position", "short_period", "cadence_without_skin",
                                  "band_ratio", "block"])
def test_invalid_descriptions_are_rejected(case):
    from paper_2501_05300_amd.lprdem import Bed, LprError
    kw = {}
    spec = spec_of([[0.05, 0.05, 0.01], [0.06, 0.05, 0.01]], [2e-3, 2e-3])
    if case == "empty":
        spec = spec_of(np.zeros((0, 3)), np.zeros(0))
    elif case == "negative_radius":
        spec.radius[1] = -1e-3
    elif case == "nan_position":
        spec.pos[0, 2] = float("nan")
    elif case == "short_period":
        spec.box = (0.005, 0.1, 0.0)  # must exceed 2 (r_i + r_j)
    elif case == "cadence_without_skin":
        kw = dict(rebuild_every=4, skin=0.0)
    elif case == "band_ratio":
        kw = dict(band_ratio=1.0)
    elif case == "block":
        kw = dict(block=100)
    with pytest.raises(LprError) as e:
        Bed(spec, **kw)
    assert e.value.status == -1


def test_more_partners_than_slots_latches_capacity():
    """A 1 mm sphere overlapped by 20 spheres of 2 mm owns all 20 pairs (the
    smaller radius owns), more than its 16 slots: the step reports the
    capacity fault and the bed stays latched."""
    from paper_2501_05300_amd.lprdem import Bed, CapacityError, LprError
    c = np.array([0.05, 0.05, 0.05])
    golden = math.pi * (3.0 - math.sqrt(5.0))
    pts = []
    for q in range(20):  # Fibonacci points on a sphere of radius 2.9 mm
        z = 1.0 - 2.0 * (q + 0.5) / 20
        rr = math.sqrt(1.0 - z * z)
        pts.append(c + 2.9e-3 * np.array([rr * math.cos(golden * q), rr * math.sin(golden * q), z]))
    spec = spec_of([c] + pts, [1e-3] + [2e-3] * 20, params=beds.paper_params(E=1e6))
    bed = Bed(spec)
    bed.step(1)
    with pytest.raises(CapacityError):
        bed.sync()
    with pytest.raises(LprError):
        bed.step(1)
        bed.sync()
    x, _, _ = bed.state()  # the state stays readable
    assert np.all(np.isfinite(x))


def test_exactly_as_many_partners_as_slots():
    """A 1 mm sphere overlapped by 16 spheres of 2 mm owns exactly its 16
    slots: no capacity fault, and the step matches the oracle (the larger
    spheres also press into one another)."""
    from paper_2501_05300_amd.lprdem import Bed
    c = np.array([0.05, 0.05, 0.05])
    golden = math.pi * (3.0 - math.sqrt(5.0))
    pts = []
    for q in range(16):  # Fibonacci points on a sphere of radius 2.9 mm
        z = 1.0 - 2.0 * (q + 0.5) / 16
        rr = math.sqrt(1.0 - z * z)
        pts.append(c + 2.9e-3 * np.array([rr * math.cos(golden * q), rr * math.sin(golden * q), z]))
    spec = spec_of([c] + pts, [1e-3] + [2e-3] * 16, params=beds.paper_params(E=1e6))
    bed = Bed(spec, record_forces=True)
    res = compare_one_step(spec, bed)
    bed.sync()  # raises if a fault latched
    print({k: v for k, v in res.items() if k not in ("only_gpu", "only_oracle")})
    assert_parity(res, 1e-5)
    got = bed.contacts()
    assert int(np.sum(got[:, 0] == 0)) == 16  # stable id 0 is the small sphere
    # from rest there is no tangential motion, so the torques vanish up to
    # rounding: compare them with the force scale times the lever arm
    F, T = bed.forces()
    assert float(np.abs(T).max()) <= 1e-5 * float(np.abs(F).max()) * 2e-3


def test_crowded_cells_take_the_exact_walk():
    """One radius band spanning a factor 8 (band ratio 8): a cell of the
    2.2 mm spheres' size holds hundreds of 0.3 mm spheres, so every row of
    cells is longer than the search's packed row table takes and every lane
    walks the FP64 records instead; the large spheres also collect hundreds
    of partner-side entries.  Contacts, forces and torques match the oracle."""
    import numpy as np
    from paper_2501_05300_amd.lprdem import Bed
    rng = np.random.default_rng(11)
    n_small, n_large, side, height = 8000, 6, 0.012, 0.008
    pos = np.stack([rng.uniform(0, side, n_small + n_large), rng.uniform(0, side, n_small + n_large),
                    rng.uniform(0, height, n_small + n_large)], 1)
    radius = np.concatenate([rng.uniform(0.28e-3, 0.32e-3, n_small), np.full(n_large, 2.2e-3)])
    spec = spec_of(pos, radius, box=(side, side, 0.0), periodic=3, params=beds.paper_params(E=1e6))
    bed = Bed(spec, record_forces=True, band_ratio=8.0)
    res = compare_one_step(spec, bed)
    bed.sync()
    print({k: v for k, v in res.items() if k not in ("only_gpu", "only_oracle")})
    assert_parity(res, 1e-5)
    got = bed.contacts()
    large = np.arange(n_small, n_small + n_large)
    assert int(np.isin(got[:, 1], large).sum()) > 100 * n_large  # long partner-side lists
    # from rest the torques vanish up to rounding (see above)
    F, T = bed.forces()
    assert float(np.abs(T).max()) <= 1e-5 * float(np.abs(F).max()) * 2.2e-3


def test_coincident_spheres_match_oracle():
    """d = 0: the pair's normal is +z (the reading for a degenerate
    direction); the force on the pair and a third, ordinary contact match
    the oracle."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = spec_of([[0.05, 0.05, 0.05], [0.05, 0.05, 0.05], [0.0535, 0.05, 0.05]], [2e-3, 2e-3, 1.5e-3],
                   params=beds.paper_params(E=1e6))
    bed = Bed(spec, record_forces=True)
    res = compare_one_step(spec, bed)
    print(res)
    assert_parity(res, 1e-5)
    assert res["n_contacts"] == 3
    F, _ = bed.forces()
    # stable id 0 owns the coincident pair (equal radii, smaller id) and is
    # pushed along -n = -z, its partner along +z
    assert F[0, 2] < 0 < F[1, 2]


@pytest.mark.parametrize("mu,rolls", [(0.5, True), (0.05, False)])
def test_explicit_step_on_an_incline_on_the_gpu(mu, rolls):
    """The tilted-plane closed forms through the HIP explicit step (rolling
    without slip at (5/7) g sin theta, sliding at g (sin theta - mu cos theta))."""
    import math
    from paper_2501_05300_amd.lprdem import Bed
    from test_oracle_spook import incline
    theta = math.radians(20.0)
    spec, down = incline(theta, mu, dt=2e-6)
    bed = Bed(spec)
    bed.step(5000)
    a = float(bed.state()[1][0].astype(np.float64) @ down) / (5000 * 2e-6)
    ref = (5.0 / 7.0) * 9.81 * math.sin(theta) if rolls else 9.81 * (math.sin(theta) - mu * math.cos(theta))
    assert abs(a / ref - 1.0) < 1e-3, (a, ref)


def test_stuck_contact_vibrates_with_the_spring_stiffnesses_on_the_gpu():
    """A sphere resting on the floor, nudged sideways with friction too high
    to slip and no damping, through the HIP step: it follows the
    two-degree-of-freedom oscillator that the tangential spring
    k_t = kappa_t dF_n/d(delta) at the lever r - delta/2 and the rolling
    spring k_r = k_t r^2 make, iterated here on its own (FP32 law and
    velocities: to 2e-3 of the initial speed over 13 periods)."""
    from paper_2501_05300_amd.lprdem import Bed
    prm = beds.Params(rho=2600.0, mu_t=10.0, mu_r=10.0, gamma_factor=0.0, dt=2e-6)
    r = float(np.float32(1.5e-3))
    m = prm.rho * 4.0 / 3.0 * math.pi * r ** 3
    inertia = 0.4 * m * r * r
    kn = prm.E / (2 * (1 - prm.nu ** 2)) * math.sqrt(2 * r) / 3.0
    dstat = (m * 9.81 / kn) ** (2.0 / 3.0)
    spec = spec_of([[0.01, 0.01, r - dstat]], [r], box=(1.0, 1.0, 0.0), periodic=0, params=prm,
                   walls=[beds.floor_wall()])
    spec.vel[0, 0] = 1e-4
    bed = Bed(spec)
    p0, v0, w0 = bed.state()
    delta = r - float(p0[0, 2])
    kt = prm.kappa() * 1.5 * kn * math.sqrt(delta)
    kr = kt * r * r
    la = r - 0.5 * delta
    dt = prm.dt
    v, w, xt, xr = float(v0[0, 0]), float(w0[0, 1]), 0.0, 0.0
    dv, dw, vmin = 0.0, 0.0, 0.0
    for _ in range(2000):
        bed.step(1)
        xt += dt * (v - la * w)
        xr += dt * w
        F = -kt * xt
        tq = -la * F - kr * xr
        v += dt * F / m
        w += dt * tq / inertia
        _, vg, wg = bed.state()
        dv = max(dv, abs(float(vg[0, 0]) - v))
        dw = max(dw, abs(float(wg[0, 1]) - w))
        vmin = min(vmin, v)
    assert vmin < -0.5e-4
    assert dv < 2e-3 * 1e-4, dv
    assert dw < 2e-3 * 1e-4 / r, dw


def test_sphere_through_the_floor_latches():
    """A sphere whose centre is set below the floor by more than its radius
    has tunnelled: the step latches LPR_E_DOMAIN, reported at lpr_sync; the
    state stays readable at the last complete step."""
    from paper_2501_05300_amd.lprdem import Bed, LprError
    spec = spec_of([[0.05, 0.05, 0.002], [0.02, 0.02, 0.002]], [2e-3, 2e-3], walls=[beds.floor_wall()])
    bed = Bed(spec)
    bed.step(5)
    bed.sync()
    x, v, w = bed.state()
    x[1, 2] = -0.0025
    bed.set_state(x, v, w)
    bed.step(3)
    with pytest.raises(LprError) as e:
        bed.sync()
    assert e.value.status == -7
    x2, _, _ = bed.state()
    assert x2[1, 2] == -0.0025   # no step completed after the set
    with pytest.raises(LprError):
        bed.step(1)


def test_sphere_outside_its_level_grid_is_counted_and_still_found():
    """A sphere thrown far above the planned extent of its level's grid is
    binned into the edge cell: the step still matches the oracle, and the
    binning is counted."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = beds.add_plate(beds.two_layer_bed(41), diameter=0.04, speed=0.5)
    bed = Bed(spec, record_forces=True)
    bed.step(100)
    x, v, w = bed.state()
    # two spheres high above the bed, overlapping slightly
    reach = 0.98 * float(spec.radius[0] + spec.radius[1])
    x[0] = (0.03, 0.03, 0.5)
    x[1] = (0.03 + reach, 0.03, 0.5)
    bed.set_state(x, v, w)
    res = compare_one_step(spec, bed)
    print({k: v for k, v in res.items() if k not in ("only_gpu", "only_oracle")})
    assert_parity(res, 1e-5)
    assert (0, 1) in set(map(tuple, bed.contacts().tolist()))
    assert bed.stats()["outside_grid"] >= 2
