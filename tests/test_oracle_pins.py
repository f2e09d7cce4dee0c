"""Pins of the FP64 oracle to results fixed outside it (CPU only).

Each test checks the oracle against something other than its own formulas:
brute-force geometry, an independent neighbour library, closed-form contact
mechanics, conservation laws, and printed values from the paper.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import oracle as O
from paper_2501_05300_amd import beds

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def make_spec(pos, rad, vel=None, omg=None, box=(1.0, 1.0, 0.0), periodic=0, params=None, walls=(),
              bodies=None):
    n = len(rad)
    return beds.BedSpec(pos=np.ascontiguousarray(pos, np.float64), radius=np.asarray(rad, np.float32),
                        vel=np.zeros((n, 3), np.float32) if vel is None else np.asarray(vel, np.float32),
                        omega=np.zeros((n, 3), np.float32) if omg is None else np.asarray(omg, np.float32),
                        box=box, periodic=periodic, params=params or beds.paper_params(), walls=list(walls),
                        bodies=bodies or [beds.Body()])


def pairs_set(a):
    return set(map(tuple, np.asarray(a).tolist()))


# ---------------------------------------------------------------------------
# P-1: the contact set


@pytest.mark.parametrize("periodic,side", [(3, 0.05), (0, 0.05), (1, 0.05), (3, 0.021)])
def test_grid_equals_brute_force(periodic, side):
    spec = beds.random_cloud(1500, side, 0.04, 0.5e-3, 5e-3, seed=periodic + int(side * 1e3), periodic=periodic)
    b = O.OracleBed(spec)
    brute = b.contact_set(0)
    grid = b.contact_set(1)
    assert len(brute) > 100
    np.testing.assert_array_equal(brute, grid)


def test_contact_set_matches_independent_kdtree():
    """scipy's periodic k-d tree gives the same pairs (ties excluded)."""
    side, height = 0.04, 0.03
    spec = beds.random_cloud(2000, side, height, 0.4e-3, 4e-3, seed=7, periodic=3)
    b = O.OracleBed(spec)
    got = pairs_set(b.contact_set(0))
    p = spec.pos
    r = spec.radius.astype(np.float64)
    tree = cKDTree(np.c_[p[:, 0], p[:, 1], p[:, 2]], boxsize=[side, side, 100.0])
    cand = tree.query_pairs(2 * r.max(), output_type="ndarray")
    d = p[cand[:, 0]] - p[cand[:, 1]]
    d[:, :2] -= side * np.round(d[:, :2] / side)
    dist = np.linalg.norm(d, axis=1)
    R = r[cand[:, 0]] + r[cand[:, 1]]
    ok = np.abs(dist - R) > 1e-12 * R
    ref = set()
    for (i, j), c in zip(cand[ok], (dist < R)[ok]):
        if c:
            a, bb = (i, j) if (r[i], i) < (r[j], j) else (j, i)
            ref.add((int(a), int(bb)))
    ties = {(min(i, j), max(i, j)) for i, j in cand[~ok].tolist()}
    got_noties = {q for q in got if (min(q), max(q)) not in ties}
    assert len(ref) > 500
    assert got_noties == ref


def test_touching_spheres_are_not_in_contact():
    """Contact needs a strictly positive overlap: exactly touching spheres
    (d = r_i + r_j, all values exact binary fractions) are apart, and moving
    one sphere by one ulp closer makes them touch."""
    rad = [0.5, 0.5]
    box = (8.0, 8.0, 0.0)
    for periodic in (0, 3):
        spec = make_spec([[2.0, 2.0, 2.0], [3.0, 2.0, 2.0]], rad, box=box, periodic=periodic)
        assert len(O.OracleBed(spec).contact_set(0)) == 0
        spec = make_spec([[2.0, 2.0, 2.0], [np.nextafter(3.0, 0.0), 2.0, 2.0]], rad, box=box, periodic=periodic)
        assert pairs_set(O.OracleBed(spec).contact_set(0)) == {(0, 1)}
    # across the periodic seam: image distance exactly 1 -> apart; 1 - ulp -> contact
    spec = make_spec([[0.25, 2.0, 2.0], [7.25, 2.0, 2.0]], rad, box=box, periodic=1)
    assert len(O.OracleBed(spec).contact_set(0)) == 0
    spec = make_spec([[0.25, 2.0, 2.0], [np.nextafter(7.25, 8.0), 2.0, 2.0]], rad, box=box, periodic=1)
    assert pairs_set(O.OracleBed(spec).contact_set(0)) == {(0, 1)}


def test_owner_is_smaller_radius_then_id():
    spec = make_spec([[0.1, 0.1, 0.1], [0.1009, 0.1, 0.1], [0.1, 0.1016, 0.1]], [1e-3, 0.5e-3, 1e-3])
    cs = pairs_set(O.OracleBed(spec).contact_set(0))
    assert cs == {(1, 0), (0, 2)}


def test_wall_contacts_follow_the_signed_distance():
    p = beds.paper_params()
    walls = [beds.floor_wall(),
             beds.Wall(kind=beds.WALL_DISK, body=1, axis=(0, 0, -1), dims=(0.01, 0, 0)),
             beds.Wall(kind=beds.WALL_BOX, body=1, origin=(0.03, 0.0, 0.0), dims=(0.002, 0.002, 0.002))]
    bodies = [beds.Body(), beds.Body(origin=(0.05, 0.05, 0.02))]
    pos = [[0.2, 0.2, 0.0009],     # floor: z < r -> contact
           [0.3, 0.3, float(np.float32(1e-3))],  # floor: z == r -> no contact
           [0.05, 0.05, 0.0191],   # disk face from below
           [0.052, 0.052, 0.0209], # above the disk (back side) -> no
           [0.0605, 0.05, 0.0195], # disk rim
           [0.08, 0.05, 0.02],     # box centre inside -> contact
           [0.0829, 0.05, 0.02]]   # box face at distance 0.0009 < r
    spec = make_spec(pos, [1e-3] * len(pos), box=(1, 1, 0), walls=walls, bodies=bodies, params=p)
    cs = pairs_set(O.OracleBed(spec).contact_set(0))
    assert cs == {(0, -1), (2, -2), (4, -2), (5, -3), (6, -3)}


# ---------------------------------------------------------------------------
# P-2, P-3: two-sphere collisions against closed forms


def _collide(params, r=1.5e-3, v0=0.1, steps=400):
    """Head-on collision of two equal spheres; returns the overlap history and
    the final relative velocity."""
    pos = [[0.1, 0.1, 0.1], [0.1 + 2 * r + 1e-9, 0.1, 0.1]]
    vel = [[0.5 * v0, 0, 0], [-0.5 * v0, 0, 0]]
    spec = make_spec(pos, [r, r], vel=vel, params=params)
    b = O.OracleBed(spec)
    dl = []
    for _ in range(steps):
        b.step(1)
        x, v, _ = b.state()
        dl.append(2 * float(np.float32(r)) - np.linalg.norm(x[1] - x[0]))
        if dl[-1] < -1e-7 and len(dl) > 10:
            break
    return np.array(dl), v[0, 0] - v[1, 0]


def test_hertz_impact_closed_form():
    """Undamped Hertz impact: delta_max = (5 m* v0^2 / (4 k_n))^(2/5) and
    contact time 2.94328 delta_max / v0, restitution 1."""
    prm = beds.Params(rho=2600.0, mu_t=0.0, mu_r=0.0, gamma_factor=0.0, g=(0.0, 0.0, 0.0))
    r = float(np.float32(1.5e-3))
    Estar = prm.E / (2 * (1 - prm.nu ** 2))
    kn = Estar * math.sqrt(r) / 3.0      # d* = r for equal spheres of radius r
    mstar = 0.5 * prm.rho * 4.0 / 3.0 * math.pi * r ** 3
    v0 = 0.1
    dmax = (5 * mstar * v0 ** 2 / (4 * kn)) ** 0.4
    tc = 2.94328 * dmax / v0
    assert abs(dmax - 4.1360e-6) < 2e-9
    errs = []
    for dt in (2e-6, 1e-6):
        dl, vrel = _collide(prm.replace(dt=dt), r=r, v0=v0, steps=int(4 * tc / dt))
        errs.append(abs(dl.max() - dmax) / dmax)
        steps_in_contact = int(np.sum(dl > 0))
        assert abs(steps_in_contact * dt - tc) <= 2.5 * dt
        assert abs(abs(vrel) / v0 - 1.0) < 5e-3
    assert errs[0] < 5e-3
    assert errs[1] < 0.6 * errs[0] + 1e-5


def test_linear_damped_contact_closed_form():
    """e_H = 1: m* delta'' = -k_n (delta + gamma_n delta'), so delta(t) =
    (v0/w_d) exp(-zeta w0 t) sin(w_d t) while the force stays positive."""
    v0 = 0.1
    r = float(np.float32(1.5e-3))
    errs = []
    for dt in (1e-6, 5e-7):
        prm = beds.Params(rho=2600.0, E=1e6, mu_t=0.0, mu_r=0.0, e_H=1.0, g=(0, 0, 0), dt=dt)
        Estar = prm.E / (2 * (1 - prm.nu ** 2))
        kn = Estar * math.sqrt(r) / 3.0
        mstar = 0.5 * prm.rho * 4.0 / 3.0 * math.pi * r ** 3
        w0 = math.sqrt(kn / mstar)
        zeta = 0.2
        gn = 2 * zeta / w0
        prm = prm.replace(gamma_factor=gn / dt)
        wd = w0 * math.sqrt(1 - zeta ** 2)
        dl, _ = _collide(prm, r=r, v0=v0, steps=int(2 * math.pi / wd / dt))
        t = dt * np.arange(1, len(dl) + 1)
        exact = (v0 / wd) * np.exp(-zeta * w0 * t) * np.sin(wd * t)
        force_pos = (exact + gn * np.gradient(exact, t)) > 0
        sel = (dl > 0) & force_pos
        sel[: 3] = False
        errs.append(np.max(np.abs(dl[sel] - exact[sel])) / exact.max())
    assert errs[0] < 0.02
    assert errs[1] < 0.6 * errs[0]


# ---------------------------------------------------------------------------
# P-4, P-5: a sphere on the floor (textbook rigid-body results)


def _sphere_on_floor(mu_t, mu_r, v0, w0, steps, dt=2e-6, sample_every=1):
    prm = beds.Params(rho=2600.0, mu_t=mu_t, mu_r=mu_r, dt=dt)
    r = float(np.float32(1.5e-3))
    m = prm.rho * 4.0 / 3.0 * math.pi * r ** 3
    Estar = prm.E / (2 * (1 - prm.nu ** 2))
    kn = Estar * math.sqrt(2 * r) / 3.0
    dstat = (m * 9.81 / kn) ** (2.0 / 3.0)
    spec = make_spec([[0.01, 0.01, r - dstat]], [r], vel=[[v0, 0, 0]], omg=[[0, w0, 0]], params=prm,
                     walls=[beds.floor_wall()], box=(1, 1, 0))
    b = O.OracleBed(spec)
    vs, ws = [], []
    for _ in range(steps // sample_every):
        b.step(sample_every)
        _, v, w = b.state()
        vs.append(v[0, 0]); ws.append(w[0, 1])
    return np.array(vs), np.array(ws), r


def test_sliding_sphere_starts_rolling_at_textbook_time():
    """Coulomb sliding: rolling starts at t* = 2 v0 / (7 mu g) with v = 5 v0 / 7."""
    mu, v0, dt = 0.4, 0.1, 2e-6
    vs, ws, r = _sphere_on_floor(mu, 0.0, v0, 0.0, 5000, dt=dt)
    slip = vs - r * ws
    tstar = 2 * v0 / (7 * mu * 9.81)
    assert abs(tstar - 7.2812e-3) < 1e-6
    k = int(np.argmax(slip < 1e-3 * v0))
    assert abs((k + 1) * dt - tstar) < 0.01 * tstar
    assert abs(vs[-1] - 5 * v0 / 7) < 2e-3 * v0


def test_rolling_resistance_deceleration():
    """Rolling under a rolling-resistance moment at its cap mu_r r m g:
    a = -(5/7) mu_r g."""
    mu_r, v0 = 0.02, 0.05
    vs, ws, r = _sphere_on_floor(0.4, mu_r, v0, v0 / 1.5e-3, 6000)
    t = 2e-6 * np.arange(len(vs))
    sel = t > 2e-3
    a = np.polyfit(t[sel], vs[sel], 1)[0]
    assert abs(a - (-(5.0 / 7.0) * mu_r * 9.81)) < 0.01 * (5.0 / 7.0) * mu_r * 9.81


def test_stuck_contact_vibrates_with_the_spring_stiffnesses():
    """A sphere resting on the floor is nudged sideways, with friction high
    enough that its springs never slip and no damping.  The tangential spring
    k_t = kappa_t dF_n/d(delta) (kappa_t the Mindlin ratio 2(1 - nu)/(2 - nu)
    of the material's nu) at the contact point, a lever r - delta/2 below the
    centre, and the rolling spring k_r = k_t r*^2 (r* = r on a wall) make a
    two-degree-of-freedom oscillator of the centre and the rotation.  Its
    step-by-step solution (springs advanced by the contact-point and relative
    angular velocities, then velocities, then positions) is iterated here on
    its own; a wrong stiffness, lever, torque sign or inertia changes its
    frequencies, so the oracle would drift away from it within a period."""
    prm = beds.Params(rho=2600.0, mu_t=10.0, mu_r=10.0, gamma_factor=0.0, dt=2e-6)
    r = float(np.float32(1.5e-3))
    m = prm.rho * 4.0 / 3.0 * math.pi * r ** 3
    inertia = 0.4 * m * r * r
    Estar = prm.E / (2 * (1 - prm.nu ** 2))
    kn = Estar * math.sqrt(2 * r) / 3.0
    dstat = (m * 9.81 / kn) ** (2.0 / 3.0)
    spec = make_spec([[0.01, 0.01, r - dstat]], [r], vel=[[1e-4, 0, 0]], params=prm,
                     walls=[beds.floor_wall()], box=(1, 1, 0))
    b = O.OracleBed(spec)
    p0, v0, w0 = b.state()
    delta = r - p0[0, 2]
    kt = prm.kappa() * 1.5 * kn * math.sqrt(delta)  # e_H = 5/4: F_n = k_n delta^(3/2)
    kr = kt * r * r
    la = r - 0.5 * delta
    dt = prm.dt
    v, w, xt, xr = float(v0[0, 0]), float(w0[0, 1]), 0.0, 0.0
    vmax, wmax, vmin = 0.0, 0.0, 0.0
    for _ in range(2000):
        b.step(1)
        xt += dt * (v - la * w)      # contact point slides with v - la w
        xr += dt * w
        F = -kt * xt
        tq = -la * F - kr * xr       # lever below the centre, rolling moment
        v += dt * F / m
        w += dt * tq / inertia
        _, vo, wo = b.state()
        vmax = max(vmax, abs(vo[0, 0] - v))
        wmax = max(wmax, abs(wo[0, 1] - w))
        vmin = min(vmin, v)
    assert vmin < -0.5e-4               # the motion reverses: a real oscillation
    assert vmax < 1e-6 * 1e-4
    assert wmax < 1e-6 * 1e-4 / r


# ---------------------------------------------------------------------------
# P-6: momentum balance with walls removed


def _cloud_for_momentum(periodic, seed):
    prm = beds.Params(E=1e7, g=(0.0, 0.0, 0.0), mu_t=0.3, mu_r=0.05)
    spec = beds.random_cloud(400, 0.03, 0.03, 0.8e-3, 2.0e-3, seed=seed, periodic=periodic, params=prm,
                             vel_scale=0.05, omega_scale=20.0)
    return spec


def test_linear_momentum_conserved_periodic():
    spec = _cloud_for_momentum(3, 11)
    b = O.OracleBed(spec)
    m = spec.params.rho * 4.0 / 3.0 * math.pi * spec.radius.astype(np.float64) ** 3
    _, v0, _ = b.state()
    P0 = (m[:, None] * v0).sum(0)
    b.step(300)
    assert len(b.last_contacts()) > 50
    _, v1, _ = b.state()
    P1 = (m[:, None] * v1).sum(0)
    scale = (m * np.linalg.norm(v1, axis=1)).sum()
    assert np.all(np.abs(P1 - P0) < 1e-13 * scale)


def test_angular_momentum_conserved_open_cluster():
    spec = _cloud_for_momentum(0, 12)
    spec.pos -= spec.pos.mean(0)
    b = O.OracleBed(spec)
    r = spec.radius.astype(np.float64)
    m = spec.params.rho * 4.0 / 3.0 * math.pi * r ** 3
    I = 0.4 * m * r ** 2

    def Lang():
        x, v, w = b.state()
        return (np.cross(x, m[:, None] * v) + I[:, None] * w).sum(0), (
            np.linalg.norm(x, axis=1) * m * np.linalg.norm(v, axis=1)).sum()

    L0, _ = Lang()
    b.step(300)
    L1, scale = Lang()
    assert len(b.last_contacts()) > 50
    assert np.all(np.abs(L1 - L0) < 1e-12 * scale)


# ---------------------------------------------------------------------------
# P-7: static pile


def static_columns(n_cols=3, height=6, seed=0, params=None):
    """Vertical columns of unequal spheres placed at the closed-form Hertz
    equilibrium: the contact below sphere i carries the weight W_i of the
    spheres above and including i, so its overlap is (W_i / k_n)^(2/3) with
    k_n = E* sqrt(d*) / 3 (d* = 2 r_a r_b / (r_a + r_b); 2 r against the floor)."""
    prm = params or beds.Params(rho=2600.0)
    rng = np.random.default_rng(seed)
    Estar = prm.E / (2 * (1 - prm.nu ** 2))
    pos, rad = [], []
    side = 0.03 * n_cols
    for cx in range(n_cols):
        for cy in range(n_cols):
            r = rng.uniform(1.0e-3, 3.0e-3, height).astype(np.float32).astype(np.float64)
            m = prm.rho * 4.0 / 3.0 * math.pi * r ** 3
            load = np.cumsum(m[::-1])[::-1] * 9.81
            z = np.zeros(height)
            kn = Estar * math.sqrt(2 * r[0]) / 3.0
            z[0] = r[0] - (load[0] / kn) ** (2.0 / 3.0)
            for i in range(1, height):
                ds = 2 * r[i - 1] * r[i] / (r[i - 1] + r[i])
                kn = Estar * math.sqrt(ds) / 3.0
                z[i] = z[i - 1] + r[i - 1] + r[i] - (load[i] / kn) ** (2.0 / 3.0)
            for i in range(height):
                pos.append([0.015 + 0.03 * cx, 0.015 + 0.03 * cy, z[i]])
                rad.append(r[i])
    return make_spec(pos, rad, box=(side, side, 0), periodic=3, params=prm, walls=[beds.floor_wall()])


def test_static_columns_balance_gravity():
    """Each sphere's contact force cancels its weight; the floor carries the
    total weight; the state stays at rest."""
    spec = static_columns()
    b = O.OracleBed(spec)
    b.step(1)
    r = spec.radius.astype(np.float64)
    m = spec.params.rho * 4.0 / 3.0 * math.pi * r ** 3
    F, T = b.last_forces()
    np.testing.assert_allclose(F[:, 2], m * 9.81, rtol=1e-9)
    assert np.abs(F[:, :2]).max() < 1e-12 * (m * 9.81).max()
    assert np.abs(T).max() < 1e-15
    R = b.last_reaction(0)
    W = m.sum() * 9.81
    assert abs(R[2] + W) < 1e-10 * W
    assert len(b.last_contacts()) == spec.n
    b.step(200)
    _, v, _ = b.state()
    assert np.abs(v).max() < 1e-7


# ---------------------------------------------------------------------------
# P-8: symmetry


def test_relabelling_maps_contacts_and_forces():
    spec = beds.random_cloud(600, 0.03, 0.02, 0.6e-3, 2.0e-3, seed=5, periodic=3, vel_scale=0.01,
                             omega_scale=5.0, params=beds.Params(E=1e7))
    perm = np.random.default_rng(1).permutation(spec.n)
    inv = np.argsort(perm)
    spec2 = spec.copy()
    spec2.pos, spec2.radius = spec.pos[perm], spec.radius[perm]
    spec2.vel, spec2.omega = spec.vel[perm], spec.omega[perm]
    a, b = O.OracleBed(spec), O.OracleBed(spec2)
    a.step(1); b.step(1)
    ca = pairs_set(a.last_contacts())
    cb = {(int(perm[i]), int(perm[j])) for i, j in b.last_contacts().tolist()}
    assert ca == cb and len(ca) > 100
    Fa, Ta = a.last_forces()
    Fb, Tb = b.last_forces()
    np.testing.assert_allclose(Fb[inv], Fa, rtol=1e-10, atol=1e-12 * np.abs(Fa).max())
    np.testing.assert_allclose(Tb[inv], Ta, rtol=1e-10, atol=1e-12 * np.abs(Ta).max())


def test_periodic_shift_invariance():
    spec = beds.random_cloud(600, 0.03, 0.02, 0.6e-3, 2.0e-3, seed=6, periodic=3, params=beds.Params(E=1e7))
    spec2 = spec.copy()
    spec2.pos[:, 0] = np.mod(spec.pos[:, 0] + 0.01, 0.03)
    spec2.pos[:, 1] = np.mod(spec.pos[:, 1] + 0.01, 0.03)
    a, b = O.OracleBed(spec), O.OracleBed(spec2)
    a.step(1); b.step(1)
    assert pairs_set(a.last_contacts()) == pairs_set(b.last_contacts())
    Fa, _ = a.last_forces()
    Fb, _ = b.last_forces()
    np.testing.assert_allclose(Fb, Fa, rtol=1e-6, atol=1e-9 * np.abs(Fa).max())


# ---------------------------------------------------------------------------
# P-9: the generator's count model and layer identity against the paper


def test_count_model_reproduces_uniform_bed_table():
    with open(os.path.join(GOLDEN, "uniform_bed_counts.json")) as f:
        g = json.load(f)
    Lx, Ly, Lz = g["container_mm"]
    vol = Lx * Ly * Lz * 1e-9
    for row in g["rows"]:
        n = beds.uniform_count(row["d_mm"] * 1e-3, vol)
        assert abs(n - row["particles"]) <= 0.05 * row["particles"], (row, n)


def test_layer_identity():
    """d_n = d_0 / r + gamma(r, eta) z_n with gamma = (r - 1)/(r eta)."""
    for ratio, eta in ((2.0, 5.0), (1.3, 3.0), (1.05, 10.0)):
        d, z = beds.layer_profile(3e-3, ratio, eta, 12)
        gamma = (ratio - 1) / (ratio * eta)
        np.testing.assert_allclose(d, 3e-3 / ratio + gamma * z, rtol=1e-12)


def test_generated_bed_is_overlap_free_and_graded():
    spec = beds.graded_bed(20000, seed=2)
    p, r = spec.pos, spec.radius.astype(np.float64)
    L = spec.box[0]
    tree = cKDTree(np.c_[p[:, 0], p[:, 1], p[:, 2]], boxsize=[L, L, 100.0])
    cand = tree.query_pairs(2 * r.max(), output_type="ndarray")
    d = p[cand[:, 0]] - p[cand[:, 1]]
    d[:, :2] -= L * np.round(d[:, :2] / L)
    gap = np.linalg.norm(d, axis=1) - (r[cand[:, 0]] + r[cand[:, 1]])
    assert gap.min() > 0
    assert np.all(p[:, 2] - r >= 0)
    top = p[:, 2] > np.percentile(p[:, 2], 90)
    bot = p[:, 2] < np.percentile(p[:, 2], 10)
    assert r[bot].mean() > 3 * r[top].mean()
    assert r.max() <= 8 * 1.5e-3 * 1.1 * (1 + 1e-6)


# ---------------------------------------------------------------------------
# P-10: derivatives


def test_tangent_matches_central_differences():
    """Forward-mode dJ/d(s_k, mu_t, mu_r) of a mean wall reaction against
    FP64 central differences of the oracle's own forward runs (relative
    steps 1e-3 .. 1e-5, the most accurate one is compared).  The bed rests on a floor body that rises at 2 cm/s, so the
    window holds many sphere-sphere and sphere-wall contacts."""
    rng = np.random.default_rng(4)
    pos, rad = beds.layered_bed([(100, 3e-3), (150, 1.5e-3)], 0.03, 0.03, rng)
    prm = beds.Params(dt=2e-6)
    spec = make_spec(pos, rad, box=(0.03, 0.03, 0), periodic=3, params=prm,
                     walls=[beds.Wall(kind=beds.WALL_PLANE, body=1, axis=(0, 0, 1))],
                     bodies=[beds.Body(), beds.Body(lin_vel=(0.0, 0.0, 0.02))])
    base = O.OracleBed(spec)
    k0 = 400
    base.step(k0)
    cs = base.last_contacts()
    assert np.sum(cs[:, 1] == -1) >= 5 and np.sum(cs[:, 1] >= 0) >= 50
    x, v, w = base.state()
    keys, vals = base.history()
    nsteps = 200

    def run(**kw):
        s2 = spec.copy()
        s2.params = prm.replace(**kw)
        b = O.OracleBed(s2)
        b.set_state(x, v, w)
        b.set_history(keys, vals)
        b.set_clock(k0)
        return b

    J, g = run().tangent_window(nsteps, 1)
    assert J < 0  # particles push the floor down
    for q, name in enumerate(("s_k", "mu_t", "mu_r")):
        p0 = getattr(prm, name)
        errs = []
        for rel in (1e-3, 1e-4, 1e-5):  # truncation vs. rounding: take the best step
            h = rel * p0
            acc = []
            for sgn in (+1, -1):
                b = run(**{name: p0 + sgn * h})
                tot = 0.0
                for _ in range(nsteps):
                    b.step(1)
                    tot += b.last_reaction(1)[2]
                acc.append(tot / nsteps)
            fd = (acc[0] - acc[1]) / (2 * h)
            errs.append(abs(g[q] - fd) / max(abs(fd), 1e-3 * abs(J) / p0))
        assert min(errs) <= 1e-5, (name, g[q], errs)


def test_tangent_exact_linear_cases():
    """Cases where the reaction is linear in one parameter, so dJ/dtheta = J/theta:
    (a) an immovable sphere pressed by a plate (normal force ~ s_k);
    (b) a sphere in full Coulomb slip on a floor body (tangential ~ mu_t);
    (c) a sphere spinning about z on a floor body (rolling moment ~ mu_r)."""
    r = float(np.float32(1.5e-3))
    # (a)
    prm = beds.Params(rho=1e15, g=(0, 0, 0))
    spec = make_spec([[0.05, 0.05, 0.01]], [r], params=prm, box=(1, 1, 0),
                     walls=[beds.Wall(kind=beds.WALL_PLANE, body=1, axis=(0, 0, -1))],
                     bodies=[beds.Body(), beds.Body(origin=(0, 0, 0.01 + r), lin_vel=(0, 0, -0.01))])
    b = O.OracleBed(spec)
    b.step(5)
    J, g = b.tangent_window(100, 1, 2)
    assert J > 0 and abs(g[0] - J / prm.s_k) < 1e-9 * abs(J)
    # (b) and (c): floor as a body of its own
    m = 2600 * 4 / 3 * math.pi * r ** 3
    Estar = 1e9 / (2 * (1 - 0.15 ** 2))
    dstat = (m * 9.81 / (Estar * math.sqrt(2 * r) / 3)) ** (2 / 3)
    for comp, vel, omg, q, mu in ((0, [[0.2, 0, 0]], [[0, 0, 0]], 1, "mu_t"), (5, [[0, 0, 0]], [[0, 0, 300.0]], 2, "mu_r")):
        prm = beds.Params(rho=2600.0, mu_t=0.3, mu_r=0.05)
        spec = make_spec([[0.05, 0.05, r - dstat]], [r], vel=vel, omg=omg, params=prm, box=(1, 1, 0),
                         walls=[beds.Wall(kind=beds.WALL_PLANE, body=1, axis=(0, 0, 1))],
                         bodies=[beds.Body(), beds.Body()])
        b = O.OracleBed(spec)
        b.step(50)
        J, g = b.tangent_window(200, 1, comp)
        assert abs(J) > 0
        assert abs(g[q] - J / getattr(prm, mu)) < 1e-9 * abs(J / getattr(prm, mu)), (mu, g, J)


@pytest.mark.parametrize("mu,rolls", [(0.5, True), (0.05, False)])
def test_explicit_step_on_an_incline(mu, rolls):
    """A sphere on a plane tilted by 20 degrees (a plane wall with a tilted
    normal): rolling without slip at (5/7) g sin theta, or sliding at
    g (sin theta - mu cos theta); over 5,000 steps the tangential spring's
    start-up transient stays below 1e-3 of the acceleration."""
    from test_oracle_spook import incline
    theta = math.radians(20.0)
    spec, down = incline(theta, mu, dt=2e-6)
    b = O.OracleBed(spec)
    b.step(5000)
    a = float(b.state()[1][0] @ down) / (5000 * 2e-6)
    ref = (5.0 / 7.0) * 9.81 * math.sin(theta) if rolls else 9.81 * (math.sin(theta) - mu * math.cos(theta))
    assert abs(a / ref - 1.0) < 1e-3
