"""Pins of the oracle's time-implicit (SPOOK) step (CPU).

Each check compares the oracle with something other than itself: textbook
statics and rigid-body results, conservation laws, and the complementarity
conditions of the step written out here from their definition (section
"Nonsmooth DEM and multibody dynamics": eq:g_n, eq:G_t, eq:G_r with the
SPOOK stepper)."""
import math

import numpy as np

from oracle import oracle as O
from paper_2501_05300_amd import beds
from test_oracle_pins import make_spec, static_columns

G = 9.81


def spook_bed(spec, n_iter):
    b = O.OracleBed(spec)
    b.set_stepper("spook", n_iter)
    return b


def test_static_columns_are_a_fixed_point():
    """Spheres placed at the Hertz equilibrium (contact below sphere i at
    overlap (W_i / k_n)^(2/3)) and at rest: the step's exact solution is
    v+ = 0 with every contact carrying the weight above it."""
    spec = static_columns(params=beds.Params(rho=2600.0, dt=1e-4))
    b = spook_bed(spec, 3000)
    b.step(1)
    r = spec.radius.astype(np.float64)
    m = spec.params.rho * 4.0 / 3.0 * math.pi * r ** 3
    F, T = b.last_forces()
    np.testing.assert_allclose(F[:, 2], m * G, rtol=1e-6)
    R = b.last_reaction(0)
    assert abs(R[2] + m.sum() * G) < 1e-6 * m.sum() * G
    _, v, w = b.state()
    assert np.abs(v).max() < 1e-9 and np.abs(w).max() < 1e-6


def _sphere(mu_t, mu_r, v0, w0, dt, start_overlap=1.0):
    prm = beds.Params(rho=2600.0, mu_t=mu_t, mu_r=mu_r, dt=dt)
    r = float(np.float32(1.5e-3))
    m = prm.rho * 4.0 / 3.0 * math.pi * r ** 3
    kn = prm.E / (2 * (1 - prm.nu ** 2)) * math.sqrt(2 * r) / 3.0
    dstat = (m * G / kn) ** (2.0 / 3.0)
    spec = make_spec([[0.01, 0.01, r - start_overlap * dstat]], [r], vel=[[v0, 0, 0]], omg=[[0, w0, 0]],
                     params=prm, walls=[beds.floor_wall()], box=(1, 1, 0))
    return spec, r, m, dstat


def test_sphere_settles_at_the_hertz_overlap():
    """A sphere released at half its static overlap settles where k_n
    delta^(3/2) = m g, and the floor carries m g."""
    spec, r, m, dstat = _sphere(0.4, 0.02, 0.0, 0.0, 1e-4, start_overlap=0.5)
    b = spook_bed(spec, 10)
    b.step(400)
    x, v, _ = b.state()
    assert abs((r - x[0, 2]) - dstat) < 1e-6 * dstat
    assert abs(b.last_reaction(0)[2] + m * G) < 1e-6 * m * G
    assert abs(v[0, 2]) < 1e-9


def test_sliding_sphere_starts_rolling_at_textbook_time():
    """Coulomb sliding decelerates at mu g until t* = 2 v0 / (7 mu g); the
    sphere then rolls without slip at 5 v0 / 7."""
    mu, v0, dt = 0.4, 0.1, 1e-5
    spec, r, _, _ = _sphere(mu, 0.0, v0, 0.0, dt)
    b = spook_bed(spec, 20)
    vs, ws = [], []
    for _ in range(1500):
        b.step(1)
        _, v, w = b.state()
        vs.append(v[0, 0])
        ws.append(w[0, 1])
    vs, ws = np.array(vs), np.array(ws)
    a = (vs[100] - vs[0]) / (100 * dt)
    assert abs(a + mu * G) < 1e-3 * mu * G
    tstar = 2 * v0 / (7 * mu * G)
    k = int(np.argmax(vs - r * ws < 1e-6 * v0))
    assert abs((k + 1) * dt - tstar) < 0.005 * tstar
    assert abs(vs[-1] - 5 * v0 / 7) < 1e-3 * v0


def test_rolling_resistance_deceleration():
    """Rolling under the rolling-resistance moment at its bound mu_r r m g
    decelerates at (5/7) mu_r g."""
    mu_r, v0, dt = 0.02, 0.05, 1e-5
    spec, r, _, _ = _sphere(0.4, mu_r, v0, v0 / 1.5e-3, dt)
    b = spook_bed(spec, 20)
    vs = []
    for _ in range(800):
        b.step(1)
        vs.append(b.state()[1][0, 0])
    t = dt * np.arange(len(vs))
    a = np.polyfit(t[100:], np.array(vs)[100:], 1)[0]
    assert abs(a + (5.0 / 7.0) * mu_r * G) < 0.005 * (5.0 / 7.0) * mu_r * G


def _cloud(periodic, seed):
    prm = beds.Params(E=1e7, g=(0.0, 0.0, 0.0), mu_t=0.3, mu_r=0.05, dt=1e-4)
    return beds.random_cloud(400, 0.03, 0.03, 0.8e-3, 2.0e-3, seed=seed, periodic=periodic, params=prm,
                             vel_scale=0.05, omega_scale=20.0)


def test_linear_momentum_conserved_periodic():
    spec = _cloud(3, 11)
    b = spook_bed(spec, 30)
    m = spec.params.rho * 4.0 / 3.0 * math.pi * spec.radius.astype(np.float64) ** 3
    P0 = (m[:, None] * b.state()[1]).sum(0)
    b.step(1)
    assert len(b.last_contacts()) > 50
    b.step(19)
    v1 = b.state()[1]
    scale = (m * np.linalg.norm(v1, axis=1)).sum()
    assert np.all(np.abs((m[:, None] * v1).sum(0) - P0) < 1e-13 * scale)


def test_angular_momentum_conserved_open_cluster():
    """Impulses act at shared contact points and the rolling impulses are
    equal and opposite, and x+ - x0 is parallel to v+: the angular momentum
    about the origin is unchanged by a step."""
    spec = _cloud(0, 12)
    spec.pos -= spec.pos.mean(0)
    b = spook_bed(spec, 30)
    r = spec.radius.astype(np.float64)
    m = spec.params.rho * 4.0 / 3.0 * math.pi * r ** 3
    I = 0.4 * m * r ** 2

    def L():
        x, v, w = b.state()
        return (np.cross(x, m[:, None] * v) + I[:, None] * w).sum(0), (
            np.linalg.norm(x, axis=1) * m * np.linalg.norm(v, axis=1)).sum()

    L0, _ = L()
    b.step(1)
    assert len(b.last_contacts()) > 50
    b.step(19)
    L1, scale = L()
    assert np.all(np.abs(L1 - L0) < 1e-12 * scale)


def _contact_rows(spec, x0, a, c):
    """Normal (a toward the partner), overlap and lever arms of contact (a, c)
    at positions x0; walls are floors (plane z = 0 facing +z)."""
    ra = float(spec.radius[a])
    if c >= 0:
        D = x0[c] - x0[a]
        for ax in range(2):
            if (spec.periodic >> ax) & 1:
                L = spec.box[ax]
                D[ax] -= L * np.round(D[ax] / L)
        d = np.linalg.norm(D)
        rb = float(spec.radius[c])
        delta = ra + rb - d
        return D / d, delta, ra - delta / 2, rb - delta / 2, 2 * ra * rb / (ra + rb)
    delta = ra - x0[a, 2]
    return np.array([0.0, 0.0, -1.0]), delta, ra - delta / 2, 0.0, 2 * ra


def test_converged_step_satisfies_the_complementarity_conditions():
    """After enough iterations the impulses and the new velocities satisfy,
    contact by contact: P >= 0, the SPOOK normal row >= 0 and complementary
    to P; |p_t| <= mu_t P with no tangential slip unless at the bound, where
    p_t opposes the slip; the same for the rolling impulse and mu_r r*."""
    prm = beds.Params(rho=2600.0, E=1e7, mu_t=0.3, mu_r=0.05, dt=1e-4)
    spec = beds.random_cloud(300, 0.025, 0.02, 0.8e-3, 2.0e-3, seed=3, periodic=3, params=prm,
                             vel_scale=0.05, omega_scale=20.0)
    spec.walls = [beds.floor_wall()]
    spec.pos[:, 2] += 0.5e-3    # some spheres overlap the floor
    b = spook_bed(spec, 4000)
    x0, v0, w0 = b.state()
    b.step(1)
    _, v1, w1 = b.state()
    pairs = b.last_contacts()
    keys, vals = b.history()
    hist = {(int(k[0]), int(k[1])): q for q, k in enumerate(keys)}
    assert len(pairs) > 100 and np.sum(pairs[:, 1] < 0) > 5
    h, eH, tau = prm.dt, prm.e_H, prm.gamma_factor * prm.dt
    Estar = prm.E / (2 * (1 - prm.nu ** 2))
    r = spec.radius.astype(np.float64)
    m = prm.rho * 4.0 / 3.0 * math.pi * r ** 3
    Pscale = (m * 0.05).max()
    n_slide = n_stick = 0
    for a, c in pairs:
        q = hist[(int(a), int(c))]
        J, pr = vals[q, :3], vals[q, 3:]
        n, delta, la, lb, dstar = _contact_rows(spec, x0, a, c)
        assert delta > 0

        def rel(v, w):
            u = v[a] + la * np.cross(w[a], n)
            if c >= 0:
                u = u - v[c] + lb * np.cross(w[c], n)
            return u, (w[a] - w[c]) if c >= 0 else w[a]

        P = -J @ n
        pt = J + P * n
        u1, wr1 = rel(v1, w1)
        u0, _ = rel(v0, w0)
        kn = Estar * math.sqrt(dstar) / 3.0
        S = 4.0 / (kn * eH * h * h * (1 + 4 * tau / h) * delta ** (2 * eH - 2))
        C = (u0 @ n - 4 * delta / (eH * h)) / (1 + 4 * tau / h)
        wn = -(u1 @ n) + S * P + C
        vscale = 0.05 + abs(C)
        assert P >= -1e-12 * Pscale
        assert wn >= -1e-7 * vscale
        assert min(P / Pscale, wn / vscale) < 1e-7
        ut = u1 - (u1 @ n) * n
        cap = prm.mu_t * P
        assert np.linalg.norm(pt) <= cap * (1 + 1e-9) + 1e-15
        if np.linalg.norm(pt) < cap * (1 - 1e-6):
            assert np.linalg.norm(ut) < 1e-7 * vscale
            n_stick += 1
        elif np.linalg.norm(ut) > 1e-7 * vscale and np.linalg.norm(pt) > 0:   # P = 0: p_t = 0 may slip
            cosang = (pt @ ut) / (np.linalg.norm(pt) * np.linalg.norm(ut))
            assert cosang < -1 + 1e-6
            n_slide += 1
        capr = prm.mu_r * 0.5 * dstar * P
        assert np.linalg.norm(pr) <= capr * (1 + 1e-9) + 1e-18
        if np.linalg.norm(pr) < capr * (1 - 1e-6):
            assert np.linalg.norm(wr1) < 1e-5 * 20.0
    assert n_stick > 10 and n_slide > 0


def test_fixed_point_does_not_depend_on_the_warm_start():
    """The converged step is the same whether the iteration starts from the
    stored impulses or from zero; with the stored ones a few iterations land
    closer to it."""
    spec = static_columns(params=beds.Params(rho=2600.0, dt=1e-4))
    spec.vel[:] = np.random.default_rng(0).normal(0, 1e-3, spec.vel.shape).astype(np.float32)
    warm = spook_bed(spec, 3000)
    warm.step(1)
    state, (keys, vals) = warm.state(), warm.history()
    ref = spook_bed(spec, 3000)
    ref.set_state(*state)
    ref.set_history(keys, vals)
    ref.set_clock(1)
    ref.step(1)
    cold = spook_bed(spec, 3000)
    cold.set_state(*state)
    cold.set_clock(1)
    cold.step(1)
    np.testing.assert_allclose(cold.state()[1], ref.state()[1], atol=1e-9)
    errs = []
    for hist in ((keys, vals), None):
        few = spook_bed(spec, 20)
        few.set_state(*state)
        if hist is not None:
            few.set_history(*hist)
        few.set_clock(1)
        few.step(1)
        errs.append(np.abs(few.state()[1] - ref.state()[1]).max())
    assert errs[0] < 0.1 * errs[1]


def incline(theta, mu_t, dt=1e-4):
    """A sphere resting at its static overlap on a plane through the origin
    tilted by theta about y (its surface descends along +x)."""
    prm = beds.Params(rho=2600.0, mu_t=mu_t, mu_r=0.0, dt=dt)
    r = float(np.float32(1.5e-3))
    m = prm.rho * 4.0 / 3.0 * math.pi * r ** 3
    kn = prm.E / (2 * (1 - prm.nu ** 2)) * math.sqrt(2 * r) / 3.0
    nu = np.array([math.sin(theta), 0.0, math.cos(theta)])
    delta = (m * G * math.cos(theta) / kn) ** (2.0 / 3.0)
    o = np.array([0.5, 0.5, 0.2])
    c = o + (r - delta) * nu
    wall = beds.Wall(kind=beds.WALL_PLANE, body=0, origin=tuple(o), axis=tuple(nu))
    spec = make_spec([c], [r], params=prm, walls=[wall], box=(1, 1, 0))
    return spec, np.array([math.cos(theta), 0.0, -math.sin(theta)])


def slope_acceleration(b, down, steps, dt):
    b.step(steps)
    v = b.state()[1][0]
    return float(v @ down) / (steps * dt)


def test_sphere_rolls_down_an_incline_without_slip():
    """Enough friction (mu >= (2/7) tan theta): rolling without slip at
    a = (5/7) g sin theta."""
    theta = math.radians(20.0)
    spec, down = incline(theta, 0.5)
    a = slope_acceleration(spook_bed(spec, 20), down, 200, 1e-4)
    assert abs(a / ((5.0 / 7.0) * G * math.sin(theta)) - 1.0) < 1e-3


def test_sphere_slides_down_an_incline_at_the_coulomb_bound():
    """Little friction (mu < (2/7) tan theta): sliding at g (sin theta - mu cos theta)."""
    theta, mu = math.radians(20.0), 0.05
    spec, down = incline(theta, mu)
    a = slope_acceleration(spook_bed(spec, 20), down, 200, 1e-4)
    assert abs(a / (G * (math.sin(theta) - mu * math.cos(theta))) - 1.0) < 1e-3
