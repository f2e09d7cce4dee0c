"""Parity of the HIP stepper with the FP64 oracle (GPU).

Bars: contact lists bit-exact given the same state; per-step contact forces
and torques within 1e-5 (normwise over particles); body reactions within
1e-5; short trajectories within 1e-3 r_min after 1000 steps.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2501_05300_amd import beds
from parity_util import assert_parity, compare_one_step, masses, oracle_pairs, rel_norm

pytestmark = pytest.mark.gpu

FTOL = 1e-5


def gpu_bed(spec, **kw):
    from paper_2501_05300_amd.lprdem import Bed
    kw.setdefault("record_forces", True)
    return Bed(spec, **kw)


def cloud(seed, n=3000, side=0.1, periodic=3, walls=True, ratio=10.0, vel=0.05, omg=20.0, E=1e7):
    """Random spheres (solid fraction ~0.4, radii 0.5-5 mm log-uniform) with
    floor, disk plate and a grouser box."""
    prm = beds.Params(E=E)
    spec = beds.random_cloud(n, side, 0.06, 0.5e-3, 0.5e-3 * ratio, seed=seed, periodic=periodic, params=prm,
                             vel_scale=vel, omega_scale=omg)
    if walls:
        spec.walls = [beds.floor_wall(),
                      beds.Wall(kind=beds.WALL_DISK, body=1, axis=(0, 0, -1), dims=(0.03, 0, 0)),
                      beds.Wall(kind=beds.WALL_BOX, body=1, origin=(0.0, 0.012, 0.0), dims=(0.004, 0.002, 0.003))]
        spec.bodies = [beds.Body(), beds.Body(origin=(0.5 * side, 0.5 * side, 0.04), lin_vel=(0.0, 0.0, -0.05))]
    return spec


@pytest.mark.parametrize("seed,periodic", [(1, 3), (2, 0), (3, 1)])
def test_first_step_matches_oracle(seed, periodic):
    spec = cloud(seed, periodic=periodic)
    bed = gpu_bed(spec)
    res = compare_one_step(spec, bed)
    print(res)
    assert_parity(res, FTOL)
    assert res["n_contacts"] > 500


def test_two_layer_bed_history_parity():
    """Two-layer bed (2,000 spheres): after 2,000 GPU steps (the bed's settle
    window) the state and contact history are handed to the oracle; the next
    steps must agree."""
    spec = beds.two_layer_bed(0)
    bed = gpu_bed(spec)
    bed.step(2000)
    keys, _ = bed.history()
    print("history records", len(keys))
    assert len(keys) > 200
    for _ in range(3):
        res = compare_one_step(spec, bed)
        print(res)
        assert_parity(res, FTOL)
        bed.step(50)


def test_static_columns_balance_gravity_gpu():
    from test_oracle_pins import static_columns
    spec = static_columns()
    bed = gpu_bed(spec)
    bed.step(1)
    m, _ = masses(spec)
    F, T = bed.forces()
    np.testing.assert_allclose(F[:, 2], m * 9.81, rtol=2e-5)
    R = bed.reaction(0)
    W = m.sum() * 9.81
    assert abs(R[2] + W) < 2e-5 * W
    assert len(bed.contacts()) == spec.n


def test_momentum_conserved_gpu():
    spec = cloud(5, walls=False, vel=0.05, omg=20.0)
    spec.params = spec.params.replace(g=(0.0, 0.0, 0.0))
    bed = gpu_bed(spec)
    m, _ = masses(spec)
    _, v0, _ = bed.state()
    P0 = (m[:, None] * v0).sum(0)
    bed.step(1000)
    _, v1, _ = bed.state()
    P1 = (m[:, None] * v1.astype(np.float64)).sum(0)
    scale = (m * np.linalg.norm(v1, axis=1)).sum()
    assert np.all(np.abs(P1 - P0) < 1e-6 * scale)


def test_bitwise_determinism_and_graph_replay():
    """Two beds from the same input give bitwise equal states; stepping by
    captured-graph cycles equals stepping one step at a time."""
    spec = beds.two_layer_bed(1)
    a, b = gpu_bed(spec), gpu_bed(spec)
    a.step(40)                 # graph cycles
    for _ in range(40):
        b.step(1)              # direct launches
    xa, va, wa = a.state()
    xb, vb, wb = b.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(wa, wb)
    assert np.array_equal(a.contacts(), b.contacts())


def test_short_trajectory_bound():
    """Two-layer bed, 1000 steps from the same state: the FP32 stepper stays
    within 1e-3 r_min of the FP64 oracle."""
    spec = beds.two_layer_bed(2)
    bed = gpu_bed(spec, record_forces=False)
    ob = O.OracleBed(spec)
    bed.step(1000)
    ob.step(1000)
    xg, _, _ = bed.state()
    xo, _, _ = ob.state()
    d = xg - xo
    L = spec.box[0]
    d[:, :2] -= L * np.round(d[:, :2] / L)
    err = np.linalg.norm(d, axis=1).max()
    print("max trajectory deviation", err)
    assert err < 1e-3 * float(spec.radius.min())


@pytest.mark.parametrize("opts", [dict(cell_factor=1.5), dict(band_ratio=1.5), dict(block=256), dict(block=128),
                                  dict(band_ratio=8.0, cell_factor=1.25), dict(cell_factor=3.5)])
def test_contact_list_invariant_to_broad_phase_choices(opts):
    """Cell sizes, radius bands and launch shapes change which cells and rows
    the search walks (cell factor 3.5 leaves the coarsest level two cells
    across the periodic box, where every cell is taken once, and cells far
    wider than the reach, where most rows and end cells are dropped), never
    the contact list or the forces."""
    spec = cloud(9, n=2500)
    ref = gpu_bed(spec)
    ref.step(1)
    alt = gpu_bed(spec, **opts)
    alt.step(1)
    assert np.array_equal(ref.contacts(), alt.contacts())
    Fr, _ = ref.forces()
    Fa, _ = alt.forces()
    assert rel_norm(Fa, Fr) < 1e-6


def test_plate_reaction_parity():
    """Two-layer bed with a plate pushed into it: plate reaction within 1e-5."""
    spec = beds.add_plate(beds.two_layer_bed(3), diameter=0.04, speed=0.5)
    bed = gpu_bed(spec)
    bed.step(400)
    res = compare_one_step(spec, bed)
    print(res)
    assert_parity(res, FTOL)
    R = bed.reaction(1)
    assert abs(R[2]) > 0


@pytest.mark.parametrize("skin,every", [(2e-4, 10), (1e-9, 7)])
def test_skin_lists_step_bitwise_like_every_step_search(skin, every):
    """Candidate lists with a skin, rebuilt every few steps, find the same
    contacts in the same order as a search every step, so the trajectories
    are bitwise equal; a skin too small to hold forces rebuilds (trips) and
    still gives the same result."""
    spec = beds.add_plate(beds.two_layer_bed(4), diameter=0.04, speed=0.5)
    a = gpu_bed(spec)
    b = gpu_bed(spec, rebuild_every=every, skin=skin)
    a.step(150)
    b.step(150)
    xa, va, wa = a.state()
    xb, vb, wb = b.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(wa, wb)
    assert np.array_equal(a.contacts(), b.contacts())
    # the two beds re-sort their storage at different steps, so the FP64
    # block sums of the plate reaction add the same terms in another order
    np.testing.assert_allclose(a.reaction(1), b.reaction(1), rtol=1e-12, atol=1e-12 * abs(a.reaction(1)[2]))
    st = b.stats()
    print(st)
    if skin < 1e-6:
        assert st["skin_trips"] > 0
    else:
        assert st["rebuilds"] < 150


def test_grousered_ring_parity():
    """Dead-weight grousered ring (annulus + 8 boxes, free in z, rotating)
    lowered into the two-layer bed: contacts bit-exact and forces, torques
    and the ring reaction within 1e-5 of the oracle, from the same state,
    history, clock and ring DOF."""
    spec = beds.two_layer_bed(5)
    spec = beds.add_ring(spec, r_in=0.012, r_out=0.024, grouser_len=0.012, grouser_thick=0.003,
                         grouser_depth=0.004, pressure=2e3, omega=5.0)
    spec.bodies[1].lin_vel = (0.0, 0.0, -1.0)   # thrown onto the bed
    bed = gpu_bed(spec)
    bed.step(1000)
    o, v = bed.body(1)
    assert v[2] < 0.0  # the ring sinks under its weight
    for _ in range(2):
        res = compare_one_step(spec, bed)
        print(res)
        assert_parity(res, FTOL)
        assert abs(bed.reaction(1)[5]) > 0  # the drive torque is compared too
        bed.step(100)
    n_ring = int(np.sum(bed.contacts()[:, 1] <= -2))
    assert n_ring > 0


def test_full_size_graded_bed_step_parity():
    """The 2,000,000-sphere graded bed the throughput is measured on, in the
    launch configuration the bench times (cell search every step, 256-thread
    step blocks): relaxed on the GPU until contacts form, then one step
    against the oracle on the same state. Contact lists equal, forces and
    torques within 1e-5."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = beds.metric_bed()
    relax = spec.copy()
    relax.params = beds.settle_params(spec.params).replace(dt=5e-6, gamma_factor=10.0)
    for w in relax.walls:
        w.mu_t, w.mu_r = 0.0, 0.0
    rb = Bed(relax, rebuild_every=5, skin=0.25 * float(spec.radius.min()))
    for _ in range(6):
        rb.step(5000)
        rb.sync()
    x, _, _ = rb.state()
    rb.close()
    spec.pos = x
    bed = gpu_bed(spec)
    bed.step(3)
    res = compare_one_step(spec, bed)
    print({k: v for k, v in res.items() if k not in ("only_gpu", "only_oracle")})
    assert_parity(res, FTOL)
    assert res["n_contacts"] > spec.n  # a bed in contact, not a falling cloud
