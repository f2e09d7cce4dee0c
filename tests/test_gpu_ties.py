"""Near ties of the contact predicate and moving-wall poses on the GPU.

The contact set is defined by the exact FP64 predicate (d^2 < (r_i + r_j)^2
for spheres, signed distance < r for walls); the GPU's FP32 pre-test must
never drop a pair that the predicate keeps.  These cases put pairs within a
few FP64 ulps of touching at coordinates up to 2.12 m (where an FP32 ulp is
2.4e-7 m, far above the overlaps involved), across both periodic seams, with
a size ratio of 8, and spheres within a few ulps of the floor and of a plate
face.  The wall poses of a spinning body are compared bit for bit with the
oracle's, since a last-ulp difference in a pose can flip a near-tie wall
contact.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2501_05300_amd import beds
from parity_util import assert_parity, compare_one_step

pytestmark = pytest.mark.gpu

L = 2.1225


def ulp_step(x, k):
    """x moved by k FP64 ulps."""
    for _ in range(abs(k)):
        x = np.nextafter(x, np.inf if k > 0 else -np.inf)
    return float(x)


def near_tie_bed(seed=7):
    rng = np.random.default_rng(seed)
    r32 = [float(np.float32(1.5e-3)), float(np.float32(12e-3))]
    pos, rad = [], []
    # sphere pairs on sites 0.1 m apart; the last rows and columns sit at the
    # periodic seams so that their partners wrap
    xs = list(np.linspace(0.08, L - 0.08, 19)) + [L - 1e-3]
    for xi in xs:
        for yi in xs:
            ri, rj = r32[rng.integers(2)], r32[rng.integers(2)]
            u = rng.normal(size=3)
            if xi > L - 0.01:
                u[0] = abs(u[0]) + 0.5
            if yi > L - 0.01:
                u[1] = abs(u[1]) + 0.5
            u /= np.linalg.norm(u)
            if rng.random() < 0.2:   # along an axis: d^2 is one square
                u = np.zeros(3)
                u[rng.integers(3)] = 1.0
            pi = np.array([xi, yi, 0.1 + 0.02 * rng.random()])
            pj = pi + (ri + rj) * u
            for c in range(3):
                pj[c] = ulp_step(pj[c], int(rng.integers(-3, 4)))
            for c in range(2):
                if pj[c] >= L:
                    pj[c] -= L
            pos += [pi, pj]
            rad += [ri, rj]
    # spheres within a few ulps of the floor (contact iff z < r)
    for q in range(60):
        r = r32[q % 2]
        pos.append(np.array([0.11 + 0.1 * (q % 19), 0.16 + 0.1 * (q // 19), ulp_step(r, q % 7 - 3)]))
        rad.append(r)
    # and of the face of a static plate at z = 0.3 (contact iff 0.3 - z < r)
    zp = 0.3
    cx = cy = 0.5 * L
    for q in range(25):
        r = r32[q % 2]
        x = cx + 0.026 * (q % 5 - 2)
        y = cy + 0.026 * (q // 5 - 2)
        pos.append(np.array([x, y, ulp_step(zp - r, q % 7 - 3)]))
        rad.append(r)
    pos = np.array(pos)
    n = len(rad)
    spec = beds.BedSpec(pos=pos, radius=np.array(rad, np.float32), vel=np.zeros((n, 3), np.float32),
                        omega=np.zeros((n, 3), np.float32), box=(L, L, 0.0), periodic=3,
                        params=beds.paper_params(),
                        walls=[beds.floor_wall(),
                               beds.Wall(kind=beds.WALL_DISK, body=1, axis=(0.0, 0.0, -1.0), dims=(0.08, 0.0, 0.0))],
                        bodies=[beds.Body(), beds.Body(origin=(cx, cy, zp))])
    return spec


def test_near_tie_contacts_match_oracle():
    from paper_2501_05300_amd.lprdem import Bed
    spec = near_tie_bed()
    n_pairs = 2 * 20 * 20
    bed = Bed(spec, record_forces=True)
    res = compare_one_step(spec, bed)
    print({k: v for k, v in res.items() if k not in ("only_gpu", "only_oracle")})
    assert_parity(res, 1e-5)
    got = bed.contacts()
    sph = got[(got[:, 1] >= 0) & (got[:, 0] < n_pairs)]
    floor = got[got[:, 1] == -1]
    plate = got[got[:, 1] == -2]
    print("sphere ties in contact", len(sph), "of", n_pairs // 2, "; floor", len(floor), "; plate", len(plate))
    # the ties split both ways (the test is not one-sided)
    assert 0.2 * n_pairs / 2 < len(sph) < 0.8 * n_pairs / 2
    assert 10 < len(floor) < 50 and 5 < len(plate) < 20
    # every pair across a seam that the oracle keeps is kept
    seam = [(a, b) for a, b in sph.tolist() if abs(spec.pos[a, 0] - spec.pos[b, 0]) > 1.0
            or abs(spec.pos[a, 1] - spec.pos[b, 1]) > 1.0]
    assert len(seam) > 5


def test_near_tie_contacts_after_a_shift_across_the_seams():
    """The same bed shifted by (L/3, L/3): the pairs now straddle other cells
    and other seams; contacts still match the oracle."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = near_tie_bed(8)
    spec.pos[:, :2] = np.mod(spec.pos[:, :2] + L / 3.0, L)
    o = spec.bodies[1].origin
    spec.bodies[1].origin = ((o[0] + L / 3.0) % L, (o[1] + L / 3.0) % L, o[2])
    bed = Bed(spec, record_forces=True, band_ratio=1.5)
    res = compare_one_step(spec, bed)
    print({k: v for k, v in res.items() if k not in ("only_gpu", "only_oracle")})
    assert_parity(res, 1e-5)


def spinning_ring_spec(omega):
    pos = np.array([[0.05, 0.05, 0.002], [0.35, 0.05, 0.002], [0.05, 0.35, 0.002], [0.35, 0.35, 0.002]])
    spec = beds.BedSpec(pos=pos, radius=np.full(4, 2e-3, np.float32), vel=np.zeros((4, 3), np.float32),
                        omega=np.zeros((4, 3), np.float32), box=(0.4, 0.4, 0.0), periodic=3,
                        params=beds.paper_params(), walls=[beds.floor_wall()], bodies=[beds.Body()])
    spec = beds.add_ring(spec, r_in=0.05, r_out=0.08, grouser_len=0.02, grouser_thick=0.004, grouser_depth=0.006,
                         pressure=2e3, omega=omega)
    spec.bodies[1].origin = (0.2, 0.2, 0.3)   # above the spheres: no contacts
    return spec


def test_spinning_wall_poses_match_oracle_bitwise():
    """A ring with grousers spinning at 300 rad/s about +z (0.6 mrad per
    step) and falling freely: at 60 clocks over 10 rad of rotation, every
    wall's origin, normal and frame equal the oracle's bit for bit (the
    oracle computes the pose from the clock and the body's z state)."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = spinning_ring_spec(300.0)
    bed = Bed(spec)
    ob = O.OracleBed(spec)
    mism = []
    done = 0
    for q in range(60):
        k = 17 + 271 * q - done
        bed.step(k)
        done += k
        clock = bed.clock()
        o, v = bed.body(1)
        ob.set_clock(clock)
        ob.set_body_state(1, o[2], v[2])
        for w in range(len(spec.walls)):
            g = bed.wall_pose(w)
            r = ob.wall_pose(w)
            for a, b in zip(g, r):
                if not np.array_equal(np.asarray(a), np.asarray(b)):
                    mism.append((clock, w, np.max(np.abs(np.asarray(a) - np.asarray(b)))))
    print("clocks", done, "mismatches", mism[:10])
    assert done > 15000 and 300.0 * done * spec.params.dt > 9.0
    assert not mism
