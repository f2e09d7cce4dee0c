"""Layer-by-layer emission on the GPU: a small refined bed (3 and 6 mm
layers on a 12 mm base, gamma 0.25) built, trimmed and relaxed through the
HIP library."""
import numpy as np
import pytest

from paper_2501_05300_amd import emission as E

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_emitted_bed_is_layered_trimmed_and_settled():
    d_min, r, eta, n, h, side = 3e-3, 2.0, 2.0, 2, 0.04, 0.05
    bed = E.emit_bed(d_min, r, eta, n, h, side, seed=0, max_steps=120_000, log=print)
    dg = E.diagnostics(bed, rho=2200.0)
    print(dg)
    assert dg["n"] > 500
    assert dg["top"] <= h                                   # every layer trimmed at its top
    for q, L in enumerate(bed.layers):
        sel = bed.layer == q
        assert sel.sum() > 10
        d = 2.0 * bed.radius[sel]
        assert np.all((d >= 0.9 * L.d * (1 - 1e-6)) & (d <= 1.1 * L.d * (1 + 1e-6)))
        assert abs(np.median(d) / L.d - 1.0) < 0.05
    # relaxed contacts: overlaps stay a small fraction of the radii
    x, rad = bed.pos, bed.radius.astype(np.float64)
    D = x[None, :, :] - x[:, None, :]
    D[..., :2] -= side * np.round(D[..., :2] / side)
    gap = np.linalg.norm(D, axis=2) - (rad[None, :] + rad[:, None])
    np.fill_diagonal(gap, np.inf)
    assert gap.min() > -0.02 * rad.min()
    assert np.all(x[:, 2] - rad > -0.02 * rad.min())        # nothing through the floor
    assert max(dg["mixing"]) < 0.25
    assert 0.5 * 2200 < dg["density_mean"] < 0.7 * 2200


def test_relaxing_emitted_layer_steps_like_the_oracle():
    """A finer layer emitted onto a relaxed coarse base, stopped while it
    falls and lands (section "Generation of soil samples" settings: reduced
    friction, frictionless floor, dt 5e-6 s, gamma_n = 10 dt, candidate lists
    with a skin): one more step on the GPU and in the oracle from the same
    state and spring history.  Contacts equal; forces, torques, per-contact
    loads and the floor reaction within 1e-5."""
    from paper_2501_05300_amd import beds
    from paper_2501_05300_amd.lprdem import Bed
    from parity_util import assert_parity, compare_one_step
    side = 0.04
    layers = E.plan_layers(3e-3, 2.0, 2.0, 1, 0.03)
    prm = beds.settle_params(beds.paper_params()).replace(dt=5e-6, gamma_factor=10.0)
    rng = np.random.default_rng(3)
    base = layers[0]
    pos, rad = E.emit(rng, base, side, 0.1 * base.d, E.emission_count(base, side))
    z = np.zeros((len(rad), 3), np.float32)
    pos, vel, omg, _ = E.relax(pos, rad, z, z, side, prm, v_tol=0.05, max_steps=40_000)
    keep = pos[:, 2] <= base.z_hi
    pos, rad, vel, omg = pos[keep], rad[keep], vel[keep], omg[keep]
    fine = layers[1]
    top = float(np.max(pos[:, 2] + rad))
    p1, r1 = E.emit(rng, fine, side, max(top, fine.z_lo) + 0.1 * fine.d, E.emission_count(fine, side))
    n1 = len(r1)
    spec = E.relax_spec(np.concatenate([pos, p1]), np.concatenate([rad, r1]),
                        np.concatenate([vel, np.zeros((n1, 3), np.float32)]),
                        np.concatenate([omg, np.zeros((n1, 3), np.float32)]), side, prm)
    bed = Bed(spec, record_forces=True, **E.relax_lists(spec))
    bed.step(8000)   # the lowest fine sheets have landed and bounce, the upper ones still fall
    res = compare_one_step(spec, bed)
    print({k: v for k, v in res.items() if k not in ("only_gpu", "only_oracle")})
    assert_parity(res, 1e-5)
    got = bed.contacts()
    fine_ids = np.arange(len(rad), len(rad) + n1)
    assert int(np.isin(got, fine_ids).any(axis=1).sum()) > 50   # the new layer is in contact
    assert int(np.sum(got[:, 1] < 0)) > 10                       # spheres on the floor
