"""Device re-sort of the storage order (GPU).

Particles are kept sorted by (level, Morton code of their cell) by a radix
sort on the device every few rebuilds, and the state is gathered into the new
order; per-particle results are summed in stable-id order, so the order
changes which particles share cache lines and blocks, never a particle's
result.  Body reactions are FP64 sums over blocks of the storage order: the
same terms in another order.
"""
import numpy as np
import pytest

from paper_2501_05300_amd import beds
from parity_util import assert_parity, compare_one_step

pytestmark = pytest.mark.gpu


def plate_bed(seed):
    return beds.add_plate(beds.two_layer_bed(seed), diameter=0.04, speed=0.5)


@pytest.mark.parametrize("opts", [dict(sort_every=-1), dict(sort_every=1), dict(sort_every=3, input_order=True),
                                  dict(sort_every=2, rebuild_every=5, skin=1e-4)])
def test_storage_order_never_changes_results(opts):
    """A plate pushed 0.3 mm into the two-layer bed over 300 steps: frozen
    order, a re-sort every rebuild, a scrambled start re-sorted every third
    rebuild, and skin lists re-sorted every second rebuild give bitwise equal
    states and contacts; the plate reactions agree to rounding."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = plate_bed(21)
    ref = Bed(spec, sort_every=-1)
    alt = Bed(spec, **opts)
    ref.step(300)
    alt.step(300)
    xa, va, wa = ref.state()
    xb, vb, wb = alt.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(wa, wb)
    assert np.array_equal(ref.contacts(), alt.contacts())
    Ra, Rb = ref.reaction(1), alt.reaction(1)
    np.testing.assert_allclose(Rb, Ra, rtol=1e-12, atol=1e-12 * abs(Ra[2]))
    st = alt.stats()
    print(opts, st)
    if opts.get("sort_every", 0) > 0:
        assert st["sorts"] > 0


def test_resorted_scrambled_bed_matches_oracle():
    """Storage starts in the caller's (shuffled) order and is re-sorted every
    rebuild while the plate moves the spheres; then one step against the
    oracle from the same state and spring history."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = plate_bed(22)
    bed = Bed(spec, record_forces=True, sort_every=1, input_order=True)
    bed.step(400)
    res = compare_one_step(spec, bed)
    print({k: v for k, v in res.items() if k not in ("only_gpu", "only_oracle")})
    assert_parity(res, 1e-5)
    assert bed.stats()["sorts"] >= 400


def test_resorting_is_deterministic_with_a_dynamic_body():
    """A dead-weight grousered ring (its z follows the FP64 reaction sums):
    two beds re-sorting every rebuild, one stepped by captured-graph cycles
    and one a step at a time, stay bitwise equal, reactions included."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = beds.add_ring(beds.two_layer_bed(23), r_in=0.012, r_out=0.024, grouser_len=0.012, grouser_thick=0.003,
                         grouser_depth=0.004, pressure=2e3, omega=5.0)
    spec.bodies[1].lin_vel = (0.0, 0.0, -1.0)
    a = Bed(spec, sort_every=2)
    b = Bed(spec, sort_every=2)
    a.step(600)
    for _ in range(600):
        b.step(1)
    xa, va, wa = a.state()
    xb, vb, wb = b.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(wa, wb)
    np.testing.assert_array_equal(a.reaction(1), b.reaction(1))
    np.testing.assert_array_equal(a.body(1)[0], b.body(1)[0])
    assert a.stats()["sorts"] == b.stats()["sorts"] == 300


def test_batch_resorts_each_bed_within_its_range():
    """Beds of a batch keep their storage ranges: a batch re-sorting every
    rebuild from scrambled orders steps each bed bitwise like the bed alone
    with a frozen order (prescribed plates)."""
    from paper_2501_05300_amd.lprdem import Batch, Bed
    specs = [plate_bed(24), beds.add_plate(beds.graded_bed(3000, r0=2e-3, L=0.04, k=2.0, depth=0.05, seed=25),
                                           diameter=0.03, speed=0.3)]
    batch = Batch(specs, sort_every=1, input_order=True)
    batch.step(150)
    for q, s in enumerate(specs):
        one = Bed(s, sort_every=-1)
        one.step(150)
        xa, va, _ = batch.state(bed=q)
        xb, vb, _ = one.state()
        assert np.array_equal(xa, xb) and np.array_equal(va, vb), q
        assert np.array_equal(batch.contacts(bed=q), one.contacts())
        one.close()


def test_lists_updated_in_place_equal_lists_rewritten_whole():
    """A rebuild that keeps the storage order updates the lists and springs in
    place, moving each carried spring to its new slot; one that re-sorts
    writes them whole into the other buffers.  A spinning, sinking grousered
    ring stirs the bed so that slots are inserted and dropped in the middle
    of the lists at every step: 800 steps either way are bitwise equal, and
    the lists changed at many rebuilds."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = beds.add_ring(beds.two_layer_bed(24), r_in=0.012, r_out=0.024, grouser_len=0.012, grouser_thick=0.003,
                         grouser_depth=0.004, pressure=2e3, omega=20.0)
    spec.bodies[1].lin_vel = (0.0, 0.0, -2.0)
    a = Bed(spec, sort_every=-1)
    b = Bed(spec, sort_every=1)
    changed = 0
    prev = None
    for _ in range(8):
        a.step(100)
        b.step(100)
        ca = a.contacts()
        assert np.array_equal(ca, b.contacts())
        (ka, ha), (kb, hb) = a.history(), b.history()
        assert np.array_equal(ka, kb) and np.array_equal(ha, hb)
        if prev is not None and not np.array_equal(prev, ca):
            changed += 1
        prev = ca
    xa, va, wa = a.state()
    xb, vb, wb = b.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(wa, wb)
    np.testing.assert_array_equal(a.reaction(1), b.reaction(1))
    assert changed >= 6
    assert a.stats()["sorts"] == 0 and b.stats()["sorts"] >= 800
