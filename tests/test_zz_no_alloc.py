"""The per-contact read that allocates nothing (GPU): its output equals the
allocating read's, on two calls in a row, the second on a smaller bed (the
static workspace keeps the first call's contents)."""
import numpy as np
import pytest

from paper_2501_05300_amd import beds

pytestmark = pytest.mark.gpu


def loaded(spec, steps):
    from paper_2501_05300_amd.lprdem import Bed
    bed = Bed(spec, record_forces=True)
    bed.step(steps)
    bed.sync()
    return bed


def same(a, b):
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.array_equal(x, y)


def test_noalloc_read_equals_the_allocating_read():
    big = loaded(beds.add_plate(beds.two_layer_bed(31), diameter=0.04, speed=0.5), 1500)
    ref = big.contact_loads()
    assert len(ref[0]) > 200
    got = big.contact_loads_noalloc(len(ref[0]) + 10)
    same(got, ref)
    small = loaded(beds.two_layer_bed(32, n_fine=300, n_coarse=100), 1500)
    ref2 = small.contact_loads()
    assert 0 < len(ref2[0]) < len(ref[0])
    got2 = small.contact_loads_noalloc(len(ref2[0]))
    same(got2, ref2)


def test_noalloc_read_reports_a_short_buffer():
    from paper_2501_05300_amd.lprdem import CapacityError
    bed = loaded(beds.two_layer_bed(33), 100)
    n = len(bed.contacts())
    with pytest.raises(CapacityError):
        bed.contact_loads_noalloc(n - 1)
