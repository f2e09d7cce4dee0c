"""Batched form: many uneven beds in one launch per kernel (GPU)."""
import numpy as np
import pytest

from paper_2501_05300_amd import beds
from parity_util import assert_parity, compare_one_step, oracle_pairs

pytestmark = pytest.mark.gpu


def small_family():
    """Uneven beds: a two-layer bed, two graded beds of different grading and
    size, a uniform bed, each with its own plate."""
    out = [beds.add_plate(beds.two_layer_bed(11), diameter=0.03, speed=0.3),
           beds.add_plate(beds.graded_bed(6000, r0=1.5e-3, L=0.01, k=1.0, depth=0.05, seed=12), diameter=0.03,
                          speed=0.3),
           beds.add_plate(beds.graded_bed(3000, r0=2.0e-3, L=0.04, k=2.0, depth=0.05, seed=13), diameter=0.03,
                          speed=0.3),
           beds.add_plate(beds.uniform_bed(1500, r=2.5e-3, depth=0.04, seed=14), diameter=0.03, speed=0.3)]
    out[1].params = out[1].params.replace(mu_t=0.2)
    return out


def test_batch_matches_beds_stepped_alone():
    from paper_2501_05300_amd.lprdem import Batch, Bed
    specs = small_family()
    batch = Batch(specs)
    assert len(batch) == len(specs)
    batch.step(120)
    for q, s in enumerate(specs):
        single = Bed(s)
        single.step(120)
        xa, va, wa = batch.state(bed=q)
        xb, vb, wb = single.state()
        assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(wa, wb), q
        assert np.array_equal(batch.contacts(bed=q), single.contacts())
        np.testing.assert_array_equal(batch.reaction(1, bed=q), single.reaction(1))
        single.close()


def test_batch_bed_parity_with_oracle():
    from paper_2501_05300_amd.lprdem import Batch
    specs = small_family()
    batch = Batch(specs, record_forces=True)
    batch.step(200)

    class View:  # one bed of the batch seen through the single-bed helper
        def __init__(self, b, q):
            self.b, self.q = b, q

        def __getattr__(self, name):
            f = getattr(self.b, name)
            return lambda *a, **k: f(*a, bed=self.q, **k)

        def step(self, n):
            self.b.step(n)

    for q in (1, 2):
        res = compare_one_step(specs[q], View(batch, q))
        print(q, res)
        assert_parity(res, 1e-5)


@pytest.mark.parametrize("block,persistent", [(256, False), (128, True), (256, True), (64, True)])
def test_launch_shapes_give_identical_results(block, persistent):
    from paper_2501_05300_amd.lprdem import Batch
    specs = small_family()
    a = Batch(specs)
    b = Batch(specs)
    b.set_launch(block, persistent)
    a.step(60)
    b.step(60)
    for q in range(len(specs)):
        xa, va, _ = a.state(bed=q)
        xb, vb, _ = b.state(bed=q)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)


def test_autotuner_returns_a_working_setting():
    from paper_2501_05300_amd.lprdem import Batch, autotune
    specs = small_family()
    best, trials = autotune(specs, trial_steps=5)
    print(best)
    assert len(trials) >= 11 + 2  # layouts, launch shapes, then two cell factors per radius band
    assert best["ms_per_step"] > 0 and best["block"] in (64, 128, 256)
    ref = Batch(specs)
    tuned = Batch(specs, band_ratio=best["band_ratio"], cell_factor=best["cell_factor"], block=best["block"],
                  persistent=best["persistent"], level_cell_factor=best["level_cell_factor"])
    banded = Batch(specs, level_cell_factor=[1.5, 1.25, 1.5])   # one setting per radius band
    banded.step(30)
    ref.step(30)
    tuned.step(30)
    for q in range(len(specs)):
        assert np.array_equal(ref.contacts(bed=q), tuned.contacts(bed=q))
        assert np.array_equal(ref.contacts(bed=q), banded.contacts(bed=q))
        # per-particle sums run in stable-id order, whatever the layout
        xa, va, _ = ref.state(bed=q)
        xb, vb, _ = tuned.state(bed=q)
        xc, vc, _ = banded.state(bed=q)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb), q
        assert np.array_equal(xa, xc) and np.array_equal(va, vc), q


def test_full_batch_family_beds_match_the_oracle():
    """The 36-bed family of the batched benchmark (2.24M spheres, each bed
    under its own plate), stepped 40,000 times from placement as one batch
    with skin lists (bitwise the every-step search), so that thousands of
    contacts have formed in each bed (it is still settling): then one step of the smallest bed and of the bed
    nearest 100k spheres against the oracle, from the same state and springs,
    at the per-contact and per-particle bounds."""
    from paper_2501_05300_amd.lprdem import Batch
    specs = beds.batch_family()
    rmin = min(float(s.radius.min()) for s in specs)
    batch = Batch(specs, rebuild_every=10, skin=0.25 * rmin, record_forces=True)
    batch.step(40_000)
    batch.sync()
    sizes = [s.n for s in specs]
    picks = sorted({int(np.argmin(sizes)), int(np.argmin([abs(n - 100_000) for n in sizes]))})

    class View:  # one bed of the batch seen through the single-bed helper
        def __init__(self, b, q):
            self.b, self.q = b, q

        def __getattr__(self, name):
            f = getattr(self.b, name)
            return lambda *a, **k: f(*a, bed=self.q, **k)

        def step(self, n):
            self.b.step(n)

    for q in picks:
        res = compare_one_step(specs[q], View(batch, q))
        print(q, specs[q].n, {k: v for k, v in res.items() if k not in ("only_gpu", "only_oracle")})
        assert res["n_contacts"] >= 2000
        assert_parity(res, 1e-5)
