"""Grousered plate under a dead weight on the GPU: one step against the
oracle, and the plate-test protocol end to end on a small refined bed."""
import numpy as np
import pytest

from paper_2501_05300_amd import beds
from paper_2501_05300_amd import terramech as T
from parity_util import assert_parity, compare_one_step

pytestmark = pytest.mark.gpu

SMALL = T.Plate(length=0.03, width=0.02, n_grousers=3, h_grouser=0.004, t_grouser=0.002, t_face=0.003,
                pressure=5e3)


def test_grouser_plate_step_matches_oracle():
    """Face and grouser boxes on a body free in z, moving along x."""
    from paper_2501_05300_amd.lprdem import Bed
    spec = T.add_grouser_plate(beds.two_layer_bed(0), SMALL, speed=0.2, vz0=-1.0)   # lands within the steps
    bed = Bed(spec, record_forces=True)
    bed.step(2100)
    res = compare_one_step(spec, bed)
    print(res)
    b = spec.info["plate_body"]
    assert_parity(res, 1e-5)
    assert abs(bed.reaction(b)[2]) > 0


@pytest.mark.timeout(300)
def test_protocol_on_a_small_refined_bed():
    spec = T.linear_bed(3e-3, 6e-3, 0.1, 0.04, 0.09, 0.06, seed=0)
    out = T.run_protocol(spec, SMALL, t_static=0.01, pull_speed=0.5, pull_distance=0.02, samples=20, log=print)
    # measured from grouser tips on the highest sphere under the plate, so the
    # face may sit below that reference; the lowering stops within three
    # grouser depths
    assert 0 < out["static_sinkage"] < 3 * SMALL.h_grouser
    assert out["dynamic_sinkage"] > 0
    tr = np.array(out["traction"])
    assert np.all(np.isfinite(tr)) and out["average_traction"] > 0
    assert out["peak_traction"] >= np.max(tr[: len(tr) // 3]) - 1e-12
    e = T.normalized_errors(out, out, SMALL.h_grouser, SMALL.load, SMALL.load)
    assert e["aggregate"] == 0.0
