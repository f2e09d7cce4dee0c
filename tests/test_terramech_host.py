"""The accuracy metric of the plate test (CPU) against the paper's printed
numbers (tests/golden/aggregate_error_paper.json)."""
import json
import os

import pytest

from paper_2501_05300_amd import terramech as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "aggregate_error_paper.json")


def test_aggregate_error_reproduces_the_papers_ranges():
    """The four normalised errors built from each range's printed mean
    deviations average to the printed aggregate error (the paper averages
    per bed, so agreement is to its rounding, 0.15 percentage points)."""
    g = json.load(open(GOLDEN))
    ref = g["reference"]
    r = {"static_sinkage": ref["static_sinkage_mm"] * 1e-3, "dynamic_sinkage": ref["dynamic_sinkage_mm"] * 1e-3,
         "peak_traction": ref["peak_traction"], "average_traction": ref["average_traction"]}
    for name, dv in g["ranges"].items():
        m = {"static_sinkage": r["static_sinkage"] + dv["static_dev_mm"] * 1e-3,
             "dynamic_sinkage": r["dynamic_sinkage"] + dv["dynamic_dev_mm"] * 1e-3,
             "peak_traction": r["peak_traction"] * (1 + dv["peak_rel"]),
             "average_traction": r["average_traction"] * (1 - dv["average_rel"])}
        e = T.normalized_errors(m, r, g["h_grouser_m"], g["F_N_max_N"], g["F_N_max_N"])
        print(name, e)
        assert abs(e["aggregate"] - dv["aggregate"]) < 0.0015, (name, e["aggregate"])


def test_errors_are_signed_and_the_aggregate_takes_magnitudes():
    ref = {"static_sinkage": 1e-3, "dynamic_sinkage": 0.05, "peak_traction": 0.3, "average_traction": 0.3}
    m = {"static_sinkage": 0.5e-3, "dynamic_sinkage": 0.06, "peak_traction": 0.25, "average_traction": 0.35}
    e = T.normalized_errors(m, ref, 0.01, 200.0, 100.0)
    assert e["static_sinkage"] == pytest.approx(-0.05) and e["dynamic_sinkage"] == pytest.approx(1.0)
    assert e["peak_traction"] == pytest.approx(-0.025) and e["average_traction"] == pytest.approx(0.025)
    assert e["aggregate"] == pytest.approx((0.05 + 1.0 + 0.025 + 0.025) / 4)


def test_plate_load_is_the_pressure_over_the_area():
    p = T.Plate(length=0.1, width=0.06, pressure=5e4)
    assert p.load == pytest.approx(300.0)
    # the paper's plate: 2550 N is 50 kPa over its area
    assert 2550.0 / 5e4 == pytest.approx(0.051)
