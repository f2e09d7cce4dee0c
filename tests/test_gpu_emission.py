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
