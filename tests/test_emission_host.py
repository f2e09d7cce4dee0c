"""Host logic of layer-by-layer emission (CPU): the layer plan against the
paper's layer construction, non-overlapping emission, and the diagnostics on
configurations whose answers are known in closed form."""
import math

import numpy as np
import pytest

from paper_2501_05300_amd import emission as E


@pytest.mark.parametrize("d_min,r,eta,n,h", [(8.5e-3, 1.234, 3.79, 6, 0.6), (3e-3, 2.0, 2.0, 2, 0.04)])
def test_plan_follows_the_layer_construction(d_min, r, eta, n, h):
    """Layer n (diameter r^n d_min, thickness eta d_n) has its bottom at depth
    eta d_0 (r^(n+1) - 1) / (r - 1) (the paper's geometric sum); layers are
    contiguous from the floor to the surface, the base is d_max = r^n d_min."""
    L = E.plan_layers(d_min, r, eta, n, h)
    assert len(L) == n + 1
    assert L[0].z_lo == 0.0 and math.isclose(L[-1].z_hi, h, rel_tol=1e-12)
    assert math.isclose(L[0].d, d_min * r ** n, rel_tol=1e-12)
    for a, b in zip(L, L[1:]):
        assert math.isclose(a.z_hi, b.z_lo, rel_tol=1e-12, abs_tol=1e-15)
    for k in range(n):                       # L[-1 - k] is layer k
        lay = L[-1 - k]
        assert math.isclose(lay.d, d_min * r ** k, rel_tol=1e-12)
        depth_bottom = eta * d_min * (r ** (k + 1) - 1.0) / (r - 1.0)
        assert math.isclose(h - lay.z_lo, depth_bottom, rel_tol=1e-12)
        assert math.isclose(lay.z_hi - lay.z_lo, eta * lay.d, rel_tol=1e-9)
    assert math.isclose(E.gamma_of(r, eta), (r - 1) / (r * eta))
    with pytest.raises(ValueError):
        E.plan_layers(d_min, r, eta, n, 0.5 * eta * d_min)


def test_emitted_spheres_never_overlap():
    rng = np.random.default_rng(0)
    side = 0.05
    lay = E.Layer(4e-3, 0.0, 0.01)
    n = E.emission_count(lay, side)
    pos, rad = E.emit(rng, lay, side, 0.02, n)
    assert len(rad) == n and pos.shape == (n, 3)
    assert np.all((pos[:, :2] >= 0) & (pos[:, :2] < side)) and np.all(pos[:, 2] > 0.02)
    assert np.all((rad >= 0.45 * lay.d - 1e-9) & (rad <= 0.55 * lay.d + 1e-9))
    r = rad.astype(np.float64)
    D = pos[None, :, :] - pos[:, None, :]
    D[..., :2] -= side * np.round(D[..., :2] / side)
    dist = np.linalg.norm(D, axis=2)
    gap = dist - (r[None, :] + r[:, None])
    np.fill_diagonal(gap, np.inf)
    assert gap.min() > 0.05 * lay.d


def test_emission_count_fills_the_layer():
    lay = E.Layer(3e-3, 0.0, 6e-3)
    n = E.emission_count(lay, 0.05, phi=0.6, excess=1.0)
    vol = n * (math.pi / 6) * E.EU3 * lay.d ** 3
    assert abs(vol / (0.05 ** 2 * 6e-3) - 0.6) < 0.01


def test_mixing_counts_spheres_below_their_layer():
    layers = [E.Layer(6e-3, 0.0, 0.02), E.Layer(3e-3, 0.02, 0.03)]
    rng = np.random.default_rng(1)
    z = np.concatenate([rng.uniform(0.003, 0.02, 100), rng.uniform(0.0201, 0.03, 50)])
    lay = np.concatenate([np.zeros(100, np.int32), np.ones(50, np.int32)])
    z[100:107] = 0.02 - 0.0016 - rng.uniform(0, 0.01, 7)   # 7 fine spheres deeper than half a diameter
    pos = np.stack([np.zeros_like(z), np.zeros_like(z), z], 1)
    m = E.mixing(pos, np.full(150, 1e-3), lay, layers)
    assert m[0] == 0.0 and math.isclose(m[1], 7 / 50)


def test_density_of_a_simple_cubic_lattice():
    """Spheres of radius r on a cubic lattice of spacing 2r: every slab of
    thickness 2r, at any offset, holds one sphere volume per column, so the
    bulk density is rho pi / 6."""
    r, side, rho = 1e-3, 0.02, 2200.0
    k = int(round(side / (2 * r)))
    g = (np.arange(k) + 0.5) * 2 * r
    X, Y, Z = np.meshgrid(g, g, (np.arange(20) + 0.5) * 2 * r, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    for off in (0.0, 0.37e-3, 1.3e-3):
        dens, _ = E.density_profile(pos, np.full(len(pos), r), rho, side, 0.004 + off, 0.004 + off + 10 * 2 * r, 10)
        np.testing.assert_allclose(dens, rho * math.pi / 6, rtol=1e-12)
