"""The seeded generator: determinism and the recipe's shapes (no method arithmetic)."""
import numpy as np

from synth import make_config, make_patch
from synth.survey import LYA_REST, comoving_distance


def test_deterministic_and_seed_dependent():
    a, _, _ = make_config(0, seed=3)
    b, _, _ = make_config(0, seed=3)
    c, _, _ = make_config(0, seed=4)
    for name in ("offsets", "ra", "dec", "dist", "delta", "weight", "loglam"):
        assert np.array_equal(getattr(a, name), getattr(b, name))
    assert not np.array_equal(a.delta, c.delta)


def test_pixel_model():
    F = make_patch(200, 3.0, 1)
    n = np.diff(F.offsets)
    assert n.max() <= 150 and n.min() >= 1
    lam = np.exp(F.loglam)
    assert lam.min() >= 3600.0 - 1e-9
    w = F.weight
    assert w.min() >= 1 / 0.35 - 1e-12 and w.max() <= 1 / 0.11 + 1e-12
    for f in range(F.n_forests):
        sl = F.forest_slice(f)
        assert np.all(np.diff(F.dist[sl]) > 0)  # blue-end runs, increasing lambda
        assert np.allclose(np.diff(np.log10(lam[sl])), 3e-4, rtol=1e-9)
    assert np.allclose(F.dist, comoving_distance(lam / LYA_REST - 1.0))
    L = make_patch(50, 3.0, 2, model="lin", npix_range=(300, 700))
    lam = np.exp(L.loglam)
    assert np.allclose(np.diff(lam[L.forest_slice(0)]), 0.8, rtol=1e-9)


def test_comoving_distance_limits():
    # low-z limit D ~ (c/H0) z, and flat LCDM value at z = 2 close to 3.6 Gpc/h
    assert abs(comoving_distance(1e-4) / (2997.92458 * 1e-4) - 1) < 1e-3
    assert 3500 < comoving_distance(2.0) < 3700


def test_batched_recipe():
    F, G, ex = make_config(3, seed=0, scale=0.02)
    assert F.n_realisations == len(ex["counts"])
    assert np.array_equal(np.bincount(F.realisation), ex["counts"])
