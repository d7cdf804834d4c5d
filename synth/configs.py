"""The five workload recipes, with the sizes and value models of the paper's
data (Sec. 3.2): eBOSS-like log-wavelength pixels, DESI-like linear pixels,
a many-realisation covariance run and a differentiable run.

Each recipe returns (forests, grid, extras).  ``scale`` < 1 shrinks the forest
count at constant sky density, giving the small versions the CPU tests use.
"""
from __future__ import annotations

import numpy as np

from .survey import concat_realisations, make_patch, uniform_grid

CONFIGS = {
    0: "plain FP64 xi: 100 forests, 5x5 deg, log pixels, 15x15 bins to 60 Mpc/h",
    1: "eBOSS-like: 30k forests over 400 deg^2, GRF + unit noise deltas, xi and D on 50x50 bins to 200",
    2: "DESI-like: 150k forests over 1000 deg^2, linear 0.8 A pixels, 300-700 per forest, xi on 50x50",
    3: "batched: 64 realisations of 2k-20k forests at 75 deg^-2, xi on 50x50",
    4: "differentiable xi: 10k forests over 100 deg^2, loss sum (xi - m)^2, m ~ U(-0.01, 0.01)",
}


def _width_for(n, density_per_deg2):
    return float(np.sqrt(n / density_per_deg2))


def make_config(cfg: int, seed: int = 0, scale: float = 1.0):
    extras = {}
    if cfg == 0:
        n = max(2, int(round(100 * scale)))
        F = make_patch(n, _width_for(n, 4.0), seed)
        G = uniform_grid(15, 60.0)
    elif cfg == 1:
        n = max(2, int(round(30000 * scale)))
        F = make_patch(n, _width_for(n, 75.0), seed, delta_mode="grf")
        G = uniform_grid(50, 200.0)
    elif cfg == 2:
        n = max(2, int(round(150000 * scale)))
        F = make_patch(n, _width_for(n, 150.0), seed, model="lin", npix_range=(300, 700))
        G = uniform_grid(50, 200.0)
        extras["project_deltas"] = True
    elif cfg == 3:
        rng = np.random.default_rng(seed + 7919)
        nr = max(1, int(round(64 * min(1.0, scale * 4))))
        lo, hi = max(2, int(2000 * scale)), max(3, int(20000 * scale))
        counts = rng.integers(lo, hi + 1, nr)
        parts = [make_patch(int(c), _width_for(int(c), 75.0), seed * 1000 + r)
                 for r, c in enumerate(counts)]
        F = concat_realisations(parts)
        G = uniform_grid(50, 200.0)
        extras["counts"] = counts
    elif cfg == 4:
        n = max(2, int(round(10000 * scale)))
        F = make_patch(n, _width_for(n, 100.0), seed)
        G = uniform_grid(50, 200.0)
        rng = np.random.default_rng(seed + 104729)
        extras["target"] = rng.uniform(-0.01, 0.01, G.n_bins)
    else:
        raise ValueError(cfg)
    F.meta["config"] = cfg
    return F, G, extras
