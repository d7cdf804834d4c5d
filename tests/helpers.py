"""Small input builders shared by the tests (no method arithmetic here)."""
from __future__ import annotations

import json
import os

import numpy as np

from synth import Forests, Grid, make_patch

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_json(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def forests_from_dict(d) -> Forests:
    arr = lambda k, t=np.float64: np.asarray(d[k], t)
    real = d.get("realisation")
    return Forests(arr("offsets", np.int64), arr("ra"), arr("dec"), arr("dist"), arr("delta"),
                   arr("weight"), arr("loglam"),
                   None if real is None else np.asarray(real, np.int32),
                   int(d.get("n_realisations", 1)))


def grid_from_dict(d) -> Grid:
    return Grid(np.asarray(d["edges_par"], np.float64), np.asarray(d["edges_perp"], np.float64))


def truncate(F: Forests, k: int) -> Forests:
    """Keep at most the first k pixels of every forest."""
    idx, offs = [], [0]
    for f in range(F.n_forests):
        a, b = int(F.offsets[f]), int(F.offsets[f + 1])
        ids = np.arange(a, min(b, a + k))
        idx.append(ids)
        offs.append(offs[-1] + ids.shape[0])
    idx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
    return Forests(np.asarray(offs, np.int64), F.ra.copy(), F.dec.copy(), F.dist[idx], F.delta[idx],
                   F.weight[idx], F.loglam[idx],
                   None if F.realisation is None else F.realisation.copy(), F.n_realisations)


def tiny(seed=0, n_forests=3, k=7, width_deg=0.5, z_range=(2.1, 2.3)):
    """A few short forests packed close together so many pairs are in a 60 Mpc/h grid.

    Quasars below z = 2.46 all start their forests at 3600 A, so with this
    redshift range the forests overlap along the line of sight.
    """
    return truncate(make_patch(n_forests, width_deg, seed, z_range=z_range), k)
