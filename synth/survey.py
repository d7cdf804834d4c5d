"""Survey-shaped synthetic forests.

The shapes follow the paper's data description (Sec. 3.2, Table "forecast"):
quasars at 2.1 < z < 3.5 whose Lyman-alpha region (rest frame 1040-1200 A,
observed above 3600 A) is sampled either on a constant log10-wavelength step
(eBOSS-like) or on a constant linear step (DESI-like).  Distances are flat
LCDM comoving distances in Mpc/h.  Everything is drawn from a seeded numpy
Generator, so a (config, seed) pair always gives the same arrays.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

C_OVER_H0 = 2997.92458  # Mpc/h
LYA_REST = 1215.67      # Angstrom


@dataclass
class Forests:
    """Forests in CSR layout.

    offsets[f]..offsets[f+1] index the pixels of forest f.  Angles are radians,
    distances Mpc/h, loglam = ln(lambda / Angstrom).  ``realisation`` (int32
    per forest, or None) tags independent mock realisations; forests only pair
    within one realisation.
    """
    offsets: np.ndarray
    ra: np.ndarray
    dec: np.ndarray
    dist: np.ndarray
    delta: np.ndarray
    weight: np.ndarray
    loglam: np.ndarray
    realisation: Optional[np.ndarray] = None
    n_realisations: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def n_forests(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_pix(self) -> int:
        return int(self.offsets[-1])

    def real_of(self) -> np.ndarray:
        if self.realisation is None:
            return np.zeros(self.n_forests, np.int32)
        return self.realisation

    def forest_slice(self, f: int) -> slice:
        return slice(int(self.offsets[f]), int(self.offsets[f + 1]))

    def copy(self) -> "Forests":
        return Forests(
            self.offsets.copy(), self.ra.copy(), self.dec.copy(), self.dist.copy(),
            self.delta.copy(), self.weight.copy(), self.loglam.copy(),
            None if self.realisation is None else self.realisation.copy(),
            self.n_realisations, dict(self.meta))


@dataclass
class Grid:
    """Rectangular (r_par, r_perp) bin edges, strictly increasing, Mpc/h."""
    edges_par: np.ndarray
    edges_perp: np.ndarray

    @property
    def n_par(self) -> int:
        return int(self.edges_par.shape[0] - 1)

    @property
    def n_perp(self) -> int:
        return int(self.edges_perp.shape[0] - 1)

    @property
    def n_bins(self) -> int:
        return self.n_par * self.n_perp


def uniform_grid(n_par: int, r_par_max: float, n_perp: Optional[int] = None,
                 r_perp_max: Optional[float] = None) -> Grid:
    if n_perp is None:
        n_perp = n_par
    if r_perp_max is None:
        r_perp_max = r_par_max
    return Grid(np.linspace(0.0, r_par_max, n_par + 1),
                np.linspace(0.0, r_perp_max, n_perp + 1))


_DTAB = None


def comoving_distance(z: np.ndarray, omega_m: float = 0.315) -> np.ndarray:
    """Flat LCDM line-of-sight comoving distance in Mpc/h (radiation neglected)."""
    global _DTAB
    if _DTAB is None or _DTAB[0] != omega_m:
        zz = np.linspace(0.0, 6.0, 600001)
        inv_e = 1.0 / np.sqrt(omega_m * (1.0 + zz) ** 3 + (1.0 - omega_m))
        # cumulative trapezoid on a 1e-5 step: relative error ~1e-11
        d = np.concatenate([[0.0], np.cumsum(0.5 * (inv_e[1:] + inv_e[:-1]) * np.diff(zz))])
        _DTAB = (omega_m, zz, C_OVER_H0 * d)
    _, zz, d = _DTAB
    return np.interp(np.asarray(z, np.float64), zz, d)


def _sky_positions(rng, n, width_deg, ra0_deg=150.0, dec0_deg=0.0):
    """Area-uniform positions in a square-ish patch centred on (ra0, dec0)."""
    hw = np.deg2rad(width_deg) / 2.0
    dec0 = np.deg2rad(dec0_deg)
    s_lo, s_hi = np.sin(dec0 - hw), np.sin(dec0 + hw)
    dec = np.arcsin(rng.uniform(s_lo, s_hi, n))
    ra = np.deg2rad(ra0_deg) + rng.uniform(-hw, hw, n) / max(np.cos(dec0), 1e-3)
    return ra, dec


def _pixel_lambdas(z_q: float, n_want: int, model: str, lam_min_obs=3600.0,
                   rest=(1040.0, 1200.0), dlog10=3e-4, dlin=0.8):
    lo = max(lam_min_obs, rest[0] * (1.0 + z_q))
    hi = rest[1] * (1.0 + z_q)
    if hi <= lo:
        return np.zeros(0)
    if model == "log":
        n_av = int(np.floor(np.log10(hi / lo) / dlog10)) + 1
        n = min(n_want, n_av)
        return 10.0 ** (np.log10(lo) + dlog10 * np.arange(n))
    if model == "lin":
        n_av = int(np.floor((hi - lo) / dlin)) + 1
        n = min(n_want, n_av)
        return lo + dlin * np.arange(n)
    raise ValueError(model)


def make_patch(n_forests: int, width_deg: float, seed: int, *, model: str = "log",
               npix_range=(50, 150), z_range=(2.1, 3.5), delta_sigma: float = 0.3,
               ra0_deg: float = 150.0, dec0_deg: float = 0.0,
               delta_mode: str = "iid", grf_sigma2: float = 0.1, grf_R: float = 10.0,
               grf_cell: float = 4.0, noise_sigma: float = 1.0) -> Forests:
    """One realisation of a survey patch.

    delta_mode "iid": delta ~ N(0, delta_sigma^2) independently per pixel.
    delta_mode "grf": Gaussian-smoothed white noise (variance grf_sigma2,
    smoothing length grf_R Mpc/h, sampled trilinearly from a grf_cell grid)
    plus N(0, noise_sigma^2) pixel noise.
    Weights w = 1/(sigma^2 + 0.1) with sigma ~ U(0.1, 0.5).
    """
    rng = np.random.default_rng(seed)
    ra, dec = _sky_positions(rng, n_forests, width_deg, ra0_deg, dec0_deg)
    zq = rng.uniform(z_range[0], z_range[1], n_forests)
    nwant = rng.integers(npix_range[0], npix_range[1] + 1, n_forests)
    lams = [_pixel_lambdas(zq[f], int(nwant[f]), model) for f in range(n_forests)]
    counts = np.array([len(l) for l in lams], np.int64)
    offsets = np.zeros(n_forests + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    lam = np.concatenate(lams) if n_forests else np.zeros(0)
    zpix = lam / LYA_REST - 1.0
    dist = comoving_distance(zpix)
    loglam = np.log(lam)
    npix = lam.shape[0]
    sigma = rng.uniform(0.1, 0.5, npix)
    weight = 1.0 / (sigma * sigma + 0.1)
    if delta_mode == "iid":
        delta = rng.normal(0.0, delta_sigma, npix)
    elif delta_mode == "grf":
        fidx = np.repeat(np.arange(n_forests), counts)
        cd = np.cos(dec)
        nx, ny, nz = cd * np.cos(ra), cd * np.sin(ra), np.sin(dec)
        pos = np.stack([dist * nx[fidx], dist * ny[fidx], dist * nz[fidx]], -1)
        delta = _grf_sample(rng, pos, grf_sigma2, grf_R, grf_cell) + rng.normal(0.0, noise_sigma, npix)
    else:
        raise ValueError(delta_mode)
    return Forests(offsets, ra, dec, dist, delta, weight, loglam,
                   meta=dict(n_forests=n_forests, width_deg=width_deg, seed=seed, model=model,
                             delta_mode=delta_mode))


def _grf_sample(rng, pos, sigma2, R, cell):
    """Gaussian-smoothed white noise on a regular grid, trilinearly sampled.

    The smoothed field has correlation sigma2 * exp(-r^2 / (4 R^2)) (up to the
    grid's discreteness), used only for physics sanity checks.
    """
    lo = pos.min(0) - 3 * cell
    hi = pos.max(0) + 3 * cell
    shape = tuple(int(np.ceil((hi[k] - lo[k]) / cell)) + 2 for k in range(3))
    white = rng.standard_normal(shape, dtype=np.float32)
    fk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(shape[0], d=cell) * 2 * np.pi
    ky = np.fft.fftfreq(shape[1], d=cell) * 2 * np.pi
    kz = np.fft.rfftfreq(shape[2], d=cell) * 2 * np.pi
    k2 = (kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2).astype(np.float32)
    fk *= np.exp(-0.5 * k2 * R * R)
    del k2
    field = np.fft.irfftn(fk, s=shape, axes=(0, 1, 2)).astype(np.float32)
    del fk
    field *= np.float32(np.sqrt(sigma2) / max(field.std(), 1e-30))
    u = (pos - lo) / cell
    i0 = np.floor(u).astype(np.int64)
    t = u - i0
    out = np.zeros(pos.shape[0])
    for dx in (0, 1):
        wx = t[:, 0] if dx else 1 - t[:, 0]
        for dy in (0, 1):
            wy = t[:, 1] if dy else 1 - t[:, 1]
            for dz in (0, 1):
                wz = t[:, 2] if dz else 1 - t[:, 2]
                out += wx * wy * wz * field[i0[:, 0] + dx, i0[:, 1] + dy, i0[:, 2] + dz]
    return out


def subset_forests(F: Forests, idx: Sequence[int]) -> Forests:
    """A new Forests holding only forests idx (in that order)."""
    idx = np.asarray(idx, np.int64)
    counts = F.offsets[idx + 1] - F.offsets[idx]
    offsets = np.zeros(idx.shape[0] + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    pix = np.concatenate([np.arange(F.offsets[f], F.offsets[f + 1]) for f in idx]) if idx.size else np.zeros(0, np.int64)
    real = None if F.realisation is None else F.realisation[idx].copy()
    return Forests(offsets, F.ra[idx].copy(), F.dec[idx].copy(), F.dist[pix].copy(),
                   F.delta[pix].copy(), F.weight[pix].copy(), F.loglam[pix].copy(),
                   real, F.n_realisations, dict(F.meta, subset=len(idx)))


def nearest_to_centre(F: Forests, k: int) -> np.ndarray:
    """Indices of the k forests angularly closest to the patch's mean direction."""
    cd = np.cos(F.dec)
    v = np.stack([cd * np.cos(F.ra), cd * np.sin(F.ra), np.sin(F.dec)], -1)
    m = v.mean(0)
    m /= np.linalg.norm(m)
    return np.sort(np.argsort(-(v @ m), kind="stable")[:k])


def sky_cells(F: Forests, n_ra: int, n_dec: int) -> np.ndarray:
    """Subsample id of each forest: an n_ra x n_dec grid of equal-area cells
    (uniform in RA and in sin(Dec)) over the patch's extent, a stand-in for
    the sky pixels the paper subsamples in.  int32 in [0, n_ra * n_dec)."""
    ra, sd = F.ra, np.sin(F.dec)
    def idx(v, n):
        lo, hi = float(v.min()), float(v.max())
        k = np.floor((v - lo) / max(hi - lo, 1e-300) * n).astype(np.int64)
        return np.clip(k, 0, n - 1)
    return (idx(ra, n_ra) * n_dec + idx(sd, n_dec)).astype(np.int32)


def concat_realisations(parts: List[Forests]) -> Forests:
    offs = [np.zeros(1, np.int64)]
    base = 0
    for p in parts:
        offs.append(p.offsets[1:] + base)
        base += p.n_pix
    real = np.concatenate([np.full(p.n_forests, r, np.int32) for r, p in enumerate(parts)])
    cat = lambda name: np.concatenate([getattr(p, name) for p in parts])
    return Forests(np.concatenate(offs), cat("ra"), cat("dec"), cat("dist"), cat("delta"),
                   cat("weight"), cat("loglam"), real, len(parts),
                   meta=dict(n_realisations=len(parts)))
