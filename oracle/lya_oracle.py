"""FP64 CPU oracle for the Lyman-alpha forest pair sums.

TEST INFRASTRUCTURE ONLY.  Nothing in the library may import, call or link
this module; only the tests, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code, constants or helpers with the HIP path; the
only thing both sides read is the seeded input generator (``synth``), which
contains none of the method's arithmetic.

Everything here is plain NumPy in float64, written from the paper:

* the two-point estimator xi_A = sum_A d_i w_i d_j w_j / sum_A w_i w_j over
  pixel pairs from different forests whose (r_par, r_perp) falls in the
  rectangular bin A (Sec. 2.1, eq. estimator_two);
* the distortion matrix D_AB = w_A^-1 sum_{ij in A} w_i w_j
  sum_{i'j' in B} eta_ii' eta_jj' with eta the per-forest continuum
  projection built from w and Lambda = log(lambda) (Sec. 2.2, eq. distortion
  and the eta definition that follows it);
* the gradient of xi with respect to delta and w, obtained by differentiating
  the estimator directly.

Where the paper is silent the oracle takes these readings:

* separations: r_par = |D_i - D_j| cos(theta/2), r_perp = (D_i + D_j)
  sin(theta/2), with sin(theta/2) = |n_f - n_g| / 2 from unit vectors
  (the decomposition of the pair separation about the mid line of sight; it
  satisfies r_par^2 + r_perp^2 = |x_i - x_j|^2);
* bins are half-open [e_k, e_{k+1}); the cut is rectangular; pairs are
  unordered (each pixel pair once);
* xi_A = 0 where sum w_i w_j = 0;
* eta uses the w-weighted mean of Lambda; the slope term is dropped when the
  weighted spread of Lambda vanishes (S <= 1e-24 W Lambda_bar^2); a forest
  with zero total weight keeps its deltas (it contributes nothing anyway);
* D uses a deterministic subset of forest pairs: (f, g) with f < g is kept iff
  splitmix64(seed XOR (f * 2^32 + g)) < floor(p * 2^64) (p = 1 keeps all);
  its normalisation w_A sums over the same kept pairs.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

IDENTITY, MEAN, MEAN_SLOPE = 0, 1, 2

# ---------------------------------------------------------------------------
# geometry (Sec. 2.1: separations parallel and perpendicular to the line of
# sight, in comoving coordinates)
# ---------------------------------------------------------------------------


def unit_vectors(ra, dec):
    """Unit vectors (cos dec cos ra, cos dec sin ra, sin dec), shape (N, 3)."""
    ra = np.asarray(ra, np.float64)
    dec = np.asarray(dec, np.float64)
    cd = np.cos(dec)
    return np.stack([cd * np.cos(ra), cd * np.sin(ra), np.sin(dec)], -1)


def pair_sc(nf, ng):
    """s = sin(theta/2) = |n_f - n_g| / 2 and c = cos(theta/2) = sqrt(1 - s^2).

    The chord form keeps full relative precision at small angles.
    """
    nf = np.asarray(nf, np.float64)
    ng = np.asarray(ng, np.float64)
    dx = nf[..., 0] - ng[..., 0]
    dy = nf[..., 1] - ng[..., 1]
    dz = nf[..., 2] - ng[..., 2]
    s = 0.5 * np.sqrt((dx * dx + dy * dy) + dz * dz)
    c = np.sqrt(1.0 - s * s)
    return s, c


def separations(Di, Dj, s, c):
    """(r_par, r_perp) of pixels at comoving distances Di, Dj (broadcasting)."""
    Di = np.asarray(Di, np.float64)
    Dj = np.asarray(Dj, np.float64)
    return np.abs(Di - Dj) * c, (Di + Dj) * s


def bin_index_1d(r, edges):
    """k with edges[k] <= r < edges[k+1]; -1 outside [edges[0], edges[-1])."""
    edges = np.asarray(edges, np.float64)
    k = np.searchsorted(edges, r, side="right") - 1
    k = np.where((k >= 0) & (k < edges.shape[0] - 1), k, -1)
    return k


def bin_index(rpar, rperp, grid):
    """Flat bin A = k_par * n_perp + k_perp, or -1 if outside the grid."""
    kp = bin_index_1d(rpar, grid.edges_par)
    kt = bin_index_1d(rperp, grid.edges_perp)
    return np.where((kp >= 0) & (kt >= 0), kp * grid.n_perp + kt, -1)


def near_edge(r, edges, tau):
    """True where r lies within tau of an edge other than a zero lower edge.

    Such pairs may legitimately bin differently under a different but equally
    valid rounding of the geometry; tests use this to recognise ties.
    """
    edges = np.asarray(edges, np.float64)
    e = edges[1:] if edges[0] == 0.0 else edges
    k = np.searchsorted(e, r)
    lo = np.abs(r - e[np.clip(k - 1, 0, e.shape[0] - 1)])
    hi = np.abs(e[np.clip(k, 0, e.shape[0] - 1)] - r)
    return np.minimum(lo, hi) <= tau


# ---------------------------------------------------------------------------
# forest pairs (Sec. 2.1: only pairs from different forests; the neighbour
# pre-ordering only decides which forests are visited, never the result)
# ---------------------------------------------------------------------------


def forest_extents(F):
    n = F.n_forests
    dmin = np.empty(n)
    dmax = np.empty(n)
    for f in range(n):
        sl = F.forest_slice(f)
        if sl.stop > sl.start:
            dmin[f] = F.dist[sl].min()
            dmax[f] = F.dist[sl].max()
        else:
            dmin[f] = np.inf
            dmax[f] = -np.inf
    return dmin, dmax


def forest_pairs(F, grid, prune=True):
    """All unordered (f, g), f < g, of one realisation; optionally pruned.

    The prune drops a pair only when no pixel pair can be in the grid: every
    r_perp >= (Dmin_f + Dmin_g) s and every r_par >= gap(f, g) c, evaluated
    with the same floating-point operations as the separations themselves, so
    the rounding is monotone and the cut is exact.
    """
    N = F.n_forests
    real = F.real_of()
    n = unit_vectors(F.ra, F.dec)
    dmin, dmax = forest_extents(F)
    out = []
    for f in range(N):
        g = np.arange(f + 1, N)
        g = g[real[g] == real[f]]
        g = g[(F.offsets[g + 1] > F.offsets[g])]
        if F.offsets[f + 1] == F.offsets[f] or g.size == 0:
            continue
        if prune:
            s, c = pair_sc(n[f][None, :], n[g])
            rperp_min = (dmin[f] + dmin[g]) * s
            gap = np.maximum(0.0, np.maximum(dmin[g] - dmax[f], dmin[f] - dmax[g]))
            rpar_min = gap * c
            keep = (rperp_min < grid.edges_perp[-1]) & (rpar_min < grid.edges_par[-1])
            g = g[keep]
        out.append(np.stack([np.full(g.shape[0], f, np.int64), g.astype(np.int64)], -1))
    if not out:
        return np.zeros((0, 2), np.int64)
    return np.concatenate(out, 0)


# ---------------------------------------------------------------------------
# eta: per-forest continuum projection (Sec. 2.2, the eta_ii' definition)
# ---------------------------------------------------------------------------


@dataclass
class EtaParams:
    W: float
    lbar: float
    S: float
    a: np.ndarray      # Lambda_i - Lambda_bar
    u: np.ndarray      # w_i / W
    b: np.ndarray      # w_i a_i / S (0 when the slope term is dropped)
    slope: bool


def eta_params(w, loglam, mode=MEAN_SLOPE) -> EtaParams:
    """Weighted sums that define eta_ii' = delta_ii' - u_i' - a_i b_i'."""
    w = np.asarray(w, np.float64)
    L = np.asarray(loglam, np.float64)
    n = w.shape[0]
    W = float(np.sum(w))
    if mode == IDENTITY or W == 0.0 or n == 0:
        z = np.zeros(n)
        return EtaParams(W, 0.0, 0.0, z, z.copy(), z.copy(), False)
    lbar = float(np.sum(w * L) / W)
    a = L - lbar
    S = float(np.sum(w * a * a))
    u = w / W
    slope = mode == MEAN_SLOPE and S > 1e-24 * W * lbar * lbar
    b = w * a / S if slope else np.zeros(n)
    return EtaParams(W, lbar, S, a, u, b, slope)


def eta_matrix(w, loglam, mode=MEAN_SLOPE):
    """Dense eta for one forest (brute-force reference)."""
    w = np.asarray(w, np.float64)
    n = w.shape[0]
    if mode == IDENTITY or n == 0 or np.sum(w) == 0.0:
        return np.eye(n)
    P = eta_params(w, loglam, mode)
    eta = np.eye(n) - P.u[None, :]
    if P.slope:
        eta = eta - P.a[:, None] * P.b[None, :]
    return eta


def project_forest(delta, w, loglam, mode=MEAN_SLOPE):
    """(eta delta)_i = delta_i - sum_i' u_i' delta_i' - a_i sum_i' b_i' delta_i'."""
    delta = np.asarray(delta, np.float64)
    if mode == IDENTITY:
        return delta.copy()
    P = eta_params(w, loglam, mode)
    if P.W == 0.0:
        return delta.copy()
    out = delta - np.sum(P.u * delta)
    if P.slope:
        out = out - P.a * np.sum(P.b * delta)
    return out


def projected_deltas(F, mode=MEAN_SLOPE):
    out = np.empty_like(F.delta)
    for f in range(F.n_forests):
        sl = F.forest_slice(f)
        out[sl] = project_forest(F.delta[sl], F.weight[sl], F.loglam[sl], mode)
    return out


# ---------------------------------------------------------------------------
# compensated accumulation of per-forest partial histograms
# ---------------------------------------------------------------------------


class _Neumaier:
    """Element-wise Neumaier (improved Kahan) summation of arrays."""

    def __init__(self, shape):
        self.s = np.zeros(shape)
        self.c = np.zeros(shape)

    def add(self, x, where=None):
        if where is not None:
            s = self.s[where]
            t = s + x
            self.c[where] += np.where(np.abs(s) >= np.abs(x), (s - t) + x, (x - t) + s)
            self.s[where] = t
            return
        t = self.s + x
        self.c += np.where(np.abs(self.s) >= np.abs(x), (self.s - t) + x, (x - t) + self.s)
        self.s = t

    def value(self):
        return self.s + self.c


# ---------------------------------------------------------------------------
# xi sums (Sec. 2.1, eq. estimator_two)
# ---------------------------------------------------------------------------


@dataclass
class XiSums:
    num: np.ndarray      # [R, n_bins]  sum w_i d_i w_j d_j
    wsum: np.ndarray     # [R, n_bins]  sum w_i w_j
    npairs: np.ndarray   # [R, n_bins]  pair counts (int64)
    absnum: np.ndarray   # [R, n_bins]  sum |w_i d_i w_j d_j| (conditioning)
    n_near_edge: int     # pairs within edge_tau * max(1, r) of an interior or upper edge
    rpsum: Optional[np.ndarray] = None   # [R, n_bins]  sum w_i w_j r_par      (means=True)
    rtsum: Optional[np.ndarray] = None   # [R, n_bins]  sum w_i w_j r_perp
    zsum: Optional[np.ndarray] = None    # [R, n_bins]  sum w_i w_j (z_i + z_j) / 2

    @property
    def xi(self):
        return xi_from_sums(self.num, self.wsum)


LYA_ALPHA_ANGSTROM = 1215.67   # rest wavelength of the Lyman-alpha transition


def pixel_redshift(loglam):
    """z of a forest pixel: lambda / lambda_Lya - 1 with lambda = exp(loglam) in
    Angstrom (natural log; only the bin-mean redshift needs the base)."""
    return np.exp(np.asarray(loglam, np.float64)) / LYA_ALPHA_ANGSTROM - 1.0


def bin_means(X: "XiSums"):
    """Weighted bin-mean coordinates (the r_par, r_perp and z columns of the
    correlation output that a model fitter reads next to xi):
    sum w_i w_j r / sum w_i w_j per bin, 0 where the bin is empty."""
    def mean(t):
        out = np.zeros_like(t)
        nz = X.wsum != 0.0
        out[nz] = t[nz] / X.wsum[nz]
        return out
    return mean(X.rpsum), mean(X.rtsum), mean(X.zsum)


def xi_from_sums(num, wsum):
    num = np.asarray(num, np.float64)
    wsum = np.asarray(wsum, np.float64)
    out = np.zeros_like(num)
    nz = wsum != 0.0
    out[nz] = num[nz] / wsum[nz]
    return out


def _partner_arrays(F, g_list, n_vec, nf_vec):
    """Concatenate the pixels of forests g_list with their per-pair (s, c)."""
    starts = F.offsets[g_list]
    counts = F.offsets[g_list + 1] - starts
    idx = np.concatenate([np.arange(a, a + k) for a, k in zip(starts, counts)])
    s, c = pair_sc(nf_vec[None, :], n_vec[g_list])
    return idx, np.repeat(s, counts), np.repeat(c, counts)


def _chunks_by_pixels(F, g_list, budget):
    out, cur, tot = [], [], 0
    for g in g_list:
        k = int(F.offsets[g + 1] - F.offsets[g])
        if cur and tot + k > budget:
            out.append(np.array(cur, np.int64))
            cur, tot = [], 0
        cur.append(g)
        tot += k
    if cur:
        out.append(np.array(cur, np.int64))
    return out


def xi_sums(F, grid, *, project=False, eta_mode=MEAN_SLOPE, prune=True,
            edge_tau=1e-12, pairs=None, chunk_elems=2_000_000, sub=None, n_sub=1,
            means=False) -> XiSums:
    """Pair sums of eq. estimator_two for every realisation.

    For each forest f the pixels of all its partners g > f are concatenated
    and the n_f x sum(n_g) separations are binned at once; the per-forest
    partial histograms are combined with Neumaier summation so the result is
    accurate to a few ulps of sum |terms| per bin.

    With `sub` (one subsample id in [0, n_sub) per forest) the sums are split
    by subsample: every pair (f, g), f < g, goes to slab r * n_sub + sub[f]
    (the errors of Sec. 2.1 and of the 3PCF figure come from subsamples of the
    forests in sky pixels); the first axis of the outputs is then R * n_sub.

    With `means`, also the weighted coordinate sums sum w_i w_j r_par,
    sum w_i w_j r_perp and sum w_i w_j (z_i + z_j) / 2 per bin (``bin_means``).
    """
    n_sub = int(n_sub) if sub is not None else 1
    R = max(1, int(F.n_realisations)) * n_sub
    nb = grid.n_bins
    delta = projected_deltas(F, eta_mode) if project else F.delta
    wd = F.weight * delta
    n_vec = unit_vectors(F.ra, F.dec)
    real = F.real_of()
    num = _Neumaier((R, nb))
    wsum = _Neumaier((R, nb))
    absn = _Neumaier((R, nb))
    npairs = np.zeros((R, nb), np.int64)
    msum = [_Neumaier((R, nb)) for _ in range(3)] if means else None
    zpix = pixel_redshift(F.loglam) if means else None
    n_near = 0

    def result():
        X = XiSums(num.value(), wsum.value(), npairs, absn.value(), n_near)
        if means:
            X.rpsum, X.rtsum, X.zsum = (m.value() for m in msum)
        return X

    if pairs is None:
        pairs = forest_pairs(F, grid, prune)
    if pairs.shape[0] == 0:
        return result()
    order = np.argsort(pairs[:, 0], kind="stable")
    pairs = pairs[order]
    firsts, starts = np.unique(pairs[:, 0], return_index=True)
    ends = np.append(starts[1:], pairs.shape[0])
    for f, a, b in zip(firsts, starts, ends):
        sl = F.forest_slice(int(f))
        nf = sl.stop - sl.start
        r = int(real[f]) * n_sub + (int(sub[f]) if sub is not None else 0)
        budget = max(1, chunk_elems // max(nf, 1))
        for gch in _chunks_by_pixels(F, pairs[a:b, 1], budget):
            idx, s, c = _partner_arrays(F, gch, n_vec, n_vec[f])
            rpar, rperp = separations(F.dist[sl][:, None], F.dist[idx][None, :], s[None, :], c[None, :])
            A = bin_index(rpar, rperp, grid)
            m = A >= 0
            if edge_tau > 0:
                near = (near_edge(rpar, grid.edges_par, edge_tau * np.maximum(1.0, rpar))
                        | near_edge(rperp, grid.edges_perp, edge_tau * np.maximum(1.0, rperp)))
                inside = (rpar < grid.edges_par[-1] + 1.0) & (rperp < grid.edges_perp[-1] + 1.0)
                n_near += int(np.count_nonzero(near & inside))
            Am = A[m]
            prod = (wd[sl][:, None] * wd[idx][None, :])[m]
            ww = (F.weight[sl][:, None] * F.weight[idx][None, :])[m]
            num.add(np.bincount(Am, weights=prod, minlength=nb), where=(r,))
            wsum.add(np.bincount(Am, weights=ww, minlength=nb), where=(r,))
            absn.add(np.bincount(Am, weights=np.abs(prod), minlength=nb), where=(r,))
            npairs[r] += np.bincount(Am, minlength=nb)
            if means:
                zz = (0.5 * (zpix[sl][:, None] + zpix[idx][None, :]))[m]
                for acc, v in zip(msum, (rpar[m], rperp[m], zz)):
                    acc.add(np.bincount(Am, weights=ww * v, minlength=nb), where=(r,))
    return result()


def covariance(num, wsum):
    """Subsample covariance of xi from [n_sub, n_bins] sums: with totals
    N_A, W_A and xi_A = N_A / W_A (0 where W_A = 0),
      C_AB = sum_s W_sA W_sB (xi_sA - xi_A)(xi_sB - xi_B) / (W_A W_B),
    written as sum_s x_sA x_sB / (W_A W_B) with x_sA = N_sA - W_sA xi_A, and 0
    where W_A W_B = 0.  The paper estimates its errors from subsamples of the
    forests in sky pixels (Sec. 2.1, the 3PCF figure) without printing the
    formula; this weighted form is the reading."""
    num = np.asarray(num, np.float64)
    wsum = np.asarray(wsum, np.float64)
    N = num.sum(axis=0)
    W = wsum.sum(axis=0)
    xi = np.where(W != 0, N / np.where(W != 0, W, 1.0), 0.0)
    x = num - wsum * xi[None, :]
    d = np.outer(W, W)
    cov = np.where(d != 0, (x.T @ x) / np.where(d != 0, d, 1.0), 0.0)
    return xi, cov


def xi_pairs_brute(F, grid, delta=None):
    """Pure-Python triple loop over pixel pairs of different forests (tiny inputs)."""
    import math
    R = max(1, int(F.n_realisations))
    nb = grid.n_bins
    if delta is None:
        delta = F.delta
    real = F.real_of()
    n = unit_vectors(F.ra, F.dec)
    num = [[[] for _ in range(nb)] for _ in range(R)]
    ws = [[[] for _ in range(nb)] for _ in range(R)]
    cnt = np.zeros((R, nb), np.int64)
    N = F.n_forests
    for f in range(N):
        for g in range(f + 1, N):
            if real[f] != real[g]:
                continue
            s, c = pair_sc(n[f], n[g])
            s, c = float(s), float(c)
            for i in range(F.offsets[f], F.offsets[f + 1]):
                for j in range(F.offsets[g], F.offsets[g + 1]):
                    rpar = abs(float(F.dist[i]) - float(F.dist[j])) * c
                    rperp = (float(F.dist[i]) + float(F.dist[j])) * s
                    kp = int(bin_index_1d(np.array([rpar]), grid.edges_par)[0])
                    kt = int(bin_index_1d(np.array([rperp]), grid.edges_perp)[0])
                    if kp < 0 or kt < 0:
                        continue
                    A = kp * grid.n_perp + kt
                    rr = int(real[f])
                    num[rr][A].append(float(F.weight[i]) * float(delta[i]) * float(F.weight[j]) * float(delta[j]))
                    ws[rr][A].append(float(F.weight[i]) * float(F.weight[j]))
                    cnt[rr, A] += 1
    N_ = np.array([[math.fsum(v) for v in row] for row in num])
    W_ = np.array([[math.fsum(v) for v in row] for row in ws])
    return N_, W_, cnt


# ---------------------------------------------------------------------------
# distortion matrix (Sec. 2.2, eq. distortion)
# ---------------------------------------------------------------------------


def xi_means_brute(F, grid):
    """Bin-mean r_par, r_perp and z by a pure-Python loop over pixel pairs
    (tiny inputs), with the separations taken from the 3-D positions
    x = D n: r_par = |(x_j - x_i) . m| along the mid line of sight
    m = (n_f + n_g) / |n_f + n_g| and r_perp the length of the rest."""
    import math
    R = max(1, int(F.n_realisations))
    nb = grid.n_bins
    real = F.real_of()
    n = unit_vectors(F.ra, F.dec)
    z = pixel_redshift(F.loglam)
    acc = {k: [[[] for _ in range(nb)] for _ in range(R)] for k in ("w", "rp", "rt", "z")}
    for f in range(F.n_forests):
        for g in range(f + 1, F.n_forests):
            if real[f] != real[g]:
                continue
            mid = n[f] + n[g]
            mid = mid / math.sqrt(float(np.dot(mid, mid)))
            for i in range(F.offsets[f], F.offsets[f + 1]):
                for j in range(F.offsets[g], F.offsets[g + 1]):
                    sep = F.dist[j] * n[g] - F.dist[i] * n[f]
                    along = float(np.dot(sep, mid))
                    rest = sep - along * mid
                    rpar, rperp = abs(along), math.sqrt(float(np.dot(rest, rest)))
                    kp = int(bin_index_1d(np.array([rpar]), grid.edges_par)[0])
                    kt = int(bin_index_1d(np.array([rperp]), grid.edges_perp)[0])
                    if kp < 0 or kt < 0:
                        continue
                    A, r = kp * grid.n_perp + kt, int(real[f])
                    ww = float(F.weight[i]) * float(F.weight[j])
                    acc["w"][r][A].append(ww)
                    acc["rp"][r][A].append(ww * rpar)
                    acc["rt"][r][A].append(ww * rperp)
                    acc["z"][r][A].append(ww * 0.5 * (z[i] + z[j]))
    tot = {k: np.array([[math.fsum(v) for v in row] for row in a]) for k, a in acc.items()}
    W = tot["w"]
    out = []
    for k in ("rp", "rt", "z"):
        m = np.zeros_like(W)
        m[W != 0] = tot[k][W != 0] / W[W != 0]
        out.append(m)
    return tuple(out)


def splitmix64(x):
    """SplitMix64 output for state x (Steele, Lea & Flood 2014; Vigna's
    reference form): z = x + 0x9E3779B97F4A7C15, then two xor-shift-multiply
    rounds and a final xor-shift.  uint64 arrays, wrapping arithmetic."""
    x = np.asarray(x, np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def keep_threshold(p):
    """floor(p * 2^64) as a Python int (None means keep every pair)."""
    if p >= 1.0:
        return None
    return int(np.ldexp(np.float64(p), 64))


def keep_pair_mask(f, g, p, seed):
    thr = keep_threshold(p)
    f = np.asarray(f, np.uint64)
    g = np.asarray(g, np.uint64)
    if thr is None:
        return np.ones(np.broadcast(f, g).shape, bool)
    key = (f << np.uint64(32)) | g
    h = splitmix64(np.uint64(seed) ^ key)
    return h < np.uint64(thr)


def dmat_pairs(F, grid, keep_fraction=1.0, seed=0, prune=True):
    pairs = forest_pairs(F, grid, prune)
    if pairs.shape[0] == 0:
        return pairs
    return pairs[keep_pair_mask(pairs[:, 0], pairs[:, 1], keep_fraction, seed)]


def _pair_bins(F, grid, f, g, n_vec):
    sf, sg = F.forest_slice(f), F.forest_slice(g)
    s, c = pair_sc(n_vec[f], n_vec[g])
    rpar, rperp = separations(F.dist[sf][:, None], F.dist[sg][None, :], s, c)
    return bin_index(rpar, rperp, grid)


@dataclass
class DmatResult:
    num: np.ndarray   # [R, nb, nb]
    wd: np.ndarray    # [R, nb]

    @property
    def D(self):
        out = np.zeros_like(self.num)
        nz = self.wd != 0.0
        for r in range(self.num.shape[0]):
            out[r][nz[r]] = self.num[r][nz[r]] / self.wd[r][nz[r]][:, None]
        return out


def dmat_brute(F, grid, pairs, eta_mode=MEAN_SLOPE):
    """Eq. distortion written out as four nested sums (tiny inputs only)."""
    R = max(1, int(F.n_realisations))
    nb = grid.n_bins
    num = np.zeros((R, nb, nb))
    wd = np.zeros((R, nb))
    real = F.real_of()
    n_vec = unit_vectors(F.ra, F.dec)
    for f, g in pairs:
        f, g = int(f), int(g)
        r = int(real[f])
        sf, sg = F.forest_slice(f), F.forest_slice(g)
        A = _pair_bins(F, grid, f, g, n_vec)
        ef = eta_matrix(F.weight[sf], F.loglam[sf], eta_mode)
        eg = eta_matrix(F.weight[sg], F.loglam[sg], eta_mode)
        wf, wg = F.weight[sf], F.weight[sg]
        nf, ng = wf.shape[0], wg.shape[0]
        for i in range(nf):
            for j in range(ng):
                a = A[i, j]
                if a < 0:
                    continue
                wd[r, a] += wf[i] * wg[j]
                for ip in range(nf):
                    for jp in range(ng):
                        b = A[ip, jp]
                        if b < 0:
                            continue
                        num[r, a, b] += wf[i] * wg[j] * ef[i, ip] * eg[j, jp]
    return DmatResult(num, wd)


def dmat_definition(F, grid, pairs, eta_mode=MEAN_SLOPE):
    """Eq. distortion with the inner double sum done as eta_f M^B eta_g^T.

    M^B[i', j'] = 1 when pixel pair (i', j') falls in bin B, so
    sum_{i'j' in B} eta_ii' eta_jj' = (eta_f M^B eta_g^T)[i, j]; the outer
    sum over (i, j) in A is then a weighted histogram.  Small inputs only.
    """
    R = max(1, int(F.n_realisations))
    nb = grid.n_bins
    num = np.zeros((R, nb, nb))
    wd = np.zeros((R, nb))
    real = F.real_of()
    n_vec = unit_vectors(F.ra, F.dec)
    for f, g in pairs:
        f, g = int(f), int(g)
        r = int(real[f])
        sf, sg = F.forest_slice(f), F.forest_slice(g)
        A = _pair_bins(F, grid, f, g, n_vec)
        m = A >= 0
        if not m.any():
            continue
        ef = eta_matrix(F.weight[sf], F.loglam[sf], eta_mode)
        eg = eta_matrix(F.weight[sg], F.loglam[sg], eta_mode)
        ww = F.weight[sf][:, None] * F.weight[sg][None, :]
        wd[r] += np.bincount(A[m], weights=ww[m], minlength=nb)
        for B in np.unique(A[m]):
            MB = (A == B).astype(np.float64)
            PB = ef @ MB @ eg.T
            num[r, :, B] += np.bincount(A[m], weights=(ww * PB)[m], minlength=nb)
    return DmatResult(num, wd)


def dmat(F, grid, pairs, eta_mode=MEAN_SLOPE):
    """Eq. distortion in factorised form (pinned against the two above).

    With eta_ii' = delta_ii' - p_i . q_i', p_i = (1, a_i), q_i' = (u_i', b_i'):
      num_AB = w_A^{fg} delta_AB
             - sum_i w_i sum_l R^l_i[A] G^l_i[B]     (i fixed, j and j' vary)
             - sum_j w_j sum_k C^k_j[A] F^k_j[B]     (j fixed, i and i' vary)
             + sum_kl H^kl_A Q^kl_B
    R^l_i[A] = sum_{j: beta(i,j)=A} w_j p_j^l, G^l_i[B] = sum_{j': beta(i,j')=B} q_j'^l,
    C, F likewise over i, H^kl_A = sum_{beta=A} w_i p_i^k w_j p_j^l,
    Q^kl_B = sum_{beta=B} q_i^k q_j^l.
    """
    R_ = max(1, int(F.n_realisations))
    nb = grid.n_bins
    num = np.zeros((R_, nb, nb))
    wd = np.zeros((R_, nb))
    real = F.real_of()
    n_vec = unit_vectors(F.ra, F.dec)
    cache = {}

    def params(f):
        if f not in cache:
            sl = F.forest_slice(f)
            P = eta_params(F.weight[sl], F.loglam[sl], eta_mode)
            w = F.weight[sl]
            if eta_mode == IDENTITY or P.W == 0.0:
                p = np.zeros((w.shape[0], 2))
                q = np.zeros((w.shape[0], 2))
            else:
                p = np.stack([np.ones(w.shape[0]), P.a], -1)
                q = np.stack([P.u, P.b], -1)
            cache[f] = (w, p, q)
        return cache[f]

    for f, g in pairs:
        f, g = int(f), int(g)
        r = int(real[f])
        A = _pair_bins(F, grid, f, g, n_vec)
        m = A >= 0
        if not m.any():
            continue
        wf, pf, qf = params(f)
        wg, pg, qg = params(g)
        nf, ng = wf.shape[0], wg.shape[0]
        touched = np.unique(A[m])
        T = touched.shape[0]
        loc = np.full(nb, -1, np.int64)
        loc[touched] = np.arange(T)
        ii, jj = np.nonzero(m)
        la = loc[A[ii, jj]]
        row_key = ii * T + la
        col_key = jj * T + la
        blk = np.zeros((T, T))
        for l in range(2):
            Rl = np.bincount(row_key, weights=wg[jj] * pg[jj, l], minlength=nf * T).reshape(nf, T)
            Gl = np.bincount(row_key, weights=qg[jj, l], minlength=nf * T).reshape(nf, T)
            blk -= (Rl * wf[:, None]).T @ Gl
            Cl = np.bincount(col_key, weights=wf[ii] * pf[ii, l], minlength=ng * T).reshape(ng, T)
            Fl = np.bincount(col_key, weights=qf[ii, l], minlength=ng * T).reshape(ng, T)
            blk -= (Cl * wg[:, None]).T @ Fl
        H00 = None
        for k in range(2):
            for l in range(2):
                H = np.bincount(la, weights=wf[ii] * pf[ii, k] * wg[jj] * pg[jj, l], minlength=T)
                Q = np.bincount(la, weights=qf[ii, k] * qg[jj, l], minlength=T)
                blk += np.outer(H, Q)
        H00 = np.bincount(la, weights=wf[ii] * wg[jj], minlength=T)
        blk[np.arange(T), np.arange(T)] += H00
        num[r][np.ix_(touched, touched)] += blk
        wd[r, touched] += H00
    return DmatResult(num, wd)


# ---------------------------------------------------------------------------
# gradient of xi (differentiating eq. estimator_two)
# ---------------------------------------------------------------------------


def xi_grad(F, grid, grad_xi, xi, wsum, pairs=None, prune=True):
    """Back-propagate dL/dxi_A to delta and w (deltas taken as given).

    With gamma_A = (dL/dxi_A) / W_A (0 where W_A = 0):
      dL/d delta_i = w_i sum_j gamma_{beta(i,j)} w_j delta_j
      dL/d w_i     = sum_j gamma_{beta(i,j)} w_j (delta_i delta_j - xi_{beta(i,j)})
    summed over every partner pixel j of every other forest (both orders).
    """
    R = max(1, int(F.n_realisations))
    nb = grid.n_bins
    grad_xi = np.asarray(grad_xi, np.float64).reshape(R, nb)
    xi = np.asarray(xi, np.float64).reshape(R, nb)
    wsum = np.asarray(wsum, np.float64).reshape(R, nb)
    gamma = np.zeros((R, nb))
    nz = wsum != 0.0
    gamma[nz] = grad_xi[nz] / wsum[nz]
    gx = gamma * xi
    gd = np.zeros(F.n_pix)
    gw = np.zeros(F.n_pix)
    real = F.real_of()
    n_vec = unit_vectors(F.ra, F.dec)
    if pairs is None:
        pairs = forest_pairs(F, grid, prune)
    wdel = F.weight * F.delta
    for f, g in pairs:
        f, g = int(f), int(g)
        r = int(real[f])
        sf, sg = F.forest_slice(f), F.forest_slice(g)
        A = _pair_bins(F, grid, f, g, n_vec)
        m = A >= 0
        if not m.any():
            continue
        Ac = np.where(m, A, 0)
        Gm = np.where(m, gamma[r][Ac], 0.0)
        GXm = np.where(m, gx[r][Ac], 0.0)
        t_f = Gm @ wdel[sg]
        t_g = Gm.T @ wdel[sf]
        gd[sf] += F.weight[sf] * t_f
        gd[sg] += F.weight[sg] * t_g
        gw[sf] += F.delta[sf] * t_f - GXm @ F.weight[sg]
        gw[sg] += F.delta[sg] * t_g - GXm.T @ F.weight[sf]
    return gd, gw


def projection_jacobians(delta, w, loglam, mode=MEAN_SLOPE):
    """Jacobians of one forest's projected deltas delta' = eta(w, Lambda) delta
    (Sec. 2.2, the eta definition) with respect to delta and to w.

    J_delta = eta.  J_w[i, k] = sum_i' (d eta_ii' / d w_k) delta_i', each
    entry of eta differentiated as written, with every w-dependent quantity
    moving: W = sum w, Lambda_bar = sum w Lambda / W (so a_i moves by
    -a_k / W), S = sum w a^2.  Identity mode, W = 0 and a dropped slope term
    follow the same readings as the forward projection (the branch in use is
    differentiated).
    """
    delta = np.asarray(delta, np.float64)
    w = np.asarray(w, np.float64)
    L = np.asarray(loglam, np.float64)
    n = delta.shape[0]
    P = eta_params(w, L, mode)
    if mode == IDENTITY or n == 0 or P.W == 0.0:
        return np.eye(n), np.zeros((n, n))
    W, a, S = P.W, P.a, P.S
    da = -a[None, :] / W                          # da_i / dw_k (same for every i)
    dS = a * a + 2.0 * np.sum(w * a) * da[0]      # dS / dw_k = a_k^2 + sum_l 2 w_l a_l da_l/dw_k
    # mean term: eta_ii' contains -w_i' / W
    #   d/dw_k (-w_i' / W) = -[i' = k] / W + w_i' / W^2
    Jw = -np.ones((n, 1)) * delta[None, :] / W + np.sum(w * delta) / (W * W)
    if P.slope:
        # slope term: eta_ii' contains -a_i w_i' a_i' / S
        wad = np.sum(w * a * delta)               # sum_i' w_i' a_i' delta_i'
        wd = np.sum(w * delta)
        for k in range(n):
            d_term = (da[0, k] * wad                        # d a_i
                      + a * a[k] * delta[k]                 # d w_i' at i' = k
                      + a * da[0, k] * wd                   # d a_i'
                      ) / S - a * wad * dS[k] / (S * S)     # d S
            Jw[:, k] -= d_term
    return eta_matrix(w, L, mode), Jw


def xi_grad_projected(F, grid, grad_xi, xi, wsum, eta_mode=MEAN_SLOPE, pairs=None, prune=True):
    """Gradient of L(xi) with respect to the raw delta and w when xi is built
    from the projected deltas delta' = eta delta of each forest (the forward
    of ``xi_sums(..., project=True)``).

    The chain rule with explicit per-forest Jacobians: with g' = dL/d delta'
    and h' = dL/dw at fixed delta' (``xi_grad`` on the projected deltas),
      dL/d delta = J_delta^T g',   dL/dw = h' + J_w^T g'.
    xi and wsum are those of the projected forward.
    """
    Fp = F.copy()
    Fp.delta = projected_deltas(F, eta_mode)
    gp, hp = xi_grad(Fp, grid, grad_xi, xi, wsum, pairs=pairs, prune=prune)
    gd = np.zeros(F.n_pix)
    gw = hp.copy()
    for f in range(F.n_forests):
        sl = F.forest_slice(f)
        Jd, Jw = projection_jacobians(F.delta[sl], F.weight[sl], F.loglam[sl], eta_mode)
        gd[sl] = Jd.T @ gp[sl]
        gw[sl] += Jw.T @ gp[sl]
    return gd, gw


def loss(xi, target):
    """L = sum_A (xi_A - m_A)^2."""
    d = np.asarray(xi, np.float64).ravel() - np.asarray(target, np.float64).ravel()
    return float(np.sum(d * d))


def loss_grad_xi(xi, target):
    return 2.0 * (np.asarray(xi, np.float64) - np.asarray(target, np.float64).reshape(np.shape(xi)))


# ---------------------------------------------------------------------------
# error metrics used by the parity tests
# ---------------------------------------------------------------------------


def err_xi(xi_test, xi_ref, wsum_ref, absnum_ref):
    """max_A |dxi_A| W_A / sum_A |w d w d| (relative to the bin's condition)."""
    xi_test = np.asarray(xi_test, np.float64)
    m = np.asarray(absnum_ref) > 0
    if not m.any():
        return 0.0
    return float(np.max(np.abs(xi_test - xi_ref)[m] * np.asarray(wsum_ref)[m] / np.asarray(absnum_ref)[m]))


def err_rel(test, ref):
    """max |d| / |ref| over entries with ref != 0 (and test must be 0 elsewhere)."""
    test = np.asarray(test, np.float64)
    ref = np.asarray(ref, np.float64)
    m = ref != 0
    e = 0.0
    if m.any():
        e = float(np.max(np.abs(test[m] - ref[m]) / np.abs(ref[m])))
    if (~m).any():
        e = max(e, float(np.max(np.abs(test[~m]))) if np.any(test[~m]) else 0.0)
    return e


def err_rows(test, ref):
    """max_A max_B |dD_AB| / max_B |D_AB| (row-normwise)."""
    test = np.asarray(test, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.max(np.abs(ref), axis=-1, keepdims=True)
    scale = np.where(scale == 0, 1.0, scale)
    return float(np.max(np.abs(test - ref) / scale))


def err_norm(test, ref):
    """max |d| / max |ref| (normwise)."""
    ref = np.asarray(ref, np.float64)
    s = float(np.max(np.abs(ref)))
    return float(np.max(np.abs(np.asarray(test, np.float64) - ref)) / (s if s else 1.0))


# ---------------------------------------------------------------------------
# anisotropic three-point function (Sec. 2.3, eq. estimator_three)
# ---------------------------------------------------------------------------
#
# xi3_A = sum_A w_i d_i w_j d_j w_k d_k / sum_A w_i w_j w_k over triplets of
# pixels from three distinct forests (quasars).  A triangle is described from
# one vertex i by its two sides r1 = x_j - x_i and r2 = x_k - x_i (x = D n):
# their lengths r1, r2, their angles theta1, theta2 to the line of sight, and
# the cosine of the opening angle alpha between them (Sec. 2.3 and the 3PCF
# figure, which bins r in [0, r_max), theta in [0, pi] and cos alpha in
# [-1, 1]).  Readings where the paper is silent:
#  * the line of sight is the direction of the vertex's quasar, n_f(i);
#  * every vertex of a triplet is used (the paper records the same triangle
#    for each choice of main vertex) and both orders of the two sides, so an
#    unordered triplet enters six times and the histogram is symmetric under
#    (r1, theta1) <-> (r2, theta2);
#  * r bins are half-open [e_k, e_k+1) with r >= r_max outside; theta and
#    cos alpha bins are half-open except the last, which is closed (theta = pi,
#    cos alpha = 1 belong to the grid);
#  * a side of zero length has no direction: such triplets are left out;
#  * the flat index follows the figure's order (r1, r2, cos alpha, theta1,
#    theta2): A = (((k_r1 n_r + k_r2) n_c + k_c) n_t + k_t1) n_t + k_t2.


@dataclass
class Grid3:
    r_edges: np.ndarray      # side lengths, Mpc/h, strictly increasing, r_edges[0] >= 0
    theta_edges: np.ndarray  # angle of a side to the line of sight, radians, 0 .. pi
    cos_edges: np.ndarray    # cosine of the opening angle, -1 .. 1

    @property
    def n_r(self):
        return len(self.r_edges) - 1

    @property
    def n_t(self):
        return len(self.theta_edges) - 1

    @property
    def n_c(self):
        return len(self.cos_edges) - 1

    @property
    def n_bins(self):
        return self.n_r * self.n_r * self.n_c * self.n_t * self.n_t

    def index(self, kr1, kr2, kc, kt1, kt2):
        return (((kr1 * self.n_r + kr2) * self.n_c + kc) * self.n_t + kt1) * self.n_t + kt2


def closed_bin_index(x, edges):
    """k with edges[k] <= x < edges[k+1], the last bin closed at edges[-1];
    -1 outside [edges[0], edges[-1]]."""
    edges = np.asarray(edges, np.float64)
    n = edges.shape[0] - 1
    k = np.searchsorted(edges, x, side="right") - 1
    k = np.where(np.asarray(x) == edges[-1], n - 1, k)
    return np.where((k >= 0) & (k < n), k, -1)


@dataclass
class Xi3Sums:
    num: np.ndarray      # [R, n_bins] sum w_i d_i w_j d_j w_k d_k
    wsum: np.ndarray     # [R, n_bins] sum w_i w_j w_k
    ntrip: np.ndarray    # [R, n_bins] number of (vertex, side, side) entries
    n_near_edge: int     # entries with a coordinate within tau of an interior edge
    absnum: Optional[np.ndarray] = None  # [R, n_bins] sum |w d w d w d| (conditioning)

    @property
    def xi(self):
        return xi_from_sums(self.num, self.wsum)


def _near(x, e, tau):
    """True where x lies within tau of one of the edges e."""
    e = np.asarray(e, np.float64)
    if e.size == 0:
        return np.zeros(np.shape(x), bool)
    return np.any(np.abs(np.asarray(x)[..., None] - e) <= np.asarray(tau)[..., None], axis=-1)


def xi3_sums(F, g3: Grid3, edge_tau=1e-12, sub=None, n_sub=1, vertices=None) -> Xi3Sums:
    """Triplet sums of eq. estimator_three, vertex by vertex.

    For a vertex pixel i the partners are the pixels of every other forest of
    its realisation with side length in [r_edges[0], r_edges[-1]) (and > 0);
    each ordered pair of partners from two different forests is one entry.
    The per-vertex histograms are combined with Neumaier summation.

    With `sub` (a subsample id in [0, n_sub) per forest) the sums are split
    by subsample for the dispersion of the 3PCF figure (subsamples of the
    forests in sky pixels): every entry goes to slab r * n_sub + sub[f] of
    its main vertex's forest f; the first axis is then R * n_sub.

    With `vertices` (forest indices) only the pixels of those forests act as
    the main vertex; their partners still come from every forest.  The entries
    of one vertex do not depend on the others, so this is the restriction of
    the same sums to those vertices (it keeps checks at survey density cheap).
    """
    n_sub = int(n_sub) if sub is not None else 1
    R = max(1, int(F.n_realisations)) * n_sub
    nb = g3.n_bins
    rmax = float(g3.r_edges[-1])
    vset = None if vertices is None else set(int(v) for v in vertices)
    n_vec = unit_vectors(F.ra, F.dec)
    fid = np.repeat(np.arange(F.n_forests), np.diff(F.offsets))
    pos = F.dist[:, None] * n_vec[fid]
    wd = F.weight * F.delta
    real = F.real_of()
    num = _Neumaier((R, nb))
    wsum = _Neumaier((R, nb))
    absn = _Neumaier((R, nb))
    cnt = np.zeros((R, nb), np.int64)
    n_near = 0
    # candidate forests: pairs that can hold a side shorter than r_max
    from types import SimpleNamespace
    box = SimpleNamespace(edges_par=np.array([0.0, rmax]), edges_perp=np.array([0.0, rmax]))
    nbrs = [[] for _ in range(F.n_forests)]
    for f, g in forest_pairs(F, box, prune=True):
        nbrs[int(f)].append(int(g))
        nbrs[int(g)].append(int(f))
    for f in range(F.n_forests):
        if not nbrs[f] or F.offsets[f + 1] == F.offsets[f] or (vset is not None and f not in vset):
            continue
        g_list = np.array(sorted(nbrs[f]), np.int64)
        idx = np.concatenate([np.arange(F.offsets[g], F.offsets[g + 1]) for g in g_list])
        r = int(real[f]) * n_sub + (int(sub[f]) if sub is not None else 0)
        los = n_vec[f]
        for i in range(F.offsets[f], F.offsets[f + 1]):
            d = pos[idx] - pos[i]
            rr = np.sqrt(np.sum(d * d, axis=1))
            kr = bin_index_1d(rr, g3.r_edges)
            keep = (kr >= 0) & (rr > 0.0)
            if np.count_nonzero(keep) < 2:
                continue
            p = idx[keep]
            kr = kr[keep]
            rr = rr[keep]
            u = d[keep] / rr[:, None]
            ct = np.clip(u @ los, -1.0, 1.0)
            th = np.arccos(ct)
            kt = closed_bin_index(th, g3.theta_edges)
            side = kt >= 0          # a side outside the theta range leaves the grid
            if np.count_nonzero(side) < 2:
                continue
            p, kr, rr, u, th, kt = p[side], kr[side], rr[side], u[side], th[side], kt[side]
            ca = np.clip(u @ u.T, -1.0, 1.0)
            kc = closed_bin_index(ca, g3.cos_edges)
            ok = (fid[p][:, None] != fid[p][None, :]) & (kc >= 0)
            A = g3.index(kr[:, None], kr[None, :], kc, kt[:, None], kt[None, :])[ok]
            prod = (wd[i] * wd[p][:, None] * wd[p][None, :])[ok]
            num.add(np.bincount(A, weights=prod, minlength=nb), where=(r,))
            absn.add(np.bincount(A, weights=np.abs(prod), minlength=nb), where=(r,))
            wsum.add(np.bincount(A, weights=(F.weight[i] * F.weight[p][:, None] * F.weight[p][None, :])[ok],
                                 minlength=nb), where=(r,))
            cnt[r] += np.bincount(A, minlength=nb)
            if edge_tau > 0:
                re = g3.r_edges if g3.r_edges[0] > 0 else g3.r_edges[1:]
                side_near = (_near(rr, re, edge_tau * np.maximum(1.0, rr))
                             | _near(th, g3.theta_edges[1:-1], edge_tau))
                pair_near = (side_near[:, None] | side_near[None, :]
                             | _near(ca, g3.cos_edges[1:-1], edge_tau))
                n_near += int(np.count_nonzero(pair_near[ok]))
    return Xi3Sums(num.value(), wsum.value(), cnt, n_near, absn.value())


def xi3_brute(F, g3: Grid3, sub=None, n_sub=1):
    """Pure-Python loop over ordered pixel triplets (i; j, k) of three distinct
    forests (tiny inputs), with every angle from math.acos and every bin found
    by scanning the edge list; with `sub`, triplet (i; j, k) goes to slab
    r * n_sub + sub[forest of i]."""
    import math
    n_sub = int(n_sub) if sub is not None else 1
    R = max(1, int(F.n_realisations)) * n_sub
    nb = g3.n_bins
    real = F.real_of()
    fid = np.repeat(np.arange(F.n_forests), np.diff(F.offsets))
    nv = unit_vectors(F.ra, F.dec)
    P = [[float(F.dist[i]) * float(nv[fid[i]][a]) for a in range(3)] for i in range(F.n_pix)]

    def scan(x, edges, closed):
        for k in range(len(edges) - 1):
            if edges[k] <= x < edges[k + 1] or (closed and k == len(edges) - 2 and x == edges[-1]):
                return k
        return -1

    num = [[[] for _ in range(nb)] for _ in range(R)]
    ws = [[[] for _ in range(nb)] for _ in range(R)]
    cnt = np.zeros((R, nb), np.int64)
    for i in range(F.n_pix):
        los = [float(v) for v in nv[fid[i]]]
        side = {}
        for j in range(F.n_pix):
            if fid[j] == fid[i] or real[fid[j]] != real[fid[i]]:
                continue
            d = [P[j][a] - P[i][a] for a in range(3)]
            r = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
            kr = scan(r, list(g3.r_edges), False)
            if kr < 0 or r == 0.0:
                continue
            u = [v / r for v in d]
            th = math.acos(max(-1.0, min(1.0, sum(u[a] * los[a] for a in range(3)))))
            kt = scan(th, list(g3.theta_edges), True)
            if kt >= 0:
                side[j] = (kr, kt, u)
        for j, (kr1, kt1, u1) in side.items():
            for k, (kr2, kt2, u2) in side.items():
                if fid[j] == fid[k]:
                    continue
                ca = max(-1.0, min(1.0, sum(u1[a] * u2[a] for a in range(3))))
                kc = scan(ca, list(g3.cos_edges), True)
                if kc < 0:
                    continue
                A = (((kr1 * g3.n_r + kr2) * g3.n_c + kc) * g3.n_t + kt1) * g3.n_t + kt2
                r = int(real[fid[i]]) * n_sub + (int(sub[fid[i]]) if sub is not None else 0)
                num[r][A].append(float(F.weight[i] * F.delta[i] * F.weight[j] * F.delta[j] * F.weight[k] * F.delta[k]))
                ws[r][A].append(float(F.weight[i] * F.weight[j] * F.weight[k]))
                cnt[r, A] += 1
    N_ = np.array([[math.fsum(v) for v in row] for row in num])
    W_ = np.array([[math.fsum(v) for v in row] for row in ws])
    return N_, W_, cnt
