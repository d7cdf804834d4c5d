"""Pins for the FP64 oracle: each test checks it against something other than
itself (hand-worked values, exact rational arithmetic, closed forms,
invariants, statistics), chosen so that a dropped term, a wrong sign or index
or a transposed operand in the oracle fails at least one of them."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from synth import Grid, concat_realisations, make_patch, subset_forests, uniform_grid
from synth.survey import Forests

from helpers import forests_from_dict, grid_from_dict, load_json, tiny, truncate

G60 = uniform_grid(15, 60.0)


# ------------------------------------------------------------------ O1 geometry


def test_separation_identity_and_chord():
    """r_par^2 + r_perp^2 = |x_i - x_j|^2 and s = sin(theta/2) (Sec. 2.1)."""
    rng = np.random.default_rng(3)
    ra = rng.uniform(0, 2 * np.pi, 200)
    dec = np.arcsin(rng.uniform(-1, 1, 200))
    n = O.unit_vectors(ra, dec)
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-15)
    f, g = rng.integers(0, 200, 500), rng.integers(0, 200, 500)
    s, c = O.pair_sc(n[f], n[g])
    Di, Dj = rng.uniform(3000, 5000, 500), rng.uniform(3000, 5000, 500)
    rpar, rperp = O.separations(Di, Dj, s, c)
    d2 = np.sum((Di[:, None] * n[f] - Dj[:, None] * n[g]) ** 2, axis=1)
    assert np.allclose(rpar ** 2 + rperp ** 2, d2, rtol=1e-9, atol=1e-6)
    # independent angle: arctan2(|n_f x n_g|, n_f . n_g)
    theta = np.arctan2(np.linalg.norm(np.cross(n[f], n[g]), axis=1), np.sum(n[f] * n[g], axis=1))
    assert np.allclose(s, np.sin(theta / 2), rtol=1e-9, atol=1e-15)
    assert np.allclose(c, np.cos(theta / 2), rtol=1e-12)


def test_separation_special_cases():
    n = O.unit_vectors([0.3, 0.3], [0.2, 0.2])
    s, c = O.pair_sc(n[0], n[1])
    assert s == 0.0 and c == 1.0
    rpar, rperp = O.separations(4000.0, 4012.5, s, c)
    assert rpar == 12.5 and rperp == 0.0
    n = O.unit_vectors([0.0, 0.01], [0.0, 0.0])
    s, c = O.pair_sc(n[0], n[1])
    rpar, rperp = O.separations(4000.0, 4000.0, s, c)
    assert rpar == 0.0
    assert rperp == pytest.approx(8000.0 * np.sin(0.005), rel=1e-12)


# ------------------------------------------------------------------ O2 binning


def test_bin_edges_half_open():
    e = np.array([0.0, 4.0, 8.0, 12.0])
    r = np.array([0.0, 1.0, 3.999999, 4.0, 7.5, 8.0, 11.99, 12.0, 13.0, -1e-300])
    assert O.bin_index_1d(r, e).tolist() == [0, 0, 0, 1, 1, 2, 2, -1, -1, -1]


def test_golden_handworked_xi():
    d = load_json("xi_handworked_two_forests.json")
    F, G = forests_from_dict(d["forests"]), grid_from_dict(d["grid"])
    X = O.xi_sums(F, G, prune=False)
    exp = d["expected"]
    assert X.npairs[0].tolist() == exp["npairs"]
    assert np.allclose(X.num[0], exp["num"], rtol=0, atol=1e-12)
    assert np.allclose(X.wsum[0], exp["wsum"], rtol=0, atol=1e-12)
    assert np.allclose(X.xi[0], exp["xi"], rtol=1e-15)
    Xp = O.xi_sums(F, G, prune=True)
    assert (Xp.npairs == X.npairs).all()


def test_golden_handworked_bin_means():
    """Bin-mean r_par, r_perp, z of the hand-worked example (values derived by
    hand in the fixture; z of a pixel is lambda / lambda_Lya - 1)."""
    d = load_json("xi_handworked_two_forests.json")
    F, G = forests_from_dict(d["forests"]), grid_from_dict(d["grid"])
    rp, rt, z = O.bin_means(O.xi_sums(F, G, prune=False, means=True))
    exp = d["expected_means"]
    assert np.allclose(rp[0], exp["rpar"], rtol=1e-14, atol=0)
    assert np.allclose(rt[0], exp["rperp"], rtol=0, atol=1e-9)
    zl = np.exp(np.asarray(exp["z_loglam"])) / 1215.67 - 1.0
    assert np.allclose(z[0], np.asarray(exp["z_weights"]) @ zl, rtol=1e-14, atol=0)


@pytest.mark.parametrize("seed", [0, 3])
def test_bin_means_vs_geometric_brute(seed):
    """Vectorised bin means against a pure-Python pair loop that measures the
    separations on 3-D positions (projection on the mid line of sight)."""
    F = tiny(seed, n_forests=4, k=8)
    X = O.xi_sums(F, G60, means=True)
    rp, rt, z = O.bin_means(X)
    brp, brt, bz = O.xi_means_brute(F, G60)
    assert X.npairs.sum() > 20
    assert np.allclose(rp, brp, rtol=1e-9, atol=1e-9)
    assert np.allclose(rt, brt, rtol=1e-9, atol=1e-9)
    assert np.allclose(z, bz, rtol=1e-13, atol=1e-13)


def test_bin_means_lie_in_their_bins():
    """A weighted mean of values in [e_k, e_k+1) lies in that interval; the
    mean pair redshift lies within the pixels' redshift range; empty bins are 0."""
    F = make_patch(40, 2.0, 12)
    X = O.xi_sums(F, G60, means=True)
    rp, rt, z = O.bin_means(X)
    kp, kt = np.divmod(np.arange(G60.n_bins), G60.n_perp)
    ne = X.wsum[0] > 0
    assert ne.sum() > 0.9 * G60.n_bins
    ep, et = G60.edges_par, G60.edges_perp
    assert np.all(rp[0][ne] >= ep[kp][ne]) and np.all(rp[0][ne] <= ep[kp + 1][ne])
    assert np.all(rt[0][ne] >= et[kt][ne]) and np.all(rt[0][ne] <= et[kt + 1][ne])
    zp = O.pixel_redshift(F.loglam)
    assert np.all(z[0][ne] >= zp.min()) and np.all(z[0][ne] <= zp.max())
    assert np.all(rp[0][~ne] == 0) and np.all(z[0][~ne] == 0)


# ------------------------------------------------------------------ O3 xi sums


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_xi_vs_python_brute(seed):
    F = tiny(seed, n_forests=4, k=8)
    N_, W_, cnt = O.xi_pairs_brute(F, G60)
    X = O.xi_sums(F, G60)
    assert cnt.sum() > 20
    assert (cnt == X.npairs).all()
    assert np.allclose(X.num, N_, rtol=1e-14, atol=1e-13)
    assert np.allclose(X.wsum, W_, rtol=1e-14, atol=1e-13)


def test_xi_exact_rational():
    """Exact sums in rational arithmetic with bins decided by the same geometry."""
    F = tiny(5, n_forests=4, k=8)
    rng = np.random.default_rng(9)
    # dyadic values so the float inputs are exactly the rationals
    F.delta = rng.integers(-64, 64, F.n_pix) / 32.0
    F.weight = rng.integers(1, 64, F.n_pix) / 16.0
    n = O.unit_vectors(F.ra, F.dec)
    nb = G60.n_bins
    N_ = [Fraction(0)] * nb
    W_ = [Fraction(0)] * nb
    for f in range(F.n_forests):
        for g in range(f + 1, F.n_forests):
            s, c = O.pair_sc(n[f], n[g])
            for i in range(F.offsets[f], F.offsets[f + 1]):
                for j in range(F.offsets[g], F.offsets[g + 1]):
                    rp, rt = O.separations(F.dist[i], F.dist[j], s, c)
                    A = int(O.bin_index(np.array([rp]), np.array([rt]), G60)[0])
                    if A < 0:
                        continue
                    wi, wj = Fraction(F.weight[i]), Fraction(F.weight[j])
                    N_[A] += wi * Fraction(F.delta[i]) * wj * Fraction(F.delta[j])
                    W_[A] += wi * wj
    X = O.xi_sums(F, G60)
    for A in range(nb):
        assert X.num[0, A] == float(N_[A])
        assert X.wsum[0, A] == float(W_[A])


def test_single_bin_closed_form():
    """With one bin that holds every pair: N = ((sum S_f)^2 - sum S_f^2) / 2."""
    F = make_patch(40, 3.0, 11)
    G = Grid(np.array([0.0, 1e5]), np.array([0.0, 1e5]))
    X = O.xi_sums(F, G)
    S = np.array([np.sum(F.weight[F.forest_slice(f)] * F.delta[F.forest_slice(f)]) for f in range(F.n_forests)])
    Wf = np.array([np.sum(F.weight[F.forest_slice(f)]) for f in range(F.n_forests)])
    n = np.diff(F.offsets)
    assert X.num[0, 0] == pytest.approx((S.sum() ** 2 - np.sum(S ** 2)) / 2, rel=1e-11)
    assert X.wsum[0, 0] == pytest.approx((Wf.sum() ** 2 - np.sum(Wf ** 2)) / 2, rel=1e-12)
    assert X.npairs[0, 0] == (n.sum() ** 2 - np.sum(n ** 2)) // 2
    # mean-projected deltas have S_f = 0 in every forest, so N vanishes
    Xp = O.xi_sums(F, G, project=True, eta_mode=O.MEAN)
    assert abs(Xp.num[0, 0]) < 1e-9 * X.absnum[0, 0]


def test_invariances():
    F = make_patch(30, 2.0, 4)
    X = O.xi_sums(F, G60)
    assert X.npairs.sum() > 1000 and X.n_near_edge == 0
    # permute forests and pixels within forests
    rng = np.random.default_rng(1)
    perm = rng.permutation(F.n_forests)
    P = subset_forests(F, perm)
    for f in range(P.n_forests):
        sl = P.forest_slice(f)
        q = sl.start + rng.permutation(sl.stop - sl.start)
        for name in ("dist", "delta", "weight", "loglam"):
            getattr(P, name)[sl] = getattr(P, name)[q]
    Xp = O.xi_sums(P, G60)
    assert (Xp.npairs == X.npairs).all()
    assert np.allclose(Xp.num, X.num, rtol=1e-12, atol=1e-12 * X.absnum.max())
    # rotate the whole sky about an arbitrary axis
    n = O.unit_vectors(F.ra, F.dec)
    a, b, c = 0.7, -1.1, 0.4
    Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(b), -np.sin(b)], [0, np.sin(b), np.cos(b)]])
    Ry = np.array([[np.cos(c), 0, np.sin(c)], [0, 1, 0], [-np.sin(c), 0, np.cos(c)]])
    m = n @ (Rz @ Rx @ Ry).T
    Rot = F.copy()
    Rot.ra = np.arctan2(m[:, 1], m[:, 0])
    Rot.dec = np.arcsin(np.clip(m[:, 2], -1, 1))
    Xr = O.xi_sums(Rot, G60)
    assert (Xr.npairs == X.npairs).all()
    assert np.allclose(Xr.xi, X.xi, rtol=1e-10, atol=1e-12)
    # w -> 3w leaves xi unchanged; delta -> -2 delta scales it by 4
    S = F.copy()
    S.weight = 3.0 * S.weight
    S.delta = -2.0 * S.delta
    Xs = O.xi_sums(S, G60)
    assert np.allclose(Xs.xi, 4.0 * X.xi, rtol=1e-12, atol=1e-14)
    # prune on/off
    Xn = O.xi_sums(F, G60, prune=False)
    assert (Xn.npairs == X.npairs).all()


def test_same_forest_pairs_excluded_and_realisations_separate():
    F = tiny(2, n_forests=3, k=6)
    G = Grid(np.array([0.0, 1e5]), np.array([0.0, 1e5]))
    X = O.xi_sums(F, G)
    n = np.diff(F.offsets)
    assert X.npairs[0, 0] == (n.sum() ** 2 - np.sum(n ** 2)) // 2
    # the same forests split into 3 realisations pair with nobody
    R = F.copy()
    R.realisation = np.arange(3, dtype=np.int32)
    R.n_realisations = 3
    Xr = O.xi_sums(R, G)
    assert Xr.npairs.sum() == 0


def test_xi_zero_mean_statistics():
    """iid zero-mean deltas: z_A = N_A / sqrt(sum_A (w_i s_i)^2 (w_j s_j)^2) has
    mean 0 and variance 1 exactly, because distinct cross-forest pairs are
    uncorrelated.  Double-counted or same-forest pairs would break this."""
    zs = []
    for seed in range(6):
        F = make_patch(60, 2.5, 100 + seed)
        rng = np.random.default_rng(500 + seed)
        sig = rng.uniform(0.2, 1.0, F.n_pix)
        F.delta = rng.normal(0.0, 1.0, F.n_pix) * sig
        X = O.xi_sums(F, G60)
        V = F.copy()
        V.weight = (F.weight * sig) ** 2
        var = O.xi_sums(V, G60).wsum
        m = X.npairs >= 200
        zs.append((X.num[m] / np.sqrt(var[m])))
    z = np.concatenate(zs)
    assert z.size > 600
    assert abs(z.mean()) < 5.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / z.size) + 0.05


# ------------------------------------------------------------------ O4 eta


@pytest.mark.parametrize("mode", [O.MEAN, O.MEAN_SLOPE])
def test_eta_invariants(mode):
    rng = np.random.default_rng(7)
    n = 37
    w = rng.uniform(0.5, 9.0, n)
    L = np.log(3600.0 * 10 ** (3e-4 * np.arange(n)))
    E = O.eta_matrix(w, L, mode)
    assert np.abs(E.sum(1)).max() < 1e-10            # eta 1 = 0
    assert np.abs(w @ E).max() < 1e-10                # sum_i w_i eta_ii' = 0
    assert np.abs(E @ E - E).max() < 1e-10            # idempotent
    if mode == O.MEAN_SLOPE:
        assert np.abs(E @ L).max() < 1e-10            # eta Lambda = 0
        assert np.abs(w @ (E * (L - L.mean())[:, None])).max() < 1e-9
        E2 = O.eta_matrix(w, 3.0 * L - 7.0, mode)     # any log base / offset
        assert np.abs(E2 - E).max() < 1e-9
        Em = O.eta_matrix(w, L, O.MEAN)
        assert np.abs(Em - E).max() > 1e-3           # slope term present
    d = rng.normal(size=n)
    assert np.allclose(O.project_forest(d, w, L, mode), E @ d, atol=1e-12)


def test_eta_explicit_formula_small():
    """eta_ii' = delta^K - w_i'/W - (L_i - Lb) w_i' (L_i' - Lb) / sum w (L - Lb)^2,
    evaluated exactly in rationals for a 3-pixel forest."""
    w = [Fraction(1), Fraction(2), Fraction(5, 2)]
    L = [Fraction(33, 4), Fraction(17, 2), Fraction(35, 4)]
    W = sum(w)
    Lb = sum(wi * li for wi, li in zip(w, L)) / W
    S = sum(wi * (li - Lb) ** 2 for wi, li in zip(w, L))
    E = O.eta_matrix(np.array([float(x) for x in w]), np.array([float(x) for x in L]), O.MEAN_SLOPE)
    for i in range(3):
        for k in range(3):
            exact = (1 if i == k else 0) - w[k] / W - (L[i] - Lb) * w[k] * (L[k] - Lb) / S
            assert E[i, k] == pytest.approx(float(exact), abs=1e-14)


def test_eta_degenerate_forests():
    assert np.allclose(O.eta_matrix(np.array([2.0]), np.array([8.3]), O.MEAN), 0.0)
    assert np.allclose(O.eta_matrix(np.array([2.0]), np.array([8.3]), O.MEAN_SLOPE), 0.0)
    # constant Lambda: slope term dropped, eta = I - 1 u^T
    w = np.array([1.0, 2.0, 3.0])
    E = O.eta_matrix(w, np.full(3, 8.3), O.MEAN_SLOPE)
    assert np.allclose(E, np.eye(3) - np.ones((3, 1)) * (w / w.sum())[None, :])
    assert np.allclose(O.eta_matrix(np.zeros(3), np.arange(3.0), O.MEAN_SLOPE), np.eye(3))
    assert np.allclose(O.eta_matrix(w, np.arange(3.0), O.IDENTITY), np.eye(3))


# ------------------------------------------------------------------ O5 distortion


def _tiny_dmat_case(seed, k=6, n_forests=3):
    F = tiny(seed, n_forests=n_forests, k=k)
    G = uniform_grid(4, 24.0, 3, 30.0)
    return F, G


@pytest.mark.parametrize("mode", [O.MEAN, O.MEAN_SLOPE])
@pytest.mark.parametrize("seed", [0, 1])
def test_dmat_brute_definition_factorised_agree(mode, seed):
    F, G = _tiny_dmat_case(seed)
    pairs = O.dmat_pairs(F, G)
    b = O.dmat_brute(F, G, pairs, mode)
    d = O.dmat_definition(F, G, pairs, mode)
    f = O.dmat(F, G, pairs, mode)
    scale = np.abs(b.num).max()
    assert scale > 0 and np.count_nonzero(b.wd) >= 4
    assert np.abs(d.num - b.num).max() <= 1e-13 * scale
    assert np.abs(f.num - b.num).max() <= 1e-13 * scale
    assert np.array_equal(f.wd, b.wd) or np.allclose(f.wd, b.wd, rtol=1e-15)


def test_dmat_exact_rational_brute():
    """Four nested sums in exact rationals (dyadic inputs) vs the factorised form."""
    F = tiny(3, n_forests=4, k=6, width_deg=0.2)
    G = Grid(np.array([0.0, 3.0, 6.0, 12.0, 24.0]), np.array([0.0, 5.0, 10.0, 20.0, 40.0]))
    rng = np.random.default_rng(2)
    F.weight = rng.integers(1, 16, F.n_pix) / 4.0
    F.loglam = np.round(F.loglam * 64) / 64.0
    n = O.unit_vectors(F.ra, F.dec)
    nb = G.n_bins
    num = {}
    wd = [Fraction(0)] * nb

    def eta_q(sl):
        w = [Fraction(x) for x in F.weight[sl]]
        L = [Fraction(x) for x in F.loglam[sl]]
        W = sum(w)
        Lb = sum(a * b for a, b in zip(w, L)) / W
        S = sum(a * (b - Lb) ** 2 for a, b in zip(w, L))
        m = len(w)
        return [[(1 if i == k else 0) - w[k] / W - ((L[i] - Lb) * w[k] * (L[k] - Lb) / S if S else 0)
                 for k in range(m)] for i in range(m)]

    pairs = O.dmat_pairs(F, G)
    for f, g in pairs:
        sf, sg = F.forest_slice(f), F.forest_slice(g)
        s, c = O.pair_sc(n[f], n[g])
        rp, rt = O.separations(F.dist[sf][:, None], F.dist[sg][None, :], s, c)
        A = O.bin_index(rp, rt, G)
        ef, eg = eta_q(sf), eta_q(sg)
        wf = [Fraction(x) for x in F.weight[sf]]
        wg = [Fraction(x) for x in F.weight[sg]]
        for i in range(A.shape[0]):
            for j in range(A.shape[1]):
                a = int(A[i, j])
                if a < 0:
                    continue
                wd[a] += wf[i] * wg[j]
                for ip in range(A.shape[0]):
                    for jp in range(A.shape[1]):
                        bb = int(A[ip, jp])
                        if bb < 0:
                            continue
                        num[(a, bb)] = num.get((a, bb), Fraction(0)) + wf[i] * wg[j] * ef[i][ip] * eg[j][jp]
    R = O.dmat(F, G, pairs, O.MEAN_SLOPE)
    assert len(num) >= 12
    scale = max(abs(float(v)) for v in num.values())
    for (a, bb), v in num.items():
        assert abs(R.num[0, a, bb] - float(v)) <= 1e-12 * scale
    for a in range(nb):
        assert R.wd[0, a] == float(wd[a])


def test_dmat_identity_eta_gives_identity():
    F = make_patch(20, 1.5, 8)
    pairs = O.dmat_pairs(F, G60)
    R = O.dmat(F, G60, pairs, O.IDENTITY)
    D = R.D[0]
    nz = R.wd[0] > 0
    assert nz.sum() > 50
    assert np.array_equal(D[np.ix_(nz, nz)], np.eye(int(nz.sum())))
    assert not D[~nz].any()


@pytest.mark.parametrize("mode", [O.MEAN, O.MEAN_SLOPE])
def test_dmat_covering_grid_row_sums_vanish(mode):
    """With a grid that holds every pair, sum_B D_AB = 0 because eta rows sum to 0."""
    F = tiny(4, n_forests=4, k=9)
    G = Grid(np.array([0.0, 4.0, 1e5]), np.array([0.0, 1e5]))
    pairs = O.dmat_pairs(F, G)
    R = O.dmat(F, G, pairs, mode)
    D = R.D[0]
    assert np.abs(D).max() > 0.1
    assert np.abs(D.sum(1)).max() < 1e-10


def test_dmat_independent_of_delta_and_subset_hash():
    F = make_patch(25, 1.5, 12)
    p_all = O.dmat_pairs(F, G60)
    R1 = O.dmat(F, G60, p_all)
    F2 = F.copy()
    F2.delta = np.random.default_rng(0).normal(size=F.n_pix)
    R2 = O.dmat(F2, G60, p_all)
    assert np.array_equal(R1.num, R2.num)
    # deterministic subset: about p of the pairs, same set for the same seed
    big = np.stack(np.triu_indices(400, 1), -1)
    m1 = O.keep_pair_mask(big[:, 0], big[:, 1], 0.25, 42)
    m2 = O.keep_pair_mask(big[:, 0], big[:, 1], 0.25, 42)
    m3 = O.keep_pair_mask(big[:, 0], big[:, 1], 0.25, 43)
    assert np.array_equal(m1, m2) and not np.array_equal(m1, m3)
    assert abs(m1.mean() - 0.25) < 5 * np.sqrt(0.25 * 0.75 / m1.size)
    assert O.keep_pair_mask(np.array([1]), np.array([2]), 1.0, 7).all()


def test_splitmix64_published_vector():
    lines = [l.split() for l in open(__import__("helpers").GOLDEN + "/splitmix64_seed1234567.txt")
             if l.strip() and not l.startswith("#")]
    state = np.uint64(int(lines[0][1]))
    for row in lines[1:]:
        assert int(O.splitmix64(state)) == int(row[0])
        with np.errstate(over="ignore"):
            state = state + np.uint64(0x9E3779B97F4A7C15)


# ------------------------------------------------------------------ O6 gradient


def _loss_of(F, G, target):
    X = O.xi_sums(F, G)
    return O.loss(X.xi, target), X


def test_gradient_finite_differences_and_euler():
    F = make_patch(12, 1.0, 21, z_range=(2.1, 2.3))
    G = G60
    rng = np.random.default_rng(3)
    target = rng.uniform(-0.01, 0.01, G.n_bins)
    L0, X = _loss_of(F, G, target)
    gxi = O.loss_grad_xi(X.xi, target[None, :])
    gd, gw = O.xi_grad(F, G, gxi, X.xi, X.wsum)
    # L is quadratic in each delta_i: central differences are exact up to rounding
    for i in rng.choice(F.n_pix, 12, replace=False):
        for eps in (0.5, 1e-3):
            Fp, Fm = F.copy(), F.copy()
            Fp.delta[i] += eps
            Fm.delta[i] -= eps
            fd = (_loss_of(Fp, G, target)[0] - _loss_of(Fm, G, target)[0]) / (2 * eps)
            assert fd == pytest.approx(gd[i], rel=1e-6, abs=1e-9 * np.abs(gd).max())
    for i in rng.choice(F.n_pix, 12, replace=False):
        eps = 1e-3
        Fp, Fm = F.copy(), F.copy()
        Fp.weight[i] += eps
        Fm.weight[i] -= eps
        fd = (_loss_of(Fp, G, target)[0] - _loss_of(Fm, G, target)[0]) / (2 * eps)
        assert fd == pytest.approx(gw[i], rel=1e-4, abs=1e-6 * np.abs(gw).max())
    # Euler: xi is homogeneous of degree 2 in delta and 0 in w
    xi = X.xi[0]
    assert np.dot(F.delta, gd) == pytest.approx(4.0 * np.sum(xi * (xi - target)), rel=1e-9)
    assert abs(np.dot(F.weight, gw)) < 1e-9 * np.dot(np.abs(F.weight), np.abs(gw))


def _loss_proj(F, G, target, mode):
    X = O.xi_sums(F, G, project=True, eta_mode=mode)
    return O.loss(X.xi, target), X


@pytest.mark.parametrize("mode", [O.MEAN, O.MEAN_SLOPE])
def test_projected_gradient_finite_differences(mode):
    """Gradient through the projection delta' = eta(w, Lambda) delta (Sec. 2.2)
    against central differences of the projected forward: exact up to
    rounding in delta (L stays quadratic in delta), O(eps^2) in w (eta moves
    with w through W, Lambda_bar and S)."""
    F = make_patch(12, 1.0, 23, z_range=(2.1, 2.3))
    G = G60
    rng = np.random.default_rng(5)
    target = rng.uniform(-0.01, 0.01, G.n_bins)
    L0, X = _loss_proj(F, G, target, mode)
    gxi = O.loss_grad_xi(X.xi, target[None, :])
    gd, gw = O.xi_grad_projected(F, G, gxi, X.xi, X.wsum, eta_mode=mode)
    for i in rng.choice(F.n_pix, 10, replace=False):
        for eps in (0.5, 1e-3):
            Fp, Fm = F.copy(), F.copy()
            Fp.delta[i] += eps
            Fm.delta[i] -= eps
            fd = (_loss_proj(Fp, G, target, mode)[0] - _loss_proj(Fm, G, target, mode)[0]) / (2 * eps)
            assert fd == pytest.approx(gd[i], rel=1e-6, abs=1e-9 * np.abs(gd).max())
    for i in rng.choice(F.n_pix, 10, replace=False):
        eps = 1e-3
        Fp, Fm = F.copy(), F.copy()
        Fp.weight[i] += eps
        Fm.weight[i] -= eps
        fd = (_loss_proj(Fp, G, target, mode)[0] - _loss_proj(Fm, G, target, mode)[0]) / (2 * eps)
        assert fd == pytest.approx(gw[i], rel=1e-4, abs=1e-6 * np.abs(gw).max())


@pytest.mark.parametrize("mode", [O.MEAN, O.MEAN_SLOPE])
def test_projected_gradient_invariances(mode):
    """delta -> delta + c (and + c Lambda with the slope term) per forest leaves
    delta' unchanged, so the delta-gradient sums to zero over each forest
    (and against Lambda); xi is homogeneous of degree 2 in delta and 0 in w,
    also through eta (Euler identities)."""
    F = make_patch(15, 1.2, 31, z_range=(2.1, 2.4))
    G = G60
    rng = np.random.default_rng(8)
    target = rng.uniform(-0.01, 0.01, G.n_bins)
    _, X = _loss_proj(F, G, target, mode)
    gxi = O.loss_grad_xi(X.xi, target[None, :])
    gd, gw = O.xi_grad_projected(F, G, gxi, X.xi, X.wsum, eta_mode=mode)
    scale = np.abs(gd).max() * 200
    for f in range(F.n_forests):
        sl = F.forest_slice(f)
        assert abs(np.sum(gd[sl])) <= 1e-12 * scale
        if mode == O.MEAN_SLOPE:
            lc = F.loglam[sl] - F.loglam[sl].mean()
            assert abs(np.dot(lc, gd[sl])) <= 1e-12 * scale
    xi = X.xi[0]
    assert np.dot(F.delta, gd) == pytest.approx(4.0 * np.sum(xi * (xi - target)), rel=1e-9)
    assert abs(np.dot(F.weight, gw)) < 1e-9 * np.dot(np.abs(F.weight), np.abs(gw))
    # without the projection term the delta-gradient is not orthogonal to 1
    gp, _ = O.xi_grad(F, G, gxi, X.xi, X.wsum)
    assert max(abs(np.sum(gp[F.forest_slice(f)])) for f in range(F.n_forests)) > 1e-6 * scale


def test_projected_gradient_identity_mode_is_plain():
    F = make_patch(10, 1.0, 41, z_range=(2.1, 2.3))
    rng = np.random.default_rng(2)
    X = O.xi_sums(F, G60)
    gxi = rng.normal(size=(1, G60.n_bins))
    a = O.xi_grad(F, G60, gxi, X.xi, X.wsum)
    b = O.xi_grad_projected(F, G60, gxi, X.xi, X.wsum, eta_mode=O.IDENTITY)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


# ---------------------------------------------------------------- subsamples
G_TINY = uniform_grid(12, 60.0)


def test_subsample_sums_partition_the_pairs():
    """Keying the sums by subsample splits every pair into exactly one slab:
    the slabs add up to the unsplit sums (counts exactly)."""
    from synth import sky_cells
    F = tiny(3, n_forests=9, k=7, width_deg=1.0)
    sub = sky_cells(F, 2, 2)
    assert len(np.unique(sub)) > 1
    whole = O.xi_sums(F, G_TINY)
    split = O.xi_sums(F, G_TINY, sub=sub, n_sub=4)
    assert split.npairs.shape == (4, G_TINY.n_bins)
    np.testing.assert_array_equal(split.npairs.sum(0), whole.npairs[0])
    np.testing.assert_allclose(split.num.sum(0), whole.num[0], rtol=0, atol=1e-13 * whole.absnum.max())
    np.testing.assert_allclose(split.wsum.sum(0), whole.wsum[0], rtol=1e-13)


def test_subsample_owner_is_smaller_index():
    """A pair is credited to the subsample of the forest with the smaller input
    index: with all forests but forest 0 in subsample 1, slab 0 holds exactly
    forest 0's pairs."""
    F = tiny(4, n_forests=5, k=6)
    sub = np.ones(F.n_forests, np.int32)
    sub[0] = 0
    split = O.xi_sums(F, G_TINY, sub=sub, n_sub=2)
    only0 = O.xi_sums(F, G_TINY, pairs=np.array([[0, g] for g in range(1, F.n_forests)]))
    np.testing.assert_array_equal(split.npairs[0], only0.npairs[0])


def test_covariance_hand_worked():
    d = load_json("covariance_two_subsamples.json")
    xi, cov = O.covariance(d["num"], d["wsum"])
    np.testing.assert_allclose(xi, d["xi"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(cov, d["cov"], rtol=0, atol=1e-15)


def test_covariance_properties():
    rng = np.random.default_rng(5)
    num = rng.normal(size=(12, 7))
    wsum = rng.uniform(0.5, 2.0, size=(12, 7))
    wsum[:, 3] = 0.0          # an empty bin
    num[:, 3] = 0.0
    xi, cov = O.covariance(num, wsum)
    assert np.all(cov[3] == 0) and np.all(cov[:, 3] == 0) and xi[3] == 0
    np.testing.assert_allclose(cov, cov.T, rtol=0, atol=1e-15)
    assert np.linalg.eigvalsh(cov).min() > -1e-12          # positive semi-definite
    _, cov2 = O.covariance(3.0 * num, wsum)
    np.testing.assert_allclose(cov2, 9.0 * cov, rtol=1e-12, atol=0)   # quadratic in N
    _, cov1 = O.covariance(num[:1], wsum[:1])
    assert np.abs(cov1).max() < 1e-28                         # one subsample: no scatter (rounding only)


# ------------------------------------------------------ anisotropic 3PCF


def _grid3(r_max=30.0, n_r=3, n_t=4, n_c=5):
    return O.Grid3(np.linspace(0.0, r_max, n_r + 1), np.linspace(0.0, np.pi, n_t + 1),
                   np.linspace(-1.0, 1.0, n_c + 1))


def test_xi3_golden_handworked():
    """One triplet of single-pixel forests binned by hand from each vertex and
    both side orders (derivation in the fixture)."""
    d = load_json("xi3_handworked_three_forests.json")
    F = forests_from_dict(d["forests"])
    g = d["grid3"]
    G3 = O.Grid3(np.array(g["r_edges"]), np.array(g["theta_edges"]), np.array(g["cos_edges"]))
    X = O.xi3_sums(F, G3)
    exp = d["expected"]
    assert G3.n_bins == exp["n_bins"]
    assert np.nonzero(X.ntrip[0])[0].tolist() == exp["bins"]
    assert np.all(X.ntrip[0][exp["bins"]] == exp["ntrip"])
    assert np.allclose(X.num[0][exp["bins"]], exp["num"], rtol=1e-15)
    assert np.allclose(X.wsum[0][exp["bins"]], exp["wsum"], rtol=1e-15)
    assert X.n_near_edge == 0


@pytest.mark.parametrize("seed,partial", [(0, False), (1, False), (1, True)])
def test_xi3_vs_python_brute(seed, partial):
    """Vectorised triplet sums against a pure-Python loop over ordered
    triplets (math.acos, edge scans); also with theta and cos alpha grids that
    cover only part of their range (sides and triangles outside drop out)."""
    F = tiny(seed, n_forests=5, k=5, width_deg=0.3)
    G3 = _grid3()
    if partial:
        G3 = O.Grid3(np.linspace(5.0, 30.0, 4), np.linspace(0.2, 2.0, 4), np.linspace(-0.5, 1.0, 4))
    X = O.xi3_sums(F, G3)
    N_, W_, C_ = O.xi3_brute(F, G3)
    assert X.n_near_edge == 0 and C_.sum() > 200
    assert (X.ntrip == C_).all()
    assert np.allclose(X.num, N_, rtol=1e-13, atol=1e-13 * np.abs(N_).max())
    assert np.allclose(X.wsum, W_, rtol=1e-13, atol=1e-13 * np.abs(W_).max())


def test_xi3_subsample_split_vs_python_brute():
    """Sums split by the subsample of the main vertex's forest against the
    pure-Python loop with the same split, over two realisations; the slabs
    add up to the unsplit sums, and a vertex forest's triplets land only in
    its own subsample (pins the slab index r * n_sub + sub[f])."""
    parts = [tiny(10 + r, n_forests=5, k=4, width_deg=0.3) for r in range(2)]
    F = concat_realisations(parts)
    G3 = _grid3()
    sub = np.array([0, 2, 1, 2, 0, 1, 1, 0, 2, 2], np.int32)[:F.n_forests]
    X = O.xi3_sums(F, G3, sub=sub, n_sub=3)
    N_, W_, C_ = O.xi3_brute(F, G3, sub=sub, n_sub=3)
    assert X.ntrip.shape == (2 * 3, G3.n_bins) and C_.sum() > 100
    assert (X.ntrip == C_).all()
    assert np.allclose(X.num, N_, rtol=1e-13, atol=1e-13 * np.abs(N_).max())
    assert np.allclose(X.wsum, W_, rtol=1e-13, atol=1e-13 * np.abs(W_).max())
    U = O.xi3_sums(F, G3)
    assert (X.ntrip.reshape(2, 3, -1).sum(axis=1) == U.ntrip).all()
    assert np.allclose(X.wsum.reshape(2, 3, -1).sum(axis=1), U.wsum, rtol=1e-13, atol=0)
    # only the vertex forests of subsample 1 contribute to its slabs
    keep = [f for f in range(F.n_forests) if sub[f] == 1]
    assert X.ntrip.reshape(2, 3, -1)[:, 1].sum() == sum(
        int(O.xi3_brute(F, G3, sub=(np.arange(F.n_forests) == f).astype(np.int32), n_sub=2)[2][1::2].sum())
        for f in keep)


def test_xi3_vertex_restriction_vs_python_brute():
    """Restricting the main vertex to some forests gives the pure-Python loop's
    slab for a subsample split that puts exactly those forests in slab 0, and
    the restrictions to a set and to its complement add up to the whole."""
    F = tiny(21, n_forests=6, k=4, width_deg=0.3)
    G3 = _grid3()
    chosen = [1, 4]
    V = O.xi3_sums(F, G3, vertices=chosen)
    sub = np.array([0 if f in chosen else 1 for f in range(F.n_forests)], np.int32)
    N_, W_, C_ = O.xi3_brute(F, G3, sub=sub, n_sub=2)
    assert C_[0].sum() > 20
    assert (V.ntrip[0] == C_[0]).all()
    assert np.allclose(V.num[0], N_[0], rtol=1e-13, atol=1e-13 * np.abs(N_[0]).max())
    assert np.allclose(V.wsum[0], W_[0], rtol=1e-13, atol=1e-13 * np.abs(W_[0]).max())
    rest = O.xi3_sums(F, G3, vertices=[f for f in range(F.n_forests) if f not in chosen])
    U = O.xi3_sums(F, G3)
    assert (V.ntrip + rest.ntrip == U.ntrip).all()
    assert np.allclose(V.wsum + rest.wsum, U.wsum, rtol=1e-13, atol=0)


def test_xi3_single_bin_closed_form():
    """With one bin holding every triangle, the sums run over all ordered
    triples of distinct forests: sum S_f S_g S_h = S1^3 - 3 S1 S2 + 2 S3 with
    the power sums S_p = sum_f S_f^p of the per-forest sums S_f."""
    F = tiny(4, n_forests=6, k=6, width_deg=0.3)
    G3 = O.Grid3(np.array([0.0, 1e6]), np.array([0.0, np.pi]), np.array([-1.0, 1.0]))
    X = O.xi3_sums(F, G3)
    fid = np.repeat(np.arange(F.n_forests), np.diff(F.offsets))

    def triple(a):
        S = np.bincount(fid, weights=a, minlength=F.n_forests)
        return S.sum() ** 3 - 3 * S.sum() * np.sum(S ** 2) + 2 * np.sum(S ** 3)
    assert X.num[0, 0] == pytest.approx(triple(F.weight * F.delta), rel=1e-12)
    assert X.wsum[0, 0] == pytest.approx(triple(F.weight), rel=1e-12)
    assert X.ntrip[0, 0] == round(triple(np.ones(F.n_pix)))


def test_xi3_symmetry_and_invariances():
    """Both side orders are entered, so the sums are symmetric under
    (r1, theta1) <-> (r2, theta2); delta -> -delta flips N, w -> 2 w scales N
    and W by 8 and leaves xi3; a realisation id keeps triplets apart."""
    F = tiny(2, n_forests=6, k=6, width_deg=0.3)
    G3 = _grid3()
    X = O.xi3_sums(F, G3)
    sh = (G3.n_r, G3.n_r, G3.n_c, G3.n_t, G3.n_t)
    N = X.num[0].reshape(sh)
    assert np.allclose(N, N.transpose(1, 0, 2, 4, 3), rtol=1e-13, atol=1e-15 * np.abs(N).max())
    assert np.array_equal(X.ntrip[0].reshape(sh), X.ntrip[0].reshape(sh).transpose(1, 0, 2, 4, 3))
    Fm = F.copy()
    Fm.delta = -Fm.delta
    assert np.allclose(O.xi3_sums(Fm, G3).num, -X.num, rtol=1e-13, atol=1e-15 * np.abs(X.num).max())
    F2 = F.copy()
    F2.weight = 2.0 * F2.weight
    X2 = O.xi3_sums(F2, G3)
    assert np.allclose(X2.num, 8 * X.num, rtol=1e-13, atol=1e-15 * np.abs(X.num).max())
    assert np.allclose(X2.xi, X.xi, rtol=1e-12, atol=1e-15)
    from synth import concat_realisations
    Rr = concat_realisations([F, F])
    XR = O.xi3_sums(Rr, G3)
    assert XR.ntrip.shape == (2, G3.n_bins)
    assert np.array_equal(XR.ntrip[0], X.ntrip[0]) and np.array_equal(XR.ntrip[1], X.ntrip[0])
