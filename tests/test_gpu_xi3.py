"""GPU parity of lya_xi3 (the anisotropic three-point function of Sec. 2.3,
eq. estimator_three) against the FP64 oracle, for the three kernels (variant 0
sums each vertex's entries in LDS before the global atomics, variant 1 adds
every entry to the global sums, variant 2 is variant 0 with the partner
lists in global scratch for vertex pixels with many partners).  Entry counts must match exactly; N and W to
1e-12 of the bin's absolute sum (FP64 throughout, only the summation order
differs)."""
import numpy as np
import pytest

import oracle as O
from synth import concat_realisations, make_config, make_patch, subset_forests
from synth.survey import nearest_to_centre

from helpers import forests_from_dict, load_json, tiny, truncate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lib():
    from paper_2507_00129_amd import Library
    L = Library(0)
    yield L
    L.close()


def grid3(r_max=30.0, n_r=3, n_t=4, n_c=5, r0=0.0, t=(0.0, np.pi), c=(-1.0, 1.0)):
    return O.Grid3(np.linspace(r0, r_max, n_r + 1), np.linspace(t[0], t[1], n_t + 1),
                   np.linspace(c[0], c[1], n_c + 1))


def run3(lib, F, G3, expect_variant=None, **kw):
    from paper_2507_00129_amd import DeviceForests
    out = lib.xi3(DeviceForests.from_host(F, "cuda:0"), G3, **kw)
    torch.cuda.synchronize()
    if expect_variant is not None:
        assert lib.last_stats()["variant"] == expect_variant
    return {k: v.cpu().numpy() for k, v in out.items()}


def check3(out, ref, what):
    print(f"[xi3 {what}] entries={int(ref.ntrip.sum())} bins={int((ref.ntrip > 0).sum())} "
          f"near_edge={ref.n_near_edge}", flush=True)
    assert ref.n_near_edge == 0, "input has entries within 1e-12 of an edge; choose another seed"
    np.testing.assert_array_equal(out["ntrip"], ref.ntrip)
    m = ref.absnum > 0
    e_n = float(np.max(np.abs(out["num"] - ref.num)[m] / ref.absnum[m])) if m.any() else 0.0
    e_w = O.err_rel(out["wsum"], ref.wsum)
    print(f"    e_N={e_n:.2e} e_W={e_w:.2e}", flush=True)
    assert e_n <= TOL and e_w <= TOL
    np.testing.assert_allclose(out["xi"], ref.xi, rtol=0, atol=TOL * max(1.0, float(np.abs(ref.xi).max())) * 1e3)


def test_xi3_golden_handworked(lib):
    d = load_json("xi3_handworked_three_forests.json")
    F = forests_from_dict(d["forests"])
    g = d["grid3"]
    G3 = O.Grid3(np.array(g["r_edges"]), np.array(g["theta_edges"]), np.array(g["cos_edges"]))
    out = run3(lib, F, G3)
    exp = d["expected"]
    assert out["ntrip"].shape == (1, exp["n_bins"])
    assert np.nonzero(out["ntrip"][0])[0].tolist() == exp["bins"]
    assert np.all(out["ntrip"][0][exp["bins"]] == exp["ntrip"])
    assert np.allclose(out["num"][0][exp["bins"]], exp["num"], rtol=1e-15)
    assert np.allclose(out["wsum"][0][exp["bins"]], exp["wsum"], rtol=1e-15)


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_xi3_tiny_vs_oracle(lib, seed, variant):
    F = tiny(seed, n_forests=6, k=8, width_deg=0.3)
    G3 = grid3()
    check3(run3(lib, F, G3, variant=variant, expect_variant=variant), O.xi3_sums(F, G3), f"tiny{seed} v{variant}")


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_xi3_partial_ranges_vs_oracle(lib, variant):
    """r from 5 Mpc/h, theta in [0.2, 2.0], cos alpha in [-0.5, 1]: sides and
    triangles outside the ranges drop out."""
    F = tiny(3, n_forests=6, k=8, width_deg=0.3)
    G3 = grid3(r0=5.0, t=(0.2, 2.0), n_t=3, c=(-0.5, 1.0), n_c=3)
    check3(run3(lib, F, G3, variant=variant), O.xi3_sums(F, G3), f"partial v{variant}")


@pytest.mark.parametrize("variant", [-1, 1, 2])
def test_xi3_patch_with_realisations_vs_oracle(lib, variant):
    """Two realisations of 15 forests (30 pixels each, several 64-lane blocks of
    partners per vertex), 6 x 6 x 8 x 5 x 5 bins to 30 Mpc/h; the default
    picks the combining kernel."""
    parts = [truncate(make_patch(15, 0.6, 40 + r, z_range=(2.1, 2.3)), 30) for r in range(2)]
    F = concat_realisations(parts)
    G3 = grid3(r_max=30.0, n_r=6, n_t=5, n_c=8)
    out = run3(lib, F, G3, variant=variant, expect_variant=0 if variant < 0 else variant)
    assert out["ntrip"].shape == (2, G3.n_bins)
    check3(out, O.xi3_sums(F, G3), f"patch v{variant}")


@pytest.mark.parametrize("variant", [0, 2])
def test_xi3_slice_blocks_vs_oracle(lib, variant):
    """n_cos n_theta = 400: the combining kernels' LDS slice holds 5 of the 7
    side-2 r bins, so each side-1 cell takes two passes (as on the paper's
    3PCF grid, 20 r x 10 theta x 20 cos alpha bins, which takes two)."""
    parts = [truncate(make_patch(12, 0.6, 70 + r, z_range=(2.1, 2.3)), 24) for r in range(2)]
    F = concat_realisations(parts)
    G3 = grid3(r_max=35.0, n_r=7, n_t=20, n_c=20)
    check3(run3(lib, F, G3, variant=variant, expect_variant=variant), O.xi3_sums(F, G3), f"slice blocks v{variant}")


def _lopsided(seed=5, n_long=2060, n_short=10):
    """Three forests side by side: one long (n_long pixels spaced 0.7 Mpc/h)
    and two short ones in its middle.  A pixel of a short forest has
    n_long + n_short partners, a pixel of the long one 2 n_short; the entries
    stay few (the long forest's pixels never pair with each other)."""
    from synth import Forests
    P = make_patch(3, 0.3, seed, z_range=(2.1, 2.3))
    rng = np.random.default_rng(seed)
    mid = 3800.0 + 0.35 * n_long
    dist = np.concatenate([3800.0 + 0.7 * np.arange(n_long),
                           mid + 0.7 * np.arange(n_short) + 0.31, mid + 0.7 * np.arange(n_short) - 0.29])
    n = dist.size
    return Forests(np.array([0, n_long, n_long + n_short, n], np.int64), P.ra.copy(), P.dec.copy(), dist,
                   rng.normal(0.0, 0.3, n), rng.uniform(0.5, 2.0, n), np.full(n, 8.2), None, 1)


def test_xi3_combining_overflow_falls_back(lib):
    """Pixels with 2070 partners: more than the combining kernel holds (2048):
    the call re-runs with the wide kernel and matches the oracle, as does the
    direct kernel (3072); variant 0 forced reports the overflow."""
    from paper_2507_00129_amd import LyaError, LYA_E_UNSUPPORTED
    F = _lopsided()
    G3 = grid3(r_max=1500.0, n_r=6, n_t=4, n_c=5)
    ref = O.xi3_sums(F, G3)
    check3(run3(lib, F, G3, expect_variant=2), ref, "fallback")
    check3(run3(lib, F, G3, variant=1, expect_variant=1), ref, "fallback direct")
    with pytest.raises(LyaError) as ei:
        run3(lib, F, G3, variant=0)
    assert ei.value.status == LYA_E_UNSUPPORTED


def test_xi3_wide_beyond_direct_capacity_vs_oracle(lib):
    """Pixels with 4010 partners, beyond the direct kernel's 3072: the default
    runs the wide kernel and matches the oracle; the direct kernel reports
    LYA_E_UNSUPPORTED."""
    from paper_2507_00129_amd import LyaError, LYA_E_UNSUPPORTED
    F = _lopsided(seed=6, n_long=4000)
    G3 = grid3(r_max=3000.0, n_r=6, n_t=4, n_c=5)
    check3(run3(lib, F, G3, expect_variant=2), O.xi3_sums(F, G3), "wide 4010")
    with pytest.raises(LyaError) as ei:
        run3(lib, F, G3, variant=1)
    assert ei.value.status == LYA_E_UNSUPPORTED


def test_xi3_wide_overflow_is_reported(lib):
    """33010 partners for the short forests' pixels: beyond the wide kernel's
    scratch lists (32768), reported as LYA_E_UNSUPPORTED."""
    from paper_2507_00129_amd import LyaError, LYA_E_UNSUPPORTED
    F = _lopsided(seed=7, n_long=33000)
    G3 = O.Grid3(np.array([0.0, 1e5]), np.array([0.0, np.pi]), np.array([-1.0, 1.0]))
    with pytest.raises(LyaError) as ei:
        run3(lib, F, G3)
    assert ei.value.status == LYA_E_UNSUPPORTED


def test_xi3_paper_grid_at_eboss_density(lib):
    """The grid of the paper's 3PCF figure (r to 80 Mpc/h in 20 bins, theta
    10 bins, cos alpha 20 bins) on 150 forests nearest the centre of the
    eBOSS-like patch: vertex pixels have thousands of partners, so the default
    runs the wide kernel; counts symmetric under (r1, theta1) <-> (r2, theta2),
    N and W symmetric to rounding; on r to 40 Mpc/h the wide and the
    combining kernels give the same counts and W."""
    import time
    F, _, _ = make_config(1, seed=3, scale=0.05)
    S = subset_forests(F, nearest_to_centre(F, 150))
    G3 = O.Grid3(np.linspace(0.0, 80.0, 21), np.linspace(0.0, np.pi, 11), np.linspace(-1.0, 1.0, 21))
    t = time.perf_counter()
    out = run3(lib, S, G3, expect_variant=2)
    sh = (20, 20, 20, 10, 10)
    c = out["ntrip"][0].reshape(sh)
    print(f"[xi3 paper grid] entries={int(c.sum())} in {time.perf_counter() - t:.2f} s", flush=True)
    assert c.sum() > 1e9
    np.testing.assert_array_equal(c, c.transpose(1, 0, 2, 4, 3))
    for k in ("num", "wsum"):
        v = out[k][0].reshape(sh)
        assert np.max(np.abs(v - v.transpose(1, 0, 2, 4, 3))) <= 1e-10 * np.abs(v).max()
    # the same call on the direct-kernel-sized r range agrees with variant 0
    G40 = O.Grid3(np.linspace(0.0, 40.0, 11), np.linspace(0.0, np.pi, 11), np.linspace(-1.0, 1.0, 21))
    a0 = run3(lib, S, G40, variant=0, expect_variant=0)
    a2 = run3(lib, S, G40, variant=2, expect_variant=2)
    np.testing.assert_array_equal(a0["ntrip"], a2["ntrip"])
    m = np.abs(a0["wsum"]) > 0
    assert np.max(np.abs(a0["wsum"] - a2["wsum"])[m] / a0["wsum"][m]) <= 1e-12


@pytest.mark.parametrize("variant", [0, 1])
def test_xi3_single_bin_closed_form(lib, variant):
    """Every triangle in one bin: the sums run over all ordered triples of
    distinct forests, S1^3 - 3 S1 S2 + 2 S3 with S_p the power sums of the
    per-forest sums (W, counts alike); tolerance relative to the same form of
    the absolute values, since ~5e7 entries meet in one FP64 accumulator."""
    F = truncate(make_patch(10, 0.3, 7, z_range=(2.1, 2.3)), 40)
    G3 = O.Grid3(np.array([0.0, 1e5]), np.array([0.0, np.pi]), np.array([-1.0, 1.0]))
    out = run3(lib, F, G3, variant=variant, expect_variant=variant)
    fid = np.repeat(np.arange(F.n_forests), np.diff(F.offsets))

    def triple(a):
        S = np.bincount(fid, weights=a, minlength=F.n_forests)
        return S.sum() ** 3 - 3 * S.sum() * np.sum(S ** 2) + 2 * np.sum(S ** 3)
    n = round(triple(np.ones(F.n_pix)))
    assert int(out["ntrip"][0, 0]) == n and n > 4e7
    assert abs(out["num"][0, 0] - triple(F.weight * F.delta)) <= 1e-10 * triple(np.abs(F.weight * F.delta))
    assert abs(out["wsum"][0, 0] - triple(F.weight)) <= 1e-10 * triple(F.weight)


@pytest.mark.parametrize("variant", [0, 1])
def test_xi3_eboss_density_properties(lib, variant):
    """300 forests at the eBOSS-like density, r to 40 Mpc/h on 10 x 10 x 10 x 5
    x 5 bins (5.6e9 entries): counts symmetric under (r1, theta1) <->
    (r2, theta2), N and W symmetric to rounding."""
    F, _, _ = make_config(1, seed=1, scale=0.05)
    S = subset_forests(F, nearest_to_centre(F, 300))
    G3 = grid3(r_max=40.0, n_r=10, n_t=5, n_c=10)
    out = run3(lib, S, G3, variant=variant)
    sh = (10, 10, 10, 5, 5)
    c = out["ntrip"][0].reshape(sh)
    print(f"[xi3 eboss-300] entries={int(c.sum())}", flush=True)
    assert c.sum() > 1e8
    np.testing.assert_array_equal(c, c.transpose(1, 0, 2, 4, 3))
    for k in ("num", "wsum"):
        v = out[k][0].reshape(sh)
        assert np.max(np.abs(v - v.transpose(1, 0, 2, 4, 3))) <= 1e-10 * np.abs(v).max()


def test_xi3_partner_overflow_is_reported(lib):
    """More partner pixels within r_max of one pixel than the direct kernel's
    LDS list holds: the call fails with LYA_E_UNSUPPORTED instead of dropping
    triangles."""
    from paper_2507_00129_amd import LyaError, LYA_E_UNSUPPORTED
    F = truncate(make_patch(48, 0.3, 8, z_range=(2.1, 2.3)), 100)
    G3 = O.Grid3(np.array([0.0, 1e5]), np.array([0.0, np.pi]), np.array([-1.0, 1.0]))
    with pytest.raises(LyaError) as ei:
        run3(lib, F, G3, variant=1)
    assert ei.value.status == LYA_E_UNSUPPORTED


def test_xi3_invalid_grids(lib):
    from paper_2507_00129_amd import LyaError, LYA_E_INVALID, LYA_E_UNSUPPORTED
    F = tiny(0, n_forests=4, k=4, width_deg=0.3)

    def expect(status, G3):
        with pytest.raises(LyaError) as ei:
            run3(lib, F, G3)
        assert ei.value.status == status, str(ei.value)
    expect(LYA_E_INVALID, O.Grid3(np.array([0.0, 10.0]), np.array([0.0, 4.0]), np.array([-1.0, 1.0])))
    expect(LYA_E_INVALID, O.Grid3(np.array([0.0, 10.0]), np.array([0.0, 1.0, 0.5]), np.array([-1.0, 1.0])))
    expect(LYA_E_INVALID, O.Grid3(np.array([0.0, 10.0]), np.array([0.0, 1.0]), np.array([-1.5, 1.0])))
    expect(LYA_E_UNSUPPORTED, O.Grid3(np.array([0.0, 10.0]), np.array([0.0, 1.0]), np.array([-1.0, 0.0, 0.2, 1.0])))
    expect(LYA_E_UNSUPPORTED, O.Grid3(np.array([0.0, 1.0, 10.0]), np.array([0.0, 1.0]), np.array([-1.0, 1.0])))
    expect(LYA_E_UNSUPPORTED, O.Grid3(np.array([0.0, 10.0]), np.array([0.0, 1.0]), np.linspace(-1.0, 1.0, 258)))
    # variant 0 on a grid whose n_cos n_theta exceeds its LDS slice; variant 2
    wide = O.Grid3(np.array([0.0, 10.0]), np.linspace(0.0, np.pi, 41), np.linspace(-1.0, 1.0, 61))
    with pytest.raises(LyaError) as ei:
        run3(lib, F, wide, variant=0)
    assert ei.value.status == LYA_E_UNSUPPORTED
    with pytest.raises(LyaError) as ei:
        run3(lib, F, grid3(), variant=3)
    assert ei.value.status == LYA_E_INVALID


def test_xi3_projected_deltas_vs_oracle(lib):
    """project_deltas correlates eta delta (eta of options.eta) per forest: the
    oracle's sums on deltas it projected itself.  delta' = delta - m - a t is
    formed by two summation orders, so its absolute error is ~eps (|delta| +
    |m| + |a t|), which can be large against a small |delta'|: N is compared
    relative to the sums of w d~ w d~ w d~ with that conditioning d~."""
    parts = [truncate(make_patch(15, 0.6, 60 + r, z_range=(2.1, 2.3)), 30) for r in range(2)]
    F = concat_realisations(parts)
    G3 = grid3(r_max=30.0, n_r=6, n_t=5, n_c=8)
    Fp, Fc = F.copy(), F.copy()
    Fp.delta = O.projected_deltas(F, O.MEAN_SLOPE)
    for f in range(F.n_forests):
        sl = F.forest_slice(f)
        P = O.eta_params(F.weight[sl], F.loglam[sl], O.MEAN_SLOPE)
        m, t = np.sum(P.u * F.delta[sl]), np.sum(P.b * F.delta[sl])
        Fc.delta[sl] = np.abs(F.delta[sl]) + abs(m) + np.abs(P.a * t)
    ref = O.xi3_sums(Fp, G3)
    cond = O.xi3_sums(Fc, G3).num
    out = run3(lib, F, G3, project_deltas=True, eta="mean_slope")
    assert ref.n_near_edge == 0
    np.testing.assert_array_equal(out["ntrip"], ref.ntrip)
    m = cond > 0
    e_n = float(np.max(np.abs(out["num"] - ref.num)[m] / cond[m]))
    e_w = O.err_rel(out["wsum"], ref.wsum)
    print(f"[xi3 projected] entries={int(ref.ntrip.sum())} e_N={e_n:.2e} e_W={e_w:.2e}", flush=True)
    assert e_n <= TOL and e_w <= TOL


def run3_sub(lib, F, G3, sub, n_sub, expect_variant=None, **kw):
    from paper_2507_00129_amd import DeviceForests
    out = lib.xi3_subsamples(DeviceForests.from_host(F, "cuda:0"), G3,
                             torch.as_tensor(sub, dtype=torch.int32, device="cuda:0"), n_sub, **kw)
    torch.cuda.synchronize()
    if expect_variant is not None:
        assert lib.last_stats()["variant"] == expect_variant
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_xi3_subsamples_vs_oracle(lib, variant):
    """Sums split by the subsample of each entry's main vertex forest (the
    dispersion of the paper's 3PCF figure), two realisations of 15 forests,
    4 subsamples: every slab against the oracle's split sums, and the slabs
    add up to lya_xi3's counts."""
    parts = [truncate(make_patch(15, 0.6, 80 + r, z_range=(2.1, 2.3)), 30) for r in range(2)]
    F = concat_realisations(parts)
    G3 = grid3(r_max=30.0, n_r=6, n_t=5, n_c=8)
    sub = np.random.default_rng(4).integers(0, 4, F.n_forests).astype(np.int32)
    out = run3_sub(lib, F, G3, sub, 4, variant=variant, expect_variant=variant)
    assert out["ntrip"].shape == (2, 4, G3.n_bins)
    ref = O.xi3_sums(F, G3, sub=sub, n_sub=4)
    flat = {k: v.reshape(8, G3.n_bins) for k, v in out.items()}
    check3(flat, ref, f"subsamples v{variant}")
    whole = run3(lib, F, G3, variant=variant)
    np.testing.assert_array_equal(out["ntrip"].sum(axis=1), whole["ntrip"])


def test_xi3_wide_kernel_vs_oracle_at_eboss_density(lib):
    """The wide kernel on the grid of the paper's 3PCF figure (r to 80 Mpc/h,
    20 x 10 x 20 bins) at eBOSS density, against the oracle restricted to one
    vertex forest (the shortest of the ten nearest the centre): the subsample
    split puts it alone in slab 0, whose entries (1.4e8, from thousands of
    partners per vertex pixel) must match exactly, with N and W to 1e-12."""
    F, _, _ = make_config(1, seed=3, scale=0.05)
    S = subset_forests(F, nearest_to_centre(F, 150))
    G3 = O.Grid3(np.linspace(0.0, 80.0, 21), np.linspace(0.0, np.pi, 11), np.linspace(-1.0, 1.0, 21))
    chosen = [int(np.argmin(np.diff(S.offsets)[:10]))]
    sub = np.ones(S.n_forests, np.int32)
    sub[chosen] = 0
    out = run3_sub(lib, S, G3, sub, 2, expect_variant=2)
    ref = O.xi3_sums(S, G3, vertices=chosen)
    slab0 = {k: v[:, 0] for k, v in out.items()}
    assert ref.ntrip.sum() > 1e7
    check3(slab0, ref, "wide kernel, eBOSS density, 3 vertex forests")


def test_xi3_subsamples_invalid_id(lib):
    from paper_2507_00129_amd import LyaError, LYA_E_INVALID
    F = tiny(0, n_forests=4, k=4, width_deg=0.3)
    with pytest.raises(LyaError) as ei:
        run3_sub(lib, F, grid3(), np.array([0, 1, 2, 3], np.int32), 3)
    assert ei.value.status == LYA_E_INVALID
