"""GPU parity of lya_dmat against the FP64 oracle (Sec. 2.2, eq. distortion).
Tolerances: e_D = max_A max_B |dD_AB| / max_B |D_AB| (row-normwise) and the
max relative error of w_A, 1e-12 for the FP64 form and 1e-5 for FP32."""
import numpy as np
import pytest

import oracle as O
from synth import Grid, concat_realisations, make_config, make_patch, subset_forests, uniform_grid
from synth.survey import nearest_to_centre

from helpers import tiny, truncate
from test_gpu_xi import _ragged_forests

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
G60 = uniform_grid(15, 60.0)
# kernel variants: 0 the 8-wave kernel with a full tile; 1 and 2 the
# upper-triangle tile kernels (large tile: two waves per workgroup in the FP32
# form, one in FP64; small tile: one wave); 3 the hybrid launch (small tile for
# one-tile windows, large tile for the rest)
VARIANTS = [0, 1, 2, 3]
ETA = {"identity": O.IDENTITY, "mean": O.MEAN, "mean_slope": O.MEAN_SLOPE}


@pytest.fixture(scope="module")
def lib():
    from paper_2507_00129_amd import Library
    L = Library(0)
    yield L
    L.close()


def run_dmat(lib, F, G, **kw):
    """A launch with the work counters (the first pass of a window then takes
    every pixel within r_par reach, and the counters check that every in-grid
    pixel pair falls inside its forest pair's r_perp window), then the launch
    as timed, without counters (every pass of a wide window takes only the
    pixels that can reach its blocks); both outputs are returned."""
    from paper_2507_00129_amd import DeviceForests
    dF = DeviceForests.from_host(F, "cuda:0")
    counted = lib.dmat(dF, G, timing=True, counters=True, **kw)
    torch.cuda.synchronize()
    st = lib.last_stats()
    assert st["lost_pairs"] == 0, st
    out = {k + "_counted": v.cpu().numpy() for k, v in counted.items()}
    del counted
    plain = lib.dmat(dF, G, timing=True, **kw)
    torch.cuda.synchronize()
    out.update({k: v.cpu().numpy() for k, v in plain.items()})
    return out


def check(out, ref, prec, what):
    for sfx in ("", "_counted"):
        e_d = O.err_rows(out["dmat" + sfx], ref.D)
        e_w = O.err_rel(out["wsum_d" + sfx], ref.wd)
        print(f"[{what}{sfx} {prec}] rows={int((ref.wd > 0).sum())} e_D={e_d:.3e} e_W={e_w:.3e}", flush=True)
        assert e_d <= TOL[prec] and e_w <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("eta", ["mean", "mean_slope"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_tiny_against_four_nested_sums(lib, prec, eta, variant):
    F = tiny(0, n_forests=3, k=6)
    G = uniform_grid(4, 24.0, 3, 30.0)
    pairs = O.dmat_pairs(F, G)
    ref = O.dmat_brute(F, G, pairs, ETA[eta])
    out = run_dmat(lib, F, G, precision=prec, eta=eta, variant=variant, autotune=False)
    check(out, ref, prec, f"tiny-{eta}-v{variant}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_config0(lib, prec, variant):
    F, G, _ = make_config(0, seed=0)
    ref = O.dmat(F, G, O.dmat_pairs(F, G))
    out = run_dmat(lib, F, G, precision=prec, variant=variant, autotune=False)
    check(out, ref, prec, f"config0-v{variant}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_identity_eta_gives_identity(lib, prec, variant):
    F, G, _ = make_config(0, seed=1, scale=0.5)
    out = run_dmat(lib, F, G, precision=prec, eta="identity", variant=variant, autotune=False)
    D, wd = out["dmat"][0], out["wsum_d"][0]
    rows = wd > 0
    assert rows.sum() > 50
    sub = D[np.ix_(rows, rows)]
    assert np.abs(np.diag(sub) - 1.0).max() < 1e-13
    assert not (sub - np.diag(np.diag(sub))).any()
    assert not D[~rows].any()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("eta", ["mean", "mean_slope"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_covering_grid_row_sums(lib, prec, eta, variant):
    """A uniform grid holding every pair of these compact forests (r < 400
    Mpc/h): the eta rows sum to zero, so every row of D does too."""
    F = tiny(4, n_forests=6, k=40)
    G = uniform_grid(50, 400.0)
    ref = O.xi_sums(F, G)
    n = np.diff(F.offsets)
    assert ref.npairs.sum() == (n.sum() ** 2 - np.sum(n ** 2)) // 2
    out = run_dmat(lib, F, G, precision=prec, eta=eta, variant=variant, autotune=False)
    D = out["dmat"][0]
    assert np.abs(D).max() > 0.1
    assert np.abs(D.sum(1)).max() <= (1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_keep_fraction_subset(lib, prec):
    F, G, _ = make_config(0, seed=2)
    p, seed = 0.35, 11
    ref = O.dmat(F, G, O.dmat_pairs(F, G, p, seed))
    out = run_dmat(lib, F, G, precision=prec, keep_fraction=p, seed=seed)
    check(out, ref, prec, "subset")
    full = run_dmat(lib, F, G, precision=prec)
    assert O.err_rows(full["dmat"], ref.D) > 1e-3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ragged(lib, prec):
    F = _ragged_forests(7)
    ref = O.dmat(F, G60, O.dmat_pairs(F, G60))
    for v in VARIANTS:
        out = run_dmat(lib, F, G60, precision=prec, variant=v, autotune=False)
        check(out, ref, prec, f"ragged-v{v}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_realisations(lib, prec, variant):
    parts = [make_patch(n, 2.0, 60 + r) for r, n in enumerate((20, 33, 27))]
    F = concat_realisations(parts)
    ref = O.dmat(F, G60, O.dmat_pairs(F, G60))
    out = run_dmat(lib, F, G60, precision=prec, variant=variant, autotune=False)
    assert out["dmat"].shape == (3, G60.n_bins, G60.n_bins)
    check(out, ref, prec, f"realisations-v{variant}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config1_compact_subpatch(lib, prec):
    """eBOSS-like forests on the 50x50 grid to 200 Mpc/h (pairs touching more
    bins than one LDS tile holds)."""
    F, G, _ = make_config(1, seed=0, scale=0.02)
    S = subset_forests(F, nearest_to_centre(F, 60))
    ref = O.dmat(S, G, O.dmat_pairs(S, G))
    for v in VARIANTS:
        out = run_dmat(lib, S, G, precision=prec, variant=v, autotune=False)
        check(out, ref, prec, f"config1-sub-v{v}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n_par", [100, 120])
def test_windows_wider_than_one_tile(lib, prec, n_par):
    """n_par r_par bins of 2 Mpc/h make every r_perp window n_par, 2 n_par or
    3 n_par bins wide; windows wider than a tile (variant 0: 160 bins in the
    FP64 form, 224 in the FP32 form; variants 1 and 2: 112 and 80 (FP64), 160
    and 128 (FP32)) are covered by several tiles and passes per run, diagonal
    and rectangle passes in variants 1 and 2."""
    F, _, _ = make_config(1, seed=3, scale=0.02)
    S = subset_forests(F, nearest_to_centre(F, 40))
    G = uniform_grid(n_par, 2.0 * n_par, 12, 60.0)
    ref = O.dmat(S, G, O.dmat_pairs(S, G))
    for v in VARIANTS:
        out = run_dmat(lib, S, G, precision=prec, variant=v, autotune=False)
        check(out, ref, prec, f"wide-windows-v{v}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wide_windows_nonzero_first_edges(lib, prec):
    """Windows of one and two k_perp rows of 100 bins (up to 15 passes on the
    smallest tile) on a grid whose first r_par and r_perp edges are not zero
    (the kernels' general range tests), against the oracle: the per-pass pixel
    ranges map window blocks to r_perp through the edges from the window's
    first k_perp row."""
    F, _, _ = make_config(1, seed=4, scale=0.02)
    S = subset_forests(F, nearest_to_centre(F, 40))
    G = Grid(np.linspace(1.0, 201.0, 101), np.linspace(2.0, 62.0, 16))
    ref = O.dmat(S, G, O.dmat_pairs(S, G))
    for v in VARIANTS:
        out = run_dmat(lib, S, G, precision=prec, variant=v, autotune=False)
        check(out, ref, prec, f"wide-offset-v{v}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_config0_against_definition(lib, prec, variant):
    """Config 0 against eq. distortion with each forest pair's inner double sum
    formed as eta_f M^B eta_g^T (oracle.dmat_definition): no factorisation in
    common with the kernels."""
    F, G, _ = make_config(0, seed=0)
    ref = O.dmat_definition(F, G, O.dmat_pairs(F, G))
    out = run_dmat(lib, F, G, precision=prec, variant=variant, autotune=False)
    check(out, ref, prec, f"config0-definition-v{variant}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_realisations_against_definition(lib, prec, variant):
    """Three realisations of short forests (a few hundred pixels each, many
    touched bins per forest pair) against the definition form."""
    parts = [truncate(make_patch(n, 1.0, 90 + r, z_range=(2.1, 2.4)), 40) for r, n in enumerate((9, 14, 11))]
    F = concat_realisations(parts)
    G = uniform_grid(12, 60.0, 10, 40.0)
    ref = O.dmat_definition(F, G, O.dmat_pairs(F, G))
    assert (ref.wd > 0).sum() > 100
    out = run_dmat(lib, F, G, precision=prec, variant=variant, autotune=False)
    check(out, ref, prec, f"realisations-definition-v{variant}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_config1_subpatch_120(lib, prec, variant):
    """The 120 forests nearest the centre of an eBOSS-like patch on the 50x50
    grid to 200 Mpc/h (7e3 forest pairs, long runs of pairs per tile)."""
    F, G, _ = make_config(1, seed=0, scale=0.02)
    S = subset_forests(F, nearest_to_centre(F, 120))
    ref = O.dmat(S, G, O.dmat_pairs(S, G))
    out = run_dmat(lib, S, G, precision=prec, variant=variant, autotune=False)
    check(out, ref, prec, f"config1-sub120-v{variant}")


def test_full_config1_fp32_vs_fp64(lib):
    """The full eBOSS-like patch (30k forests, all 1.9e7 forest pairs): the
    FP32 form's D against the FP64 form's, row-normwise within 1e-5, w_A
    within 1e-5 (launches as timed, without counters), and no in-grid pixel
    pair outside its window (launches with counters)."""
    import time
    from paper_2507_00129_amd import DeviceForests
    F, G, _ = make_config(1, seed=0)
    dF = DeviceForests.from_host(F, "cuda:0")
    out = {}
    for prec in ("fp64", "fp32"):
        t = time.perf_counter()
        o = lib.dmat(dF, G, precision=prec, timing=True, counters=True)
        torch.cuda.synchronize()
        st = lib.last_stats()
        assert st["lost_pairs"] == 0, st
        del o
        o = lib.dmat(dF, G, precision=prec, timing=True)
        torch.cuda.synchronize()
        out[prec] = {k: v.cpu().numpy() for k, v in o.items()}
        print(f"[dmat full {prec}] forest pairs={st['forest_pairs']} in-grid pairs={st['ingrid_pairs']:.4e} "
              f"kernel={st['ms_main']:.0f} ms call={(time.perf_counter() - t) * 1e3:.0f} ms", flush=True)
        del o
    e_d = O.err_rows(out["fp32"]["dmat"], out["fp64"]["dmat"])
    e_w = O.err_rel(out["fp32"]["wsum_d"], out["fp64"]["wsum_d"])
    print(f"[dmat full] fp32 vs fp64: e_D={e_d:.2e} e_W={e_w:.2e}", flush=True)
    assert e_d <= 1e-5 and e_w <= 1e-5
