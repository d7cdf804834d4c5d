"""options.deterministic of lya_xi (the sums of Sec. 2.1, eq. estimator_two
with order-independent fixed-point accumulation): parity with the FP64 oracle
at the bar of each precision, bitwise-identical repeats, and a realisation's
sums bitwise identical whether it runs alone or batched with others."""
import numpy as np
import pytest

import oracle as O
from synth import concat_realisations, make_config, make_patch, uniform_grid

from test_gpu_xi import _ragged_forests, check, run_xi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G60 = uniform_grid(15, 60.0)


@pytest.fixture(scope="module")
def lib():
    from paper_2507_00129_amd import Library
    L = Library(0)
    yield L
    L.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deterministic_config0_vs_oracle(lib, prec):
    F, G, _ = make_config(0, seed=0)
    check(run_xi(lib, F, G, precision=prec, deterministic=True), O.xi_sums(F, G), prec, "det config0")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deterministic_ragged_and_projected_vs_oracle(lib, prec):
    F = _ragged_forests(21)
    check(run_xi(lib, F, G60, precision=prec, deterministic=True), O.xi_sums(F, G60), prec, "det ragged")
    Fp = F.copy()
    Fp.delta = O.projected_deltas(F, O.MEAN_SLOPE)
    out = run_xi(lib, F, G60, precision=prec, deterministic=True, project_deltas=True, eta="mean_slope")
    ref = O.xi_sums(Fp, G60)
    np.testing.assert_array_equal(out["npairs"], ref.npairs)
    assert O.err_rel(out["wsum"], ref.wsum) <= {"fp64": 1e-12, "fp32": 1e-5}[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deterministic_repeats_are_bitwise_identical(lib, prec):
    """The eBOSS-like density on 2000 forests: two calls give the same bits
    (the default form's FP64 atomics need not)."""
    from synth import subset_forests
    from synth.survey import nearest_to_centre
    F, G, _ = make_config(1, seed=2, scale=0.1)
    S = subset_forests(F, nearest_to_centre(F, 2000))
    a = run_xi(lib, S, G, precision=prec, deterministic=True)
    b = run_xi(lib, S, G, precision=prec, deterministic=True)
    for k in ("num", "wsum", "npairs", "xi"):
        assert np.array_equal(a[k].view(np.uint64), b[k].view(np.uint64)), k
    d = run_xi(lib, S, G, precision=prec)
    np.testing.assert_array_equal(d["npairs"], a["npairs"])
    absn = run_xi(lib, _abs(S), G, precision="fp64")["num"]
    m = absn > 0
    e = float(np.max(np.abs(a["num"] - d["num"])[m] / absn[m]))
    print(f"[det repeats {prec}] pairs={int(a['npairs'].sum())} det vs default e_N={e:.2e}", flush=True)
    assert e <= {"fp64": 1e-12, "fp32": 1e-5}[prec]


def _abs(F):
    G = F.copy()
    G.delta = np.abs(F.delta)
    return G


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deterministic_batched_equals_separate_bitwise(lib, prec):
    """Five realisations of different sizes and value ranges in one call: each
    realisation's outputs carry the same bits as the realisation run alone."""
    parts = []
    for r, (n, scale) in enumerate(((40, 1.0), (70, 1e-3), (25, 50.0), (55, 1.0), (10, 7.0))):
        P = make_patch(n, 2.0, 300 + r)
        P.weight = P.weight * scale
        parts.append(P)
    F = concat_realisations(parts)
    bat = run_xi(lib, F, G60, precision=prec, deterministic=True)
    assert bat["num"].shape == (5, G60.n_bins)
    for r, P in enumerate(parts):
        sep = run_xi(lib, P, G60, precision=prec, deterministic=True)
        for k in ("num", "wsum", "npairs", "xi"):
            assert np.array_equal(sep[k][0].view(np.uint64), bat[k][r].view(np.uint64)), (r, k)
    print(f"[det batched {prec}] pairs={int(bat['npairs'].sum())} bitwise equal", flush=True)


def test_deterministic_rejected_by_other_calls(lib):
    from paper_2507_00129_amd import DeviceForests, LyaError, LYA_E_UNSUPPORTED
    F, G, _ = make_config(0, seed=0)
    dF = DeviceForests.from_host(F, "cuda:0")
    sub = torch.zeros(F.n_forests, dtype=torch.int32, device="cuda:0")
    g3 = O.Grid3(np.linspace(0.0, 20.0, 3), np.linspace(0.0, np.pi, 3), np.linspace(-1.0, 1.0, 3))
    calls = [lambda: lib.xi_means(dF, G, deterministic=True),
             lambda: lib.xi_subsamples(dF, G, sub, 1, deterministic=True),
             lambda: lib.dmat(dF, G, deterministic=True),
             lambda: lib.xi3(dF, g3, deterministic=True)]
    for c in calls:
        with pytest.raises(LyaError) as ei:
            c()
        assert ei.value.status == LYA_E_UNSUPPORTED


def test_full_batched_workload_deterministic_bitwise(lib):
    """The full batched covariance workload (64 realisations of 2k-20k
    forests, ~6.7e7 pixels, FP32 form) in one deterministic launch against 64
    separate deterministic launches: every realisation's N, W, counts and xi
    carry the same bits."""
    import time
    from paper_2507_00129_amd import DeviceForests
    from test_gpu_batched import realisation
    F, G, _ = make_config(3, seed=0)
    assert F.n_realisations == 64
    dF = DeviceForests.from_host(F)
    t = time.perf_counter()
    out = lib.xi(dF, G, precision="fp32", deterministic=True, timing=True)
    torch.cuda.synchronize()
    st = lib.last_stats()
    bat = {k: v.cpu().numpy() for k, v in out.items()}
    del dF, out
    print(f"[det batched full] pixels={F.n_pix} pairs={int(bat['npairs'].sum()):.4e} "
          f"kernel={st['ms_main']:.1f} ms call={(time.perf_counter() - t) * 1e3:.1f} ms", flush=True)
    for r in range(F.n_realisations):
        S = realisation(F, r)
        sep = {k: v.cpu().numpy() for k, v in lib.xi(DeviceForests.from_host(S), G, precision="fp32",
                                                      deterministic=True).items()}
        for k in ("num", "wsum", "npairs", "xi"):
            assert np.array_equal(sep[k][0].view(np.uint64), bat[k][r].view(np.uint64)), (r, k)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deterministic_batched_with_different_min_distance(lib, prec):
    """A high-redshift realisation (its pixels start above 3600 A, so its
    smallest distance is larger than the other realisations') in a batch: the
    sky index's strip height follows the smallest distance of the whole call,
    so it differs between the batched and the separate run, yet the
    realisation's sums keep their bits (the row forest of a pair is the one
    with the smaller input index, whatever the strips)."""
    parts = [make_patch(80, 2.0, 411, z_range=(3.0, 3.5)), make_patch(80, 2.0, 412),
             make_patch(50, 2.0, 413, z_range=(2.1, 2.3))]
    assert parts[0].dist.min() > parts[1].dist.min() + 200.0
    F = concat_realisations(parts)
    bat = run_xi(lib, F, G60, precision=prec, deterministic=True)
    for r, P in enumerate(parts):
        sep = run_xi(lib, P, G60, precision=prec, deterministic=True)
        assert sep["npairs"].sum() > 0
        for k in ("num", "wsum", "npairs", "xi"):
            assert np.array_equal(sep[k][0].view(np.uint64), bat[k][r].view(np.uint64)), (r, k)
    print(f"[det min-distance {prec}] pairs={int(bat['npairs'].sum())} bitwise equal", flush=True)
