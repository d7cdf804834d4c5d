"""Batched multi-realisation launches: many independent mock realisations of
uneven size in one persistent launch, checked against the FP64 oracle on a
small case and against separate single-realisation runs at larger scale."""
import numpy as np
import pytest

import oracle as O
from synth import make_config, subset_forests

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2507_00129_amd import Library
    L = Library(0)
    yield L
    L.close()


def realisation(F, r):
    idx = np.nonzero(F.realisation == r)[0]
    S = subset_forests(F, idx)
    S.realisation = None
    S.n_realisations = 1
    return S


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_small_batched_vs_oracle(lib, prec, tol):
    from paper_2507_00129_amd import DeviceForests
    F, G, _ = make_config(3, seed=1, scale=0.01)
    assert F.n_realisations >= 2
    ref = O.xi_sums(F, G)
    out = lib.xi(DeviceForests.from_host(F), G, precision=prec)
    n = out["npairs"].cpu().numpy()
    np.testing.assert_array_equal(n, ref.npairs)
    e = O.err_xi(out["xi"].cpu().numpy(), ref.xi, ref.wsum, ref.absnum)
    print(f"[batched-oracle {prec}] R={F.n_realisations} pairs={int(n.sum())} e_xi={e:.2e}", flush=True)
    assert e <= tol


def test_batched_matches_separate_runs(lib):
    """26 realisations of 200-2000 forests in one launch vs 26 launches: pair
    counts identical, sums within 1e-6 of each bin's absolute sum (FP32)."""
    from paper_2507_00129_amd import DeviceForests
    F, G, ex = make_config(3, seed=0, scale=0.1)
    R = F.n_realisations
    dF = DeviceForests.from_host(F)
    bat = {k: v.cpu().numpy() for k, v in lib.xi(dF, G, precision="fp32").items()}
    absn = lib.xi(dF.with_values(delta=dF.delta.abs()), G, precision="fp64")["num"].cpu().numpy()
    worst = 0.0
    for r in range(R):
        S = realisation(F, r)
        sep = {k: v.cpu().numpy() for k, v in lib.xi(DeviceForests.from_host(S), G, precision="fp32").items()}
        np.testing.assert_array_equal(sep["npairs"][0], bat["npairs"][r])
        m = absn[r] > 0
        worst = max(worst, float(np.max(np.abs(sep["num"][0] - bat["num"][r])[m] / absn[r][m])))
        assert O.err_rel(sep["wsum"][0], bat["wsum"][r]) <= 1e-6
    print(f"[batched-vs-separate] R={R} forests={F.n_forests} worst e_N={worst:.2e}", flush=True)
    assert worst <= 1e-6


def test_batched_dmat_and_backward_match_separate(lib):
    """D and the xi gradient of a batched launch equal those of separate runs
    (all forest pairs kept; FP64 form)."""
    from paper_2507_00129_amd import DeviceForests
    F, G, _ = make_config(3, seed=2, scale=0.02)
    R = F.n_realisations
    assert R >= 3
    dF = DeviceForests.from_host(F)
    Dall = lib.dmat(dF, G, precision="fp64")["dmat"].cpu().numpy()
    bx = lib.xi(dF, G, precision="fp64")
    gd, gw = lib.xi_backward(dF, G, 2.0 * (bx["xi"] - 0.002), bx["xi"], bx["wsum"], precision="fp64")
    gd, gw = gd.cpu().numpy(), gw.cpu().numpy()
    for r in range(R):
        idx = np.nonzero(F.realisation == r)[0]
        dS = DeviceForests.from_host(realisation(F, r))
        sd = lib.dmat(dS, G, precision="fp64")["dmat"].cpu().numpy()[0]
        assert O.err_rows(sd, Dall[r]) <= 1e-12
        sx = lib.xi(dS, G, precision="fp64")
        sgd, sgw = lib.xi_backward(dS, G, 2.0 * (sx["xi"] - 0.002), sx["xi"], sx["wsum"], precision="fp64")
        pix = np.concatenate([np.arange(F.offsets[f], F.offsets[f + 1]) for f in idx])
        assert O.err_norm(sgd.cpu().numpy(), gd[pix]) <= 1e-12
        assert O.err_norm(sgw.cpu().numpy(), gw[pix]) <= 1e-12
    print(f"[batched D/backward] R={R} forests={F.n_forests}", flush=True)


def test_full_batched_workload_vs_separate_runs(lib):
    """The full batched covariance workload: 64 realisations of 2k-20k forests
    (~7e5 forests, ~6.7e7 pixels) in one persistent launch (FP32, the launch
    the autotuner picks) against 64 separate single-realisation launches:
    pair counts identical, sums within 1e-6 of each bin's absolute sum."""
    import time
    from paper_2507_00129_amd import DeviceForests
    F, G, ex = make_config(3, seed=0)
    R = F.n_realisations
    assert R == 64
    dF = DeviceForests.from_host(F)
    lib.xi(dF, G, precision="fp32")  # autotune and warm up
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = lib.xi(dF, G, precision="fp32", timing=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    st = lib.last_stats()
    bat = {k: v.cpu().numpy() for k, v in out.items()}
    pairs = int(bat["npairs"].sum())
    print(f"[batched full] R={R} forests={F.n_forests} pixels={F.n_pix} pairs={pairs:.4e} "
          f"kernel={st['ms_main']:.1f} ms ({pairs / st['ms_main'] * 1e3:.3e} pairs/s) call={wall * 1e3:.1f} ms",
          flush=True)
    absn = lib.xi(dF.with_values(delta=dF.delta.abs()), G, precision="fp64")["num"].cpu().numpy()
    del dF
    worst_n = worst_w = 0.0
    for r in range(R):
        S = realisation(F, r)
        sep = {k: v.cpu().numpy() for k, v in lib.xi(DeviceForests.from_host(S), G, precision="fp32").items()}
        np.testing.assert_array_equal(sep["npairs"][0], bat["npairs"][r])
        m = absn[r] > 0
        worst_n = max(worst_n, float(np.max(np.abs(sep["num"][0] - bat["num"][r])[m] / absn[r][m])))
        worst_w = max(worst_w, O.err_rel(sep["wsum"][0], bat["wsum"][r]))
    print(f"[batched full] separate vs batched: e_N={worst_n:.2e} e_W={worst_w:.2e}", flush=True)
    assert worst_n <= 1e-6 and worst_w <= 1e-6
