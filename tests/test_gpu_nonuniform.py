"""Grids with non-uniform bin edges (any strictly increasing edges for the
(r_par, r_perp) bins of Sec. 2.1): xi, the bin means, the gradient and D on the
GPU against the FP64 oracle, which bins by searching the edge arrays.  On such
a grid every pair in range is binned by searching the FP64 edge arrays on the
GPU too, so pair counts must match exactly, also for pairs placed exactly on
an edge.  Tolerances as for the uniform grids: 1e-12 (FP64 form), 1e-5 (FP32
form)."""
import numpy as np
import pytest

import oracle as O
from synth import Grid, make_config, subset_forests
from synth.survey import nearest_to_centre

from test_gpu_xi import check as check_xi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
GRIDS = {
    # the covering grid of the oracle pins: one 4 Mpc/h bin and one that holds
    # every other separation on each axis
    "covering": Grid(np.array([0.0, 4.0, 1e5]), np.array([0.0, 4.0, 1e5])),
    # graded widths, a non-zero first r_perp edge
    "graded": Grid(np.array([0.0, 2.0, 5.0, 9.0, 14.0, 20.0, 27.0, 35.0, 44.0, 54.0, 60.0]),
                   np.array([0.5, 3.0, 7.0, 12.0, 18.0, 25.0, 33.0, 42.0, 52.0, 60.0])),
    # a uniform grid with one interior edge moved by 1e-7 Mpc/h (2.5e-8 of a bin)
    "nudged": Grid(np.linspace(0.0, 60.0, 16) + np.where(np.arange(16) == 7, 1e-7, 0.0),
                   np.linspace(0.0, 60.0, 16)),
}


@pytest.fixture(scope="module")
def lib():
    from paper_2507_00129_amd import Library
    L = Library(0)
    yield L
    L.close()


def dev(F):
    from paper_2507_00129_amd import DeviceForests
    return DeviceForests.from_host(F, "cuda:0")


def host(out):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("grid", sorted(GRIDS))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_xi_vs_oracle(lib, grid, prec):
    G = GRIDS[grid]
    F, _, _ = make_config(0, seed=5)
    ref = O.xi_sums(F, G)
    for v in (0, 3):
        out = host(lib.xi(dev(F), G, precision=prec, variant=v, autotune=False))
        check_xi(out, ref, prec, f"{grid} v{v}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pairs_exactly_on_edges(lib, prec):
    """Interior edges set to separations that pixel pairs of the input have
    exactly (in FP64): each such pair belongs to the bin above the edge."""
    F, _, _ = make_config(0, seed=6)
    n = O.unit_vectors(F.ra, F.dec)
    # the first forest pair with in-grid separations on both axes
    for f in range(F.n_forests):
        g = f + 1 + int(np.argmin(np.sum((n[f + 1:] - n[f]) ** 2, axis=1)))
        s, c = O.pair_sc(n[f], n[g])
        rp, rt = O.separations(F.dist[F.forest_slice(f)][:, None], F.dist[F.forest_slice(g)][None, :], s, c)
        ok = (rp < 55.0) & (rt < 55.0)
        rp, rt = np.unique(rp[ok]), np.unique(rt[ok])
        if rp.size >= 6 and rt.size >= 2:
            break
    assert rp.size >= 6 and rt.size >= 2, "choose another seed"
    ep = np.unique(np.concatenate([[0.0], rp[:: max(1, rp.size // 5)][1:6], [60.0]]))
    et = np.unique(np.concatenate([[0.0], rt[:2], [60.0]]))
    G = Grid(ep, et)
    ref = O.xi_sums(F, G)
    out = host(lib.xi(dev(F), G, precision=prec))
    np.testing.assert_array_equal(out["npairs"], ref.npairs)
    assert O.err_xi(out["xi"], ref.xi, ref.wsum, ref.absnum) <= TOL[prec]
    assert O.err_rel(out["wsum"], ref.wsum) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_means_vs_oracle(lib, prec):
    """Bin-mean coordinates: within 1e-12 (FP64) or 1e-4 (FP32) of the mean bin
    width, as on uniform grids (the FP32 form's means come from coordinates in
    units of the mean width, with the same error bound)."""
    G = GRIDS["graded"]
    F, _, _ = make_config(0, seed=7)
    ref = O.xi_sums(F, G, means=True)
    out = host(lib.xi_means(dev(F), G, precision=prec))
    np.testing.assert_array_equal(out["npairs"], ref.npairs)
    rp, rt, z = O.bin_means(ref)
    wp = (G.edges_par[-1] - G.edges_par[0]) / G.n_par
    wt = (G.edges_perp[-1] - G.edges_perp[0]) / G.n_perp
    tol_r, tol_z = {"fp64": (1e-12, 1e-12), "fp32": (1e-4, 1e-6)}[prec]
    assert float(np.max(np.abs(out["rpar"] - rp))) / wp <= tol_r
    assert float(np.max(np.abs(out["rperp"] - rt))) / wt <= tol_r
    assert O.err_rel(out["z"], z) <= tol_z


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gradient_vs_oracle(lib, prec):
    G = GRIDS["graded"]
    F, _, _ = make_config(0, seed=8)
    target = np.random.default_rng(8).uniform(-0.01, 0.01, G.n_bins)
    X = O.xi_sums(F, G)
    rd, rw = O.xi_grad(F, G, O.loss_grad_xi(X.xi, target[None, :]), X.xi, X.wsum)
    dF = dev(F)
    o = lib.xi(dF, G, precision=prec)
    gxi = 2.0 * (o["xi"] - torch.as_tensor(target, device="cuda:0")[None, :])
    gd, gw = lib.xi_backward(dF, G, gxi, o["xi"], o["wsum"], precision=prec)
    torch.cuda.synchronize()
    assert O.err_norm(gd.cpu().numpy(), rd) <= TOL[prec]
    assert O.err_norm(gw.cpu().numpy(), rw) <= TOL[prec]


@pytest.mark.parametrize("grid", ["graded", "covering"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_dmat_vs_oracle(lib, grid, prec, variant):
    """Row-normwise error, except for the FP32 form on the covering grid: there
    two bins take nearly every pair and the projection cancels almost all of
    their rows (D_AA ~ 0.005 from terms of order 1), so the FP32 form is held to
    1e-5 of D's natural scale (the identity) instead, max |dD_AB| <= 1e-5."""
    G = GRIDS[grid]
    F, _, _ = make_config(0, seed=9)
    F = subset_forests(F, nearest_to_centre(F, 40))
    ref = O.dmat(F, G, O.dmat_pairs(F, G))
    dF = dev(F)
    host(lib.dmat(dF, G, precision=prec, variant=variant, autotune=False, counters=True))
    assert lib.last_stats()["lost_pairs"] == 0
    out = host(lib.dmat(dF, G, precision=prec, variant=variant, autotune=False))
    e_d, e_w = O.err_rows(out["dmat"], ref.D), O.err_rel(out["wsum_d"], ref.wd)
    if grid == "covering" and prec == "fp32":
        e_d = float(np.max(np.abs(out["dmat"] - ref.D)))
    print(f"[{grid} {prec} v{variant}] e_D={e_d:.3e} e_W={e_w:.3e}", flush=True)
    assert e_d <= TOL[prec] and e_w <= TOL[prec]
