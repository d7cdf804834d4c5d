"""Pair sums split by subsample and the subsample covariance of xi (the
errors of Sec. 2.1 come from subsamples of the forests in sky pixels), on the
GPU against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from synth import concat_realisations, make_config, make_patch, sky_cells, uniform_grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
G60 = uniform_grid(15, 60.0)


@pytest.fixture(scope="module")
def lib():
    from paper_2507_00129_amd import Library
    L = Library(0)
    yield L
    L.close()


def run_sub(lib, F, G, sub, n_sub, **kw):
    from paper_2507_00129_amd import DeviceForests
    out = lib.xi_subsamples(DeviceForests.from_host(F), G, torch.from_numpy(sub).cuda(), n_sub, **kw)
    return {k: v.cpu().numpy() for k, v in out.items()}


def errors(out, ref, R, n_sub, nb):
    """(pair counts identical, max |dN| / sum |w d w d| per bin, max relative dW)"""
    assert ref.n_near_edge == 0, "input has pairs within 1e-12 of an edge; choose another seed"
    n = ref.npairs.reshape(R, n_sub, nb)
    dn = np.abs(out["num"].reshape(-1, nb) - ref.num)
    e_n = float(np.max(dn / np.where(ref.absnum > 0, ref.absnum, 1.0)))
    e_w = O.err_rel(out["wsum"].reshape(-1, nb), ref.wsum)
    return np.array_equal(out["npairs"], n), e_n, e_w


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_subsample_sums_vs_oracle(lib, prec):
    F, G, _ = make_config(0, seed=2)
    sub = sky_cells(F, 3, 3)
    ref = O.xi_sums(F, G, sub=sub, n_sub=9)
    out = run_sub(lib, F, G, sub, 9, precision=prec)
    same, e_n, e_w = errors(out, ref, 1, 9, G.n_bins)
    print(f"[subsamples {prec}] slabs={int((ref.npairs.sum(1) > 0).sum())} e_N={e_n:.2e} e_W={e_w:.2e}", flush=True)
    assert same and e_n <= TOL[prec] and e_w <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_subsample_sums_with_realisations(lib, prec):
    parts = [make_patch(n, 3.0, 80 + r) for r, n in enumerate((40, 55))]
    F = concat_realisations(parts)
    sub = sky_cells(F, 2, 2)
    ref = O.xi_sums(F, G60, sub=sub, n_sub=4)
    out = run_sub(lib, F, G60, sub, 4, precision=prec)
    assert out["num"].shape == (2, 4, G60.n_bins)
    same, e_n, e_w = errors(out, ref, 2, 4, G60.n_bins)
    assert same and e_n <= TOL[prec] and e_w <= TOL[prec]


def test_slabs_add_up_to_xi(lib):
    from paper_2507_00129_amd import DeviceForests
    F, G, _ = make_config(0, seed=3)
    sub = sky_cells(F, 4, 2)
    split = run_sub(lib, F, G, sub, 8, precision="fp64")
    whole = {k: v.cpu().numpy() for k, v in lib.xi(DeviceForests.from_host(F), G, precision="fp64").items()}
    ref = O.xi_sums(F, G)
    np.testing.assert_array_equal(split["npairs"].sum(1), whole["npairs"])
    dn = np.abs(split["num"].sum(1) - whole["num"])
    assert float(np.max(dn / np.where(ref.absnum > 0, ref.absnum, 1.0))) <= 1e-12
    assert O.err_rel(split["wsum"].sum(1), whole["wsum"]) <= 1e-12


def test_covariance_kernel_on_oracle_sums(lib):
    """The covariance kernel applied to the oracle's sums equals the oracle's
    covariance (FP64)."""
    F, G, _ = make_config(0, seed=4)
    sub = sky_cells(F, 4, 4)
    ref = O.xi_sums(F, G, sub=sub, n_sub=16)
    xi_o, cov_o = O.covariance(ref.num, ref.wsum)
    xi_g, cov_g = lib.xi_covariance(torch.from_numpy(ref.num).cuda(), torch.from_numpy(ref.wsum).cuda())
    scale = np.abs(cov_o).max()
    assert scale > 0
    assert np.abs(cov_g.cpu().numpy() - cov_o).max() <= 1e-12 * scale
    np.testing.assert_allclose(xi_g.cpu().numpy(), xi_o, rtol=1e-14, atol=1e-14 * np.abs(xi_o).max())


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-3)])
def test_covariance_end_to_end(lib, prec, tol):
    """GPU sums -> GPU covariance against oracle sums -> oracle covariance.
    x_sA = N_sA - W_sA xi_A cancels, so the tolerance is relative to max |C|
    and looser than the sums' (the sums agree to e_N of the bin's absolute sum)."""
    F, G, _ = make_config(0, seed=5)
    sub = sky_cells(F, 3, 3)
    ref = O.xi_sums(F, G, sub=sub, n_sub=9)
    _, cov_o = O.covariance(ref.num, ref.wsum)
    from paper_2507_00129_amd import DeviceForests
    out = lib.xi_subsamples(DeviceForests.from_host(F), G, torch.from_numpy(sub).cuda(), 9, precision=prec)
    _, cov_g = lib.xi_covariance(out["num"][0], out["wsum"][0])
    e = np.abs(cov_g.cpu().numpy() - cov_o).max() / np.abs(cov_o).max()
    print(f"[covariance {prec}] e_C={e:.2e}", flush=True)
    assert e <= tol


def test_invalid_subsample_ids(lib):
    from paper_2507_00129_amd import DeviceForests, LyaError
    F = make_patch(12, 2.0, 9)
    sub = np.zeros(F.n_forests, np.int32)
    sub[5] = 3
    with pytest.raises(LyaError):
        lib.xi_subsamples(DeviceForests.from_host(F), G60, torch.from_numpy(sub).cuda(), 3)
    sub[5] = -1
    with pytest.raises(LyaError):
        lib.xi_subsamples(DeviceForests.from_host(F), G60, torch.from_numpy(sub).cuda(), 3)
