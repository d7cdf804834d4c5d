"""The forest-pair work list on wide footprints (the neighbour pre-ordering of
Sec. 2.1): candidates are bounded by declination strip and by right-ascension
window, so forests straddling RA = 0, near a pole or spread over the whole sky
must still give exactly the oracle's forest pairs and pair counts, for the
one-sided lists of xi and D and the two-sided lists of the backward pass."""
import numpy as np
import pytest

import oracle as O
from synth import make_patch, uniform_grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G60 = uniform_grid(15, 60.0)


@pytest.fixture(scope="module")
def lib():
    from paper_2507_00129_amd import Library
    L = Library(0)
    yield L
    L.close()


def placed(kind, n=300, seed=0):
    """Forests of the config-0 pixel model moved to a footprint."""
    rng = np.random.default_rng(seed)
    F = make_patch(n, 5.0, seed)
    if kind == "ra_wrap":      # a 30 x 12 deg band centred on RA = 0
        ra, dec = np.deg2rad(rng.uniform(-15.0, 15.0, n)) % (2 * np.pi), np.deg2rad(rng.uniform(-6.0, 6.0, n))
    elif kind == "north_cap":  # dec above 82 deg, all RA
        ra, dec = rng.uniform(0.0, 2 * np.pi, n), np.deg2rad(rng.uniform(82.0, 90.0, n))
    elif kind == "south_edge":  # dec below -80 deg, RA just under 2 pi
        ra, dec = 2 * np.pi - np.deg2rad(rng.uniform(0.0, 20.0, n)), np.deg2rad(rng.uniform(-90.0, -80.0, n))
    else:                      # whole sky, with clumps of coincident positions
        ra, dec = rng.uniform(0.0, 2 * np.pi, n), np.arcsin(rng.uniform(-1.0, 1.0, n))
        ra[: n // 3] = np.repeat(ra[: n // 30], 10)
        dec[: n // 3] = np.repeat(dec[: n // 30], 10)
    F.ra, F.dec = ra.astype(np.float64), dec.astype(np.float64)
    return F


def dev(F):
    from paper_2507_00129_amd import DeviceForests
    return DeviceForests.from_host(F, "cuda:0")


@pytest.mark.parametrize("kind", ["ra_wrap", "north_cap", "south_edge", "sky"])
def test_xi_pairs_on_wide_footprints(lib, kind):
    F = placed(kind)
    ref = O.xi_sums(F, G60)
    n_fp = int(O.forest_pairs(F, G60).shape[0])
    out = lib.xi(dev(F), G60, precision="fp64")
    torch.cuda.synchronize()
    st = lib.last_stats()
    print(f"[{kind}] forest pairs {n_fp} pixel pairs {int(ref.npairs.sum())}", flush=True)
    assert st["forest_pairs"] == n_fp
    np.testing.assert_array_equal(out["npairs"].cpu().numpy(), ref.npairs)
    assert O.err_xi(out["xi"].cpu().numpy(), ref.xi, ref.wsum, ref.absnum) <= 1e-12


@pytest.mark.parametrize("kind", ["ra_wrap", "north_cap"])
def test_backward_and_dmat_on_wide_footprints(lib, kind):
    F = placed(kind, n=160, seed=1)
    X = O.xi_sums(F, G60)
    target = np.random.default_rng(3).uniform(-0.01, 0.01, G60.n_bins)
    rd, rw = O.xi_grad(F, G60, O.loss_grad_xi(X.xi, target[None, :]), X.xi, X.wsum)
    dF = dev(F)
    o = lib.xi(dF, G60, precision="fp64")
    gd, gw = lib.xi_backward(dF, G60, 2.0 * (o["xi"] - torch.as_tensor(target, device="cuda:0")[None, :]),
                             o["xi"], o["wsum"], precision="fp64")
    torch.cuda.synchronize()
    assert O.err_norm(gd.cpu().numpy(), rd) <= 1e-12 and O.err_norm(gw.cpu().numpy(), rw) <= 1e-12
    ref = O.dmat(F, G60, O.dmat_pairs(F, G60))
    d = lib.dmat(dF, G60, precision="fp64")
    torch.cuda.synchronize()
    assert lib.last_stats()["forest_pairs"] == int(O.dmat_pairs(F, G60).shape[0])
    assert O.err_rows(d["dmat"].cpu().numpy(), ref.D) <= 1e-12
