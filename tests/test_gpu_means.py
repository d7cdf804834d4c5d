"""Weighted bin-mean coordinates (r_par, r_perp, z columns of the correlation
output) from lya_xi_means, on the GPU against the FP64 oracle.

Tolerances.  FP64 form: 1e-12 of the bin width for r_par, r_perp and 1e-12
relative for z.  FP32 form: the means come from the FP32 bin coordinates the
binning computes; each is within the x-space error bound of the exact value,
u ((2 M + 3 |e0|) / dr + 3 (N + 2)) bins for r_par and less for r_perp
(u = 2^-24, M = max |D - dc| <= 1000 Mpc/h, dr = 4, N = 15 or 50), i.e.
below 6e-5 bins here, so the tolerance is 1e-4 of the bin width; z is packed
in FP32 (relative error 6e-8), tolerance 1e-6 relative.  The sums and counts
obey the same bar as lya_xi."""
import numpy as np
import pytest

import oracle as O
from synth import concat_realisations, make_config, make_patch, subset_forests, uniform_grid
from synth.survey import nearest_to_centre

from helpers import forests_from_dict, grid_from_dict, load_json
from test_gpu_xi import _ragged_forests, check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_R = {"fp64": 1e-12, "fp32": 1e-4}
TOL_Z = {"fp64": 1e-12, "fp32": 1e-6}
G60 = uniform_grid(15, 60.0)


@pytest.fixture(scope="module")
def lib():
    from paper_2507_00129_amd import Library
    L = Library(0)
    yield L
    L.close()


def run_means(lib, F, G, **kw):
    from paper_2507_00129_amd import DeviceForests
    out = lib.xi_means(DeviceForests.from_host(F, "cuda:0"), G, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def check_means(out, ref, G, prec, what=""):
    rp, rt, z = O.bin_means(ref)
    dp = G.edges_par[1] - G.edges_par[0]
    dt = G.edges_perp[1] - G.edges_perp[0]
    e_p = float(np.max(np.abs(out["rpar"] - rp))) / dp
    e_t = float(np.max(np.abs(out["rperp"] - rt))) / dt
    nz = z != 0
    e_z = float(np.max(np.abs(out["z"] - z)[nz] / np.abs(z[nz]))) if nz.any() else 0.0
    print(f"[means {what} {prec}] e_rpar={e_p:.2e} e_rperp={e_t:.2e} e_z={e_z:.2e} bins={int(nz.sum())}",
          flush=True)
    assert np.all(out["rpar"][ref.wsum == 0] == 0) and np.all(out["z"][ref.wsum == 0] == 0)
    assert e_p <= TOL_R[prec] and e_t <= TOL_R[prec] and e_z <= TOL_Z[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_golden_handworked_means(lib, prec):
    d = load_json("xi_handworked_two_forests.json")
    F, G = forests_from_dict(d["forests"]), grid_from_dict(d["grid"])
    out = run_means(lib, F, G, precision=prec)
    exp = d["expected_means"]
    assert out["npairs"][0].tolist() == d["expected"]["npairs"]
    assert np.allclose(out["rpar"][0], exp["rpar"], rtol=TOL_R[prec], atol=0)
    assert np.allclose(out["rperp"][0], exp["rperp"], rtol=0, atol=1e-9)
    zl = np.exp(np.asarray(exp["z_loglam"])) / 1215.67 - 1.0
    assert np.allclose(out["z"][0], np.asarray(exp["z_weights"]) @ zl, rtol=TOL_Z[prec], atol=0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config0_means_vs_oracle(lib, prec):
    F, G, _ = make_config(0, seed=0)
    ref = O.xi_sums(F, G, means=True)
    out = run_means(lib, F, G, precision=prec)
    check(out, ref, prec, "means config0")
    check_means(out, ref, G, prec, "config0")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_means_ragged_and_realisations(lib, prec):
    F = _ragged_forests(11)
    ref = O.xi_sums(F, G60, means=True)
    out = run_means(lib, F, G60, precision=prec)
    check(out, ref, prec, "means ragged")
    check_means(out, ref, G60, prec, "ragged")
    parts = [make_patch(n, 2.0, 90 + r) for r, n in enumerate((30, 45))]
    R = concat_realisations(parts)
    ref = O.xi_sums(R, G60, means=True)
    out = run_means(lib, R, G60, precision=prec)
    assert out["rpar"].shape == (2, G60.n_bins)
    check(out, ref, prec, "means realisations")
    check_means(out, ref, G60, prec, "realisations")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config1_subpatch_means(lib, prec):
    """eBOSS-like density on the 50x50 grid to 200 Mpc/h (150 forests nearest
    the centre of a config-1 patch)."""
    F, G, _ = make_config(1, seed=0, scale=0.02)
    S = subset_forests(F, nearest_to_centre(F, 150))
    ref = O.xi_sums(S, G, means=True)
    out = run_means(lib, S, G, precision=prec)
    check(out, ref, prec, "means config1-sub")
    check_means(out, ref, G, prec, "config1-sub")


def test_full_config1_means_properties(lib):
    """Full eBOSS-like patch: the means form bins every pair as lya_xi does,
    every bin mean lies inside its bin, z inside the pixels' range, and the
    FP32 means agree with the FP64 ones to the FP32 bound."""
    from paper_2507_00129_amd import DeviceForests
    F, G, _ = make_config(1, seed=0)
    dF = DeviceForests.from_host(F, "cuda:0")
    plain = lib.xi(dF, G, precision="fp32")["npairs"].cpu().numpy()
    m32 = {k: v.cpu().numpy() for k, v in lib.xi_means(dF, G, precision="fp32").items()}
    m64 = {k: v.cpu().numpy() for k, v in lib.xi_means(dF, G, precision="fp64").items()}
    np.testing.assert_array_equal(m32["npairs"], plain)
    np.testing.assert_array_equal(m64["npairs"], plain)
    ne = m64["wsum"][0] > 0
    assert ne.sum() > 0.99 * G.n_bins
    kp, kt = np.divmod(np.arange(G.n_bins), G.n_perp)
    for m in (m32, m64):
        rp, rt = m["rpar"][0][ne], m["rperp"][0][ne]
        assert np.all(rp >= G.edges_par[kp][ne]) and np.all(rp <= G.edges_par[kp + 1][ne])
        assert np.all(rt >= G.edges_perp[kt][ne]) and np.all(rt <= G.edges_perp[kt + 1][ne])
    zp = O.pixel_redshift(F.loglam)
    assert np.all(m64["z"][0][ne] >= zp.min()) and np.all(m64["z"][0][ne] <= zp.max())
    dr = G.edges_par[1] - G.edges_par[0]
    e_p = float(np.max(np.abs(m32["rpar"] - m64["rpar"]))) / dr
    e_t = float(np.max(np.abs(m32["rperp"] - m64["rperp"]))) / dr
    e_z = float(np.max(np.abs(m32["z"] - m64["z"])[m64["z"] != 0] / np.abs(m64["z"][m64["z"] != 0])))
    print(f"[means full config1] fp32 vs fp64: e_rpar={e_p:.2e} e_rperp={e_t:.2e} e_z={e_z:.2e}", flush=True)
    assert e_p <= TOL_R["fp32"] and e_t <= TOL_R["fp32"] and e_z <= TOL_Z["fp32"]
