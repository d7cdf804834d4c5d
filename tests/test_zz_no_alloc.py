"""lya_xi_noalloc (the entry point that allocates no device memory) against
lya_xi on the same inputs, two calls in a row with the second input smaller,
so the second call runs in scratch memory that still holds the first call's
work space."""
import numpy as np
import pytest

import oracle
from paper_2507_00129_amd import DeviceForests, Library
from paper_2507_00129_amd.lya import LyaError, LYA_E_UNSUPPORTED
from synth import Forests, make_config

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _outputs(R, nb, dev):
    import torch
    return {k: torch.full((R, nb), -7, dtype=torch.int64 if k == "npairs" else torch.float64, device=dev)
            for k in ("num", "wsum", "npairs", "xi")}


@pytest.fixture(scope="module")
def lib():
    L = Library(0)
    yield L
    L.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_xi_two_calls(lib, prec):
    import torch
    for call, (scale, seed) in enumerate(((1.0, 11), (0.45, 12))):
        F, G, _ = make_config(0, seed=seed, scale=scale)
        print(f"noalloc {prec} call {call}: {F.n_forests} forests, {F.n_pix} pixels", flush=True)
        dF = DeviceForests.from_host(F, "cuda:0")
        ref = lib.xi(dF, G, precision=prec)
        out = lib.xi_noalloc(dF, G, _outputs(1, G.n_bins, "cuda:0"), precision=prec)
        torch.cuda.synchronize()
        n_ref, n_out = ref["npairs"].cpu().numpy(), out["npairs"].cpu().numpy()
        assert np.array_equal(n_out, n_ref)
        o = oracle.xi_sums(F, G)
        assert np.array_equal(n_out[0], o.npairs[0])
        # both GPU results against the oracle, to the form's bound
        for res in (ref, out):
            e = oracle.err_xi(res["xi"].cpu().numpy(), o.xi, o.wsum, o.absnum)
            assert e <= TOL[prec], (call, e)
        # and the two GPU paths against each other, relative to the bin's condition
        dnum = np.abs(out["num"].cpu().numpy() - ref["num"].cpu().numpy())
        assert np.all(dnum <= TOL[prec] * o.absnum + 1e-300)
        dw = np.abs(out["wsum"].cpu().numpy() - ref["wsum"].cpu().numpy())
        assert np.all(dw <= TOL[prec] * o.wsum + 1e-300)


def test_noalloc_deterministic_bitwise(lib):
    import torch
    for call, (scale, seed) in enumerate(((1.0, 21), (0.5, 22))):
        F, G, _ = make_config(0, seed=seed, scale=scale)
        dF = DeviceForests.from_host(F, "cuda:0")
        ref = lib.xi(dF, G, precision="fp32", deterministic=True)
        out = lib.xi_noalloc(dF, G, _outputs(1, G.n_bins, "cuda:0"), precision="fp32", deterministic=True)
        torch.cuda.synchronize()
        for k in ("num", "wsum", "npairs", "xi"):
            assert torch.equal(out[k], ref[k]), (call, k)


def test_noalloc_rejects_oversized_input(lib):
    # 6e6 pixels: the packed pixel records alone exceed the scratch array
    n_f, k = 60000, 100
    npix = n_f * k
    rng = np.random.default_rng(5)
    F = Forests(np.arange(0, npix + 1, k, dtype=np.int64), rng.uniform(0, 0.1, n_f), rng.uniform(0, 0.1, n_f),
                np.tile(np.linspace(3000.0, 3300.0, k), n_f), rng.normal(0, 0.3, npix),
                np.ones(npix), np.log(np.tile(np.linspace(3600.0, 4000.0, k), n_f)))
    _, G, _ = make_config(0, seed=0, scale=0.1)
    dF = DeviceForests.from_host(F, "cuda:0")
    with pytest.raises(LyaError) as ei:
        lib.xi_noalloc(dF, G, _outputs(1, G.n_bins, "cuda:0"), precision="fp32")
    assert ei.value.status == LYA_E_UNSUPPORTED
    assert "scratch" in str(ei.value)
    # the context still works afterwards, in both entry points
    F2, G2, _ = make_config(0, seed=31, scale=0.3)
    d2 = DeviceForests.from_host(F2, "cuda:0")
    a = lib.xi(d2, G2, precision="fp64")
    b = lib.xi_noalloc(d2, G2, _outputs(1, G2.n_bins, "cuda:0"), precision="fp64")
    assert np.array_equal(a["npairs"].cpu().numpy(), b["npairs"].cpu().numpy())
