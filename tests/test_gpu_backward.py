"""GPU parity of lya_xi_backward (the hand-written gradient of xi, also
through the continuum projection) against the FP64 oracle gradient, central
finite differences, invariances and Euler identities.
e_g = max |dg| / max |g| (normwise): 1e-12 for the FP64 form, 1e-5 for FP32."""
import numpy as np
import pytest

import oracle as O
from synth import concat_realisations, make_config, make_patch, subset_forests, uniform_grid
from synth.survey import nearest_to_centre

from test_gpu_xi import _ragged_forests

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


def gpu_grad(lib, F, G, target, prec):
    from paper_2507_00129_amd import DeviceForests
    dF = DeviceForests.from_host(F, "cuda:0")
    out = lib.xi(dF, G, precision=prec)
    t = torch.as_tensor(target, device="cuda:0").reshape(out["xi"].shape)
    gxi = 2.0 * (out["xi"] - t)
    gd, gw = lib.xi_backward(dF, G, gxi, out["xi"], out["wsum"], precision=prec)
    torch.cuda.synchronize()
    return gd.cpu().numpy(), gw.cpu().numpy(), out["xi"].cpu().numpy(), out["wsum"].cpu().numpy()


_ORACLE_CACHE = {}


def oracle_grad(F, G, target, key=None):
    if key is not None and key in _ORACLE_CACHE:
        return _ORACLE_CACHE[key]
    X = O.xi_sums(F, G)
    gxi = O.loss_grad_xi(X.xi, np.asarray(target).reshape(X.xi.shape))
    gd, gw = O.xi_grad(F, G, gxi, X.xi, X.wsum)
    if key is not None:
        _ORACLE_CACHE[key] = (gd, gw, X)
    return gd, gw, X


def check(gd, gw, rd, rw, prec, what):
    ed, ew = O.err_norm(gd, rd), O.err_norm(gw, rw)
    print(f"[{what} {prec}] e_gdelta={ed:.3e} e_gw={ew:.3e}", flush=True)
    assert ed <= TOL[prec] and ew <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config4_subset_vs_oracle(lib, prec):
    """The 200 forests nearest the centre of the differentiable workload."""
    F, G, ex = make_config(4, seed=0, scale=0.05)
    S = subset_forests(F, nearest_to_centre(F, 200))
    rd, rw, _ = oracle_grad(S, G, ex["target"], key="config4-200")
    gd, gw, _, _ = gpu_grad(lib, S, G, ex["target"], prec)
    check(gd, gw, rd, rw, prec, "config4-200")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ragged_and_realisations(lib, prec):
    F = _ragged_forests(3)
    target = np.random.default_rng(1).uniform(-0.01, 0.01, G60.n_bins)
    rd, rw, _ = oracle_grad(F, G60, target)
    gd, gw, _, _ = gpu_grad(lib, F, G60, target, prec)
    check(gd, gw, rd, rw, prec, "ragged")
    parts = [make_patch(n, 2.0, 80 + r) for r, n in enumerate((25, 40))]
    R = concat_realisations(parts)
    tgt = np.random.default_rng(2).uniform(-0.01, 0.01, (2, G60.n_bins))
    rd, rw, _ = oracle_grad(R, G60, tgt)
    gd, gw, _, _ = gpu_grad(lib, R, G60, tgt, prec)
    check(gd, gw, rd, rw, prec, "realisations")


def test_finite_differences_on_gpu(lib):
    """L is quadratic in each delta_i, so central differences of the GPU loss
    (FP64 form) are exact up to rounding; in w they are O(eps^2)."""
    from paper_2507_00129_amd import DeviceForests
    F, G, ex = make_config(4, seed=1, scale=0.02)
    dF = DeviceForests.from_host(F, "cuda:0")
    tgt = torch.as_tensor(ex["target"], device="cuda:0")[None, :]

    def loss(d, w):
        x = lib.xi(dF.with_values(delta=d, weight=w), G, precision="fp64")["xi"]
        return float(((x - tgt) ** 2).sum())

    out = lib.xi(dF, G, precision="fp64")
    gd, gw = lib.xi_backward(dF, G, 2.0 * (out["xi"] - tgt), out["xi"], out["wsum"], precision="fp64")
    gd, gw = gd.cpu().numpy(), gw.cpu().numpy()
    rng = np.random.default_rng(5)
    eps = 1e-3
    for i in rng.choice(F.n_pix, 16, replace=False):
        d = dF.delta.clone()
        d[i] += eps
        lp = loss(d, dF.weight)
        d[i] -= 2 * eps
        lm = loss(d, dF.weight)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - gd[i]) <= 1e-7 * max(1.0, abs(gd[i])) + 1e-9 * np.abs(gd).max(), (i, fd, gd[i])
    for i in rng.choice(F.n_pix, 16, replace=False):
        w = dF.weight.clone()
        w[i] += eps
        lp = loss(dF.delta, w)
        w[i] -= 2 * eps
        lm = loss(dF.delta, w)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - gw[i]) <= 1e-4 * abs(gw[i]) + 1e-6 * np.abs(gw).max(), (i, fd, gw[i])


def test_finite_differences_fp32_on_gpu(lib):
    """The FP32 form's forward and backward, central differences with eps =
    1e-3.  Binning is identical in the two evaluations and the products of
    unperturbed pixel pairs are bitwise equal, so the difference carries only
    the FP32 rounding of the perturbed pixel's products and of the run sums
    that hold them: ~6e-8 |w delta_i| sum_j |w delta_j| per bin against a
    change of 2 eps w_i sum_j w delta_j, i.e. ~3e-5 |delta_i| times the
    cancellation ratio sum |w delta| / |sum w delta| of the pixel's partners.
    Tolerance 2e-4 relative plus 2e-6 of the largest gradient (the same for
    w, where the O(eps^2) truncation is far smaller)."""
    from paper_2507_00129_amd import DeviceForests
    F, G, ex = make_config(4, seed=1, scale=0.02)
    dF = DeviceForests.from_host(F, "cuda:0")
    tgt = torch.as_tensor(ex["target"], device="cuda:0")[None, :]

    def loss(d, w):
        x = lib.xi(dF.with_values(delta=d, weight=w), G, precision="fp32")["xi"]
        return float(((x - tgt) ** 2).sum())

    out = lib.xi(dF, G, precision="fp32")
    gd, gw = lib.xi_backward(dF, G, 2.0 * (out["xi"] - tgt), out["xi"], out["wsum"], precision="fp32")
    gd, gw = gd.cpu().numpy(), gw.cpu().numpy()
    rng = np.random.default_rng(6)
    eps = 1e-3
    worst = 0.0
    for which, g in (("delta", gd), ("weight", gw)):
        for i in rng.choice(F.n_pix, 16, replace=False):
            d, w = dF.delta.clone(), dF.weight.clone()
            v = d if which == "delta" else w
            v[i] += eps
            lp = loss(d, w)
            v[i] -= 2 * eps
            lm = loss(d, w)
            fd = (lp - lm) / (2 * eps)
            err = abs(fd - g[i]) / (2e-4 * abs(g[i]) + 2e-6 * np.abs(g).max())
            worst = max(worst, err)
            assert err <= 1.0, (which, i, fd, g[i])
    print(f"[fd fp32] worst error / tolerance = {worst:.3f}", flush=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_euler_identities_full_size(lib, prec):
    """Full differentiable workload (10k forests, 50x50 bins): xi is homogeneous
    of degree 2 in delta and 0 in w, so sum delta_i g_delta_i = 4 sum xi (xi - m)
    and sum w_i g_w_i = 0."""
    F, G, ex = make_config(4, seed=0)
    gd, gw, xi, _ = gpu_grad(lib, F, G, ex["target"], prec)
    lhs = float(np.dot(F.delta, gd))
    rhs = 4.0 * float(np.sum(xi[0] * (xi[0] - ex["target"])))
    scale = float(np.dot(np.abs(F.delta), np.abs(gd)))
    print(f"[euler {prec}] {lhs:.12e} vs {rhs:.12e} (|diff| / scale = {abs(lhs - rhs) / scale:.2e}); "
          f"w.gw = {np.dot(F.weight, gw):.3e} (relative {abs(np.dot(F.weight, gw)) / float(np.dot(np.abs(F.weight), np.abs(gw))):.2e})", flush=True)
    assert abs(lhs - rhs) <= TOL[prec] * scale
    assert abs(np.dot(F.weight, gw)) <= TOL[prec] * float(np.dot(np.abs(F.weight), np.abs(gw)))


def test_autograd_function(lib):
    from paper_2507_00129_amd import DeviceForests, differentiable_xi
    F, G, ex = make_config(4, seed=2, scale=0.02)
    dF = DeviceForests.from_host(F, "cuda:0")
    d = dF.delta.clone().requires_grad_(True)
    w = dF.weight.clone().requires_grad_(True)
    xi = differentiable_xi(d, w, lib, dF, G, "fp64")
    tgt = torch.as_tensor(ex["target"], device="cuda:0")[None, :]
    L = ((xi - tgt) ** 2).sum()
    L.backward()
    gd, gw, _, _ = gpu_grad(lib, F, G, ex["target"], "fp64")
    assert np.allclose(d.grad.cpu().numpy(), gd, rtol=1e-12, atol=1e-14 * np.abs(gd).max())
    assert np.allclose(w.grad.cpu().numpy(), gw, rtol=1e-12, atol=1e-14 * np.abs(gw).max())


# ----------------------------------------------- gradient through the projection


def gpu_grad_proj(lib, F, G, target, prec, eta):
    from paper_2507_00129_amd import DeviceForests
    dF = DeviceForests.from_host(F, "cuda:0")
    opts = dict(precision=prec, project_deltas=True, eta=eta)
    out = lib.xi(dF, G, **opts)
    t = torch.as_tensor(target, device="cuda:0").reshape(out["xi"].shape)
    gd, gw = lib.xi_backward(dF, G, 2.0 * (out["xi"] - t), out["xi"], out["wsum"], **opts)
    torch.cuda.synchronize()
    return gd.cpu().numpy(), gw.cpu().numpy(), out["xi"].cpu().numpy()


def oracle_grad_proj(F, G, target, eta):
    mode = {"mean": O.MEAN, "mean_slope": O.MEAN_SLOPE, "identity": O.IDENTITY}[eta]
    X = O.xi_sums(F, G, project=True, eta_mode=mode)
    gxi = O.loss_grad_xi(X.xi, np.asarray(target).reshape(X.xi.shape))
    return O.xi_grad_projected(F, G, gxi, X.xi, X.wsum, eta_mode=mode)


@pytest.mark.parametrize("eta", ["mean_slope", "mean"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_projected_config4_subset_vs_oracle(lib, prec, eta):
    """Gradient with respect to the raw delta and w when xi correlates the
    projected deltas eta delta (eta moving with w), on the 200 forests nearest
    the centre of the differentiable workload."""
    F, G, ex = make_config(4, seed=0, scale=0.05)
    S = subset_forests(F, nearest_to_centre(F, 200))
    key = ("proj", eta)
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle_grad_proj(S, G, ex["target"], eta)
    rd, rw = _ORACLE_CACHE[key]
    gd, gw, _ = gpu_grad_proj(lib, S, G, ex["target"], prec, eta)
    check(gd, gw, rd, rw, prec, f"projected {eta} config4-200")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_projected_ragged_and_degenerate(lib, prec):
    """Empty, one-pixel (slope term dropped) and zero-weight (eta = I) forests,
    forests of up to 700 pixels, and the identity projection."""
    F = _ragged_forests(5)
    target = np.random.default_rng(4).uniform(-0.01, 0.01, G60.n_bins)
    for eta in ("mean_slope", "identity"):
        rd, rw = oracle_grad_proj(F, G60, target, eta)
        gd, gw, _ = gpu_grad_proj(lib, F, G60, target, prec, eta)
        check(gd, gw, rd, rw, prec, f"projected {eta} ragged")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_projected_invariances_full_size(lib, prec):
    """Full differentiable workload with projected deltas: adding a constant or
    a multiple of Lambda to one forest's deltas leaves eta delta unchanged, so
    the delta-gradient sums to zero over every forest and against Lambda; the
    Euler identities hold through eta."""
    F, G, ex = make_config(4, seed=0)
    gd, gw, xi = gpu_grad_proj(lib, F, G, ex["target"], prec, "mean_slope")
    c = np.repeat(np.arange(F.n_forests), np.diff(F.offsets))
    n = np.maximum(np.bincount(c, minlength=F.n_forests), 1)
    lc = F.loglam - (np.bincount(c, F.loglam, F.n_forests) / n)[c]
    s0 = np.abs(np.bincount(c, gd, F.n_forests))
    s1 = np.abs(np.bincount(c, lc * gd, F.n_forests))
    a0 = np.bincount(c, np.abs(gd), F.n_forests)
    a1 = np.bincount(c, np.abs(lc * gd), F.n_forests)
    e0 = float(np.max(s0 / np.maximum(a0, 1e-300)))
    e1 = float(np.max(s1 / np.maximum(a1, 1e-300)))
    lhs = float(np.dot(F.delta, gd))
    rhs = 4.0 * float(np.sum(xi[0] * (xi[0] - ex["target"])))
    scale = float(np.dot(np.abs(F.delta), np.abs(gd)))
    wg = abs(np.dot(F.weight, gw)) / float(np.dot(np.abs(F.weight), np.abs(gw)))
    print(f"[projected invariances {prec}] sum={e0:.2e} lambda={e1:.2e} euler={abs(lhs - rhs) / scale:.2e} "
          f"w.gw={wg:.2e}", flush=True)
    assert e0 <= 1e-12 and e1 <= 1e-10
    assert abs(lhs - rhs) <= TOL[prec] * scale
    assert wg <= TOL[prec]


def test_projected_finite_differences_on_gpu(lib):
    """Central differences of the GPU loss with projected deltas (FP64 form):
    exact up to rounding in delta, O(eps^2) in w."""
    from paper_2507_00129_amd import DeviceForests
    F, G, ex = make_config(4, seed=1, scale=0.02)
    dF = DeviceForests.from_host(F, "cuda:0")
    tgt = torch.as_tensor(ex["target"], device="cuda:0")[None, :]
    opts = dict(precision="fp64", project_deltas=True, eta="mean_slope")

    def loss(d, w):
        x = lib.xi(dF.with_values(delta=d, weight=w), G, **opts)["xi"]
        return float(((x - tgt) ** 2).sum())

    out = lib.xi(dF, G, **opts)
    gd, gw = lib.xi_backward(dF, G, 2.0 * (out["xi"] - tgt), out["xi"], out["wsum"], **opts)
    gd, gw = gd.cpu().numpy(), gw.cpu().numpy()
    rng = np.random.default_rng(6)
    eps = 1e-3
    for i in rng.choice(F.n_pix, 12, replace=False):
        d = dF.delta.clone()
        d[i] += eps
        lp = loss(d, dF.weight)
        d[i] -= 2 * eps
        lm = loss(d, dF.weight)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - gd[i]) <= 1e-7 * max(1.0, abs(gd[i])) + 1e-9 * np.abs(gd).max(), (i, fd, gd[i])
    for i in rng.choice(F.n_pix, 12, replace=False):
        w = dF.weight.clone()
        w[i] += eps
        lp = loss(dF.delta, w)
        w[i] -= 2 * eps
        lm = loss(dF.delta, w)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - gw[i]) <= 1e-4 * abs(gw[i]) + 1e-6 * np.abs(gw).max(), (i, fd, gw[i])


def test_projected_autograd_function(lib):
    from paper_2507_00129_amd import DeviceForests, differentiable_xi
    F, G, ex = make_config(4, seed=2, scale=0.02)
    dF = DeviceForests.from_host(F, "cuda:0")
    d = dF.delta.clone().requires_grad_(True)
    w = dF.weight.clone().requires_grad_(True)
    xi = differentiable_xi(d, w, lib, dF, G, "fp64", project_deltas=True)
    tgt = torch.as_tensor(ex["target"], device="cuda:0")[None, :]
    ((xi - tgt) ** 2).sum().backward()
    gd, gw, _ = gpu_grad_proj(lib, F, G, ex["target"], "fp64", "mean_slope")
    assert np.allclose(d.grad.cpu().numpy(), gd, rtol=1e-12, atol=1e-14 * np.abs(gd).max())
    assert np.allclose(w.grad.cpu().numpy(), gw, rtol=1e-12, atol=1e-14 * np.abs(gw).max())


@pytest.mark.parametrize("project", [False, True])
def test_gradcheck_tiny_fp64(lib, project):
    """torch.autograd.gradcheck of the differentiable xi (FP64 forward and
    backward kernels) with respect to delta and w on four 6-pixel forests:
    the backward kernel's Jacobian-vector products against central
    differences of the forward kernel, with and without the projection."""
    from helpers import tiny
    from paper_2507_00129_amd import DeviceForests, differentiable_xi
    F = tiny(4, n_forests=4, k=6, width_deg=0.3)
    dF = DeviceForests.from_host(F, "cuda:0")
    d = dF.delta.clone().requires_grad_(True)
    w = dF.weight.clone().requires_grad_(True)

    def f(d, w):
        return differentiable_xi(d, w, lib, dF, G60, "fp64", project_deltas=project)
    assert f(d, w).abs().sum().item() > 0
    # FP64 atomics make repeated backward calls differ in the last bits
    assert torch.autograd.gradcheck(f, (d, w), eps=1e-6, atol=1e-7, rtol=1e-5, nondet_tol=1e-12)
