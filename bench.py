#!/usr/bin/env python3
"""Throughput of the Lyman-alpha pair accumulation on one MI355X.

One step = one pass of the whole hot path over the eBOSS-like workload
(30k forests over 400 deg^2, 50x50 bins to 200 Mpc/h): per-forest precompute,
device work list, the xi pair kernel and its finalisation, then the
distortion matrix over the kept forest pairs and its finalisation.  Inputs are
synthetic (seeded), resident in HBM before the timed region.

value = in-grid pixel pairs of the step (xi pairs + pairs of the kept D forest
pairs) / step time, for the FP32 form.  The FP64 form is timed the same way
and reported beside it, with the FP32 form's error against FP64 at full size
and both forms' errors against the FP64 CPU oracle on a compact sub-patch.

Prints ONE JSON line.  --gpus N > 1 is not supported by this build.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# one non-packed VALU op per lane per clock: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz (the
# 157.3 TFLOP/s FP32 vector figure with an FMA as two flops; a SIMD issues a 64-lane FP32
# instruction in two clocks, which the instruction counters of the xi kernel confirm)
PEAK_ALU_OPS = 256 * 4 * 32 * 2.4e9
PEAK_MFMA_F64 = 78.6e12                   # dense FP64 matrix peak (flop/s)
PEAK_MFMA_F32 = 157.3e12                  # dense FP32 matrix peak (flop/s)
PEAK_HBM = 8.0e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters.json")
WORKLOADS = {
    1: "eBOSS-like patch: 30k forests over 400 deg^2, log-lambda pixels (50-150 per forest), "
       "GRF + unit-noise deltas; xi and D on 50x50 bins to 200 Mpc/h",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_step(lib, dF, G, prec, keep, seed, stream, xv, dv, counters=False):
    xo = lib.xi(dF, G, precision=prec, timing=True, stream=stream, variant=xv, autotune=False)
    sx = lib.last_stats()
    do = lib.dmat(dF, G, precision=prec, timing=True, keep_fraction=keep, seed=seed, stream=stream,
                  variant=dv, autotune=False, counters=counters)
    sd = lib.last_stats()
    return xo, do, sx, sd


def time_form(lib, dF, G, prec, keep, seed, steps, warmup, xv, dv):
    """Times `steps` steps after `warmup` untimed ones.  The distortion kernel's
    work counters (in-grid pairs, outer-product FMAs) are collected on the first
    warm-up step only, so the timed launches run without them."""
    import torch
    stream = torch.cuda.current_stream()
    counted = None
    for w in range(max(1, warmup)):
        _, _, _, sdw = run_step(lib, dF, G, prec, keep, seed, stream, xv, dv, counters=(w == 0))
        counted = counted or sdw
        torch.cuda.synchronize()
        log(f"[bench] {prec} warmup {w + 1}/{max(1, warmup)} done")
    sx_all, sd_all = [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(steps):
        xo, do, sx, sd = run_step(lib, dF, G, prec, keep, seed, stream, xv, dv)
        sx_all.append(sx)
        sd_all.append(sd)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1)
    log(f"[bench] {prec}: {steps} steps in {wall:.3f} s wall, {dev_ms:.1f} ms device")
    return xo, do, sx_all, sd_all, wall, counted


def mean(xs):
    return sum(xs) / max(1, len(xs))


def source_digest(name):
    import hashlib
    path = os.path.join(ROOT, "paper_2507_00129_amd", "csrc", name)
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, source):
    """HBM bytes per launch of `kernel` from the hardware counters recorded in
    profiles/traffic.json, or None when absent or taken on another version of
    the kernel's source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_digest(source):
        return None
    return rec.get("bytes_per_launch")


def issued_valu_frac(kernel, source, ms):
    """Issued VALU lane-ops per second over the peak, from the instruction
    counters recorded in profiles/counters.json for this kernel source (None
    when absent or taken on another version of the source)."""
    try:
        with open(COUNTERS_FILE) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_digest(source):
        return None
    return rec["insts_valu_per_launch"] * 64 / (ms / 1e3) / PEAK_ALU_OPS


def xi_roofline(r):
    ops = 6.0 * r["cand"] + 7.0 * r["xi_pairs"]
    achieved = ops / (r["ms_xi_kernel"] / 1e3) / 1e12
    return dict(kernel="xi_kernel<float>", bound="alu", achieved=achieved, peak=PEAK_ALU_OPS / 1e12,
                unit="TFLOP/s", frac=achieved / (PEAK_ALU_OPS / 1e12),
                traffic=measured_traffic("xi_kernel", "k_xi.hip"),
                work=f"6 ops x {r['cand']} candidate pairs + 7 ops x {r['xi_pairs']} in-grid pairs",
                issued_valu_frac=issued_valu_frac("xi_kernel", "k_xi.hip", r["ms_xi_kernel"]),
                ms=r["ms_xi_kernel"])


def d_roofline(r):
    flops = 2.0 * r["d_fmas"]
    achieved = flops / (r["ms_d_kernel"] / 1e3) / 1e12
    # the FP32 form's contraction runs as FP32 MFMA steps: its own dtype's peak
    return dict(kernel="dmat_kernel<float>", bound="mfma", achieved=achieved, peak=PEAK_MFMA_F32 / 1e12,
                unit="TFLOP/s", frac=achieved / (PEAK_MFMA_F32 / 1e12),
                traffic=measured_traffic("dmat_kernel", "k_dmat.hip"),
                work=f"2 x {r['d_fmas']} FMAs of the sparse row outer products and the rank-4 pair term "
                     f"(FP32 MFMA steps into FP32 accumulators, added to the FP64 numerator once per run)",
                ms=r["ms_d_kernel"])


def cpu_baseline_and_sample_errors(lib, F, G, keep, seed, n_xi, n_d, xv, dv):
    """The FP64 oracle on a compact sub-patch (timed on one host thread), and the
    GPU forms' errors against it on the same sample.  These launches use kernels
    other than the timed FP32 ones (the other xi variant, the FP64 distortion
    form), so the profiler's averages for the timed kernels cover full-size
    launches only; the FP32 distortion form is compared with the FP64 form at
    full size instead, and every variant is parity-tested."""
    import numpy as np
    import oracle
    from paper_2507_00129_amd import DeviceForests
    from synth import subset_forests
    from synth.survey import nearest_to_centre
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:  # pragma: no cover
        limiter = None
    Sx = subset_forests(F, nearest_to_centre(F, n_xi))
    Sd = subset_forests(F, nearest_to_centre(F, n_d))
    t0 = time.perf_counter()
    X = oracle.xi_sums(Sx, G)
    t1 = time.perf_counter()
    pairs = oracle.dmat_pairs(Sd, G, keep, seed)
    Dr = oracle.dmat(Sd, G, pairs)
    t2 = time.perf_counter()
    d_pairs = int(oracle.xi_sums(Sd, G, pairs=pairs).npairs.sum())
    if limiter is not None:
        limiter.unregister()
    xi_pairs = int(X.npairs.sum())
    errs = {}
    dSx, dSd = DeviceForests.from_host(Sx), DeviceForests.from_host(Sd)
    for prec in ("fp32", "fp64"):
        o = lib.xi(dSx, G, precision=prec, variant=xv, autotune=False)
        xi = o["xi"].cpu().numpy()
        same = bool(np.array_equal(o["npairs"].cpu().numpy(), X.npairs))
        errs[prec] = dict(e_xi=oracle.err_xi(xi, X.xi, X.wsum, X.absnum),
                          e_W=oracle.err_rel(o["wsum"].cpu().numpy(), X.wsum),
                          npairs_exact=same)
        if prec == "fp64":
            d = lib.dmat(dSd, G, precision=prec, keep_fraction=keep, seed=seed, variant=dv, autotune=False)
            errs[prec]["e_D"] = oracle.err_rows(d["dmat"].cpu().numpy(), Dr.D)
    value = (xi_pairs + d_pairs) / ((t1 - t0) + (t2 - t1))
    base = dict(value=value, unit="pixel pairs/s", cores=1, kind="oracle",
                sample=f"FP64 NumPy oracle, one thread: xi on the {n_xi} forests nearest the patch centre "
                       f"({xi_pairs} in-grid pairs, {t1 - t0:.2f} s) + D on the {n_d} nearest "
                       f"({d_pairs} in-grid pairs of {len(pairs)} kept forest pairs, {t2 - t1:.2f} s)")
    return base, errs


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1, choices=sorted(WORKLOADS))
    ap.add_argument("--keep", type=float, default=1.0, help="distortion-matrix forest-pair keep fraction")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the full-size FP32-vs-FP64 comparison")
    ap.add_argument("--no-means", action="store_true", help="skip timing the bin-means form of the xi kernel")
    ap.add_argument("--no-xi3", action="store_true", help="skip timing the three-point kernel")
    ap.add_argument("--xi3-forests", type=int, default=1500,
                    help="forests nearest the patch centre used for the three-point timing")
    ap.add_argument("--xi3-wide-forests", type=int, default=500,
                    help="forests for the three-point timing on the paper's 80 Mpc/h grid")
    ap.add_argument("--cpu-xi-forests", type=int, default=400)
    ap.add_argument("--cpu-d-forests", type=int, default=120)
    ap.add_argument("--xi-variant", type=int, default=3,
                    help="xi kernel variant (3 = 512 threads with run-length sums, the autotuner's "
                         "choice for this workload on MI355X)")
    ap.add_argument("--d-variant", type=int, default=0,
                    help="distortion kernel variant (0 = 8 waves, the autotuner's choice)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a known-size "
                         "reference for hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs the hot path on one GPU only; --gpus N > 1 is not "
              "supported (the work list would be sharded across GPUs with one all-reduce of the "
              "sums, which is not built here)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2507_00129_amd import DeviceForests, Library
    from synth import make_config

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
    log(f"[bench] generating config {args.config} (seed {args.seed})")
    F, G, extras = make_config(args.config, seed=args.seed)
    lib = Library(0)
    dF = DeviceForests.from_host(F, "cuda:0")
    torch.cuda.synchronize()
    log(f"[bench] {F.n_forests} forests, {F.n_pix} pixels resident on the GPU")

    res = {}
    forms = ["fp32"] if args.no_fp64 else ["fp32", "fp64"]
    for prec in forms:
        xo, do, sx, sd, wall, sdc = time_form(lib, dF, G, prec, args.keep, args.seed, args.steps,
                                              args.warmup, args.xi_variant, args.d_variant)
        xi_pairs = int(xo["npairs"].sum().item())
        d_pairs = int(sdc["ingrid_pairs"])
        res[prec] = dict(out_xi={k: v.cpu().numpy() for k, v in xo.items()},
                         out_d={k: v.cpu().numpy() for k, v in do.items()},
                         xi_pairs=xi_pairs, d_pairs=d_pairs, wall=wall,
                         ms_step=1e3 * wall / args.steps,
                         ms_xi_kernel=mean([s["ms_main"] for s in sx]),
                         ms_d_kernel=mean([s["ms_main"] for s in sd]),
                         ms_xi_kernel_median=float(np.median([s["ms_main"] for s in sx])),
                         ms_d_kernel_median=float(np.median([s["ms_main"] for s in sd])),
                         ms_xi_total=mean([s["ms_precompute"] + s["ms_worklist"] + s["ms_main"] + s["ms_finalize"] for s in sx]),
                         ms_d_total=mean([s["ms_precompute"] + s["ms_worklist"] + s["ms_main"] + s["ms_finalize"] for s in sd]),
                         cand=int(sx[-1]["candidate_pairs"]), d_fmas=int(sdc["outer_fmas"]),
                         d_forest_pairs=int(sd[-1]["forest_pairs"]), xi_variant=int(sx[-1]["variant"]),
                         d_variant=int(sd[-1]["variant"]))
        r = res[prec]
        r["value"] = (xi_pairs + d_pairs) / (r["ms_step"] / 1e3)
        log(f"[bench] {prec}: {r['value']:.4e} pairs/s; xi kernel {r['ms_xi_kernel']:.2f} ms "
            f"({xi_pairs / r['ms_xi_kernel'] * 1e3:.3e} pairs/s), D kernel {r['ms_d_kernel']:.2f} ms "
            f"({d_pairs / max(r['ms_d_kernel'], 1e-9) * 1e3:.3e} pairs/s)")

    means = None
    if not args.no_means:
        # the xi kernel form that also sums the bin-mean coordinates (FP32),
        # one warm-up and three timed calls outside the step
        ms = []
        for k in range(4):
            lib.xi_means(dF, G, precision="fp32", timing=True)
            if k:
                ms.append(lib.last_stats()["ms_main"])
        torch.cuda.synchronize()
        mm = mean(ms)
        means = dict(ms_kernel=mm, pairs_per_s_kernel=res["fp32"]["xi_pairs"] / (mm / 1e3),
                     time_over_xi_kernel=mm / res["fp32"]["ms_xi_kernel"])
        log(f"[bench] xi with bin means (fp32): kernel {mm:.2f} ms")

    xi3 = None
    if not args.no_xi3:
        # anisotropic 3PCF (FP64) on the forests nearest the patch centre, sides to
        # 40 Mpc/h in 10 bins, theta in 10 bins over [0, pi], cos alpha in 20 bins
        from types import SimpleNamespace
        from synth import subset_forests
        from synth.survey import nearest_to_centre
        S = subset_forests(F, nearest_to_centre(F, args.xi3_forests))
        dS = DeviceForests.from_host(S, "cuda:0")
        g3 = SimpleNamespace(r_edges=np.linspace(0.0, 40.0, 11), theta_edges=np.linspace(0.0, np.pi, 11),
                             cos_edges=np.linspace(-1.0, 1.0, 21))
        ms = []
        for k in range(2):
            o3 = lib.xi3(dS, g3, timing=True)
            ms.append(lib.last_stats()["ms_main"])
        variant = lib.last_stats()["variant"]
        torch.cuda.synchronize()
        entries = int(o3["ntrip"].sum().item())
        t3 = ms[-1] / 1e3
        # ms_kernel: the triplet kernel plus the sum of the per-XCD copies
        xi3 = dict(workload=f"{S.n_forests} forests nearest the centre of the eBOSS-like patch "
                            f"({S.n_pix} pixels); r to 40 Mpc/h (10 bins), theta 10 bins, cos alpha 20 bins",
                   kernel="xi3c_kernel (entries summed in LDS per side-1 cell)" if variant == 0
                   else "xi3_kernel (global atomics per entry)",
                   entries=entries, ms_kernel=ms[-1], entries_per_s=entries / t3, dtype="f64")
        log(f"[bench] xi3: {entries:.3e} entries in {ms[-1]:.1f} ms ({entries / t3:.3e} entries/s)")
        del dS, o3
        # the grid of the paper's 3PCF figure: r to 80 Mpc/h in 20 bins, theta
        # 10 bins, cos alpha 20 bins; vertex pixels have thousands of partners
        S = subset_forests(F, nearest_to_centre(F, args.xi3_wide_forests))
        dS = DeviceForests.from_host(S, "cuda:0")
        g80 = SimpleNamespace(r_edges=np.linspace(0.0, 80.0, 21), theta_edges=np.linspace(0.0, np.pi, 11),
                              cos_edges=np.linspace(-1.0, 1.0, 21))
        o3 = lib.xi3(dS, g80, timing=True)
        st3 = lib.last_stats()
        torch.cuda.synchronize()
        e80 = int(o3["ntrip"].sum().item())
        xi3["paper_grid"] = dict(
            workload=f"{S.n_forests} forests nearest the centre ({S.n_pix} pixels); r to 80 Mpc/h (20 bins), "
                     f"theta 10 bins, cos alpha 20 bins",
            kernel={0: "xi3c_kernel", 1: "xi3_kernel", 2: "xi3w_kernel (partner lists in global scratch)"}[
                st3["variant"]],
            entries=e80, ms_kernel=st3["ms_main"], entries_per_s=e80 / (st3["ms_main"] / 1e3))
        log(f"[bench] xi3 paper grid: {e80:.3e} entries in {st3['ms_main']:.1f} ms")
        del dS, o3

    r32 = res["fp32"]
    # dominant kernel and its roofline (algorithmic work / kernel time from HIP
    # events recorded around the launch on its stream)
    roof = xi_roofline(r32) if r32["ms_xi_kernel"] >= r32["ms_d_kernel"] else d_roofline(r32)

    line = dict(metric="pixel pairs/sec for xi + distortion matrix, FP32 vs FP64 at stated rel. error",
                value=r32["value"], unit="pixel pairs/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                ms_per_step=r32["ms_step"], higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32", data="synthetic",
                config=dict(workload=WORKLOADS[args.config], forests=F.n_forests, pixels=F.n_pix,
                            n_bins=G.n_bins, dmat_keep_fraction=args.keep, precision="FP32_COMP",
                            xi_pairs=r32["xi_pairs"], d_pairs=r32["d_pairs"],
                            d_forest_pairs=r32["d_forest_pairs"], candidate_pairs=r32["cand"]),
                roofline=roof)
    line["roofline_xi"] = xi_roofline(r32)
    line["xi_pairs_per_s_kernel"] = r32["xi_pairs"] / (r32["ms_xi_kernel"] / 1e3)
    line["d_pairs_per_s_kernel"] = r32["d_pairs"] / max(r32["ms_d_kernel"] / 1e3, 1e-12)
    # whole calls (precompute, work list, kernel, finalise; device time of the
    # timed steps) and the spread of the kernel times over the timed steps
    line["xi_pairs_per_s_call"] = r32["xi_pairs"] / (r32["ms_xi_total"] / 1e3)
    line["d_pairs_per_s_call"] = r32["d_pairs"] / max(r32["ms_d_total"] / 1e3, 1e-12)
    line["kernel_ms"] = dict(xi_mean=r32["ms_xi_kernel"], xi_median=r32["ms_xi_kernel_median"],
                             d_mean=r32["ms_d_kernel"], d_median=r32["ms_d_kernel_median"])
    if means is not None:
        line["xi_means_fp32"] = means
    if xi3 is not None:
        line["xi3_fp64"] = xi3
    if "fp64" in res:
        r64 = res["fp64"]
        d64 = 2.0 * r64["d_fmas"] / max(r64["ms_d_kernel"] / 1e3, 1e-12)
        line["fp64"] = dict(value=r64["value"], ms_per_step=r64["ms_step"],
                            xi_pairs_per_s_kernel=r64["xi_pairs"] / (r64["ms_xi_kernel"] / 1e3),
                            d_pairs_per_s_kernel=r64["d_pairs"] / max(r64["ms_d_kernel"] / 1e3, 1e-12),
                            xi_pairs_per_s_call=r64["xi_pairs"] / (r64["ms_xi_total"] / 1e3),
                            d_pairs_per_s_call=r64["d_pairs"] / max(r64["ms_d_total"] / 1e3, 1e-12),
                            kernel_ms=dict(xi_mean=r64["ms_xi_kernel"], xi_median=r64["ms_xi_kernel_median"],
                                           d_mean=r64["ms_d_kernel"], d_median=r64["ms_d_kernel_median"]),
                            d_mfma_tflops=d64 / 1e12, d_mfma_frac_of_f64_peak=d64 / PEAK_MFMA_F64)
        line["fp32_over_fp64"] = r32["value"] / r64["value"]
        if not args.no_check:
            a32, a64 = r32["out_xi"], r64["out_xi"]
            absn = lib.xi(dF.with_values(delta=dF.delta.abs()), G, precision="fp64")["num"].cpu().numpy()
            m = absn > 0
            d32, d64 = r32["out_d"]["dmat"], r64["out_d"]["dmat"]
            scale = np.max(np.abs(d64), axis=-1, keepdims=True)
            scale[scale == 0] = 1.0
            line["fp32_vs_fp64_full"] = dict(
                npairs_identical=bool(np.array_equal(a32["npairs"], a64["npairs"])),
                e_xi=float(np.max(np.abs(a32["num"] - a64["num"])[m] / absn[m])),
                e_W=float(np.max(np.abs(a32["wsum"] - a64["wsum"])[a64["wsum"] > 0] / a64["wsum"][a64["wsum"] > 0])),
                e_D=float(np.max(np.abs(d32 - d64) / scale)))
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a compact sub-patch")
        base, errs = cpu_baseline_and_sample_errors(lib, F, G, args.keep, args.seed,
                                                    args.cpu_xi_forests, args.cpu_d_forests,
                                                    0 if args.xi_variant != 0 else 1, args.d_variant)
        line["cpu_baseline"] = base
        line["vs_oracle_sample"] = errs
    print(json.dumps(line), flush=True)
    lib.close()


if __name__ == "__main__":
    main()
