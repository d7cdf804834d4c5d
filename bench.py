#!/usr/bin/env python3
"""Throughput of the Lyman-alpha pair accumulation on one MI355X.

One step = one pass of the whole hot path over the eBOSS-like workload
(30k forests over 400 deg^2, 50x50 bins to 200 Mpc/h): per-forest precompute,
device work list, the xi pair kernel and its finalisation, then the
distortion matrix over the kept forest pairs and its finalisation.  Inputs are
synthetic (seeded), resident in HBM before the timed region.

value = in-grid pixel pairs of the step (xi pairs + pairs of the kept D forest
pairs) / step time, for the FP32 form.  Kernel variants are the autotuner's
choice, made during the first warm-up step.  The FP64 form is timed the same
way (fewer steps) and reported beside it, with the FP32 form's error against
FP64 at full size and both forms' errors against the FP64 CPU oracle on a
compact sub-patch.  Extra keys time the batched 64-realisation xi launch and
the differentiable workload (forward and backward, gradient error against the
oracle on a 200-forest subset).

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

# ALU peak from the chip's unit counts: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz =
# 7.86e13 lane-ops/s.  On gfx950 a SIMD retires a 64-lane non-packed FP32 or u32
# add (mul, compare, logic) in two clocks and an FMA in four: lya_measure_peaks
# times 6.8e13 lane-adds/s and 3.8e13 lane-FMAs/s, and the xi kernel's
# arithmetic is adds, multiplies and compares.  (The 157.3 TFLOP/s FP32 vector
# figure is the FMA rate with packed FMAs; packed FP32 is not used here.)
PEAK_VALU_LANE_OPS = 256 * 4 * 32 * 2.4e9
# FP64 VALU: one 64-lane FP64 add, multiply or FMA per SIMD every four clocks
PEAK_VALU_F64_LANE_OPS = 256 * 4 * 16 * 2.4e9
PEAK_MFMA_F64 = 78.6e12                   # dense FP64 matrix peak (flop/s)
PEAK_MFMA_F32 = 157.3e12                  # dense FP32 matrix peak (flop/s)
PEAK_HBM = 8.0e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters.json")
WORKLOADS = {
    1: "eBOSS-like patch: 30k forests over 400 deg^2, log-lambda pixels (50-150 per forest), "
       "GRF + unit-noise deltas; xi and D on 50x50 bins to 200 Mpc/h",
}
# the paper's own wall-clock figures (context only: other hardware, other
# workloads, no precision stated)
PAPER_TIMINGS = {
    "2pcf_desi_y5_2xA100": "4.3 h including 2.3 h of FITS extraction (Table cpu_equiv)",
    "dmat_desi_y5_2xA100": "6.4 h on a subset of forest pairs of unstated size (Table cpu_equiv)",
    "2pcf_dr16_rtx2070_fit": "t = 0.3 + 18.6 min (N / 210005)^1.9 (Table Nforests)",
    "2pcf_plus_dmat_dr16_rtx2070_fit": "t = 1.3 + 35.5 min (N / 210005)^1.8 (Table Nforests)",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def mean(xs):
    return sum(xs) / max(1, len(xs))


# ---------------------------------------------------------------------------
# the FP64 CPU oracle on the host cores (test infrastructure: timed as the CPU
# baseline and used for the sample errors, never on the measured path)
# ---------------------------------------------------------------------------

_ORACLE_INPUT = {}


def _worker_init():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass


def _oracle_xi_part(args):
    import oracle
    key, pairs = args
    F, G = _ORACLE_INPUT[key]
    X = oracle.xi_sums(F, G, pairs=pairs)
    return X.num, X.wsum, X.npairs, X.absnum


def _oracle_d_part(args):
    import oracle
    key, pairs = args
    F, G = _ORACLE_INPUT[key]
    R = oracle.dmat(F, G, pairs)
    return R.num, R.wd


def _oracle_grad_part(args):
    import oracle
    key, pairs, gxi, xi, wsum = args
    F, G = _ORACLE_INPUT[key]
    return oracle.xi_grad(F, G, gxi, xi, wsum, pairs=pairs)


def _split_pairs(F, pairs, parts):
    """Contiguous runs of the pair list (ordered by first forest) with about
    equal pixel-pair counts."""
    import numpy as np
    if pairs.shape[0] == 0:
        return [pairs]
    pairs = pairs[np.argsort(pairs[:, 0], kind="stable")]
    n = np.diff(F.offsets)
    cost = np.cumsum(n[pairs[:, 0]].astype(np.float64) * n[pairs[:, 1]])
    cuts = np.searchsorted(cost, cost[-1] * np.arange(1, parts) / parts)
    return [p for p in np.split(pairs, cuts) if p.shape[0]]


class OraclePool:
    """The oracle run over chunks of the forest-pair list in worker processes
    forked from this one (before the GPU is initialised), one NumPy thread each."""

    def __init__(self, workers):
        import multiprocessing as mp
        self.workers = workers
        self.pool = mp.get_context("fork").Pool(workers, initializer=_worker_init)

    def xi_sums(self, key, F, G, pairs):
        import numpy as np
        parts = self.pool.map(_oracle_xi_part, [(key, p) for p in _split_pairs(F, pairs, 4 * self.workers)])
        return [np.sum([p[i] for p in parts], axis=0) for i in range(4)]

    def dmat(self, key, F, G, pairs):
        import numpy as np
        # one chunk per worker: each result carries a dense n_bins^2 numerator
        parts = self.pool.map(_oracle_d_part, [(key, p) for p in _split_pairs(F, pairs, self.workers)])
        num, wd = np.sum([p[0] for p in parts], axis=0), np.sum([p[1] for p in parts], axis=0)
        D = np.zeros_like(num)
        for r in range(num.shape[0]):
            nz = wd[r] != 0
            D[r][nz] = num[r][nz] / wd[r][nz][:, None]
        return D

    def xi_grad(self, key, F, G, pairs, gxi, xi, wsum):
        import numpy as np
        parts = self.pool.map(_oracle_grad_part,
                              [(key, p, gxi, xi, wsum) for p in _split_pairs(F, pairs, 4 * self.workers)])
        return np.sum([p[0] for p in parts], axis=0), np.sum([p[1] for p in parts], axis=0)

    def close(self):
        self.pool.close()
        self.pool.join()


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_stage(F, G, keep, seed, n_xi, n_d, F4, G4, target4, workers):
    """CPU baseline: xi on the n_xi forests nearest the patch centre and D on the
    n_d nearest, timed (pair list + pooled oracle); then, untimed, the
    distortion sample's in-grid pair count and the config-4 subset gradient."""
    import numpy as np
    import oracle
    from synth import subset_forests
    from synth.survey import nearest_to_centre
    Sx = subset_forests(F, nearest_to_centre(F, n_xi))
    Sd = subset_forests(F, nearest_to_centre(F, n_d))
    _ORACLE_INPUT["xi"] = (Sx, G)
    _ORACLE_INPUT["d"] = (Sd, G)
    S4 = None
    if F4 is not None:
        S4 = subset_forests(F4, nearest_to_centre(F4, 200))
        _ORACLE_INPUT["c4"] = (S4, G4)
    pool = OraclePool(workers)
    try:
        t0 = time.perf_counter()
        px = oracle.forest_pairs(Sx, G)
        num, wsum, npairs, absnum = pool.xi_sums("xi", Sx, G, px)
        t1 = time.perf_counter()
        pd = oracle.dmat_pairs(Sd, G, keep, seed)
        Dref = pool.dmat("d", Sd, G, pd)
        t2 = time.perf_counter()
        d_pairs = int(pool.xi_sums("d", Sd, G, pd)[2].sum())
        xi_ref = oracle.xi_from_sums(num, wsum)
        grad = None
        if S4 is not None:
            p4 = oracle.forest_pairs(S4, G4)
            n4, w4, c4, a4 = pool.xi_sums("c4", S4, G4, p4)
            x4 = oracle.xi_from_sums(n4, w4)
            gxi = oracle.loss_grad_xi(x4, np.asarray(target4).reshape(x4.shape))
            gd, gw = pool.xi_grad("c4", S4, G4, p4, gxi, x4, w4)
            grad = dict(S=S4, gd=gd, gw=gw, pairs=int(c4.sum()))
    finally:
        pool.close()
    xi_pairs = int(npairs.sum())
    base = dict(value=(xi_pairs + d_pairs) / (t2 - t0), unit="pixel pairs/s", cores=workers, kind="oracle",
                sample=f"FP64 NumPy oracle in {workers} worker processes (one thread each) over chunks of the "
                       f"forest-pair list: xi on the {n_xi} forests nearest the patch centre ({xi_pairs} in-grid "
                       f"pairs, {t1 - t0:.2f} s) + D on the {n_d} nearest ({d_pairs} in-grid pairs of "
                       f"{len(pd)} kept forest pairs, {t2 - t1:.2f} s)")
    ref = dict(Sx=Sx, Sd=Sd, num=num, wsum=wsum, npairs=npairs, absnum=absnum, xi=xi_ref, D=Dref)
    return base, ref, grad


def gpu_sample_errors(lib, ref, G, keep, seed, xv, dv64):
    """Both GPU forms against the oracle on the sample.  These launches use a
    kernel other than the timed FP32 ones (another xi variant, the FP64
    distortion form), so the profiler's averages for the timed kernels cover
    full-size launches only."""
    import numpy as np
    import oracle
    from paper_2507_00129_amd import DeviceForests
    errs = {}
    dSx, dSd = DeviceForests.from_host(ref["Sx"]), DeviceForests.from_host(ref["Sd"])
    for prec in ("fp32", "fp64"):
        o = lib.xi(dSx, G, precision=prec, variant=xv, autotune=False)
        same = bool(np.array_equal(o["npairs"].cpu().numpy(), ref["npairs"]))
        errs[prec] = dict(e_xi=oracle.err_xi(o["xi"].cpu().numpy(), ref["xi"], ref["wsum"], ref["absnum"]),
                          e_W=oracle.err_rel(o["wsum"].cpu().numpy(), ref["wsum"]),
                          npairs_exact=same)
        if prec == "fp64":
            d = lib.dmat(dSd, G, precision=prec, keep_fraction=keep, seed=seed, variant=dv64, autotune=False)
            errs[prec]["e_D"] = oracle.err_rows(d["dmat"].cpu().numpy(), ref["D"])
    return errs


# ---------------------------------------------------------------------------
# the timed step
# ---------------------------------------------------------------------------


def run_step(lib, dF, G, prec, keep, seed, stream, xv, dv, counters=False):
    tune = xv < 0 or dv < 0
    xo = lib.xi(dF, G, precision=prec, timing=True, stream=stream, variant=xv, autotune=tune)
    sx = lib.last_stats()
    do = lib.dmat(dF, G, precision=prec, timing=True, keep_fraction=keep, seed=seed, stream=stream,
                  variant=dv, autotune=tune, counters=counters)
    sd = lib.last_stats()
    return xo, do, sx, sd


def time_form(lib, dF, G, prec, keep, seed, steps, warmup, xv, dv):
    """Times `steps` steps after `warmup` untimed ones.  The first warm-up step
    lets the autotuner pick the variants (where not forced) and collects the
    distortion kernel's work counters (in-grid pairs, outer-product FMAs); the
    timed launches run with the chosen variants and without counters."""
    import torch
    stream = torch.cuda.current_stream()
    counted = None
    for w in range(max(1, warmup)):
        _, _, sxw, sdw = run_step(lib, dF, G, prec, keep, seed, stream, xv, dv, counters=(w == 0))
        if w == 0:
            counted = sdw
            xv, dv = int(sxw["variant"]), int(sdw["variant"])
        torch.cuda.synchronize()
        log(f"[bench] {prec} warmup {w + 1}/{max(1, warmup)} done (xi variant {xv}, D variant {dv})")
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


def source_digest(name):
    import hashlib
    path = os.path.join(ROOT, "paper_2507_00129_amd", "csrc", name)
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _profile_record(path, kernel, source):
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_digest(source):
        return None
    return rec


def measured_traffic(kernel, source):
    """HBM bytes per launch of `kernel` from the hardware counters recorded in
    profiles/traffic.json, or None when absent or taken on another version of
    the kernel's source."""
    rec = _profile_record(TRAFFIC_FILE, kernel, source)
    return None if rec is None else rec.get("bytes_per_launch")


def issued_valu_frac(kernel, source, ms):
    """Issued VALU lane-ops per second over the peak, from the instruction
    counters recorded in profiles/counters.json for this kernel source (None
    when absent or taken on another version of the source)."""
    rec = _profile_record(COUNTERS_FILE, kernel, source)
    if rec is None:
        return None
    return rec["insts_valu_per_launch"] * 64 / (ms / 1e3) / PEAK_VALU_LANE_OPS


XI_KERNELS = {0: "xi_kernel<float, 256, false, true, false, false>", 1: "xi_kernel<float, 512, false, true, false, false>",
              2: "xi_kernel<float, 256, true, true, false, false>", 3: "xi_kernel<float, 512, true, true, false, false>"}


def xi_roofline(r, peaks):
    ops = 6.0 * r["cand"] + 7.0 * r["xi_pairs"]
    t = r["ms_xi_kernel"] / 1e3
    achieved = ops / t / 1e12
    kname = XI_KERNELS.get(r["xi_variant"], "xi_kernel")
    return dict(kernel=f"{kname} ({r['xi_variant_name']})", bound="alu", achieved=achieved,
                peak=PEAK_VALU_LANE_OPS / 1e12, unit="TFLOP/s", frac=achieved / (PEAK_VALU_LANE_OPS / 1e12),
                traffic=measured_traffic(kname, "k_xi.hip"),
                work=f"6 ops x {r['cand']} candidate pairs + 7 ops x {r['xi_pairs']} in-grid pairs "
                     f"(lane-operations; peak = a 64-lane add per SIMD every two clocks)",
                frac_of_measured_add_rate=ops / t / peaks["valu_add_f32"] if peaks else None,
                issued_valu_frac=issued_valu_frac(kname, "k_xi.hip", r["ms_xi_kernel"]),
                ms=r["ms_xi_kernel"])


def xi_lds_roofline(r, peaks):
    """LDS-atomic side of the xi kernel: each in-grid pair contributes two FP64
    adds (N, W) and one u32 add (n) to the LDS histograms; frac is the time the
    LDS would need for them at the measured conflict-free rates over the
    kernel's time (the kernel itself merges runs of same-bin pairs first)."""
    if not peaks:
        return None
    t = r["ms_xi_kernel"] / 1e3
    p = float(r["xi_pairs"])
    busy = 2.0 * p / peaks["lds_add_f64"] + p / peaks["lds_add_u32"]
    return dict(kernel=f"{XI_KERNELS.get(r['xi_variant'], 'xi_kernel')} ({r['xi_variant_name']})", bound="lds_atomic",
                achieved=2.0 * p / t / 1e12, peak=peaks["lds_add_f64"] / 1e12, unit="T FP64 adds/s",
                frac=busy / t, work=f"2 FP64 + 1 u32 LDS adds x {r['xi_pairs']} in-grid pairs",
                peak_u32=peaks["lds_add_u32"] / 1e12, ms=r["ms_xi_kernel"])


def xi3_roofline(entries, ms, peaks):
    """Per entry (triplet i; j, k) the 3PCF kernels compute cos alpha = u_j . u_k
    (3 multiplies, 2 adds), the products w_i d_i w_j d_j w_k d_k and w_i w_j w_k
    (4 multiplies) and add them to the running sums (2 adds): 11 FP64 lane-ops;
    unmerged, an entry would also be 2 FP64 and 1 u32 LDS atomic adds."""
    t = ms / 1e3
    ops = 11.0 * entries
    out = dict(bound="alu", achieved=ops / t / 1e12, peak=PEAK_VALU_F64_LANE_OPS / 1e12, unit="TFLOP/s",
               frac=ops / t / PEAK_VALU_F64_LANE_OPS, work=f"11 FP64 lane-ops x {entries} entries")
    if peaks:
        out["lds_atomic_frac"] = entries * (2.0 / peaks["lds_add_f64"] + 1.0 / peaks["lds_add_u32"]) / t
    return out


# FP32 distortion kernels by variant index: the 8-wave kernel, the two
# single-wave tiles, and the hybrid launch of both single-wave kernels
D_KERNELS = {0: ["dmat_kernel<float, 512, true>"], 1: ["dmat_wave_kernel<float, 10, 4, 2, true, 2>"],
             2: ["dmat_wave_kernel<float, 8, 4, 2, true, 1>"],
             3: ["dmat_wave_kernel<float, 10, 4, 2, true, 2>", "dmat_wave_kernel<float, 8, 4, 2, true, 1>"]}


def d_roofline(r):
    flops = 2.0 * r["d_fmas"]
    achieved = flops / (r["ms_d_kernel"] / 1e3) / 1e12
    names = D_KERNELS.get(r["d_variant"], [])
    src = "k_dmat.hip" if r["d_variant"] == 0 else "k_dmat_wave.hip"
    parts = [measured_traffic(n, src) for n in names]
    traffic = sum(parts) if parts and all(p is not None for p in parts) else None
    # the FP32 form's contraction runs as FP32 MFMA steps: its own dtype's peak
    return dict(kernel=" + ".join(names) + f" ({r['d_variant_name']})", bound="mfma", achieved=achieved,
                peak=PEAK_MFMA_F32 / 1e12, unit="TFLOP/s", frac=achieved / (PEAK_MFMA_F32 / 1e12),
                traffic=traffic,
                work=f"2 x {r['d_fmas']} FMAs of the sparse row outer products and the rank-4 pair term "
                     f"(FP32 MFMA steps into FP32 accumulators, added to the FP64 numerator once per run)",
                ms=r["ms_d_kernel"])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1, choices=sorted(WORKLOADS))
    ap.add_argument("--keep", type=float, default=1.0, help="distortion-matrix forest-pair keep fraction")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=3, help="timed steps of the FP64 form (at most --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the full-size FP32-vs-FP64 comparison")
    ap.add_argument("--no-means", action="store_true", help="skip timing the bin-means form of the xi kernel")
    ap.add_argument("--no-xi3", action="store_true", help="skip timing the three-point kernel")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-realisation batched xi launch")
    ap.add_argument("--no-grad", action="store_true", help="skip the differentiable (forward + backward) workload")
    ap.add_argument("--no-peaks", action="store_true", help="skip the peak-rate microbenchmarks")
    ap.add_argument("--xi3-forests", type=int, default=1500,
                    help="forests nearest the patch centre used for the three-point timing")
    ap.add_argument("--xi3-wide-forests", type=int, default=500,
                    help="forests for the three-point timing on the paper's 80 Mpc/h grid")
    ap.add_argument("--cpu-xi-forests", type=int, default=600)
    ap.add_argument("--cpu-d-forests", type=int, default=200)
    ap.add_argument("--xi-variant", type=int, default=-1, help="xi kernel variant (-1: the autotuner's choice)")
    ap.add_argument("--d-variant", type=int, default=-1,
                    help="distortion kernel variant (-1: the autotuner's choice)")
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
    from synth import make_config

    log(f"[bench] generating config {args.config} (seed {args.seed})")
    F, G, extras = make_config(args.config, seed=args.seed)
    F4 = G4 = ex4 = None
    if not args.no_grad:
        F4, G4, ex4 = make_config(4, seed=args.seed)

    # the CPU oracle runs first: its worker processes are forked before this
    # process initialises the GPU
    base = oref = gref = None
    if not args.no_cpu_baseline:
        workers = host_cores()
        log(f"[bench] timing the CPU oracle on a compact sub-patch ({workers} processes)")
        base, oref, gref = oracle_stage(F, G, args.keep, args.seed, args.cpu_xi_forests, args.cpu_d_forests,
                                        F4, G4, None if ex4 is None else ex4["target"], workers)
        log(f"[bench] oracle: {base['value']:.3e} pairs/s on {workers} cores")

    from paper_2507_00129_amd import DeviceForests, Library
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
    lib = Library(0)
    peaks = None
    if not args.no_peaks:
        peaks = lib.measure_peaks()
        log("[bench] measured peaks: " + ", ".join(f"{k}={v:.3e}" for k, v in peaks.items()))
    dF = DeviceForests.from_host(F, "cuda:0")
    torch.cuda.synchronize()
    log(f"[bench] {F.n_forests} forests, {F.n_pix} pixels resident on the GPU")

    res = {}
    d64_variant = -1
    forms = ["fp32"] if args.no_fp64 else ["fp32", "fp64"]
    for prec in forms:
        steps = args.steps if prec == "fp32" else max(1, min(args.steps, args.fp64_steps))
        warm = args.warmup if prec == "fp32" else 1
        xo, do, sx, sd, wall, sdc = time_form(lib, dF, G, prec, args.keep, args.seed, steps, warm,
                                              args.xi_variant, args.d_variant)
        xi_pairs = int(xo["npairs"].sum().item())
        d_pairs = int(sdc["ingrid_pairs"])
        xv, dv = int(sx[-1]["variant"]), int(sd[-1]["variant"])
        res[prec] = dict(out_xi={k: v.cpu().numpy() for k, v in xo.items()},
                         out_d={k: v.cpu().numpy() for k, v in do.items()},
                         xi_pairs=xi_pairs, d_pairs=d_pairs, wall=wall, steps=steps, warmup=warm,
                         ms_step=1e3 * wall / steps,
                         ms_xi_kernel=mean([s["ms_main"] for s in sx]),
                         ms_d_kernel=mean([s["ms_main"] for s in sd]),
                         ms_xi_kernel_median=float(np.median([s["ms_main"] for s in sx])),
                         ms_d_kernel_median=float(np.median([s["ms_main"] for s in sd])),
                         ms_xi_total=mean([s["ms_precompute"] + s["ms_worklist"] + s["ms_main"] + s["ms_finalize"] for s in sx]),
                         ms_d_total=mean([s["ms_precompute"] + s["ms_worklist"] + s["ms_main"] + s["ms_finalize"] for s in sd]),
                         cand=int(sx[-1]["candidate_pairs"]), d_fmas=int(sdc["outer_fmas"]),
                         d_forest_pairs=int(sd[-1]["forest_pairs"]), xi_variant=xv, d_variant=dv,
                         xi_variant_name=lib.variant_name("xi", xv), d_variant_name=lib.variant_name("dmat", dv))
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
                   entries=entries, ms_kernel=ms[-1], entries_per_s=entries / t3, dtype="f64",
                   roofline=xi3_roofline(entries, ms[-1], peaks))
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
            entries=e80, ms_kernel=st3["ms_main"], entries_per_s=e80 / (st3["ms_main"] / 1e3),
            roofline=xi3_roofline(e80, st3["ms_main"], peaks))
        log(f"[bench] xi3 paper grid: {e80:.3e} entries in {st3['ms_main']:.1f} ms")
        del dS, o3

    r32 = res["fp32"]
    # dominant kernel and its roofline (algorithmic work / kernel time from HIP
    # events recorded around the launch on its stream)
    roof = xi_roofline(r32, peaks) if r32["ms_xi_kernel"] >= r32["ms_d_kernel"] else d_roofline(r32)

    line = dict(metric="pixel pairs/sec for xi + distortion matrix, FP32 vs FP64 at stated rel. error",
                value=r32["value"], unit="pixel pairs/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                ms_per_step=r32["ms_step"], higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32", data="synthetic",
                config=dict(workload=WORKLOADS[args.config], forests=F.n_forests, pixels=F.n_pix,
                            n_bins=G.n_bins, dmat_keep_fraction=args.keep, precision="FP32_COMP",
                            xi_pairs=r32["xi_pairs"], d_pairs=r32["d_pairs"],
                            d_forest_pairs=r32["d_forest_pairs"], candidate_pairs=r32["cand"]),
                roofline=roof)
    line["roofline_xi"] = xi_roofline(r32, peaks)
    line["roofline_xi_lds"] = xi_lds_roofline(r32, peaks)
    line["roofline_d"] = d_roofline(r32)
    line["variants"] = dict(xi=r32["xi_variant_name"], d=r32["d_variant_name"], chosen_by="autotuner"
                            if args.xi_variant < 0 and args.d_variant < 0 else "command line")
    if peaks:
        line["measured_peaks_lane_ops_per_s"] = peaks
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
        line["fp64"] = dict(value=r64["value"], ms_per_step=r64["ms_step"], steps=r64["steps"],
                            warmup=r64["warmup"], variants=dict(xi=r64["xi_variant_name"], d=r64["d_variant_name"]),
                            xi_pairs_per_s_kernel=r64["xi_pairs"] / (r64["ms_xi_kernel"] / 1e3),
                            d_pairs_per_s_kernel=r64["d_pairs"] / max(r64["ms_d_kernel"] / 1e3, 1e-12),
                            xi_pairs_per_s_call=r64["xi_pairs"] / (r64["ms_xi_total"] / 1e3),
                            d_pairs_per_s_call=r64["d_pairs"] / max(r64["ms_d_total"] / 1e3, 1e-12),
                            kernel_ms=dict(xi_mean=r64["ms_xi_kernel"], xi_median=r64["ms_xi_kernel_median"],
                                           d_mean=r64["ms_d_kernel"], d_median=r64["ms_d_kernel_median"]),
                            d_mfma_tflops=d64 / 1e12, d_mfma_frac_of_f64_peak=d64 / PEAK_MFMA_F64)
        d64_variant = r64["d_variant"]
        line["fp32_over_fp64"] = r32["value"] / r64["value"]
        line["fp32_over_fp64_xi_kernel"] = r64["ms_xi_kernel"] / r32["ms_xi_kernel"]
        line["fp32_over_fp64_d_kernel"] = r64["ms_d_kernel"] / r32["ms_d_kernel"]
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
    del dF, res

    if not args.no_grad:
        # differentiable workload: 10k forests over 100 deg^2, FP32 forward and
        # the hand-written backward of sum_b (xi_b - m_b)^2
        import oracle
        dF4 = DeviceForests.from_host(F4, "cuda:0")
        tgt = torch.as_tensor(ex4["target"], device="cuda:0")[None, :]
        fw, bw = [], []
        for k in range(4):
            o4 = lib.xi(dF4, G4, precision="fp32", timing=True)
            fw.append(lib.last_stats())
            gxi = 2.0 * (o4["xi"] - tgt)
            lib.xi_backward(dF4, G4, gxi, o4["xi"], o4["wsum"], precision="fp32", timing=True)
            bw.append(lib.last_stats())
        torch.cuda.synchronize()
        p4 = int(o4["npairs"].sum().item())
        fms, bms = mean([s["ms_main"] for s in fw[1:]]), mean([s["ms_main"] for s in bw[1:]])
        grad = dict(workload="10k forests over 100 deg^2, 50x50 bins to 200 Mpc/h, loss sum_b (xi_b - m_b)^2",
                    in_grid_pairs=p4, fwd_ms_kernel=fms, bwd_ms_kernel=bms,
                    fwd_pairs_per_s_kernel=p4 / (fms / 1e3), bwd_pairs_per_s_kernel=p4 / (bms / 1e3),
                    note="the backward visits every in-grid pair once per direction")
        if gref is not None:
            dS4 = DeviceForests.from_host(gref["S"], "cuda:0")
            for prec in ("fp32", "fp64"):
                o = lib.xi(dS4, G4, precision=prec)
                gd, gw = lib.xi_backward(dS4, G4, 2.0 * (o["xi"] - tgt), o["xi"], o["wsum"], precision=prec)
                grad[f"e_g_{prec}"] = dict(delta=oracle.err_norm(gd.cpu().numpy(), gref["gd"]),
                                           weight=oracle.err_norm(gw.cpu().numpy(), gref["gw"]),
                                           subset="200 forests nearest the centre", pairs=gref["pairs"])
            del dS4
        line["config4_grad"] = grad
        log(f"[bench] config 4: forward {fms:.2f} ms, backward {bms:.2f} ms ({p4} in-grid pairs)")
        del dF4, o4

    if not args.no_batched:
        # 64 realisations with 2k-20k forests each in one persistent launch
        F3, G3, ex3 = make_config(3, seed=args.seed)
        dF3 = DeviceForests.from_host(F3, "cuda:0")
        st = []
        for k in range(3):
            o3 = lib.xi(dF3, G3, precision="fp32", timing=True)
            st.append(lib.last_stats())
        torch.cuda.synchronize()
        p3 = int(o3["npairs"].sum().item())
        kms = mean([s["ms_main"] for s in st[1:]])
        cms = mean([s["ms_precompute"] + s["ms_worklist"] + s["ms_main"] + s["ms_finalize"] for s in st[1:]])
        line["config3_batched"] = dict(
            workload=f"{F3.n_realisations} realisations, {F3.n_forests} forests, {F3.n_pix} pixels; "
                     f"xi on 50x50 bins to 200 Mpc/h, FP32 form",
            in_grid_pairs=p3, ms_kernel=kms, ms_call=cms, pairs_per_s_kernel=p3 / (kms / 1e3),
            pairs_per_s_call=p3 / (cms / 1e3), variant=lib.variant_name("xi", st[-1]["variant"]))
        log(f"[bench] config 3: {p3:.3e} pairs, kernel {kms:.1f} ms")
        del dF3, o3

    if base is not None:
        line["cpu_baseline"] = base
        xv = r32["xi_variant"]
        line["vs_oracle_sample"] = gpu_sample_errors(lib, oref, G, args.keep, args.seed, 0 if xv != 0 else 1,
                                                     d64_variant)
    line["paper_timings"] = PAPER_TIMINGS
    print(json.dumps(line), flush=True)
    lib.close()


if __name__ == "__main__":
    main()
