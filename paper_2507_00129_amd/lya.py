"""ctypes binding of the C ABI in include/lya.h.

Argument marshalling only: every step of the computation runs in the HIP
library.  Device arrays are torch CUDA tensors (used for memory and streams);
grid edges stay on the host.  Importing works without a GPU; calls need one.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "liblya.so")

LYA_OK, LYA_E_INVALID, LYA_E_NOMEM, LYA_E_DEVICE, LYA_E_UNSUPPORTED = 0, 1, 2, 3, 4
FP32_COMP, FP64 = 0, 1
ETA_IDENTITY, ETA_MEAN, ETA_MEAN_SLOPE = 0, 1, 2

_PRECISION = {"fp32": FP32_COMP, "fp32_comp": FP32_COMP, "fp64": FP64, FP32_COMP: FP32_COMP, FP64: FP64}
_ETA = {"identity": ETA_IDENTITY, "mean": ETA_MEAN, "mean_slope": ETA_MEAN_SLOPE,
        ETA_IDENTITY: ETA_IDENTITY, ETA_MEAN: ETA_MEAN, ETA_MEAN_SLOPE: ETA_MEAN_SLOPE}


class LyaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lya status {status}: {msg}")
        self.status = status


class lya_forests(ctypes.Structure):
    _fields_ = [
        ("n_forests", ctypes.c_int64), ("n_pix", ctypes.c_int64),
        ("offsets", ctypes.c_void_p), ("ra", ctypes.c_void_p), ("dec", ctypes.c_void_p),
        ("dist", ctypes.c_void_p), ("delta", ctypes.c_void_p), ("weight", ctypes.c_void_p),
        ("loglam", ctypes.c_void_p), ("realisation", ctypes.c_void_p),
        ("n_realisations", ctypes.c_int32),
    ]


class lya_grid(ctypes.Structure):
    _fields_ = [("n_par", ctypes.c_int32), ("n_perp", ctypes.c_int32),
                ("edges_par", ctypes.c_void_p), ("edges_perp", ctypes.c_void_p)]


class lya_grid3(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int32), ("n_theta", ctypes.c_int32), ("n_cos", ctypes.c_int32),
                ("r_edges", ctypes.c_void_p), ("theta_edges", ctypes.c_void_p), ("cos_edges", ctypes.c_void_p)]


class lya_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("eta", ctypes.c_int32), ("project_deltas", ctypes.c_int32),
        ("autotune", ctypes.c_int32), ("validate", ctypes.c_int32), ("timing", ctypes.c_int32),
        ("variant", ctypes.c_int32), ("counters", ctypes.c_int32),
        ("dmat_keep_fraction", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("deterministic", ctypes.c_int32),
    ]


class lya_stats(ctypes.Structure):
    _fields_ = [
        ("forest_pairs", ctypes.c_int64), ("work_items", ctypes.c_int64),
        ("candidate_pairs", ctypes.c_int64), ("variant", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32), ("ms_precompute", ctypes.c_float),
        ("ms_worklist", ctypes.c_float), ("ms_main", ctypes.c_float), ("ms_finalize", ctypes.c_float),
        ("ingrid_pairs", ctypes.c_int64), ("outer_fmas", ctypes.c_int64),
        ("lost_pairs", ctypes.c_int64),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads liblya.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run paper_2507_00129_amd.build)")
    # torch first: its HIP runtime is then the one the library binds to (same
    # soname), so streams and device pointers from torch are valid in the
    # library; loaded the other way round, the process would hold two HIP
    # runtimes
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.lya_options_default.argtypes = [ctypes.POINTER(lya_options)]
    lib.lya_options_default.restype = None
    lib.lya_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
    lib.lya_create.restype = I32
    lib.lya_destroy.argtypes = [P]
    lib.lya_destroy.restype = None
    lib.lya_last_error.argtypes = [P]
    lib.lya_last_error.restype = ctypes.c_char_p
    lib.lya_last_stats.argtypes = [P, ctypes.POINTER(lya_stats)]
    lib.lya_last_stats.restype = I32
    FP, GP, OP = ctypes.POINTER(lya_forests), ctypes.POINTER(lya_grid), ctypes.POINTER(lya_options)
    lib.lya_xi.argtypes = [P, FP, GP, OP, P, P, P, P, P]
    lib.lya_xi.restype = I32
    lib.lya_xi_noalloc.argtypes = [P, FP, GP, OP, P, P, P, P, P]
    lib.lya_xi_noalloc.restype = I32
    lib.lya_dmat.argtypes = [P, FP, GP, OP, P, P, P]
    lib.lya_dmat.restype = I32
    lib.lya_xi_backward.argtypes = [P, FP, GP, OP, P, P, P, P, P, P]
    lib.lya_xi_backward.restype = I32
    lib.lya_xi_subsamples.argtypes = [P, FP, GP, OP, P, P, I32, P, P, P, P]
    lib.lya_xi_subsamples.restype = I32
    lib.lya_xi3.argtypes = [P, FP, ctypes.POINTER(lya_grid3), OP, P, P, P, P, P]
    lib.lya_xi3.restype = I32
    lib.lya_xi3_subsamples.argtypes = [P, FP, ctypes.POINTER(lya_grid3), OP, P, P, I32, P, P, P, P]
    lib.lya_xi3_subsamples.restype = I32
    lib.lya_xi_means.argtypes = [P, FP, GP, OP, P, P, P, P, P, P, P, P]
    lib.lya_xi_means.restype = I32
    lib.lya_xi_covariance.argtypes = [P, P, P, I64, I64, P, P, P]
    lib.lya_xi_covariance.restype = I32
    lib.lya_variant_name.argtypes = [I32, I32]
    lib.lya_variant_name.restype = ctypes.c_char_p
    lib.lya_measure_peaks.argtypes = [P, P, ctypes.POINTER(ctypes.c_double)]
    lib.lya_measure_peaks.restype = I32
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


@dataclass
class DeviceForests:
    """Forests resident on the GPU as torch tensors (CSR layout of lya.h)."""
    offsets: "object"
    ra: "object"
    dec: "object"
    dist: "object"
    delta: "object"
    weight: "object"
    loglam: "object"
    realisation: "object" = None
    n_realisations: int = 1
    offsets_host: Optional[np.ndarray] = None

    @property
    def n_forests(self):
        return int(self.ra.shape[0])

    @property
    def n_pix(self):
        return int(self.dist.shape[0])

    @classmethod
    def from_host(cls, F, device="cuda"):
        import torch
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)
        real = None if getattr(F, "realisation", None) is None else t(F.realisation, torch.int32)
        return cls(t(F.offsets, torch.int64), t(F.ra, torch.float64), t(F.dec, torch.float64),
                   t(F.dist, torch.float64), t(F.delta, torch.float64), t(F.weight, torch.float64),
                   t(F.loglam, torch.float64), real, int(getattr(F, "n_realisations", 1)),
                   np.asarray(F.offsets, np.int64).copy())

    def with_values(self, delta=None, weight=None):
        return DeviceForests(self.offsets, self.ra, self.dec, self.dist,
                             self.delta if delta is None else delta,
                             self.weight if weight is None else weight,
                             self.loglam, self.realisation, self.n_realisations, self.offsets_host)

    def c_struct(self) -> lya_forests:
        for name in ("ra", "dec", "dist", "delta", "weight", "loglam"):
            v = getattr(self, name)
            if not v.is_contiguous() or str(v.dtype) != "torch.float64":
                raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
        return lya_forests(self.n_forests, self.n_pix, _ptr(self.offsets), _ptr(self.ra), _ptr(self.dec),
                           _ptr(self.dist), _ptr(self.delta), _ptr(self.weight), _ptr(self.loglam),
                           _ptr(self.realisation), int(self.n_realisations))


class HostGrid:
    """Keeps the edge arrays alive for the duration of a call."""

    def __init__(self, grid):
        self.ep = np.ascontiguousarray(grid.edges_par, np.float64)
        self.et = np.ascontiguousarray(grid.edges_perp, np.float64)
        self.n_bins = (self.ep.shape[0] - 1) * (self.et.shape[0] - 1)

    def c_struct(self) -> lya_grid:
        return lya_grid(self.ep.shape[0] - 1, self.et.shape[0] - 1,
                        self.ep.ctypes.data, self.et.ctypes.data)


class HostGrid3:
    """Edge arrays of a three-point grid (any object with r_edges, theta_edges
    and cos_edges), kept alive for the duration of a call."""

    def __init__(self, grid):
        self.er = np.ascontiguousarray(grid.r_edges, np.float64)
        self.et = np.ascontiguousarray(grid.theta_edges, np.float64)
        self.ec = np.ascontiguousarray(grid.cos_edges, np.float64)
        nr, nt, nc = (e.shape[0] - 1 for e in (self.er, self.et, self.ec))
        self.n_bins = nr * nr * nc * nt * nt

    def c_struct(self) -> lya_grid3:
        return lya_grid3(self.er.shape[0] - 1, self.et.shape[0] - 1, self.ec.shape[0] - 1,
                         self.er.ctypes.data, self.et.ctypes.data, self.ec.ctypes.data)


class Library:
    """One lya_context bound to a CUDA device."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        import torch
        self.device = int(device)
        torch.cuda.init()
        self.ctx = ctypes.c_void_p()
        s = self.lib.lya_create(ctypes.byref(self.ctx), self.device)
        if s != LYA_OK:
            raise LyaError(s, f"lya_create(device={device}) failed: {self.lib.lya_last_error(None).decode()}")

    def close(self):
        if self.ctx:
            self.lib.lya_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def options(self, precision="fp32", eta="mean_slope", project_deltas=False, autotune=True,
                validate=True, timing=False, keep_fraction=1.0, seed=0, variant=-1,
                counters=False, deterministic=False) -> lya_options:
        o = lya_options()
        self.lib.lya_options_default(ctypes.byref(o))
        o.precision = _PRECISION[precision]
        o.eta = _ETA[eta]
        o.project_deltas = int(bool(project_deltas))
        o.autotune = int(bool(autotune))
        o.validate = int(bool(validate))
        o.timing = int(bool(timing))
        o.counters = int(bool(counters))
        o.dmat_keep_fraction = float(keep_fraction)
        o.seed = int(seed)
        o.variant = int(variant)
        o.deterministic = int(bool(deterministic))
        return o

    def _check(self, status):
        if status != LYA_OK:
            raise LyaError(status, self.lib.lya_last_error(self.ctx).decode())

    def _stream(self, stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(int(stream.cuda_stream))

    def last_stats(self) -> dict:
        st = lya_stats()
        self._check(self.lib.lya_last_stats(self.ctx, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in lya_stats._fields_}

    def xi(self, forests: DeviceForests, grid, stream=None, out=None, **opts):
        """Pair sums and xi; returns dict of [n_realisations, n_bins] tensors."""
        import torch
        g = HostGrid(grid)
        R = int(forests.n_realisations)
        dev = forests.dist.device
        if out is None:
            out = dict(num=torch.empty((R, g.n_bins), dtype=torch.float64, device=dev),
                       wsum=torch.empty((R, g.n_bins), dtype=torch.float64, device=dev),
                       npairs=torch.empty((R, g.n_bins), dtype=torch.int64, device=dev),
                       xi=torch.empty((R, g.n_bins), dtype=torch.float64, device=dev))
        fs, gs, o = forests.c_struct(), g.c_struct(), self.options(**opts)
        self._check(self.lib.lya_xi(self.ctx, ctypes.byref(fs), ctypes.byref(gs), ctypes.byref(o),
                                    self._stream(stream), _ptr(out["num"]), _ptr(out["wsum"]),
                                    _ptr(out["npairs"]), _ptr(out.get("xi"))))
        return out

    def xi_noalloc(self, forests: DeviceForests, grid, out, stream=None, **opts):
        """lya_xi_noalloc: xi into caller-given outputs (dict of [R, n_bins]
        tensors num, wsum, npairs and optionally xi) with no device allocation
        in the library."""
        g = HostGrid(grid)
        fs, gs, o = forests.c_struct(), g.c_struct(), self.options(**opts)
        self._check(self.lib.lya_xi_noalloc(self.ctx, ctypes.byref(fs), ctypes.byref(gs), ctypes.byref(o),
                                            self._stream(stream), _ptr(out["num"]), _ptr(out["wsum"]),
                                            _ptr(out["npairs"]), _ptr(out.get("xi"))))
        return out

    def xi3(self, forests: DeviceForests, grid3, stream=None, out=None, **opts):
        """Triplet sums and xi3 of the anisotropic three-point function (FP64);
        returns dict of [n_realisations, n_bins] tensors."""
        import torch
        g = HostGrid3(grid3)
        R = int(forests.n_realisations)
        dev = forests.dist.device
        if out is None:
            out = {k: torch.empty((R, g.n_bins), dtype=torch.int64 if k == "ntrip" else torch.float64, device=dev)
                   for k in ("num", "wsum", "ntrip", "xi")}
        fs, gs, o = forests.c_struct(), g.c_struct(), self.options(**opts)
        self._check(self.lib.lya_xi3(self.ctx, ctypes.byref(fs), ctypes.byref(gs), ctypes.byref(o),
                                     self._stream(stream), _ptr(out["num"]), _ptr(out["wsum"]),
                                     _ptr(out["ntrip"]), _ptr(out.get("xi"))))
        return out

    def xi3_subsamples(self, forests: DeviceForests, grid3, subsample, n_sub, stream=None, out=None, **opts):
        """Triplet sums of the 3PCF split by the subsample of each entry's main
        vertex forest; returns dict of [R, n_sub, n_bins] tensors.  `subsample`
        is an int32 device tensor [n_forests] with ids in [0, n_sub)."""
        import torch
        g = HostGrid3(grid3)
        R = int(forests.n_realisations)
        dev = forests.dist.device
        sub = subsample.to(device=dev, dtype=torch.int32).contiguous()
        if sub.numel() != forests.n_forests:
            raise ValueError("subsample must have one entry per forest")
        shape = (R, int(n_sub), g.n_bins)
        if out is None:
            out = {k: torch.empty(shape, dtype=torch.int64 if k == "ntrip" else torch.float64, device=dev)
                   for k in ("num", "wsum", "ntrip", "xi")}
        fs, gs, o = forests.c_struct(), g.c_struct(), self.options(**opts)
        self._check(self.lib.lya_xi3_subsamples(self.ctx, ctypes.byref(fs), ctypes.byref(gs), ctypes.byref(o),
                                                self._stream(stream), _ptr(sub), int(n_sub), _ptr(out["num"]),
                                                _ptr(out["wsum"]), _ptr(out["ntrip"]), _ptr(out.get("xi"))))
        return out

    def xi_means(self, forests: DeviceForests, grid, stream=None, out=None, **opts):
        """Pair sums, xi and the weighted bin-mean r_par, r_perp and z (z needs
        loglam = ln(lambda / Angstrom)); returns dict of [R, n_bins] tensors."""
        import torch
        g = HostGrid(grid)
        R = int(forests.n_realisations)
        dev = forests.dist.device
        if out is None:
            out = {k: torch.empty((R, g.n_bins), dtype=torch.int64 if k == "npairs" else torch.float64, device=dev)
                   for k in ("num", "wsum", "npairs", "xi", "rpar", "rperp", "z")}
        fs, gs, o = forests.c_struct(), g.c_struct(), self.options(**opts)
        self._check(self.lib.lya_xi_means(self.ctx, ctypes.byref(fs), ctypes.byref(gs), ctypes.byref(o),
                                          self._stream(stream), _ptr(out["num"]), _ptr(out["wsum"]),
                                          _ptr(out["npairs"]), _ptr(out.get("xi")), _ptr(out["rpar"]),
                                          _ptr(out["rperp"]), _ptr(out["z"])))
        return out

    def xi_subsamples(self, forests: DeviceForests, grid, subsample, n_sub, stream=None, out=None, **opts):
        """Pair sums split by the subsample of each pair's owning forest (the one
        with the smaller input index); returns dict of [R, n_sub, n_bins] tensors.
        `subsample` is an int32 device tensor [n_forests] with ids in [0, n_sub)."""
        import torch
        g = HostGrid(grid)
        R = int(forests.n_realisations)
        dev = forests.dist.device
        sub = subsample.to(device=dev, dtype=torch.int32).contiguous()
        if sub.numel() != forests.n_forests:
            raise ValueError("subsample must have one entry per forest")
        shape = (R, int(n_sub), g.n_bins)
        if out is None:
            out = dict(num=torch.empty(shape, dtype=torch.float64, device=dev),
                       wsum=torch.empty(shape, dtype=torch.float64, device=dev),
                       npairs=torch.empty(shape, dtype=torch.int64, device=dev),
                       xi=torch.empty(shape, dtype=torch.float64, device=dev))
        fs, gs, o = forests.c_struct(), g.c_struct(), self.options(**opts)
        self._check(self.lib.lya_xi_subsamples(self.ctx, ctypes.byref(fs), ctypes.byref(gs), ctypes.byref(o),
                                               self._stream(stream), _ptr(sub), int(n_sub), _ptr(out["num"]),
                                               _ptr(out["wsum"]), _ptr(out["npairs"]), _ptr(out.get("xi"))))
        return out

    def xi_covariance(self, num, wsum, stream=None):
        """Subsample covariance of xi from one realisation's [n_sub, n_bins] sums;
        returns (xi [n_bins], cov [n_bins, n_bins])."""
        import torch
        num = num.contiguous().to(torch.float64)
        wsum = wsum.contiguous().to(torch.float64)
        n_sub, nb = int(num.shape[0]), int(num.shape[1])
        xi = torch.empty(nb, dtype=torch.float64, device=num.device)
        cov = torch.empty((nb, nb), dtype=torch.float64, device=num.device)
        self._check(self.lib.lya_xi_covariance(self.ctx, _ptr(num), _ptr(wsum), n_sub, nb, self._stream(stream),
                                               _ptr(xi), _ptr(cov)))
        return xi, cov

    PEAK_KEYS = ("valu_fma_f32", "valu_fma_f64", "lds_add_f32", "lds_add_f64", "lds_add_u32",
                 "lds_add_f32_4per_address", "lds_store_b32", "valu_add_f32", "valu_add_u32")

    def variant_name(self, kernel: str, variant: int) -> str:
        """Name of a main-kernel variant; kernel is "xi" or "dmat"."""
        n = self.lib.lya_variant_name({"xi": 0, "dmat": 1}[kernel], int(variant))
        if n is None:
            raise ValueError(f"no {kernel} variant {variant}")
        return n.decode()

    def measure_peaks(self, stream=None) -> dict:
        """Measured whole-chip lane-operations per second (lya_measure_peaks)."""
        buf = (ctypes.c_double * len(self.PEAK_KEYS))()
        self._check(self.lib.lya_measure_peaks(self.ctx, self._stream(stream), buf))
        return {k: float(buf[i]) for i, k in enumerate(self.PEAK_KEYS)}

    def dmat(self, forests: DeviceForests, grid, stream=None, out=None, **opts):
        """Distortion matrix; returns dict(dmat [R, nb, nb], wsum_d [R, nb])."""
        import torch
        g = HostGrid(grid)
        R = int(forests.n_realisations)
        dev = forests.dist.device
        if out is None:
            out = dict(dmat=torch.empty((R, g.n_bins, g.n_bins), dtype=torch.float64, device=dev),
                       wsum_d=torch.empty((R, g.n_bins), dtype=torch.float64, device=dev))
        fs, gs, o = forests.c_struct(), g.c_struct(), self.options(**opts)
        self._check(self.lib.lya_dmat(self.ctx, ctypes.byref(fs), ctypes.byref(gs), ctypes.byref(o),
                                      self._stream(stream), _ptr(out["dmat"]), _ptr(out["wsum_d"])))
        return out

    def xi_backward(self, forests: DeviceForests, grid, grad_xi, xi, wsum, stream=None, out=None, **opts):
        """dL/ddelta and dL/dw for dL/dxi = grad_xi; returns (grad_delta, grad_weight)."""
        import torch
        g = HostGrid(grid)
        dev = forests.dist.device
        if out is None:
            out = (torch.empty(forests.n_pix, dtype=torch.float64, device=dev),
                   torch.empty(forests.n_pix, dtype=torch.float64, device=dev))
        gx, x, w = (t.contiguous().to(torch.float64) for t in (grad_xi, xi, wsum))
        fs, gs, o = forests.c_struct(), g.c_struct(), self.options(**opts)
        self._check(self.lib.lya_xi_backward(self.ctx, ctypes.byref(fs), ctypes.byref(gs), ctypes.byref(o),
                                             self._stream(stream), _ptr(gx), _ptr(x), _ptr(w),
                                             _ptr(out[0]), _ptr(out[1])))
        return out
