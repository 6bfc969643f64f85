"""Python binding of libheget (include/heget.h): argument marshalling only.

Every step of the |M|^2 / cross-section path runs in the HIP kernels of the
in-tree ``libheget.so``; there is no CPU fallback.  Importing this package
fails loudly if the library has not been built
(``python paper_0908_4403_amd/build.py``).

The library is opened on the first call, after importing torch when it is
installed: torch ships its own HIP runtime, and loading it first makes
libheget bind to that same runtime, so the process has one HIP runtime
whichever module the caller imported first.

Host-array calls take and return numpy arrays (event layout [npoints, n+2, 4]).
Device calls take torch tensors on the GPU (SoA layout [(n+2)*4, npoints],
float64) and enqueue on ``torch.cuda.current_stream()`` unless a stream is
given; torch only provides memory and streams here.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libheget.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_0908_4403_amd/build.py`")


OK, WARN_NONFINITE = 0, 1
ERR_ARG, ERR_RANGE, ERR_ALLOC, ERR_DEVICE = -1, -2, -3, -4
FP64, FP32 = 0, 1
FIXED_SHAT, UNIFORM_SQRTSHAT, PP_TOY = 0, 1, 2
OBS_PT_MAX, OBS_DR_MIN = 0, 1

EXPORTS = ["heget_gen_points", "heget_gen_points_device", "heget_me2", "heget_me2_device",
           "heget_me2_async",
           "heget_xsec", "heget_xsec_async", "heget_xsec_device", "heget_xsec_device_noalloc",
           "heget_xsec_hist",
           "heget_xsec_events",
           "heget_xsec_batch",
           "heget_set_batch_schedule", "heget_batch_schedule_in_use",
           "heget_set_couplings",
           "heget_timing_enable",
           "heget_timing_read", "heget_me2_flops", "heget_autotune", "heget_kernel_shapes",
           "heget_set_kernel_shape", "heget_valu_peak",
           "heget_helas_sizes", "heget_helas", "heget_helas_device",
           "heget_me2_frame", "heget_me2_frame_device",
           "heget_last_error", "heget_shutdown"]


class Cuts(C.Structure):
    _fields_ = [("pt_min", C.c_double), ("eta_max", C.c_double), ("dr_min", C.c_double)]


class _Config(C.Structure):
    _fields_ = [("mode", C.c_int32), ("prec", C.c_int32), ("seed", C.c_uint64),
                ("npoints", C.c_int64), ("sqrt_s", C.c_double), ("sqrt_shat_lo", C.c_double),
                ("sqrt_shat_hi", C.c_double), ("cuts", Cuts), ("alpha", C.c_double),
                ("charge", C.c_double), ("helicity_sampling", C.c_int32), ("reserved", C.c_int32)]


class Shape(C.Structure):
    _fields_ = [("unrolled", C.c_int32), ("helicities_per_walk", C.c_int32),
                ("closing", C.c_int32), ("waves_per_block", C.c_int32), ("prefetch", C.c_int32),
                ("waves_per_simd", C.c_int32), ("points_per_lane", C.c_int32),
                ("prefix_sets", C.c_int32)]

    def as_tuple(self):
        return (self.unrolled, self.helicities_per_walk, self.closing, self.waves_per_block,
                self.prefetch, self.waves_per_simd, self.points_per_lane, self.prefix_sets)


class Result(C.Structure):
    _fields_ = [("sigma_fb", C.c_double), ("err_fb", C.c_double), ("sum_w", C.c_double),
                ("sum_w_comp", C.c_double), ("sum_w2", C.c_double), ("n_gen", C.c_int64),
                ("n_acc", C.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_dp = C.POINTER(C.c_double)
_st = C.c_int
_handle = None


def _load():
    global _handle
    if _handle is not None:
        return _handle
    try:
        import torch  # noqa: F401  (its HIP runtime first; see the module docstring)
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    lib.heget_gen_points.argtypes = [C.c_int, C.c_double, C.POINTER(Cuts), C.c_uint64, C.c_int64,
                                     _dp, _dp]
    lib.heget_gen_points_device.argtypes = [C.c_int, C.c_double, C.POINTER(Cuts), C.c_uint64,
                                            C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.heget_me2.argtypes = [C.c_int, C.c_int64, _dp, _dp, C.c_int]
    lib.heget_me2_device.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_int,
                                     C.c_void_p]
    lib.heget_me2_async.argtypes = lib.heget_me2_device.argtypes
    lib.heget_xsec.argtypes = [C.c_int, C.POINTER(_Config), C.POINTER(Result)]
    lib.heget_xsec_async.argtypes = [C.c_int, C.POINTER(_Config), C.POINTER(Result), C.c_void_p]
    lib.heget_set_batch_schedule.argtypes = [C.c_int]
    lib.heget_xsec_hist.argtypes = [C.c_int, C.POINTER(_Config), C.c_int, C.c_int, C.c_double,
                                    C.c_double, _dp, C.POINTER(Result)]
    lib.heget_batch_schedule_in_use.argtypes = [C.POINTER(C.c_int), C.POINTER(_Config), C.c_int,
                                                C.POINTER(C.c_int)]
    lib.heget_xsec_device.argtypes = [C.c_int, C.POINTER(_Config), C.c_void_p, C.c_void_p]
    lib.heget_xsec_device_noalloc.argtypes = lib.heget_xsec_device.argtypes
    lib.heget_xsec_batch.argtypes = [C.POINTER(C.c_int), C.POINTER(_Config), C.c_int,
                                     C.POINTER(Result)]
    lib.heget_set_couplings.argtypes = [C.c_double, C.c_double]
    lib.heget_timing_enable.argtypes = [C.c_int]
    lib.heget_timing_read.argtypes = [_dp, C.POINTER(C.c_int64), C.c_int]
    lib.heget_me2_flops.argtypes = [C.c_int, C.c_int, _dp, C.POINTER(Shape)]
    lib.heget_autotune.argtypes = [C.c_int, C.c_int, C.c_int64, C.POINTER(Shape), _dp]
    lib.heget_kernel_shapes.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(Shape),
                                        C.POINTER(C.c_int)]
    lib.heget_set_kernel_shape.argtypes = [C.c_int, C.c_int, C.POINTER(Shape)]
    lib.heget_valu_peak.argtypes = [_dp, _dp]
    lib.heget_helas_sizes.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.heget_helas.argtypes = [C.c_int, C.c_int64, _dp, _dp, C.c_int]
    lib.heget_helas_device.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_int,
                                       C.c_void_p]
    lib.heget_me2_frame.argtypes = [C.c_int, C.c_int64, _dp, _dp, C.c_int]
    lib.heget_me2_frame_device.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_int,
                                           C.c_void_p]
    lib.heget_last_error.restype = C.c_char_p
    lib.heget_shutdown.restype = None
    for f in EXPORTS[:-2]:
        getattr(lib, f).restype = _st
    _handle = lib
    return lib


class _LazyLib:
    def __getattr__(self, name):
        return getattr(_load(), name)


_lib = _LazyLib()


class HegetError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where} failed with status {status}: {last_error()}")


def last_error() -> str:
    return _lib.heget_last_error().decode()


def _check(status: int, where: str) -> int:
    if status < 0:
        raise HegetError(status, where)
    return status


def _cuts(cuts) -> Cuts | None:
    if cuts is None:
        return None
    if isinstance(cuts, Cuts):
        return cuts
    return Cuts(*[float(x) for x in cuts])


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# ---- host-array calls -------------------------------------------------------

def gen_points(n: int, sqrt_s: float, cuts=(20.0, 2.5, 0.4), seed: int = 0, npoints: int = 1024):
    """(momenta[npoints, n+2, 4], weight[npoints]) at fixed sqrt(shat)."""
    mom = np.zeros((npoints, n + 2, 4))
    w = np.zeros(npoints)
    c = _cuts(cuts)
    _check(_lib.heget_gen_points(n, sqrt_s, C.byref(c) if c else None, seed, npoints,
                                 _ptr(mom), _ptr(w)), "heget_gen_points")
    return mom, w


def me2(momenta, prec: int = FP64, return_status: bool = False):
    """Helicity-summed |M|^2 at momenta[npoints, n+2, 4] (host arrays)."""
    p = np.ascontiguousarray(momenta, dtype=np.float64)
    if p.ndim != 3 or p.shape[2] != 4:
        raise ValueError("momenta must have shape [npoints, n+2, 4]")
    n = p.shape[1] - 2
    out = np.zeros(p.shape[0])
    st = _check(_lib.heget_me2(n, p.shape[0], _ptr(p), _ptr(out), prec), "heget_me2")
    return (out, st) if return_status else out


@dataclass
class Config:
    mode: int = FIXED_SHAT
    prec: int = FP32
    seed: int = 0
    npoints: int = 16384
    sqrt_s: float = 500.0
    sqrt_shat_lo: float = 0.0
    sqrt_shat_hi: float = 0.0
    pt_min: float = 20.0
    eta_max: float = 2.5
    dr_min: float = 0.4
    alpha: float = 1.0 / 137.0
    charge: float = 2.0 / 3.0
    helicity_sampling: int = 0  # 1: one drawn helicity configuration per point

    def c(self) -> _Config:
        return _Config(self.mode, self.prec, self.seed, self.npoints, self.sqrt_s,
                       self.sqrt_shat_lo, self.sqrt_shat_hi,
                       Cuts(self.pt_min, self.eta_max, self.dr_min), self.alpha, self.charge,
                       self.helicity_sampling, 0)


def xsec(n: int, cfg: Config, return_status: bool = False) -> dict:
    r = Result()
    c = cfg.c()
    st = _check(_lib.heget_xsec(n, C.byref(c), C.byref(r)), "heget_xsec")
    d = r.as_dict()
    return (d, st) if return_status else d


# The library writes an async result when the stream reaches it, so the
# Result storage must outlive the Python handle: the last _MAX_INFLIGHT are
# kept here (the library's staging ring holds 256 calls in flight).
_MAX_INFLIGHT = 1024
_inflight: "collections.deque" = None


def xsec_batch(ns, cfgs, return_status: bool = False):
    """Cross sections of several configurations in one device pass (list of dicts)."""
    k = len(ns)
    na = (C.c_int * k)(*ns)
    ca = (_Config * k)(*[c.c() for c in cfgs])
    ra = (Result * k)()
    st = _check(_lib.heget_xsec_batch(na, ca, k, ra), "heget_xsec_batch")
    out = [r.as_dict() for r in ra]
    return (out, st) if return_status else out


def xsec_device(n: int, cfg: Config, out, stream=None) -> None:
    """Enqueue the cross section with its result record written by the device into
    `out`: a contiguous torch tensor of >= 56 bytes on the GPU or in pinned host
    memory (layout of Result; read it back with result_from_bytes)."""
    if out.numel() * out.element_size() < C.sizeof(Result) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous tensor of at least {C.sizeof(Result)} bytes")
    if not (out.is_cuda or _is_pinned(out)):
        raise ValueError("out must be GPU memory or pinned host memory")
    c = cfg.c()
    _check(_lib.heget_xsec_device(n, C.byref(c), C.c_void_p(out.data_ptr()), _stream(stream)),
           "heget_xsec_device")


def xsec_device_noalloc(n: int, cfg: Config, out, stream=None) -> None:
    """heget_xsec_device_noalloc: xsec_device on the library's fixed static
    workspace (no device allocation); same arguments.  Raises (ERR_RANGE) when
    the configuration's buffers exceed that workspace."""
    if out.numel() * out.element_size() < C.sizeof(Result) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous tensor of at least {C.sizeof(Result)} bytes")
    if not (out.is_cuda or _is_pinned(out)):
        raise ValueError("out must be GPU memory or pinned host memory")
    c = cfg.c()
    _check(_lib.heget_xsec_device_noalloc(n, C.byref(c), C.c_void_p(out.data_ptr()), _stream(stream)),
           "heget_xsec_device_noalloc")


def result_from_bytes(buf) -> dict:
    """Decode a Result record (56 bytes, e.g. from xsec_device) into a dict."""
    raw = bytes(buf[:C.sizeof(Result)])
    return Result.from_buffer_copy(raw).as_dict()


BATCH_AUTO, BATCH_PERSISTENT, BATCH_BRANCHES = 0, 1, 2


def set_batch_schedule(schedule: int) -> None:
    _check(_lib.heget_set_batch_schedule(schedule), "heget_set_batch_schedule")


def batch_schedule_in_use(ns, cfgs) -> int:
    k = len(ns)
    na = (C.c_int * k)(*ns)
    ca = (_Config * k)(*[c.c() for c in cfgs])
    s = C.c_int()
    _check(_lib.heget_batch_schedule_in_use(na, ca, k, C.byref(s)), "heget_batch_schedule_in_use")
    return s.value


class XsecAsync:
    """Handle of an enqueued heget_xsec_async; .result() after the stream completes.

    At most 256 calls may be in flight at once (the library's staging ring)."""

    def __init__(self, n: int, cfg: Config, stream=None):
        global _inflight
        import collections
        if _inflight is None:
            _inflight = collections.deque(maxlen=_MAX_INFLIGHT)
        self._res = Result()
        self._cfg = cfg.c()
        _inflight.append(self._res)
        _check(_lib.heget_xsec_async(n, C.byref(self._cfg), C.byref(self._res), _stream(stream)),
               "heget_xsec_async")

    def result(self) -> dict:
        return self._res.as_dict()


# ---- device calls (torch tensors) -------------------------------------------

def me2_device(n: int, mom_soa, out, prec: int = FP32, stream=None) -> None:
    """|M|^2 of the points in mom_soa[(n+2)*4, npoints] (float64, GPU) into out[npoints]."""
    _device_f64(mom_soa, out)
    if mom_soa.dim() != 2 or out.dim() != 1 or mom_soa.shape[0] != (n + 2) * 4 or out.shape[0] != mom_soa.shape[1]:
        raise ValueError("shape mismatch: mom_soa[(n+2)*4, npoints], out[npoints]")
    _check(_lib.heget_me2_device(n, mom_soa.shape[1], mom_soa.data_ptr(), out.data_ptr(), prec,
                                 _stream(stream)), "heget_me2_device")


def me2_async(n: int, mom_soa, out, prec: int = FP32, stream=None) -> None:
    """heget_me2_async: the stream-ordered form of me2, same arguments as me2_device."""
    _device_f64(mom_soa, out)
    if mom_soa.dim() != 2 or out.dim() != 1 or mom_soa.shape[0] != (n + 2) * 4 \
            or out.shape[0] != mom_soa.shape[1]:
        raise ValueError("shape mismatch: mom_soa[(n+2)*4, npoints], out[npoints]")
    _check(_lib.heget_me2_async(n, mom_soa.shape[1], mom_soa.data_ptr(), out.data_ptr(), prec,
                                _stream(stream)), "heget_me2_async")


def gen_points_device(n: int, sqrt_s: float, mom_soa, weight, cuts=(20.0, 2.5, 0.4), seed: int = 0,
                      first: int = 0, stream=None) -> None:
    """Points first..first+npoints-1 into mom_soa[(n+2)*4, npoints] and their
    phase-space weights into weight[npoints] (float64, GPU)."""
    _device_f64(mom_soa, weight)
    if mom_soa.dim() != 2 or weight.dim() != 1 or mom_soa.shape[0] != (n + 2) * 4 or weight.shape[0] != mom_soa.shape[1]:
        raise ValueError("shape mismatch: mom_soa[(n+2)*4, npoints], weight[npoints]")
    c = _cuts(cuts)
    _check(_lib.heget_gen_points_device(n, sqrt_s, C.byref(c) if c else None, seed, first,
                                        mom_soa.shape[1], mom_soa.data_ptr(), weight.data_ptr(),
                                        _stream(stream)), "heget_gen_points_device")


# ---- misc --------------------------------------------------------------------

def set_couplings(alpha: float = 1.0 / 137.0, charge: float = 2.0 / 3.0) -> None:
    _check(_lib.heget_set_couplings(alpha, charge), "heget_set_couplings")


def timing_enable(on: bool = True) -> None:
    _check(_lib.heget_timing_enable(int(on)), "heget_timing_enable")


def timing_read(reset: bool = True):
    ms, cnt = C.c_double(), C.c_int64()
    _check(_lib.heget_timing_read(C.byref(ms), C.byref(cnt), int(reset)), "heget_timing_read")
    return ms.value, cnt.value


SHAPE_FIELDS = ("unrolled", "helicities_per_walk", "closing", "waves_per_block", "prefetch",
                "waves_per_simd", "points_per_lane", "prefix_sets")


def me2_flops(n: int, prec: int = FP32):
    """(algorithmic flops per point, shape tuple) of the kernel in use for (n, prec)."""
    f, s = C.c_double(), Shape()
    _check(_lib.heget_me2_flops(n, prec, C.byref(f), C.byref(s)), "heget_me2_flops")
    return f.value, s.as_tuple()


def autotune(n: int, prec: int = FP32, npoints: int = 1 << 18) -> dict:
    """Time every compiled kernel shape for (n, prec) and keep the fastest."""
    s, ms = Shape(), C.c_double()
    _check(_lib.heget_autotune(n, prec, npoints, C.byref(s), C.byref(ms)), "heget_autotune")
    d = dict(zip(SHAPE_FIELDS, s.as_tuple()))
    d["ms"] = ms.value
    return d


def kernel_shapes(n: int, prec: int = FP32):
    """Compiled shapes for (n, prec) as tuples (unrolled, helicities_per_walk,
    closing, waves_per_block, prefetch), the shape in use first."""
    cnt = C.c_int()
    _check(_lib.heget_kernel_shapes(n, prec, 0, None, C.byref(cnt)), "heget_kernel_shapes")
    arr = (Shape * cnt.value)()
    _check(_lib.heget_kernel_shapes(n, prec, cnt.value, arr, C.byref(cnt)), "heget_kernel_shapes")
    return [s.as_tuple() for s in arr]


def set_kernel_shape(n: int, prec: int, shape=None) -> None:
    """Force a compiled shape (tuple as from kernel_shapes); None = default."""
    if shape is None:
        _check(_lib.heget_set_kernel_shape(n, prec, None), "heget_set_kernel_shape")
    else:
        s = Shape(*shape)
        _check(_lib.heget_set_kernel_shape(n, prec, C.byref(s)), "heget_set_kernel_shape")


def shutdown() -> None:
    _lib.heget_shutdown()


def lib():
    return _lib


def valu_peak() -> dict:
    """Measured FP32 and FP64 FMA ceilings of the device (TFLOP/s)."""
    f32, f64 = C.c_double(0.0), C.c_double(0.0)
    _check(_lib.heget_valu_peak(C.byref(f32), C.byref(f64)), "heget_valu_peak")
    return {"fp32_tflops": f32.value, "fp64_tflops": f64.value}


def xsec_hist(n: int, cfg: Config, observable: int, nbins: int, lo: float, hi: float):
    """(hist[nbins + 2] = [underflow, bins on [lo, hi), overflow] in fb per bin,
    result dict) for the observable over the points of heget_xsec."""
    h = np.zeros(nbins + 2)
    r = Result()
    c = cfg.c()
    _check(_lib.heget_xsec_hist(n, C.byref(c), observable, nbins, lo, hi, _ptr(h), C.byref(r)),
           "heget_xsec_hist")
    return h, r.as_dict()


def xsec_events(n: int, cfg: Config, momenta: bool = False, rapidity: bool = False,
                helicity: bool = False) -> dict:
    """heget_xsec plus per-event records: dict(result, weight[npoints] and, if
    asked for, momenta[npoints, n+2, 4] (partonic CM frame), rapidity[npoints],
    helicity[npoints] (uint16: bit 0 quark pair, bit 1 + j photon j is +1))."""
    npts = max(int(cfg.npoints), 0)
    out = {"weight": np.zeros(npts)}
    if momenta:
        out["momenta"] = np.zeros((npts, n + 2, 4))
    if rapidity:
        out["rapidity"] = np.zeros(npts)
    if helicity:
        out["helicity"] = np.zeros(npts, dtype=np.uint16)
    r = Result()
    c = cfg.c()
    opt = lambda k: _ptr(out[k]) if k in out else None
    hp = out["helicity"].ctypes.data_as(C.POINTER(C.c_uint16)) if helicity else None
    _check(_lib.heget_xsec_events(n, C.byref(c), C.byref(r), _ptr(out["weight"]), opt("momenta"),
                                  opt("rapidity"), hp), "heget_xsec_events")
    out["result"] = r.as_dict()
    return out


# ---- the massless HELAS set (Appendix B) as a device library

HELAS_FUNCS = ["ixxxx0", "ixxxx1", "ixxxx2", "oxxxx0", "oxxxx1", "oxxxx2", "vxxxx0", "vxxxx1",
               "vxxxx2", "iovxxx", "fvixx0", "fvoxx0", "jioxx0"]


def helas_sizes(func) -> tuple:
    """(input doubles, output doubles) per record of a HELAS function."""
    f = HELAS_FUNCS.index(func) if isinstance(func, str) else int(func)
    ni, no = C.c_int(), C.c_int()
    _check(_lib.heget_helas_sizes(f, C.byref(ni), C.byref(no)), "heget_helas_sizes")
    return ni.value, no.value


def helas(func, records, prec: int = FP64) -> np.ndarray:
    """Evaluate one HELAS function on the device over records[count, in_doubles]."""
    f = HELAS_FUNCS.index(func) if isinstance(func, str) else int(func)
    ni, no = helas_sizes(f)
    x = np.ascontiguousarray(records, dtype=np.float64)
    if x.ndim != 2 or x.shape[1] != ni:
        raise ValueError(f"records must have shape [count, {ni}]")
    out = np.zeros((x.shape[0], no))
    _check(_lib.heget_helas(f, x.shape[0], _ptr(x), _ptr(out), prec), "heget_helas")
    return out


def _is_pinned(t) -> bool:
    try:
        return bool(t.is_pinned())
    except RuntimeError:  # no device runtime to ask: not pinned memory
        return False


def _device_f64(*ts) -> None:
    if any(str(t.dtype) != "torch.float64" for t in ts):
        raise TypeError("device buffers must be float64")
    for t in ts:
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("device buffers must be contiguous GPU tensors")


def helas_device(func, records, out, prec: int = FP64, stream=None) -> None:
    """Device form of helas: records[count, in_doubles] and out[count, out_doubles] on the GPU."""
    f = HELAS_FUNCS.index(func) if isinstance(func, str) else int(func)
    ni, no = helas_sizes(f)
    _device_f64(records, out)
    if records.dim() != 2 or records.shape[1] != ni or tuple(out.shape) != (records.shape[0], no):
        raise ValueError(f"shape mismatch: records[count, {ni}], out[count, {no}]")
    _check(_lib.heget_helas_device(f, records.shape[0], records.data_ptr(), out.data_ptr(), prec,
                                   _stream(stream)), "heget_helas_device")


def me2_frame(momenta, prec: int = FP64, return_status: bool = False):
    """Helicity-summed |M|^2 of u ubar -> n photons (n <= 5) at momenta[npoints, n+2, 4] in any frame."""
    p = np.ascontiguousarray(momenta, dtype=np.float64)
    if p.ndim != 3 or p.shape[2] != 4:
        raise ValueError("momenta must have shape [npoints, n+2, 4]")
    n = p.shape[1] - 2
    out = np.zeros(p.shape[0])
    st = _check(_lib.heget_me2_frame(n, p.shape[0], _ptr(p), _ptr(out), prec), "heget_me2_frame")
    return (out, st) if return_status else out


def me2_frame_device(n: int, mom_soa, out, prec: int = FP32, stream=None) -> None:
    """Device form: mom_soa[(n+2)*4, npoints] and out[npoints], float64 on the GPU."""
    _device_f64(mom_soa, out)
    if mom_soa.shape[0] != (n + 2) * 4 or out.shape[0] != mom_soa.shape[1]:
        raise ValueError("shape mismatch: mom_soa[(n+2)*4, npoints], out[npoints]")
    _check(_lib.heget_me2_frame_device(n, out.shape[0], mom_soa.data_ptr(), out.data_ptr(), prec,
                                       _stream(stream)), "heget_me2_frame_device")
