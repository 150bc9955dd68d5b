"""Python binding of libfdas, the MI355X FDAS correlation hot path.

Argument marshalling only: every step of the search runs in the HIP kernels
behind the C ABI declared in include/fdas.h.  PyTorch supplies device memory
(tensors' data pointers) and streams (``torch.cuda.current_stream()``); the
library raises ``ImportError`` when libfdas.so has not been built -- there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "FdasError", "load", "lib_path", "CAND_DTYPE", "Bank", "Plan", "TdPlan", "Server",
    "make_templates", "autotune", "threshold", "significance", "dft_c64", "dedisperse", "pinned_candidates",
    "IN_SERIES", "IN_SPECTRUM",
    "IN_SPECTRUM_NORMALISED",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfdas.so")
_lib = None

IN_SERIES = 0
IN_SPECTRUM = 1
IN_SPECTRUM_NORMALISED = 2

_c_i32, _c_i64, _c_dbl, _c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class _Cand(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("iz", ctypes.c_int32), ("nharm", ctypes.c_int32),
                ("r", ctypes.c_double), ("z", ctypes.c_double), ("power", ctypes.c_float),
                ("sigma", ctypes.c_float)]


class _Opts(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("nharm_max", ctypes.c_int32),
                ("median_window", ctypes.c_int32), ("cand_capacity", ctypes.c_int64),
                ("templates_per_block", ctypes.c_int32), ("correlator", ctypes.c_int32),
                ("refine_levels", ctypes.c_int32), ("interbin", ctypes.c_int32),
                ("batch_launch", ctypes.c_int32)]


CAND_DTYPE = np.dtype([("k", "<i8"), ("iz", "<i4"), ("nharm", "<i4"), ("r", "<f8"), ("z", "<f8"),
                       ("power", "<f4"), ("sigma", "<f4")])
assert CAND_DTYPE.itemsize == ctypes.sizeof(_Cand) == 40

STATUS = {0: "FDAS_OK", -1: "FDAS_E_INVAL", -2: "FDAS_E_NOMEM", -3: "FDAS_E_DEVICE",
          -4: "FDAS_E_OVERFLOW", -5: "FDAS_E_BUSY", -6: "FDAS_E_TIMEOUT"}


class FdasError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Load libfdas.so (built by ``python -m paper_1511_07343_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run python -m paper_1511_07343_amd.build")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "fdas_default_opts": (None, [P(_Opts)]),
        "fdas_make_templates": (_c_i32, [_c_dbl, _c_dbl, P(_c_vp)]),
        "fdas_bank_nz": (_c_i32, [_c_vp]),
        "fdas_bank_halfwidth": (_c_i32, [_c_vp]),
        "fdas_bank_z": (_c_dbl, [_c_vp, _c_i32]),
        "fdas_bank_taps": (_c_i32, [_c_vp, _c_i32, P(_c_dbl)]),
        "fdas_bank_destroy": (None, [_c_vp]),
        "fdas_threshold": (_c_i32, [_c_dbl, _c_i32, P(_c_dbl)]),
        "fdas_significance": (_c_i32, [_c_dbl, _c_i32, P(_c_dbl)]),
        "fdas_plan": (_c_i32, [_c_vp, _c_i64, _c_i32, P(_Opts), P(_c_vp)]),
        "fdas_td_plan": (_c_i32, [_c_i64, _c_dbl, _c_i32, P(_Opts), P(_c_vp)]),
        "fdas_dedisperse": (_c_i32, [_c_vp, _c_i32, _c_i64, _c_dbl, _c_dbl, _c_dbl, P(_c_dbl), _c_i32, _c_i64,
                                     _c_vp, _c_vp]),
        "fdas_plan_nbins": (_c_i64, [_c_vp]),
        "fdas_plan_rows": (_c_i32, [_c_vp]),
        "fdas_plan_row_value": (_c_dbl, [_c_vp, _c_i32]),
        "fdas_plan_device_bytes": (_c_i64, [_c_vp]),
        "fdas_plan_destroy": (None, [_c_vp]),
        "fdas_search": (_c_i32, [_c_vp, _c_i32, _c_vp, _c_vp, P(_Cand), _c_i64, P(_c_i64), _c_vp]),
        "fdas_search_host": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, P(_Cand), _c_i64, P(_c_i64), _c_vp]),
        "fdas_search_batch": (_c_i32, [_c_vp, _c_i32, P(_c_vp), P(_c_i64), P(_Cand), P(_c_i64),
                                       P(_c_i64), _c_vp]),
        "fdas_plan_fetch_spectrum": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp]),
        "fdas_interp_power": (_c_i32, [_c_vp, _c_i64, P(_c_dbl), P(_c_dbl), P(_c_i32), P(_c_dbl), _c_vp]),
        "fdas_refine": (_c_i32, [_c_vp, _c_vp, _c_i64, _c_i32, _c_vp]),
        "fdas_refine_noalloc": (_c_i32, [_c_vp, _c_vp, _c_i64, _c_i32, _c_vp]),
        "fdas_plan_enable_timing": (_c_i32, [_c_vp, _c_i32]),
        "fdas_plan_stage_times": (_c_i32, [_c_vp, P(_c_dbl), P(_c_i64)]),
        "fdas_plan_search_counts": (_c_i32, [_c_vp, P(_c_i64)]),
        "fdas_dft_c64": (_c_i32, [_c_i32, _c_i32, _c_i64, _c_vp, _c_vp, _c_vp]),
        "fdas_autotune": (_c_i32, [_c_vp, _c_i64, P(_Opts), ctypes.c_char_p, P(_c_i32), P(_c_i32),
                                   P(_c_dbl)]),
        "fdas_server_create": (_c_i32, [_c_vp, _c_i32, P(_Opts), _c_i64, ctypes.c_size_t, _c_i32,
                                        P(_c_vp)]),
        "fdas_submit": (_c_i32, [_c_vp, _c_vp, _c_i64, ctypes.c_uint64]),
        "fdas_poll": (_c_i32, [_c_vp, P(ctypes.c_uint64), P(_Cand), _c_i64, P(_c_i64), P(_c_dbl),
                               _c_i32]),
        "fdas_server_outstanding": (_c_i64, [_c_vp]),
        "fdas_server_destroy": (None, [_c_vp]),
        "fdas_strerror": (ctypes.c_char_p, [_c_i32]),
        "fdas_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, allow=()):
    if status == 0 or status in allow:
        return status
    msg = load().fdas_last_error().decode(errors="replace")
    raise FdasError(status, msg)


def _stream_handle(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# Correlators (fdas_opts.correlator): FP32 overlap-save FFTs, or Eq. (1) as a
# matrix product with BF16 / FP16 operands and FP32 accumulation.
CORRELATORS = {"fft": 0, "bf16": 1, "f16": 2}
# fdas_search_batch launch forms (fdas_opts.batch_launch)
BATCH_LAUNCH = {"streams": 0, "persistent": 1}


def _opts(sigma=6.0, nharm_max=16, median_window=1024, cand_capacity=0, templates_per_block=0, correlator="fft",
          refine_levels=0, interbin=False, batch_launch="streams"):
    o = _Opts()
    load().fdas_default_opts(ctypes.byref(o))
    o.sigma = float(sigma)
    o.nharm_max = int(nharm_max)
    o.median_window = int(median_window)
    o.cand_capacity = int(cand_capacity)
    o.templates_per_block = int(templates_per_block)
    if correlator not in CORRELATORS:
        raise ValueError(f"correlator must be one of {sorted(CORRELATORS)}")
    o.correlator = CORRELATORS[correlator]
    o.refine_levels = int(refine_levels)
    o.interbin = int(bool(interbin))
    if batch_launch not in BATCH_LAUNCH:
        raise ValueError(f"batch_launch must be one of {sorted(BATCH_LAUNCH)}")
    o.batch_launch = BATCH_LAUNCH[batch_launch]
    return o


def _cands_to_numpy(buf, n: int) -> np.ndarray:
    return np.frombuffer(ctypes.string_at(ctypes.addressof(buf), n * 40), dtype=CAND_DTYPE).copy() \
        if n > 0 else np.zeros(0, dtype=CAND_DTYPE)


class _CandBuffer:
    """Reusable uninitialised host buffer of candidate records."""

    def __init__(self):
        self.arr = np.empty(0, dtype=CAND_DTYPE)

    def get(self, n: int) -> np.ndarray:
        if self.arr.shape[0] < n:
            self.arr = np.empty(n, dtype=CAND_DTYPE)
        return self.arr

    @staticmethod
    def ptr(a: np.ndarray):
        return ctypes.cast(ctypes.c_void_p(a.ctypes.data), ctypes.POINTER(_Cand))


def threshold(sigma: float, nharm: int) -> float:
    out = ctypes.c_double()
    _check(load().fdas_threshold(sigma, nharm, ctypes.byref(out)))
    return out.value


def significance(power: float, nharm: int) -> float:
    out = ctypes.c_double()
    _check(load().fdas_significance(power, nharm, ctypes.byref(out)))
    return out.value


class Bank:
    """Template bank (host FP64): z = -zmax + iz dz, taps q = -h..h."""

    def __init__(self, zmax: float, dz: float):
        h = ctypes.c_void_p()
        _check(load().fdas_make_templates(zmax, dz, ctypes.byref(h)))
        self._h = h
        self.zmax, self.dz = float(zmax), float(dz)

    @property
    def handle(self):
        return self._h

    @property
    def nz(self) -> int:
        return load().fdas_bank_nz(self._h)

    @property
    def h(self) -> int:
        return load().fdas_bank_halfwidth(self._h)

    def z(self, iz: int) -> float:
        return load().fdas_bank_z(self._h, iz)

    def taps(self, iz: int) -> np.ndarray:
        n = 2 * self.h + 1
        buf = (ctypes.c_double * (2 * n))()
        _check(load().fdas_bank_taps(self._h, iz, buf))
        a = np.frombuffer(buf, dtype=np.float64).copy()
        return a[0::2] + 1j * a[1::2]

    def close(self):
        if self._h:
            load().fdas_bank_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_templates(zmax: float, dz: float) -> Bank:
    return Bank(zmax, dz)


def autotune(bank: Bank, nsamp: int, cache_path: Optional[str] = None, **opts):
    """Fastest (segment length, templates per block, ms) for this bank and
    series length (see fdas_autotune)."""
    seg = ctypes.c_int32()
    tpb = ctypes.c_int32()
    ms = ctypes.c_double()
    o = _opts(**opts)
    _check(load().fdas_autotune(bank.handle, int(nsamp), ctypes.byref(o),
                                cache_path.encode() if cache_path else None, ctypes.byref(seg),
                                ctypes.byref(tpb), ctypes.byref(ms)))
    return seg.value, tpb.value, ms.value


class Plan:
    """Device-resident plan for one (bank, nsamp, seg)."""

    def __init__(self, bank: Bank, nsamp: int, seg: int, **opts):
        h = ctypes.c_void_p()
        o = _opts(**opts)
        _check(load().fdas_plan(bank.handle, int(nsamp), int(seg), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.bank = bank
        self.rows = bank.nz
        self.nsamp, self.seg = int(nsamp), int(seg)
        self.opts = o
        self._buf = _CandBuffer()
        self._staged = None

    @property
    def nbins(self) -> int:
        return load().fdas_plan_nbins(self._h)

    @property
    def plane_columns(self) -> int:
        """Columns of the plane: nbins, or 2 nbins for a half-bin plane."""
        return self.nbins * (2 if self.opts.interbin else 1)

    @property
    def device_bytes(self) -> int:
        return load().fdas_plan_device_bytes(self._h)

    def search(self, inp, kind: int = IN_SERIES, plane=None, cap: int = 1 << 22, stream=None,
               allow_overflow: bool = False, out: Optional[np.ndarray] = None):
        """Run the hot path on a device tensor; returns (candidates, n_found).

        ``out``: optional CAND_DTYPE array (e.g. from ``pinned_candidates``)
        that receives the records; the result is then a view of it.
        """
        buf = out if out is not None else self._buf.get(max(cap, 1))
        if out is not None:
            cap = min(cap, out.shape[0])
        if plane is not None and plane.numel() * plane.element_size() < 4 * self.rows * self.plane_columns:
            raise ValueError(f"plane must hold float32[{self.rows}][{self.plane_columns}]")
        n = ctypes.c_int64()
        st = load().fdas_search(self._h, kind, ctypes.c_void_p(inp.data_ptr()),
                                ctypes.c_void_p(plane.data_ptr() if plane is not None else 0),
                                _CandBuffer.ptr(buf), cap, ctypes.byref(n), _stream_handle(stream))
        _check(st, allow=(-4,) if allow_overflow else ())
        m = min(n.value, cap)
        return (buf[:m] if out is not None else buf[:m].copy()), n.value

    def search_host(self, series, next=None, plane=None, cap: int = 1 << 22, stream=None,
                    allow_overflow: bool = False, out: Optional[np.ndarray] = None):
        """Search a float32 series held in host memory (a numpy array or a CPU
        tensor, page-locked for the copy to overlap), copying it to the device
        as part of the call; ``next`` (same kinds, may be None) is the series of
        the following call, whose copy starts now and overlaps this search.
        The binding keeps ``next`` alive until that call.  Returns
        (candidates, n_found) like ``search``."""
        def ptr(a):
            if a is None:
                return 0, None
            if hasattr(a, "data_ptr"):
                if a.is_cuda or a.dtype != __import__("torch").float32 or not a.is_contiguous():
                    raise TypeError("host series must be a contiguous float32 CPU tensor or array")
                if a.numel() != self.nsamp:
                    raise ValueError(f"host series must hold {self.nsamp} samples")
                return a.data_ptr(), a
            a = np.ascontiguousarray(a, dtype=np.float32)
            if a.shape != (self.nsamp,):
                raise ValueError(f"host series must hold {self.nsamp} samples")
            return a.ctypes.data, a
        p_cur, keep_cur = ptr(series)
        p_next, keep_next = ptr(next)
        buf = out if out is not None else self._buf.get(max(cap, 1))
        if out is not None:
            cap = min(cap, out.shape[0])
        if plane is not None and plane.numel() * plane.element_size() < 4 * self.rows * self.plane_columns:
            raise ValueError(f"plane must hold float32[{self.rows}][{self.plane_columns}]")
        n = ctypes.c_int64()
        st = load().fdas_search_host(self._h, ctypes.c_void_p(p_cur), ctypes.c_void_p(p_next),
                                     ctypes.c_void_p(plane.data_ptr() if plane is not None else 0),
                                     _CandBuffer.ptr(buf), cap, ctypes.byref(n), _stream_handle(stream))
        self._staged = keep_next  # its copy is in flight until the next call
        del keep_cur
        _check(st, allow=(-4,) if allow_overflow else ())
        m = min(n.value, cap)
        return (buf[:m] if out is not None else buf[:m].copy()), n.value

    def search_batch(self, series: Sequence, caps: Optional[Sequence[int]] = None, stream=None,
                     out: Optional[np.ndarray] = None):
        """Several device float32 series; returns a list of candidate arrays
        (views of ``out`` when given, which must hold sum(caps) records)."""
        k = len(series)
        caps = list(caps) if caps is not None else [1 << 20] * k
        ptrs = (ctypes.c_void_p * k)(*[s.data_ptr() for s in series])
        ns = (ctypes.c_int64 * k)(*[int(s.numel()) for s in series])
        cp = (ctypes.c_int64 * k)(*caps)
        nc = (ctypes.c_int64 * k)()
        if out is not None and out.shape[0] < sum(caps):
            raise ValueError("out holds fewer records than sum(caps)")
        buf = out if out is not None else self._buf.get(max(1, sum(caps)))
        _check(load().fdas_search_batch(self._h, k, ptrs, ns, _CandBuffer.ptr(buf), cp, nc,
                                        _stream_handle(stream)))
        res, off = [], 0
        for i in range(k):
            v = buf[off: off + min(nc[i], caps[i])]
            res.append(v if out is not None else v.copy())
            off += caps[i]
        return res

    def fetch_spectrum(self, spectrum=None, medians=None, stream=None):
        _check(load().fdas_plan_fetch_spectrum(
            self._h, ctypes.c_void_p(spectrum.data_ptr() if spectrum is not None else 0),
            ctypes.c_void_p(medians.data_ptr() if medians is not None else 0), _stream_handle(stream)))

    def interp_power(self, r, z, nharm, stream=None) -> np.ndarray:
        """Fourier-interpolated harmonic sums S(r, z) (FP64) with nharm
        harmonics on the normalised spectrum of the last search."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        nh = np.ascontiguousarray(np.broadcast_to(np.asarray(nharm, dtype=np.int32), r.shape))
        if z.shape != r.shape:
            raise ValueError("r and z must have the same shape")
        out = np.empty(r.shape, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(load().fdas_interp_power(
            self._h, r.size, r.ctypes.data_as(dp), z.ctypes.data_as(dp),
            nh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), out.ctypes.data_as(dp), _stream_handle(stream)))
        return out

    def refine(self, cands: np.ndarray, levels: int = 6, stream=None) -> np.ndarray:
        """Refined copies of the given candidate records (on the last search's
        spectrum)."""
        out = np.ascontiguousarray(cands, dtype=CAND_DTYPE).copy()
        _check(load().fdas_refine(self._h, ctypes.c_void_p(out.ctypes.data if out.size else 0), out.size,
                                  int(levels), _stream_handle(stream)))
        return out

    REFINE_NOALLOC_MAX = 16384  # FDAS_REFINE_NOALLOC_MAX

    def refine_noalloc(self, cands: np.ndarray, levels: int = 6, stream=None) -> np.ndarray:
        """``refine`` through the allocation-free entry point (records staged in
        the library's fixed device array; at most REFINE_NOALLOC_MAX)."""
        out = np.ascontiguousarray(cands, dtype=CAND_DTYPE).copy()
        _check(load().fdas_refine_noalloc(self._h, ctypes.c_void_p(out.ctypes.data if out.size else 0), out.size,
                                          int(levels), _stream_handle(stream)))
        return out

    STAGES = ("r2c", "unpack_median", "segment_dft", "correlate", "harmonic_sum", "refine")

    def enable_timing(self, enable: bool = True):
        _check(load().fdas_plan_enable_timing(self._h, int(enable)))

    def stage_times(self):
        """(dict stage -> total ms, number of timed searches)."""
        ms = (ctypes.c_double * len(self.STAGES))()
        n = ctypes.c_int64()
        _check(load().fdas_plan_stage_times(self._h, ms, ctypes.byref(n)))
        return dict(zip(self.STAGES, list(ms))), n.value

    def search_counts(self):
        """(candidates, cells passed by the harmonic-sum screen, their
        16-column groups) of the last search."""
        out = (ctypes.c_int64 * 3)()
        _check(load().fdas_plan_search_counts(self._h, out))
        return tuple(out)

    def close(self):
        if self._h:
            load().fdas_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



class TdPlan(Plan):
    """Time-domain resampling search over nalpha acceleration trials
    alpha_i = -alpha_max + i 2 alpha_max / (nalpha - 1); ``search`` takes a
    float32 series and fills a float32[nalpha][nbins] plane."""

    def __init__(self, nsamp: int, alpha_max: float, nalpha: int, **opts):
        h = ctypes.c_void_p()
        o = _opts(**opts)
        _check(load().fdas_td_plan(int(nsamp), float(alpha_max), int(nalpha), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.bank = None
        self.rows = int(nalpha)
        self.nsamp, self.seg = int(nsamp), 0
        self.alpha_max = float(alpha_max)
        self.opts = o
        self._buf = _CandBuffer()
        self._staged = None

    @property
    def alphas(self) -> np.ndarray:
        """The acceleration trial of every plane row, as the library defines them."""
        lib = load()
        return np.array([lib.fdas_plan_row_value(self._h, i) for i in range(lib.fdas_plan_rows(self._h))],
                        dtype=np.float64)


class Server:
    """Continuous-batching request loop (host series in, candidates out)."""

    def __init__(self, bank: Bank, seg: int, max_nsamp: int, hbm_budget: int = 0, max_slots: int = 4,
                 **opts):
        h = ctypes.c_void_p()
        o = _opts(**opts)
        _check(load().fdas_server_create(bank.handle, int(seg), ctypes.byref(o), int(max_nsamp),
                                         int(hbm_budget), int(max_slots), ctypes.byref(h)))
        self._h = h
        self.bank = bank
        self._buf = _CandBuffer()

    def submit(self, series: np.ndarray, tag: int):
        x = np.ascontiguousarray(series, dtype=np.float32)
        _check(load().fdas_submit(self._h, ctypes.c_void_p(x.ctypes.data), x.shape[0], int(tag)))

    def poll(self, timeout_ms: int = -1, cap: int = 1 << 22):
        """Returns (tag, candidates, n_found, latency_s), or None on timeout."""
        tag = ctypes.c_uint64()
        n = ctypes.c_int64()
        lat = ctypes.c_double()
        buf = self._buf.get(max(cap, 1))
        st = load().fdas_poll(self._h, ctypes.byref(tag), _CandBuffer.ptr(buf), cap, ctypes.byref(n),
                              ctypes.byref(lat), int(timeout_ms))
        if st == -6:
            return None
        _check(st)
        return tag.value, buf[:min(n.value, cap)].copy(), n.value, lat.value

    @property
    def outstanding(self) -> int:
        return load().fdas_server_outstanding(self._h)

    def close(self):
        if self._h:
            load().fdas_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _PinnedArray(np.ndarray):
    """ndarray that keeps the torch tensor owning its page-locked memory alive."""

    owner = None


def pinned_candidates(n: int):
    """A CAND_DTYPE array of n records in page-locked host memory (torch
    allocates it), for fast device-to-host candidate copies."""
    import torch
    t = torch.empty(n * CAND_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True)
    arr = t.numpy().view(CAND_DTYPE).view(_PinnedArray)
    arr.owner = t
    return arr


def dft_c64(x, inverse: bool = False, out=None, stream=None):
    """Batched unnormalised complex DFT along the last axis (length 2^6..2^13)."""
    import torch
    if x.dtype != torch.complex64 or not x.is_cuda:
        raise TypeError("dft_c64 needs a complex64 CUDA tensor")
    n = x.shape[-1]
    log2n = int(n).bit_length() - 1
    x = x.contiguous()
    if out is None:
        out = torch.empty_like(x)
    batch = x.numel() // n
    _check(load().fdas_dft_c64(log2n, int(inverse), batch, ctypes.c_void_p(x.data_ptr()),
                               ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def dedisperse(fil, f_top: float, foff: float, tsamp: float, dms, nout: int, out=None, stream=None):
    """De-disperse a channel-major uint8 CUDA filterbank (nchan x nsamp, channel
    c at f_top - c foff MHz) for each DM: float32 CUDA tensor [ndm, nout]."""
    import torch
    if fil.dtype != torch.uint8 or not fil.is_cuda or fil.dim() != 2:
        raise TypeError("dedisperse needs a 2-d uint8 CUDA tensor (channels x samples)")
    fil = fil.contiguous()
    dms = np.ascontiguousarray(dms, dtype=np.float64)
    if out is None:
        out = torch.empty((dms.size, int(nout)), dtype=torch.float32, device=fil.device)
    elif out.dtype != torch.float32 or out.numel() < dms.size * int(nout) or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of ndm x nout")
    _check(load().fdas_dedisperse(ctypes.c_void_p(fil.data_ptr()), fil.shape[0], fil.shape[1], float(f_top),
                                  float(foff), float(tsamp), dms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  dms.size, int(nout), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out
