"""Python binding of the gfx950 Fourier-domain dedispersion library (libfdd.so).

Argument marshalling only: every stage of the path runs in the library's HIP kernels.  PyTorch
provides device memory (inputs, outputs, the plan workspace) and the HIP stream.  There is no
CPU fallback: if the library is missing or no GPU is present, calls fail loudly.

Low-level functions carry the C ABI names (fdd_plan, fdd_execute, fdd_power_spectrum, ...);
`Plan` wraps them for tensors.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "FDD_OK", "FDD_IN_U8_TIME_MAJOR", "FDD_IN_F32_CHAN_MAJOR", "FDD_FP32", "FDD_FP16_SPLIT",
    "FDD_BF16_SPLIT", "FDD_DELAY_EXACT", "FDD_DELAY_ROUND", "FDD_PLAN_DRY_RUN",
    "FDD_PLAN_EXTERNAL_WORKSPACE", "FDD_PLAN_POWER_ONLY", "FDD_PLAN_SCALED_DM", "FddError", "PlanDesc", "PlanGeometry", "library", "library_path",
    "exported_symbols", "fdd_plan", "fdd_plan_info", "fdd_set_workspace", "fdd_execute", "fdd_execute_noalloc",
    "fdd_power_spectrum", "fdd_power_spectrum_scaled", "fdd_tdd_execute", "fdd_destroy", "fdd_profile_enable", "fdd_profile_read",
    "fdd_dispersion_delays", "fdd_plan_delays", "fdd_plan_output_offsets", "fdd_smearing_factors",
    "fdd_plan_kernel", "fdd_plan_factors", "fdd_status_string",
    "fdd_last_error", "fdd_version", "Plan", "FDD_BATCH_NO_GRAPH", "FDD_BATCH_NO_AUTOTUNE", "FDD_BATCH_SHARE_PHASORS", "BatchDesc",
    "fdd_batch_create", "fdd_batch_execute", "fdd_batch_info", "fdd_batch_describe", "fdd_batch_destroy", "Batch",
]

FDD_OK = 0
FDD_IN_U8_TIME_MAJOR, FDD_IN_F32_CHAN_MAJOR = 0, 1
FDD_FP32, FDD_FP16_SPLIT, FDD_BF16_SPLIT = 0, 1, 2
FDD_DELAY_EXACT, FDD_DELAY_ROUND = 0, 1
FDD_PLAN_DRY_RUN, FDD_PLAN_EXTERNAL_WORKSPACE, FDD_PLAN_POWER_ONLY, FDD_PLAN_SCALED_DM = 1, 2, 4, 8
FDD_BATCH_NO_GRAPH, FDD_BATCH_NO_AUTOTUNE, FDD_BATCH_SHARE_PHASORS = 1, 2, 4

_HERE = os.path.dirname(os.path.abspath(__file__))
# FDD_LIBRARY overrides the in-tree build (e.g. to compare two builds of the library)
library_path = os.environ.get("FDD_LIBRARY") or os.path.join(_HERE, "lib", "libfdd.so")


class FddError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {fdd_status_string(status)} ({status}): {fdd_last_error()}")


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n_chan", ctypes.c_int32),
        ("chan_freq_mhz", ctypes.POINTER(ctypes.c_double)),
        ("ref_freq_mhz", ctypes.c_double),
        ("tsamp_s", ctypes.c_double),
        ("n_dm", ctypes.c_int32),
        ("dm", ctypes.POINTER(ctypes.c_double)),
        ("n_samp", ctypes.c_int64),
        ("chunk_len", ctypes.c_int64),
        ("overlap", ctypes.c_int64),
        ("single_chunk", ctypes.c_int32),
        ("input", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("delay_mode", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("downsample", ctypes.POINTER(ctypes.c_int32)),
    ]


class PlanGeometry(ctypes.Structure):
    _fields_ = [
        ("chunk_len", ctypes.c_int64),
        ("stride", ctypes.c_int64),
        ("overlap", ctypes.c_int64),
        ("n_chunks", ctypes.c_int64),
        ("n_bins", ctypes.c_int64),
        ("bins_padded", ctypes.c_int64),
        ("max_delay", ctypes.c_double),
        ("n_valid", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_size_t),
        ("out_samples", ctypes.c_int64),
        ("n_segments", ctypes.c_int32),
        ("scaled_min_bin", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchDesc(ctypes.Structure):
    _fields_ = [
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_int32),
        ("scratch_limit", ctypes.c_size_t),
        ("tune_cache", ctypes.c_char_p),
    ]


_lib = None

_SIGNATURES = {
    "fdd_plan": (ctypes.c_int, [ctypes.POINTER(PlanDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "fdd_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PlanGeometry)]),
    "fdd_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "fdd_execute": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fdd_execute_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fdd_power_spectrum": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fdd_tdd_execute": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fdd_power_spectrum_scaled": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fdd_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "fdd_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "fdd_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "fdd_dispersion_delays": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "fdd_plan_delays": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "fdd_plan_output_offsets": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "fdd_smearing_factors": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                            ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32)]),
    "fdd_plan_kernel": (ctypes.c_char_p, [ctypes.c_void_p]),
    "fdd_plan_factors": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "fdd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "fdd_last_error": (ctypes.c_char_p, []),
    "fdd_version": (ctypes.c_char_p, []),
    "fdd_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(BatchDesc),
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "fdd_batch_execute": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "fdd_batch_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(ctypes.c_size_t)]),
    "fdd_batch_describe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t,
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "fdd_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}


def library() -> ctypes.CDLL:
    """Load libfdd.so (built by paper_2110_03482_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise RuntimeError(f"{library_path} is missing: build it with `python -m paper_2110_03482_amd.build`")
        lib = ctypes.CDLL(library_path)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols() -> list:
    return sorted(_SIGNATURES)


def _check(status: int, where: str) -> None:
    if status != FDD_OK:
        raise FddError(status, where)


def _dptr(a) -> ctypes.POINTER(ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------------------------- C ABI mirrors

def fdd_status_string(status: int) -> str:
    return library().fdd_status_string(int(status)).decode()


def fdd_last_error() -> str:
    return library().fdd_last_error().decode()


def fdd_version() -> str:
    return library().fdd_version().decode()


def fdd_plan(desc: PlanDesc) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(library().fdd_plan(ctypes.byref(desc), ctypes.byref(h)), "fdd_plan")
    return h


def fdd_plan_info(plan) -> PlanGeometry:
    g = PlanGeometry()
    _check(library().fdd_plan_info(plan, ctypes.byref(g)), "fdd_plan_info")
    return g


def fdd_set_workspace(plan, ptr: int, nbytes: int) -> None:
    _check(library().fdd_set_workspace(plan, ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes)), "fdd_set_workspace")


def fdd_execute(plan, d_in: int, d_out: int, stream: int = 0) -> None:
    _check(library().fdd_execute(plan, ctypes.c_void_p(d_in), ctypes.c_void_p(d_out), ctypes.c_void_p(stream)),
           "fdd_execute")


def fdd_execute_noalloc(plan, d_in: int, d_out: int, stream: int = 0) -> None:
    _check(library().fdd_execute_noalloc(plan, ctypes.c_void_p(d_in), ctypes.c_void_p(d_out), ctypes.c_void_p(stream)),
           "fdd_execute_noalloc")


def fdd_power_spectrum(plan, d_in: int, d_out: int, stream: int = 0) -> None:
    _check(library().fdd_power_spectrum(plan, ctypes.c_void_p(d_in), ctypes.c_void_p(d_out),
                                        ctypes.c_void_p(stream)), "fdd_power_spectrum")


def fdd_power_spectrum_scaled(plan, d_in: int, d_out: int, stream: int = 0) -> None:
    _check(library().fdd_power_spectrum_scaled(plan, ctypes.c_void_p(d_in), ctypes.c_void_p(d_out),
                                               ctypes.c_void_p(stream)), "fdd_power_spectrum_scaled")


def fdd_tdd_execute(plan, d_in: int, d_out: int, stream: int = 0) -> None:
    _check(library().fdd_tdd_execute(plan, ctypes.c_void_p(d_in), ctypes.c_void_p(d_out), ctypes.c_void_p(stream)),
           "fdd_tdd_execute")


def fdd_destroy(plan) -> None:
    _check(library().fdd_destroy(plan), "fdd_destroy")


def fdd_profile_enable(plan, depth: int) -> None:
    _check(library().fdd_profile_enable(plan, int(depth)), "fdd_profile_enable")


def fdd_profile_read(plan):
    """(mean ms per stage [transpose, forward FFT, phasor sum, inverse FFT], calls averaged)."""
    ms = (ctypes.c_float * 4)()
    n = ctypes.c_int32()
    _check(library().fdd_profile_read(plan, ms, ctypes.byref(n)), "fdd_profile_read")
    return [float(v) for v in ms], int(n.value)


def fdd_dispersion_delays(freqs_mhz: Sequence[float], ref_freq_mhz: float, tsamp_s: float, dm: float) -> np.ndarray:
    f = np.ascontiguousarray(freqs_mhz, dtype=np.float64)
    out = np.empty_like(f)
    _check(library().fdd_dispersion_delays(int(f.size), _dptr(f), float(ref_freq_mhz), float(tsamp_s), float(dm),
                                           _dptr(out)), "fdd_dispersion_delays")
    return out


def fdd_plan_delays(plan, n_dm: int, n_chan: int) -> np.ndarray:
    out = np.empty((n_dm, n_chan), dtype=np.float64)
    _check(library().fdd_plan_delays(plan, _dptr(out)), "fdd_plan_delays")
    return out


def fdd_plan_output_offsets(plan, n_dm: int) -> np.ndarray:
    """Start of every output row of fdd_execute (n_dm + 1 entries, the last = out_samples)."""
    out = np.empty(n_dm + 1, dtype=np.int64)
    _check(library().fdd_plan_output_offsets(plan, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
           "fdd_plan_output_offsets")
    return out


def fdd_smearing_factors(freqs_mhz, tsamp_s: float, dms, max_factor: int) -> np.ndarray:
    """Per-DM down-sampling factors from the smearing across the lowest channel."""
    f = np.ascontiguousarray(freqs_mhz, dtype=np.float64)
    d = np.ascontiguousarray(dms, dtype=np.float64)
    out = np.empty(d.size, dtype=np.int32)
    _check(library().fdd_smearing_factors(int(f.size), _dptr(f), float(tsamp_s), int(d.size), _dptr(d),
                                          int(max_factor), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
           "fdd_smearing_factors")
    return out


def fdd_plan_kernel(plan) -> str:
    return library().fdd_plan_kernel(plan).decode()


def fdd_plan_factors(plan) -> tuple:
    """(fine, coarse, col_tiles) of the plan's DM factorisation; zeros if it is not factorised."""
    v = [ctypes.c_int32() for _ in range(3)]
    _check(library().fdd_plan_factors(plan, *[ctypes.byref(x) for x in v]), "fdd_plan_factors")
    return tuple(int(x.value) for x in v)


def fdd_batch_create(plans: Sequence, desc: BatchDesc) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * len(plans))(*[ctypes.c_void_p(p) if isinstance(p, int) else p for p in plans])
    out = ctypes.c_void_p()
    _check(library().fdd_batch_create(len(plans), arr, ctypes.byref(desc), ctypes.byref(out)), "fdd_batch_create")
    return out


def fdd_batch_execute(batch, d_in: Sequence[int], d_out: Sequence[int], stream: int = 0) -> None:
    ins = (ctypes.c_void_p * len(d_in))(*d_in)
    outs = (ctypes.c_void_p * len(d_out))(*d_out)
    _check(library().fdd_batch_execute(batch, ins, outs, ctypes.c_void_p(stream)), "fdd_batch_execute")


def fdd_batch_info(batch):
    w, sb, tb = ctypes.c_int32(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(library().fdd_batch_info(batch, ctypes.byref(w), ctypes.byref(sb), ctypes.byref(tb)), "fdd_batch_info")
    return int(w.value), int(sb.value), int(tb.value)


def fdd_batch_describe(batch) -> dict:
    import json
    need = ctypes.c_size_t()
    library().fdd_batch_describe(batch, None, 0, ctypes.byref(need))
    buf = ctypes.create_string_buffer(int(need.value))
    _check(library().fdd_batch_describe(batch, buf, int(need.value), None), "fdd_batch_describe")
    return json.loads(buf.value.decode())


def fdd_batch_destroy(batch) -> None:
    _check(library().fdd_batch_destroy(batch), "fdd_batch_destroy")


# ----------------------------------------------------------------------------- tensor wrapper

_PRECISIONS = {"fp32": FDD_FP32, "fp16_split": FDD_FP16_SPLIT, "bf16_split": FDD_BF16_SPLIT}
_MODES = {"exact": FDD_DELAY_EXACT, "round": FDD_DELAY_ROUND}
_INPUTS = {"u8": FDD_IN_U8_TIME_MAJOR, "f32": FDD_IN_F32_CHAN_MAJOR}


class Plan:
    """A dedispersion plan with a workspace allocated from torch on `device`.

    Input tensors: uint8 [n_samp][n_chan] (input="u8") or float32 [n_chan][n_samp] ("f32").
    """

    def __init__(self, freqs_mhz, ref_freq_mhz: float, tsamp_s: float, dms, n_samp: int, chunk_len: int,
                 overlap: int = 0, single_chunk: bool = False, input: str = "f32", precision: str = "fp32",
                 mode: str = "exact", device=None, dry_run: bool = False, power_only: bool = False,
                 workspace: bool = True, downsample=None, scaled_dm: bool = False):
        self._freqs = np.ascontiguousarray(freqs_mhz, dtype=np.float64)
        self._dms = np.ascontiguousarray(dms, dtype=np.float64)
        self._ds = None if downsample is None else np.ascontiguousarray(downsample, dtype=np.int32)
        self.n_chan = int(self._freqs.size)
        self.n_dm = int(self._dms.size)
        self.n_samp = int(n_samp)
        self.input = input
        self.single_chunk = bool(single_chunk)
        d = PlanDesc()
        d.n_chan = self.n_chan
        d.chan_freq_mhz = _dptr(self._freqs)
        d.ref_freq_mhz = float(ref_freq_mhz)
        d.tsamp_s = float(tsamp_s)
        d.n_dm = self.n_dm
        d.dm = _dptr(self._dms)
        d.n_samp = self.n_samp
        d.chunk_len = int(chunk_len)
        d.overlap = int(overlap)
        d.single_chunk = int(self.single_chunk)
        d.input = _INPUTS[input]
        d.precision = _PRECISIONS[precision]
        d.delay_mode = _MODES[mode]
        d.flags = ((FDD_PLAN_DRY_RUN if dry_run else FDD_PLAN_EXTERNAL_WORKSPACE) | (FDD_PLAN_POWER_ONLY if power_only else 0)
                   | (FDD_PLAN_SCALED_DM if scaled_dm else 0))
        if self._ds is not None:
            if self._ds.size != self.n_dm:
                raise ValueError("downsample needs one factor per DM")
            d.downsample = self._ds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self._handle = fdd_plan(d)
        self.geometry = fdd_plan_info(self._handle)
        self.downsampled = int(self.geometry.out_samples) != self.n_dm * self.n_samp
        self.kernel = fdd_plan_kernel(self._handle)
        self.factors = fdd_plan_factors(self._handle)
        self.workspace = None
        self.device = None
        if not dry_run:
            import torch
            if not torch.cuda.is_available():
                fdd_destroy(self._handle)
                self._handle = None
                raise RuntimeError("no GPU visible: the FDD library has no CPU path")
            self.device = torch.device("cuda") if device is None else torch.device(device)
            if workspace:   # without one the plan only describes a beam of a Batch
                self.workspace = torch.empty(int(self.geometry.workspace_bytes), dtype=torch.uint8, device=self.device)
                fdd_set_workspace(self._handle, self.workspace.data_ptr(), self.workspace.numel())

    # -- helpers
    @property
    def handle(self):
        return self._handle

    def delays(self) -> np.ndarray:
        return fdd_plan_delays(self._handle, self.n_dm, self.n_chan)

    def _check_input(self, x):
        import torch
        if self.input == "u8":
            want = (torch.uint8, (self.n_samp, self.n_chan))
        else:
            want = (torch.float32, (self.n_chan, self.n_samp))
        if x.dtype != want[0] or tuple(x.shape) != want[1] or not x.is_contiguous() or x.device.type != "cuda":
            raise ValueError(f"input must be a contiguous {want[0]} tensor of shape {want[1]} on {self.device}")

    @staticmethod
    def _stream(stream) -> int:
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        return int(s.cuda_stream)

    def output_offsets(self) -> np.ndarray:
        """Start of every DM's output row in the flat output (n_dm + 1 entries)."""
        return fdd_plan_output_offsets(self._handle, self.n_dm)

    def rows(self, out):
        """The DM rows of a flat down-sampled output, as views."""
        off = self.output_offsets()
        return [out[int(off[j]): int(off[j + 1])] for j in range(self.n_dm)]

    def execute(self, x, out=None, stream=None):
        """Dedispersed series float32 [n_dm][n_samp]; with down-sampling a flat float32
        [out_samples] holding the DM rows one after another (see rows())."""
        import torch
        self._check_input(x)
        shape = (int(self.geometry.out_samples),) if self.downsampled else (self.n_dm, self.n_samp)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        elif out.dtype != torch.float32 or tuple(out.shape) != shape or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float32 tensor of shape {shape}")
        fdd_execute(self._handle, x.data_ptr(), out.data_ptr(), self._stream(stream))
        return out

    def execute_noalloc(self, x, out, stream=None):
        """execute() with the workspace in the library's static device scratch (no device
        allocation by the call; dry-run plans accepted).  out: float32 as execute() returns."""
        import torch
        self._check_input(x)
        shape = (int(self.geometry.out_samples),) if self.downsampled else (self.n_dm, self.n_samp)
        if out.dtype != torch.float32 or tuple(out.shape) != shape or not out.is_contiguous() or out.device != x.device:
            raise ValueError(f"out must be a contiguous float32 tensor of shape {shape} on the input's device")
        fdd_execute_noalloc(self._handle, x.data_ptr(), out.data_ptr(), self._stream(stream))
        return out

    def tdd(self, x, out=None, stream=None):
        """Brute-force time-domain dedispersion with the plan's nearest-sample delays, [n_dm][n_samp]."""
        import torch
        self._check_input(x)
        if out is None:
            out = torch.empty((self.n_dm, self.n_samp), dtype=torch.float32, device=self.device)
        elif out.dtype != torch.float32 or tuple(out.shape) != (self.n_dm, self.n_samp) or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor [n_dm][n_samp]")
        fdd_tdd_execute(self._handle, x.data_ptr(), out.data_ptr(), self._stream(stream))
        return out

    def power_spectrum(self, x, out=None, stream=None):
        """Power spectra float32 [n_dm][L/2] (single-chunk plans)."""
        import torch
        self._check_input(x)
        nb = int(self.geometry.chunk_len) // 2
        if out is None:
            out = torch.empty((self.n_dm, nb), dtype=torch.float32, device=self.device)
        elif out.dtype != torch.float32 or tuple(out.shape) != (self.n_dm, nb) or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor [n_dm][L/2]")
        fdd_power_spectrum(self._handle, x.data_ptr(), out.data_ptr(), self._stream(stream))
        return out

    def power_spectrum_scaled(self, x, out=None, stream=None):
        """Power spectra float32 [n_dm][L/2] with spin-frequency-scaled DMs (approximate above
        geometry.scaled_min_bin; plans made with scaled_dm=True)."""
        import torch
        self._check_input(x)
        nb = int(self.geometry.chunk_len) // 2
        if out is None:
            out = torch.empty((self.n_dm, nb), dtype=torch.float32, device=self.device)
        elif out.dtype != torch.float32 or tuple(out.shape) != (self.n_dm, nb) or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor [n_dm][L/2]")
        fdd_power_spectrum_scaled(self._handle, x.data_ptr(), out.data_ptr(), self._stream(stream))
        return out

    def profile(self, depth: int = 1) -> None:
        """Record per-stage HIP events for the next `depth` calls (0 disables)."""
        fdd_profile_enable(self._handle, depth)

    def stage_ms(self):
        """Mean ms per call of [transpose, forward FFT, phasor sum, inverse FFT], and the call count."""
        return fdd_profile_read(self._handle)

    def close(self) -> None:
        if getattr(self, "_handle", None) is not None:
            fdd_destroy(self._handle)
            self._handle = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many plans (beams) dedispersed together by grouped launches replayed from one HIP graph.

    The plans may be made with workspace=False: the batch owns its own scratch.  The first
    execute runs the autotuner (unless autotune=False) and captures the graph; later calls
    with the same tensors replay it.
    """

    def __init__(self, plans: Sequence[Plan], graph: bool = True, autotune: bool = True, scratch_limit: int = 0,
                 tune_cache: Optional[str] = None, share_phasors: bool = False):
        self.plans = list(plans)
        d = BatchDesc()
        d.flags = ((0 if graph else FDD_BATCH_NO_GRAPH) | (0 if autotune else FDD_BATCH_NO_AUTOTUNE) |
                   (FDD_BATCH_SHARE_PHASORS if share_phasors else 0))
        d.reserved = 0
        d.scratch_limit = int(scratch_limit)
        self._cache = tune_cache.encode() if tune_cache else None
        d.tune_cache = self._cache
        self._handle = fdd_batch_create([p.handle for p in self.plans], d)
        self.n_waves, self.scratch_bytes, self.table_bytes = fdd_batch_info(self._handle)

    @property
    def handle(self):
        return self._handle

    def describe(self) -> dict:
        return fdd_batch_describe(self._handle)

    def execute(self, inputs, outputs=None, stream=None):
        """Dedisperse every beam; returns the list of float32 [n_dm][n_samp] outputs."""
        import torch
        if len(inputs) != len(self.plans):
            raise ValueError("one input per plan expected")
        for p, x in zip(self.plans, inputs):
            p._check_input(x)
        if outputs is None:
            outputs = [torch.empty((p.n_dm, p.n_samp), dtype=torch.float32, device=x.device)
                       for p, x in zip(self.plans, inputs)]
        for p, y in zip(self.plans, outputs):
            if y.dtype != torch.float32 or tuple(y.shape) != (p.n_dm, p.n_samp) or not y.is_contiguous():
                raise ValueError("outputs must be contiguous float32 tensors [n_dm][n_samp]")
        fdd_batch_execute(self._handle, [x.data_ptr() for x in inputs], [y.data_ptr() for y in outputs],
                          Plan._stream(stream))
        return outputs

    def close(self) -> None:
        if getattr(self, "_handle", None) is not None:
            fdd_batch_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
