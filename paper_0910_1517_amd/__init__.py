"""Python binding of libcorr, the MI355X (gfx950) FX correlator of
Roy et al., "A real-time software backend for the GMRT" (arXiv:0910.1517).

This module only marshals arguments into the C ABI declared in
``include/corr.h``: every step of the correlator runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.  There is no fallback:
if ``libcorr.so`` is missing the import of the handle raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcorr.so")

FP32, INT8, FP8_E4M3 = 0, 1, 2
SCALE_HOLD, SCALE_COMPUTE = 0, 1
DUMP, RESET = 1, 2
BEAM_INTENSITY, BEAM_FULLPOL, BEAM_VOLTAGE = 0, 1, 2  # coherent beam products (corr_beamform)
MAX_BEAMS = 4
MAX_INT8_SPECTRA = 66572

STATUS = {
    0: "OK", -1: "INVALID", -2: "NULL", -3: "ALIGN", -4: "UNSUPPORTED", -5: "WORKSPACE",
    -6: "OVERFLOW", -7: "DEVICE", -8: "NOMEM", -9: "STATE", -10: "DEVICE_ARG", -11: "IO",
}
CNN_PARAMS = 2625
TILE_SPECTRA, TILE_CHANNELS = 64, 256

# corr_geom_t: {int32 D; float frac; double psi0; double rate} (24 bytes)
GEOM_DTYPE = np.dtype([("D", "<i4"), ("frac", "<f4"), ("psi0", "<f8"), ("rate", "<f8")])
assert GEOM_DTYPE.itemsize == 24


class CorrDesc(ctypes.Structure):
    _fields_ = [
        ("n_signals", ctypes.c_int32),
        ("fft_len", ctypes.c_int32),
        ("n_spectra", ctypes.c_int64),
        ("max_delay", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("sideband", ctypes.c_int32),
        ("scale_mode", ctypes.c_int32),
        ("sample_rate", ctypes.c_double),
        ("nu_bb", ctypes.c_double),
        ("x_split", ctypes.c_int32),
        ("phase_lut", ctypes.c_int32),
        ("power_fp16", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 5),
    ]


class CorrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


_lib = None

# Exported symbols of include/corr.h (checked by the tests).
SYMBOLS = [
    "corr_plan_create", "corr_plan_destroy", "corr_plan_workspace_bytes", "corr_plan_spectra_bytes",
    "corr_plan_acc_bytes", "corr_plan_state_bytes", "corr_plan_vis_bytes", "corr_plan_x_splits",
    "corr_plan_bind_workspace", "corr_fengine", "corr_xpack", "corr_xengine", "corr_integrate",
    "corr_check_device_errors", "corr_status_string", "corr_last_error",
    "corr_mad_flag", "corr_apply_flags", "corr_pair_counts", "corr_plan_power_bytes",
    "corr_plan_flags_bytes", "corr_plan_keep_bytes", "corr_beamform",
    "corr_batch_create", "corr_batch_destroy", "corr_batch_plan", "corr_batch_set_io", "corr_batch_run",
    "corr_batch_capture", "corr_batch_launch", "corr_batch_last_error",
    "corr_autotune_scratch_bytes", "corr_autotune_x_split",
    "corr_cnn_create", "corr_cnn_destroy", "corr_cnn_workspace_bytes", "corr_cnn_bind_workspace",
    "corr_cnn_forward", "corr_cnn_loss_grad", "corr_cnn_adam", "corr_cnn_train_step",
    "corr_cnn_check_device_errors", "corr_cnn_infer", "corr_cnn_infer_f16", "corr_cnn_infer_guarded", "corr_cnn_save", "corr_cnn_load", "corr_cnn_last_error",
    "corr_blank_voltages", "corr_blank_noise_table", "corr_blank_last_error",
    "corr_adc_unpack", "corr_adc_last_error", "corr_xengine_gated", "corr_pulsar_gates",
    "corr_dedisperse", "corr_dedisperse_workspace_bytes", "corr_dedisperse_last_error",
    "corr_geom_from_model", "corr_dedisperse_noalloc", "corr_plan_fengine_kernel", "corr_requantize", "corr_fix16_spectra", "corr_fix16_xengine",
]


class CnnDesc(ctypes.Structure):
    _fields_ = [("max_tiles", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("reserved", ctypes.c_int32 * 7)]


class BatchIO(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("row_stride", ctypes.c_int64), ("geom", ctypes.c_void_p),
                ("spectrum0", ctypes.c_int64), ("spec", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("acc", ctypes.c_void_p), ("state", ctypes.c_void_p), ("vis", ctypes.c_void_p),
                ("flags", ctypes.c_uint32)]


def lib():
    """Load libcorr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcorr.so not built: run `python -m paper_0910_1517_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, st, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    L.corr_plan_create.argtypes = [ctypes.POINTER(CorrDesc), ctypes.POINTER(P)]
    L.corr_plan_create.restype = st
    L.corr_plan_destroy.argtypes = [P]
    L.corr_plan_destroy.restype = None
    for n in ("workspace", "spectra", "acc", "state", "vis", "power", "flags", "keep"):
        f = getattr(L, "corr_plan_%s_bytes" % n)
        f.argtypes = [P]
        f.restype = sz
    L.corr_plan_x_splits.argtypes = [P]
    L.corr_plan_x_splits.restype = ctypes.c_int32
    L.corr_plan_fengine_kernel.argtypes = [P]
    L.corr_plan_fengine_kernel.restype = ctypes.c_char_p
    L.corr_requantize.argtypes = [P, P, P, P, P]
    L.corr_requantize.restype = st
    L.corr_plan_bind_workspace.argtypes = [P, P, sz, P]
    L.corr_plan_bind_workspace.restype = st
    L.corr_fengine.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int64, P, P, P, P]
    L.corr_mad_flag.argtypes = [P, P, ctypes.c_float, P, P]
    L.corr_mad_flag.restype = st
    L.corr_apply_flags.argtypes = [P, P, P, P, P]
    L.corr_apply_flags.restype = st
    L.corr_pair_counts.argtypes = [P, P, P, P]
    L.corr_pair_counts.restype = st
    L.corr_fengine.restype = st
    L.corr_xpack.argtypes = [P, P, P, P]
    L.corr_xpack.restype = st
    L.corr_xengine.argtypes = [P, P, P, P, P, P]
    L.corr_xengine.restype = st
    L.corr_beamform.argtypes = [P, P, P, P, P, P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, P]
    L.corr_beamform.restype = st
    L.corr_integrate.argtypes = [P, P, P, P, P, ctypes.c_uint32, P]
    L.corr_integrate.restype = st
    L.corr_check_device_errors.argtypes = [P, P]
    L.corr_check_device_errors.restype = st
    L.corr_batch_create.argtypes = [ctypes.POINTER(CorrDesc), ctypes.c_int, ctypes.POINTER(P)]
    L.corr_batch_create.restype = st
    L.corr_batch_destroy.argtypes = [P]
    L.corr_batch_destroy.restype = None
    L.corr_batch_plan.argtypes = [P, ctypes.c_int]
    L.corr_batch_plan.restype = P
    L.corr_batch_set_io.argtypes = [P, ctypes.c_int, ctypes.POINTER(BatchIO)]
    L.corr_batch_set_io.restype = st
    for n in ("run", "capture", "launch"):
        f = getattr(L, "corr_batch_" + n)
        f.argtypes = [P, P]
        f.restype = st
    L.corr_batch_last_error.argtypes = [P]
    L.corr_batch_last_error.restype = ctypes.c_char_p
    L.corr_autotune_scratch_bytes.argtypes = [ctypes.POINTER(CorrDesc)]
    L.corr_autotune_scratch_bytes.restype = sz
    L.corr_autotune_x_split.argtypes = [ctypes.POINTER(CorrDesc), P, sz, P, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_float)]
    L.corr_autotune_x_split.restype = st
    i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.corr_cnn_create.argtypes = [ctypes.POINTER(CnnDesc), ctypes.POINTER(P)]
    L.corr_cnn_destroy.argtypes = [P]
    L.corr_cnn_destroy.restype = None
    L.corr_cnn_workspace_bytes.argtypes = [P]
    L.corr_cnn_workspace_bytes.restype = sz
    L.corr_cnn_bind_workspace.argtypes = [P, P, sz]
    L.corr_cnn_forward.argtypes = [P, P, P, i32, i64, i32, P, i32, P, P]
    L.corr_cnn_loss_grad.argtypes = [P, P, P, P, i32, i64, i32, P, i32, P, P, P]
    L.corr_cnn_adam.argtypes = [P, P, P, P, P, i64, P]
    L.corr_cnn_train_step.argtypes = [P, P, P, P, i64, P, P, i32, i64, i32, P, i32, P, P]
    L.corr_cnn_check_device_errors.argtypes = [P, P]
    L.corr_cnn_infer.argtypes = [P, P, i32, i64, i32, f32, P, P, P]
    L.corr_cnn_infer_f16.argtypes = [P, P, i32, i64, i32, f32, P, P, P]
    L.corr_cnn_infer_f16.restype = ctypes.c_int32
    L.corr_cnn_infer_guarded.argtypes = [P, P, i32, i32, i64, i32, f32, f32, P, P, P]
    L.corr_cnn_infer_guarded.restype = ctypes.c_int32
    L.corr_cnn_save.argtypes = [ctypes.c_char_p, P, P, P, i64]
    L.corr_cnn_load.argtypes = [ctypes.c_char_p, P, P, P, ctypes.POINTER(i64)]
    for n in ("create", "bind_workspace", "forward", "loss_grad", "adam", "train_step", "check_device_errors",
              "infer", "save", "load"):
        getattr(L, "corr_cnn_" + n).restype = st
    L.corr_cnn_last_error.argtypes = [P]
    L.corr_cnn_last_error.restype = ctypes.c_char_p
    L.corr_blank_voltages.argtypes = [P, i64, i32, i64, i32, f32, P, i64, i64, P, P, P, P]
    L.corr_blank_voltages.restype = st
    L.corr_blank_noise_table.argtypes = [ctypes.c_uint64, i32, i64, P, P]
    L.corr_blank_noise_table.restype = st
    L.corr_blank_last_error.argtypes = []
    L.corr_blank_last_error.restype = ctypes.c_char_p
    L.corr_xengine_gated.argtypes = [P, P, P, i32, P, P]
    L.corr_xengine_gated.restype = st
    L.corr_pulsar_gates.argtypes = [i64, i64, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, i32, P, P]
    L.corr_pulsar_gates.restype = st
    L.corr_dedisperse.argtypes = [P, i32, i64, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, i32, P, P, P]
    L.corr_dedisperse.restype = st
    L.corr_dedisperse_noalloc.argtypes = [P, i32, i64, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, i32,
                                          P, P]
    L.corr_dedisperse_noalloc.restype = st
    L.corr_fix16_spectra.argtypes = [P, P, P, i64, P, P, P, P]
    L.corr_fix16_spectra.restype = st
    L.corr_fix16_xengine.argtypes = [P, P, P, P, P, P]
    L.corr_fix16_xengine.restype = st
    L.corr_dedisperse_workspace_bytes.argtypes = [i32, i64, i32]
    L.corr_dedisperse_workspace_bytes.restype = ctypes.c_size_t
    L.corr_dedisperse_last_error.argtypes = []
    L.corr_dedisperse_last_error.restype = ctypes.c_char_p
    L.corr_adc_unpack.argtypes = [P, i64, i32, i64, i32, P, i64, P]
    L.corr_adc_unpack.restype = st
    L.corr_adc_last_error.argtypes = []
    L.corr_adc_last_error.restype = ctypes.c_char_p
    dbl = ctypes.c_double
    L.corr_geom_from_model.argtypes = [i32, P, P, dbl, dbl, dbl, dbl, i32, P]
    L.corr_geom_from_model.restype = st
    L.corr_status_string.argtypes = [st]
    L.corr_status_string.restype = ctypes.c_char_p
    L.corr_last_error.argtypes = [P]
    L.corr_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _avail(t, rows: bool = False) -> int:
    """Bytes a call may use from t.data_ptr(): the tensor's own extent (a 2-D
    array of rows: up to the last row's end rounded to a 16-byte chunk),
    never past the end of its storage."""
    el = t.element_size()
    store = t.untyped_storage().nbytes() - t.storage_offset() * el
    if rows and t.dim() == 2 and t.shape[0] > 0:
        view = (t.shape[0] - 1) * t.stride(0) * el + (t.shape[1] * el + 15) // 16 * 16
    else:
        view = t.numel() * el
    return min(store, view)


def _need(t, name: str, nbytes: int, dtype=None, *, optional: bool = False, rows: bool = False):
    """Check a caller buffer before its raw pointer crosses the C-ABI (which
    cannot see sizes): a device tensor, of dtype when given (a dtype or a
    tuple of them), dense -- contiguous, or with rows=True a 2-D array of rows
    with unit stride along a row (or a contiguous flat buffer that the call's
    row stride divides into rows) -- and with at least nbytes addressable
    from its data pointer.  None passes when optional."""
    if t is None:
        if optional:
            return
        raise ValueError("%s is required" % name)
    if not getattr(t, "is_cuda", False):
        raise ValueError("%s must be a device tensor" % name)
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if rows and t.dim() == 2:
        if t.shape[1] > 1 and t.stride(1) != 1:
            raise ValueError("%s must be a 2-D array of rows with unit stride along a row" % name)
    elif rows and t.dim() != 1:
        raise ValueError("%s must be a 2-D array of rows or a flat buffer" % name)
    elif not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    have = _avail(t, rows)
    if have < nbytes:
        raise ValueError("%s holds %d bytes, needs %d" % (name, have, nbytes))


def _rows_bytes(n_rows: int, row_stride: int, row_len: int, elsize: int = 1) -> int:
    """Bytes from the first row's start to the end of the last row's row_len
    elements, rounded up to whole 16-byte chunks (the kernels read whole
    chunks)."""
    if n_rows <= 0:
        return 0
    return ((n_rows - 1) * row_stride * elsize + row_len * elsize + 15) // 16 * 16


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_desc(n_signals, fft_len, n_spectra, *, max_delay=16, precision=FP32, sideband=1,
              scale_mode=SCALE_HOLD, sample_rate=66.666666e6, nu_bb=0.0, x_split=0, phase_lut=0,
              power_fp16=0) -> CorrDesc:
    d = CorrDesc()
    d.n_signals, d.fft_len, d.n_spectra = n_signals, fft_len, n_spectra
    d.max_delay, d.precision, d.sideband, d.scale_mode = max_delay, precision, sideband, scale_mode
    d.sample_rate, d.nu_bb, d.x_split, d.phase_lut = sample_rate, nu_bb, x_split, phase_lut
    d.power_fp16 = power_fp16
    return d


class Plan:
    """A correlator plan (corr_plan_t) with its workspace bound to device memory."""

    def __init__(self, n_signals: int, fft_len: int, n_spectra: int, *, max_delay: int = 16,
                 precision: int = FP32, sideband: int = 1, scale_mode: int = SCALE_HOLD,
                 sample_rate: float = 66.666666e6, nu_bb: float = 0.0, x_split: int = 0, phase_lut: int = 0,
                 power_fp16: int = 0, device=None, bind: bool = True, _handle=None):
        L = lib()
        self.desc = make_desc(n_signals, fft_len, n_spectra, max_delay=max_delay, precision=precision,
                              sideband=sideband, scale_mode=scale_mode, sample_rate=sample_rate,
                              nu_bb=nu_bb, x_split=x_split, phase_lut=phase_lut, power_fp16=power_fp16)
        self._owned = _handle is None
        if _handle is None:
            h = ctypes.c_void_p()
            rc = L.corr_plan_create(ctypes.byref(self.desc), ctypes.byref(h))
            if rc != 0:
                raise CorrError(rc, L.corr_last_error(None).decode())
        else:
            h = ctypes.c_void_p(_handle)
        self._h = h
        self.S, self.N, self.T = n_signals, fft_len, n_spectra
        self.C = fft_len // 2
        self.P = n_signals * (n_signals + 1) // 2
        self.precision = precision
        self.power_fp16 = power_fp16
        self.max_delay = max_delay
        self.workspace = None
        if bind:
            self.bind(device)

    # ---------------------------------------------------------------- sizes
    @property
    def handle(self):
        return self._h

    def _size(self, n):
        return int(getattr(lib(), "corr_plan_%s_bytes" % n)(self._h))

    workspace_bytes = property(lambda self: self._size("workspace"))
    spectra_bytes = property(lambda self: self._size("spectra"))
    acc_bytes = property(lambda self: self._size("acc"))
    state_bytes = property(lambda self: self._size("state"))
    vis_bytes = property(lambda self: self._size("vis"))
    splits = property(lambda self: int(lib().corr_plan_x_splits(self._h)))
    # the F-engine kernel corr_fengine launches for this plan (as a profiler names it)
    fengine_kernel = property(lambda self: lib().corr_plan_fengine_kernel(self._h).decode())

    def _check(self, rc):
        if rc != 0:
            raise CorrError(rc, lib().corr_last_error(self._h).decode())

    # ------------------------------------------------------------- buffers
    def bind(self, device=None):
        import torch
        dev = torch.device(device or "cuda")
        self.workspace = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=dev)
        self._check(lib().corr_plan_bind_workspace(self._h, _ptr(self.workspace), self.workspace.numel(),
                                                   _stream(None)))

    def alloc(self, what: str, device=None, zero: bool = True):
        """Caller-owned device buffer of the right size: spectra | acc | state | vis."""
        import torch
        n = self._size(what)
        dt = {"spectra": torch.uint8, "acc": torch.int32 if self.precision == INT8 else torch.float32,
              "state": torch.float64, "vis": torch.float32,
              "power": torch.float16 if self.power_fp16 else torch.float32,
              "flags": torch.uint8, "keep": torch.int32}[what]
        el = torch.tensor([], dtype=dt).element_size()
        f = torch.zeros if zero else torch.empty
        return f(n // el, dtype=dt, device=device or "cuda")

    # ---------------------------------------------------------------- calls
    def fengine(self, x, geom, spec, scale=None, *, power=None, row_stride=None, spectrum0=0, stream=None):
        """x: int8 device tensor [S][row_stride]; geom: uint8 device tensor holding corr_geom_t[S]."""
        import torch
        rs = x.stride(0) if row_stride is None else row_stride
        _need(x, "x", _rows_bytes(self.S, rs, self.T * self.N + self.max_delay), (torch.int8, torch.uint8),
              rows=True)
        _need(geom, "geom", 24 * self.S)
        _need(spec, "spec", self.spectra_bytes)
        _need(scale, "scale", 4 * self.S * self.C, torch.float32, optional=self.precision == FP32)
        _need(power, "power", self._size("power"), torch.float16 if self.power_fp16 else torch.float32,
              optional=True)
        self._check(lib().corr_fengine(self._h, _ptr(x), rs, _ptr(geom), spectrum0, _ptr(spec),
                                       _ptr(scale), _ptr(power), _stream(stream)))

    def mad_flag(self, power, flags, M=3.0, stream=None):
        import torch
        _need(power, "power", self._size("power"), torch.float16 if self.power_fp16 else torch.float32)
        _need(flags, "flags", self._size("flags"), torch.uint8)
        self._check(lib().corr_mad_flag(self._h, _ptr(power), M, _ptr(flags), _stream(stream)))

    def apply_flags(self, flags, spec, keep=None, stream=None):
        """corr_apply_flags; spec None: write the keep words only (for
        xengine(..., keep=...))."""
        _need(flags, "flags", self._size("flags"))
        _need(spec, "spec", self.spectra_bytes, optional=keep is not None)
        _need(keep, "keep", self._size("keep"), optional=True)
        self._check(lib().corr_apply_flags(self._h, _ptr(flags), _ptr(spec), _ptr(keep), _stream(stream)))

    def pair_counts(self, keep, counts, stream=None):
        import torch
        _need(keep, "keep", self._size("keep"))
        _need(counts, "counts", 4 * self.C * self.P, torch.int32)
        self._check(lib().corr_pair_counts(self._h, _ptr(keep), _ptr(counts), _stream(stream)))

    def xpack(self, inp, spec, stream=None):
        _need(inp, "inp", self.S * self.T * self.C * 2 * (4 if self.precision == FP32 else 1))
        _need(spec, "spec", self.spectra_bytes)
        self._check(lib().corr_xpack(self._h, _ptr(inp), _ptr(spec), _stream(stream)))

    def requantize(self, inp, scale, out, stream=None):
        """corr_requantize: FP32 spectra [S][T][C][2] -> this plan's codes [S][T][C][2]
        (int8, or e4m3 bytes as uint8) with the F-engine's encoders."""
        import torch
        n = self.S * self.T * self.C * 2
        _need(inp, "inp", 4 * n, torch.float32)
        _need(scale, "scale", 4 * self.S * self.C, torch.float32)
        _need(out, "out", n, (torch.int8, torch.uint8))
        self._check(lib().corr_requantize(self._h, _ptr(inp), _ptr(scale), _ptr(out), _stream(stream)))

    def xengine(self, spec, acc, keep=None, counts=None, stream=None):
        """corr_xengine; keep: keep words [C/8][T/32][S][8] (uint32 or int32) whose
        cleared bits are zeroed inside the X-engine, counts: int32 [C][P]
        += the per-pair unflagged counts (needs keep)."""
        import torch
        _need(spec, "spec", self.spectra_bytes)
        _need(acc, "acc", self.acc_bytes)
        _need(keep, "keep", self._size("keep"), optional=True)
        _need(counts, "counts", 4 * self.C * self.P, torch.int32, optional=True)
        self._check(lib().corr_xengine(self._h, _ptr(spec), _ptr(keep), _ptr(acc), _ptr(counts), _stream(stream)))

    def xengine_gated(self, spec, gate, n_bins, acc, stream=None):
        """Gated X-engine: acc holds n_bins accumulators of acc_bytes each;
        gate is a uint8 device tensor [T]; see corr_xengine_gated."""
        import torch
        _need(spec, "spec", self.spectra_bytes)
        _need(gate, "gate", self.T, torch.uint8)
        _need(acc, "acc", max(int(n_bins), 0) * self.acc_bytes)
        self._check(lib().corr_xengine_gated(self._h, _ptr(spec), _ptr(gate), n_bins, _ptr(acc), _stream(stream)))

    def beamform(self, spec, scale=None, w=None, inc=None, c=None, coh=None, mode=None, tint=1, stream=None):
        """Incoherent beam (w [S] float -> inc [2][T/tint][C]) and coherent beams
        (c [n_beams][S][2] float as (re, im) -> coh [n_beams][planes][T/tint][C],
        complex64 [n_beams][2][T][C] for BEAM_VOLTAGE); see corr_beamform."""
        import torch
        n_beams = 0 if c is None else int(c.shape[0])
        mode = BEAM_FULLPOL if mode is None else mode
        tt = self.T // max(int(tint), 1)
        _need(spec, "spec", self.spectra_bytes)
        _need(scale, "scale", 4 * self.S * self.C, torch.float32, optional=self.precision == FP32)
        _need(inc, "inc", 4 * 2 * tt * self.C, torch.float32, optional=True)
        _need(w, "w", 4 * self.S, torch.float32, optional=inc is None)
        if n_beams:
            _need(c, "c", 4 * 2 * n_beams * self.S, torch.float32)
            per = {BEAM_INTENSITY: 2 * 4 * tt, BEAM_FULLPOL: 4 * 4 * tt, BEAM_VOLTAGE: 2 * 8 * self.T}.get(mode, 0)
            _need(coh, "coh", n_beams * per * self.C, (torch.float32, torch.complex64))
        self._check(lib().corr_beamform(self._h, _ptr(spec), _ptr(scale), _ptr(w), _ptr(inc), _ptr(c), n_beams,
                                        mode, _ptr(coh), tint, _stream(stream)))

    def fix16_spectra(self, spec, geom, scale, y16, q16=None, spectrum0=0, stream=None):
        """corr_fix16_spectra: 16-bit fixed-point spectra (int16 [S][T][C][2]) from the
        unrotated FP32 spectra of this FP32 plan."""
        import torch
        n = 4 * self.S * self.T * self.C
        _need(spec, "spec", self.spectra_bytes)
        _need(geom, "geom", 24 * self.S)
        _need(scale, "scale", 4 * self.S * self.C, torch.float32)
        _need(y16, "y16", n, torch.int16)
        _need(q16, "q16", n, torch.int16, optional=True)
        self._check(lib().corr_fix16_spectra(self._h, _ptr(spec), _ptr(geom), spectrum0, _ptr(scale), _ptr(q16),
                                             _ptr(y16), _stream(stream)))

    def fix16_xengine(self, y16, acc, scale=None, vis=None, stream=None):
        """corr_fix16_xengine: exact int64 sums [C][P][2] of the 16-bit spectra's
        products, and optionally the scaled FP64 visibilities."""
        import torch
        _need(y16, "y16", 4 * self.S * self.T * self.C, torch.int16)
        _need(acc, "acc", 16 * self.C * self.P, torch.int64)
        _need(vis, "vis", 16 * self.C * self.P, torch.float64, optional=True)
        _need(scale, "scale", 4 * self.S * self.C, torch.float32, optional=True)
        self._check(lib().corr_fix16_xengine(self._h, _ptr(y16), _ptr(scale), _ptr(acc), _ptr(vis), _stream(stream)))

    def integrate(self, acc, state, vis=None, scale=None, flags=DUMP, stream=None):
        import torch
        _need(acc, "acc", self.acc_bytes)
        _need(state, "state", self.state_bytes, torch.float64)
        _need(vis, "vis", self.vis_bytes, (torch.float32, torch.complex64), optional=True)
        _need(scale, "scale", 4 * self.S * self.C, torch.float32, optional=self.precision == FP32)
        self._check(lib().corr_integrate(self._h, _ptr(acc), _ptr(scale), _ptr(state), _ptr(vis), flags,
                                         _stream(stream)))

    def check_device_errors(self, stream=None):
        self._check(lib().corr_check_device_errors(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            if self._owned:
                lib().corr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several INT8 correlations of different shapes run as one unit (corr_batch_t):
    concurrent F-engines, one X-engine launch over all sub-arrays, integration;
    capturable into one HIP graph."""

    def __init__(self, shapes, *, device=None, **common):
        """shapes: list of dicts with n_signals, fft_len, n_spectra (and optional x_split)."""
        L = lib()
        self.descs = (CorrDesc * len(shapes))()
        kw = dict(precision=INT8, scale_mode=SCALE_HOLD)
        kw.update(common)
        for i, sh in enumerate(shapes):
            self.descs[i] = make_desc(sh["n_signals"], sh["fft_len"], sh["n_spectra"],
                                      x_split=sh.get("x_split", 0), **kw)
        h = ctypes.c_void_p()
        rc = L.corr_batch_create(self.descs, len(shapes), ctypes.byref(h))
        if rc != 0:
            raise CorrError(rc, L.corr_last_error(None).decode())
        self._h = h
        self.plans = []
        for i, sh in enumerate(shapes):
            d = self.descs[i]
            p = Plan(d.n_signals, d.fft_len, d.n_spectra, max_delay=d.max_delay, precision=d.precision,
                     sideband=d.sideband, scale_mode=d.scale_mode, sample_rate=d.sample_rate, nu_bb=d.nu_bb,
                     x_split=d.x_split, device=device, _handle=L.corr_batch_plan(h, i))
            self.plans.append(p)
        self._keep = {}

    def _check(self, rc):
        if rc != 0:
            raise CorrError(rc, lib().corr_batch_last_error(self._h).decode())

    def set_io(self, i, *, x, geom, spec, scale, acc, state, vis=None, flags=DUMP, row_stride=None, spectrum0=0):
        import torch
        p = self.plans[i]
        rs = x.stride(0) if row_stride is None else row_stride
        _need(x, "x", _rows_bytes(p.S, rs, p.T * p.N + p.max_delay), (torch.int8, torch.uint8), rows=True)
        _need(geom, "geom", 24 * p.S)
        _need(spec, "spec", p.spectra_bytes)
        _need(scale, "scale", 4 * p.S * p.C, torch.float32)
        _need(acc, "acc", p.acc_bytes)
        _need(state, "state", p.state_bytes, torch.float64)
        _need(vis, "vis", p.vis_bytes, (torch.float32, torch.complex64), optional=True)
        io = BatchIO(_ptr(x), x.stride(0) if row_stride is None else row_stride, _ptr(geom), spectrum0,
                     _ptr(spec), _ptr(scale), _ptr(acc), _ptr(state), _ptr(vis), flags)
        self._keep[i] = (x, geom, spec, scale, acc, state, vis)  # keep the tensors alive
        self._check(lib().corr_batch_set_io(self._h, i, ctypes.byref(io)))

    def run(self, stream=None):
        self._check(lib().corr_batch_run(self._h, _stream(stream)))

    def capture(self, stream):
        self._check(lib().corr_batch_capture(self._h, _stream(stream)))

    def launch(self, stream=None):
        self._check(lib().corr_batch_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            for p in self.plans:
                p.close()
            lib().corr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cnn_check(rc, h=None):
    if rc != 0:
        raise CorrError(rc, lib().corr_cnn_last_error(h).decode())


def _cnn_args(params, power, tiles, labels=None):
    """Buffers shared by the CNN training calls: parameters, power [S][T][C],
    the int32 tile list and, for the loss, labels [S][T][C]."""
    import torch
    _need(params, "params", 4 * CNN_PARAMS, torch.float32)
    S, T, C = power.shape
    _need(power, "power", 4 * S * T * C, torch.float32)
    _need(tiles, "tiles", 4 * tiles.numel(), torch.int32)
    if labels is not None:
        _need(labels, "labels", S * T * C, (torch.uint8, torch.bool))


def cnn_tiles(S: int, T: int, C: int) -> int:
    """Number of 64 x 256 flagging tiles of power [S][T][C]."""
    return S * (T // TILE_SPECTRA) * (C // TILE_CHANNELS)


class CNN:
    """Training handle of the learned flagger (corr_cnn_t) with its workspace
    bound to device memory.  Parameters and Adam moments are caller-owned
    device tensors of CNN_PARAMS floats."""

    def __init__(self, max_tiles: int, *, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, device=None):
        import torch
        L = lib()
        self.desc = CnnDesc()
        self.desc.max_tiles, self.desc.lr, self.desc.beta1, self.desc.beta2, self.desc.eps = (
            max_tiles, lr, beta1, beta2, eps)
        h = ctypes.c_void_p()
        _cnn_check(L.corr_cnn_create(ctypes.byref(self.desc), ctypes.byref(h)))
        self._h = h
        self.max_tiles = max_tiles
        n = int(L.corr_cnn_workspace_bytes(h))
        self.workspace = torch.empty(n, dtype=torch.uint8, device=device or "cuda")
        self._check(L.corr_cnn_bind_workspace(h, _ptr(self.workspace), n))

    def _check(self, rc):
        _cnn_check(rc, self._h)

    def forward(self, params, power, tiles, logits, stream=None):
        """FP32 logits [n][64][256] of the listed tiles of power [S][T][C]."""
        import torch
        S, T, C = power.shape
        _cnn_args(params, power, tiles)
        _need(logits, "logits", 4 * tiles.numel() * TILE_SPECTRA * TILE_CHANNELS, torch.float32)
        self._check(lib().corr_cnn_forward(self._h, _ptr(params), _ptr(power), S, T, C, _ptr(tiles),
                                           tiles.numel(), _ptr(logits), _stream(stream)))

    def loss_grad(self, params, power, labels, tiles, loss, grad=None, stream=None):
        import torch
        S, T, C = power.shape
        _cnn_args(params, power, tiles, labels)
        _need(loss, "loss", 4, torch.float32)
        _need(grad, "grad", 4 * CNN_PARAMS, torch.float32, optional=True)
        self._check(lib().corr_cnn_loss_grad(self._h, _ptr(params), _ptr(power), _ptr(labels), S, T, C,
                                             _ptr(tiles), tiles.numel(), _ptr(loss), _ptr(grad), _stream(stream)))

    def adam(self, params, m, v, step: int, grad=None, stream=None):
        import torch
        for t, nm in ((params, "params"), (m, "m"), (v, "v")):
            _need(t, nm, 4 * CNN_PARAMS, torch.float32)
        _need(grad, "grad", 4 * CNN_PARAMS, torch.float32, optional=True)
        self._check(lib().corr_cnn_adam(self._h, _ptr(params), _ptr(m), _ptr(v), _ptr(grad), step, _stream(stream)))

    def train_step(self, params, m, v, step: int, power, labels, tiles, loss, stream=None):
        import torch
        S, T, C = power.shape
        _cnn_args(params, power, tiles, labels)
        for t, nm in ((m, "m"), (v, "v")):
            _need(t, nm, 4 * CNN_PARAMS, torch.float32)
        _need(loss, "loss", 4, torch.float32)
        self._check(lib().corr_cnn_train_step(self._h, _ptr(params), _ptr(m), _ptr(v), step, _ptr(power),
                                              _ptr(labels), S, T, C, _ptr(tiles), tiles.numel(), _ptr(loss),
                                              _stream(stream)))

    def check_device_errors(self, stream=None):
        self._check(lib().corr_cnn_check_device_errors(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().corr_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cnn_infer(params, power, flags, *, threshold: float = 0.5, logits=None, guard: float = 0.0, stream=None):
    """Flags (and optionally logits) of every tile of power [S][T][C] (float32,
    or float16 as the F-engine writes it with power_fp16) from the fused FP16
    inference kernel.  guard > 0: also flag the tile columns that the MAD
    column statistic flags at M = guard (corr_cnn_infer_guarded)."""
    import torch
    S, T, C = power.shape
    f16 = power.dtype == torch.float16
    _need(params, "params", 4 * CNN_PARAMS, torch.float32)
    _need(power, "power", (2 if f16 else 4) * S * T * C, (torch.float16, torch.float32))
    _need(flags, "flags", S * T * C, torch.uint8)
    _need(logits, "logits", 4 * S * T * C, torch.float32, optional=True)
    if guard:
        _cnn_check(lib().corr_cnn_infer_guarded(_ptr(params), _ptr(power), int(f16), S, T, C, threshold, guard,
                                                _ptr(flags), _ptr(logits), _stream(stream)))
        return
    fn = lib().corr_cnn_infer_f16 if f16 else lib().corr_cnn_infer
    _cnn_check(fn(_ptr(params), _ptr(power), S, T, C, threshold, _ptr(flags), _ptr(logits), _stream(stream)))


def cnn_save(path: str, params, m=None, v=None, step: int = 0):
    import torch
    _need(params, "params", 4 * CNN_PARAMS, torch.float32)
    _need(m, "m", 4 * CNN_PARAMS, torch.float32, optional=True)
    _need(v, "v", 4 * CNN_PARAMS, torch.float32, optional=True)
    _cnn_check(lib().corr_cnn_save(path.encode(), _ptr(params), _ptr(m), _ptr(v), step))


def cnn_load(path: str, params, m=None, v=None) -> int:
    import torch
    _need(params, "params", 4 * CNN_PARAMS, torch.float32)
    _need(m, "m", 4 * CNN_PARAMS, torch.float32, optional=True)
    _need(v, "v", 4 * CNN_PARAMS, torch.float32, optional=True)
    st = ctypes.c_int64()
    _cnn_check(lib().corr_cnn_load(path.encode(), _ptr(params), _ptr(m), _ptr(v), ctypes.byref(st)))
    return st.value


def adc_unpack(raw, x, *, bits: int, n: int | None = None, stream=None):
    """Demultiplex and unpack card streams raw (uint8 [cards][raw_stride]) into
    int8 rows x [4 cards][row_stride] (first n samples; default the row
    length); see corr_adc_unpack."""
    import torch
    cards, rs_raw = raw.shape
    rows, rs = x.shape
    if rows != 4 * cards:
        raise ValueError("x has %d rows, needs 4 per card (%d)" % (rows, 4 * cards))
    nn = rs if n is None else int(n)
    _need(raw, "raw", _rows_bytes(cards, raw.stride(0), nn * bits // 2), torch.uint8, rows=True)
    _need(x, "x", _rows_bytes(rows, x.stride(0), nn), torch.int8, rows=True)
    rc = lib().corr_adc_unpack(_ptr(raw), raw.stride(0), cards, rs if n is None else n, bits, _ptr(x), x.stride(0),
                               _stream(stream))
    if rc != 0:
        raise CorrError(rc, lib().corr_adc_last_error().decode())
    return x


def pulsar_gates(spectrum0: int, n_spectra: int, fft_len: int, sample_rate: float, t0: float, period: float,
                 n_bins: int):
    """(gate uint8 [n_spectra], counts int64 [n_bins]) of consecutive spectra
    from a pulsar's period; see corr_pulsar_gates (host arithmetic)."""
    import numpy as np
    gate = np.zeros(n_spectra, dtype=np.uint8)
    counts = np.zeros(n_bins, dtype=np.int64)
    rc = lib().corr_pulsar_gates(spectrum0, n_spectra, fft_len, sample_rate, t0, period, n_bins,
                                 gate.ctypes.data_as(ctypes.c_void_p), counts.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise CorrError(rc, lib().corr_last_error(None).decode())
    return gate, counts


def dedisperse(v, *, sample_rate: float, nu0: float, dm: float, n_int: int, work=None, out=None, stream=None):
    """Coherent dedispersion of one beam's voltages v (complex64 device tensor
    [npol][T][C]); returns the detected, integrated series (float [T C /
    n_int]) and the workspace (the dedispersed voltages).  See
    corr_dedisperse."""
    import torch
    npol, T, C = v.shape
    L = T * C
    if work is None:
        work = torch.empty(npol, L, dtype=torch.complex64, device=v.device)
    if out is None:
        out = torch.empty(L // max(int(n_int), 1), dtype=torch.float32, device=v.device)
    _need(v, "v", 8 * npol * L, torch.complex64)
    _need(work, "work", 8 * npol * L, torch.complex64)
    _need(out, "out", 4 * (L // max(int(n_int), 1)), torch.float32)
    rc = lib().corr_dedisperse(_ptr(v), npol, T, C, sample_rate, nu0, dm, n_int, _ptr(work), _ptr(out),
                               _stream(stream))
    if rc != 0:
        raise CorrError(rc, lib().corr_dedisperse_last_error().decode())
    return out, work


DEDISPERSE_NOALLOC_MAX = 1 << 22  # complex samples (npol T C) of corr_dedisperse_noalloc


def dedisperse_noalloc(v, out, *, sample_rate: float, nu0: float, dm: float, n_int: int, stream=None):
    """corr_dedisperse_noalloc: the same dedispersion with the library's own
    device scratch (no workspace argument, nothing allocated by the call);
    npol T C at most DEDISPERSE_NOALLOC_MAX.  Writes out (float [T C / n_int])."""
    import torch
    npol, T, C = v.shape
    L = T * C
    _need(v, "v", 8 * npol * L, torch.complex64)
    _need(out, "out", 4 * (L // max(int(n_int), 1)), torch.float32)
    rc = lib().corr_dedisperse_noalloc(_ptr(v), npol, T, C, sample_rate, nu0, dm, n_int, _ptr(out), _stream(stream))
    if rc != 0:
        raise CorrError(rc, lib().corr_dedisperse_last_error().decode())
    return out


def _blank_check(rc):
    if rc != 0:
        raise CorrError(rc, lib().corr_blank_last_error().decode())


def blank_noise_table(seed: int, table, stream=None):
    """Fill table (float32 [S][L], L a power of two) with the blanker's
    precomputed Gaussian noise; see corr_blank_noise_table."""
    import torch
    S, L = table.shape
    _need(table, "table", 4 * S * L, torch.float32)
    _blank_check(lib().corr_blank_noise_table(int(seed) & 0xFFFFFFFFFFFFFFFF, S, L, _ptr(table), _stream(stream)))


def blank_voltages(x, table, *, block: int, M: float = 3.0, out=None, counts=None, stats=None, sample0: int = 0,
                   n: int | None = None, stream=None):
    """MAD voltage blanker on int8 rows x [S][row_stride] (first n samples of
    each row, default all); out is x (in place, the default) or a tensor of
    the same shape; counts int32 [S][nblocks] and stats int32
    [S][nblocks][2] optional.  See corr_blank_voltages."""
    import torch
    S, rs = x.shape
    if out is None:
        out = x
    nn = rs if n is None else int(n)
    nblk = -(-nn // block) if block > 0 else 0
    _need(x, "x", _rows_bytes(S, x.stride(0), nn), torch.int8, rows=True)
    _need(out, "out", _rows_bytes(S, x.stride(0), nn), torch.int8, rows=True)
    if out.stride(0) != x.stride(0):
        raise ValueError("out must have the row stride of x")
    _need(table, "table", 4 * S * table.shape[1], torch.float32)
    _need(counts, "counts", 4 * S * nblk, torch.int32, optional=True)
    _need(stats, "stats", 8 * S * nblk, torch.int32, optional=True)
    _blank_check(lib().corr_blank_voltages(_ptr(x), x.stride(0), S, rs if n is None else n, block, M, _ptr(table),
                                           table.shape[1], sample0, _ptr(out), _ptr(counts), _ptr(stats),
                                           _stream(stream)))
    return out


def _autotune_cache_path():
    base = os.environ.get("CORR_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_0910_1517_amd", "autotune.json")
    return base


def autotune_x_split(n_signals, fft_len, n_spectra, *, precision=INT8, cache=True, device=None):
    """Fastest X-engine K-split for this shape, measured on the current GPU
    (corr_autotune_x_split) and remembered in a JSON cache keyed by device
    architecture and shape.  Returns (split, ms)."""
    import json
    import torch
    arch = torch.cuda.get_device_properties(device or 0).gcnArchName.split(":")[0]
    key = "%s|S%d|N%d|T%d|P%d" % (arch, n_signals, fft_len, n_spectra, precision)
    path = _autotune_cache_path()
    table = {}
    if cache and os.path.exists(path):
        try:
            table = json.load(open(path))
        except (OSError, ValueError):
            table = {}
    if cache and key in table:
        return int(table[key]["split"]), float(table[key]["ms"])
    L = lib()
    d = make_desc(n_signals, fft_len, n_spectra, precision=precision)
    nbytes = int(L.corr_autotune_scratch_bytes(ctypes.byref(d)))
    if nbytes == 0:
        raise CorrError(-1, L.corr_last_error(None).decode())
    scratch = torch.zeros(nbytes, dtype=torch.uint8, device=device or "cuda")
    best = ctypes.c_int32()
    ms = ctypes.c_float()
    rc = L.corr_autotune_x_split(ctypes.byref(d), _ptr(scratch), nbytes, _stream(None), ctypes.byref(best),
                                 ctypes.byref(ms))
    if rc != 0:
        raise CorrError(rc, L.corr_last_error(None).decode())
    del scratch
    if cache:
        table[key] = {"split": best.value, "ms": ms.value}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        json.dump(table, open(tmp, "w"), indent=1, sort_keys=True)
        os.replace(tmp, path)
    return best.value, ms.value


def geom_array(D, frac, psi0, rate) -> np.ndarray:
    """corr_geom_t[S] as a numpy structured array (host)."""
    g = np.zeros(len(D), dtype=GEOM_DTYPE)
    g["D"], g["frac"], g["psi0"], g["rate"] = D, frac, psi0, rate
    return g


def geom_from_model(tau0, taudot, *, t0: float = 0.0, t_delay: float = 0.0, sample_rate: float,
                    nu_lo: float, max_delay: int) -> np.ndarray:
    """corr_geom_t[S] (host structured array) from the delay model
    tau_s(t) = tau0[s] + taudot[s] (t - t0); see corr_geom_from_model (host arithmetic)."""
    tau0 = np.ascontiguousarray(tau0, dtype=np.float64)
    taudot = np.ascontiguousarray(taudot, dtype=np.float64)
    if tau0.shape != taudot.shape or tau0.ndim != 1:
        raise ValueError("tau0 and taudot must be 1-D arrays of the same length")
    g = np.zeros(tau0.size, dtype=GEOM_DTYPE)
    rc = lib().corr_geom_from_model(tau0.size, tau0.ctypes.data_as(ctypes.c_void_p),
                                    taudot.ctypes.data_as(ctypes.c_void_p), t0, t_delay, sample_rate, nu_lo,
                                    max_delay, g.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise CorrError(rc, lib().corr_last_error(None).decode())
    return g


def geom_to_device(g: np.ndarray, device="cuda"):
    import torch
    return torch.from_numpy(g.view(np.uint8).copy()).to(device)


def vis_complex(vis, C: int, P: int) -> np.ndarray:
    """Dumped complex64 visibilities (device float tensor) -> numpy complex [C][P]."""
    v = vis.detach().cpu().numpy().reshape(C, P, 2)
    return v[..., 0].astype(np.float64) + 1j * v[..., 1].astype(np.float64)


def unpack_spectra(spec, precision: int, S: int, C: int, T: int) -> np.ndarray:
    """X-layout spectra (device uint8 tensor) -> numpy [S][T][C][2] (float32 / int8 / uint8 codes).

    Host-side reader for tests and diagnostics; the X-engine reads the layout directly."""
    raw = spec.detach().cpu().numpy()
    if precision == FP32:
        a = raw.view(np.float32).reshape(T // 2, C // 8, S, 8, 2, 2)  # [g][kb][s][kk][q][re/im]
        return np.ascontiguousarray(a.transpose(2, 0, 4, 1, 3, 5).reshape(S, T, C, 2))
    a = raw.reshape(T // 8, C // 8, S, 8, 2, 8)                       # [g][kb][s][kk][re/im][q]
    out = a.transpose(2, 0, 5, 1, 3, 4).reshape(S, T, C, 2)
    return np.ascontiguousarray(out.view(np.int8) if precision == INT8 else out)
