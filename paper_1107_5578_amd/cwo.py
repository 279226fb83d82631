"""Python binding of libcwo (argument marshalling only).

Every step of a propagation runs in the HIP kernels of ``libcwo.so``; this
module only converts arguments, allocates output tensors with PyTorch and
passes device pointers and the current HIP stream through the C ABI declared in
``include/cwo.h``. Importing it raises if the library has not been built.

Fields are ``torch.complex64`` tensors on a ROCm device, contiguous, shape
``[ny, nx]`` (x fastest), as the C ABI requires.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcwo.so")

CWO_OK = 0
CWO_ERR_INVALID = -1
CWO_ERR_UNSUPPORTED = -2
CWO_ERR_NOMEM = -3
CWO_ERR_DEVICE = -4
CWO_ERR_NOTFOUND = -5

ANGULAR = 1
FRESNEL_CONV = 2
FRESNEL_FOURIER = 3
FRESNEL_SHIFTED = 4

PREC_F32 = 0
PREC_F16 = 1
PREC_BF16 = 2
_PRECISIONS = {"f32": PREC_F32, "fp32": PREC_F32, "f16": PREC_F16, "fp16": PREC_F16,
               "bf16": PREC_BF16}

FLAG_NOPAD = 1
FLAG_FRESNEL_TF = 2  # Fresnel: analytic transfer function instead of the sampled kernel

STAGE_ROW_FWD = 0
STAGE_COL = 1
STAGE_ROW_INV = 2
STAGE_TABLES = 3
STAGE_COL_Z = 4
STAGE_ROW_GS = 5
STAGE_NAMES = {STAGE_ROW_FWD: "row_fwd", STAGE_COL: "col", STAGE_ROW_INV: "row_inv",
               STAGE_TABLES: "tables", STAGE_COL_Z: "col_z", STAGE_ROW_GS: "row_gs"}
KINDS = {"asm": ANGULAR, "angular": ANGULAR, "fresnel": FRESNEL_CONV}


class CwoError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        msg = strerror(status)
        super().__init__("%s: %s (status %d)" % (what, msg, status) if what else msg)


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("wavelength", ctypes.c_double), ("z", ctypes.c_double),
        ("kind", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


class Job(ctypes.Structure):
    _fields_ = [("p", Params), ("inp", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class TicketInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("footprint", ctypes.c_size_t)]


QUEUED, RUNNING, DONE = 0, 1, 2


_lib = None
_lib_lock = threading.Lock()

# name -> (restype, argtypes) for every symbol include/cwo.h declares
class Shift(ctypes.Structure):
    """cwo_shift: destination-window offset [m] and band-limit centres/widths [1/m]."""
    _fields_ = [("ox", ctypes.c_double), ("oy", ctypes.c_double),
                ("cx", ctypes.c_double), ("wx", ctypes.c_double),
                ("cy", ctypes.c_double), ("wy", ctypes.c_double)]


class PlsParams(ctypes.Structure):
    """cwo_pls_params: hologram size and pitch, wavelength, object offset [m]."""
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("px", ctypes.c_double), ("py", ctypes.c_double),
                ("wavelength", ctypes.c_double),
                ("ox", ctypes.c_double), ("oy", ctypes.c_double), ("oz", ctypes.c_double)]


class SFresnel(ctypes.Structure):
    """cwo_sfresnel: destination pitch and the two window centres [m]."""
    _fields_ = [("dx1", ctypes.c_double), ("dy1", ctypes.c_double),
                ("ox0", ctypes.c_double), ("oy0", ctypes.c_double),
                ("ox1", ctypes.c_double), ("oy1", ctypes.c_double)]


class Tuning(ctypes.Structure):
    """cwo_tuning: the schedule picked by cwo_autotune."""
    _fields_ = [("row_form", ctypes.c_int32), ("zchunk", ctypes.c_int32),
                ("us_per_plane", ctypes.c_float), ("layout", ctypes.c_int32),
                ("col_form", ctypes.c_int32)]


SIGNATURES = {
    "cwo_create": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_size_t]),
    "cwo_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "cwo_asm": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p]),
    "cwo_fresnel": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "cwo_asm_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "cwo_asm_shifted": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params),
                                         ctypes.POINTER(Shift), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "cwo_band_limit": (ctypes.c_int32, [ctypes.POINTER(Params), ctypes.POINTER(Shift)]),
    "cwo_fresnel_shifted": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params),
                                             ctypes.POINTER(SFresnel), ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "cwo_intensity": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p]),
    "cwo_asm_intensity": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params),
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cwo_fresnel_intensity": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params),
                                               ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "cwo_pls_cgh": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(PlsParams), ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "cwo_pls_field": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(PlsParams),
                                       ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "cwo_phase": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p]),
    "cwo_polar": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "cwo_scale": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_float, ctypes.c_size_t,
                                   ctypes.c_void_p]),
    "cwo_fresnel_fourier": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params),
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cwo_fresnel_fourier_pitch": (ctypes.c_int32, [ctypes.POINTER(Params),
                                                   ctypes.POINTER(ctypes.c_double),
                                                   ctypes.POINTER(ctypes.c_double)]),
    "cwo_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(Tuning)]),
    "cwo_set_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_int32,
                                        ctypes.POINTER(Tuning)]),
    "cwo_zstack": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params),
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cwo_batch": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.c_int32,
                                   ctypes.c_void_p]),
    "cwo_gs": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p]),
    "cwo_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Job),
                                    ctypes.POINTER(ctypes.c_uint64)]),
    "cwo_submit_after": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "cwo_memory_held": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "cwo_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]),
    "cwo_ticket_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.POINTER(TicketInfo)]),
    "cwo_release": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64]),
    "cwo_drain": (ctypes.c_int32, [ctypes.c_void_p]),
    "cwo_check_params": (ctypes.c_int32, [ctypes.POINTER(Params), ctypes.c_int32]),
    "cwo_scratch_bytes": (ctypes.c_size_t, [ctypes.POINTER(Params)]),
    "cwo_profile": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "cwo_profile_read": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64)]),
    "cwo_strerror": (ctypes.c_char_p, [ctypes.c_int32]),
    "cwo_version": (ctypes.c_int32, []),
}


def load():
    """Load libcwo.so (raises FileNotFoundError when it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise FileNotFoundError(
                    "libcwo.so is not built (run `python -m paper_1107_5578_amd.build`)")
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def strerror(status: int) -> str:
    return load().cwo_strerror(int(status)).decode()


def make_params(nx, ny, dx, dy=None, wavelength=633e-9, z=0.1, kind=0, precision="f32",
                nopad=False, fresnel_tf=False) -> Params:
    prec = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return Params(int(nx), int(ny), float(dx), float(dx if dy is None else dy),
                  float(wavelength), float(z), int(kind), prec,
                  (FLAG_NOPAD if nopad else 0) | (FLAG_FRESNEL_TF if fresnel_tf else 0))


def check_params(p: Params, kind: int) -> int:
    return int(load().cwo_check_params(ctypes.byref(p), int(kind)))


class Context:
    """A libcwo context on one device: scratch, twiddle tables and caches."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._lib = load()
        h = ctypes.c_void_p()
        st = self._lib.cwo_create(ctypes.byref(h), int(device), int(hbm_budget_bytes))
        if st != CWO_OK:
            raise CwoError(st, "cwo_create")
        self.handle = h
        self.device = int(device)

    def close(self):
        if getattr(self, "handle", None):
            st = self._lib.cwo_destroy(self.handle)
            self.handle = None
            if st != CWO_OK:
                raise CwoError(st, "cwo_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool):
        """Start (clearing totals) or stop per-kernel HIP-event timing."""
        st = self._lib.cwo_profile(self.handle, 1 if enable else 0)
        if st != CWO_OK:
            raise CwoError(st, "cwo_profile")

    def profile_read(self, stage: int):
        """(total milliseconds, launches) of one kernel stage since profiling started."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        st = self._lib.cwo_profile_read(self.handle, int(stage), ctypes.byref(ms), ctypes.byref(n))
        if st != CWO_OK:
            raise CwoError(st, "cwo_profile_read")
        return ms.value, n.value

    # -- helpers ------------------------------------------------------------
    @staticmethod
    def _field(u):
        import torch
        if not isinstance(u, torch.Tensor) or u.dtype != torch.complex64 or u.dim() != 2:
            raise TypeError("field must be a 2-D torch.complex64 tensor")
        if u.device.type != "cuda":
            raise TypeError("field must live on a ROCm device")
        if not u.is_contiguous():
            raise ValueError("field must be contiguous [ny, nx]")
        return u

    @staticmethod
    def _stream(u, stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(u.device)
        return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))

    def _propagate(self, fn, kind, u, dx, dy, wavelength, z, precision, nopad, out, stream,
                   fresnel_tf=False):
        import torch
        u = self._field(u)
        ny, nx = u.shape
        p = make_params(nx, ny, dx, dy, wavelength, z, kind, precision, nopad, fresnel_tf)
        if out is None:
            out = torch.empty_like(u)
        else:
            out = self._field(out)
            if out.shape != u.shape or out.device != u.device:
                raise ValueError("out must match the field's shape and device")
        st = fn(self.handle, ctypes.byref(p), ctypes.c_void_p(u.data_ptr()),
                ctypes.c_void_p(out.data_ptr()), self._stream(u, stream))
        if st != CWO_OK:
            raise CwoError(st, fn.__name__)
        return out

    def asm(self, u, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, precision="f32",
            nopad=False, out=None, stream=None):
        """Angular spectrum propagation by z (stream-ordered; returns the output tensor)."""
        return self._propagate(self._lib.cwo_asm, ANGULAR, u, dx, dy, wavelength, z, precision,
                               nopad, out, stream)

    def asm_noalloc(self, u, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, nopad=False,
                    out=None, stream=None):
        """cwo_asm through the entry point that allocates no device memory (its scratch is a
        static device array; calls that overlap on one device race). Pass `out` to keep the
        call free of allocations on the Python side too."""
        return self._propagate(self._lib.cwo_asm_noalloc, ANGULAR, u, dx, dy, wavelength, z,
                               "f32", nopad, out, stream)

    def fresnel(self, u, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, precision="f32",
                nopad=False, out=None, stream=None, fresnel_tf=False):
        """Fresnel diffraction (convolution form) by z; fresnel_tf takes the analytic
        transfer function instead of the transformed sampled kernel."""
        return self._propagate(self._lib.cwo_fresnel, FRESNEL_CONV, u, dx, dy, wavelength, z,
                               precision, nopad, out, stream, fresnel_tf)

    def fresnel_fourier(self, u, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, out=None,
                        stream=None):
        """Fresnel diffraction, Fourier form (one unpadded FFT); the destination pitch is
        fresnel_fourier_pitch(...)."""
        return self._propagate(self._lib.cwo_fresnel_fourier, FRESNEL_FOURIER, u, dx, dy,
                               wavelength, z, "f32", False, out, stream)

    # -- epilogues (Sec. 3.1, Sec. 7.1) -------------------------------------
    def _contig(self, t, dtype, name):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor" % (name, dtype))
        return t

    def intensity(self, u, stream=None):
        """|u|^2 as a float32 tensor of u's shape."""
        import torch
        u = self._contig(u, torch.complex64, "u")
        out = torch.empty(u.shape, dtype=torch.float32, device=u.device)
        st = self._lib.cwo_intensity(self.handle, ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), u.numel(),
                                     self._stream(u, stream))
        if st != CWO_OK:
            raise CwoError(st, "cwo_intensity")
        return out

    def phase(self, u, stream=None):
        """atan2(Im u, Re u) as a float32 tensor (the kinoform of u)."""
        import torch
        u = self._contig(u, torch.complex64, "u")
        out = torch.empty(u.shape, dtype=torch.float32, device=u.device)
        st = self._lib.cwo_phase(self.handle, ctypes.c_void_p(u.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), u.numel(),
                                 self._stream(u, stream))
        if st != CWO_OK:
            raise CwoError(st, "cwo_phase")
        return out

    def polar(self, phase, amp=None, stream=None):
        """amp * exp(i phase) (amp = 1 if None) as a complex64 tensor."""
        import torch
        phase = self._contig(phase, torch.float32, "phase")
        if amp is not None:
            amp = self._contig(amp, torch.float32, "amp")
            if amp.shape != phase.shape:
                raise ValueError("amp must match phase")
        out = torch.empty(phase.shape, dtype=torch.complex64, device=phase.device)
        st = self._lib.cwo_polar(self.handle, ctypes.c_void_p(phase.data_ptr()),
                                 ctypes.c_void_p(amp.data_ptr() if amp is not None else None),
                                 ctypes.c_void_p(out.data_ptr()), phase.numel(),
                                 self._stream(phase, stream))
        if st != CWO_OK:
            raise CwoError(st, "cwo_polar")
        return out

    def scale(self, x, top=255.0, u8=False, stream=None):
        """(x - min)/(max - min) * top as float32, or as uint8 codes when u8."""
        import torch
        x = self._contig(x, torch.float32, "x")
        out = torch.empty(x.shape, dtype=torch.uint8 if u8 else torch.float32, device=x.device)
        st = self._lib.cwo_scale(self.handle, ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), 1 if u8 else 0, float(top),
                                 x.numel(), self._stream(x, stream))
        if st != CWO_OK:
            raise CwoError(st, "cwo_scale")
        return out

    def fresnel_shifted(self, u, dx0=10e-6, dy0=None, dx1=10e-6, dy1=None, wavelength=633e-9,
                        z=0.1, ox0=0.0, oy0=0.0, ox1=0.0, oy1=0.0, out=None, stream=None):
        """Shifted Fresnel diffraction from a window of pitch (dx0, dy0) centred at
        (ox0, oy0) to one of pitch (dx1, dy1) centred at (ox1, oy1) [m]."""
        dy0 = dx0 if dy0 is None else dy0
        dy1 = dx1 if dy1 is None else dy1
        w = SFresnel(float(dx1), float(dy1), float(ox0), float(oy0), float(ox1), float(oy1))
        lib = self._lib

        def call(h, pp, a, b, s):
            return lib.cwo_fresnel_shifted(h, pp, ctypes.byref(w), a, b, s)

        call.__name__ = "cwo_fresnel_shifted"
        return self._propagate(call, FRESNEL_SHIFTED, u, dx0, dy0, wavelength, z, "f32", False,
                               out, stream)

    def _propagate_intensity(self, fn, kind, u, dx, dy, wavelength, z, precision, nopad, out,
                             stream, fresnel_tf=False):
        import torch
        u = self._field(u)
        ny, nx = u.shape
        p = make_params(nx, ny, dx, dy, wavelength, z, kind, precision, nopad, fresnel_tf)
        if out is None:
            out = torch.empty((ny, nx), dtype=torch.float32, device=u.device)
        elif (out.dtype != torch.float32 or tuple(out.shape) != (ny, nx)
              or not out.is_contiguous() or out.device != u.device):
            raise ValueError("out must be a contiguous float32 [ny, nx] tensor on the field's device")
        st = fn(self.handle, ctypes.byref(p), ctypes.c_void_p(u.data_ptr()),
                ctypes.c_void_p(out.data_ptr()), self._stream(u, stream))
        if st != CWO_OK:
            raise CwoError(st, fn.__name__)
        return out

    def asm_intensity(self, u, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, precision="f32",
                      nopad=False, out=None, stream=None):
        """|ASM propagation of u|^2, the intensity stored by the last pass (float [ny, nx])."""
        return self._propagate_intensity(self._lib.cwo_asm_intensity, ANGULAR, u, dx, dy,
                                         wavelength, z, precision, nopad, out, stream)

    def fresnel_intensity(self, u, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, precision="f32",
                          nopad=False, out=None, stream=None, fresnel_tf=False):
        """|Fresnel propagation of u|^2, the intensity stored by the last pass."""
        return self._propagate_intensity(self._lib.cwo_fresnel_intensity, FRESNEL_CONV, u, dx,
                                         dy, wavelength, z, precision, nopad, out, stream,
                                         fresnel_tf)

    def _pls(self, fn, points, nx, ny, px, py, wavelength, ox, oy, oz, out, stream, field):
        import torch
        if (not isinstance(points, torch.Tensor) or points.dtype != torch.float32
                or points.dim() != 2 or points.shape[1] != 4 or not points.is_contiguous()
                or points.device.type != "cuda"):
            raise ValueError("points must be a contiguous float32 [N, 4] CUDA tensor (X, Y, Z, A)")
        py = px if py is None else py
        dtype = torch.complex64 if field else torch.float32
        if out is None:
            out = torch.empty((int(ny), int(nx)), dtype=dtype, device=points.device)
        elif (out.dtype != dtype or tuple(out.shape) != (int(ny), int(nx))
              or not out.is_contiguous() or out.device != points.device):
            raise ValueError("out must be a contiguous [ny, nx] tensor of the right dtype")
        p = PlsParams(int(nx), int(ny), float(px), float(py), float(wavelength), float(ox),
                      float(oy), float(oz))
        st = fn(self.handle, ctypes.byref(p), ctypes.c_void_p(points.data_ptr()),
                int(points.shape[0]), ctypes.c_void_p(out.data_ptr()),
                self._stream(points, stream))
        if st != CWO_OK:
            raise CwoError(st, fn.__name__)
        return out

    def pls_cgh(self, points, nx, ny, px=10e-6, py=None, wavelength=633e-9, ox=0.0, oy=0.0,
                oz=0.1, out=None, stream=None):
        """Point-light-source hologram I = sum_j A_j cos(pi r_j^2/(lambda z_j)), float
        [ny, nx]; points: float32 [N, 4] (X, Y, Z, A) relative to the offset (ox, oy, oz)."""
        return self._pls(self._lib.cwo_pls_cgh, points, nx, ny, px, py, wavelength, ox, oy, oz,
                         out, stream, False)

    def pls_field(self, points, nx, ny, px=10e-6, py=None, wavelength=633e-9, ox=0.0, oy=0.0,
                  oz=0.1, out=None, stream=None):
        """Point-light-source complex field exp(i k oz)/(i lambda oz) sum_j A_j
        exp(i pi r_j^2/(lambda z_j)), complex64 [ny, nx]."""
        return self._pls(self._lib.cwo_pls_field, points, nx, ny, px, py, wavelength, ox, oy,
                         oz, out, stream, True)

    def asm_shifted(self, u, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, ox=0.0, oy=0.0,
                    cx=0.0, wx=0.0, cy=0.0, wy=0.0, nopad=False, out=None, stream=None,
                    precision="f32"):
        """Shifted angular spectrum propagation: window offset (ox, oy) [m], band limits
        Rect((fx - cx)/wx) Rect((fy - cy)/wy) [1/m] (a width <= 0: no limit)."""
        sh = Shift(float(ox), float(oy), float(cx), float(wx), float(cy), float(wy))
        lib = self._lib

        def call(h, pp, a, b, s):
            return lib.cwo_asm_shifted(h, pp, ctypes.byref(sh), a, b, s)

        call.__name__ = "cwo_asm_shifted"
        return self._propagate(call, ANGULAR, u, dx, dy, wavelength, z, precision, nopad, out,
                               stream)


    def autotune(self, u, nz=1, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, kind="asm",
                 precision="f32", nopad=False, stream=None):
        """Pick and keep the fastest schedule for this parameter set (cwo_autotune);
        returns (row_form, zchunk, us_per_plane, layout, col_form)."""
        import torch
        u = self._field(u)
        ny, nx = u.shape
        k = KINDS[kind] if isinstance(kind, str) else int(kind)
        p = make_params(nx, ny, dx, dy, wavelength, z, k, precision, nopad)
        out = torch.empty((int(nz), ny, nx), dtype=torch.complex64, device=u.device)
        t = Tuning()
        st = self._lib.cwo_autotune(self.handle, ctypes.byref(p), int(nz),
                                    ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    self._stream(u, stream), ctypes.byref(t))
        if st != CWO_OK:
            raise CwoError(st, "cwo_autotune")
        return t.row_form, t.zchunk, t.us_per_plane, t.layout, t.col_form

    def set_tuning(self, nx, ny, nz=1, kind="asm", precision="f32", nopad=False, row_form=0,
                   zchunk=0, layout=0, clear=False, col_form=0):
        """Install a schedule for this parameter set (cwo_set_tuning), or remove it."""
        k = KINDS[kind] if isinstance(kind, str) else int(kind)
        p = make_params(nx, ny, 10e-6, None, 633e-9, 0.1, k, precision, nopad)
        t = Tuning(int(row_form), int(zchunk), 0.0, int(layout), int(col_form))
        st = self._lib.cwo_set_tuning(self.handle, ctypes.byref(p), int(nz),
                                      None if clear else ctypes.byref(t))
        if st != CWO_OK:
            raise CwoError(st, "cwo_set_tuning")

    def zstack(self, u, z, dx=10e-6, dy=None, wavelength=633e-9, kind="asm", precision="f32",
               nopad=False, out=None, stream=None, fresnel_tf=False):
        """Propagate one field to every distance in z; returns [nz, ny, nx] planes."""
        import torch
        u = self._field(u)
        ny, nx = u.shape
        zs = [float(v) for v in z]
        k = KINDS[kind] if isinstance(kind, str) else int(kind)
        p = make_params(nx, ny, dx, dy, wavelength, 0.0, k, precision, nopad, fresnel_tf)
        if out is None:
            out = torch.empty((len(zs), ny, nx), dtype=torch.complex64, device=u.device)
        elif (out.dtype != torch.complex64 or tuple(out.shape) != (len(zs), ny, nx)
              or not out.is_contiguous() or out.device != u.device):
            raise ValueError("out must be a contiguous complex64 [nz, ny, nx] tensor")
        zarr = (ctypes.c_double * max(len(zs), 1))(*zs)
        st = self._lib.cwo_zstack(self.handle, ctypes.byref(p), zarr, len(zs),
                                  ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  self._stream(u, stream))
        if st != CWO_OK:
            raise CwoError(st, "cwo_zstack")
        return out

    def gs(self, u, a1, a2, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, iterations=1,
           errors=True, precision="f32", stream=None):
        """Ping-pong iteration in place on u (complex64 [ny, nx]); a1, a2 float32 amplitude
        targets at the two planes. Returns the float32 tensor of E_k (or None)."""
        import torch
        u = self._field(u)
        ny, nx = u.shape
        for a in (a1, a2):
            if (not isinstance(a, torch.Tensor) or a.dtype != torch.float32 or a.shape != u.shape
                    or not a.is_contiguous() or a.device != u.device):
                raise ValueError("amplitude targets must be contiguous float32 [ny, nx] on the "
                                 "field's device")
        p = make_params(nx, ny, dx, dy, wavelength, z, ANGULAR, precision)
        err = torch.empty(max(int(iterations), 1), dtype=torch.float32, device=u.device) \
            if errors else None
        st = self._lib.cwo_gs(self.handle, ctypes.byref(p), ctypes.c_void_p(a1.data_ptr()),
                              ctypes.c_void_p(a2.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                              int(iterations),
                              ctypes.c_void_p(err.data_ptr() if err is not None else 0),
                              self._stream(u, stream))
        if st != CWO_OK:
            raise CwoError(st, "cwo_gs")
        return err[:int(iterations)] if err is not None else None

    # -- serving --------------------------------------------------------------
    def submit(self, kind, u, out, dx=10e-6, dy=None, wavelength=633e-9, z=0.1,
               precision="f32", stream=None):
        """Queue one propagation; returns a ticket. u and out must stay alive (and out
        untouched) until done. The job waits for the work already enqueued on `stream`
        (torch's current stream of u's device by default), so u may come straight from
        asynchronous kernels."""
        u = self._field(u)
        out = self._field(out)
        ny, nx = u.shape
        k = KINDS[kind] if isinstance(kind, str) else int(kind)
        job = Job()
        job.p = make_params(nx, ny, dx, dy, wavelength, z, k, precision)
        job.inp = u.data_ptr()
        job.out = out.data_ptr()
        t = ctypes.c_uint64()
        st = self._lib.cwo_submit_after(self.handle, ctypes.byref(job), self._stream(u, stream),
                                        ctypes.byref(t))
        if st != CWO_OK:
            raise CwoError(st, "cwo_submit_after")
        return t.value

    def memory_held(self):
        """Bytes of device memory the context holds (tables, workspaces, serving slots)."""
        b = ctypes.c_size_t()
        st = self._lib.cwo_memory_held(self.handle, ctypes.byref(b))
        if st != CWO_OK:
            raise CwoError(st, "cwo_memory_held")
        return b.value

    def poll(self, ticket):
        state = ctypes.c_int32()
        st = self._lib.cwo_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(state))
        if st != CWO_OK:
            raise CwoError(st, "cwo_poll")
        return state.value

    def info(self, ticket):
        i = TicketInfo()
        st = self._lib.cwo_ticket_info(self.handle, ctypes.c_uint64(ticket), ctypes.byref(i))
        if st != CWO_OK:
            raise CwoError(st, "cwo_ticket_info")
        return {"state": i.state, "t_submit": i.t_submit, "t_start": i.t_start,
                "t_done": i.t_done, "footprint": i.footprint}

    def release(self, ticket):
        st = self._lib.cwo_release(self.handle, ctypes.c_uint64(ticket))
        if st != CWO_OK:
            raise CwoError(st, "cwo_release")

    def drain(self):
        st = self._lib.cwo_drain(self.handle)
        if st != CWO_OK:
            raise CwoError(st, "cwo_drain")

    def batch(self, jobs, stream=None):
        """Run a list of (kind, u, out, dict(dx=, dy=, wavelength=, z=, ...)) jobs in order."""
        if not jobs:
            return
        arr = (Job * len(jobs))()
        first = None
        for i, (kind, u, out, kw) in enumerate(jobs):
            u = self._field(u)
            out = self._field(out)
            first = first if first is not None else u
            ny, nx = u.shape
            k = KINDS[kind] if isinstance(kind, str) else int(kind)
            arr[i].p = make_params(nx, ny, kw.get("dx", 10e-6), kw.get("dy"),
                                   kw.get("wavelength", 633e-9), kw.get("z", 0.1), k,
                                   kw.get("precision", "f32"), kw.get("nopad", False),
                                   kw.get("fresnel_tf", False))
            arr[i].inp = u.data_ptr()
            arr[i].out = out.data_ptr()
        st = self._lib.cwo_batch(self.handle, arr, len(jobs), self._stream(first, stream))
        if st != CWO_OK:
            raise CwoError(st, "cwo_batch")


_default = {}


def fresnel_fourier_pitch(nx, ny, dx, dy=None, wavelength=633e-9, z=0.1):
    """(dx2, dy2): destination pitch of the Fresnel Fourier form [m]."""
    p = make_params(nx, ny, dx, dy, wavelength, z, FRESNEL_FOURIER, "f32", False)
    a, b = ctypes.c_double(), ctypes.c_double()
    st = load().cwo_fresnel_fourier_pitch(ctypes.byref(p), ctypes.byref(a), ctypes.byref(b))
    if st != CWO_OK:
        raise CwoError(st, "cwo_fresnel_fourier_pitch")
    return a.value, b.value


def band_limit(nx, ny, dx, dy=None, wavelength=633e-9, z=0.1, nopad=False):
    """(wx, wy): full widths [1/m] of the on-axis band limit (cwo_band_limit)."""
    p = make_params(nx, ny, dx, dy, wavelength, z, ANGULAR, "f32", nopad)
    sh = Shift()
    st = load().cwo_band_limit(ctypes.byref(p), ctypes.byref(sh))
    if st != CWO_OK:
        raise CwoError(st, "cwo_band_limit")
    return sh.wx, sh.wy


def context(device: int = 0) -> Context:
    """The process-wide default context of a device."""
    c = _default.get(device)
    if c is None:
        c = Context(device)
        _default[device] = c
    return c


def asm(u, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, **kw):
    return context(u.device.index or 0).asm(u, dx, dy, wavelength, z, **kw)


def fresnel(u, dx=10e-6, dy=None, wavelength=633e-9, z=0.1, **kw):
    return context(u.device.index or 0).fresnel(u, dx, dy, wavelength, z, **kw)


def algorithmic_bytes(nx: int, ny: int, intermediate_bytes: int = 8) -> int:
    """Bytes one padded propagation must move: read the field, write and re-read the
    Ny x 2Nx spectrum plane twice (row pass, column pass), write the field."""
    mx = 2 * nx
    field = 8 * nx * ny
    plane = intermediate_bytes * ny * mx
    return field + plane + 2 * plane + plane + field  # row, column (r+w), row-inverse (r)


__all__ = ["Context", "CwoError", "Params", "make_params", "check_params", "context", "asm",
           "fresnel", "load", "strerror", "algorithmic_bytes", "math"]
