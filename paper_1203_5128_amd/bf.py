"""Thin ctypes binding of libbf.so (include/bf.h).

Argument marshalling only: every step of the filter runs in the HIP kernels of
libbf.so.  PyTorch supplies device memory and streams.  If the library is
missing the import fails loudly; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbf.so")

BF_OK = 0
BF_ERR_INVALID_ARG = 1
BF_ERR_UNSUPPORTED = 2
BF_ERR_OUT_OF_MEMORY = 3
BF_ERR_DEVICE = 4
BF_ERR_NOT_FINITE = 5
BF_ERR_RANGE = 6

BF_U8, BF_U16, BF_F32 = 0, 1, 2
BF_T_GLOBAL, BF_T_LOCAL = 0, 1
BF_BLUR_AUTO = 0
BF_BLUR_IIR_F32 = 1
BF_BLUR_TOEPLITZ_F16 = 2
BF_BLUR_TOEPLITZ_BF16 = 3
BF_BLUR_TOEPLITZ_F16X2 = 4
BF_BLUR_TOEPLITZ_BF16X2 = 5

DTYPES = {"u8": BF_U8, "u16": BF_U16, "f32": BF_F32}
BLURS = {"auto": BF_BLUR_AUTO, "iir_f32": BF_BLUR_IIR_F32, "toeplitz_f16": BF_BLUR_TOEPLITZ_F16,
         "toeplitz_bf16": BF_BLUR_TOEPLITZ_BF16, "toeplitz_f16x2": BF_BLUR_TOEPLITZ_F16X2,
         "toeplitz_bf16x2": BF_BLUR_TOEPLITZ_BF16X2}
BLUR_NAMES = {v: k for k, v in BLURS.items()}

EXPORTS = ["bf_plan", "bf_filter", "bf_filter_batch", "bf_dynamic_range", "bf_profile", "bf_profile_read",
           "bf_plan_destroy", "bf_status_string", "bf_last_error_detail", "bf_filter_noalloc"]
STAGES = ["range", "v_iir", "v_toeplitz", "h_combine"]


class bf_params(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("in_pitch", ctypes.c_int64), ("out_pitch", ctypes.c_int64),
                ("dtype", ctypes.c_int), ("sigma_s", ctypes.c_double),
                ("sigma_r", ctypes.c_double), ("eps", ctypes.c_double),
                ("radius", ctypes.c_int32), ("t_mode", ctypes.c_int),
                ("t_value", ctypes.c_double), ("value_range", ctypes.c_double),
                ("blur", ctypes.c_int), ("spatial", ctypes.c_int), ("range_kernel", ctypes.c_int),
                ("patch_size", ctypes.c_int32), ("patch_dy", ctypes.c_int32 * 4), ("patch_dx", ctypes.c_int32 * 4)]


class bf_report(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("T_used", ctypes.c_int32), ("N", ctypes.c_int32),
                ("M", ctypes.c_int32), ("kept", ctypes.c_int32), ("pairs", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("q_nonpos", ctypes.c_int64), ("ms", ctypes.c_float)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["variant"] = BLUR_NAMES.get(d["variant"], d["variant"])
        return d


class BFError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{bf_status_string(status)} ({status}): {detail}")
        self.status = status
        self.detail = detail


_lib = None


def lib():
    """Load libbf.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.bf_plan.argtypes = [ctypes.POINTER(bf_params), ctypes.c_int32, ctypes.POINTER(P)]
        L.bf_plan.restype = ctypes.c_int
        L.bf_filter.argtypes = [P, P, P, P, ctypes.POINTER(bf_report)]
        L.bf_filter.restype = ctypes.c_int
        L.bf_filter_noalloc.argtypes = [P, P, P, P, ctypes.POINTER(bf_report)]
        L.bf_filter_noalloc.restype = ctypes.c_int
        L.bf_filter_batch.argtypes = [P, ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(P), P,
                                      ctypes.POINTER(bf_report)]
        L.bf_filter_batch.restype = ctypes.c_int
        L.bf_dynamic_range.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_double)]
        L.bf_dynamic_range.restype = ctypes.c_int
        L.bf_profile.argtypes = [P, ctypes.c_int32]
        L.bf_profile.restype = ctypes.c_int
        L.bf_profile_read.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.bf_profile_read.restype = ctypes.c_int
        L.bf_plan_destroy.argtypes = [P]
        L.bf_plan_destroy.restype = None
        L.bf_status_string.argtypes = [ctypes.c_int]
        L.bf_status_string.restype = ctypes.c_char_p
        L.bf_last_error_detail.argtypes = []
        L.bf_last_error_detail.restype = ctypes.c_char_p
        _lib = L
    return _lib


def bf_status_string(status: int) -> str:
    return lib().bf_status_string(int(status)).decode()


def bf_last_error_detail() -> str:
    return lib().bf_last_error_detail().decode()


def _check(status: int):
    if status != BF_OK:
        raise BFError(status, bf_last_error_detail())


SPATIALS = {"gaussian": 0, "box": 1, "gaussian_fir": 2}
RANGE_KERNELS = {"raised_cosine": 0, "polynomial": 1}


def make_params(H, W, dtype="u8", sigma_s=3.0, sigma_r=30.0, eps=1e-3, radius=0, t_mode="local",
                t_value=0.0, value_range=0.0, blur="iir_f32", in_pitch=0, out_pitch=0,
                spatial="gaussian", range_kernel="raised_cosine", patch=None) -> bf_params:
    """patch: None for the bilateral filter, or the non-local-means patch as
    a list of (dy, dx) offsets starting with (0, 0)."""
    p = bf_params()
    p.height, p.width = int(H), int(W)
    p.in_pitch, p.out_pitch = int(in_pitch), int(out_pitch)
    p.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    p.sigma_s, p.sigma_r, p.eps = float(sigma_s), float(sigma_r), float(eps)
    p.radius = int(radius)
    p.t_mode = {"global": BF_T_GLOBAL, "local": BF_T_LOCAL}[t_mode] if isinstance(t_mode, str) else int(t_mode)
    p.t_value, p.value_range = float(t_value), float(value_range)
    p.blur = BLURS[blur] if isinstance(blur, str) else int(blur)
    p.spatial = SPATIALS[spatial] if isinstance(spatial, str) else int(spatial)
    p.range_kernel = RANGE_KERNELS[range_kernel] if isinstance(range_kernel, str) else int(range_kernel)
    if patch:
        p.patch_size = len(patch)
        for k, (dy, dx) in enumerate(patch[:4]):
            p.patch_dy[k], p.patch_dx[k] = int(dy), int(dx)
    return p


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def bf_plan(params) -> int:
    """Create a plan from one bf_params or a list of them; returns the handle."""
    if isinstance(params, bf_params):
        params = [params]
    arr = (bf_params * len(params))(*params)
    h = ctypes.c_void_p()
    _check(lib().bf_plan(arr, len(params), ctypes.byref(h)))
    return h.value


def bf_filter(plan: int, d_in: int, d_out: int, stream=None, report: bool = True):
    rep = bf_report() if report else None
    st = lib().bf_filter(plan, d_in, d_out, _stream_handle(stream),
                         ctypes.byref(rep) if rep is not None else None)
    _check(st)
    return rep.as_dict() if rep is not None else None


def bf_filter_noalloc(plan: int, d_in: int, d_out: int, stream=None, report: bool = True):
    rep = bf_report() if report else None
    st = lib().bf_filter_noalloc(plan, d_in, d_out, _stream_handle(stream),
                                 ctypes.byref(rep) if rep is not None else None)
    _check(st)
    return rep.as_dict() if rep is not None else None


def bf_filter_batch(plan: int, d_ins, d_outs, stream=None, report: bool = True):
    n = len(d_ins)
    ins = (ctypes.c_void_p * n)(*d_ins)
    outs = (ctypes.c_void_p * n)(*d_outs)
    reps = (bf_report * n)() if report else None
    _check(lib().bf_filter_batch(plan, n, ins, outs, _stream_handle(stream), reps))
    return [r.as_dict() for r in reps] if reps is not None else None


def bf_dynamic_range(plan: int, d_in: int, stream=None) -> float:
    T = ctypes.c_double()
    _check(lib().bf_dynamic_range(plan, d_in, _stream_handle(stream), ctypes.byref(T)))
    return T.value


def bf_profile(plan: int, enable: bool):
    _check(lib().bf_profile(plan, int(bool(enable))))


def bf_profile_read(plan: int):
    """{stage: (milliseconds, launches)} since the last read."""
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_int64 * len(STAGES))()
    _check(lib().bf_profile_read(plan, ms, n))
    return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}


def bf_plan_destroy(plan: int):
    lib().bf_plan_destroy(plan)


# ----------------------------------------------------------- torch helpers
_TORCH_DTYPES = {BF_U8: ("uint8",), BF_U16: ("uint16", "int16"), BF_F32: ("float32",)}


def _check_tensor(name, t, H, W, pitch, dts):
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dim() != 2 or tuple(t.shape) != (H, W):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, the plan expects ({H}, {W})")
    if str(t.dtype).replace("torch.", "") not in dts:
        raise ValueError(f"{name} has dtype {t.dtype}, the plan expects {' or '.join(dts)}")
    if t.stride(1) != 1 or (H > 1 and t.stride(0) != (pitch if pitch > 0 else W)):
        raise ValueError(f"{name} strides {t.stride()} do not match the plan's pitch "
                         f"({pitch if pitch > 0 else W} elements per row, unit column stride)")


def check_tensors(p: bf_params, img, out=None):
    """The buffers handed to the C ABI must be what the plan's parameters
    describe: the library reads H x W elements of the input type with the
    plan's pitch and writes float32 with the output pitch, so a wrong shape,
    dtype, stride or device would be read or written out of place.  Raises
    ValueError on any mismatch (nothing is launched)."""
    _check_tensor("input", img, p.height, p.width, p.in_pitch, _TORCH_DTYPES[p.dtype])
    if out is not None:
        _check_tensor("output", out, p.height, p.width, p.out_pitch, ("float32",))
        if img.device != out.device:
            raise ValueError("input and output are on different devices")


@dataclass
class Plan:
    """Owns a plan handle; images are torch tensors on the GPU."""
    handle: int
    params: tuple = ()

    @classmethod
    def create(cls, params):
        plist = [params] if isinstance(params, bf_params) else list(params)
        return cls(bf_plan(plist), tuple(plist))

    def filter(self, img, out=None, stream=None, report=True):
        import torch
        if out is None:
            out = torch.empty(img.shape, dtype=torch.float32, device=img.device)
        if self.params:
            check_tensors(self.params[0], img, out)
        rep = bf_filter(self.handle, img.data_ptr(), out.data_ptr(), stream, report)
        return out, rep

    def filter_noalloc(self, img, out, stream=None, report=True):
        """bf_filter_noalloc: the caller passes the output buffer; the call
        itself allocates nothing on the device."""
        if self.params:
            check_tensors(self.params[0], img, out)
        rep = bf_filter_noalloc(self.handle, img.data_ptr(), out.data_ptr(), stream, report)
        return out, rep

    def filter_batch(self, imgs, outs=None, stream=None, report=True):
        import torch
        if outs is None:
            outs = [torch.empty(i.shape, dtype=torch.float32, device=i.device) for i in imgs]
        if len(imgs) != len(outs) or (self.params and len(imgs) > len(self.params)):
            raise ValueError("the number of inputs and outputs must match and not exceed the plan's images")
        for i, (a, b) in enumerate(zip(imgs, outs)):
            if self.params:
                check_tensors(self.params[i], a, b)
        reps = bf_filter_batch(self.handle, [i.data_ptr() for i in imgs], [o.data_ptr() for o in outs],
                               stream, report)
        return outs, reps

    def profile(self, enable=True):
        bf_profile(self.handle, enable)

    def profile_read(self):
        return bf_profile_read(self.handle)

    def dynamic_range(self, img, stream=None):
        if self.params:
            check_tensors(self.params[0], img)
        return bf_dynamic_range(self.handle, img.data_ptr(), stream)

    def close(self):
        if self.handle:
            bf_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def torch_dtype_name(t) -> str:
    import torch
    return {torch.uint8: "u8", torch.uint16: "u16", torch.int16: "u16", torch.float32: "f32"}[t.dtype]


def bilateral_filter(img, sigma_s, sigma_r, eps=1e-3, radius=0, t_mode="local", t_value=0.0,
                     value_range=0.0, blur="iir_f32", stream=None):
    """Filter one 2-D torch tensor (uint8, uint16 or float32) on the GPU."""
    H, W = img.shape
    p = make_params(H, W, torch_dtype_name(img), sigma_s, sigma_r, eps, radius, t_mode, t_value,
                    value_range, blur)
    plan = Plan.create(p)
    try:
        return plan.filter(img.contiguous(), stream=stream)
    finally:
        plan.close()
