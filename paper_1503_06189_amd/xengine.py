"""ctypes binding of libxengine.so (the HIP path), same names as the C ABI.

Argument marshalling only: every step of the correlation runs in the
library's kernels.  PyTorch supplies device memory and the current stream.
There is no fallback: if the library is missing, importing the functions
below raises :class:`XEngineUnavailable`.
"""

from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxengine.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "xengine.h")

XE_OK = 0
XE_ERR_ARG = -1
XE_ERR_ALIGN = -2
XE_ERR_OVERFLOW = -3
XE_ERR_WORKSPACE = -4
XE_ERR_HIP = -5
XE_ERR_UNSUPPORTED = -6
XE_ERR_NO_DEVICE = -7
XE_MAX_N = 4096
XE_MAX_SAMPLES = 16777215
XE_DEVICE_NONE = -1

#: every function the header declares
EXPORTS = ("xe_create", "xe_destroy", "xe_status_string", "xe_last_error",
           "xe_correlate_frame", "xe_accumulate", "xe_normalize",
           "xe_accumulate_batch", "xe_plan_query")


class XEngineUnavailable(RuntimeError):
    """libxengine.so is not built or cannot be loaded."""


class XEngineError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"xengine status {status}: {msg}")
        self.status = status


class PlanInfo(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("splits", ctypes.c_int32), ("steps_per_split", ctypes.c_int32),
                ("workgroups", ctypes.c_int64), ("mfma_tiles", ctypes.c_int64)]


class Instance(ctypes.Structure):
    _fields_ = [("packed", ctypes.c_void_p), ("loss_mask", ctypes.c_void_p),
                ("N", ctypes.c_int32), ("F", ctypes.c_int32), ("T", ctypes.c_int32),
                ("B", ctypes.c_int32), ("vis", ctypes.c_void_p), ("count", ctypes.c_void_p)]


_lib = None
_lib_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    """The loaded library (loaded once)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise XEngineUnavailable(
                    f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                    "python paper_1503_06189_amd/build.py")
            try:
                L = ctypes.CDLL(LIB_PATH)
            except OSError as e:
                raise XEngineUnavailable(str(e)) from e
            i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
            L.xe_create.restype = i32
            L.xe_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_size_t]
            L.xe_destroy.restype = i32
            L.xe_destroy.argtypes = [vp]
            L.xe_status_string.restype = ctypes.c_char_p
            L.xe_status_string.argtypes = [i32]
            L.xe_last_error.restype = ctypes.c_char_p
            L.xe_last_error.argtypes = [vp]
            for name in ("xe_correlate_frame", "xe_accumulate"):
                fn = getattr(L, name)
                fn.restype = i32
                fn.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, vp, vp]
            L.xe_normalize.restype = i32
            L.xe_normalize.argtypes = [vp, vp, vp, i32, i32, vp, vp]
            L.xe_accumulate_batch.restype = i32
            L.xe_accumulate_batch.argtypes = [vp, ctypes.POINTER(Instance), i32, vp]
            L.xe_plan_query.restype = i32
            L.xe_plan_query.argtypes = [i32, i32, i32, i32, i32, ctypes.POINTER(PlanInfo)]
            _lib = L
        return _lib


def status_string(s: int) -> str:
    return lib().xe_status_string(s).decode()


def plan_query(N: int, F: int, T: int, B: int = 256, n_cu: int = 256) -> PlanInfo:
    info = PlanInfo()
    s = lib().xe_plan_query(N, F, T, B, n_cu, ctypes.byref(info))
    if s != XE_OK:
        raise XEngineError(s, status_string(s))
    return info


class Handle:
    """Owns one xe_handle (and its pre-allocated workspace)."""

    def __init__(self, device: Optional[int] = None, workspace_bytes: int = 0):
        if device is None:
            import torch
            device = torch.cuda.current_device()
        self.device = device
        h = ctypes.c_void_p()
        s = lib().xe_create(ctypes.byref(h), device, workspace_bytes)
        if s != XE_OK:
            raise XEngineError(s, status_string(s))
        self._h = h

    @property
    def ptr(self):
        return self._h

    def check(self, s: int) -> None:
        if s != XE_OK:
            msg = lib().xe_last_error(self._h).decode() or status_string(s)
            raise XEngineError(s, msg)

    def close(self) -> None:
        if self._h:
            lib().xe_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles = {}


def default_handle(device: Optional[int] = None) -> Handle:
    import torch
    if device is None:
        device = torch.cuda.current_device()
    h = _handles.get(device)
    if h is None:
        h = _handles[device] = Handle(device)
    return h


# ---------------------------------------------------------------------------
# tensor-level API
# ---------------------------------------------------------------------------

def _stream_ptr(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_frame(packed, mask, B):
    import torch
    if packed.dtype != torch.uint8 or packed.dim() != 3 or not packed.is_cuda:
        raise ValueError("packed must be a CUDA uint8 tensor [T, F, N]")
    if not packed.is_contiguous():
        raise ValueError("packed must be contiguous")
    T, F, N = packed.shape
    if mask is not None:
        nblk = (T + B - 1) // B
        if mask.dtype != torch.uint8 or tuple(mask.shape) != (F, nblk) or \
                not mask.is_cuda or not mask.is_contiguous():
            raise ValueError(f"mask must be a contiguous CUDA uint8 tensor [{F}, {nblk}]")
    return T, F, N


def new_accumulators(N: int, F: int, device=None):
    import torch
    P = N * (N + 1) // 2
    dev = device if device is not None else torch.device("cuda")
    return (torch.zeros((F, P, 2), dtype=torch.int32, device=dev),
            torch.zeros((F,), dtype=torch.int64, device=dev))


def _check_acc(vis, count, N, F):
    import torch
    P = N * (N + 1) // 2
    if vis.dtype != torch.int32 or tuple(vis.shape) != (F, P, 2) or not vis.is_contiguous():
        raise ValueError(f"vis must be contiguous int32 [{F}, {P}, 2]")
    if count.dtype != torch.int64 or tuple(count.shape) != (F,) or not count.is_contiguous():
        raise ValueError(f"count must be contiguous int64 [{F}]")


def correlate_frame(packed, mask=None, B: int = 256, vis=None, count=None,
                    handle: Optional[Handle] = None, stream=None):
    """V and n of one frame (overwrites ``vis``/``count`` when given)."""
    T, F, N = _check_frame(packed, mask, B)
    if vis is None or count is None:
        vis, count = new_accumulators(N, F, packed.device)
    _check_acc(vis, count, N, F)
    h = handle or default_handle(packed.device.index)
    h.check(lib().xe_correlate_frame(
        h.ptr, ctypes.c_void_p(packed.data_ptr()),
        ctypes.c_void_p(mask.data_ptr() if mask is not None else None),
        N, F, T, B, ctypes.c_void_p(vis.data_ptr()), ctypes.c_void_p(count.data_ptr()),
        _stream_ptr(stream)))
    return vis, count


def accumulate(packed, mask, B: int, vis, count, handle: Optional[Handle] = None,
               stream=None):
    """vis += V(frame), count += n(frame), in place on the device."""
    T, F, N = _check_frame(packed, mask, B)
    _check_acc(vis, count, N, F)
    h = handle or default_handle(packed.device.index)
    h.check(lib().xe_accumulate(
        h.ptr, ctypes.c_void_p(packed.data_ptr()),
        ctypes.c_void_p(mask.data_ptr() if mask is not None else None),
        N, F, T, B, ctypes.c_void_p(vis.data_ptr()), ctypes.c_void_p(count.data_ptr()),
        _stream_ptr(stream)))
    return vis, count


def normalize(vis, count, out=None, handle: Optional[Handle] = None, stream=None):
    """float32 V / n per channel (0 where n == 0)."""
    import torch
    F, P, two = vis.shape
    N = int(round(((8 * P + 1) ** 0.5 - 1) / 2))
    if two != 2 or N * (N + 1) // 2 != P:
        raise ValueError("vis must be [F, N(N+1)/2, 2]")
    _check_acc(vis, count, N, F)
    if out is None:
        out = torch.empty((F, P, 2), dtype=torch.float32, device=vis.device)
    if out.dtype != torch.float32 or tuple(out.shape) != (F, P, 2) or not out.is_contiguous():
        raise ValueError("out must be contiguous float32 [F, P, 2]")
    h = handle or default_handle(vis.device.index)
    h.check(lib().xe_normalize(h.ptr, ctypes.c_void_p(vis.data_ptr()),
                               ctypes.c_void_p(count.data_ptr()), N, F,
                               ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def accumulate_batch(items: Sequence[Tuple], handle: Optional[Handle] = None, stream=None):
    """items: (packed, mask, B, vis, count) per instance; one library call."""
    arr = (Instance * len(items))()
    dev = None
    for k, (packed, mask, B, vis, count) in enumerate(items):
        T, F, N = _check_frame(packed, mask, B)
        _check_acc(vis, count, N, F)
        dev = packed.device.index
        arr[k] = Instance(packed.data_ptr(), mask.data_ptr() if mask is not None else None,
                          N, F, T, B, vis.data_ptr(), count.data_ptr())
    h = handle or default_handle(dev)
    h.check(lib().xe_accumulate_batch(h.ptr, arr, len(items), _stream_ptr(stream)))
