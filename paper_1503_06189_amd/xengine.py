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
import weakref
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
XE_GEOM_AUTO = 0
XE_GEOM_SUPER = 1
XE_GEOM_HALVES = 2
#: tile geometries of frames with N <= 128, by name
GEOMETRIES = {"auto": XE_GEOM_AUTO, "super": XE_GEOM_SUPER, "halves": XE_GEOM_HALVES}

#: every function the header declares
EXPORTS = ("xe_create", "xe_destroy", "xe_status_string", "xe_last_error", "xe_set_geometry",
           "xe_correlate_frame", "xe_accumulate", "xe_normalize",
           "xe_accumulate_batch", "xe_batch_plan", "xe_batch_run", "xe_batch_release",
           "xe_batch_query", "xe_plan_query",
           "xe_flag_accumulate", "xe_apply_flags", "xe_normalize_flagged",
           "xe_assemble_frame", "xe_time_shift", "xe_accumulate_noalloc")


class XEngineUnavailable(RuntimeError):
    """libxengine.so is not built or cannot be loaded."""


class XEngineError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"xengine status {status}: {msg}")
        self.status = status


# Samples integrated into each accumulator since it was last cleared.  int32
# sums are exact for at most XE_MAX_SAMPLES accumulated samples (|Re V| <= 128
# per sample); calls that would pass that bound are refused before launching,
# and a call's samples are charged only once the library has accepted it.
# correlate_frame and new_accumulators start a count; callers that clear sums
# themselves call reset_integration.  Replays of a captured graph bypass this
# bookkeeping.
#
# An entry is keyed by the sums' device address but holds a weak reference to
# the tensor that owns the count: once that tensor is freed the entry is
# stale, so a new tensor that the allocator places at the same address starts
# from 0 instead of inheriting the old count.  A view of a live accumulator
# (same address) shares its count.
_integrated = {}
_integrated_lock = threading.Lock()


def _entry_count(key: int) -> int:
    e = _integrated.get(key)
    if e is None:
        return 0
    ref, n = e
    t = ref()
    if t is None or t.data_ptr() != key:
        del _integrated[key]
        return 0
    return n


def _set_count(vis, n: int) -> None:
    key = vis.data_ptr()
    e = _integrated.get(key)
    if e is not None:
        owner = e[0]()
        if owner is not None and owner.data_ptr() == key:
            _integrated[key] = (e[0], n)
            return
    _integrated[key] = (weakref.ref(vis), n)


def reset_integration(vis) -> None:
    """Mark the sums in ``vis`` as cleared (0 samples integrated)."""
    with _integrated_lock:
        _set_count(vis, 0)


def integrated_samples(vis) -> int:
    """Samples integrated into ``vis`` since it was last cleared."""
    with _integrated_lock:
        return _entry_count(vis.data_ptr())


def snapshot(vis, count, stream=None) -> dict:
    """Checkpoint of an integration in progress: its sums and counts copied to
    host memory, with the samples integrated so far.  The integration state
    is exactly the output plus the counts (Sec. II-C), so restoring the
    snapshot into any accumulators of the same shape and continuing gives
    the uninterrupted result (accumulation is linear in time)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    with torch.cuda.stream(s):
        v = vis.to("cpu", non_blocking=False)
        c = count.to("cpu", non_blocking=False)
    return {"vis": v.numpy(), "count": c.numpy(), "samples": integrated_samples(vis)}


def restore(state: dict, vis, count, stream=None) -> None:
    """Load a snapshot into ``vis``/``count`` (same shapes) on the device.
    Raises ValueError for a snapshot of another shape or element type, or
    whose sample count lies outside 0 .. the int32 integration bound."""
    import numpy as np
    import torch
    sv, sc = np.asarray(state["vis"]), np.asarray(state["count"])
    if sv.dtype != np.int32 or sc.dtype != np.int64:
        raise ValueError(f"snapshot types {sv.dtype}/{sc.dtype}, expected int32/int64")
    samples = int(state["samples"])
    if not 0 <= samples <= XE_MAX_SAMPLES:
        raise ValueError(f"snapshot of {samples} samples, outside 0..{XE_MAX_SAMPLES}")
    v = torch.from_numpy(np.ascontiguousarray(sv))
    c = torch.from_numpy(np.ascontiguousarray(sc))
    if tuple(v.shape) != tuple(vis.shape) or tuple(c.shape) != tuple(count.shape):
        raise ValueError("snapshot shape differs from the accumulators")
    s = torch.cuda.current_stream() if stream is None else stream
    with torch.cuda.stream(s):
        vis.copy_(v)
        count.copy_(c)
    s.synchronize()
    with _integrated_lock:
        _set_count(vis, samples)


def _charge(pairs, call):
    """Run ``call`` (which returns an xe_status and raises on failure) only if
    adding T samples to each (vis, T) keeps every count within the bound;
    the counts are updated after the call succeeded."""
    with _integrated_lock:
        new = {}
        owners = {}
        for vis, T in pairs:
            key = vis.data_ptr()
            n = new.get(key, _entry_count(key)) + int(T)
            if n > XE_MAX_SAMPLES:
                raise XEngineError(XE_ERR_OVERFLOW,
                                   f"{n} samples would exceed the int32 integration bound "
                                   f"{XE_MAX_SAMPLES}; normalise and clear the sums first")
            new[key] = n
            owners[key] = vis
    result = call()
    with _integrated_lock:
        for key, n in new.items():
            _set_count(owners[key], n)
    return result


class PlanInfo(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("splits", ctypes.c_int32), ("steps_per_split", ctypes.c_int32),
                ("workgroups", ctypes.c_int64), ("mfma_tiles", ctypes.c_int64)]


class Instance(ctypes.Structure):
    _fields_ = [("packed", ctypes.c_void_p), ("loss_mask", ctypes.c_void_p),
                ("N", ctypes.c_int32), ("F", ctypes.c_int32), ("T", ctypes.c_int32),
                ("B", ctypes.c_int32), ("vis", ctypes.c_void_p), ("count", ctypes.c_void_p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("items", ctypes.c_int64), ("instances", ctypes.c_int32),
                ("unaligned", ctypes.c_int32), ("chunk_steps", ctypes.c_int32),
                ("partial_bytes", ctypes.c_int64)]


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
            L.xe_set_geometry.restype = i32
            L.xe_set_geometry.argtypes = [vp, i32]
            for name in ("xe_correlate_frame", "xe_accumulate"):
                fn = getattr(L, name)
                fn.restype = i32
                fn.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, vp, vp]
            L.xe_accumulate_noalloc.restype = i32
            L.xe_accumulate_noalloc.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, vp]
            L.xe_normalize.restype = i32
            L.xe_normalize.argtypes = [vp, vp, vp, i32, i32, vp, vp]
            L.xe_flag_accumulate.restype = i32
            L.xe_flag_accumulate.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, vp]
            L.xe_apply_flags.restype = i32
            L.xe_apply_flags.argtypes = [vp, vp, vp, i32, i32, i32, vp]
            L.xe_normalize_flagged.restype = i32
            L.xe_normalize_flagged.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp, vp]
            L.xe_time_shift.restype = i32
            L.xe_time_shift.argtypes = [vp, vp, vp, vp, i32, i32, i32, vp, vp, vp]
            L.xe_assemble_frame.restype = i32
            L.xe_assemble_frame.argtypes = [vp, vp, ctypes.c_int64, i32, i32, i32,
                                            ctypes.c_int64, i32, vp, vp, vp, vp, vp]
            L.xe_accumulate_batch.restype = i32
            L.xe_accumulate_batch.argtypes = [vp, ctypes.POINTER(Instance), i32, vp]
            L.xe_batch_plan.restype = i32
            L.xe_batch_plan.argtypes = [vp, ctypes.POINTER(Instance), i32, i32,
                                        ctypes.POINTER(i32)]
            L.xe_batch_run.restype = i32
            L.xe_batch_run.argtypes = [vp, i32, vp]
            L.xe_batch_release.restype = i32
            L.xe_batch_release.argtypes = [vp, i32]
            L.xe_batch_query.restype = i32
            L.xe_batch_query.argtypes = [ctypes.POINTER(Instance), i32, i32, i32,
                                         ctypes.POINTER(BatchInfo)]
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
        self.geometry = XE_GEOM_AUTO

    @property
    def ptr(self):
        return self._h

    def check(self, s: int) -> None:
        if s != XE_OK:
            msg = lib().xe_last_error(self._h).decode() or status_string(s)
            raise XEngineError(s, msg)

    def set_geometry(self, geometry) -> None:
        """Tile geometry of frames with N <= 128 for later calls and plans:
        "auto", "super" or "halves", or an XE_GEOM_* value."""
        g = GEOMETRIES[geometry] if isinstance(geometry, str) else int(geometry)
        self.check(lib().xe_set_geometry(self._h, g))
        self.geometry = g

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
    vis = torch.zeros((F, P, 2), dtype=torch.int32, device=dev)
    reset_integration(vis)
    return vis, torch.zeros((F,), dtype=torch.int64, device=dev)


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
    with _integrated_lock:
        _set_count(vis, T)
    return vis, count


def accumulate(packed, mask, B: int, vis, count, handle: Optional[Handle] = None,
               stream=None):
    """vis += V(frame), count += n(frame), in place on the device."""
    T, F, N = _check_frame(packed, mask, B)
    _check_acc(vis, count, N, F)
    h = handle or default_handle(packed.device.index)
    _charge([(vis, T)], lambda: h.check(lib().xe_accumulate(
        h.ptr, ctypes.c_void_p(packed.data_ptr()),
        ctypes.c_void_p(mask.data_ptr() if mask is not None else None),
        N, F, T, B, ctypes.c_void_p(vis.data_ptr()), ctypes.c_void_p(count.data_ptr()),
        _stream_ptr(stream))))
    return vis, count


def accumulate_noalloc(packed, mask, B: int, vis, count, stream=None):
    """As :func:`accumulate`, through xe_accumulate_noalloc: no handle, no
    device allocation (time-chunk sums in the library's static scratch
    array of the current device).  Calls overlapping on one GPU race."""
    import torch
    T, F, N = _check_frame(packed, mask, B)
    _check_acc(vis, count, N, F)
    if torch.cuda.current_device() != packed.device.index:
        raise ValueError("the frame must be on the current device")

    def call():
        s = lib().xe_accumulate_noalloc(
            ctypes.c_void_p(packed.data_ptr()),
            ctypes.c_void_p(mask.data_ptr() if mask is not None else None),
            N, F, T, B, ctypes.c_void_p(vis.data_ptr()), ctypes.c_void_p(count.data_ptr()),
            _stream_ptr(stream))
        if s != XE_OK:
            raise XEngineError(s, status_string(s))
    _charge([(vis, T)], call)
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


# -- per-input flags (Sec. II-C) ---------------------------------------------

def _check_flags(flags, F, T, N):
    import torch
    W = (N + 31) // 32
    if flags.dtype != torch.int32 or tuple(flags.shape) != (F, T, W) or \
            not flags.is_cuda or not flags.is_contiguous():
        raise ValueError(f"flags must be a contiguous CUDA int32 tensor [{F}, {T}, {W}] "
                         "holding the uint32 bit-fields")


def new_flag_counts(N: int, F: int, device=None):
    """Zeroed int32 [F, P] intersection counts for flag_accumulate."""
    import torch
    dev = device if device is not None else torch.device("cuda")
    return torch.zeros((F, N * (N + 1) // 2), dtype=torch.int32, device=dev)


def flag_accumulate(flags, mask, B: int, N: int, dcount, handle: Optional[Handle] = None,
                    stream=None):
    """dcount += per-baseline flag intersections of one frame (diagonal: the
    per-input flag counters); ``flags`` int32 [F, T, ceil(N/32)] bit-fields."""
    import torch
    F, T = int(flags.shape[0]), int(flags.shape[1])
    _check_flags(flags, F, T, N)
    if mask is not None:
        nblk = (T + B - 1) // B
        if mask.dtype != torch.uint8 or tuple(mask.shape) != (F, nblk) or \
                not mask.is_cuda or not mask.is_contiguous():
            raise ValueError(f"mask must be a contiguous CUDA uint8 tensor [{F}, {nblk}]")
    P = N * (N + 1) // 2
    if dcount.dtype != torch.int32 or tuple(dcount.shape) != (F, P) or \
            not dcount.is_contiguous():
        raise ValueError(f"dcount must be contiguous int32 [{F}, {P}]")
    h = handle or default_handle(flags.device.index)
    h.check(lib().xe_flag_accumulate(
        h.ptr, ctypes.c_void_p(flags.data_ptr()),
        ctypes.c_void_p(mask.data_ptr() if mask is not None else None),
        N, F, T, B, ctypes.c_void_p(dcount.data_ptr()), _stream_ptr(stream)))
    return dcount


def apply_flags(packed, flags, handle: Optional[Handle] = None, stream=None):
    """Zero the flagged points of ``packed`` in place (byte 0x88)."""
    T, F, N = _check_frame(packed, None, 1)
    _check_flags(flags, F, T, N)
    h = handle or default_handle(packed.device.index)
    h.check(lib().xe_apply_flags(h.ptr, ctypes.c_void_p(packed.data_ptr()),
                                 ctypes.c_void_p(flags.data_ptr()), N, F, T,
                                 _stream_ptr(stream)))
    return packed


def normalize_flagged(vis, count, dcount, out=None, n_out=None,
                      handle: Optional[Handle] = None, stream=None):
    """float32 V / n_ij per baseline, n_ij = count - d_ii - d_jj + d_ij
    (0 where n_ij == 0); ``n_out`` (optional int32 [F, P]) receives n_ij."""
    import torch
    F, P, two = vis.shape
    N = int(round(((8 * P + 1) ** 0.5 - 1) / 2))
    if two != 2 or N * (N + 1) // 2 != P:
        raise ValueError("vis must be [F, N(N+1)/2, 2]")
    _check_acc(vis, count, N, F)
    if dcount.dtype != torch.int32 or tuple(dcount.shape) != (F, P) or \
            not dcount.is_contiguous():
        raise ValueError(f"dcount must be contiguous int32 [{F}, {P}]")
    if out is None:
        out = torch.empty((F, P, 2), dtype=torch.float32, device=vis.device)
    if out.dtype != torch.float32 or tuple(out.shape) != (F, P, 2) or not out.is_contiguous():
        raise ValueError("out must be contiguous float32 [F, P, 2]")
    if n_out is not None and (n_out.dtype != torch.int32 or tuple(n_out.shape) != (F, P)
                              or not n_out.is_contiguous()):
        raise ValueError("n_out must be contiguous int32 [F, P]")
    h = handle or default_handle(vis.device.index)
    h.check(lib().xe_normalize_flagged(
        h.ptr, ctypes.c_void_p(vis.data_ptr()), ctypes.c_void_p(count.data_ptr()),
        ctypes.c_void_p(dcount.data_ptr()), N, F, ctypes.c_void_p(out.data_ptr()),
        ctypes.c_void_p(n_out.data_ptr() if n_out is not None else None),
        _stream_ptr(stream)))
    return out


# -- frame assembly from packets (Sec. II-A) ---------------------------------

def packet_bytes(N: int) -> int:
    """XE_PACKET_BYTES(N): header + [4][8][N] data + [4][8][ceil(N/32)] flag words."""
    return 16 + 32 * N + 128 * ((N + 31) // 32)


def assemble_frame(packets, N: int, n_streams: int, stream_base: int, seq0: int, T: int,
                   packed=None, mask=None, flags=None, stats=None, with_flags: bool = True,
                   handle: Optional[Handle] = None, stream=None):
    """Frame, loss mask (B = 4), flags and counters from a CUDA uint8 tensor
    of packets [n, packet_bytes(N)] in arrival order."""
    import torch
    pb = packet_bytes(N)
    if packets.dtype != torch.uint8 or packets.dim() != 2 or not packets.is_cuda or \
            not packets.is_contiguous() or (packets.shape[0] and packets.shape[1] != pb):
        raise ValueError(f"packets must be a contiguous CUDA uint8 tensor [n, {pb}]")
    dev = packets.device
    F, W = 8 * n_streams, (N + 31) // 32
    if packed is None:
        packed = torch.empty((T, F, N), dtype=torch.uint8, device=dev)
    if mask is None:
        mask = torch.empty((F, T // 4), dtype=torch.uint8, device=dev)
    if flags is None and with_flags:
        flags = torch.empty((F, T, W), dtype=torch.int32, device=dev)
    if stats is None:
        stats = torch.empty(6, dtype=torch.int64, device=dev)
    if tuple(packed.shape) != (T, F, N) or packed.dtype != torch.uint8 or \
            not packed.is_contiguous():
        raise ValueError(f"packed must be contiguous uint8 [{T}, {F}, {N}]")
    if tuple(mask.shape) != (F, T // 4) or mask.dtype != torch.uint8 or not mask.is_contiguous():
        raise ValueError(f"mask must be contiguous uint8 [{F}, {T // 4}]")
    if flags is not None and (tuple(flags.shape) != (F, T, W) or flags.dtype != torch.int32
                              or not flags.is_contiguous()):
        raise ValueError(f"flags must be contiguous int32 [{F}, {T}, {W}]")
    if stats.dtype != torch.int64 or stats.numel() != 6 or not stats.is_contiguous():
        raise ValueError("stats must be contiguous int64 [6]")
    h = handle or default_handle(dev.index)
    h.check(lib().xe_assemble_frame(
        h.ptr, ctypes.c_void_p(packets.data_ptr()), int(packets.shape[0]), N, n_streams,
        stream_base, seq0, T, ctypes.c_void_p(packed.data_ptr()),
        ctypes.c_void_p(mask.data_ptr()),
        ctypes.c_void_p(flags.data_ptr() if flags is not None else None),
        ctypes.c_void_p(stats.data_ptr()), _stream_ptr(stream)))
    return packed, mask, flags, stats


# -- per-input time shifting ---------------------------------------------------

def time_shift(packed, delays, flags=None, out=None, flags_out=None, with_flags: bool = True,
               handle: Optional[Handle] = None, stream=None):
    """Input i delayed by delays[i] samples (CUDA int32 [N]); samples
    shifted in from outside the frame are 0 + 0i and flagged in flags_out."""
    import torch
    T, F, N = _check_frame(packed, None, 1)
    W = (N + 31) // 32
    if delays.dtype != torch.int32 or tuple(delays.shape) != (N,) or not delays.is_cuda or \
            not delays.is_contiguous():
        raise ValueError(f"delays must be a contiguous CUDA int32 tensor [{N}]")
    if flags is not None:
        _check_flags(flags, F, T, N)
    if out is None:
        out = torch.empty_like(packed)
    if flags_out is None and with_flags:
        flags_out = torch.empty((F, T, W), dtype=torch.int32, device=packed.device)
    if flags_out is not None:
        _check_flags(flags_out, F, T, N)
    h = handle or default_handle(packed.device.index)
    h.check(lib().xe_time_shift(
        h.ptr, ctypes.c_void_p(packed.data_ptr()),
        ctypes.c_void_p(flags.data_ptr() if flags is not None else None),
        ctypes.c_void_p(delays.data_ptr()), N, F, T, ctypes.c_void_p(out.data_ptr()),
        ctypes.c_void_p(flags_out.data_ptr() if flags_out is not None else None),
        _stream_ptr(stream)))
    return out, flags_out


def _instances(items: Sequence[Tuple]):
    """ctypes array of xe_instance from (packed, mask, B, vis, count) tuples."""
    arr = (Instance * max(1, len(items)))()
    dev = None
    for k, (packed, mask, B, vis, count) in enumerate(items):
        T, F, N = _check_frame(packed, mask, B)
        _check_acc(vis, count, N, F)
        if dev is not None and packed.device.index != dev:
            raise ValueError("all instances of a batch must be on one device")
        dev = packed.device.index
        arr[k] = Instance(packed.data_ptr(), mask.data_ptr() if mask is not None else None,
                          N, F, T, B, vis.data_ptr(), count.data_ptr())
    return arr, dev


def accumulate_batch(items: Sequence[Tuple], handle: Optional[Handle] = None, stream=None):
    """items: (packed, mask, B, vis, count) per instance; one persistent launch."""
    arr, dev = _instances(items)
    h = handle or default_handle(dev)
    _charge([(v, p.shape[0]) for p, m, B, v, c in items],
            lambda: h.check(lib().xe_accumulate_batch(h.ptr, arr, len(items),
                                                      _stream_ptr(stream))))


class BatchPlan:
    """A work list kept on the device; :meth:`run` only enqueues kernels, so
    it can be captured into a CUDA/HIP graph and replayed.  The instances'
    tensors are referenced here so they outlive the plan."""

    def __init__(self, items: Sequence[Tuple], chunk_steps: int = 0,
                 handle: Optional[Handle] = None, geometry=None):
        arr, dev = _instances(items)
        self.handle = handle or default_handle(dev)
        self.items = list(items)
        pid = ctypes.c_int32(-1)
        # the plan keeps the tile geometry it is built with; the handle's
        # own setting is restored afterwards
        before = self.handle.geometry
        if geometry is not None:
            self.handle.set_geometry(geometry)
        try:
            self.handle.check(lib().xe_batch_plan(self.handle.ptr, arr, len(items), chunk_steps,
                                                  ctypes.byref(pid)))
        finally:
            if geometry is not None:
                self.handle.set_geometry(before)
        self.geometry = self.handle.geometry if geometry is None else (
            GEOMETRIES[geometry] if isinstance(geometry, str) else int(geometry))
        self.plan_id = pid.value

    def run(self, stream=None) -> None:
        _charge([(v, p.shape[0]) for p, m, B, v, c in self.items],
                lambda: self.handle.check(lib().xe_batch_run(self.handle.ptr, self.plan_id,
                                                             _stream_ptr(stream))))

    def release(self) -> None:
        if self.plan_id >= 0:
            lib().xe_batch_release(self.handle.ptr, self.plan_id)
            self.plan_id = -1

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def batch_query(shapes: Sequence[Tuple[int, int, int, int]], n_cu: int = 256,
                chunk_steps: int = 0, aligned: Sequence[bool] = ()) -> BatchInfo:
    """Work-list shape for instances (N, F, T, B), host only.  Fake,
    disjoint, suitably aligned pointers stand in for device buffers
    (``aligned[k]`` False offsets instance k's frame by one byte)."""
    arr = (Instance * max(1, len(shapes)))()
    base = 1 << 40
    for k, (N, F, T, B) in enumerate(shapes):
        P = N * (N + 1) // 2
        off = 0 if (k >= len(aligned) or aligned[k]) else 1
        vis = base
        cnt = vis + ((F * P * 8 + 255) & ~255)
        arr[k] = Instance(base + off + (1 << 36), None, N, F, T, B, vis, cnt)
        base = cnt + ((F * 8 + 255) & ~255)
    info = BatchInfo()
    s = lib().xe_batch_query(arr, len(shapes), n_cu, chunk_steps, ctypes.byref(info))
    if s != XE_OK:
        raise XEngineError(s, status_string(s))
    return info
