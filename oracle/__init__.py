"""Oracle for the X-engine correlation path -- TEST INFRASTRUCTURE ONLY.

A plain CPU implementation (``xcorr_oracle.c``: int64 loops over channel,
input pair and time sample, FP64 normalisation) with a ctypes wrapper.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the HIP path and never
imports the product package.

``build()`` compiles the C file with gcc (OpenMP over the outer loops);
``load()`` returns an :class:`Oracle` bound to a built library, building it
first when none exists.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "xcorr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build(src: str = SRC, out: str = LIB, extra: Sequence[str] = ()) -> str:
    """Compile the oracle into a shared library; returns its path."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
           "-Wall", "-Wextra", *extra, src, "-o", out + ".tmp"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(out + ".tmp", out)
    return out


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_p)


class Oracle:
    """numpy-level access to one built oracle library."""

    def __init__(self, path: str):
        self.path = path
        lib = ctypes.CDLL(path)
        self._lib = lib
        lib.oracle_tri_index.restype = _i64
        lib.oracle_tri_index.argtypes = [_i64, _i64, _i64]
        lib.oracle_num_pairs.restype = _i64
        lib.oracle_num_pairs.argtypes = [_i64]
        lib.oracle_decode.restype = None
        lib.oracle_decode.argtypes = [ctypes.c_uint8, ctypes.POINTER(_i32),
                                      ctypes.POINTER(_i32)]
        lib.oracle_valid_counts.restype = None
        lib.oracle_valid_counts.argtypes = [_p, _i32, _i32, _i32, _p]
        for name in ("oracle_correlate", "oracle_accumulate"):
            fn = getattr(lib, name)
            fn.restype = None
            fn.argtypes = [_p, _p, _i32, _i32, _i32, _i32, _p, _p]
        lib.oracle_correlate_full.restype = None
        lib.oracle_correlate_full.argtypes = [_p, _p, _i32, _i32, _i32, _i32, _p]
        lib.oracle_correlate_pairs.restype = None
        lib.oracle_correlate_pairs.argtypes = [_p, _p, _i32, _i32, _i32, _i32,
                                               _p, _p, _p, _i64, _p]
        lib.oracle_normalize.restype = None
        lib.oracle_normalize.argtypes = [_p, _p, _i32, _i32, _p]
        lib.oracle_flag_counters.restype = None
        lib.oracle_flag_counters.argtypes = [_p, _p, _i32, _i32, _i32, _i32, _p, _p]
        lib.oracle_flag_norm.restype = None
        lib.oracle_flag_norm.argtypes = [_p, _p, _p, _i32, _i32, _p]
        lib.oracle_apply_flags.restype = None
        lib.oracle_apply_flags.argtypes = [_p, _p, _i32, _i32, _i32]
        lib.oracle_correlate_flagged.restype = None
        lib.oracle_correlate_flagged.argtypes = [_p, _p, _p, _i32, _i32, _i32, _i32,
                                                 _p, _p]
        lib.oracle_normalize_pairs.restype = None
        lib.oracle_normalize_pairs.argtypes = [_p, _p, _i32, _i32, _p]
        lib.oracle_time_shift.restype = None
        lib.oracle_time_shift.argtypes = [_p, _p, _p, _i32, _i32, _i32, _p, _p]
        lib.oracle_assemble.restype = None
        lib.oracle_assemble.argtypes = [_p, _i64, _i32, _i32, _i32, _i64, _i32, _p, _p, _p, _p]

    # -- helpers ---------------------------------------------------------
    @staticmethod
    def _frame_args(packed: np.ndarray, mask: Optional[np.ndarray], B: int):
        packed = np.ascontiguousarray(packed, dtype=np.uint8)
        if packed.ndim != 3:
            raise ValueError("packed must be [T][F][N]")
        T, F, N = packed.shape
        if mask is not None:
            mask = np.ascontiguousarray(mask, dtype=np.uint8)
            if mask.shape != (F, (T + B - 1) // B):
                raise ValueError("mask must be [F][ceil(T/B)]")
        return packed, mask, N, F, T

    @staticmethod
    def _flag_args(flags: np.ndarray, T: int, F: int, N: int) -> np.ndarray:
        flags = np.ascontiguousarray(flags, dtype=np.uint32)
        if flags.shape != (F, T, (N + 31) // 32):
            raise ValueError("flags must be uint32 [F][T][ceil(N/32)]")
        return flags

    # -- API ---------------------------------------------------------------
    def tri_index(self, N: int, i: int, j: int) -> int:
        return int(self._lib.oracle_tri_index(N, i, j))

    def num_pairs(self, N: int) -> int:
        return int(self._lib.oracle_num_pairs(N))

    def decode(self, byte: int) -> Tuple[int, int]:
        re, im = _i32(), _i32()
        self._lib.oracle_decode(byte, ctypes.byref(re), ctypes.byref(im))
        return re.value, im.value

    def valid_counts(self, mask: Optional[np.ndarray], F: int, T: int, B: int) -> np.ndarray:
        out = np.zeros(F, dtype=np.int64)
        if mask is not None:
            mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self._lib.oracle_valid_counts(_ptr(mask), F, T, B, _ptr(out))
        return out

    def correlate(self, packed, mask=None, B: int = 256):
        packed, mask, N, F, T = self._frame_args(packed, mask, B)
        vis = np.zeros((F, N * (N + 1) // 2, 2), dtype=np.int64)
        cnt = np.zeros(F, dtype=np.int64)
        self._lib.oracle_correlate(_ptr(packed), _ptr(mask), N, F, T, B,
                                   _ptr(vis), _ptr(cnt))
        return vis, cnt

    def accumulate(self, packed, mask, B: int, vis: np.ndarray, cnt: np.ndarray) -> None:
        packed, mask, N, F, T = self._frame_args(packed, mask, B)
        if vis.dtype != np.int64 or not vis.flags.c_contiguous or \
                vis.shape != (F, N * (N + 1) // 2, 2):
            raise ValueError("vis must be contiguous int64 [F][P][2]")
        if cnt.dtype != np.int64 or cnt.shape != (F,):
            raise ValueError("count must be int64 [F]")
        self._lib.oracle_accumulate(_ptr(packed), _ptr(mask), N, F, T, B,
                                    _ptr(vis), _ptr(cnt))

    def correlate_full(self, packed, mask=None, B: int = 256) -> np.ndarray:
        packed, mask, N, F, T = self._frame_args(packed, mask, B)
        out = np.zeros((F, N, N, 2), dtype=np.int64)
        self._lib.oracle_correlate_full(_ptr(packed), _ptr(mask), N, F, T, B, _ptr(out))
        return out

    def correlate_pairs(self, packed, mask, B: int, fs, is_, js) -> np.ndarray:
        packed, mask, N, F, T = self._frame_args(packed, mask, B)
        fs = np.ascontiguousarray(fs, dtype=np.int32)
        is_ = np.ascontiguousarray(is_, dtype=np.int32)
        js = np.ascontiguousarray(js, dtype=np.int32)
        n = fs.size
        if not (is_.size == n and js.size == n):
            raise ValueError("index arrays differ in length")
        if n and (fs.min() < 0 or fs.max() >= F or is_.min() < 0 or js.min() < 0
                  or is_.max() >= N or js.max() >= N):
            raise ValueError("index out of range")
        out = np.zeros((n, 2), dtype=np.int64)
        self._lib.oracle_correlate_pairs(_ptr(packed), _ptr(mask), N, F, T, B,
                                         _ptr(fs), _ptr(is_), _ptr(js), n, _ptr(out))
        return out

    def normalize(self, vis: np.ndarray, cnt: np.ndarray) -> np.ndarray:
        vis = np.ascontiguousarray(vis, dtype=np.int64)
        cnt = np.ascontiguousarray(cnt, dtype=np.int64)
        F, P, two = vis.shape
        N = int(round((np.sqrt(8 * P + 1) - 1) / 2))
        if two != 2 or N * (N + 1) // 2 != P or cnt.shape != (F,):
            raise ValueError("vis must be [F][N(N+1)/2][2], count [F]")
        out = np.zeros((F, P, 2), dtype=np.float32)
        self._lib.oracle_normalize(_ptr(vis), _ptr(cnt), N, F, _ptr(out))
        return out

    # -- per-input flags (Sec. II-C) -----------------------------------------
    def flag_counters(self, flags, mask, N: int, B: int = 256, c=None, d=None):
        """Counters c [F][N] and intersections d [F][P] (diagonal = c) of
        one frame's flags, added into ``c``/``d`` when given."""
        flags = np.asarray(flags)
        F, T = flags.shape[:2]
        flags = self._flag_args(flags, T, F, N)
        if mask is not None:
            mask = np.ascontiguousarray(mask, dtype=np.uint8)
            if mask.shape != (F, (T + B - 1) // B):
                raise ValueError("mask must be [F][ceil(T/B)]")
        P = N * (N + 1) // 2
        c = np.zeros((F, N), dtype=np.int64) if c is None else c
        d = np.zeros((F, P), dtype=np.int64) if d is None else d
        if c.dtype != np.int64 or c.shape != (F, N) or not c.flags.c_contiguous:
            raise ValueError("c must be contiguous int64 [F][N]")
        if d.dtype != np.int64 or d.shape != (F, P) or not d.flags.c_contiguous:
            raise ValueError("d must be contiguous int64 [F][P]")
        self._lib.oracle_flag_counters(_ptr(flags), _ptr(mask), N, F, T, B,
                                       _ptr(c), _ptr(d))
        return c, d

    def flag_norm(self, count, c, d) -> np.ndarray:
        """Normalisation matrix n [F][P] = count_f - c_i - c_j + d_ij."""
        count = np.ascontiguousarray(count, dtype=np.int64)
        c = np.ascontiguousarray(c, dtype=np.int64)
        d = np.ascontiguousarray(d, dtype=np.int64)
        F, N = c.shape
        if count.shape != (F,) or d.shape != (F, N * (N + 1) // 2):
            raise ValueError("count [F], c [F][N], d [F][P] expected")
        n = np.zeros_like(d)
        self._lib.oracle_flag_norm(_ptr(count), _ptr(c), _ptr(d), N, F, _ptr(n))
        return n

    def apply_flags(self, packed, flags) -> np.ndarray:
        """Copy of the frame with every flagged point set to 0 + 0i."""
        out = np.array(packed, dtype=np.uint8, order="C", copy=True)
        T, F, N = out.shape
        flags = self._flag_args(flags, T, F, N)
        self._lib.oracle_apply_flags(_ptr(out), _ptr(flags), N, F, T)
        return out

    def correlate_flagged(self, packed, mask, flags, B: int = 256):
        packed, mask, N, F, T = self._frame_args(packed, mask, B)
        flags = self._flag_args(flags, T, F, N)
        vis = np.zeros((F, N * (N + 1) // 2, 2), dtype=np.int64)
        cnt = np.zeros(F, dtype=np.int64)
        self._lib.oracle_correlate_flagged(_ptr(packed), _ptr(mask), _ptr(flags),
                                           N, F, T, B, _ptr(vis), _ptr(cnt))
        return vis, cnt

    def normalize_pairs(self, vis, n) -> np.ndarray:
        vis = np.ascontiguousarray(vis, dtype=np.int64)
        n = np.ascontiguousarray(n, dtype=np.int64)
        F, P, two = vis.shape
        N = int(round((np.sqrt(8 * P + 1) - 1) / 2))
        if two != 2 or N * (N + 1) // 2 != P or n.shape != (F, P):
            raise ValueError("vis must be [F][P][2], n [F][P]")
        out = np.zeros((F, P, 2), dtype=np.float32)
        self._lib.oracle_normalize_pairs(_ptr(vis), _ptr(n), N, F, _ptr(out))
        return out

    # -- frame assembly from packets (Sec. II-A) -----------------------------
    def assemble(self, packets, N: int, n_streams: int, stream_base: int, seq0: int, T: int):
        """(packed [T][F][N], mask [F][T/4], flags [F][T][W], stats [6]) from
        packets uint8 [n][packet_bytes] in arrival order."""
        packets = np.ascontiguousarray(packets, dtype=np.uint8)
        W = (N + 31) // 32
        pb = 16 + 32 * N + 128 * W
        if packets.ndim != 2 or (packets.shape[0] and packets.shape[1] != pb):
            raise ValueError(f"packets must be uint8 [n][{pb}]")
        if T % 4:
            raise ValueError("T must be a multiple of 4")
        F = 8 * n_streams
        # outputs start as garbage: the assembler must write every element
        packed = np.full((T, F, N), 0x5A, dtype=np.uint8)
        mask = np.full((F, T // 4), 7, dtype=np.uint8)
        flags = np.full((F, T, W), 0xDEADBEEF, dtype=np.uint32)
        stats = np.full(6, -1, dtype=np.int64)
        self._lib.oracle_assemble(_ptr(packets), packets.shape[0], N, n_streams, stream_base,
                                  seq0, T, _ptr(packed), _ptr(mask), _ptr(flags), _ptr(stats))
        return packed, mask, flags, stats

    # -- per-input time shifting ------------------------------------------------
    def time_shift(self, packed, flags, delays):
        """(out [T][F][N], flags_out [F][T][W]): input i delayed by delays[i]."""
        packed = np.ascontiguousarray(packed, dtype=np.uint8)
        T, F, N = packed.shape
        if flags is not None:
            flags = self._flag_args(flags, T, F, N)
        delays = np.ascontiguousarray(delays, dtype=np.int32)
        if delays.shape != (N,):
            raise ValueError("delays must be int32 [N]")
        out = np.full_like(packed, 0x5A)
        fo = np.full((F, T, (N + 31) // 32), 0xDEADBEEF, dtype=np.uint32)
        self._lib.oracle_time_shift(_ptr(packed), _ptr(flags), _ptr(delays), N, F, T,
                                    _ptr(out), _ptr(fo))
        return out, fo


_cached: Optional[Oracle] = None


def load(path: Optional[str] = None) -> Oracle:
    """The oracle bound to ``path`` (default: the in-tree build, built on
    first use when missing)."""
    global _cached
    if path is not None:
        return Oracle(path)
    if _cached is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _cached = Oracle(LIB)
    return _cached
