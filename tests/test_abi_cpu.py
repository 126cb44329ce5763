"""The C ABI on the host: exports, status strings, argument checks, plan.

No compute call reaches a GPU here: the handle is validation-only
(XE_DEVICE_NONE), so every compute entry point validates its arguments and
returns XE_ERR_NO_DEVICE when they are good.
"""

import ctypes
import re

import pytest

from paper_1503_06189_amd import xengine as xe


@pytest.fixture(scope="module")
def L():
    return xe.lib()


@pytest.fixture()
def h(L):
    p = ctypes.c_void_p()
    assert L.xe_create(ctypes.byref(p), xe.XE_DEVICE_NONE, 0) == xe.XE_OK
    yield p
    assert L.xe_destroy(p) == xe.XE_OK


def test_every_declared_symbol_is_exported(L):
    text = open(xe.HEADER).read()
    declared = set(re.findall(r"\b(xe_[a-z_]+)\s*\(", text))
    assert declared == set(xe.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_status_strings(L):
    for s in (0, -1, -2, -3, -4, -5, -6, -7):
        assert xe.status_string(s) not in ("", "unknown status")
    assert xe.status_string(42) == "unknown status"


def _call(L, h, N=16, F=2, T=64, B=16, packed=0x1000, mask=None, vis=0x2000, count=0x3000,
          fn="xe_accumulate"):
    f = getattr(L, fn)
    return f(h, ctypes.c_void_p(packed), ctypes.c_void_p(mask), N, F, T, B,
             ctypes.c_void_p(vis), ctypes.c_void_p(count), None)


@pytest.mark.parametrize("fn", ["xe_accumulate", "xe_correlate_frame"])
def test_argument_checks(L, h, fn):
    assert _call(L, h, fn=fn) == xe.XE_ERR_NO_DEVICE
    assert _call(L, None, fn=fn) == xe.XE_ERR_ARG
    for bad in (dict(N=0), dict(N=4097), dict(F=0), dict(T=0), dict(B=0), dict(T=-5),
                dict(packed=0), dict(vis=0), dict(count=0)):
        assert _call(L, h, fn=fn, **bad) == xe.XE_ERR_ARG, bad
        assert L.xe_last_error(h)
    assert _call(L, h, fn=fn, T=xe.XE_MAX_SAMPLES + 1) == xe.XE_ERR_OVERFLOW
    assert _call(L, h, fn=fn, T=xe.XE_MAX_SAMPLES) == xe.XE_ERR_NO_DEVICE
    assert _call(L, h, fn=fn, vis=0x2004) == xe.XE_ERR_ALIGN
    assert _call(L, h, fn=fn, count=0x3002) == xe.XE_ERR_ALIGN
    assert _call(L, h, fn=fn, N=4096, F=1, T=1) == xe.XE_ERR_NO_DEVICE


def test_normalize_checks(L, h):
    f = L.xe_normalize
    vp = ctypes.c_void_p
    assert f(h, vp(0x10000), vp(0x20000), 16, 2, vp(0x30000), None) == xe.XE_ERR_NO_DEVICE
    assert f(h, vp(0), vp(0x20000), 16, 2, vp(0x30000), None) == xe.XE_ERR_ARG
    assert f(h, vp(0x10000), vp(0x20000), 0, 2, vp(0x30000), None) == xe.XE_ERR_ARG
    assert f(h, vp(0x10004), vp(0x20000), 16, 2, vp(0x30000), None) == xe.XE_ERR_ALIGN
    # out overlapping vis
    assert f(h, vp(0x10000), vp(0x20000), 16, 2, vp(0x10100), None) == xe.XE_ERR_ARG


def test_batch_checks(L, h):
    arr = (xe.Instance * 2)()
    arr[0] = xe.Instance(0x1000, None, 16, 1, 64, 16, 0x2000, 0x3000)
    arr[1] = xe.Instance(0x1000, None, 16, 1, 64, 16, 0x2000, 0x3000)
    assert L.xe_accumulate_batch(h, arr, 2, None) == xe.XE_ERR_NO_DEVICE
    arr[1].N = 0
    assert L.xe_accumulate_batch(h, arr, 2, None) == xe.XE_ERR_ARG
    assert L.xe_accumulate_batch(h, arr, -1, None) == xe.XE_ERR_ARG


def test_create_without_gpu_is_clean(L):
    # device 0 does not exist in a GPU-less container: an error, never a crash
    p = ctypes.c_void_p()
    s = L.xe_create(ctypes.byref(p), 0, 0)
    if s == xe.XE_OK:
        L.xe_destroy(p)
    else:
        assert s in (xe.XE_ERR_HIP, xe.XE_ERR_UNSUPPORTED)
    assert L.xe_create(None, 0, 0) == xe.XE_ERR_ARG


def test_plan_query_shapes():
    # pathfinder share: one diagonal group per channel, split in time to
    # cover 256 compute units
    p = xe.plan_query(256, 64, 16384, 256, 256)
    assert (p.blocks, p.groups, p.splits) == (8, 1, 4)
    assert p.workgroups == 256 and p.mfma_tiles == 36
    assert p.splits * p.steps_per_split * 32 >= 16384
    # large N: 8 super-rows -> 64 groups per channel, no split needed
    p = xe.plan_query(2048, 16, 8192, 256, 256)
    assert (p.blocks, p.groups, p.splits) == (64, 64, 1)
    assert p.mfma_tiles == 8 * 36 + 8 * 7 * 32
    # tiny
    p = xe.plan_query(16, 8, 256, 256, 256)
    assert p.blocks == 1 and p.groups == 1 and p.splits == 1
    with pytest.raises(xe.XEngineError):
        xe.plan_query(0, 1, 1, 1, 256)


def test_tile_groups_cover_the_triangle_once():
    """Host model of the tile decomposition (eight waves per group): every
    (I <= J) block pair of the triangle is owned by exactly one tile of one
    wave of one group, for many N, and every wave has 16 MFMAs per step."""
    def groups(nb):
        ns = -(-nb // 8)
        out = []
        for gid in range(ns * ns):
            if gid < ns:
                slots = [8 * gid + s for s in range(8)]
                for w in range(8):
                    tiles, mfmas = [], 0
                    if w < 4:
                        tiles += [(w, w + 1 + k) for k in range(4)]
                        mfmas = 2 * 4
                    else:
                        p = w - 4
                        tiles += [(p, p), (7 - p, 7 - p)]
                        tiles += [(p, p + 5 + k) for k in range(3 - p)]
                        tiles += [(7 - p, 8 - p + k) for k in range(p)]
                        mfmas = 2 + 2 * 3
                    assert mfmas == 8 and len(set(tiles)) == len(tiles)
                    out += [(slots[r], slots[c]) for r, c in tiles]
            else:
                q = gid - ns
                p, half = q // 2, q % 2
                R = 0
                while p >= ns - 1 - R:
                    p -= ns - 1 - R
                    R += 1
                C = R + 1 + p
                slots = [8 * R + 4 * half + s for s in range(4)] + [8 * C + s for s in range(8)]
                for w in range(8):
                    c0 = 4 + 4 * (w % 2)
                    out += [(slots[w // 2], slots[c0 + k]) for k in range(4)]
        return out
    for nb in (1, 2, 3, 7, 8, 9, 15, 16, 17, 33, 64, 128):
        allt = groups(nb)
        assert all(i <= j for i, j in allt)
        tiles = [t for t in allt if t[0] < nb and t[1] < nb]
        want = [(i, j) for i in range(nb) for j in range(i, nb)]
        assert sorted(tiles) == want, nb
