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
    arr[1] = xe.Instance(0x1000, None, 16, 1, 64, 16, 0x4000, 0x5000)
    assert L.xe_accumulate_batch(h, arr, 2, None) == xe.XE_ERR_NO_DEVICE
    assert L.xe_accumulate_batch(h, arr, 0, None) == xe.XE_ERR_NO_DEVICE
    pid = ctypes.c_int32(-1)
    assert L.xe_batch_plan(h, arr, 2, 0, ctypes.byref(pid)) == xe.XE_ERR_NO_DEVICE
    assert L.xe_batch_plan(h, arr, 2, -1, ctypes.byref(pid)) == xe.XE_ERR_ARG
    assert L.xe_batch_run(h, 0, None) == xe.XE_ERR_ARG       # no such plan
    assert L.xe_batch_run(h, 7, None) == xe.XE_ERR_ARG
    assert L.xe_batch_release(h, 5) == xe.XE_ERR_ARG
    # the second instance's sums overlap the first's (16 inputs: 1088 bytes)
    arr[1].vis = 0x2000 + 1024
    assert L.xe_accumulate_batch(h, arr, 2, None) == xe.XE_ERR_ARG
    assert b"share" in L.xe_last_error(h)
    arr[1].vis = 0x4000
    arr[1].count = 0x2000 + 8 * 136 - 8
    assert L.xe_accumulate_batch(h, arr, 2, None) == xe.XE_ERR_ARG
    arr[1].count = 0x5000
    arr[1].N = 0
    assert L.xe_accumulate_batch(h, arr, 2, None) == xe.XE_ERR_ARG
    assert L.xe_accumulate_batch(h, arr, -1, None) == xe.XE_ERR_ARG
    assert L.xe_accumulate_batch(h, None, 2, None) == xe.XE_ERR_ARG


def _model_items(shapes, chunk, n_cu=256):
    """Work items of a batch in the default (halves) geometry: F * groups *
    time chunks per instance, where instances of N <= 128 (their own
    launch) take chunks of about their total work / n_cu steps, between 32
    and the common length."""
    def work(N, F, T):
        nb = -(-N // 32)
        return F * (-(-nb // 8)) ** 2 * -(-T // 32)
    small_work = sum(work(N, F, T) for N, F, T, B in shapes if N <= 128)
    small_chunk = max(32, min(chunk, -(-small_work // n_cu)))
    items = 0
    for N, F, T, B in shapes:
        nb = -(-N // 32)
        G = (-(-nb // 8)) ** 2
        steps = -(-T // 32)
        sps = min(small_chunk if N <= 128 else chunk, steps)
        items += F * G * -(-steps // sps)
    return items, small_chunk


def test_batch_query_work_list():
    """Work items = sum over instances of F * groups * time chunks; the
    automatic chunk length gives about four items per compute unit, and the
    halves-geometry instances (N <= 128), which drain in a launch of their
    own, about one per compute unit."""
    import random
    rng = random.Random(7)
    shapes = [(rng.choice([64, 128, 256, 512, 1024]), 1, 256 * rng.randint(4, 256), 256)
              for _ in range(128)]
    info = xe.batch_query(shapes, n_cu=256)
    assert info.instances == 128 and info.unaligned == 0
    work = sum(F * (-(-(-(-N // 32)) // 8)) ** 2 * -(-T // 32) for N, F, T, B in shapes)
    assert info.chunk_steps == max(32, work // (4 * 256))
    items, small_chunk = _model_items(shapes, info.chunk_steps)
    assert info.items == items
    assert small_chunk < info.chunk_steps
    small = sum(1 for N, F, T, B in shapes if N <= 128)
    small_items = items - _model_items([x for x in shapes if x[0] > 128], info.chunk_steps)[0]
    assert small <= small_items and 256 <= small_items <= 256 + small
    assert 256 * 3 <= info.items <= 256 * 7
    # an explicit chunk length
    info2 = xe.batch_query(shapes, n_cu=256, chunk_steps=2 * info.chunk_steps)
    assert info2.chunk_steps == 2 * info.chunk_steps and info2.items < info.items
    # N not a multiple of 4 or an unaligned frame: a plain launch
    info3 = xe.batch_query([(18, 2, 1000, 256), (64, 1, 4096, 256), (64, 1, 4096, 256)],
                           aligned=[True, True, False])
    assert (info3.instances, info3.unaligned) == (1, 2)
    # partial sums of every chunked (channel, group) must fit the workspace
    with pytest.raises(xe.XEngineError):
        xe.batch_query([(4096, 64, 1 << 20, 256)], chunk_steps=32)
    assert xe.batch_query([], n_cu=256).items == 0


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
    """Host model of the tile decomposition (eight waves per group, waves w
    and w + 4 on one SIMD): every (I <= J) block pair of the triangle is
    owned by exactly one tile of one wave of one group, for many N; every
    wave runs 16 MFMAs per step (a diagonal tile is one chain, an
    off-diagonal tile two) and holds at most 128 accumulator registers; the
    staging work of a step is dealt evenly to the four SIMDs."""
    def roles(diag):
        out = []
        for w in range(8):
            if diag:
                if w < 4:                       # row block w x columns 4..7
                    q, pairs, upt = [], [(w, 4 + c) for c in range(4)], 1
                elif w % 2 == 0:                # half A of triangle 0..3 / 4..7
                    b = 2 * (w - 4)
                    q, pairs, upt = [b, b + 1], [(b, b + c) for c in (1, 2, 3)], 1
                else:                           # half B
                    b = 2 * (w - 5)
                    q = [b + 2, b + 3]
                    pairs = [(b + 1, b + 2), (b + 1, b + 3), (b + 2, b + 3)]
                    upt = 1
            else:                               # row slot w % 4 x 4 column slots
                c0 = 4 + 4 * (w // 4)
                q, pairs, upt = [], [(w % 4, c0 + c) for c in range(4)], 2 if w < 4 else 1
            out.append((q, pairs, upt))
        return out

    for diag in (True, False):
        rs = roles(diag)
        for q, pairs, upt in rs:
            assert 2 * (len(q) + 2 * len(pairs)) == 16        # MFMAs per 32-sample step
            assert 16 * len(q) + 32 * len(pairs) <= 128       # accumulator registers
        units = [rs[w][2] + rs[w + 4][2] for w in range(4)]
        assert len(set(units)) == 1                           # per-SIMD staging share
        assert sum(r[2] for r in rs) * 64 == (8 if diag else 12) * 64  # units per step

    def groups(nb):
        ns = -(-nb // 8)
        out = []
        for gid in range(ns * ns):
            if gid < ns:
                slots = [8 * gid + s for s in range(8)]
                for q, pairs, _ in roles(True):
                    tiles = [(b, b) for b in q] + pairs
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
                for _, pairs, _ in roles(False):
                    out += [(slots[r], slots[c]) for r, c in pairs]
        return out
    for nb in (1, 2, 3, 7, 8, 9, 15, 16, 17, 33, 64, 128):
        allt = groups(nb)
        assert all(i <= j for i, j in allt)
        tiles = [t for t in allt if t[0] < nb and t[1] < nb]
        want = [(i, j) for i in range(nb) for j in range(i, nb)]
        assert sorted(tiles) == want, nb


def test_halves_geometry_model():
    """Host model of the halves geometry (N <= 128): slots 0..3 hold blocks
    0..3 at the even 32-sample step of a pair, slots 4..7 the same blocks at
    the odd one.  Waves 4..7 keep their triangle roles: waves 4, 5 cover the
    10 tiles of the 4-block triangle over the even steps and waves 6, 7 over
    the odd ones, each tile exactly once per step, never pairing slots of
    different steps; the rectangle waves (0..3) would pair different steps,
    so they stage only."""
    def tri(w):
        if w % 2 == 0:
            b = 2 * (w - 4)
            return [(b, b), (b + 1, b + 1)] + [(b, b + c) for c in (1, 2, 3)]
        b = 2 * (w - 5)
        return [(b + 2, b + 2), (b + 3, b + 3), (b + 1, b + 2), (b + 1, b + 3), (b + 2, b + 3)]
    block, step = (lambda s: s % 4), (lambda s: s // 4)
    want = sorted((i, j) for i in range(4) for j in range(i, 4))
    for parity, waves in ((0, (4, 5)), (1, (6, 7))):
        tiles = []
        for w in waves:
            for r, c in tri(w):
                assert step(r) == step(c) == parity
                tiles.append((block(r), block(c)))
        assert sorted(tiles) == want
    for w in range(4):                       # rectangle: row slot w x slots 4..7
        assert all(step(w) != step(4 + c) for c in range(4))


def test_set_geometry_checks(L, h):
    for g in (xe.XE_GEOM_AUTO, xe.XE_GEOM_SUPER, xe.XE_GEOM_HALVES):
        assert L.xe_set_geometry(h, g) == xe.XE_OK
    assert L.xe_set_geometry(h, 3) == xe.XE_ERR_ARG
    assert L.xe_set_geometry(h, -1) == xe.XE_ERR_ARG
    assert L.xe_set_geometry(None, 0) == xe.XE_ERR_ARG


def test_flag_checks(L, h):
    def acc(flags=0x1000, mask=None, N=40, F=2, T=64, B=16, d=0x200000, hh=h):
        return L.xe_flag_accumulate(hh, ctypes.c_void_p(flags), ctypes.c_void_p(mask), N, F,
                                    T, B, ctypes.c_void_p(d), None)
    assert acc() == xe.XE_ERR_NO_DEVICE
    assert acc(hh=None) == xe.XE_ERR_ARG
    for bad in (dict(flags=0), dict(d=0), dict(N=0), dict(F=0), dict(T=0), dict(B=0)):
        assert acc(**bad) == xe.XE_ERR_ARG, bad
    assert acc(flags=0x1002) == xe.XE_ERR_ALIGN
    assert acc(d=0x200002) == xe.XE_ERR_ALIGN
    assert acc(T=xe.XE_MAX_SAMPLES + 1) == xe.XE_ERR_OVERFLOW

    def app(packed=0x100000, flags=0x1000, N=40, F=2, T=64):
        return L.xe_apply_flags(h, ctypes.c_void_p(packed), ctypes.c_void_p(flags), N, F, T,
                                None)
    assert app() == xe.XE_ERR_NO_DEVICE
    assert app(packed=0) == xe.XE_ERR_ARG
    assert app(flags=0x1001) == xe.XE_ERR_ALIGN
    assert app(packed=0x1000 + 64) == xe.XE_ERR_ARG   # overlaps the flags

    def nrm(vis=0x100000, count=0x200000, d=0x300000, out=0x400000, n_out=None, N=40, F=2):
        return L.xe_normalize_flagged(h, ctypes.c_void_p(vis), ctypes.c_void_p(count),
                                      ctypes.c_void_p(d), N, F, ctypes.c_void_p(out),
                                      ctypes.c_void_p(n_out), None)
    assert nrm() == xe.XE_ERR_NO_DEVICE
    assert nrm(n_out=0x500000) == xe.XE_ERR_NO_DEVICE
    for bad in (dict(vis=0), dict(count=0), dict(d=0), dict(out=0), dict(N=0)):
        assert nrm(**bad) == xe.XE_ERR_ARG, bad
    assert nrm(out=0x100000 + 8) == xe.XE_ERR_ARG      # out overlaps vis
    assert nrm(n_out=0x300000) == xe.XE_ERR_ARG        # n_out overlaps dcount
    assert nrm(vis=0x100004) == xe.XE_ERR_ALIGN
    assert nrm(d=0x300002) == xe.XE_ERR_ALIGN
    assert nrm(n_out=0x500002) == xe.XE_ERR_ALIGN


def test_assemble_checks(L, h):
    def asm(packets=0x100000, n=10, N=40, S=2, base=0, seq0=0, T=64, packed=0x200000,
            mask=0x300000, flags=0x400000, stats=0x500000, hh=h):
        return L.xe_assemble_frame(hh, ctypes.c_void_p(packets), n, N, S, base, seq0, T,
                                   ctypes.c_void_p(packed), ctypes.c_void_p(mask),
                                   ctypes.c_void_p(flags), ctypes.c_void_p(stats), None)
    assert asm() == xe.XE_ERR_NO_DEVICE
    assert asm(flags=0) == xe.XE_ERR_NO_DEVICE          # flags are optional
    assert asm(n=0, packets=0) == xe.XE_ERR_NO_DEVICE   # an empty batch: every place lost
    assert asm(hh=None) == xe.XE_ERR_ARG
    for bad in (dict(packets=0), dict(packed=0), dict(mask=0), dict(stats=0), dict(N=0),
                dict(S=0), dict(T=62), dict(T=0), dict(n=-1)):
        assert asm(**bad) == xe.XE_ERR_ARG, bad
    assert asm(packets=0x100002) == xe.XE_ERR_ALIGN
    assert asm(stats=0x500004) == xe.XE_ERR_ALIGN
    assert xe.packet_bytes(256) == 16 + 8192 + 1024
    assert xe.packet_bytes(37) == 16 + 32 * 37 + 128 * 2


def test_time_shift_checks(L, h):
    def sh(pin=0x100000, fin=0x200000, d=0x300000, N=40, F=2, T=64, pout=0x400000,
           fout=0x500000, hh=h):
        return L.xe_time_shift(hh, ctypes.c_void_p(pin), ctypes.c_void_p(fin),
                               ctypes.c_void_p(d), N, F, T, ctypes.c_void_p(pout),
                               ctypes.c_void_p(fout), None)
    assert sh() == xe.XE_ERR_NO_DEVICE
    assert sh(fin=0, fout=0) == xe.XE_ERR_NO_DEVICE     # flags optional
    assert sh(hh=None) == xe.XE_ERR_ARG
    for bad in (dict(pin=0), dict(d=0), dict(pout=0), dict(N=0), dict(T=0)):
        assert sh(**bad) == xe.XE_ERR_ARG, bad
    assert sh(pout=0x100000 + 16) == xe.XE_ERR_ARG       # overlaps the input frame
    assert sh(fout=0x200000 + 4) == xe.XE_ERR_ARG        # overlaps the input flags
    assert sh(d=0x300002) == xe.XE_ERR_ALIGN
    assert sh(fout=0x500002) == xe.XE_ERR_ALIGN


def test_integration_bound_bookkeeping():
    """Samples integrated per accumulator are counted and a call that would
    pass the int32 bound is refused before anything is launched."""
    torch = pytest.importorskip("torch")
    ok = lambda: 0                               # noqa: E731  (a call that succeeds)
    vis = torch.zeros(4, dtype=torch.int32)
    other = torch.zeros(4, dtype=torch.int32)
    xe.reset_integration(vis)
    xe._charge([(vis, xe.XE_MAX_SAMPLES - 10)], ok)
    assert xe.integrated_samples(vis) == xe.XE_MAX_SAMPLES - 10
    xe._charge([(vis, 10)], ok)                  # exactly at the bound: allowed
    ran = []
    with pytest.raises(xe.XEngineError) as e:    # one over: the whole call is refused
        xe._charge([(other, 5), (vis, 1)], lambda: ran.append(1))
    assert e.value.status == xe.XE_ERR_OVERFLOW
    assert not ran                               # ... before the call was made
    assert xe.integrated_samples(other) == 0     # nothing was charged
    xe.reset_integration(vis)
    xe._charge([(vis, 1), (vis, 2)], ok)         # the same sums twice in one batch
    assert xe.integrated_samples(vis) == 3


def test_integration_bound_failed_call_charges_nothing():
    """A call the library rejects adds no samples to the count."""
    torch = pytest.importorskip("torch")
    vis = torch.zeros(4, dtype=torch.int32)
    xe.reset_integration(vis)

    def rejected():
        raise xe.XEngineError(xe.XE_ERR_ARG, "rejected")
    with pytest.raises(xe.XEngineError):
        xe._charge([(vis, 100)], rejected)
    assert xe.integrated_samples(vis) == 0


def test_integration_bound_not_inherited_at_a_recycled_address():
    """The count belongs to the tensor: once it is freed, a tensor at the
    same address starts from 0; a live view of the same sums shares it."""
    torch = pytest.importorskip("torch")
    import gc
    vis = torch.zeros(64, dtype=torch.int32)
    xe.reset_integration(vis)
    xe._charge([(vis, 1000)], lambda: 0)
    view = vis.view(8, 8)
    assert xe.integrated_samples(view) == 1000   # same memory, same count
    addr = vis.data_ptr()
    del vis, view
    gc.collect()

    class Stand:                                 # a new tensor at the old address
        def data_ptr(self):
            return addr
    assert xe.integrated_samples(Stand()) == 0


def test_noalloc_rejects_frames_beyond_its_scratch():
    """xe_accumulate_noalloc refuses, on the host and before any device
    call, a frame whose fewest possible time chunks need more partial sums
    than its static array holds; argument errors come first.  (No device
    here: an acceptable frame then fails at the device lookup.)"""
    L = xe.lib()
    vp = ctypes.c_void_p
    fake = vp(0x10000000)

    def call(N, F, T, B=256, packed=fake, vis=fake, count=fake):
        return L.xe_accumulate_noalloc(packed, None, N, F, T, B, vis, count, None)

    # 16 channels of 256 inputs over 8M samples: at most 16,376 steps per
    # chunk, so at least 17 chunks, 16 x 16 x 327,680 B > 64 MiB
    assert call(256, 16, 8 << 20) == xe.XE_ERR_WORKSPACE
    assert call(256, 16, 100, packed=None) == xe.XE_ERR_ARG
    assert call(0, 16, 100) == xe.XE_ERR_ARG
    assert call(256, 16, xe.XE_MAX_SAMPLES + 1) == xe.XE_ERR_OVERFLOW
    assert call(256, 16, 100, vis=vp(0x10000004)) == xe.XE_ERR_ALIGN
    import torch
    if not torch.cuda.is_available():
        assert call(256, 16, 1000) in (xe.XE_ERR_HIP, xe.XE_ERR_UNSUPPORTED)
