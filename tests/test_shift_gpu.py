"""Per-input time shifting on the GPU against the oracle: shifted frame and
moved flags bit for bit, and a shifted frame integrated with per-input
flags end to end (zero flagged points, correlate, count intersections,
normalise per baseline) against the oracle's chain."""

import sys

import numpy as np
import pytest

import oracle
from paper_1503_06189_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def xe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_06189_amd import xengine
    xengine.lib()   # fails loudly if the library is missing
    return xengine


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def _delays(rng, N, T):
    d = rng.integers(-9, 10, N).astype(np.int32)
    d[:3] = (T + 2, -T - 1, 0)
    return d


@pytest.mark.parametrize("N,with_flags", [(37, True), (64, False), (256, True)])
def test_time_shift_matches_oracle(xe, orc, N, with_flags):
    rng = np.random.default_rng(100 + N)
    T, F = 300, 3
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    flags = synth.random_flags(rng, T, F, N, 0.1, garbage_padding=True) if with_flags else None
    d = _delays(rng, N, T)
    _say(f"time shift N={N} flags={with_flags}")
    want, wflags = orc.time_shift(packed, flags, d)
    out, fo = xe.time_shift(_dev(packed), _dev(d), _dev(flags) if with_flags else None)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    assert np.array_equal(fo.cpu().numpy().view(np.uint32), wflags)


def test_shifted_flagged_integration(xe, orc):
    rng = np.random.default_rng(120)
    T, F, N, B = 512, 2, 300, 64
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    mask = synth.bernoulli_mask(rng, F, T, B, 0.1)
    bits = synth.unpack_flags(synth.fengine_flags(rng, T, F, N, 0.01), N)
    lost = np.repeat(mask != 0, B, axis=1)[:, :T].T          # [T][F]
    flags = synth.pack_flags(bits | lost[:, :, None])        # losses as flagged points
    d = _delays(rng, N, T)
    _say("shifted flagged integration N=300")
    sp, sf = orc.time_shift(packed, flags, d)
    ev, en = orc.correlate_flagged(sp, None, sf, B)
    c, dd = orc.flag_counters(sf, None, N, B)
    n = orc.flag_norm(en, c, dd)
    eout = orc.normalize_pairs(ev, n)

    out, fo = xe.time_shift(_dev(packed), _dev(d), _dev(flags))
    xe.apply_flags(out, fo)
    vis, cnt = xe.new_accumulators(N, F)
    dcount = xe.new_flag_counts(N, F)
    xe.accumulate(out, None, B, vis, cnt)
    xe.flag_accumulate(fo, None, B, N, dcount)
    nn = torch.empty_like(dcount)
    res = xe.normalize_flagged(vis, cnt, dcount, n_out=nn)
    torch.cuda.synchronize()
    assert np.array_equal(vis.cpu().numpy().astype(np.int64), ev)
    assert np.array_equal(nn.cpu().numpy().astype(np.int64), n)
    assert np.array_equal(res.cpu().numpy(), eout)


def _shift_both(xe, orc, packed, flags, d):
    want, wflags = orc.time_shift(packed, flags, d)
    out, fo = xe.time_shift(_dev(packed), _dev(d), _dev(flags) if flags is not None else None)
    torch.cuda.synchronize()
    got, gflags = out.cpu().numpy(), fo.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    assert np.array_equal(gflags, wflags)
    return got, gflags


@pytest.mark.parametrize("N,spread", [(64, 16), (64, 32), (64, 33), (512, 32), (300, 20),
                                      (300, 33)])
def test_time_shift_staged_and_unstaged_tiles(xe, orc, N, spread):
    """Every tile of 256 inputs whose delays lie within 32 samples of each
    other stages its source rows in LDS; a wider spread reads the frame
    directly.  Both paths, on the 16-byte (N % 16 == 0) and byte copies,
    against the oracle, with a ragged last time tile (T = 300)."""
    rng = np.random.default_rng(150 + N + spread)
    T, F = 300, 2
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    flags = synth.random_flags(rng, T, F, N, 0.1, garbage_padding=True)
    lo = -(spread // 2)
    d = rng.integers(lo, lo + spread + 1, N).astype(np.int32)
    for t0 in range(0, N, 256):
        d[t0], d[min(t0 + 1, N - 1)] = lo, lo + spread    # the tile's full spread
    _say(f"time shift staged/unstaged N={N} spread={spread}")
    _shift_both(xe, orc, packed, flags, d)


@pytest.mark.parametrize("N,F,T", [(1, 1, 1), (1, 2, 5), (16, 1, 1), (33, 3, 31),
                                   (4096, 1, 3)])
def test_time_shift_degenerate(xe, orc, N, F, T):
    """Smallest frames, the widest input count, zero delays (the frame and
    the flags pass through unchanged) and delays at the int32 limits (every
    sample shifted in from outside: 0 + 0i and flagged)."""
    rng = np.random.default_rng(170 + N + T)
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    flags = synth.random_flags(rng, T, F, N, 0.3, garbage_padding=True)
    _say(f"time shift degenerate N={N} F={F} T={T}")
    got, gflags = _shift_both(xe, orc, packed, flags, np.zeros(N, np.int32))
    assert np.array_equal(got, packed)
    assert np.array_equal(synth.unpack_flags(gflags, N), synth.unpack_flags(flags, N))
    ext = np.where(np.arange(N) % 2 == 0, np.iinfo(np.int32).max,
                   np.iinfo(np.int32).min).astype(np.int32)
    got, gflags = _shift_both(xe, orc, packed, flags, ext)
    assert (got == 0x88).all()
    assert synth.unpack_flags(gflags, N).all()


def test_time_shift_pathfinder_full_size(xe, orc):
    """The pathfinder share (N=256, F=64, T=16384) with delays in [-8, 8]
    samples and bursty flags, the configuration the shift is timed on:
    the whole shifted frame and its flags against the oracle."""
    fr = synth.pathfinder()
    rng = np.random.default_rng(31)
    flags = synth.fengine_flags(rng, fr.T, fr.F, fr.N, 1e-3)
    d = rng.integers(-8, 9, fr.N).astype(np.int32)
    _say("time shift pathfinder full size")
    _shift_both(xe, orc, fr.packed, flags, d)
