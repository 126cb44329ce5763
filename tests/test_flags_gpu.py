"""Per-input flags on the GPU against the oracle (Sec. II-C).

* xe_flag_accumulate's counts (diagonal = per-input counters, off-diagonal =
  intersections) are compared bit-exactly with the oracle's counters, which
  follow the method's own listing of flagged inputs per sample;
* xe_apply_flags must zero exactly the bytes the oracle zeroes;
* the flagged integration end to end (zero, correlate, count, normalise
  per baseline) must match the oracle's flagged correlation and
  normalisation matrix bit for bit, and its float output exactly (both
  divide in double and round once).

Shapes cover one and several 256-input super blocks (off-diagonal pairs),
ragged N, T not a multiple of the 128-sample stage, lost blocks, dense and
bursty flags, flags in the padding bits, no flags and every point flagged.
"""

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


def _case(seed, N, F, T, B, kind="dense", p=0.2, p_loss=0.1):
    rng = np.random.default_rng(seed)
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    mask = synth.bernoulli_mask(rng, F, T, B, p_loss) if p_loss > 0 else None
    if kind == "dense":
        flags = synth.random_flags(rng, T, F, N, p, garbage_padding=True)
    elif kind == "bursty":
        flags = synth.fengine_flags(rng, T, F, N, p, mean_run=32.0, garbage_padding=True)
    elif kind == "none":
        flags = np.zeros((F, T, synth.flag_words(N)), dtype=np.uint32)
    elif kind == "all":
        flags = np.full((F, T, synth.flag_words(N)), 0xFFFFFFFF, dtype=np.uint32)
    else:
        raise ValueError(kind)
    return packed, mask, flags


def _oracle_d(orc, flags, mask, N, B):
    c, d = orc.flag_counters(flags, mask, N, B)
    iu = np.triu_indices(N)
    diag = np.flatnonzero(iu[0] == iu[1])
    assert (d[:, diag] == c).all()   # the oracle's own diagonal reading
    return c, d


COUNT_CASES = [
    # (seed, N, F, T, B, kind, p)
    (1, 37, 3, 700, 64, "dense", 0.2),
    (2, 256, 4, 1000, 256, "bursty", 0.01),
    (3, 256, 2, 640, 128, "dense", 0.5),
    (4, 300, 2, 513, 100, "dense", 0.1),      # two super blocks, ragged
    (5, 600, 1, 300, 64, "bursty", 0.02),     # three super blocks
    (6, 64, 2, 1, 1, "dense", 0.5),           # one sample
    (7, 1, 1, 200, 16, "dense", 0.5),         # one input
    (8, 256, 2, 384, 128, "none", 0.0),       # nothing flagged: every stage skipped
    (9, 96, 2, 260, 32, "all", 1.0),          # every point flagged
    (10, 512, 1, 4096, 256, "bursty", 0.001), # sparse, off-diagonal pair
]


@pytest.mark.parametrize("case", COUNT_CASES, ids=[f"n{c[1]}_f{c[2]}_t{c[3]}_{c[5]}"
                                                  for c in COUNT_CASES])
def test_flag_counts_match_oracle(xe, orc, case):
    seed, N, F, T, B, kind, p = case
    _say(f"flag counts seed={seed} N={N} F={F} T={T} B={B} kind={kind}")
    packed, mask, flags = _case(seed, N, F, T, B, kind, p)
    _, d = _oracle_d(orc, flags, mask, N, B)
    dcount = xe.new_flag_counts(N, F)
    xe.flag_accumulate(_dev(flags), _dev(mask) if mask is not None else None, B, N, dcount)
    torch.cuda.synchronize()
    got = dcount.cpu().numpy().astype(np.int64)
    assert np.array_equal(got, d), np.argwhere(got != d)[:5]


def _sparse_words(rng, F, T, N, k):
    """[F][T][W] flag words with each bit set with probability 2^-k (the AND
    of k random words), garbage in the padding bits, and a flag-free span."""
    shape = (F, T, synth.flag_words(N))
    w = rng.integers(0, 2 ** 32, shape, dtype=np.uint32)
    for _ in range(k - 1):
        w &= rng.integers(0, 2 ** 32, shape, dtype=np.uint32)
    w[:, T // 3:T // 2] = 0
    return w


@pytest.mark.parametrize("seed,N,F,T,B,k", [(14, 32, 512, 40000, 100, 3),
                                            (15, 290, 180, 33000, 7, 7)])
def test_flag_counts_window_capped_chunks(xe, orc, seed, N, F, T, B, k):
    """Frames long enough that one time chunk would pass the kernel's
    1024-word validity window (32,768 samples), with enough channels that
    the occupancy target alone asks for one chunk: the window cap splits
    the frame (ragged last stage), on the diagonal kernel and, at N = 290,
    the off-diagonal one too."""
    rng = np.random.default_rng(seed)
    flags = _sparse_words(rng, F, T, N, k)
    mask = synth.bernoulli_mask(rng, F, T, B, 0.05)
    _say(f"flag counts window cap N={N} F={F} T={T} B={B}")
    _, d = _oracle_d(orc, flags, mask, N, B)
    dcount = xe.new_flag_counts(N, F)
    xe.flag_accumulate(_dev(flags), _dev(mask), B, N, dcount)
    torch.cuda.synchronize()
    got = dcount.cpu().numpy().astype(np.int64)
    assert np.array_equal(got, d), np.argwhere(got != d)[:5]


def test_flag_counts_accumulate_over_frames(xe, orc):
    N, F, B = 300, 2, 64
    dcount = _dev(np.random.default_rng(11).integers(0, 1000, (F, N * (N + 1) // 2),
                                                     dtype=np.int32))
    want = dcount.cpu().numpy().astype(np.int64)
    for seed, T in ((12, 500), (13, 131)):
        _say(f"flag accumulate frame seed={seed} T={T}")
        packed, mask, flags = _case(seed, N, F, T, B, "dense", 0.15)
        _, d = _oracle_d(orc, flags, mask, N, B)
        want += d
        xe.flag_accumulate(_dev(flags), _dev(mask), B, N, dcount)
    torch.cuda.synchronize()
    assert np.array_equal(dcount.cpu().numpy().astype(np.int64), want)


@pytest.mark.parametrize("N", [37, 256])
def test_apply_flags_matches_oracle(xe, orc, N):
    _say(f"apply flags N={N}")
    packed, mask, flags = _case(20 + N, N, 3, 300, 64, "dense", 0.3)
    want = orc.apply_flags(packed, flags)
    dp = _dev(packed)
    xe.apply_flags(dp, _dev(flags))
    torch.cuda.synchronize()
    assert np.array_equal(dp.cpu().numpy(), want)


@pytest.mark.parametrize("case", [(30, 37, 3, 700, 64, "dense", 0.2),
                                  (31, 300, 2, 513, 100, "bursty", 0.05)],
                         ids=["n37", "n300"])
def test_flagged_integration_end_to_end(xe, orc, case):
    seed, N, F, T, B, kind, p = case
    _say(f"flagged integration seed={seed} N={N} F={F} T={T}")
    packed, mask, flags = _case(seed, N, F, T, B, kind, p)
    ev, en = orc.correlate_flagged(packed, mask, flags, B)
    c, d = _oracle_d(orc, flags, mask, N, B)
    n = orc.flag_norm(en, c, d)
    eout = orc.normalize_pairs(ev, n)

    dp, dm, dfl = _dev(packed), _dev(mask), _dev(flags)
    xe.apply_flags(dp, dfl)
    vis, cnt = xe.new_accumulators(N, F)
    dcount = xe.new_flag_counts(N, F)
    xe.accumulate(dp, dm, B, vis, cnt)
    xe.flag_accumulate(dfl, dm, B, N, dcount)
    n_out = torch.empty_like(dcount)
    out = xe.normalize_flagged(vis, cnt, dcount, n_out=n_out)
    torch.cuda.synchronize()
    assert np.array_equal(vis.cpu().numpy().astype(np.int64), ev)
    assert np.array_equal(cnt.cpu().numpy(), en)
    assert np.array_equal(dcount.cpu().numpy().astype(np.int64), d)
    assert np.array_equal(n_out.cpu().numpy().astype(np.int64), n)
    got = out.cpu().numpy()
    assert np.array_equal(got, eout), np.abs(got - eout).max()
    assert (n < en[:, None]).any()   # the flags did change some baselines


def test_normalize_flagged_random_values(xe, orc):
    """Arbitrary int32 sums (not from a frame) with the counts of a random
    flag frame in which input 5 is flagged at every sample (its baselines
    have n = 0): rounding and the n == 0 case against the oracle."""
    rng = np.random.default_rng(40)
    N, F, T, B = 70, 3, 300, 50
    P = N * (N + 1) // 2
    mask = synth.bernoulli_mask(rng, F, T, B, 0.2)
    bits = rng.random((T, F, N)) < 0.1
    bits[:, :, 5] = True
    flags = synth.pack_flags(bits)
    count = orc.valid_counts(mask, F, T, B)
    c, d = orc.flag_counters(flags, mask, N, B)
    n = orc.flag_norm(count, c, d)
    assert (n >= 0).all() and (n == 0).any() and (n > 0).any()
    vis = rng.integers(-2 ** 31 + 1, 2 ** 31 - 1, (F, P, 2)).astype(np.int32)
    want = orc.normalize_pairs(vis.astype(np.int64), n)
    dn = torch.empty((F, P), dtype=torch.int32, device="cuda")
    out = xe.normalize_flagged(_dev(vis), _dev(count), _dev(d.astype(np.int32)), n_out=dn)
    torch.cuda.synchronize()
    assert np.array_equal(dn.cpu().numpy().astype(np.int64), n)
    assert np.array_equal(out.cpu().numpy(), want)


def test_flag_counts_pathfinder_full_size(xe, orc):
    """N=256, 64 channels, 16384 samples with bursty flags at 0.1% and 1%
    block loss: every count against the oracle, and the zeroed frame byte for
    byte."""
    fr = synth.pathfinder()
    rng = np.random.default_rng(50)
    flags = synth.fengine_flags(rng, fr.T, fr.F, fr.N, 1e-3, mean_run=32.0)
    _say(f"flag counts full size N={fr.N} F={fr.F} T={fr.T}")
    _, d = _oracle_d(orc, flags, fr.mask, fr.N, fr.B)
    dcount = xe.new_flag_counts(fr.N, fr.F)
    dfl = _dev(flags)
    xe.flag_accumulate(dfl, _dev(fr.mask), fr.B, fr.N, dcount)
    dp = _dev(fr.packed)
    xe.apply_flags(dp, dfl)
    torch.cuda.synchronize()
    assert np.array_equal(dcount.cpu().numpy().astype(np.int64), d)
    assert np.array_equal(dp.cpu().numpy(), orc.apply_flags(fr.packed, flags))
