"""HIP path vs the oracle, element by element (GPU).

Integer visibilities and counts must be bit-exact.  The stated tolerance of
the normalised float32 output is 1e-6 relative to the oracle's FP64
normalisation; both sides divide the same integers in double and round once
to float32, so the tests require the float32 values to be identical, which
implies that tolerance.  The full-size workloads are compared over their
whole output, in the launch configuration the benchmark times.
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
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_gpu(xe, fr, normalize=False):
    packed = _dev(fr.packed)
    mask = _dev(fr.mask) if fr.mask is not None else None
    vis, cnt = xe.correlate_frame(packed, mask, fr.B)
    out = xe.normalize(vis, cnt) if normalize else None
    torch.cuda.synchronize()
    res = (vis.cpu().numpy().astype(np.int64), cnt.cpu().numpy())
    if normalize:
        res = res + (out.cpu().numpy(),)
    return res


def assert_same_floats(got, want):
    """float32 outputs identical bit for bit (within 1e-6 relative a fortiori)."""
    assert got.dtype == np.float32 and want.dtype == np.float32
    assert got.shape == want.shape
    bad = np.argwhere(got.view(np.uint32) != want.view(np.uint32))
    assert bad.size == 0, f"{len(bad)} normalised values differ, first {bad[:5].tolist()}"
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=0)


def check_full(xe, orc, fr, normalize=True, expect=None):
    _say(f"case {fr.name} N={fr.N} F={fr.F} T={fr.T} B={fr.B} seed={fr.seed}")
    got = run_gpu(xe, fr, normalize)
    ev, en = expect if expect is not None else orc.correlate(fr.packed, fr.mask, fr.B)
    assert np.array_equal(got[1], en), "counts differ"
    bad = np.argwhere(got[0] != ev)
    assert bad.size == 0, f"{len(bad)} visibilities differ, first {bad[:5].tolist()}"
    if normalize:
        assert_same_floats(got[2], orc.normalize(ev, en))


# ---------------------------------------------------------------------------
# small and ragged shapes, whole output
# ---------------------------------------------------------------------------

def test_tiny_config(xe, orc):
    check_full(xe, orc, synth.tiny())


SHAPES = [
    # N, F, T, B, p_loss
    (1, 1, 1, 1, 0.0),
    (2, 3, 5, 2, 0.3),
    (3, 2, 33, 4, 0.3),
    (16, 4, 31, 256, 0.0),
    (31, 2, 100, 7, 0.2),
    (32, 2, 64, 16, 0.1),
    (33, 3, 97, 32, 0.2),
    (64, 2, 300, 50, 0.1),
    (100, 2, 257, 64, 0.2),
    (255, 1, 129, 128, 0.1),
    (256, 2, 1000, 256, 0.05),
    (257, 1, 200, 3, 0.2),
    (300, 1, 95, 1000, 0.0),
    (513, 1, 70, 16, 0.2),
    # few channels over long frames: dozens of time chunks merged, counts
    # taken by the merge
    (64, 1, 20000, 100, 0.1),
    (300, 2, 9001, 37, 0.1),
]


@pytest.mark.parametrize("N,F,T,B,p", SHAPES, ids=[f"N{s[0]}_F{s[1]}_T{s[2]}_B{s[3]}" for s in SHAPES])
def test_shapes_random_bytes(xe, orc, N, F, T, B, p):
    """Uniform random bytes (every code, -8 included), garbage in lost
    blocks, ragged N, T and B."""
    fr = synth.random_bytes_frame(1000 + N + T, N, F, T, B, p_loss=p, fill="garbage")
    check_full(xe, orc, fr)


def test_all_lost_channel_and_no_mask(xe, orc):
    fr = synth.random_bytes_frame(5, 40, 3, 300, 64, p_loss=0.0)
    fr.mask = np.zeros((3, 5), dtype=np.uint8)
    fr.mask[1, :] = 1
    check_full(xe, orc, fr)
    fr.mask = None
    check_full(xe, orc, fr)


def test_accumulate_linearity(xe, orc):
    """accumulate(F1) + accumulate(F2) on the device == oracle of F1 then F2."""
    N, F, B = 96, 3, 32
    fr = synth.random_bytes_frame(77, N, F, 640, B, p_loss=0.1)
    T1 = 224
    vis, cnt = xe.new_accumulators(N, F)
    xe.accumulate(_dev(fr.packed[:T1]), _dev(fr.mask[:, :T1 // B]), B, vis, cnt)
    xe.accumulate(_dev(fr.packed[T1:]), _dev(fr.mask[:, T1 // B:]), B, vis, cnt)
    torch.cuda.synchronize()
    ev, en = orc.correlate(fr.packed, fr.mask, B)
    assert np.array_equal(vis.cpu().numpy().astype(np.int64), ev)
    assert np.array_equal(cnt.cpu().numpy(), en)


def test_unaligned_packed_pointer(xe, orc):
    """A frame that starts at an odd address takes the byte-load path."""
    fr = synth.random_bytes_frame(9, 64, 2, 100, 16, p_loss=0.2)
    buf = torch.zeros(fr.packed.size + 1, dtype=torch.uint8, device="cuda")
    buf[1:] = _dev(fr.packed.reshape(-1))
    packed = buf[1:].view(fr.T, fr.F, fr.N)
    assert packed.data_ptr() % 4 == 1
    vis, cnt = xe.correlate_frame(packed, _dev(fr.mask), fr.B)
    torch.cuda.synchronize()
    ev, en = orc.correlate(fr.packed, fr.mask, fr.B)
    assert np.array_equal(vis.cpu().numpy().astype(np.int64), ev)


# ---------------------------------------------------------------------------
# full-size workloads: sampled baselines + properties that hold at any size
# ---------------------------------------------------------------------------

def _sample_pairs(rng, N, F, n):
    fs = rng.integers(0, F, n)
    i = rng.integers(0, N, n)
    j = rng.integers(0, N, n)
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    # always include the corners and the diagonal
    fs = np.concatenate([fs, [0, F - 1, F - 1, 0]])
    lo = np.concatenate([lo, [0, 0, N - 1, N - 1]])
    hi = np.concatenate([hi, [0, N - 1, N - 1, N - 1]])
    return fs, lo, hi


def check_sampled(xe, orc, fr, n_pairs=3000):
    _say(f"case {fr.name} N={fr.N} F={fr.F} T={fr.T} B={fr.B} seed={fr.seed} (sampled)")
    vis, cnt, out = run_gpu(xe, fr, normalize=True)
    N, F = fr.N, fr.F
    # counts: samples outside lost blocks (numpy, independent of the oracle)
    if fr.mask is not None:
        lost_per_blk = np.minimum(fr.B, fr.T - np.arange(fr.nblk) * fr.B)
        exp_n = fr.T - (fr.mask.astype(np.int64) * lost_per_blk[None, :]).sum(1)
    else:
        exp_n = np.full(F, fr.T)
    assert np.array_equal(cnt, exp_n)
    rng = np.random.default_rng(fr.seed)
    fs, i, j = _sample_pairs(rng, N, F, n_pairs)
    exp = orc.correlate_pairs(fr.packed, fr.mask, fr.B, fs, i, j)
    idx = i * N - i * (i - 1) // 2 + (j - i)
    got = vis[fs, idx]
    bad = np.argwhere((got != exp).any(axis=1))
    assert bad.size == 0, f"{len(bad)} sampled baselines differ: {bad[:5].ravel().tolist()}"
    # autocorrelations: real, non-negative, at every input of every channel
    di = np.arange(N)
    dia = di * N - di * (di - 1) // 2
    assert not vis[:, dia, 1].any()
    assert (vis[:, dia, 0] >= 0).all()
    # normalisation on the sampled baselines: each sample as a one-input
    # "channel" of the oracle's normalisation
    eo = orc.normalize(exp.reshape(-1, 1, 2), exp_n[fs])
    np.testing.assert_allclose(out[fs, idx], eo[:, 0, :], rtol=1e-6, atol=0)


@pytest.fixture(scope="module")
def pathfinder(orc):
    fr = synth.pathfinder()
    _say(f"oracle: {fr.name} N={fr.N} F={fr.F} T={fr.T} (whole frame)")
    return fr, orc.correlate(fr.packed, fr.mask, fr.B)


def test_pathfinder_full_size(xe, orc, pathfinder):
    """N=256, 64 channels, 16384 samples, 1% block loss (the bench workload):
    every visibility, count and normalised value of the frame."""
    fr, expect = pathfinder
    check_full(xe, orc, fr, expect=expect)


def test_pathfinder_accumulate_as_benched(xe, orc, pathfinder):
    """The benchmark's call: xe_accumulate into resident sums (its time-
    chunked launch and merge), three frames, then xe_normalize; the whole
    integration equals three times the oracle's frame."""
    fr, (ev, en) = pathfinder
    _say(f"case {fr.name} accumulate x3 (whole frame)")
    plan = xe.plan_query(fr.N, fr.F, fr.T, fr.B)
    assert plan.splits > 1    # the chunked path with its merge kernel
    packed, mask = _dev(fr.packed), _dev(fr.mask)
    vis, cnt = xe.new_accumulators(fr.N, fr.F, packed.device)
    for _ in range(3):
        xe.accumulate(packed, mask, fr.B, vis, cnt)
    out = xe.normalize(vis, cnt)
    torch.cuda.synchronize()
    assert np.array_equal(cnt.cpu().numpy(), 3 * en)
    got = vis.cpu().numpy()
    bad = np.argwhere(got != 3 * ev)
    assert bad.size == 0, f"{len(bad)} visibilities differ, first {bad[:5].tolist()}"
    assert_same_floats(out.cpu().numpy(), orc.normalize(3 * ev, 3 * en))


def test_pathfinder_sampled_pairs(xe, orc):
    """Sampled baselines through the oracle's per-pair routine and the
    autocorrelation properties, on the same frame."""
    check_sampled(xe, orc, synth.pathfinder())


def test_large_n_full_size(xe, orc):
    """N=2048, 16 channels, 8192 samples, 0.5% loss: the whole output
    (2,098,176 baselines per channel)."""
    fr = synth.large_n()
    _say(f"oracle: {fr.name} N={fr.N} F={fr.F} T={fr.T} (whole frame, about a minute)")
    check_full(xe, orc, fr)


def test_large_n_sampled_pairs(xe, orc):
    check_sampled(xe, orc, synth.large_n(), n_pairs=2000)


def test_max_n(xe, orc):
    """N=4096 (the largest a call takes), whole output."""
    fr = synth.random_bytes_frame(4096, 4096, 1, 40, 16, p_loss=0.2)
    check_full(xe, orc, fr)


def test_block_longer_than_frame(xe, orc):
    """A loss block longer than the frame (up to INT32_MAX samples) is one
    block covering it: its single mask entry decides every sample."""
    for B in (301, 1 << 20, 2**31 - 1):
        fr = synth.random_bytes_frame(31, 40, 3, 300, B, p_loss=0.0, fill="garbage")
        fr.mask = np.array([[0], [1], [0]], dtype=np.uint8)
        check_full(xe, orc, fr)


def test_overflow_edge(xe):
    """All bytes 0x00 (x = -8-8i) over the longest frame a call accepts:
    Re V = 128 T = 2,147,483,520 (fits int32), Im V = 0 everywhere."""
    T, F, N = 16_777_215, 1, 16
    _say(f"case overflow_edge N={N} F={F} T={T}")
    packed = torch.zeros((T, F, N), dtype=torch.uint8, device="cuda")
    vis, cnt = xe.correlate_frame(packed, None, 256)
    torch.cuda.synchronize()
    v = vis.cpu().numpy()
    assert int(cnt.cpu()[0]) == T
    assert (v[..., 0] == 128 * T).all() and not v[..., 1].any()
    del packed


def test_bad_arguments_raise(xe):
    packed = torch.zeros((4, 1, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        xe.correlate_frame(packed, torch.zeros((1, 3), dtype=torch.uint8, device="cuda"), 2)
    with pytest.raises(xe.XEngineError):
        xe.correlate_frame(torch.zeros((0, 1, 8), dtype=torch.uint8, device="cuda"), None, 2)


def test_integration_bound_refused(xe):
    """An accumulate that would pass the int32 integration bound raises
    XE_ERR_OVERFLOW and leaves the sums untouched; correlate_frame starts a
    new count."""
    fr = synth.tiny()
    packed = _dev(fr.packed)
    vis, cnt = xe.new_accumulators(fr.N, fr.F, packed.device)
    xe.accumulate(packed, None, fr.B, vis, cnt)
    torch.cuda.synchronize()
    before = vis.clone()
    xe._charge([(vis, xe.XE_MAX_SAMPLES - fr.T - 1)], lambda: 0)
    with pytest.raises(xe.XEngineError) as e:
        xe.accumulate(packed, None, fr.B, vis, cnt)
    assert e.value.status == xe.XE_ERR_OVERFLOW
    torch.cuda.synchronize()
    assert torch.equal(vis, before)
    xe.correlate_frame(packed, None, fr.B, vis, cnt)
    assert xe.integrated_samples(vis) == fr.T
