"""Generator determinism and shapes (CPU)."""

import numpy as np

from paper_1503_06189_amd import synth


def test_seed_determinism():
    a = synth.pathfinder(N=8, F=3, T=700, B=64)
    b = synth.pathfinder(N=8, F=3, T=700, B=64)
    assert np.array_equal(a.packed, b.packed) and np.array_equal(a.mask, b.mask)
    c = synth.pathfinder(seed=5, N=8, F=3, T=700, B=64)
    assert not np.array_equal(a.packed, c.packed)


def test_shapes_and_partial_block():
    fr = synth.large_n(N=32, F=2, T=1000, B=256)
    assert fr.packed.shape == (1000, 2, 32) and fr.mask.shape == (2, 4)
    t = synth.tiny()
    assert t.packed.shape == (256, 8, 16) and not t.mask.any()


def test_values_clipped_and_zero_fill():
    fr = synth.pathfinder(N=16, F=4, T=2048, B=256, p_loss=0.3)
    hi = (fr.packed >> 4).astype(int) - 8
    lo = (fr.packed & 15).astype(int) - 8
    assert hi.min() >= -7 and hi.max() <= 7 and lo.min() >= -7 and lo.max() <= 7
    for f, b in zip(*np.nonzero(fr.mask)):
        assert (fr.packed[b * 256:(b + 1) * 256, f] == synth.ZERO_BYTE).all()


def test_encode_rejects_out_of_range():
    import pytest
    with pytest.raises(ValueError):
        synth.encode(np.array([8]), np.array([0]))


def test_gilbert_elliott_cap_and_rate():
    rng = np.random.default_rng(0)
    m = synth.gilbert_elliott_mask(rng, 200, 16, 0.05, 4.0, 0.10)
    assert m.shape == (200, 16)
    assert (m.sum(axis=1) <= 1).all()        # floor(0.10 * 16) = 1
    m2 = synth.gilbert_elliott_mask(np.random.default_rng(1), 50, 4000, 0.05, 4.0, 1.0)
    assert 0.03 < m2.mean() < 0.07


def test_batched_and_streams():
    specs = synth.batched_specs(n_inst=16)
    assert len(specs) == 16
    for s in specs:
        assert s.N in (64, 128, 256, 512, 1024) and 1024 <= s.T <= 65536 and s.T % 256 == 0
    st = synth.streaming_streams()
    assert len(st) == 8 and abs(sum(s.rate_bps for s in st) - 51.2e9) < 1
    fr = synth.stream_frame(st[0], 3)
    assert fr.packed.shape == (4096, st[0].F, st[0].N)
