"""The capture-safe entry points inside a HIP graph: frame assembly, flag
zeroing, correlation, flag intersections and per-baseline normalisation
captured once and replayed several times, with eager work and
synchronisation between replays; every replay must give the eager result
(integer sums grow by exactly one frame's worth per replay)."""

import sys

import numpy as np
import pytest

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


def test_flag_pipeline_graph_replays(xe):
    rng = np.random.default_rng(140)
    N, S, T = 96, 2, 512
    F = 8 * S
    packed0 = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    flags0 = synth.random_flags(rng, T, F, N, 0.05)
    pk = synth.network_faults(rng, synth.packetize(packed0, flags0), p_drop=0.05,
                              p_dup=0.05, window=8)
    dev = torch.device("cuda")
    dpk = torch.from_numpy(pk).to(dev)
    packed, mask, fl, stats = xe.assemble_frame(dpk, N, S, 0, 0, T)
    vis, cnt = xe.new_accumulators(N, F, dev)
    dc = xe.new_flag_counts(N, F, dev)
    out = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.float32, device=dev)

    def frame(stream):
        xe.assemble_frame(dpk, N, S, 0, 0, T, packed, mask, fl, stats, stream=stream)
        xe.apply_flags(packed, fl, stream=stream)
        xe.accumulate(packed, mask, 4, vis, cnt, stream=stream)
        xe.flag_accumulate(fl, mask, 4, N, dc, stream=stream)
        xe.normalize_flagged(vis, cnt, dc, out=out, stream=stream)

    # eager reference: one frame from zero
    _say("graph: eager frame")
    frame(torch.cuda.current_stream())
    torch.cuda.synchronize()
    v1, c1, d1, o1 = vis.clone(), cnt.clone(), dc.clone(), out.clone()
    vis.zero_(); cnt.zero_(); dc.zero_()
    torch.cuda.synchronize()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            frame(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    # capture does not run the work: sums still zero
    assert not vis.any() and not cnt.any() and not dc.any()
    for k in range(1, 5):
        _say(f"graph: replay {k}")
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(vis, v1 * k), k
        assert torch.equal(cnt, c1 * k), k
        assert torch.equal(dc, d1 * k), k
        assert torch.equal(out, o1), k          # V/n is the same after k equal frames
        junk = torch.randint(0, 256, packed.shape, dtype=torch.uint8, device=dev)
        packed.copy_(junk)                       # eager work between replays
        torch.cuda.synchronize()
    del g


def test_time_shift_graph_replays(xe):
    rng = np.random.default_rng(141)
    T, F, N = 256, 3, 64
    dev = torch.device("cuda")
    packed = torch.from_numpy(rng.integers(0, 256, (T, F, N), dtype=np.uint8)).to(dev)
    flags = torch.from_numpy(synth.random_flags(rng, T, F, N, 0.1).view(np.int32)).to(dev)
    d = torch.from_numpy(rng.integers(-5, 6, N).astype(np.int32)).to(dev)
    out, fo = xe.time_shift(packed, d, flags)
    torch.cuda.synchronize()
    want, wfo = out.clone(), fo.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            xe.time_shift(packed, d, flags, out, fo, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    for k in range(3):
        _say(f"graph shift: replay {k}")
        out.fill_(0x11)
        fo.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want) and torch.equal(fo, wfo), k
    del g
