"""Both tile geometries of frames with N <= 128 against the oracle (GPU).

A frame of at most four 32-input blocks runs either as a padded 256-input
super-block ("super": 36 tiles, one 32-sample step per loop step) or in the
halves geometry ("halves": the 10 tiles of the 4-block triangle over two
consecutive 32-sample steps per loop step, the odd-step sums handed to the
even-step waves through LDS).  Every case below runs under both and must
equal the oracle bit for bit: single frames (overwrite and accumulate, one
time chunk and many, an odd number of 32-sample steps, ragged N, lost
blocks, the unaligned byte path), a frame whose one chunk passes the
kernel's 2048-step validity window, and batches built and replayed under
each geometry.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1503_06189_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GEOMS = ("super", "halves")


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


@pytest.fixture(scope="module")
def handles(xe):
    out = {}
    for g in GEOMS:
        h = xe.Handle(0)
        h.set_geometry(g)
        out[g] = h
    yield out
    for h in out.values():
        h.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_plan_tiles_per_geometry(xe):
    """The plan reports 10 tiles for a 4-block frame in the halves geometry
    (the default) and the padded 36 otherwise; larger frames are unchanged."""
    assert xe.plan_query(128, 4, 4096).mfma_tiles == 10
    assert xe.plan_query(33, 4, 4096).mfma_tiles == 10
    assert xe.plan_query(129, 4, 4096).mfma_tiles == 36
    assert xe.plan_query(256, 4, 4096).mfma_tiles == 36


def test_set_geometry_rejects_unknown(xe):
    h = xe.Handle(0)
    try:
        with pytest.raises(xe.XEngineError):
            h.set_geometry(7)
    finally:
        h.close()


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("N,F,T,B,p", [
    (128, 3, 5024, 256, 0.1),   # 157 steps: an odd count, many chunks
    (64, 256, 8192, 256, 0.05),  # one chunk of 256 steps
    (100, 2, 700, 64, 0.2),     # ragged N and T
    (37, 5, 33, 16, 0.3),       # ragged, unaligned byte path (N % 4 != 0)
    (4, 1, 96, 32, 0.0),        # one block, three steps
    (1, 2, 1, 1, 0.0),          # one input, one sample
    (32, 300, 65, 64, 0.1),     # one block, many channels, 3 steps
])
def test_geometry_matches_oracle(xe, orc, handles, geom, N, F, T, B, p):
    h = handles[geom]
    fr = synth.random_bytes_frame(seed=400 + N + T + F, N=N, F=F, T=T, B=B, p_loss=p)
    _say(f"geometry {geom} N={N} F={F} T={T} B={B}")
    ev, en = orc.correlate(fr.packed, fr.mask, fr.B)
    packed = _dev(fr.packed)
    mask = _dev(fr.mask) if fr.mask is not None else None
    vis, cnt = xe.correlate_frame(packed, mask, fr.B, handle=h)
    torch.cuda.synchronize()
    assert np.array_equal(cnt.cpu().numpy(), en)
    got = vis.cpu().numpy().astype(np.int64)
    bad = np.argwhere(got != ev)
    assert bad.size == 0, f"{len(bad)} visibilities differ, first {bad[:5].tolist()}"
    # accumulate on top: twice the sums
    xe.accumulate(packed, mask, fr.B, vis, cnt, handle=h)
    torch.cuda.synchronize()
    assert np.array_equal(vis.cpu().numpy().astype(np.int64), 2 * ev)
    assert np.array_equal(cnt.cpu().numpy(), 2 * en)


@pytest.mark.parametrize("geom", GEOMS)
def test_geometry_long_chunk_passes_validity_window(xe, orc, handles, geom):
    """256 channels fill the GPU with one time chunk each; 70,016 samples are
    2,188 steps, past the kernel's 2,048-word validity window, with lost
    blocks on both sides of the window's edge.  Channels 0, 1 and 255 are
    compared with the oracle."""
    N, F, T, B = 64, 256, 70016, 256
    rng = np.random.default_rng(77)
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    mask = synth.bernoulli_mask(rng, F, T, B, 0.05)
    mask[:, 255:258] = 1    # blocks around sample 65,536
    info = xe.plan_query(N, F, T, B)
    assert info.splits == 1
    _say(f"geometry {geom} long chunk N={N} F={F} T={T}")
    vis, cnt = xe.correlate_frame(_dev(packed), _dev(mask), B, handle=handles[geom])
    torch.cuda.synchronize()
    got_v = vis.cpu().numpy().astype(np.int64)
    got_n = cnt.cpu().numpy()
    for f in (0, 1, 255):
        ev, en = orc.correlate(np.ascontiguousarray(packed[:, f:f + 1, :]),
                               np.ascontiguousarray(mask[f:f + 1]), B)
        assert got_n[f] == en[0], f"channel {f} count"
        assert np.array_equal(got_v[f], ev[0]), f"channel {f} visibilities"


def _batch(xe, frames):
    insts = []
    for fr in frames:
        p = _dev(fr.packed)
        m = _dev(fr.mask) if fr.mask is not None else None
        v, c = xe.new_accumulators(fr.N, fr.F, p.device)
        insts.append((fr, p, m, v, c))
    return insts


@pytest.mark.parametrize("geom", GEOMS)
def test_geometry_batch_plan_matches_oracle(xe, orc, handles, geom):
    """An uneven batch of 24 instances (N from 64 to 512, small ones under
    the chosen geometry) built as a plan and replayed twice."""
    specs = synth.batched_specs(synth.SEEDS["batched"] + 3, 24, 0.125,
                                (64, 96, 128, 256, 512))
    frames = [synth.instance_frame(s) for s in specs]
    insts = _batch(xe, frames)
    items = [(p, m, fr.B, v, c) for fr, p, m, v, c in insts]
    _say(f"geometry {geom} batch of {len(items)}")
    plan = xe.BatchPlan(items, handle=handles[geom], geometry=geom)
    try:
        plan.run()
        plan.run()
        torch.cuda.synchronize()
    finally:
        plan.release()
    for k, (fr, p, m, v, c) in enumerate(insts):
        ev, en = orc.correlate(fr.packed, fr.mask, fr.B)
        assert np.array_equal(c.cpu().numpy(), 2 * en), f"instance {k} N={fr.N} counts"
        assert np.array_equal(v.cpu().numpy().astype(np.int64), 2 * ev), \
            f"instance {k} N={fr.N} visibilities"
