"""Streaming server on the GPU: results alone equal results in the mix,
both equal the oracle, and a tight HBM budget delays frames without
changing any result."""

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
def srv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_06189_amd import serve, xengine
    xengine.lib()
    return serve


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.fixture(scope="module")
def specs():
    return synth.streaming_streams(n_streams=4, total_bps=4 * 2e9, T=1024,
                                   n_choices=(64, 128), f_range=(2, 4), l_range=(2, 3),
                                   max_loss=0.10)


@pytest.fixture(scope="module")
def pool(specs):
    return {s.stream_id: [synth.stream_frame(s, k, 256) for k in range(2)] for s in specs}


def _expected(orc, spec, pool, sequence, index):
    L = spec.frames_per_integration
    vis = cnt = None
    for k in sequence[index * L:(index + 1) * L]:
        fr = pool[spec.stream_id][k]
        v, n = orc.correlate(fr.packed, fr.mask, fr.B)
        vis = v if vis is None else vis + v
        cnt = n if cnt is None else cnt + n
    return vis, cnt, orc.normalize(vis, cnt)


def _by_stream(res):
    return {sid: [(r.index, r.vis, r.count, r.out) for r in lst]
            for sid, lst in res.server.results.items()}


def test_mix_equals_alone_and_oracle(srv, orc, specs, pool):
    n_int = 2
    mix = srv.run_load(specs, integrations=n_int, speed=50.0, pool=pool)
    _say(f"mix: {mix.stats}")
    assert mix.stats["frames"] == sum(n_int * s.frames_per_integration for s in specs)
    assert mix.stats["mean_batch"] > 1.0      # frames of several streams shared launches
    got_mix = _by_stream(mix)
    for s in specs:
        alone = srv.run_load([s], integrations=n_int, speed=50.0, pool=pool)
        got_alone = _by_stream(alone)[s.stream_id]
        assert len(got_alone) == n_int and len(got_mix[s.stream_id]) == n_int
        for (ia, va, ca, oa), (im, vm, cm, om) in zip(got_alone, got_mix[s.stream_id]):
            assert ia == im
            assert np.array_equal(va, vm) and np.array_equal(ca, cm)
            assert np.array_equal(oa.view(np.uint32), om.view(np.uint32))
        for idx, v, c, o in got_mix[s.stream_id]:
            ev, en, eo = _expected(orc, s, pool, mix.sequence[s.stream_id], idx)
            assert np.array_equal(c, en), f"stream {s.stream_id} integration {idx} counts"
            assert np.array_equal(v.astype(np.int64), ev), f"stream {s.stream_id} vis"
            assert np.array_equal(o.view(np.uint32), eo.view(np.uint32))


def test_streaming_shapes_mix_equals_alone_and_oracle(srv, orc):
    """Streams of the serving workload's shapes (N 128, 256 and 512; 16 to
    64 channels; 4096-sample frames; bursty loss up to 10% per frame), one
    whole integration of distinct frames each: every result in the mix
    equals the result alone and the oracle, bit for bit."""
    from paper_1503_06189_amd.synth import StreamSpec, stream_frame
    base = synth.SEEDS["streaming"] * 1000 + 500
    specs = [StreamSpec(0, 128, 64, 4096, 3, 0.05, 6.4e9, base + 0),
             StreamSpec(1, 256, 16, 4096, 3, 0.03, 6.4e9, base + 1),
             StreamSpec(2, 512, 24, 4096, 3, 0.05, 6.4e9, base + 2)]
    pool = {s.stream_id: [stream_frame(s, k, 256) for k in range(3)] for s in specs}
    _say("streaming shapes: " + " ".join(f"N={s.N},F={s.F}" for s in specs))
    mix = srv.run_load(specs, integrations=1, distinct=3, speed=float("inf"), pool=pool)
    assert mix.stats["mean_batch"] > 1.0
    got_mix = _by_stream(mix)
    for s in specs:
        assert mix.sequence[s.stream_id] == [0, 1, 2]    # three distinct frames
        alone = _by_stream(srv.run_load([s], integrations=1, distinct=3,
                                        speed=float("inf"), pool=pool))[s.stream_id]
        ((ia, va, ca, oa),) = alone
        ((im, vm, cm, om),) = got_mix[s.stream_id]
        assert ia == im == 0
        assert np.array_equal(va, vm) and np.array_equal(ca, cm)
        assert np.array_equal(oa.view(np.uint32), om.view(np.uint32))
        ev, en, eo = _expected(orc, s, pool, mix.sequence[s.stream_id], 0)
        assert np.array_equal(cm, en), f"stream {s.stream_id} counts"
        assert np.array_equal(vm.astype(np.int64), ev), f"stream {s.stream_id} vis"
        assert np.array_equal(om.view(np.uint32), eo.view(np.uint32)), \
            f"stream {s.stream_id} normalised"


def test_tight_budget_delays_but_does_not_change(srv, specs, pool):
    """A frame pool of two slots, each holding a 256-sample slice of the
    largest frame: frames wait for slots (admission waits), the HBM in use
    never passes the budget, and every result equals the roomy run's."""
    from paper_1503_06189_amd.serve import SlotPool, StreamConfig, _Stream
    cfgs = [StreamConfig(s.stream_id, s.N, s.F, s.T, 256, s.frames_per_integration)
            for s in specs]
    resident = sum(_Stream.resident_bytes_for(c) for c in cfgs)
    slot = max(256 * c.F * c.N for c in cfgs)
    pool_bytes = 2 * (slot + SlotPool.MASK_BYTES)
    budget = resident + pool_bytes
    free = srv.run_load(specs, integrations=1, speed=float("inf"), pool=pool)
    tight = srv.run_load(specs, integrations=1, speed=float("inf"), pool=pool,
                         hbm_budget=budget, slot_bytes=slot, pool_bytes=pool_bytes)
    _say(f"tight: {tight.stats}")
    assert tight.stats["hbm_peak_used"] <= budget
    assert tight.stats["admission_waits"] > 0
    a, b = _by_stream(free), _by_stream(tight)
    for sid in a:
        assert len(a[sid]) == len(b[sid]) == 1
        for (i1, v1, c1, o1), (i2, v2, c2, o2) in zip(a[sid], b[sid]):
            assert i1 == i2 and np.array_equal(v1, v2) and np.array_equal(c1, c2)
            assert np.array_equal(o1.view(np.uint32), o2.view(np.uint32))


def test_sliced_copies_equal_whole_frames_and_oracle(srv, orc, specs, pool):
    """Frames copied and accumulated in 256-sample time slices (4 per
    frame) give the same integrations as whole frames, bit for bit, and the
    oracle's."""
    n_int = 2
    whole = srv.run_load(specs, integrations=n_int, speed=50.0, pool=pool)
    sliced = srv.run_load(specs, integrations=n_int, speed=50.0, pool=pool, slice_samples=256)
    assert sliced.stats["batches"] > whole.stats["batches"]
    a, b = _by_stream(whole), _by_stream(sliced)
    for s in specs:
        assert len(a[s.stream_id]) == len(b[s.stream_id]) == n_int
        for (i1, v1, c1, o1), (i2, v2, c2, o2) in zip(a[s.stream_id], b[s.stream_id]):
            assert i1 == i2 and np.array_equal(v1, v2) and np.array_equal(c1, c2)
            assert np.array_equal(o1.view(np.uint32), o2.view(np.uint32))
            ev, en, eo = _expected(orc, s, pool, sliced.sequence[s.stream_id], i2)
            assert np.array_equal(c2, en) and np.array_equal(v2.astype(np.int64), ev)
    bd = sliced.stats["latency_breakdown"]
    assert set(bd) == {"wait", "copy", "finish"}


def test_budget_too_small(srv, specs):
    """A budget whose frame pool holds no slot, and one whose pool leaves no
    room for a stream's accumulators, are refused up front."""
    from paper_1503_06189_amd.serve import SlotPool, StreamConfig, StreamServer
    s = specs[0]
    with pytest.raises(MemoryError):
        StreamServer(hbm_budget=1 << 16)
    slot = 256 * s.F * s.N
    server = StreamServer(hbm_budget=slot + SlotPool.MASK_BYTES + 1024, slot_bytes=slot,
                          pool_bytes=slot + SlotPool.MASK_BYTES)
    with pytest.raises(MemoryError):
        server.open(StreamConfig(s.stream_id, s.N, s.F, s.T, 256, s.frames_per_integration))


def test_device_resident_serving_accounts_every_frame(srv, specs, pool):
    """Serving loop with frames already in HBM (no host link, whole frames,
    no copies): every frame is served once, its bytes counted once, and the
    latency statistics are consistent (a rate comparison with plain
    launches is the benchmark's, not a test's)."""
    n = 12
    res = srv.run_load(specs, frames_per_stream=n, speed=float("inf"), pool=pool,
                       device_resident=True, hbm_budget=1 << 34, max_inflight=2)
    plain = srv.run_plain(specs, pool, n)
    _say(f"served {res.stats['gbps']:.1f} Gb/s vs plain {plain['gbps']:.1f} Gb/s")
    assert res.stats["frames"] == n * len(specs) == plain["frames"]
    assert res.server.samples_done == n * sum(s.N * s.F * s.T for s in specs)
    assert res.stats["p50_ms"] is not None and res.stats["p50_ms"] <= res.stats["p99_ms"]
    assert res.stats["latency_breakdown"]["copy"]["p99_ms"] == 0.0


def test_aligned_streams_combined_by_stream_id(srv, orc):
    """Streams of one correlator (same N, their own channels) integrate over
    sequence-number windows of 2 frames; the combiner joins each window's
    results in stream-id order.  One stream misses its first frame (its
    window 0 holds one frame), frames are submitted with the streams
    interleaved in a scrambled order, and every combined window equals the
    oracle's sums of exactly the frames of that window, channel by channel;
    the .npz dump reads back the same."""
    import os
    import tempfile
    from paper_1503_06189_amd.serve import Combiner, Frame, StreamConfig, StreamServer
    from paper_1503_06189_amd.synth import StreamSpec, stream_frame
    N, T, B, L = 64, 512, 64, 2
    specs = [StreamSpec(7, N, 3, T, L, 0.05, 1e9, 9001),
             StreamSpec(2, N, 2, T, L, 0.05, 1e9, 9002),
             StreamSpec(5, N, 4, T, L, 0.05, 1e9, 9003)]
    seqs = {7: [0, 1, 2, 3, 4, 5], 2: [0, 1, 2, 3, 4, 5], 5: [1, 2, 3, 4, 5]}
    frames = {s.stream_id: {q: stream_frame(s, q, B) for q in seqs[s.stream_id]} for s in specs}
    comb = Combiner([s.stream_id for s in specs])
    server = StreamServer(hbm_budget=1 << 30, on_result=comb.add)
    for s in specs:
        server.open(StreamConfig(s.stream_id, N, s.F, T, B, L, aligned=True))
    order = [(q, s.stream_id) for q in range(6) for s in specs if q in seqs[s.stream_id]]
    rng = np.random.default_rng(4)
    # scramble across streams, keeping each stream's own frames in order
    keys = {k: rng.random() for k in order}
    order.sort(key=lambda k: (k[0] + keys[k] * 1.5))
    for q, sid in order:
        fr = frames[sid][q]
        server.submit(Frame(sid, q, torch.from_numpy(fr.packed).cuda(),
                            torch.from_numpy(fr.mask).cuda(), 0.0))
        server.step()
    server.sync()
    for s in specs:
        server.flush(s.stream_id)
    torch.cuda.synchronize()
    assert not comb.incomplete()
    assert [c.window for c in comb.combined] == [0, 1, 2]
    ids = sorted(s.stream_id for s in specs)
    for c in comb.combined:
        assert c.stream_ids == ids
        want_v, want_n, frames_per = [], [], []
        for sid in ids:
            qs = [q for q in seqs[sid] if q // L == c.window]
            frames_per.append(len(qs))
            ev = en = None
            for q in qs:
                v, n = orc.correlate(frames[sid][q].packed, frames[sid][q].mask, B)
                ev = v if ev is None else ev + v
                en = n if en is None else en + n
            want_v.append(ev)
            want_n.append(en)
        assert c.frames == frames_per
        ev, en = np.concatenate(want_v), np.concatenate(want_n)
        assert np.array_equal(c.count, en), f"window {c.window} counts"
        assert np.array_equal(c.vis.astype(np.int64), ev), f"window {c.window} vis"
        assert np.array_equal(c.out.view(np.uint32), orc.normalize(ev, en).view(np.uint32))
        with tempfile.TemporaryDirectory() as d:
            path = os.path.join(d, f"w{c.window}.npz")
            c.save(path)
            back = np.load(path)
            assert np.array_equal(back["vis"], c.vis) and np.array_equal(back["out"], c.out)
            assert list(back["stream_ids"]) == ids and int(back["window"]) == c.window
    # stream 5 lacked frame 0: its window-0 integration holds one frame
    assert comb.combined[0].frames == [2, 1, 2]


def test_snapshot_restore_equals_uninterrupted(srv, orc):
    """An integration split by a snapshot (device to host) and a restore
    into other accumulators equals the uninterrupted one and the oracle of
    the two frames concatenated in time."""
    from paper_1503_06189_amd import xengine
    a = synth.random_bytes_frame(seed=61, N=96, F=3, T=700, B=64, p_loss=0.1)
    b = synth.random_bytes_frame(seed=62, N=96, F=3, T=900, B=64, p_loss=0.1)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    v1, c1 = xengine.new_accumulators(96, 3)
    xengine.accumulate(dev(a.packed), dev(a.mask), 64, v1, c1)
    snap = xengine.snapshot(v1, c1)
    assert snap["samples"] == 700
    v2, c2 = xengine.new_accumulators(96, 3)
    xengine.restore(snap, v2, c2)
    assert xengine.integrated_samples(v2) == 700
    xengine.accumulate(dev(b.packed), dev(b.mask), 64, v2, c2)
    xengine.accumulate(dev(b.packed), dev(b.mask), 64, v1, c1)
    torch.cuda.synchronize()
    assert np.array_equal(v1.cpu().numpy(), v2.cpu().numpy())
    assert np.array_equal(c1.cpu().numpy(), c2.cpu().numpy())
    ea, na = orc.correlate(a.packed, a.mask, 64)
    eb, nb = orc.correlate(b.packed, b.mask, 64)
    assert np.array_equal(v2.cpu().numpy().astype(np.int64), ea + eb)
    assert np.array_equal(c2.cpu().numpy(), na + nb)


def _serve_frames(server, frames, sid_seq):
    from paper_1503_06189_amd.serve import Frame
    for sid, q in sid_seq:
        fr = frames[sid][q]
        server.submit(Frame(sid, q, torch.from_numpy(fr.packed).cuda(),
                            torch.from_numpy(fr.mask).cuda(), 0.0))
        server.step()
    server.sync()


def test_checkpoint_resume_across_servers(srv, orc, tmp_path):
    """Two streams integrate 3 frames each.  A server takes the first two
    frames of every stream and writes a checkpoint; a fresh server opens the
    same streams, resumes from it and takes the last frames: its results
    equal an uninterrupted server's and the oracle's."""
    from paper_1503_06189_amd.serve import StreamConfig, StreamServer
    from paper_1503_06189_amd.synth import StreamSpec, stream_frame
    specs = [StreamSpec(3, 64, 2, 512, 3, 0.05, 1e9, 7101),
             StreamSpec(9, 128, 3, 512, 3, 0.05, 1e9, 7102)]
    frames = {s.stream_id: [stream_frame(s, q, 64) for q in range(3)] for s in specs}
    cfgs = [StreamConfig(s.stream_id, s.N, s.F, s.T, 64, 3) for s in specs]

    def server():
        sv = StreamServer(hbm_budget=1 << 30)
        for c in cfgs:
            sv.open(c)
        return sv

    whole = server()
    _serve_frames(whole, frames, [(s.stream_id, q) for q in range(3) for s in specs])
    first = server()
    _serve_frames(first, frames, [(s.stream_id, q) for q in range(2) for s in specs])
    assert not any(first.results.values())
    path = str(tmp_path / "ckpt.npz")
    first.checkpoint(path)
    second = server()
    second.resume(path)
    _serve_frames(second, frames, [(s.stream_id, 2) for s in specs])
    for s in specs:
        (rw,), (rr,) = whole.results[s.stream_id], second.results[s.stream_id]
        assert rr.frames == 3 and rr.index == rw.index == 0
        assert np.array_equal(rr.vis, rw.vis) and np.array_equal(rr.count, rw.count)
        assert np.array_equal(rr.out.view(np.uint32), rw.out.view(np.uint32))
        ev = en = None
        for fr in frames[s.stream_id]:
            v, n = orc.correlate(fr.packed, fr.mask, 64)
            ev = v if ev is None else ev + v
            en = n if en is None else en + n
        assert np.array_equal(rr.vis.astype(np.int64), ev) and np.array_equal(rr.count, en)


def test_stream_dying_mid_integration(srv, orc, specs, pool):
    """One of four streams dies after part of an integration: the server
    drops its frames and open sums, returns its pool slots and closes it;
    the other streams' results still equal the oracle."""
    from paper_1503_06189_amd.serve import Frame, StreamConfig, StreamServer
    server = StreamServer(hbm_budget=1 << 30, slice_samples=256)
    for s in specs:
        server.open(StreamConfig(s.stream_id, s.N, s.F, s.T, 256, s.frames_per_integration))
    victim = specs[1].stream_id
    seq = {s.stream_id: [k % 2 for k in range(s.frames_per_integration)] for s in specs}
    for k in range(max(len(v) for v in seq.values())):
        for s in specs:
            if k >= len(seq[s.stream_id]) or (s.stream_id == victim and k >= 1):
                continue
            fr = pool[s.stream_id][seq[s.stream_id][k]]
            server.submit(Frame(s.stream_id, k, torch.from_numpy(fr.packed).pin_memory(),
                                torch.from_numpy(fr.mask).pin_memory(), 0.0))
        server.step()
        if k == 1:
            server.abort(victim)
    server.sync()
    assert victim not in server.streams and not server.results.get(victim)
    assert len(server.pool.free) == server.pool.n
    for s in specs:
        if s.stream_id == victim:
            continue
        (r,) = server.results[s.stream_id]
        ev, en, eo = _expected(orc, s, pool, seq[s.stream_id], 0)
        assert np.array_equal(r.count, en) and np.array_equal(r.vis.astype(np.int64), ev)


def _submit(server, spec, fr, seq):
    from paper_1503_06189_amd.serve import Frame
    server.submit(Frame(spec.stream_id, seq, torch.from_numpy(fr.packed).pin_memory(),
                        torch.from_numpy(fr.mask).pin_memory(), 0.0))


def test_failing_result_callback_is_raised_not_waited_for(srv, orc, specs, pool):
    """A result callback that raises: sync() raises RuntimeError with the
    callback's error as its cause instead of waiting forever for the result
    to be delivered; the result is still kept, and the server goes on."""
    from paper_1503_06189_amd.serve import StreamConfig, StreamServer
    calls = []

    def on_result(res):
        calls.append(res.index)
        if len(calls) == 1:
            raise ValueError("the consumer failed")

    server = StreamServer(hbm_budget=1 << 30, on_result=on_result)
    s = specs[0]
    server.open(StreamConfig(s.stream_id, s.N, s.F, s.T, 256, 1))
    fr = pool[s.stream_id][0]
    _say(f"failing callback, stream {s.stream_id} N={s.N} F={s.F}")
    _submit(server, s, fr, 0)
    with pytest.raises(RuntimeError) as err:
        server.sync()
    assert isinstance(err.value.__cause__, ValueError)
    _submit(server, s, fr, 1)
    server.sync()
    assert calls == [0, 1]
    ev, en = orc.correlate(fr.packed, fr.mask, fr.B)
    assert [r.index for r in server.results[s.stream_id]] == [0, 1]
    for r in server.results[s.stream_id]:
        assert np.array_equal(r.count, en) and np.array_equal(r.vis.astype(np.int64), ev)


def test_abort_and_close_see_frames_not_yet_scheduled(srv, orc, specs, pool):
    """Frames submitted for a stream aborted before the scheduler took them
    are dropped with it and counted, and later passes do not trip over
    them; close() of a stream with such frames refuses.  The surviving
    stream's integration equals the oracle."""
    from paper_1503_06189_amd.serve import StreamConfig, StreamServer
    server = StreamServer(hbm_budget=1 << 30)
    a, b, c = specs[0], specs[1], specs[2]
    for s in (a, b, c):
        server.open(StreamConfig(s.stream_id, s.N, s.F, s.T, 256, 2))
    for k in range(2):
        for s in (a, b):
            _submit(server, s, pool[s.stream_id][k], k)
    _submit(server, c, pool[c.stream_id][0], 0)
    _say(f"abort {a.stream_id} with 2 unscheduled frames")
    assert server.abort(a.stream_id) == 2
    with pytest.raises(RuntimeError):
        server.close(c.stream_id)
    server.flush(c.stream_id)
    server.sync()
    assert a.stream_id not in server.streams and not server.results.get(a.stream_id)
    (r,) = server.results[b.stream_id]
    vis = cnt = 0
    for k in range(2):
        fr = pool[b.stream_id][k]
        v, n = orc.correlate(fr.packed, fr.mask, fr.B)
        vis, cnt = vis + v, cnt + n
    assert np.array_equal(r.count, cnt) and np.array_equal(r.vis.astype(np.int64), vis)
    (rc,) = server.results[c.stream_id]
    fr = pool[c.stream_id][0]
    v, n = orc.correlate(fr.packed, fr.mask, fr.B)
    assert rc.frames == 1 and np.array_equal(rc.vis.astype(np.int64), v)
    server.close(c.stream_id)
    assert len(server.pool.free) == server.pool.n
