"""Frame assembly from F-engine packets on the GPU against the oracle
(Sec. II-A): frame bytes, loss mask, flag words and counters bit for bit.

The packet streams come from synth.packetize and synth.network_faults:
drops, duplicates with different payloads (the first arrival must win),
reordering, packets outside the frame's window, of unknown streams and
with another input count.  Output buffers start as garbage: every element
must be written.  Shapes cover the byte path (odd N) and the 16-byte path,
and the full pathfinder frame (8 streams x 8 bands, 16384 samples).
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


def _garbage_outputs(T, F, N):
    W = (N + 31) // 32
    return (torch.full((T, F, N), 0x5A, dtype=torch.uint8, device="cuda"),
            torch.full((F, T // 4), 7, dtype=torch.uint8, device="cuda"),
            torch.full((F, T, W), -559038737, dtype=torch.int32, device="cuda"),
            torch.full((6,), -1, dtype=torch.int64, device="cuda"))


def _run(xe, pk, N, S, base, seq0, T):
    packed, mask, flags, stats = _garbage_outputs(T, 8 * S, N)
    dpk = torch.from_numpy(np.ascontiguousarray(pk)).cuda()
    xe.assemble_frame(dpk, N, S, base, seq0, T, packed, mask, flags, stats)
    torch.cuda.synchronize()
    return (packed.cpu().numpy(), mask.cpu().numpy(),
            flags.cpu().numpy().view(np.uint32), stats.cpu().numpy())


def _compare(got, want):
    names = ("packed", "mask", "flags", "stats")
    for n, g, w in zip(names, got, want):
        assert np.array_equal(g, w), (n, np.argwhere(g != w)[:5] if g.shape == w.shape else "")


def _frame(seed, N, S, T):
    rng = np.random.default_rng(seed)
    F = 8 * S
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    flags = synth.random_flags(rng, T, F, N, 0.1, garbage_padding=True)
    return rng, packed, flags


@pytest.mark.parametrize("N", [37, 64, 256])
def test_assemble_in_order_and_shuffled(xe, orc, N):
    S, T, base, seq0 = 3, 128, 11, 5000
    rng, packed, flags = _frame(70 + N, N, S, T)
    pk = synth.packetize(packed, flags, stream_base=base, seq0=seq0)
    for tag, order in (("in order", np.arange(len(pk))), ("shuffled", rng.permutation(len(pk)))):
        _say(f"assemble N={N} {tag}")
        got = _run(xe, pk[order], N, S, base, seq0, T)
        _compare(got, orc.assemble(pk[order], N, S, base, seq0, T))
        assert np.array_equal(got[0], packed) and not got[1].any()


@pytest.mark.parametrize("N,seed", [(37, 80), (64, 81), (256, 82), (256, 83)])
def test_assemble_network_faults(xe, orc, N, seed):
    S, T, base, seq0 = 4, 256, 3, 1 << 33
    rng, packed, flags = _frame(seed, N, S, T)
    pk = synth.packetize(packed, flags, stream_base=base, seq0=seq0)
    pk = synth.network_faults(rng, pk, p_drop=0.1, p_dup=0.1, window=16, n_stray=5,
                              stray_seq=seq0 + T // 4)
    bad = pk[:3].copy()
    for j, (sid, nin) in enumerate(((base + S, N), (base - 1, N), (base, N + 1))):
        h = bad[j, :16].view("<u8").copy()
        h[1] = np.uint64(sid & 0xffffffff) | (np.uint64(nin) << np.uint64(32))
        bad[j, :16] = h.view(np.uint8)
    pk = np.concatenate([bad[:1], pk, bad[1:]])
    _say(f"assemble faults N={N} seed={seed} packets={len(pk)}")
    got = _run(xe, pk, N, S, base, seq0, T)
    want = orc.assemble(pk, N, S, base, seq0, T)
    _compare(got, want)
    st = want[3]
    assert st[0] > st[4] and st[1] >= 5 and st[2] == 2 and st[3] == 1 and st[5] > 0


def test_assemble_empty_batch(xe, orc):
    N, S, T = 64, 2, 32
    pk = np.zeros((0, synth.packet_bytes(N)), dtype=np.uint8)
    _say("assemble empty batch")
    packed, mask, flags, stats = _garbage_outputs(T, 8 * S, N)
    xe.assemble_frame(torch.zeros((0, synth.packet_bytes(N)), dtype=torch.uint8,
                                  device="cuda"), N, S, 0, 0, T, packed, mask, flags, stats)
    torch.cuda.synchronize()
    got = (packed.cpu().numpy(), mask.cpu().numpy(), flags.cpu().numpy().view(np.uint32),
           stats.cpu().numpy())
    _compare(got, orc.assemble(pk, N, S, 0, 0, T))
    assert got[1].all() and (got[0] == 0x88).all()


def test_assemble_pathfinder_full_size(xe, orc):
    """The pathfinder share from 8 links (8 bands each) with 1% drops,
    0.5% duplicates and reordering, then correlated: the assembled frame,
    mask and flags equal the oracle's, and so do sampled baselines of the
    correlation of the assembled frame (mask with B = 4)."""
    fr = synth.pathfinder(p_loss=0.0)
    rng = np.random.default_rng(90)
    flags = synth.fengine_flags(rng, fr.T, fr.F, fr.N, 1e-3)
    pk = synth.packetize(fr.packed, flags, stream_base=0, seq0=7)
    pk = synth.network_faults(rng, pk, p_drop=0.01, p_dup=0.005, window=64, n_stray=2)
    _say(f"assemble pathfinder packets={len(pk)}")
    S = fr.F // 8
    got = _run(xe, pk, fr.N, S, 0, 7, fr.T)
    want = orc.assemble(pk, fr.N, S, 0, 7, fr.T)
    _compare(got, want)
    # correlate the assembled frame on the GPU, check sampled baselines
    packed = torch.from_numpy(got[0]).cuda()
    mask = torch.from_numpy(got[1]).cuda()
    vis, cnt = xe.correlate_frame(packed, mask, 4)
    torch.cuda.synchronize()
    fs = rng.integers(0, fr.F, 64)
    is_ = rng.integers(0, fr.N, 64)
    js = rng.integers(0, fr.N, 64)
    lo, hi = np.minimum(is_, js), np.maximum(is_, js)
    ev = orc.correlate_pairs(want[0], want[1], 4, fs, lo, hi)
    idx = lo * fr.N - lo * (lo - 1) // 2 + (hi - lo)
    v = vis.cpu().numpy()
    assert np.array_equal(v[fs, idx].astype(np.int64), ev)
    assert np.array_equal(cnt.cpu().numpy(), orc.valid_counts(want[1], fr.F, fr.T, 4))


def _set_seq(pk, j, seq):
    h = pk[j, :16].view("<u8").copy()
    h[0] = np.uint64(seq)
    pk[j, :16] = h.view(np.uint8)


@pytest.mark.parametrize("N", [4095, 4096])
def test_assemble_widest_packets(xe, orc, N):
    """The widest input count (packets of 147 KB, 128 flag words per row),
    on the byte path (N odd) and the 16-byte path, with drops and
    duplicates."""
    S, T, base, seq0 = 1, 32, 2, 40
    rng, packed, flags = _frame(200 + N, N, S, T)
    pk = synth.packetize(packed, flags, stream_base=base, seq0=seq0)
    pk = synth.network_faults(rng, pk, p_drop=0.25, p_dup=0.5, window=4, n_stray=1,
                              stray_seq=seq0 + T // 4)
    _say(f"assemble widest N={N} packets={len(pk)}")
    _compare(_run(xe, pk, N, S, base, seq0, T), orc.assemble(pk, N, S, base, seq0, T))


def test_assemble_sequence_limits(xe, orc):
    """A window that starts just below 2^63, with packets one before it and
    at the largest uint64 sequence number (both outside, counted as such)."""
    N, S, T, base = 48, 2, 64, 0
    seq0 = (1 << 63) - 100
    rng, packed, flags = _frame(210, N, S, T)
    pk = synth.packetize(packed, flags, stream_base=base, seq0=seq0)
    pk = synth.network_faults(rng, pk, p_drop=0.1, p_dup=0.1, window=8)
    extra = pk[:2].copy()
    _set_seq(extra, 0, seq0 - 1)
    _set_seq(extra, 1, (1 << 64) - 1)
    pk = np.concatenate([extra[:1], pk, extra[1:]])
    _say(f"assemble sequence limits packets={len(pk)}")
    got = _run(xe, pk, N, S, base, seq0, T)
    want = orc.assemble(pk, N, S, base, seq0, T)
    _compare(got, want)
    assert want[3][1] == 2


def test_assemble_without_flags(xe, orc):
    """Flags are optional: frame, mask and counters as with them."""
    N, S, T, base, seq0 = 64, 2, 64, 5, 9
    rng, packed, flags = _frame(220, N, S, T)
    pk = synth.packetize(packed, flags, stream_base=base, seq0=seq0)
    pk = synth.network_faults(rng, pk, p_drop=0.2, p_dup=0.2, window=8)
    _say("assemble without flags")
    p, m, _, st = _garbage_outputs(T, 8 * S, N)
    xe.assemble_frame(torch.from_numpy(pk).cuda(), N, S, base, seq0, T, p, m, None, st,
                      with_flags=False)
    torch.cuda.synchronize()
    want = orc.assemble(pk, N, S, base, seq0, T)
    _compare((p.cpu().numpy(), m.cpu().numpy(), want[2], st.cpu().numpy()), want)
