"""Pins that tie the oracle to facts other than its own code.

Each ``pin_*`` takes an :class:`oracle.Oracle` and raises ``AssertionError``
when the oracle disagrees with what the mathematics or the method fixes:

* a library routine (numpy complex128 matrix product) and pure-Python
  complex arithmetic on small inputs built from *values*, never from the
  oracle's own decoding of bytes;
* closed forms (constant input, quarter-rate tone, all-(-8-8i) overflow
  edge, tone normalised after loss);
* invariants (Hermitian symmetry, real non-negative autocorrelations,
  linearity across frames, nibble swap = conjugation, i*x and -x leave V
  unchanged, input permutation permutes V, garbage in lost blocks changes
  nothing);
* exact rational arithmetic for the normalisation's rounding.

``tests/test_oracle_pins.py`` runs them on the oracle; the planted-mistake
test runs them on altered copies of it and requires each copy to fail one.
"""

from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np

from paper_1503_06189_amd import synth


# ---------------------------------------------------------------------------
# helpers that build frames from complex *values* (no decoding involved)
# ---------------------------------------------------------------------------

def _values(rng, shape, lo=-8, hi=7):
    re = rng.integers(lo, hi + 1, shape)
    im = rng.integers(lo, hi + 1, shape)
    return re, im


def _frame_from_values(re, im):
    return synth.encode(re, im)


def _expand_mask(mask, T, B):
    """[F][nblk] block flags -> [T][F] boolean validity, by repetition."""
    if mask is None:
        return None
    rep = np.repeat(mask != 0, B, axis=1)[:, :T]   # [F][T]
    return ~rep.T


def _numpy_vis(re, im, valid=None):
    """Upper-triangle V from values with numpy's complex matrix product."""
    T, F, N = re.shape
    x = re.astype(np.complex128) + 1j * im.astype(np.complex128)
    if valid is not None:
        x = x * valid[:, :, None]
    out = []
    iu, ju = np.triu_indices(N)
    for f in range(F):
        X = x[:, f, :]                       # [T][N]
        V = X.T @ X.conj()                   # V[i][j] = sum_t x_i conj(x_j)
        out.append(np.stack([V[iu, ju].real, V[iu, ju].imag], axis=-1))
    return np.rint(np.array(out)).astype(np.int64)


# ---------------------------------------------------------------------------
# pins
# ---------------------------------------------------------------------------

def pin_decode_roundtrip(orc):
    """Every (re, im) in [-8, 7]^2 survives the independent encoder, and the
    256 byte codes map one-to-one onto those 256 values."""
    seen = set()
    for re, im in itertools.product(range(-8, 8), repeat=2):
        b = int(_frame_from_values(np.array(re), np.array(im)))
        assert orc.decode(b) == (re, im), (re, im, b)
        seen.add(orc.decode(b))
    assert len({orc.decode(b) for b in range(256)}) == 256
    assert len(seen) == 256


def pin_tri_index(orc):
    """Row-major packed upper triangle incl. diagonal is a bijection onto
    0..P-1 and consecutive along each row."""
    for N in (1, 2, 3, 16, 256):
        P = N * (N + 1) // 2
        assert orc.num_pairs(N) == P
        idx = [orc.tri_index(N, i, j) for i in range(N) for j in range(i, N)]
        assert idx == list(range(P)), N


def pin_numpy_matmul(orc):
    """Random values incl. -8, random loss with garbage in lost blocks:
    oracle == numpy complex128 X^T conj(X) over the valid samples (exact,
    every partial sum is an integer far below 2^53)."""
    rng = np.random.default_rng(11)
    for (N, F, T, B, p) in [(1, 1, 1, 1, 0.0), (3, 2, 7, 2, 0.3), (8, 3, 64, 8, 0.25),
                            (5, 2, 33, 4, 0.5), (16, 1, 40, 256, 0.0)]:
        re, im = _values(rng, (T, F, N))
        packed = _frame_from_values(re, im)
        mask = (rng.random((F, (T + B - 1) // B)) < p).astype(np.uint8)
        valid = _expand_mask(mask, T, B)
        # garbage in lost blocks: the oracle must not read it
        noise = rng.integers(0, 256, packed.shape, dtype=np.uint8)
        packed = np.where(valid[:, :, None], packed, noise).astype(np.uint8)
        vis, cnt = orc.correlate(packed, mask, B)
        exp = _numpy_vis(re, im, valid)
        assert np.array_equal(vis, exp), (N, F, T, B)
        assert np.array_equal(cnt, valid.sum(axis=0)), (N, F, T, B)


def pin_python_brute_force(orc):
    """Pure-Python complex loops on a handful of samples."""
    rng = np.random.default_rng(12)
    T, F, N = 5, 2, 4
    re, im = _values(rng, (T, F, N))
    vis, _ = orc.correlate(_frame_from_values(re, im), None, 4)
    p = 0
    for i in range(N):
        for j in range(i, N):
            for f in range(F):
                s = 0j
                for t in range(T):
                    xi = complex(int(re[t, f, i]), int(im[t, f, i]))
                    xj = complex(int(re[t, f, j]), int(im[t, f, j]))
                    s += xi * xj.conjugate()
                assert vis[f, p, 0] == s.real and vis[f, p, 1] == s.imag, (f, i, j)
            p += 1


def pin_hermitian_autocorr(orc):
    """Full matrix: V_ji = conj(V_ij); Im V_ii = 0; Re V_ii = sum |x_i|^2;
    the packed triangle is the upper half of the full matrix."""
    rng = np.random.default_rng(13)
    T, F, N, B = 48, 2, 6, 16
    re, im = _values(rng, (T, F, N))
    mask = np.array([[0, 1, 0], [0, 0, 1]], dtype=np.uint8)
    packed = _frame_from_values(re, im)
    full = orc.correlate_full(packed, mask, B)
    vis, _ = orc.correlate(packed, mask, B)
    valid = _expand_mask(mask, T, B)
    assert np.array_equal(full[..., 0], full[..., 0].transpose(0, 2, 1))
    assert np.array_equal(full[..., 1], -full[..., 1].transpose(0, 2, 1))
    power = ((re.astype(np.int64) ** 2 + im.astype(np.int64) ** 2) * valid[:, :, None]).sum(0)
    for f in range(F):
        assert np.array_equal(np.diagonal(full[f, :, :, 0]), power[f])
        assert not np.diagonal(full[f, :, :, 1]).any()
        iu, ju = np.triu_indices(N)
        assert np.array_equal(full[f, iu, ju], vis[f])


def pin_constant_input(orc):
    """x_i(t) = c_i for every t: V_ij = n c_i conj(c_j), n = valid count."""
    rng = np.random.default_rng(14)
    T, F, N, B = 40, 3, 7, 8
    cr, ci = _values(rng, (F, N))
    re = np.broadcast_to(cr, (T, F, N))
    im = np.broadcast_to(ci, (T, F, N))
    mask = np.zeros((F, 5), dtype=np.uint8)
    mask[1, 2] = 1
    mask[2, :] = 1
    vis, cnt = orc.correlate(_frame_from_values(re, im), mask, B)
    assert list(cnt) == [40, 32, 0]
    p = 0
    for i in range(N):
        for j in range(i, N):
            for f in range(F):
                c_i = complex(int(cr[f, i]), int(ci[f, i]))
                c_j = complex(int(cr[f, j]), int(ci[f, j]))
                v = cnt[f] * c_i * c_j.conjugate()
                assert (vis[f, p, 0], vis[f, p, 1]) == (v.real, v.imag)
            p += 1


def _tone(rng, T, F, N):
    """x_i(t) = g_i * (1j)^t: multiplying by 1j swaps/negates the
    components, so values stay integers in [-7, 7]."""
    gr, gi = _values(rng, (F, N), -7, 7)
    g = gr + 1j * gi
    ph = (1j) ** np.arange(T)
    x = ph[:, None, None] * g[None]
    re = np.rint(x.real).astype(np.int64)
    im = np.rint(x.imag).astype(np.int64)
    return g, re, im


def pin_single_tone_and_normalize(orc):
    """Quarter-rate tone: V_ij = n g_i conj(g_j) (the phase cancels); after
    loss, V/n = g_i conj(g_j) exactly."""
    rng = np.random.default_rng(15)
    T, F, N, B = 64, 2, 5, 4
    g, re, im = _tone(rng, T, F, N)
    mask = (rng.random((F, T // B)) < 0.4).astype(np.uint8)
    vis, cnt = orc.correlate(_frame_from_values(re, im), mask, B)
    out = orc.normalize(vis, cnt)
    iu, ju = np.triu_indices(N)
    for f in range(F):
        G = np.outer(g[f], g[f].conj())[iu, ju]
        assert np.array_equal(vis[f, :, 0], cnt[f] * G.real.astype(np.int64))
        assert np.array_equal(vis[f, :, 1], cnt[f] * G.imag.astype(np.int64))
        assert np.array_equal(out[f, :, 0], G.real.astype(np.float32))
        assert np.array_equal(out[f, :, 1], G.imag.astype(np.float32))


def pin_linearity(orc):
    """accumulate(F1); accumulate(F2) == correlate(F1 then F2 in time);
    also a start from non-zero sums (resume from a snapshot)."""
    rng = np.random.default_rng(16)
    N, F, B = 6, 2, 8
    T1, T2 = 24, 40
    fr = synth.random_bytes_frame(17, N, F, T1 + T2, B, p_loss=0.3)
    m1, m2 = fr.mask[:, :T1 // B], fr.mask[:, T1 // B:]
    full_v, full_n = orc.correlate(fr.packed, fr.mask, B)
    v = np.zeros_like(full_v)
    n = np.zeros_like(full_n)
    orc.accumulate(fr.packed[:T1], m1, B, v, n)
    orc.accumulate(fr.packed[T1:], m2, B, v, n)
    assert np.array_equal(v, full_v) and np.array_equal(n, full_n)
    start_v = rng.integers(-1000, 1000, v.shape).astype(np.int64)
    start_n = rng.integers(0, 1000, n.shape).astype(np.int64)
    v2, n2 = start_v.copy(), start_n.copy()
    orc.accumulate(fr.packed, fr.mask, B, v2, n2)
    assert np.array_equal(v2, start_v + full_v) and np.array_equal(n2, start_n + full_n)


def pin_symmetries(orc):
    """Nibble swap (x -> i conj x) conjugates V for every byte; i*x and -x
    leave V unchanged; permuting inputs permutes V."""
    rng = np.random.default_rng(18)
    T, F, N, B = 32, 2, 6, 8
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    mask = (rng.random((F, T // B)) < 0.3).astype(np.uint8)
    v, _ = orc.correlate(packed, mask, B)
    swapped = ((packed >> 4) | (packed << 4)).astype(np.uint8)
    vs, _ = orc.correlate(swapped, mask, B)
    assert np.array_equal(vs[..., 0], v[..., 0]) and np.array_equal(vs[..., 1], -v[..., 1])

    re, im = _values(rng, (T, F, N), -7, 7)
    v0, _ = orc.correlate(_frame_from_values(re, im), mask, B)
    vi, _ = orc.correlate(_frame_from_values(-im, re), mask, B)      # i * x
    vn, _ = orc.correlate(_frame_from_values(-re, -im), mask, B)     # -x
    assert np.array_equal(vi, v0) and np.array_equal(vn, v0)

    perm = rng.permutation(N)
    full = orc.correlate_full(packed, mask, B)
    fullp = orc.correlate_full(packed[:, :, perm], mask, B)
    assert np.array_equal(fullp, full[:, perm][:, :, perm])


def pin_loss_and_counts(orc):
    """Lost blocks: garbage == zero fill; counts == samples outside lost
    blocks, including a partial last block; an all-lost channel gives 0."""
    for (N, F, T, B, p) in [(4, 3, 50, 8, 0.4), (3, 2, 17, 5, 0.5), (2, 4, 9, 256, 0.5)]:
        seed = 19 + T
        zero = synth.random_bytes_frame(seed, N, F, T, B, p_loss=p, fill="zero")
        junk = zero.packed.copy()
        synth.fill_lost(junk, zero.mask, B, "garbage", np.random.default_rng(seed))
        vz, nz = orc.correlate(zero.packed, zero.mask, B)
        vj, nj = orc.correlate(junk, zero.mask, B)
        assert np.array_equal(vz, vj) and np.array_equal(nz, nj)
        valid = _expand_mask(zero.mask, T, B)
        assert np.array_equal(nz, valid.sum(axis=0))
        assert np.array_equal(orc.valid_counts(zero.mask, F, T, B), nz)
    mask = np.ones((2, 3), dtype=np.uint8)
    mask[1, 1] = 0
    packed = np.full((20, 2, 3), 0x00, dtype=np.uint8)
    v, n = orc.correlate(packed, mask, 8)
    assert list(n) == [0, 8] and not v[0].any()
    assert (v[1, :, 0] == 128 * 8).all() and not v[1, :, 1].any()


def pin_overflow_edge(orc):
    """Every byte 0x00 (x = -8-8i): Re V = 128 n, Im V = 0, exactly, at the
    largest frame length whose sums still fit int32 (16,777,215)."""
    T = 16_777_215
    packed = np.zeros((T, 1, 2), dtype=np.uint8)
    vis, cnt = orc.correlate(packed, None, 256)
    assert cnt[0] == T
    assert (vis[0, :, 0] == 128 * T).all() and not vis[0, :, 1].any()
    assert 128 * T < 2 ** 31


def pin_pairs_subset(orc):
    """The sampled-pairs entry equals the full matrix for any (f, i, j),
    including i > j."""
    fr = synth.random_bytes_frame(23, 7, 3, 30, 4, p_loss=0.3)
    full = orc.correlate_full(fr.packed, fr.mask, 4)
    rng = np.random.default_rng(24)
    fs = rng.integers(0, 3, 50)
    is_ = rng.integers(0, 7, 50)
    js = rng.integers(0, 7, 50)
    got = orc.correlate_pairs(fr.packed, fr.mask, 4, fs, is_, js)
    assert np.array_equal(got, full[fs, is_, js])


def pin_normalize_rounding(orc):
    """V/n rounded to float32 lies within half an ulp (plus the double
    step's 2^-53) of the exact rational V/n; n = 0 gives exactly 0."""
    rng = np.random.default_rng(25)
    F, N = 4, 20
    P = N * (N + 1) // 2
    vis = rng.integers(-2 ** 31 + 1, 2 ** 31 - 1, (F, P, 2)).astype(np.int64)
    vis[1] = rng.integers(-2 ** 26, 2 ** 26, (P, 2))
    cnt = np.array([3, 16_777_213, 0, 7919], dtype=np.int64)
    out = orc.normalize(vis, cnt)
    assert not out[2].any()
    for f in (0, 1, 3):
        for p in range(P):
            for c in range(2):
                exact = Fraction(int(vis[f, p, c]), int(cnt[f]))
                got = Fraction(float(out[f, p, c]))
                m, e = np.frexp(np.float32(float(exact)))
                half_ulp = Fraction(2) ** (int(e) - 25)
                assert abs(got - exact) <= half_ulp * (1 + Fraction(1, 2 ** 28)), \
                    (f, p, c, float(exact), float(got))


# ---------------------------------------------------------------------------
# per-input flags (Sec. II-C)
# ---------------------------------------------------------------------------

def _flag_case(seed, N=37, F=3, T=70, B=8, p=0.25, p_loss=0.2):
    """Random values, a loss mask and dense random flags with garbage in the
    padding bits, one all-ones bit-field and one column of zero words."""
    rng = np.random.default_rng(seed)
    re, im = _values(rng, (T, F, N))
    packed = _frame_from_values(re, im)
    mask = synth.bernoulli_mask(rng, F, T, B, p_loss)
    flags = synth.random_flags(rng, T, F, N, p, garbage_padding=True)
    flags[1, 3, :] = 0xFFFFFFFF
    flags[:, 5, 0] = 0
    return re, im, packed, mask, flags, B


def pin_flag_counts_brute_force(orc):
    """Counters, intersections and the normalisation matrix against direct
    counting on unpacked bits: c_i = #valid samples with i flagged, d_ij =
    #valid samples with both flagged, n_ij = #valid samples with neither
    flagged (a 0/1 matrix product); counters add up across frames."""
    for seed, N, T in ((31, 37, 70), (32, 64, 64), (33, 5, 33)):
        re, im, packed, mask, flags, B = _flag_case(seed, N=N, T=T)
        F = packed.shape[1]
        valid = _expand_mask(mask, T, B)                       # [T][F]
        fl = synth.unpack_flags(flags, N) & valid[:, :, None]
        ok = valid[:, :, None] & ~synth.unpack_flags(flags, N)
        c, d = orc.flag_counters(flags, mask, N, B)
        cnt = orc.valid_counts(mask, F, T, B)
        n = orc.flag_norm(cnt, c, d)
        iu, ju = np.triu_indices(N)
        for f in range(F):
            A = fl[:, f, :].astype(np.int64)
            O = ok[:, f, :].astype(np.int64)
            D = A.T @ A
            G = O.T @ O
            assert (c[f] == A.sum(0)).all(), (seed, f)
            assert (d[f] == D[iu, ju]).all(), (seed, f)
            assert (n[f] == G[iu, ju]).all(), (seed, f)
        # two halves of a frame (split on a block edge) add up to the whole
        h = (T // 2) // B * B
        if 0 < h < T:
            c2, d2 = orc.flag_counters(flags[:, :h], mask[:, :h // B], N, B)
            orc.flag_counters(flags[:, h:], mask[:, h // B:], N, B, c2, d2)
            assert (c2 == c).all() and (d2 == d).all(), seed


def pin_flagged_correlation(orc):
    """Flagged points contribute nothing: V with flags equals numpy's
    complex product of the values with flagged and lost points set to 0,
    and equals the plain correlation of the frame whose flagged points
    were zeroed (0x88); zeroing touches flagged points only."""
    re, im, packed, mask, flags, B = _flag_case(34, N=37, T=70)
    T, F, N = packed.shape
    bits = synth.unpack_flags(flags, N)
    valid = _expand_mask(mask, T, B)
    vis, cnt = orc.correlate_flagged(packed, mask, flags, B)
    x = (re + 1j * im) * (valid[:, :, None] & ~bits)
    iu, ju = np.triu_indices(N)
    for f in range(F):
        X = x[:, f, :]
        V = X.T @ X.conj()
        assert (vis[f, :, 0] == np.rint(V[iu, ju].real)).all(), f
        assert (vis[f, :, 1] == np.rint(V[iu, ju].imag)).all(), f
    assert (cnt == orc.valid_counts(mask, F, T, B)).all()
    z = orc.apply_flags(packed, flags)
    assert (z[bits] == synth.ZERO_BYTE).all()
    assert (z[~bits] == packed[~bits]).all()
    vis2, cnt2 = orc.correlate(z, mask, B)
    assert (vis2 == vis).all() and (cnt2 == cnt).all()


def pin_flag_normalize(orc):
    """Input i held at a constant x_i: every baseline with n_ij > 0
    normalises to exactly x_i conj(x_j), an input flagged at every sample
    has n = 0 on its row and column and normalises to 0, and without flags
    n_ij is the channel's valid count.  Random V/n rounds to within half an
    ulp of the exact rational."""
    rng = np.random.default_rng(35)
    N, F, T, B = 40, 2, 96, 16
    xr = rng.integers(-7, 8, N)
    xi = rng.integers(-7, 8, N)
    packed = _frame_from_values(np.broadcast_to(xr, (T, F, N)),
                                np.broadcast_to(xi, (T, F, N)))
    mask = synth.bernoulli_mask(rng, F, T, B, 0.25)
    bits = rng.random((T, F, N)) < 0.3
    bits[:, 1, 7] = True
    flags = synth.pack_flags(bits)
    vis, cnt = orc.correlate_flagged(packed, mask, flags, B)
    c, d = orc.flag_counters(flags, mask, N, B)
    n = orc.flag_norm(cnt, c, d)
    out = orc.normalize_pairs(vis, n)
    iu, ju = np.triu_indices(N)
    want_re = xr[iu] * xr[ju] + xi[iu] * xi[ju]
    want_im = xi[iu] * xr[ju] - xr[iu] * xi[ju]
    for f in range(F):
        pos = n[f] > 0
        assert (out[f, pos, 0] == want_re[pos]).all(), f
        assert (out[f, pos, 1] == want_im[pos]).all(), f
        assert not out[f, ~pos].any(), f
        assert (n[f] < cnt[f]).any() and pos.any(), f
    row7 = (iu == 7) | (ju == 7)
    assert not n[1, row7].any()
    c0, d0 = orc.flag_counters(np.zeros_like(flags), mask, N, B)
    assert (orc.flag_norm(cnt, c0, d0) == cnt[:, None]).all()
    # rounding of V / n_ij for arbitrary values
    P = N * (N + 1) // 2
    rv = rng.integers(-2 ** 31 + 1, 2 ** 31 - 1, (F, P, 2)).astype(np.int64)
    rn = rng.integers(0, 2 ** 24, (F, P)).astype(np.int64)
    rn[0, :5] = 0
    ro = orc.normalize_pairs(rv, rn)
    for f in range(F):
        for p in range(0, P, 7):
            for k in range(2):
                if rn[f, p] == 0:
                    assert ro[f, p, k] == 0
                    continue
                exact = Fraction(int(rv[f, p, k]), int(rn[f, p]))
                got = Fraction(float(ro[f, p, k]))
                m, e = np.frexp(np.float32(float(exact)))
                half_ulp = Fraction(2) ** (int(e) - 25)
                assert abs(got - exact) <= half_ulp * (1 + Fraction(1, 2 ** 28)), (f, p, k)


# ---------------------------------------------------------------------------
# frame assembly from packets (Sec. II-A)
# ---------------------------------------------------------------------------

def _assembly_case(seed, N=37, n_streams=3, T=64, base=5, seq0=1000):
    rng = np.random.default_rng(seed)
    F = 8 * n_streams
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    flags = synth.random_flags(rng, T, F, N, 0.2, garbage_padding=True)
    pk = synth.packetize(packed, flags, stream_base=base, seq0=seq0)
    return rng, packed, flags, pk


def _brute_assemble(pk, N, n_streams, base, seq0, T):
    """Arrival order, first packet per (stream, slot), written with numpy
    slicing of each packet (no loop over bytes)."""
    F = 8 * n_streams
    W = (N + 31) // 32
    packed = np.full((T, F, N), synth.ZERO_BYTE, dtype=np.uint8)
    mask = np.ones((F, T // 4), dtype=np.uint8)
    flags = np.zeros((F, T, W), dtype=np.uint32)
    seen = set()
    stats = [0] * 6
    for p in pk:
        seq, sid, nin = synth.packet_header(p)
        if nin != N:
            stats[3] += 1
            continue
        s = sid - base
        if not 0 <= s < n_streams:
            stats[2] += 1
            continue
        k = seq - seq0
        if not 0 <= k < T // 4:
            stats[1] += 1
            continue
        stats[0] += 1
        if (s, k) in seen:
            continue
        seen.add((s, k))
        stats[4] += 1
        data = p[16:16 + 32 * N].reshape(4, 8, N)
        packed[4 * k:4 * k + 4, 8 * s:8 * s + 8, :] = data
        fw = p[16 + 32 * N:].view("<u4").reshape(4, 8, W)
        flags[8 * s:8 * s + 8, 4 * k:4 * k + 4, :] = fw.transpose(1, 0, 2)
        mask[8 * s:8 * s + 8, k] = 0
    stats[5] = int(mask[::8].sum())
    return packed, mask, flags, np.array(stats)


def pin_assemble_roundtrip(orc):
    """Packets cut from a frame, in order and shuffled, give the frame back:
    same bytes and flag words, nothing lost, every packet placed."""
    rng, packed, flags, pk = _assembly_case(60)
    for order in (np.arange(len(pk)), rng.permutation(len(pk))):
        got = orc.assemble(pk[order], 37, 3, 5, 1000, 64)
        assert np.array_equal(got[0], packed)
        assert np.array_equal(got[2], flags)
        assert not got[1].any()
        assert list(got[3]) == [len(pk), 0, 0, 0, len(pk), 0]


def pin_assemble_faults(orc):
    """Drops, duplicates with different payloads, reordering, packets from
    outside the window, of unknown streams and with a wrong input count:
    the first arrival of each (stream, slot) is placed, empty places read
    0 + 0i with no flags and a lost block, against a direct reconstruction."""
    for seed, N in ((61, 37), (62, 64)):
        rng, packed, flags, pk = _assembly_case(seed, N=N)
        pk = synth.network_faults(rng, pk, p_drop=0.15, p_dup=0.2, window=6, n_stray=3)
        bad = pk[:2].copy()
        h = bad[0, :16].view("<u8").copy()
        h[1] = np.uint64(99) | (np.uint64(N) << np.uint64(32))      # unknown stream
        bad[0, :16] = h.view(np.uint8)
        h = bad[1, :16].view("<u8").copy()
        h[1] = (h[1] & np.uint64(0xffffffff)) | (np.uint64(N + 1) << np.uint64(32))
        bad[1, :16] = h.view(np.uint8)                               # wrong input count
        early = pk[:1].copy()
        h = early[0, :16].view("<u8").copy()
        h[0] = np.uint64(999)                                        # before the window
        early[0, :16] = h.view(np.uint8)
        pk = np.concatenate([pk[:5], bad, early, pk[5:]])
        got = orc.assemble(pk, N, 3, 5, 1000, 64)
        want = _brute_assemble(pk, N, 3, 5, 1000, 64)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), seed
        st = got[3]
        assert st[1] >= 4 and st[2] >= 1 and st[3] >= 1 and st[5] > 0 and st[0] > st[4]


# ---------------------------------------------------------------------------
# per-input time shifting
# ---------------------------------------------------------------------------

def pin_time_shift(orc):
    """Zero delays copy the frame and its flags; each input's column equals
    numpy's shifted slice with 0x88 and a flag where the source lies
    outside; one common delay d leaves V over the frame equal to V of the
    first T - d samples of the original (same pairs, fewer samples)."""
    rng = np.random.default_rng(70)
    T, F, N = 40, 3, 37
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    flags = synth.random_flags(rng, T, F, N, 0.2, garbage_padding=True)
    bits = synth.unpack_flags(flags, N)
    out, fo = orc.time_shift(packed, flags, np.zeros(N, np.int32))
    assert np.array_equal(out, packed)
    assert np.array_equal(synth.unpack_flags(fo, N), bits)
    assert np.array_equal(fo, synth.pack_flags(bits))           # padding bits cleared
    d = rng.integers(-6, 7, N).astype(np.int32)
    d[0], d[1] = T + 3, -T
    out, fo = orc.time_shift(packed, flags, d)
    ob = synth.unpack_flags(fo, N)
    for i in range(N):
        for t in range(T):
            src = t - d[i]
            if 0 <= src < T:
                assert (out[t, :, i] == packed[src, :, i]).all()
                assert (ob[t, :, i] == bits[src, :, i]).all()
            else:
                assert (out[t, :, i] == synth.ZERO_BYTE).all() and ob[t, :, i].all()
    out, fo = orc.time_shift(packed, None, np.full(N, 5, np.int32))
    vs, _ = orc.correlate(out)
    vo, _ = orc.correlate(packed[:T - 5])
    assert np.array_equal(vs, vo)
    assert synth.unpack_flags(fo, N)[:5].all() and not synth.unpack_flags(fo, N)[5:].any()


def pin_time_shift_aligns_delayed_copy(orc):
    """What the shift is for: input 1 carries input 0's signal D samples
    later, and shifting input 1 by -D lines the two up.  Then the (0, 1)
    visibility over the frame is input 0's autocorrelation over the
    samples both still hold (the first T - D), real, with zero imaginary
    part; unshifted it is not.  Input 1's last D samples are flagged."""
    rng = np.random.default_rng(71)
    T, F, N, D = 64, 2, 4, 9
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    packed[D:, :, 1] = packed[:T - D, :, 0]
    d = np.zeros(N, np.int32)
    d[1] = -D
    out, fo = orc.time_shift(packed, None, d)
    vs, _ = orc.correlate(out)
    auto, _ = orc.correlate(packed[:T - D])
    assert np.array_equal(vs[:, 1], auto[:, 0])     # pair (0, 1) vs pair (0, 0)
    assert (vs[:, 1, 1] == 0).all() and (vs[:, 1, 0] > 0).all()
    vu, _ = orc.correlate(packed)
    assert not np.array_equal(vu[:, 1], auto[:, 0])
    fb = synth.unpack_flags(fo, N)
    assert fb[T - D:, :, 1].all() and not fb[:T - D, :, 1].any() and not fb[:, :, 0].any()


PINS = [
    pin_decode_roundtrip,
    pin_tri_index,
    pin_numpy_matmul,
    pin_python_brute_force,
    pin_hermitian_autocorr,
    pin_constant_input,
    pin_single_tone_and_normalize,
    pin_linearity,
    pin_symmetries,
    pin_loss_and_counts,
    pin_overflow_edge,
    pin_pairs_subset,
    pin_normalize_rounding,
    pin_flag_counts_brute_force,
    pin_flagged_correlation,
    pin_flag_normalize,
    pin_assemble_roundtrip,
    pin_assemble_faults,
    pin_time_shift,
    pin_time_shift_aligns_delayed_copy,
]
