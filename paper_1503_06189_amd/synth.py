"""Seeded synthetic inputs for the X-engine correlator.

This module only *makes* inputs: complex voltages drawn from numpy's PCG64,
quantised to the 4+4-bit offset encoding, laid out as the frames the
correlator consumes, plus packet-loss masks.  It holds none of the
correlation arithmetic and imports nothing else from this package, so the
oracle (test infrastructure) and the HIP path can both consume its bytes
without sharing any code of the method.

Data layout (Sec. II-A, the packet carries all inputs of each band for a few
time samples and is used by the GPU unmodified):

* ``packed``  ``uint8[T][F][N]`` -- time-major, then channel, then input.
  One byte per complex sample: high nibble = real part, low nibble =
  imaginary part, each offset-encoded ``0..15`` meaning ``-8..7``.
* ``mask``    ``uint8[F][ceil(T/B)]`` -- one flag per channel and packet block
  of ``B`` samples, non-zero = the block was lost.  The last block may be
  partial.  Lost samples are written as ``0x88`` (value zero, the paper's
  zero fill, Sec. II-A.2) unless a test asks for garbage bytes there.
* ``flags``   ``uint32[F][T][ceil(N/32)]`` -- per-input F-engine flags as
  bit-fields, channel-major, bit ``i % 32`` of word ``i // 32`` set when
  input ``i`` is flagged at that channel and sample (Sec. II-C).

Workload recipes (sizes from Sec. I, Sec. II-A, Sec. III and Table I: N=256
inputs, 64 channels per server, 32-256 MB frames, N=16 and N=2048 scaling
points) are the functions ``tiny``, ``pathfinder``, ``large_n``,
``batched`` and ``streaming_streams`` below.  No public dataset exists for
this method; these synthetic frames stand in for live F-engine data.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

#: byte that encodes the complex value 0 + 0i (both nibbles = 8)
ZERO_BYTE = 0x88

#: per-recipe default seeds
SEEDS = {"tiny": 101, "pathfinder": 102, "large_n": 103, "batched": 104,
         "streaming": 105}

#: time samples drawn per noise chunk; part of the recipe (fixes draw order)
CHUNK = 1024


@dataclasses.dataclass
class Frame:
    """One frame of packed samples plus its loss mask."""

    packed: np.ndarray          # uint8 [T][F][N]
    mask: Optional[np.ndarray]  # uint8 [F][nblk] or None (= nothing lost)
    N: int
    F: int
    T: int
    B: int
    name: str = ""
    seed: int = 0

    @property
    def nblk(self) -> int:
        return (self.T + self.B - 1) // self.B

    @property
    def nbytes(self) -> int:
        return self.T * self.F * self.N


def encode(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Integers in [-8, 7] -> offset-encoded bytes (hi nibble re, lo nibble im)."""
    re = np.asarray(re, dtype=np.int16)
    im = np.asarray(im, dtype=np.int16)
    if re.size and (re.min() < -8 or re.max() > 7 or im.min() < -8 or im.max() > 7):
        raise ValueError("components must lie in [-8, 7]")
    return (((re + 8) << 4) | (im + 8)).astype(np.uint8)


def quantize(z_re: np.ndarray, z_im: np.ndarray, clip: int = 7) -> np.ndarray:
    """Round half-to-even, clip each component to [-clip, clip], encode."""
    re = np.clip(np.rint(z_re), -clip, clip).astype(np.int16)
    im = np.clip(np.rint(z_im), -clip, clip).astype(np.int16)
    return encode(re, im)


def nblocks(T: int, B: int) -> int:
    return (T + B - 1) // B


def bernoulli_mask(rng: np.random.Generator, F: int, T: int, B: int,
                   p: float) -> np.ndarray:
    """Independent loss per (channel, block) with probability p."""
    return (rng.random((F, nblocks(T, B))) < p).astype(np.uint8)


def gilbert_elliott_mask(rng: np.random.Generator, F: int, nblk: int,
                         rate: float, mean_burst: float = 4.0,
                         cap: float = 0.10) -> np.ndarray:
    """Bursty loss: two-state Markov chain per channel over blocks.

    The bad state lasts ``mean_burst`` blocks on average and the long-run
    fraction of lost blocks is ``rate``; each channel's loss in this frame
    is capped at ``cap`` of its blocks (extra lost blocks are un-flagged
    from the end).
    """
    mask = np.zeros((F, nblk), dtype=np.uint8)
    if rate <= 0:
        return mask
    p_bg = 1.0 / mean_burst                      # bad -> good
    p_gb = rate * p_bg / max(1e-12, 1.0 - rate)  # good -> bad
    state = rng.random(F) < rate
    for b in range(nblk):
        mask[:, b] = state
        u = rng.random(F)
        state = np.where(state, u >= p_bg, u < p_gb)
    limit = int(math.floor(cap * nblk))
    for f in range(F):
        lost = np.flatnonzero(mask[f])
        if lost.size > limit:
            mask[f, lost[limit:]] = 0
    return mask


def fill_lost(packed: np.ndarray, mask: Optional[np.ndarray], B: int,
              fill: str = "zero", rng: Optional[np.random.Generator] = None) -> None:
    """Overwrite the samples of lost blocks in place.

    ``fill='zero'`` writes 0x88 (the zero value, as the network thread of
    Sec. II-A.2 does); ``fill='garbage'`` writes random bytes, which a
    correct correlator must ignore because it applies the mask itself.
    """
    if mask is None:
        return
    T, F, N = packed.shape
    if fill == "garbage" and rng is None:
        rng = np.random.default_rng(0)
    for f, b in zip(*np.nonzero(mask)):
        t0, t1 = int(b) * B, min(T, (int(b) + 1) * B)
        if fill == "zero":
            packed[t0:t1, f, :] = ZERO_BYTE
        elif fill == "garbage":
            packed[t0:t1, f, :] = rng.integers(0, 256, (t1 - t0, N), dtype=np.uint8)
        else:
            raise ValueError(fill)


# ---------------------------------------------------------------------------
# per-input flags (F-engine range / sampling faults, Sec. II-C)
# ---------------------------------------------------------------------------

def flag_words(N: int) -> int:
    """32-bit words per (sample, channel) bit-field."""
    return (N + 31) // 32


def pack_flags(bits: np.ndarray) -> np.ndarray:
    """bool [T][F][N] (frame order) -> uint32 [F][T][ceil(N/32)] bit-fields;
    bit i%32 of word i/32."""
    bits = np.asarray(bits, dtype=bool).transpose(1, 0, 2)
    F, T, N = bits.shape
    W = flag_words(N)
    padded = np.zeros((F, T, W * 32), dtype=np.uint8)
    padded[:, :, :N] = bits
    by = np.packbits(padded.reshape(F, T, W, 4, 8), axis=-1, bitorder="little")
    return np.ascontiguousarray(by.reshape(F, T, W, 4)).view("<u4").reshape(F, T, W)


def unpack_flags(words: np.ndarray, N: int) -> np.ndarray:
    """uint32 [F][T][W] bit-fields -> bool [T][F][N] in frame order
    (padding bits dropped)."""
    words = np.ascontiguousarray(words, dtype="<u4")
    F, T, W = words.shape
    by = words.view(np.uint8).reshape(F, T, W * 4)
    bits = np.unpackbits(by, axis=-1, bitorder="little")
    return bits[:, :, :N].astype(bool).transpose(1, 0, 2)


def fengine_flags(rng: np.random.Generator, T: int, F: int, N: int,
                  rate: float, mean_run: float = 32.0,
                  garbage_padding: bool = False) -> np.ndarray:
    """Bursty per-input flags as uint32 bit-fields [F][T][ceil(N/32)].

    Each (channel, input) sees flag runs (a saturating ADC, a range fault)
    that start as a Poisson process in time with ``rate / mean_run`` starts
    per sample and last a geometric number of samples of mean
    ``mean_run``, so about ``rate`` of all points are flagged.  With
    ``garbage_padding`` the bits past input N-1 of the last word are
    random, which a consumer must ignore.  Draw order: run counts, starts,
    lengths, padding.
    """
    bits = np.zeros((T, F, N), dtype=bool)
    if rate > 0 and T > 0:
        lam = rate * T / mean_run
        runs = rng.poisson(lam, (F, N))
        total = int(runs.sum())
        fi = np.repeat(np.arange(F * N), runs.ravel())
        start = rng.integers(0, T, total)
        length = rng.geometric(1.0 / mean_run, total)
        for k in range(total):
            f, i = divmod(int(fi[k]), N)
            bits[start[k]:start[k] + length[k], f, i] = True
    words = pack_flags(bits)
    if garbage_padding and N % 32:
        pad = ~np.uint32((1 << (N % 32)) - 1)
        junk = rng.integers(0, 2 ** 32, (F, T), dtype=np.uint32) & pad
        words[:, :, -1] |= junk
    return words


def random_flags(rng: np.random.Generator, T: int, F: int, N: int,
                 p: float, garbage_padding: bool = True) -> np.ndarray:
    """Independent flags with probability p per point (dense stress case)."""
    words = pack_flags(rng.random((T, F, N)) < p)
    if garbage_padding and N % 32:
        pad = ~np.uint32((1 << (N % 32)) - 1)
        words[:, :, -1] |= rng.integers(0, 2 ** 32, (F, T), dtype=np.uint32) & pad
    return words


# ---------------------------------------------------------------------------
# UDP packets of the F-engine (Sec. II-A)
# ---------------------------------------------------------------------------

#: time samples and frequency bands per packet (Sec. II-A)
PKT_SAMPLES = 4
PKT_BANDS = 8
#: header: uint64 sequence number, uint32 stream id, uint32 input count
PKT_HEADER = 16


def packet_bytes(N: int) -> int:
    """Header + data [4][8][N] bytes + footer flags [4][8][ceil(N/32)] uint32."""
    return PKT_HEADER + PKT_SAMPLES * PKT_BANDS * N + PKT_SAMPLES * PKT_BANDS * flag_words(N) * 4


def packetize(packed: np.ndarray, flags: Optional[np.ndarray] = None,
              stream_base: int = 0, seq0: int = 0) -> np.ndarray:
    """Cut a frame into packets, uint8 [n_packets][packet_bytes], in time
    order with the streams of one time slot next to each other.

    Stream s carries channels 8 s .. 8 s + 7; packet k of stream s holds
    samples 4 k .. 4 k + 3 of those channels with sequence number seq0 + k.
    ``flags`` (uint32 [F][T][W], optional) fills the footers.
    """
    T, F, N = packed.shape
    if T % PKT_SAMPLES or F % PKT_BANDS:
        raise ValueError("T must be a multiple of 4 and F of 8")
    W = flag_words(N)
    S, n_slot = F // PKT_BANDS, T // PKT_SAMPLES
    pb = packet_bytes(N)
    out = np.zeros((n_slot * S, pb), dtype=np.uint8)
    data = packed.reshape(n_slot, PKT_SAMPLES, S, PKT_BANDS, N).transpose(0, 2, 1, 3, 4)
    out[:, PKT_HEADER:PKT_HEADER + PKT_SAMPLES * PKT_BANDS * N] = \
        data.reshape(n_slot * S, -1)
    if flags is not None:
        fw = np.ascontiguousarray(flags, dtype="<u4").reshape(S, PKT_BANDS, n_slot,
                                                              PKT_SAMPLES, W)
        fw = fw.transpose(2, 0, 3, 1, 4).reshape(n_slot * S, -1)   # [k][s][4][8][W]
        out[:, PKT_HEADER + PKT_SAMPLES * PKT_BANDS * N:] = fw.view(np.uint8)
    hdr = np.zeros((n_slot * S, 2), dtype="<u8")
    k = np.repeat(np.arange(n_slot, dtype=np.uint64), S)
    sid = np.tile(np.arange(S, dtype=np.uint64), n_slot) + np.uint64(stream_base)
    hdr[:, 0] = np.uint64(seq0) + k
    hdr[:, 1] = sid | (np.uint64(N) << np.uint64(32))
    out[:, :PKT_HEADER] = hdr.view(np.uint8).reshape(-1, PKT_HEADER)
    return out


def packet_header(pkt: np.ndarray):
    """(seq, stream_id, n_inputs) of one packet."""
    h = np.frombuffer(pkt[:PKT_HEADER].tobytes(), dtype="<u8")
    return int(h[0]), int(h[1] & 0xffffffff), int(h[1] >> np.uint64(32))


def network_faults(rng: np.random.Generator, packets: np.ndarray, p_drop: float = 0.01,
                   p_dup: float = 0.005, window: int = 64, n_stray: int = 0,
                   stray_seq: int = 1 << 40) -> np.ndarray:
    """What UDP does to a packet stream: drop each packet with p_drop,
    duplicate each with p_dup (the copy arrives up to ``window`` packets
    later, before or after the jittered original, and carries a different
    payload so that the rule "the first arrival wins" is visible), reorder by
    jittering arrival positions within ``window``, and append ``n_stray``
    packets from outside the frame (sequence numbers near ``stray_seq``).
    Draw order: drops, duplicates, duplicate payload, jitter, strays."""
    n = packets.shape[0]
    keep = rng.random(n) >= p_drop
    dup = (rng.random(n) < p_dup) & keep
    rows = list(np.flatnonzero(keep))
    pos = [float(i) for i in rows]
    extra = []
    for i in np.flatnonzero(dup):
        copy = packets[i].copy()
        copy[PKT_HEADER:] = rng.integers(0, 256, copy.size - PKT_HEADER, dtype=np.uint8)
        extra.append(copy)
        pos.append(float(i) + 1 + rng.uniform(0, window))
    jitter = rng.uniform(0, window, len(rows))
    for j in range(len(rows)):
        pos[j] += jitter[j]
    allp = [packets[i] for i in rows] + extra
    for k in range(n_stray):
        st = packets[k % max(n, 1)].copy() if n else np.zeros(packets.shape[1], np.uint8)
        h = np.frombuffer(st[:PKT_HEADER].tobytes(), dtype="<u8").copy()
        h[0] = np.uint64(stray_seq + k)
        st[:PKT_HEADER] = h.view(np.uint8)
        allp.append(st)
        pos.append(rng.uniform(0, n))
    order = np.argsort(np.array(pos), kind="stable")
    out = np.stack([allp[i] for i in order]) if allp else packets[:0].copy()
    return out


# ---------------------------------------------------------------------------
# generic helpers for tests
# ---------------------------------------------------------------------------

def random_bytes_frame(seed: int, N: int, F: int, T: int, B: int = 256,
                       p_loss: float = 0.0, fill: str = "garbage") -> Frame:
    """Uniform random bytes (all 256 codes, including -8 components)."""
    rng = np.random.default_rng(seed)
    packed = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    mask = bernoulli_mask(rng, F, T, B, p_loss) if p_loss > 0 else None
    fill_lost(packed, mask, B, fill, rng)
    return Frame(packed, mask, N, F, T, B, "random_bytes", seed)


def gaussian_frame(seed: int, N: int, F: int, T: int, B: int = 256,
                   sigma: float = 2.5, p_loss: float = 0.0,
                   fill: str = "zero") -> Frame:
    """Gaussian noise per component, rounded and clipped to [-7, 7]."""
    rng = np.random.default_rng(seed)
    mask = bernoulli_mask(rng, F, T, B, p_loss) if p_loss > 0 else None
    packed = np.empty((T, F, N), dtype=np.uint8)
    for t0 in range(0, T, CHUNK):
        t1 = min(T, t0 + CHUNK)
        re = rng.standard_normal((t1 - t0, F, N), dtype=np.float32) * sigma
        im = rng.standard_normal((t1 - t0, F, N), dtype=np.float32) * sigma
        packed[t0:t1] = quantize(re, im)
    fill_lost(packed, mask, B, fill, rng)
    return Frame(packed, mask, N, F, T, B, "gaussian", seed)


# ---------------------------------------------------------------------------
# the workload recipes
# ---------------------------------------------------------------------------

def tiny(seed: int = SEEDS["tiny"]) -> Frame:
    """N=16 inputs, 8 channels, 256 samples, sigma=2.5 noise, no loss."""
    fr = gaussian_frame(seed, N=16, F=8, T=256, B=256, sigma=2.5)
    fr.mask = np.zeros((8, 1), dtype=np.uint8)
    fr.name = "tiny_n16_f8_t256"
    return fr


def pathfinder(seed: int = SEEDS["pathfinder"], N: int = 256, F: int = 64,
               T: int = 16384, B: int = 256, p_loss: float = 0.01,
               tone_amp: float = 2.0, sigma: float = 2.5,
               fill: str = "zero") -> Frame:
    """One server's share of the pathfinder: N=256, 64 channels, 16384 samples.

    Noise sigma=2.5 per component plus one sky tone per channel,
    ``s_f(t) = A exp(i(2 pi nu_f t + phi_f))``, seen by input i through a
    complex gain ``g_i = r_i exp(i theta_i)`` with r ~ U(0.5, 1.5),
    theta ~ U(0, 2 pi) shared by all channels.  1% of the 256-sample blocks
    of each channel are lost.  Draw order: gains, tone parameters, mask,
    then noise chunk by chunk (real, then imaginary).
    """
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.5, 1.5, N)
    theta = rng.uniform(0.0, 2 * np.pi, N)
    gain = (r * np.exp(1j * theta)).astype(np.complex64)          # [N]
    nu = rng.uniform(-0.5, 0.5, F)
    phi = rng.uniform(0.0, 2 * np.pi, F)
    mask = bernoulli_mask(rng, F, T, B, p_loss)
    packed = np.empty((T, F, N), dtype=np.uint8)
    for t0 in range(0, T, CHUNK):
        t1 = min(T, t0 + CHUNK)
        t = np.arange(t0, t1, dtype=np.float64)[:, None]
        tone = (tone_amp * np.exp(1j * (2 * np.pi * nu[None, :] * t + phi[None, :])))
        sky = tone.astype(np.complex64)[:, :, None] * gain[None, None, :]
        re = rng.standard_normal((t1 - t0, F, N), dtype=np.float32) * sigma + sky.real
        im = rng.standard_normal((t1 - t0, F, N), dtype=np.float32) * sigma + sky.imag
        packed[t0:t1] = quantize(re, im)
    fill_lost(packed, mask, B, fill, np.random.default_rng(seed + 7919))
    return Frame(packed, mask, N, F, T, B, f"pathfinder_n{N}_f{F}_t{T}", seed)


def large_n(seed: int = SEEDS["large_n"], N: int = 2048, F: int = 16,
            T: int = 8192, B: int = 256, p_loss: float = 0.005,
            n_src: int = 4, sigma: float = 2.5) -> Frame:
    """Large-N scaling point: N=2048, 16 channels, 8192 samples.

    Noise sigma=2.5 plus ``n_src`` point sources; source k emits
    ``s_k(f, t) ~ CN(0, 1)`` and reaches input i with phase
    ``exp(i phi_{k,i})``, phi ~ U(0, 2 pi).  0.5% of 256-sample blocks lost.
    """
    rng = np.random.default_rng(seed)
    phase = np.exp(1j * rng.uniform(0.0, 2 * np.pi, (n_src, N))).astype(np.complex64)
    mask = bernoulli_mask(rng, F, T, B, p_loss)
    packed = np.empty((T, F, N), dtype=np.uint8)
    for t0 in range(0, T, CHUNK):
        t1 = min(T, t0 + CHUNK)
        n = t1 - t0
        s = ((rng.standard_normal((n, F, n_src)) + 1j * rng.standard_normal((n, F, n_src)))
             / np.sqrt(2.0)).astype(np.complex64)
        sky = np.einsum("tfk,ki->tfi", s, phase)
        re = rng.standard_normal((n, F, N), dtype=np.float32) * sigma + sky.real
        im = rng.standard_normal((n, F, N), dtype=np.float32) * sigma + sky.imag
        packed[t0:t1] = quantize(re, im)
    fill_lost(packed, mask, B, "zero")
    return Frame(packed, mask, N, F, T, B, f"large_n{N}_f{F}_t{T}", seed)


@dataclasses.dataclass
class InstanceSpec:
    N: int
    T: int
    sigma: float
    p_loss: float
    seed: int


def batched_specs(seed: int = SEEDS["batched"], n_inst: int = 128,
                  t_scale: float = 1.0,
                  n_choices=(64, 128, 256, 512, 1024)) -> List[InstanceSpec]:
    """Uneven single-channel instances: N from ``n_choices``, T log-uniform
    in [1024, 65536] rounded to a multiple of 256 (times ``t_scale``, for
    cheaper test runs), sigma ~ U(1.5, 3.5), loss p ~ U(0, 0.05)."""
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(n_inst):
        N = int(rng.choice(n_choices))
        T = 256 * int(round(math.exp(rng.uniform(math.log(1024), math.log(65536))) / 256))
        T = max(1, int(round(T * t_scale)))
        sigma = float(rng.uniform(1.5, 3.5))
        p = float(rng.uniform(0.0, 0.05))
        specs.append(InstanceSpec(N, T, sigma, p, int(seed * 100003 + k)))
    return specs


def instance_frame(spec: InstanceSpec, B: int = 256) -> Frame:
    fr = gaussian_frame(spec.seed, spec.N, 1, spec.T, B, spec.sigma, spec.p_loss)
    if fr.mask is None:
        fr.mask = np.zeros((1, fr.nblk), dtype=np.uint8)
    fr.name = f"inst_n{spec.N}_t{spec.T}"
    return fr


def batched(seed: int = SEEDS["batched"], n_inst: int = 128,
            t_scale: float = 1.0) -> List[Frame]:
    return [instance_frame(s) for s in batched_specs(seed, n_inst, t_scale)]


@dataclasses.dataclass
class StreamSpec:
    stream_id: int
    N: int
    F: int
    T: int                 # samples per frame
    frames_per_integration: int
    loss_rate: float       # long-run fraction of lost blocks
    rate_bps: float        # offered input rate, bits of 4-bit sky data per second
    seed: int

    @property
    def frame_bytes(self) -> int:
        return self.T * self.F * self.N

    @property
    def frame_rate(self) -> float:
        """Mean frames per second for the offered rate (8 bits per sample)."""
        return self.rate_bps / (8.0 * self.frame_bytes)


def streaming_streams(seed: int = SEEDS["streaming"], n_streams: int = 8,
                      total_bps: float = 51.2e9, T: int = 4096,
                      n_choices=(128, 256, 512), f_range=(16, 64),
                      l_range=(10, 100), max_loss: float = 0.05) -> List[StreamSpec]:
    """Several concurrent streams sharing one GPU; each is offered an equal
    share of ``total_bps`` (the per-host rate of Table I by default)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_streams):
        N = int(rng.choice(n_choices))
        F = int(rng.integers(f_range[0], f_range[1] + 1))
        L = int(rng.integers(l_range[0], l_range[1] + 1))
        loss = float(rng.uniform(0.0, max_loss))
        out.append(StreamSpec(s, N, F, T, L, loss, total_bps / n_streams,
                              int(seed * 1000 + s)))
    return out


def stream_frame(spec: StreamSpec, index: int, B: int = 256, sigma: float = 2.5,
                 burst: float = 4.0, cap: float = 0.10) -> Frame:
    """Frame ``index`` of a stream: Gaussian noise plus bursty block loss."""
    rng = np.random.default_rng([spec.seed, index])
    nblk = nblocks(spec.T, B)
    mask = gilbert_elliott_mask(rng, spec.F, nblk, spec.loss_rate, burst, cap)
    packed = np.empty((spec.T, spec.F, spec.N), dtype=np.uint8)
    for t0 in range(0, spec.T, CHUNK):
        t1 = min(spec.T, t0 + CHUNK)
        re = rng.standard_normal((t1 - t0, spec.F, spec.N), dtype=np.float32) * sigma
        im = rng.standard_normal((t1 - t0, spec.F, spec.N), dtype=np.float32) * sigma
        packed[t0:t1] = quantize(re, im)
    fill_lost(packed, mask, B, "zero")
    return Frame(packed, mask, spec.N, spec.F, spec.T, B,
                 f"stream{spec.stream_id}_frame{index}", spec.seed)


def stream_frame_variant(spec: StreamSpec, base: Frame, index: int, B: int = 256,
                         burst: float = 4.0, cap: float = 0.10) -> Frame:
    """Frame ``index`` of a stream derived from an already generated frame:
    its samples rolled in time and across inputs by steps that depend on
    the index, with a loss mask of its own (lost blocks zero).  The
    statistics are the base frame's; the data differ from it."""
    rng = np.random.default_rng([spec.seed, index, 1])
    shift = (index * 1013) % max(1, spec.T)
    packed = np.roll(np.roll(base.packed, shift, axis=0), (index * 37) % spec.N, axis=2)
    mask = gilbert_elliott_mask(rng, spec.F, nblocks(spec.T, B), spec.loss_rate, burst, cap)
    fill_lost(packed, mask, B, "zero")
    return Frame(packed, mask, spec.N, spec.F, spec.T, B,
                 f"stream{spec.stream_id}_frame{index}", spec.seed)
