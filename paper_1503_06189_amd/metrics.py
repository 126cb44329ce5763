"""Rate and work definitions used when reporting throughput.

Input rate counts every 4+4-bit sample of every input and channel, lost or
not, at 8 bits per sample: the "4-bit sky data" rate of Table I (one link
= 8 bands x 256 inputs x 390,625 samples/s x 8 bit = 6.4 Gb/s).  The
algorithmic work is 8 integer operations (4 multiplies, 4 adds) per
complex multiply-accumulate, over the upper triangle including the
autocorrelations, per channel and sample.
"""

#: F-engine sample rate per channel: 400 MHz split into 1024 bins (Sec. I)
SAMPLE_RATE_HZ = 400e6 / 1024


def num_pairs(N: int) -> int:
    """Baselines in the upper triangle including autocorrelations."""
    return N * (N + 1) // 2


def input_bits(N: int, F: int, T: int) -> int:
    """Bits of packed input for T samples of N inputs in F channels."""
    return 8 * N * F * T


def input_gbps(N: int, F: int, T: int, seconds: float) -> float:
    return input_bits(N, F, T) / seconds / 1e9


def int_ops(N: int, F: int, T: int) -> int:
    """Algorithmic integer ops: 8 per (channel, upper-triangle pair, sample)."""
    return 8 * num_pairs(N) * F * T


def input_bytes(N: int, F: int, T: int) -> int:
    return N * F * T


def output_bytes(N: int, F: int) -> int:
    """int32 (re, im) per baseline and channel."""
    return 8 * num_pairs(N) * F
