"""Planted mistakes: each altered copy of the oracle must fail a pin.

Every mutant is a plausible slip in the C oracle (a dropped term, a wrong
sign or index, a transposed operand, ignored loss, float instead of double
rounding ...).  The copy is built in a temporary directory and run against
the pins; the real oracle source is never touched.
"""

import os

import pytest

import oracle
from tests import oracle_pins

# (name, original text, replacement, occurrences to replace: 0 = all)
MUTANTS = [
    ("drop_bb_term", "re += (int64_t)ai * aj + (int64_t)bi * bj;", "re += (int64_t)ai * aj;", 1),
    ("im_sign", "im += (int64_t)bi * aj - (int64_t)ai * bj;",
     "im += (int64_t)ai * bj - (int64_t)bi * aj;", 1),
    ("no_conjugate", "im += (int64_t)bi * aj - (int64_t)ai * bj;",
     "im += (int64_t)bi * aj + (int64_t)ai * bj;", 1),
    ("swap_nibbles", "return (int)(byte >> 4) - 8; }", "return (int)(byte & 15) - 8; }", 1),
    ("offset_7", "return (int)(byte & 15) - 8; }", "return (int)(byte & 15) - 7; }", 1),
    ("mask_block_index", "+ t / B]", "+ (t + 1) / B % nblk]", 1),
    ("mask_transposed", "mask[(int64_t)f * nblk + t / B]", "mask[(int64_t)(t / B) * F + f]", 1),
    ("loss_ignored", "            continue;\n        if (flags != NULL", "            ;\n        if (flags != NULL", 1),
    ("count_ignores_loss", "            n += sample_valid(mask, F, T, B, f, t);\n        count[f] = n;",
     "            n += 1;\n        count[f] = n;", 1),
    ("transposed_operand",
     "pair_sum(packed, mask, N, F, T, B, f, i, j, &out[0], &out[1]);\n            }\n    oracle_valid_counts",
     "pair_sum(packed, mask, N, F, T, B, f, j, i, &out[0], &out[1]);\n            }\n    oracle_valid_counts", 1),
    ("diagonal_dropped", "for (int j = i; j < N; ++j)", "for (int j = i + 1; j < N; ++j)", 0),
    ("accumulate_overwrites", "out[0] += re;", "out[0] = re;", 1),
    ("accumulate_count_overwrites", "count[f] += n;", "count[f] = n;", 1),
    ("normalize_float_division", "(float)((double)vis[k] / (double)n)", "(float)vis[k] / (float)n", 1),
    ("normalize_zero_count", "n == 0 ? 0.0f : ", "", 1),
    ("tri_index_column_major", "return i * N - i * (i - 1) / 2 + (j - i);",
     "return j * (j + 1) / 2 + i;", 1),
    # per-input flags (Sec. II-C)
    ("flag_no_intersection",
     "d[(int64_t)f * P + oracle_tri_index(N, i, listed[l])] += 1;", "(void)l;", 1),
    ("flag_diagonal_missing",
     "d[(int64_t)f * P + oracle_tri_index(N, i, i)] += 1;", ";", 1),
    ("flag_counts_lost_samples",
     "continue;\n            const uint32_t *field", ";\n            const uint32_t *field", 1),
    ("flag_bit_order", "if ((word >> b) & 1u)", "if ((word >> (31 - b)) & 1u)", 1),
    ("flag_fast_path_inverted", "if (word == 0)\n                    continue;",
     "if (word != 0)\n                    continue;", 1),
    ("flag_norm_intersection_sign", "+ d[p];", "- d[p];", 1),
    ("flag_norm_one_counter", " - c[(int64_t)f * N + j] + d[p];", " + d[p];", 1),
    ("flag_zero_byte", "packed[((int64_t)t * F + f) * N + i] = 0x88;",
     "packed[((int64_t)t * F + f) * N + i] = 0x00;", 1),
    ("flagged_one_side", "(input_flagged(flags, N, T, f, t, i) ||\n", "(0 ||\n", 1),
    ("flag_word_bit", "i / 32] >> (i % 32))", "i / 32] >> (31 - i % 32))", 1),
    ("normalize_pairs_float",
     "(float)((double)vis[2 * q + k] / (double)m)", "(float)vis[2 * q + k] / (float)m", 1),
    ("normalize_pairs_zero", "m == 0 ? 0.0f : ", "", 1),
    # frame assembly (Sec. II-A)
    ("assemble_last_wins", "if (filled[s * slots + k])\n            continue;",
     "if (0)\n            continue;", 1),
    ("assemble_zero_byte", "packed[(t * F + f) * N + i] = 0x88;", "packed[(t * F + f) * N + i] = 0;", 1),
    ("assemble_mask_not_set", "mask[f * slots + k] = (uint8_t)lost;", "mask[f * slots + k] = 0;", 1),
    ("assemble_band_order", "int64_t t = k * S + smp, f = s * NB + b;",
     "int64_t t = k * S + smp, f = s * NB + (NB - 1 - b);", 1),
    ("assemble_footer_order", "(((int64_t)smp * NB + b) * W) * 4;", "(((int64_t)b * S + smp) * W) * 4;", 1),
    ("assemble_window_start", "if (seq < (uint64_t)seq0 ||", "if (seq <= (uint64_t)seq0 ||", 1),
    ("assemble_stream_base", "int64_t s = (int64_t)sid - stream_base;", "int64_t s = (int64_t)sid;", 1),
    ("assemble_lost_flags_kept", "flags[(f * T + t) * W + w] = 0;", ";", 1),
    # per-input time shifting
    ("shift_sign", "int64_t src = t - delays[i];", "int64_t src = t + delays[i];", 1),
    ("shift_edge_not_flagged", "int flagged = 1;", "int flagged = 0;", 1),
    ("shift_flags_not_moved", "input_flagged(flags_in, N, T, (int)f, (int)src, i);",
     "input_flagged(flags_in, N, T, (int)f, (int)t, i);", 1),
    ("shift_edge_byte", ": 0x88;", ": 0x00;", 1),
]


def _mutant_source(orig, new, count):
    src = open(oracle.SRC).read()
    n = src.count(orig)
    assert n >= 1, f"mutation anchor not found: {orig!r}"
    if count:
        assert n == count, (orig, n)
        return src.replace(orig, new, count)
    return src.replace(orig, new)


@pytest.mark.parametrize("name,orig,new,count", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, orig, new, count):
    src = tmp_path / "mutant.c"
    src.write_text(_mutant_source(orig, new, count))
    lib = oracle.build(str(src), str(tmp_path / f"lib_{name}.so"))
    orc = oracle.load(lib)
    failed = []
    for pin in oracle_pins.PINS:
        try:
            pin(orc)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
