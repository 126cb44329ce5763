/*
 * Oracle for the X-engine correlation path.  TEST INFRASTRUCTURE ONLY.
 *
 * A deliberately plain, slow CPU implementation of what the correlator
 * computes.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may build, load or call it; the product library never links,
 * includes or calls anything in this directory, and this file includes no
 * header of the product.
 *
 * The method reaches an exact result with a plain definition, so the oracle
 * is that definition written out, with int64 accumulators:
 *
 *   sample    x[t][f][i] = a + i*b, one byte per complex sample, high nibble
 *             a+8, low nibble b+8 (4+4-bit complex values, Sec. I and
 *             Sec. II-A: all inputs of one band take one byte each).
 *   loss      a sample whose packet block is flagged lost contributes
 *             nothing, whatever its bytes hold (Sec. II-A.2: lost data are
 *             zeros).  Blocks are B samples of one channel.
 *   correlate for each channel f and 0 <= i <= j < N,
 *             V[f][i][j] = sum over valid t of x[t][f][i] * conj(x[t][f][j])
 *             stored as a row-major packed upper triangle including the
 *             diagonal, index(i,j) = i*N - i*(i-1)/2 + (j-i), (re, im).
 *   count     n[f] = number of valid samples of channel f (Sec. II-C: packet
 *             loss is tracked as one counter added to every point).
 *   accumulate adds V and n of a frame into running sums: the correlation
 *             kernels add into the output of the previous run (Sec. II-B).
 *   normalize out = (float)((double)V / (double)n), 0 when n == 0: the
 *             fraction of lost data is applied to the correlation matrix at
 *             the end of the integration (Sec. II-C).
 *
 *   flags     per-input F-engine flags (Sec. II-C), bit-fields beside the
 *             frame: flagged points are zeroed before correlation, and the
 *             normalisation matrix counts, per baseline, the valid samples
 *             where neither input is flagged.  The bookkeeping follows the
 *             method's own steps (per-input counters, intersections per
 *             sample, then count - c_i - c_j + d_ij); the flagged
 *             correlation is the plain definition with both conditions.
 *
 * Loop order follows the definition: channel, i, j >= i, then the sum over
 * t.  OpenMP may split the (f, i) loop across threads; every sum is exact,
 * so the thread count does not change any result.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

/* value of the high (real) nibble and of the low (imaginary) nibble */
static int re_part(uint8_t byte) { return (int)(byte >> 4) - 8; }
static int im_part(uint8_t byte) { return (int)(byte & 15) - 8; }

/* 1 when sample t of channel f is valid (its block is not flagged lost) */
static int sample_valid(const uint8_t *mask, int F, int T, int B, int f, int t)
{
    (void)F;
    if (mask == NULL)
        return 1;
    int64_t nblk = ((int64_t)T + B - 1) / B;
    return mask[(int64_t)f * nblk + t / B] == 0;
}

int64_t oracle_tri_index(int64_t N, int64_t i, int64_t j)
{
    return i * N - i * (i - 1) / 2 + (j - i);
}

int64_t oracle_num_pairs(int64_t N)
{
    return N * (N + 1) / 2;
}

void oracle_decode(uint8_t byte, int32_t *re, int32_t *im)
{
    *re = re_part(byte);
    *im = im_part(byte);
}

/* n[f] = number of valid samples of channel f in this frame */
void oracle_valid_counts(const uint8_t *mask, int32_t F, int32_t T, int32_t B,
                         int64_t *count)
{
    for (int f = 0; f < F; ++f) {
        int64_t n = 0;
        for (int t = 0; t < T; ++t)
            n += sample_valid(mask, F, T, B, f, t);
        count[f] = n;
    }
}

/* 1 when the per-input flag bit-fields (described below, Sec. II-C) mark
 * input i of channel f at sample t */
static int input_flagged(const uint32_t *flags, int N, int T, int f, int t,
                         int i)
{
    int64_t W = ((int64_t)N + 31) / 32;
    return (int)((flags[((int64_t)f * T + t) * W + i / 32] >> (i % 32)) & 1u);
}

/* sum over valid t of x_i * conj(x_j) for one channel and one pair; with
 * per-input flags, samples where either input is flagged are skipped too */
static void pair_sum_flagged(const uint8_t *packed, const uint8_t *mask,
                             const uint32_t *flags, int N, int F, int T, int B,
                             int f, int i, int j, int64_t *re_out,
                             int64_t *im_out)
{
    int64_t re = 0, im = 0;
    for (int t = 0; t < T; ++t) {
        if (!sample_valid(mask, F, T, B, f, t))
            continue;
        if (flags != NULL && (input_flagged(flags, N, T, f, t, i) ||
                              input_flagged(flags, N, T, f, t, j)))
            continue;
        const uint8_t *row = packed + ((int64_t)t * F + f) * N;
        int ai = re_part(row[i]), bi = im_part(row[i]);
        int aj = re_part(row[j]), bj = im_part(row[j]);
        /* (ai + i bi)(aj - i bj) = (ai aj + bi bj) + i (bi aj - ai bj) */
        re += (int64_t)ai * aj + (int64_t)bi * bj;
        im += (int64_t)bi * aj - (int64_t)ai * bj;
    }
    *re_out = re;
    *im_out = im;
}

static void pair_sum(const uint8_t *packed, const uint8_t *mask, int N, int F,
                     int T, int B, int f, int i, int j, int64_t *re_out,
                     int64_t *im_out)
{
    pair_sum_flagged(packed, mask, NULL, N, F, T, B, f, i, j, re_out, im_out);
}

/* V over one frame, overwriting vis [F][P][2] and count [F] */
void oracle_correlate(const uint8_t *packed, const uint8_t *mask, int32_t N,
                      int32_t F, int32_t T, int32_t B, int64_t *vis,
                      int64_t *count)
{
    int64_t P = oracle_num_pairs(N);
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int f = 0; f < F; ++f)
        for (int i = 0; i < N; ++i)
            for (int j = i; j < N; ++j) {
                int64_t *out = vis + ((int64_t)f * P + oracle_tri_index(N, i, j)) * 2;
                pair_sum(packed, mask, N, F, T, B, f, i, j, &out[0], &out[1]);
            }
    oracle_valid_counts(mask, F, T, B, count);
}

/* running integration: vis += V(frame), count += n(frame) */
void oracle_accumulate(const uint8_t *packed, const uint8_t *mask, int32_t N,
                       int32_t F, int32_t T, int32_t B, int64_t *vis,
                       int64_t *count)
{
    int64_t P = oracle_num_pairs(N);
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int f = 0; f < F; ++f)
        for (int i = 0; i < N; ++i)
            for (int j = i; j < N; ++j) {
                int64_t re, im;
                pair_sum(packed, mask, N, F, T, B, f, i, j, &re, &im);
                int64_t *out = vis + ((int64_t)f * P + oracle_tri_index(N, i, j)) * 2;
                out[0] += re;
                out[1] += im;
            }
    for (int f = 0; f < F; ++f) {
        int64_t n = 0;
        for (int t = 0; t < T; ++t)
            n += sample_valid(mask, F, T, B, f, t);
        count[f] += n;
    }
}

/* every ordered pair (i, j), full matrix [F][N][N][2]; used for checks
 * that need both triangles (Hermitian symmetry) */
void oracle_correlate_full(const uint8_t *packed, const uint8_t *mask,
                           int32_t N, int32_t F, int32_t T, int32_t B,
                           int64_t *vis_full)
{
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int f = 0; f < F; ++f)
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                int64_t *out = vis_full + (((int64_t)f * N + i) * N + j) * 2;
                pair_sum(packed, mask, N, F, T, B, f, i, j, &out[0], &out[1]);
            }
}

/* V for a list of (f, i, j) triples only, out [n][2]; lets a test check a
 * sample of baselines of a frame too large for the full loop */
void oracle_correlate_pairs(const uint8_t *packed, const uint8_t *mask,
                            int32_t N, int32_t F, int32_t T, int32_t B,
                            const int32_t *fs, const int32_t *is,
                            const int32_t *js, int64_t n, int64_t *out)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t k = 0; k < n; ++k)
        pair_sum(packed, mask, N, F, T, B, fs[k], is[k], js[k], &out[2 * k],
                 &out[2 * k + 1]);
}

/* out [F][P][2] = V / n in double, rounded once to float; 0 when n == 0 */
void oracle_normalize(const int64_t *vis, const int64_t *count, int32_t N,
                      int32_t F, float *out)
{
    int64_t P = oracle_num_pairs(N);
    for (int f = 0; f < F; ++f) {
        int64_t n = count[f];
        for (int64_t p = 0; p < 2 * P; ++p) {
            int64_t k = (int64_t)f * 2 * P + p;
            out[k] = n == 0 ? 0.0f : (float)((double)vis[k] / (double)n);
        }
    }
}

/* ---------------------------------------------------------------------
 * Per-input flags (Sec. II-C).  Besides whole lost packets, the F-engine
 * flags single data points (range or sampling faults); those points are
 * zeroed before the correlator sees them, so baseline (i, j) integrates
 * fewer samples than its channel's valid count.  The flags arrive as
 * bit-fields: flags[f][t][w] is a 32-bit word, W = ceil(N/32) words per
 * (channel, sample), bit i%32 of word i/32 set when input i is flagged.
 * Bits past input N-1 in the last word carry nothing.  A lost sample
 * (packet mask) brings no footer, so its flags are never counted: the
 * loss counter already removes that sample from every baseline.
 * --------------------------------------------------------------------- */

/* Flag bookkeeping as the method describes it, added into c and d:
 *   c[f][i]           number of valid samples where input i is flagged
 *                     (the per-input, per-frequency counters);
 *   d[f][tri(i, j)]   for i < j, number of valid samples where i and j are
 *                     flagged together (the intersections recorded per
 *                     sample); on the diagonal d[f][tri(i, i)] = c[f][i],
 *                     an input meeting itself in every flagged sample.
 * Each sample's bit-field is read a 32-bit word at a time and bits are
 * extracted only from non-zero words; the flagged inputs of the sample are
 * listed and every pair of the list is counted, O(E^2) for E flags. */
void oracle_flag_counters(const uint32_t *flags, const uint8_t *mask,
                          int32_t N, int32_t F, int32_t T, int32_t B,
                          int64_t *c, int64_t *d)
{
    int64_t W = ((int64_t)N + 31) / 32;
    int64_t P = oracle_num_pairs(N);
    int *listed = (int *)malloc(((size_t)N + 1) * sizeof(int));
    if (listed == NULL)
        return;
    for (int f = 0; f < F; ++f) {
        for (int t = 0; t < T; ++t) {
            if (!sample_valid(mask, F, T, B, f, t))
                continue;
            const uint32_t *field = flags + ((int64_t)f * T + t) * W;
            int E = 0;
            for (int64_t w = 0; w < W; ++w) {
                uint32_t word = field[w];
                if (word == 0)
                    continue;
                for (int b = 0; b < 32 && w * 32 + b < N; ++b)
                    if ((word >> b) & 1u)
                        listed[E++] = (int)(w * 32 + b);
            }
            for (int k = 0; k < E; ++k) {
                int i = listed[k];
                c[(int64_t)f * N + i] += 1;
                d[(int64_t)f * P + oracle_tri_index(N, i, i)] += 1;
                for (int l = k + 1; l < E; ++l)
                    d[(int64_t)f * P + oracle_tri_index(N, i, listed[l])] += 1;
            }
        }
    }
    free(listed);
}

/* Normalisation matrix, overwriting n [F][P]: the channel's valid-sample
 * count (frame samples less the packet-loss counter) less the flag
 * counters of both inputs, plus their intersection, which was subtracted
 * twice:  n_ij = count_f - c_i - c_j + d_ij, and n_ii = count_f - c_i. */
void oracle_flag_norm(const int64_t *count, const int64_t *c, const int64_t *d,
                      int32_t N, int32_t F, int64_t *n)
{
    int64_t P = oracle_num_pairs(N);
    for (int f = 0; f < F; ++f)
        for (int i = 0; i < N; ++i)
            for (int j = i; j < N; ++j) {
                int64_t p = (int64_t)f * P + oracle_tri_index(N, i, j);
                n[p] = count[f] - c[(int64_t)f * N + i] - c[(int64_t)f * N + j] + d[p];
            }
}

/* Zero every flagged data point of a frame in place: byte 0x88 decodes to
 * 0 + 0i.  This is what happens to flagged points before correlation. */
void oracle_apply_flags(uint8_t *packed, const uint32_t *flags, int32_t N,
                        int32_t F, int32_t T)
{
    for (int t = 0; t < T; ++t)
        for (int f = 0; f < F; ++f)
            for (int i = 0; i < N; ++i)
                if (input_flagged(flags, N, T, f, t, i))
                    packed[((int64_t)t * F + f) * N + i] = 0x88;
}

/* V of a frame with per-input flags, overwriting vis [F][P][2] and count
 * [F]: the sum over samples that are valid and where neither input is
 * flagged; count is the channel's valid-sample count, as without flags. */
void oracle_correlate_flagged(const uint8_t *packed, const uint8_t *mask,
                              const uint32_t *flags, int32_t N, int32_t F,
                              int32_t T, int32_t B, int64_t *vis,
                              int64_t *count)
{
    int64_t P = oracle_num_pairs(N);
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int f = 0; f < F; ++f)
        for (int i = 0; i < N; ++i)
            for (int j = i; j < N; ++j) {
                int64_t *out = vis + ((int64_t)f * P + oracle_tri_index(N, i, j)) * 2;
                pair_sum_flagged(packed, mask, flags, N, F, T, B, f, i, j,
                                 &out[0], &out[1]);
            }
    oracle_valid_counts(mask, F, T, B, count);
}

/* out [F][P][2] = V / n_ij per baseline, in double rounded once to float;
 * 0 where n_ij == 0 */
void oracle_normalize_pairs(const int64_t *vis, const int64_t *n, int32_t N,
                            int32_t F, float *out)
{
    int64_t P = oracle_num_pairs(N);
    for (int64_t q = 0; q < (int64_t)F * P; ++q)
        for (int k = 0; k < 2; ++k) {
            int64_t m = n[q];
            out[2 * q + k] = m == 0 ? 0.0f : (float)((double)vis[2 * q + k] / (double)m);
        }
}

/* ---------------------------------------------------------------------
 * Frame assembly from UDP packets (Sec. II-A: the network thread places
 * each packet's data by its sequence number; missing packets leave zeros,
 * out-of-order packets go to their own place, duplicates are ignored).
 *
 * Packet layout (the paper's figure of it is not available; this one keeps
 * its contents): a 16-byte header (uint64 sequence number, uint32 stream
 * id, uint32 input count N), then the data of 4 samples x 8 bands x N
 * inputs, one byte each, in that order, then the flag bit-fields of the 4 x
 * 8 (sample, band) pairs, W = ceil(N/32) uint32 words each.  Stream
 * stream_base + s carries channels 8 s .. 8 s + 7 of the frame; the packet
 * with sequence number seq0 + k holds samples 4 k .. 4 k + 3.
 *
 * stats [6]: packets in the frame's window, outside it, of an unknown
 * stream, with a wrong input count, placed, and (stream, slot) places left
 * empty.  Duplicates = in window - placed.
 * --------------------------------------------------------------------- */
void oracle_assemble(const uint8_t *packets, int64_t n_packets, int32_t N,
                     int32_t n_streams, int32_t stream_base, int64_t seq0,
                     int32_t T, uint8_t *packed, uint8_t *mask,
                     uint32_t *flags, int64_t *stats)
{
    const int S = 4, NB = 8;
    int64_t W = ((int64_t)N + 31) / 32;
    int64_t F = (int64_t)NB * n_streams;
    int64_t slots = T / S;
    int64_t pbytes = 16 + (int64_t)S * NB * N + (int64_t)S * NB * W * 4;
    char *filled = (char *)calloc((size_t)(n_streams * slots), 1);
    if (filled == NULL)
        return;
    for (int k = 0; k < 6; ++k)
        stats[k] = 0;
    /* every packet in arrival order */
    for (int64_t p = 0; p < n_packets; ++p) {
        const uint8_t *pkt = packets + p * pbytes;
        uint64_t seq = 0;
        uint32_t sid = 0, nin = 0;
        for (int b = 0; b < 8; ++b)
            seq |= (uint64_t)pkt[b] << (8 * b);
        for (int b = 0; b < 4; ++b) {
            sid |= (uint32_t)pkt[8 + b] << (8 * b);
            nin |= (uint32_t)pkt[12 + b] << (8 * b);
        }
        if (nin != (uint32_t)N) {
            stats[3] += 1;
            continue;
        }
        int64_t s = (int64_t)sid - stream_base;
        if (s < 0 || s >= n_streams) {
            stats[2] += 1;
            continue;
        }
        if (seq < (uint64_t)seq0 || seq - (uint64_t)seq0 >= (uint64_t)slots) {
            stats[1] += 1;
            continue;
        }
        stats[0] += 1;
        int64_t k = (int64_t)(seq - (uint64_t)seq0);
        if (filled[s * slots + k])
            continue;          /* a duplicate: the first arrival stays */
        filled[s * slots + k] = 1;
        stats[4] += 1;
        for (int smp = 0; smp < S; ++smp)
            for (int b = 0; b < NB; ++b) {
                int64_t t = k * S + smp, f = s * NB + b;
                for (int i = 0; i < N; ++i)
                    packed[(t * F + f) * N + i] = pkt[16 + ((int64_t)smp * NB + b) * N + i];
                const uint8_t *fw = pkt + 16 + (int64_t)S * NB * N +
                                    (((int64_t)smp * NB + b) * W) * 4;
                for (int64_t w = 0; w < W; ++w) {
                    uint32_t v = 0;
                    for (int c = 0; c < 4; ++c)
                        v |= (uint32_t)fw[w * 4 + c] << (8 * c);
                    flags[(f * T + t) * W + w] = v;
                }
            }
    }
    /* places no packet reached: zeros in the data, no flags, block lost */
    for (int64_t s = 0; s < n_streams; ++s)
        for (int64_t k = 0; k < slots; ++k) {
            int lost = !filled[s * slots + k];
            stats[5] += lost;
            for (int b = 0; b < NB; ++b) {
                int64_t f = s * NB + b;
                mask[f * slots + k] = (uint8_t)lost;
                if (!lost)
                    continue;
                for (int smp = 0; smp < S; ++smp) {
                    int64_t t = k * S + smp;
                    for (int i = 0; i < N; ++i)
                        packed[(t * F + f) * N + i] = 0x88;
                    for (int64_t w = 0; w < W; ++w)
                        flags[(f * T + t) * W + w] = 0;
                }
            }
        }
    free(filled);
}

/* ---------------------------------------------------------------------
 * Per-input time shifting (the caption of Fig. 4, Sec. II-B, names time
 * shifting among the extra operations of the GPU kernel stage and gives no
 * algorithm; the reading here is an integer sample delay per input).  Input i of every channel is delayed
 * by delays[i] samples: out[t][f][i] = in[t - d_i][f][i] when 0 <= t - d_i
 * < T.  A sample shifted in from outside the frame has no data: it becomes
 * 0x88 (0 + 0i) and a flagged point, so the per-baseline normalisation
 * counts it out.  F-engine flags move with their data: flags_out[f][t] of
 * input i = flags_in[f][t - d_i] of input i (flags_in may be NULL = none),
 * or 1 outside the frame.  Bits past input N-1 are written as 0.
 * --------------------------------------------------------------------- */
void oracle_time_shift(const uint8_t *packed, const uint32_t *flags_in,
                       const int32_t *delays, int32_t N, int32_t F, int32_t T,
                       uint8_t *out, uint32_t *flags_out)
{
    int64_t W = ((int64_t)N + 31) / 32;
    for (int64_t f = 0; f < F; ++f)
        for (int64_t t = 0; t < T; ++t)
            for (int64_t w = 0; w < W; ++w)
                flags_out[(f * T + t) * W + w] = 0;
    for (int64_t t = 0; t < T; ++t)
        for (int64_t f = 0; f < F; ++f)
            for (int i = 0; i < N; ++i) {
                int64_t src = t - delays[i];
                int inside = src >= 0 && src < T;
                out[(t * F + f) * N + i] = inside ? packed[(src * F + f) * N + i] : 0x88;
                int flagged = 1;
                if (inside)
                    flagged = flags_in != NULL &&
                              input_flagged(flags_in, N, T, (int)f, (int)src, i);
                if (flagged)
                    flags_out[(f * T + t) * W + i / 32] |= 1u << (i % 32);
            }
}
