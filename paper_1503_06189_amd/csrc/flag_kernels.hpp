// flag_kernels.hpp -- gfx950 kernels for per-input flags (Sec. II-C).
//
// The F-engine flags single data points (range or sampling faults).  Flagged
// points are zeroed before correlation, so baseline (i, j) of channel f
// integrates
//     n_ij = count_f - c_i - c_j + d_ij
// samples: count_f valid samples of the channel, c_i of them with input i
// flagged, d_ij with both flagged (d_ii = c_i).  The method keeps c and d on
// the host, listing the flagged inputs of every sample, O(E^2) per sample.
// Here d, diagonal included, is one 0/1 Gram matrix per channel,
//     D = A A^T over valid samples,  A[i][t] = flag bit of input i at t,
// on the int8 matrix cores: exact, and its cost does not grow with the
// number of points a sample flags.
//
// Flags arrive as bit-fields flags[f][t][w], W = ceil(N/32) words, bit i % 32
// of word i / 32 = input i.  A workgroup takes one channel, one pair of
// 256-input super blocks (R <= C) and one chunk of time; its waves take the
// chunk's 32-sample steps in turn and never wait for each other:
//   1. a wave loads the words of its next 8 steps at once (0 for lost
//      samples, samples past the chunk and inputs past N) and finds, with one
//      ballot per word, which 32-input blocks hold a flag in each step; a
//      step without any ends there, the counterpart of the method's test of
//      whole 32-bit words before extracting bits;
//   2. for a flagged step, the wave turns every flagged block's 32 x 32 bits
//      into the operand of v_mfma_i32_32x32x32_i8 (lane l: input l % 32, 16
//      samples of half l / 32 as 0/1 bytes) by byte selection and a shift,
//      and runs one MFMA per tile whose two blocks both hold a flag;
//   3. the tile's counts are added into the workgroup's LDS counts (16 bits
//      each, two per word), and at the end the nonzero ones into d with
//      integer atomics, so the order of waves and chunks does not matter.
// A chunk without any flag costs only its loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace xe {
namespace flag {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kSuper = 8;           // 32-input blocks per super block
constexpr int kWindow = 1024;       // validity words per chunk: chunks <= 32768 samples

struct Args {
    const uint32_t *flags;   // [F][T][W]
    const uint8_t *mask;     // [F][nblk], may be null
    int32_t *d;              // [F][P]
    int N, F, T, B, W, nblk;
    int ns;                  // super blocks, ceil(N / 256)
    int chunks;              // time chunks per (channel, pair)
    int chunk_samples;       // samples per chunk, a multiple of 32, <= 32 kWindow
    uint64_t b_magic;        // ceil(2^40 / B) when B <= 2^16, else 0
};

// t / B for 0 <= t < 2^24: (t * ceil(2^40 / B)) >> 40 is exact when B <= 2^16
// (the rounding adds less than 2^-16 to t / B, whose fraction is at most
// 1 - 1/B); larger B divides.
__device__ __forceinline__ int block_of(const Args &a, int t) {
    return a.b_magic ? (int)(((uint64_t)(uint32_t)t * a.b_magic) >> 40) : t / a.B;
}

// A diagonal pair (R == C) has 36 tiles of 32 x 32 counts (blocks bi <= bj)
// and runs 16 waves; an off-diagonal pair (R < C) has 64 and runs 8 waves,
// and every wave loads the words of both super blocks.
template <bool kOff>
struct Shape {
    static constexpr int kSides = kOff ? 2 : 1;
    static constexpr int kWaves = kOff ? 8 : 16;
    static constexpr int kThreads = 64 * kWaves;
    static constexpr int kTiles = kOff ? 64 : 36;
    static constexpr int kBatch = kOff ? 4 : 8;   // steps a wave loads before it uses the first
    static constexpr int kPitch = kOff ? 8 : 9;   // 64-bit words per tile column in LDS
    static constexpr int kTileQuads = 32 * kPitch;
};

// Counts of the chunk in LDS as four 16-bit fields per 64-bit word (a chunk
// holds at most 32768 samples, so no field carries into the next): tile k,
// column j, rows 4 Q .. 4 Q + 3 at acc[k][j * kPitch + Q], row 4 Q in the
// low field.  The diagonal pair's odd pitch spreads the two half-waves of
// an MFMA result over different banks.
template <bool kOff>
struct Lds {
    using S = Shape<kOff>;
    uint64_t acc[S::kTiles * S::kTileQuads];
    uint32_t words[S::kWaves][S::kSides][kSuper][32];  // per wave: its current step
    uint32_t valid[kWindow];   // bit k of word s: sample 32 s + k of the chunk
};

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

__device__ __forceinline__ v16i mfma(v4i a, v4i b, v16i c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int64_t tri(int64_t N, int64_t i, int64_t j) {
    return i * N - i * (i - 1) / 2 + (j - i);
}

// Operand of block b of one step, from the 32 words of its samples
// (src[t] = word of sample t): byte q of this lane's 16 is the flag of input
// l % 32 at sample 16 (l / 32) + q.  Each group of 4 words gives one dword:
// byte (i / 8) of each word is gathered with two byte permutes, then bit
// (i % 8) of every byte is shifted down and masked.
__device__ __forceinline__ v4i build_op(const uint32_t *src, int lane) {
    const int i = lane & 31, h = lane >> 5;
    const uint32_t bi = (uint32_t)(i >> 3), bb = (uint32_t)(i & 7);
    const uint32_t sel_lo = 0x0c0c0000u | ((4u + bi) << 8) | bi;
    const uint32_t sel_hi = ((4u + bi) << 24) | (bi << 16) | 0x0c0cu;
    const v4i *p = (const v4i *)(src + h * 16);
    v4i out;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const v4i w = p[d];
        const uint32_t x = perm((uint32_t)w.y, (uint32_t)w.x, sel_lo) |
                           perm((uint32_t)w.w, (uint32_t)w.z, sel_hi);
        out[d] = (int)((x >> bb) & 0x01010101u);
    }
    return out;
}

// Add a 32 x 32 block of counts (an MFMA result: element v at row
// 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32) into LDS tile `t`, four rows
// per 64-bit word.
template <int PITCH>
__device__ __forceinline__ void add_tile(uint64_t *t, const v16i &c, int lane) {
    uint64_t *col = t + (lane & 31) * PITCH + (lane >> 5);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint64_t lo = (uint32_t)c[4 * q] | ((uint32_t)c[4 * q + 1] << 16);
        const uint64_t hi = (uint32_t)c[4 * q + 2] | ((uint32_t)c[4 * q + 3] << 16);
        atomicAdd((unsigned long long *)(col + 2 * q), (unsigned long long)(lo | (hi << 32)));
    }
}

// Validity of the chunk's samples, one bit each, in LDS: 1 inside the chunk
// and outside lost blocks.  All threads take part; a barrier must follow.
template <bool kOff>
__device__ __forceinline__ void fill_window(const Args &a, Lds<kOff> &L, int f, int t_begin,
                                            int t_end, int tid) {
    const int words = (t_end - t_begin + 31) >> 5;
    for (int s = tid; s < words; s += Shape<kOff>::kThreads) {
        const int t = t_begin + 32 * s;
        const int n = min(32, t_end - t);
        uint32_t bits = n == 32 ? 0xffffffffu : (1u << n) - 1u;
        if (a.mask) {
            // the blocks touching the word's samples, eight loads at a time,
            // all issued before the first is used (indices clamped)
            const uint8_t *row = a.mask + (int64_t)f * a.nblk;
            const int first = block_of(a, t), last = block_of(a, t + n - 1);
            for (int b0 = first; b0 <= last; b0 += 8) {
                uint32_t v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = row[min(b0 + q, last)];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int b = b0 + q;
                    if (b > last || v[q] == 0u) continue;
                    const int lo = max(t, b * a.B) - t;
                    const int hi = min(t + n, (b + 1) * a.B) - t;    // exclusive
                    const uint64_t span = ((1ull << hi) - 1ull) & ~((1ull << lo) - 1ull);
                    bits &= ~(uint32_t)span;
                }
            }
        }
        L.valid[s] = bits;
    }
}

// The words of kBatch steps, step q at byte row0 + q * step_bytes of the
// buffer (steps past its range read 0), all loads issued before any is
// used: four dwords per side, or one 16-byte load when kVec (the four words
// of a side are contiguous and 16-byte aligned).
template <bool kVec, int kBatch, int SIDES>
__device__ __forceinline__ void load_batch(uint32_t (&raw)[kBatch][SIDES][4],
                                           __amdgpu_buffer_rsrc_t rsrc,
                                           const uint32_t (&off)[SIDES][4], uint32_t row0,
                                           uint32_t step_bytes) {
#pragma unroll
    for (int q = 0; q < kBatch; ++q)
#pragma unroll
        for (int side = 0; side < SIDES; ++side) {
            const uint32_t o = row0 + q * step_bytes;
            if (kVec) {
                const v4i v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(o + off[side][0]),
                                                                    0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) raw[q][side][r] = (uint32_t)v[r];
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    raw[q][side][r] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(
                        rsrc, (int)(o + off[side][r]), 0, 0);
            }
        }
}

// Workgroup b runs on XCD b % 8; consecutive work items (the chunks of one
// channel and pair) are numbered onto one XCD so they share its L2.
__device__ __forceinline__ int64_t xcd_local(int64_t b, int64_t total) {
    const int64_t per = total / 8, rem = total % 8;
    const int64_t x = b % 8, idx = b / 8;
    return x * per + (x < rem ? x : rem) + idx;
}

// One workgroup: channel f, super-block pair (R, C), one time chunk.  Every
// wave takes its own 32-sample steps of the chunk (wave, wave + waves, ...),
// kBatch steps' loads in flight at once (the first batch issued before the
// workgroup's set-up), and never waits for another wave:
//   * lane l holds sample l / 2 of the step and words 4 (l % 2) .. +3 of
//     each super block, masked by the sample's validity and the inputs < N;
//   * one ballot tells whether the step holds any flag; a step without any
//     (the common case for the sparse flags of the method) ends there, the
//     counterpart of the method's test of whole 32-bit words;
//   * otherwise one ballot per word tells which 32-input blocks hold a flag,
//     the wave stores the step's words in its own LDS slot, builds the MFMA
//     operand of every flagged block, and runs one v_mfma_i32_32x32x32_i8 per
//     tile whose two blocks both hold a flag, adding the 32 x 32 counts into
//     the workgroup's LDS counts.
// After a barrier, the nonzero counts are added into d with integer atomics
// (time chunks of one pair add into the same counts; the order does not
// matter).
template <bool kOff, bool kVec>
__global__ __launch_bounds__(Shape<kOff>::kThreads) void gram_kernel(Args a) {
    using S = Shape<kOff>;
    constexpr int SIDES = S::kSides;
    __shared__ __attribute__((aligned(16))) Lds<kOff> L;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int pairs = kOff ? a.ns * (a.ns - 1) / 2 : a.ns;
    const int64_t total = (int64_t)a.F * pairs * a.chunks;
    const int64_t w = xcd_local(blockIdx.x, total);
    const int chunk = (int)(w % a.chunks);
    const int64_t rest = w / a.chunks;
    const int g = (int)(rest % pairs);
    const int f = __builtin_amdgcn_readfirstlane((int)(rest / pairs));
    int R = g, C = g;
    if (kOff) {
        // g -> (R, C), R < C, row-major over the strict upper triangle
        int rem = g;
        R = 0;
        while (rem >= a.ns - 1 - R) {
            rem -= a.ns - 1 - R;
            ++R;
        }
        C = R + 1 + rem;
    }
    R = __builtin_amdgcn_readfirstlane(R);
    C = __builtin_amdgcn_readfirstlane(C);
    const int t_begin = __builtin_amdgcn_readfirstlane(chunk * a.chunk_samples);
    const int t_end = __builtin_amdgcn_readfirstlane(min(a.T, t_begin + a.chunk_samples));
    const int nsteps = (t_end - t_begin + 31) >> 5;

    // the chunk's rows of this channel's flags through a buffer resource
    // whose range ends at the chunk's last sample: loads past it return 0
    // without a memory access
    const uint32_t row_bytes = 4u * (uint32_t)a.W;
    const uint64_t base = (uint64_t)(uintptr_t)(a.flags + ((int64_t)f * a.T + t_begin) * a.W);
    const uint32_t extent =
        __builtin_amdgcn_readfirstlane((uint32_t)(t_end - t_begin) * row_bytes);
    // (readfirstlane returns int: both halves go through uint32_t so the low
    // one is not sign-extended into the high one)
    const uint32_t base_lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t base_hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    void *bp = (void *)(uintptr_t)(((uint64_t)base_hi << 32) | base_lo);
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(bp, (short)0, (int)extent, 0x00020000);
    // per lane: byte offset of each word within a row and the bits of
    // inputs < N; a word past the row reads the last word (kVec: the last
    // four), masked to 0
    uint32_t off[SIDES][4], pad[SIDES][4];
#pragma unroll
    for (int side = 0; side < SIDES; ++side)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gw = (side == 0 ? R : C) * kSuper + 4 * (lane & 1) + r;
            const int left = a.N - gw * 32;
            off[side][r] = kVec ? 4u * (uint32_t)min(gw - r, a.W - 4) + 4u * r
                                : 4u * (uint32_t)min(gw, a.W - 1);
            pad[side][r] = left >= 32 ? 0xffffffffu : left > 0 ? (1u << left) - 1u : 0u;
        }
    const uint32_t smp = (uint32_t)(lane >> 1);
    const uint32_t step_bytes = 32u * S::kWaves * row_bytes;
    auto batch_row = [&](int j0) {
        return (32u * (uint32_t)(wave + S::kWaves * j0) + smp) * row_bytes;
    };
    uint32_t raw[S::kBatch][SIDES][4];
    load_batch<kVec, S::kBatch, SIDES>(raw, rsrc, off, batch_row(0), step_bytes);

    // clear the counts, build the validity window
    {
        uint4 *z = (uint4 *)L.acc;
        for (int e = tid; e < S::kTiles * S::kTileQuads / 2; e += S::kThreads)
            z[e] = (uint4){0u, 0u, 0u, 0u};
    }
    fill_window(a, L, f, t_begin, t_end, tid);
    __syncthreads();   // counts cleared, validity window visible

    constexpr uint64_t kEven = 0x5555555555555555ull;
    constexpr int cs = SIDES - 1;   // side of the column blocks
    uint32_t(*slot)[kSuper][32] = L.words[wave];
    for (int j0 = 0; wave + S::kWaves * j0 < nsteps; j0 += S::kBatch) {
        if (j0 > 0) load_batch<kVec, S::kBatch, SIDES>(raw, rsrc, off, batch_row(j0), step_bytes);
#pragma unroll
        for (int q = 0; q < S::kBatch; ++q) {
            const int s = wave + S::kWaves * (j0 + q);
            if (s >= nsteps) continue;
            const uint32_t keep = 0u - ((L.valid[s] >> smp) & 1u);
            uint32_t seen[SIDES];
#pragma unroll
            for (int side = 0; side < SIDES; ++side) {
                seen[side] = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    raw[q][side][r] &= pad[side][r] & keep;
                    seen[side] |= raw[q][side][r];
                }
            }
            bool flagged = true;
#pragma unroll
            for (int side = 0; side < SIDES; ++side) flagged = flagged && __ballot(seen[side] != 0u) != 0;
            if (!flagged) continue;
            // bit b of blk[side]: block b of the side holds a flag
            uint32_t blk[SIDES];
#pragma unroll
            for (int side = 0; side < SIDES; ++side) {
                uint32_t bits = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint64_t m = __ballot(raw[q][side][r] != 0u);
                    bits |= ((m & kEven) != 0 ? 1u : 0u) << r;
                    bits |= ((m & ~kEven) != 0 ? 1u : 0u) << (4 + r);
                }
                blk[side] = __builtin_amdgcn_readfirstlane(bits);
            }
            // the step's words in this wave's slot, [side][block][sample]
#pragma unroll
            for (int side = 0; side < SIDES; ++side)
#pragma unroll
                for (int r = 0; r < 4; ++r) slot[side][4 * (lane & 1) + r][smp] = raw[q][side][r];
            // operands of the column side's flagged blocks; a row block's
            // operand is the same (diagonal pair) or built when its row of
            // tiles comes
            v4i op[kSuper];
#pragma unroll
            for (int b = 0; b < kSuper; ++b)
                if ((blk[cs] >> b) & 1u) op[b] = build_op(slot[cs][b], lane);
            const v16i zero = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int bi = 0; bi < kSuper; ++bi) {
                if (((blk[0] >> bi) & 1u) == 0u) continue;
                const v4i row_op = kOff ? build_op(slot[0][bi], lane) : op[bi];
#pragma unroll
                for (int bj = kOff ? 0 : bi; bj < kSuper; ++bj) {
                    if (((blk[cs] >> bj) & 1u) == 0u) continue;
                    const int k = kOff ? bi * kSuper + bj
                                       : bi * kSuper - bi * (bi - 1) / 2 + (bj - bi);
                    add_tile<S::kPitch>(L.acc + k * S::kTileQuads, mfma(row_op, op[bj], zero),
                                        lane);
                }
            }
        }
    }
    __syncthreads();   // every wave's counts added

    // the nonzero counts into d
    const int64_t P = (int64_t)a.N * (a.N + 1) / 2;
    int32_t *dst = a.d + (int64_t)f * P;
    for (int e = tid; e < S::kTiles * 256; e += S::kThreads) {
        const int k = e >> 8, j = (e >> 3) & 31, Q = e & 7;
        const uint64_t word = L.acc[k * S::kTileQuads + j * S::kPitch + Q];
        if (word == 0u) continue;
        int bi, bj;
        if (kOff) {
            bi = k >> 3;
            bj = k & 7;
        } else {
            int kk = k;
            bi = 0;
            while (kk >= kSuper - bi) {
                kk -= kSuper - bi;
                ++bi;
            }
            bj = bi + kk;
        }
        const int gi = R * 256 + bi * 32 + 4 * Q, gj = C * 256 + bj * 32 + j;
        if (gj >= a.N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int cnt = (int)((word >> (16 * r)) & 0xffffu);
            if (cnt != 0 && gi + r <= gj) atomicAdd(dst + tri(a.N, gi + r, gj), cnt);
        }
    }
}

// Zero flagged points in place: byte 0x88 is 0 + 0i.  One thread per flag
// word; a word without flags touches nothing else.  When N % 32 == 0 the 32
// bytes of a word are rewritten with two 16-byte accesses.
template <bool kVec>
__global__ void apply_kernel(uint8_t *packed, const uint32_t *flags, int N, int F, int T, int W) {
    const int64_t total = (int64_t)F * T * W;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += stride) {
        uint32_t word = flags[e];
        const int w = (int)(e % W);
        const int64_t ft = e / W;
        const int t = (int)(ft % T), f = (int)(ft / T);
        const int rest = N - w * 32;
        if (rest < 32) word &= (1u << rest) - 1u;
        if (word == 0u) continue;
        uint8_t *row = packed + ((int64_t)t * F + f) * N + w * 32;
        if (kVec) {
            uint4 *p = (uint4 *)row;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                uint4 v = p[half];
                uint32_t *d = (uint32_t *)&v;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t b4 = (word >> (16 * half + 4 * q)) & 15u;
                    uint32_t m = (b4 * 0x00204081u) & 0x01010101u;  // bit k -> byte k
                    m = (m << 8) - m;                                // -> 0xff bytes
                    d[q] = (d[q] & ~m) | (0x88888888u & m);
                }
                p[half] = v;
            }
        } else {
            for (int b = 0; b < 32; ++b)
                if ((word >> b) & 1u) row[b] = 0x88;
        }
    }
}

// out[f][p] = vis / n_ij, n_ij = count_f - d_ii - d_jj + d_ij, in double
// rounded once to float, 0 where n_ij == 0; n_out (optional) = n_ij.  One
// thread per baseline; (i, j) from p by inverting the row starts
// s(i) = i N - i (i - 1) / 2.
__global__ void normalize_kernel(const int32_t *vis, const int64_t *count, const int32_t *d,
                                 float *out, int32_t *n_out, int N, int F) {
    const int64_t P = (int64_t)N * (N + 1) / 2;
    const int64_t total = P * F;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t f = e / P, p = e % P;
        const double b = 2.0 * N + 1.0;
        int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)p)) * 0.5);
        if (i < 0) i = 0;
        if (i > N - 1) i = N - 1;
        while (i > 0 && tri(N, i, i) > p) --i;
        while (i + 1 < N && tri(N, i + 1, i + 1) <= p) ++i;
        const int64_t j = i + (p - tri(N, i, i));
        const int32_t *df = d + f * P;
        const int64_t n = count[f] - (int64_t)df[tri(N, i, i)] - (int64_t)df[tri(N, j, j)] +
                          (int64_t)df[p];
        const int2 v = *(const int2 *)(vis + 2 * e);
        float2 o;
        o.x = n == 0 ? 0.0f : (float)((double)v.x / (double)n);
        o.y = n == 0 ? 0.0f : (float)((double)v.y / (double)n);
        *(float2 *)(out + 2 * e) = o;
        if (n_out) n_out[e] = (int32_t)n;
    }
}

}  // namespace flag
}  // namespace xe
