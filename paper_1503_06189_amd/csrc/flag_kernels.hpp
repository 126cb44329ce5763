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
// 256-input super blocks (R <= C) and one chunk of time, in stages of 256
// samples:
//   1. the words of both super blocks are loaded two stages ahead (0 for
//      lost samples, samples past the chunk and inputs past N) and stored in
//      LDS with one "any flag" bit per (32-input block, 32-sample step),
//      gathered by wave ballots;
//   2. every (block, step) with a flag is turned, by one wave, from 32 x 32
//      bits into the operand of v_mfma_i32_32x32x32_i8 (lane l: input l % 32,
//      16 samples of half l / 32 as 0/1 bytes) by byte selection and a shift;
//   3. each wave runs its tiles and skips a (tile, step) when either block
//      has no flag there: the counterpart of the method's test of whole
//      32-bit words before extracting bits.
// A stage without any flag costs only its loads.  Tiles hold exact int32
// counts; the time chunks of one tile are summed into d with integer
// atomics, so their order does not matter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace xe {
namespace flag {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kThreads = 512;            // 8 waves, two per SIMD
constexpr int kWaves = kThreads / 64;
constexpr int kSuper = 8;                // 32-input blocks per super block
constexpr int kSteps = 8;                // 32-sample steps per stage
constexpr int kStage = kSteps * 32;      // samples per stage
constexpr int kPitch = kStage + 4;       // LDS words per block row (16-B aligned rows)
constexpr int kLoads = kStage * kSuper / kThreads;  // flag words per thread, stage and side

struct Args {
    const uint32_t *flags;   // [F][T][W]
    const uint8_t *mask;     // [F][nblk], may be null
    int32_t *d;              // [F][P]
    int N, F, T, B, W, nblk;
    int ns;                  // super blocks, ceil(N / 256)
    int chunks;              // time chunks per (channel, pair)
    int chunk_samples;       // samples per chunk, a multiple of kStage
    uint64_t b_magic;        // ceil(2^40 / B) when B <= 2^16, else 0
};

// t / B for 0 <= t < 2^24: (t * ceil(2^40 / B)) >> 40 is exact when B <= 2^16
// (the rounding adds less than 2^-16 to t / B, whose fraction is at most
// 1 - 1/B); larger B divides.
__device__ __forceinline__ int block_of(const Args &a, int t) {
    return a.b_magic ? (int)(((uint64_t)(uint32_t)t * a.b_magic) >> 40) : t / a.B;
}

// wave roles: in a diagonal pair (R == C) waves 0-3 take row block w against
// column blocks 4..7 (kRect), waves 4/6 and 5/7 split the two 4-block
// triangles (kTriA, kTriB); in an off-diagonal pair wave w takes row blocks
// 2 (w % 4) + {0, 1} against column blocks 4 (w / 4) + {0..3} (kOff).
// Waves w and w + 4 share a SIMD and together hold 9 (diagonal) or 16 tiles.
enum { kRect = 0, kTriA = 1, kTriB = 2, kOff = 3 };

template <int ROLE>
struct Role {
    // operands held per step: NR row blocks (side 0), NC column blocks
    static constexpr int NR = ROLE == kRect ? 1 : ROLE == kOff ? 2 : 4;
    static constexpr int NC = ROLE == kRect ? 4 : ROLE == kOff ? 4 : 0;  // 0: columns = rows
    static constexpr int NT = ROLE == kRect ? 4 : ROLE == kOff ? 8 : 5;
    // tile k = (row operand r, column operand c)
    __device__ static constexpr int r(int k) {
        return ROLE == kRect ? 0
             : ROLE == kOff  ? k / 4
             : ROLE == kTriA ? (k < 4 ? 0 : 1)
                             : (k < 2 ? 1 : k < 4 ? 2 : 3);
    }
    __device__ static constexpr int c(int k) {
        return ROLE == kRect ? k
             : ROLE == kOff  ? k % 4
             : ROLE == kTriA ? (k < 4 ? k : 1)
                             : (k == 0 ? 2 : k == 1 ? 3 : k == 2 ? 2 : 3);
    }
};

// SIDES = 1 for a diagonal pair (rows and columns are the same 256 inputs)
template <int SIDES>
struct Lds {
    uint32_t words[SIDES][kSuper][kPitch];      // [side][block][sample]
    v4i ops[SIDES][kSuper][kSteps][64];         // [side][block][step][lane]
    uint64_t any[2][SIDES][kWaves];             // [stage % 2][side][wave]: bit 8 b + s
};

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

__device__ __forceinline__ v16i mfma(v4i a, v4i b, v16i c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// bit k of an 8-bit value -> bit 8 k
__device__ __forceinline__ uint64_t spread8(uint64_t x) {
    x = (x | (x << 28)) & 0x0000000F0000000Full;
    x = (x | (x << 14)) & 0x0003000300030003ull;
    x = (x | (x << 7)) & 0x0101010101010101ull;
    return x;
}

// Operand of (side, block b, step s) for this lane: byte q of the 16 is the
// flag of input l % 32 at sample 32 s + 16 (l / 32) + q.  Each group of 4
// words gives one dword: byte (i / 8) of each word is gathered with two
// byte permutes, then bit (i % 8) of every byte is shifted down and masked.
template <int SIDES>
__device__ __forceinline__ void build_op(Lds<SIDES> &L, int side, int b, int s, int lane) {
    const int i = lane & 31, h = lane >> 5;
    const uint32_t bi = (uint32_t)(i >> 3), bb = (uint32_t)(i & 7);
    const uint32_t sel_lo = 0x0c0c0000u | ((4u + bi) << 8) | bi;
    const uint32_t sel_hi = ((4u + bi) << 24) | (bi << 16) | 0x0c0cu;
    const v4i *src = (const v4i *)&L.words[side][b][s * 32 + h * 16];
    v4i out;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        v4i w = src[d];
        uint32_t x = perm((uint32_t)w.y, (uint32_t)w.x, sel_lo) |
                     perm((uint32_t)w.w, (uint32_t)w.z, sel_hi);
        out[d] = (int)((x >> bb) & 0x01010101u);
    }
    L.ops[side][b][s][lane] = out;
}

__device__ __forceinline__ int64_t tri(int64_t N, int64_t i, int64_t j) {
    return i * N - i * (i - 1) / 2 + (j - i);
}

// Flag words of one stage, raw, in registers: element e = tid + 512 r is
// sample e / 8 of the stage, word e % 8 of the super block.  Every load is
// issued unconditionally from a clamped, in-range address and nothing is
// computed from the loaded values until the stage is stored two stages
// later (a load under a divergent branch, or arithmetic on its result, would
// be waited for right away).
// The loss byte of a sample's block is read as the aligned dword holding
// it (the same page as the byte, so always mapped) and picked out at store
// time.
template <int SIDES>
struct StageRegs {
    uint32_t w[SIDES][kLoads];
    uint32_t lost[kLoads];     // dword holding the block's loss byte
};

// byte offset of the loss byte of sample tc of channel f from the 4-aligned
// address just below the mask (0 without a mask)
__device__ __forceinline__ int64_t mask_byte(const Args &a, int f, int tc) {
    if (a.mask == nullptr) return 0;
    const int64_t mis = (int64_t)((uintptr_t)a.mask & 3u);
    return mis + (int64_t)f * a.nblk + block_of(a, tc);
}

template <int SIDES>
__device__ __forceinline__ void load_stage(const Args &a, StageRegs<SIDES> &g, int f, int R,
                                           int C, int t0, int tid) {
    // dwords of the mask, from the 4-aligned address at or below its start
    // (the flags stand in when there is no mask; the value is then unused)
    const uint32_t *mwords =
        a.mask ? (const uint32_t *)(a.mask - ((uintptr_t)a.mask & 3u)) : a.flags;
    const uint32_t *frow = a.flags + (int64_t)f * a.T * a.W;
#pragma unroll
    for (int r = 0; r < kLoads; ++r) {
        const int e = tid + kThreads * r;
        const int tc = min(t0 + (e >> 3), a.T - 1);
        g.lost[r] = mwords[mask_byte(a, f, tc) >> 2];
#pragma unroll
        for (int side = 0; side < SIDES; ++side) {
            const int gw = (side == 0 ? R : C) * kSuper + (e & 7);
            g.w[side][r] = frow[(int64_t)tc * a.W + min(gw, a.W - 1)];
        }
    }
}

// Store a stage's words in LDS (0 for lost samples, samples past the chunk
// and inputs past N) and publish, per wave, which (block, step) hold a flag:
// the 64 lanes of one load cover 8 samples of one step and lane % 8 = block,
// so a ballot folded over its 8 bytes gives the blocks.
template <int SIDES>
__device__ __forceinline__ void store_stage(const Args &a, Lds<SIDES> &L,
                                            const StageRegs<SIDES> &g, int f, int R, int C, int t0,
                                            int t_end, int buf, int wave, int lane, int tid) {
    const bool has_mask = a.mask != nullptr;
#pragma unroll
    for (int side = 0; side < SIDES; ++side) {
        uint64_t any = 0;
#pragma unroll
        for (int r = 0; r < kLoads; ++r) {
            const int e = tid + kThreads * r;
            const int gw = (side == 0 ? R : C) * kSuper + (e & 7);
            const int rest = a.N - gw * 32;
            const uint32_t pad = rest >= 32 ? 0xffffffffu : rest > 0 ? (1u << rest) - 1u : 0u;
            const int t = t0 + (e >> 3);
            const int64_t mb = mask_byte(a, f, min(t, a.T - 1));
            const uint32_t lost = (g.lost[r] >> (8 * (int)(mb & 3))) & 0xffu;
            // branch-free: 0 past the chunk or in a lost block
            const uint32_t keep = (uint32_t)(t < t_end) & (uint32_t)(!has_mask | (lost == 0u));
            const uint32_t v = g.w[side][r] & pad & (0u - keep);
            L.words[side][e & 7][e >> 3] = v;
            uint64_t m = __ballot(v != 0u);
            m |= m >> 32;
            m |= m >> 16;
            m |= m >> 8;
            const int step = (wave + kWaves * r) >> 2;
            any |= spread8(m & 0xffu) << step;
        }
        if (lane == 0) L.any[buf][side][wave] = any;
    }
}

template <int ROLE, int SIDES>
__device__ __forceinline__ void run_role(const Args &a, Lds<SIDES> &L, int f, int R, int C,
                                         int t_begin, int t_end, int wave, int lane, int tid) {
    using RL = Role<ROLE>;
    constexpr int sc = SIDES - 1;              // side of the column blocks
    const int rb0 = ROLE == kRect ? wave : ROLE == kOff ? 2 * (wave & 3)
                  : ROLE == kTriA ? (wave == 4 ? 0 : 4) : (wave == 5 ? 0 : 4);
    const int cb0 = ROLE == kRect ? 4 : ROLE == kOff ? 4 * (wave >> 2) : rb0;

    v16i acc[RL::NT];
    bool touched[RL::NT];
#pragma unroll
    for (int k = 0; k < RL::NT; ++k) {
        acc[k] = v16i{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        touched[k] = false;
    }

    const int nst = (t_end - t_begin + kStage - 1) / kStage;
    StageRegs<SIDES> g[2];
    // Stage st's words sit in g[st % 2] from two stages ahead until stored.
    // Loads and stores run for every stage, also past the chunk's end (in
    // range, read as 0): the same number of loads on every path lets each
    // store wait for its own loads only.
    load_stage(a, g[0], f, R, C, t_begin, tid);
    load_stage(a, g[1], f, R, C, t_begin + kStage, tid);
    store_stage(a, L, g[0], f, R, C, t_begin, t_end, 0, wave, lane, tid);
    load_stage(a, g[0], f, R, C, t_begin + 2 * kStage, tid);

    auto stage = [&](int st, auto parity) {
        constexpr int P = decltype(parity)::value;
        __syncthreads();  // words and flag bits of stage st visible
        uint64_t any0 = 0, any1 = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) any0 |= L.any[P][0][w];
        if (SIDES == 2) {
#pragma unroll
            for (int w = 0; w < kWaves; ++w) any1 |= L.any[P][sc][w];
        } else {
            any1 = any0;
        }
        any0 = __builtin_amdgcn_readfirstlane((uint32_t)any0) |
               ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(any0 >> 32)) << 32);
        any1 = __builtin_amdgcn_readfirstlane((uint32_t)any1) |
               ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(any1 >> 32)) << 32);
        const bool work = any0 != 0 && any1 != 0;
        if (work) {
            // operand builds: item q = 8 b + s, wave w takes q = w mod 8
#pragma unroll
            for (int side = 0; side < SIDES; ++side) {
                const uint64_t bits = side == 0 ? any0 : any1;
#pragma unroll
                for (int m = 0; m < kSuper; ++m) {
                    const int q = wave + kWaves * m;
                    if ((bits >> q) & 1u) build_op(L, side, q >> 3, q & 7, lane);
                }
            }
            __syncthreads();  // operands visible
        }
        // this stage's words are done: store the next stage, load the one after
        store_stage(a, L, g[1 - P], f, R, C, t_begin + (st + 1) * kStage, t_end, 1 - P, wave,
                    lane, tid);
        load_stage(a, g[1 - P], f, R, C, t_begin + (st + 3) * kStage, tid);
        if (work) {
            // one step at a time keeps the operands of later steps out of
            // registers (the 8-tile role holds 128 accumulators)
#pragma unroll 1
            for (int s = 0; s < kSteps; ++s) {
                v4i ro[RL::NR];
                v4i co[RL::NC > 0 ? RL::NC : 1];
#pragma unroll
                for (int r = 0; r < RL::NR; ++r)
                    if ((any0 >> ((rb0 + r) * 8 + s)) & 1u) ro[r] = L.ops[0][rb0 + r][s][lane];
#pragma unroll
                for (int c = 0; c < RL::NC; ++c)
                    if ((any1 >> ((cb0 + c) * 8 + s)) & 1u) co[c] = L.ops[sc][cb0 + c][s][lane];
#pragma unroll
                for (int k = 0; k < RL::NT; ++k) {
                    const int rbk = rb0 + RL::r(k), cbk = cb0 + RL::c(k);
                    if (((any0 >> (rbk * 8 + s)) & (any1 >> (cbk * 8 + s)) & 1u) != 0u) {
                        const v4i &bop = RL::NC > 0 ? co[RL::c(k) < RL::NC ? RL::c(k) : 0]
                                                    : ro[RL::c(k)];
                        acc[k] = mfma(ro[RL::r(k)], bop, acc[k]);
                        touched[k] = true;
                    }
                }
            }
        }
    };
    for (int st = 0; st < nst; st += 2) {
        stage(st, std::integral_constant<int, 0>{});
        if (st + 1 < nst) stage(st + 1, std::integral_constant<int, 1>{});
    }

    // add the counts into d: element v of a tile sits at
    // (8 (v / 4) + 4 (lane / 32) + v % 4, lane % 32)
    const int64_t P = (int64_t)a.N * (a.N + 1) / 2;
    int32_t *dst = a.d + (int64_t)f * P;
#pragma unroll
    for (int k = 0; k < RL::NT; ++k) {
        if (!touched[k]) continue;
        const int gi0 = R * 256 + (rb0 + RL::r(k)) * 32 + 4 * (lane >> 5);
        const int gj = C * 256 + (cb0 + RL::c(k)) * 32 + (lane & 31);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int gi = gi0 + 8 * (v >> 2) + (v & 3);
            const int val = acc[k][v];
            if (val != 0 && gi < a.N && gj < a.N && gi <= gj)
                atomicAdd(dst + tri(a.N, gi, gj), val);
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

// One launch per pair kind, so each kernel is register-allocated for its own
// roles: kOffPairs = false runs the ns diagonal pairs (R == C) of every
// channel, true the ns (ns - 1) / 2 off-diagonal pairs (R < C).
template <bool kOffPairs>
__global__ __launch_bounds__(kThreads, 1) void gram_kernel(Args a) {
    constexpr int SIDES = kOffPairs ? 2 : 1;
    __shared__ Lds<SIDES> L;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int pairs = kOffPairs ? a.ns * (a.ns - 1) / 2 : a.ns;
    const int64_t total = (int64_t)a.F * pairs * a.chunks;
    const int64_t w = xcd_local(blockIdx.x, total);
    const int chunk = (int)(w % a.chunks);
    const int64_t rest = w / a.chunks;
    const int g = (int)(rest % pairs);
    const int f = __builtin_amdgcn_readfirstlane((int)(rest / pairs));
    int R = g, C = g;
    if (kOffPairs) {
        // g -> (R, C), R < C, row-major over the strict upper triangle
        int rem = g;
        R = 0;
        while (rem >= a.ns - 1 - R) {
            rem -= a.ns - 1 - R;
            ++R;
        }
        C = R + 1 + rem;
    }
    // wave-uniform bounds keep the stage loop's branches scalar
    const int t_begin = __builtin_amdgcn_readfirstlane(chunk * a.chunk_samples);
    const int t_end = __builtin_amdgcn_readfirstlane(min(a.T, t_begin + a.chunk_samples));
    R = __builtin_amdgcn_readfirstlane(R);
    C = __builtin_amdgcn_readfirstlane(C);

    if (kOffPairs) {
        run_role<kOff>(a, L, f, R, C, t_begin, t_end, wave, lane, tid);
    } else if (wave < 4) {
        run_role<kRect>(a, L, f, R, C, t_begin, t_end, wave, lane, tid);
    } else if ((wave & 1) == 0) {
        run_role<kTriA>(a, L, f, R, C, t_begin, t_end, wave, lane, tid);
    } else {
        run_role<kTriB>(a, L, f, R, C, t_begin, t_end, wave, lane, tid);
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
