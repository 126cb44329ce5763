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
//   1. the words of both super blocks are loaded a few stages ahead (0 for
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
constexpr int kWindow = 1024;            // validity words per chunk: chunks <= 32768 samples

struct Args {
    const uint32_t *flags;   // [F][T][W]
    const uint8_t *mask;     // [F][nblk], may be null
    int32_t *d;              // [F][P]
    int N, F, T, B, W, nblk;
    int ns;                  // super blocks, ceil(N / 256)
    int chunks;              // time chunks per (channel, pair)
    int chunk_samples;       // samples per chunk, a multiple of kStage, <= 32 kWindow
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
    uint32_t valid[kWindow];                    // bit k of word s: sample 32 s + k of the chunk
};

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

__device__ __forceinline__ v16i mfma(v4i a, v4i b, v16i c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
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

// Validity of the chunk's samples, one bit each, in LDS: 1 inside the chunk
// and outside lost blocks.  All threads take part; a barrier must follow.
template <int SIDES>
__device__ __forceinline__ void fill_window(const Args &a, Lds<SIDES> &L, int f, int t_begin,
                                            int t_end, int tid) {
    const int words = (t_end - t_begin + 31) >> 5;
    for (int s = tid; s < words; s += kThreads) {
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

// Flag words of one stage, raw, in registers.  Thread tid owns sample
// tid / 2 of the stage and words 4 (tid % 2) .. +3 of each super block, so
// wave w covers step w.  The words are read through a buffer resource whose
// range ends at the chunk's last sample: loads past it return 0 without a
// memory access, so every load is issued unconditionally, and nothing is
// computed from the loaded values until the stage is stored D stages later
// (arithmetic on a load's result would be waited for right away).
template <int SIDES>
struct StageRegs {
    uint32_t w[SIDES][4];
};

// per-thread constants of the stage loop
template <int SIDES>
struct Lane {
    __amdgpu_buffer_rsrc_t rsrc;   // the chunk's rows of this channel's flags
    uint32_t row_bytes;            // 4 W
    uint32_t off[SIDES][4];        // byte offset of each word in a row (word clamped to W - 1)
    uint32_t pad[SIDES][4];        // bits of inputs < N
    int smp;                       // sample within the stage
    int k0;                        // first of the thread's 4 block rows
};

template <int SIDES>
__device__ __forceinline__ Lane<SIDES> make_lane(const Args &a, int f, int R, int C,
                                                 int t_begin, int t_end, int tid) {
    Lane<SIDES> l;
    l.smp = tid >> 1;
    l.k0 = 4 * (tid & 1);
    l.row_bytes = 4u * (uint32_t)a.W;
#pragma unroll
    for (int side = 0; side < SIDES; ++side)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gw = (side == 0 ? R : C) * kSuper + l.k0 + r;
            const int rest = a.N - gw * 32;
            l.off[side][r] = 4u * (uint32_t)min(gw, a.W - 1);
            l.pad[side][r] = rest >= 32 ? 0xffffffffu : rest > 0 ? (1u << rest) - 1u : 0u;
        }
    // wave-uniform; readfirstlane keeps the resource in scalar registers
    const uint64_t base = (uint64_t)(uintptr_t)(a.flags + ((int64_t)f * a.T + t_begin) * a.W);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    const uint32_t extent =
        __builtin_amdgcn_readfirstlane((uint32_t)(t_end - t_begin) * l.row_bytes);
    void *p = (void *)(uintptr_t)(((uint64_t)hi << 32) | lo);
    l.rsrc = __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)extent, 0x00020000);
    return l;
}

// stage starting ts samples into the chunk; offsets stay below 2^31 (a chunk
// holds at most 32768 samples of at most 512 bytes)
template <int SIDES>
__device__ __forceinline__ void load_stage(const Lane<SIDES> &l, StageRegs<SIDES> &g, int ts) {
    const uint32_t row = (uint32_t)(ts + l.smp) * l.row_bytes;
#pragma unroll
    for (int side = 0; side < SIDES; ++side)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            g.w[side][r] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(
                l.rsrc, (int)(row + l.off[side][r]), 0, 0);
}

// Store a stage's words in LDS (0 for lost samples, samples past the chunk
// and inputs past N) and publish, per wave, which (block, step) hold a flag:
// a wave's 64 lanes are the 32 samples of one step, even lanes holding block
// rows r and odd lanes rows 4 + r, so two masks of a ballot give the bits.
template <int SIDES>
__device__ __forceinline__ void store_stage(Lds<SIDES> &L, const Lane<SIDES> &l,
                                            const StageRegs<SIDES> &g, int ts, int buf,
                                            int wave, int lane) {
    const int t = ts + l.smp;   // sample within the chunk
    const uint32_t wv = t < 32 * kWindow ? L.valid[t >> 5] : 0u;
    const uint32_t keep = 0u - ((wv >> (t & 31)) & 1u);
#pragma unroll
    for (int side = 0; side < SIDES; ++side) {
        uint64_t any = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t v = g.w[side][r] & l.pad[side][r] & keep;
            L.words[side][l.k0 + r][l.smp] = v;
            const uint64_t m = __ballot(v != 0u);
            any |= (uint64_t)((m & 0x5555555555555555ull) != 0) << (r * 8 + wave);
            any |= (uint64_t)((m & 0xAAAAAAAAAAAAAAAAull) != 0) << ((4 + r) * 8 + wave);
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
    const Lane<SIDES> ln = make_lane<SIDES>(a, f, R, C, t_begin, t_end, tid);
    fill_window(a, L, f, t_begin, t_end, tid);
    // Stage j's words sit in g[j % D] from D stages ahead until stored (D =
    // 4 for a diagonal pair, two of which share a CU; 2 for the
    // register-heavy off-diagonal roles).
    // Loads and stores run for every stage, also past the chunk's end (out
    // of the buffer's range: 0, no memory access), so that every path issues
    // the same loads and each store waits for its own loads only.
    constexpr int D = SIDES == 1 ? 4 : 2;
    StageRegs<SIDES> g[D];
#pragma unroll
    for (int j = 0; j < D; ++j) load_stage(ln, g[j], j * kStage);
    __syncthreads();  // validity window visible
    store_stage(L, ln, g[0], 0, 0, wave, lane);
    load_stage(ln, g[0], D * kStage);

    auto stage = [&](int st, auto slot) {
        constexpr int J = decltype(slot)::value;        // st % D
        constexpr int P = J % 2;                        // st % 2 (D is even)
        constexpr int JN = (J + 1) % D;                 // (st + 1) % D
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
            // operand builds: wave w builds step w of all 8 blocks, every
            // block when the step holds any flag (reads issued together, no
            // wait per item); slots of flag-free blocks are never read below
            constexpr uint64_t kCol = 0x0101010101010101ull;
#pragma unroll
            for (int side = 0; side < SIDES; ++side) {
                const uint64_t bits = side == 0 ? any0 : any1;
                if (((bits >> wave) & kCol) != 0) {
#pragma unroll
                    for (int b = 0; b < kSuper; ++b) build_op(L, side, b, wave, lane);
                }
            }
            __syncthreads();  // operands visible
        }
        // this stage's words are done: store the next stage, load the one after
        store_stage(L, ln, g[JN], (st + 1) * kStage, 1 - P, wave, lane);
        load_stage(ln, g[JN], (st + 1 + D) * kStage);
        if (work) {
            // one step at a time keeps the operands of later steps out of
            // registers (the 8-tile role holds 128 accumulators); a step
            // without flags on either side is skipped, otherwise all its
            // operands are read at once and only the MFMAs are conditional
            constexpr uint64_t kCol = 0x0101010101010101ull;
#pragma unroll 1
            for (int s = 0; s < kSteps; ++s) {
                if (((any0 >> s) & kCol) == 0 || ((any1 >> s) & kCol) == 0) continue;
                v4i ro[RL::NR];
                v4i co[RL::NC > 0 ? RL::NC : 1];
#pragma unroll
                for (int r = 0; r < RL::NR; ++r) ro[r] = L.ops[0][rb0 + r][s][lane];
#pragma unroll
                for (int c = 0; c < RL::NC; ++c) co[c] = L.ops[sc][cb0 + c][s][lane];
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
    static_assert(D % 2 == 0 && D <= 6, "ring depth");
    for (int st = 0; st < nst; st += D) {
        stage(st, std::integral_constant<int, 0>{});
        if (st + 1 < nst) stage(st + 1, std::integral_constant<int, 1>{});
        if constexpr (D > 2) {
            if (st + 2 < nst) stage(st + 2, std::integral_constant<int, 2 % D>{});
            if (st + 3 < nst) stage(st + 3, std::integral_constant<int, 3 % D>{});
        }
        if constexpr (D > 4) {
            if (st + 4 < nst) stage(st + 4, std::integral_constant<int, 4 % D>{});
            if (st + 5 < nst) stage(st + 5, std::integral_constant<int, 5 % D>{});
        }
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
// channel, true the ns (ns - 1) / 2 off-diagonal pairs (R < C).  Diagonal
// pairs are built for two workgroups per CU (4 waves per SIMD, 128 VGPRs,
// 76 KB of LDS each), so one's barriers and loads overlap the other's work.
template <bool kOffPairs>
__global__ __launch_bounds__(kThreads, kOffPairs ? 1 : 4) void gram_kernel(Args a) {
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
