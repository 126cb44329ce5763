// xcorr_kernels.hpp -- gfx950 kernels of the correlator.
//
// Correlation (Sec. II-B: cross-correlate every input pair of a channel and
// add into the previous output):
//   x = a + i b.  With the real K-vector of one input laid out as the pairs
//   (a_t, b_t) and the derived vector (b_t, -a_t),
//     Re V_ij = sum_k Xr_i[k] Xr_j[k]      Im V_ij = sum_k Xp_i[k] Xr_j[k]
//   with Xr = (a, b), Xp = (b, -a): two real int8 GEMMs with K = 2T on the
//   matrix cores, exact int32 accumulation.  Only tiles with I <= J run.
//   A diagonal tile (I = J) is Hermitian, so it runs one GEMM:
//     Q = Xs Xr^T with Xs = Xr + Xp = (a + b, b - a)  (fits int8),
//     Re = (Q + Q^T) / 2,  Im = (Q - Q^T) / 2  (exact: Q + Q^T = 2 Re).
//
// A workgroup integrates one tile group (plan.hpp) of one channel over one
// chunk of time.  Per staged step of 32 samples it
//   1. loads the packed bytes of its input blocks with dword buffer loads
//      along the input axis (the buffer range ends at the chunk), kDepth
//      steps ahead, into a ring of register sets;
//   2. substitutes 0x88 (= 0) for lost samples, samples past the chunk and
//      inputs past N, transposes 4x4 byte blocks in registers so that each
//      dword holds 4 samples of one input, decodes nibbles to signed int8
//      with carry-free byte arithmetic and writes LDS in the operand layout
//      of v_mfma_i32_32x32x32_i8: per block and 16-sample sub-step, lane l
//      reads 16 bytes = 8 samples of input l % 32.  Both operands use the
//      same K order, so the order of samples inside K does not change the
//      sum;
//   3. runs its tiles: A operand (rows) in Xr, Xp (and Xs) form, B Xr.
// The loop is software-pipelined over three LDS buffers: the decode of step
// s+2 and the operand reads of step s+1 overlap the MFMAs of step s; one
// barrier per step; eight waves, two per SIMD, so that one wave's decode
// and waits overlap the other's MFMAs.
//
// Output: chunk 0 of a tile group (or its only chunk) writes its tiles with
// plain stores (overwrite) or read-add-write (accumulate).  Chunks 1.. store
// their int32 tiles in the workspace, and merge_kernel, launched next on
// the same stream, adds them into the output.  Integer sums, so the order of
// chunks does not matter and the result is exact.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.hpp"

namespace xe {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef int v2i __attribute__((ext_vector_type(2)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));

constexpr int kFragBytes = kBlk * kStep * 2;  // one decoded operand of a block per step
// A diagonal group stages Xr and Xs per block (8 slots x 2 operands), an
// off-diagonal half stages Xr only (12 slots)
constexpr int kBufBytes = 16 * kFragBytes;
// validity bits of a window of steps, one 32-bit word per step
constexpr int kMaskWindow = 2048;
// int32 (Re, Im) tiles of one wave in the workspace: 10 tiles x 32 x 64
constexpr int kWavePartial = kTilesPerWave * 32 * 64;
constexpr int64_t kGroupPartial = (int64_t)kWaves * kWavePartial;

struct CorrArgs {
    const uint8_t *packed;
    const uint8_t *mask;  // may be null
    int32_t *vis;
    int64_t *count;
    int32_t *partials;    // [F*groups][splits-1][kGroupPartial] when splits > 1
    int N, F, T, B;
    int nblk_mask;        // ceil(T / B)
    int nb;               // ceil(N / 32)
    int groups;           // groups per channel
    int splits;
    int steps_per_split;
    int halves;           // the halves geometry when N <= 128
};

// ---------------------------------------------------------------------------
// byte tricks (all carry-free per byte)
// ---------------------------------------------------------------------------

// nibble u in 0..15 per byte -> u - 8 as int8: (u + 0x78) ^ 0x80
__device__ __forceinline__ uint32_t nib_to_s8(uint32_t u) {
    return (u + 0x78787878u) ^ 0x80808080u;
}

// -x per byte for x in [-8, 7]: ((x ^ 0x7f) + 1) ^ 0x80, no byte overflows
__device__ __forceinline__ uint32_t neg_s8(uint32_t x) {
    return ((x ^ 0x7f7f7f7fu) + 0x01010101u) ^ 0x80808080u;
}

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// 4x4 byte transpose: d[e] holds inputs 0..3 of sample e; out[c] holds
// samples 0..3 of input c
__device__ __forceinline__ void transpose4(const uint32_t d[4], uint32_t out[4]) {
    uint32_t e0 = perm(d[1], d[0], 0x05010400u);  // d00 d10 d01 d11
    uint32_t e1 = perm(d[1], d[0], 0x07030602u);  // d02 d12 d03 d13
    uint32_t e2 = perm(d[3], d[2], 0x05010400u);  // d20 d30 d21 d31
    uint32_t e3 = perm(d[3], d[2], 0x07030602u);  // d22 d32 d23 d33
    out[0] = perm(e2, e0, 0x05040100u);
    out[1] = perm(e2, e0, 0x07060302u);
    out[2] = perm(e3, e1, 0x05040100u);
    out[3] = perm(e3, e1, 0x07060302u);
}

// 4 validity bits -> 4 byte masks (0xff = valid)
__device__ __forceinline__ uint32_t bits_to_bytes(uint32_t b4) {
    uint32_t m = (b4 * 0x00204081u) & 0x01010101u;  // bit k -> byte k
    return (m << 8) - m;
}

// A 16-byte operand chunk holds, for 8 samples of one input,
// (a0..3 | b0..3 | a4..7 | b4..7).  Xr chunk -> Xp chunk (b | -a).
__device__ __forceinline__ v4i make_xp(v4i x) {
    v4i p;
    p.x = x.y;
    p.y = (int)neg_s8((uint32_t)x.x);
    p.z = x.w;
    p.w = (int)neg_s8((uint32_t)x.z);
    return p;
}

__device__ __forceinline__ v16i mfma(v4i a, v4i b, v16i c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// LDS position of the 16-byte chunk c (= lane-group g * 32 + row r) of
// (block slot s, operand op, sub-step u).  The 64 chunks of one (s, op, u)
// form 1 KB; lane l of a reading wave takes chunk l, stored at
//   phys(l, s) = l ^ (s & 1) ^ (bit 4 of l) << 1,
// a permutation inside aligned groups of 4 chunks, so a wave's 16-byte
// reads stay conflict-free while the stagers' 8-byte writes (below) hit all
// 64 banks exactly once per half-wave.
__device__ __forceinline__ int phys_chunk(int c, int s) {
    return c ^ (s & 1) ^ (((c >> 4) & 1) << 1);
}
__device__ __forceinline__ int chunk_off(int slot_bytes, int s, int op, int u, int c) {
    return s * slot_bytes + op * kFragBytes + u * 1024 + (phys_chunk(c, s) << 4);
}

// ---------------------------------------------------------------------------
// staging: global packed bytes -> decoded int8 operand layout in LDS
// ---------------------------------------------------------------------------

// One staging unit = 4 inputs (n0..n0+3) x 4 samples (sample quad sq of the
// step) of block slot s.  Units come in rounds of 64 per wave: lane bits
// (q = lane & 7, s_lo = bit 3, h = bit 4, s_hi = bit 5) give input quad q,
// slot 4 sg + s_lo + 2 s_hi and sample quad 2 o + h, with the octet o and
// the slot group sg fixed per wave-round.  Coordinates do not change along
// the time loop.
struct Unit {
    int s, q, sq;
    uint32_t voff;  // byte offset of (sample 4 sq, input n0) within the chunk;
                    // out of range (reads 0) when the inputs lie past N
    bool act;       // inputs lie below N (else staged as 0)
    bool hi;        // halves geometry, slots 4..7: the odd step of the pair
    uint32_t inb;   // unaligned path: byte c of the dword lies below N
};

template <int UPT>
struct Prefetch {
    uint32_t d[UPT][4];
};

// The chunk of a workgroup: samples [t_begin, t_end) of channel f, read
// through a buffer resource whose range ends at the last byte of the chunk,
// so every load is bounds-checked by the hardware (reads past it return 0;
// such samples are replaced below anyway).
struct Chunk {
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t row_bytes;  // F * N: bytes between consecutive samples
    int t_begin, t_end;
};

__device__ __forceinline__ Chunk make_chunk(const CorrArgs &a, int f, int t_begin, int t_end) {
    Chunk c;
    // every value here is wave-uniform; readfirstlane keeps the resource in
    // scalar registers (a buffer load needs it there)
    uint64_t base = (uint64_t)(uintptr_t)(a.packed + ((int64_t)t_begin * a.F + f) * a.N);
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    uint32_t row = __builtin_amdgcn_readfirstlane((uint32_t)a.F * (uint32_t)a.N);
    uint32_t extent = __builtin_amdgcn_readfirstlane((uint32_t)(t_end - t_begin - 1) * row +
                                                     (uint32_t)a.N);
    void *p = (void *)(uintptr_t)(((uint64_t)hi << 32) | lo);
    c.rsrc = __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)extent, 0x00020000);
    c.row_bytes = row;
    c.t_begin = t_begin;
    c.t_end = t_end;
    return c;
}

// The whole byte offset goes into the vector offset, which the hardware
// checks against the resource's range (loads past the chunk read 0); the
// scalar offset stays 0.  Offsets stay below 2^31 (the host bounds a
// chunk, its lookahead included), so an inactive unit's 0x80000000 stays
// out of range.
template <bool kAligned, int UPT>
__device__ __forceinline__ void issue_loads(const Chunk &ch, int tb, const Unit (&u)[UPT],
                                            Prefetch<UPT> &p) {
    const uint32_t step_off = (uint32_t)(tb - ch.t_begin) * ch.row_bytes;
#pragma unroll
    for (int r = 0; r < UPT; ++r) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t off = u[r].voff + step_off + (uint32_t)e * ch.row_bytes;
            if (kAligned) {
                p.d[r][e] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(ch.rsrc, (int)off, 0, 0);
            } else {
                uint32_t v = 0;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    uint32_t b = (uint8_t)__builtin_amdgcn_raw_buffer_load_b8(
                        ch.rsrc, (int)(off + c), 0, 0);
                    v |= (((u[r].inb >> c) & 1u) ? b : 0x88u) << (8 * c);
                }
                p.d[r][e] = v;
            }
        }
    }
}

// Validity words of steps [s0, s0 + kMaskWindow) of the chunk into LDS: bit k
// of word s = sample t_begin + 32 s + k lies inside the chunk and not in a
// lost block.  All threads take part; call between barriers.
__device__ inline void fill_mask_window(const CorrArgs &a, int f, const Chunk &ch, int s0,
                                        int nsteps, uint32_t *words) {
    const uint8_t *m = a.mask ? a.mask + (int64_t)f * a.nblk_mask : nullptr;
    const int n = (nsteps - s0) < kMaskWindow ? (nsteps - s0) : kMaskWindow;
    for (int w = threadIdx.x; w < n; w += kThreads) {
        const int tb = ch.t_begin + (s0 + w) * kStep;
        const int left = ch.t_end - tb;
        uint32_t bits = left >= 32 ? 0xffffffffu : ((1u << left) - 1u);
        if (m) {
            int blk = tb / a.B;
            for (int k0 = blk * a.B - tb; k0 < 32 && blk < a.nblk_mask; k0 += a.B, ++blk) {
                if (m[blk]) {
                    int lo = k0 < 0 ? 0 : k0;
                    int hi = k0 + a.B > 32 ? 32 : k0 + a.B;
                    uint32_t range =
                        (hi - lo >= 32) ? 0xffffffffu : (((1u << (hi - lo)) - 1u) << lo);
                    bits &= ~range;
                }
            }
        }
        words[w] = bits;
    }
}

// Decode one prefetched step into LDS (validity words vb0 for its units, vb1
// for the odd-step units of the halves geometry).  Per input, from the
// masked nibbles
// A' = a + 8 and B' = b + 8 (4 samples per dword):
//   Xr = (a | b)             a = (A' + 0x78) ^ 0x80
//   Xs = (a + b | b - a)     a + b = (A' + B' + 0x70) ^ 0x80,
//                            b - a = ((B' | 0x80) - A') ^ 0x80
// all per byte without carries or borrows; Xs only for diagonal groups.
// A unit writes bytes 8h .. 8h+7 of its inputs' chunks (h = sq & 1).
template <bool kXs, bool kSmall, int UPT>
__device__ __forceinline__ void commit(const Unit (&u)[UPT], const Prefetch<UPT> &p,
                                       uint32_t vb0, uint32_t vb1, uint8_t *buf,
                                       int slot_bytes) {
#pragma unroll
    for (int r = 0; r < UPT; ++r) {
        uint32_t L[4];
        transpose4(p.d[r], L);
        const uint32_t vbits = kSmall && u[r].hi ? vb1 : vb0;
        const uint32_t vq = u[r].act ? (vbits >> (4 * u[r].sq)) & 15u : 0u;
        const uint32_t m = bits_to_bytes(vq);
        const int o = u[r].sq >> 1, h = u[r].sq & 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            uint32_t Lm = (L[c] & m) | (0x88888888u & ~m);
            uint32_t an = (Lm >> 4) & 0x0f0f0f0fu, bn = Lm & 0x0f0f0f0fu;
            uint8_t *dst = buf + chunk_off(slot_bytes, u[r].s, 0, o >> 1,
                                           (o & 1) * 32 + 4 * u[r].q + c) + 8 * h;
            v2u xr = {nib_to_s8(an), nib_to_s8(bn)};
            *(v2u *)dst = xr;
            if (kXs) {
                v2u xs = {(an + bn + 0x70707070u) ^ 0x80808080u,
                          ((bn | 0x80808080u) - an) ^ 0x80808080u};
                *(v2u *)(dst + kFragBytes) = xs;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// the tiles of one wave
// ---------------------------------------------------------------------------

// Three tile shapes (see plan.hpp), 16 MFMAs per 32-sample step each:
//   kRect: row block s0 x column blocks c0 .. c0+3 (4 off-diagonal tiles);
//   kTriA: of the 4 blocks s0 .. s0+3, the diagonal tiles of blocks 0 and 1
//          (as Q) and the pairs (0,1) (0,2) (0,3);
//   kTriB: the diagonal tiles of blocks 2 and 3 and the pairs (1,2) (1,3)
//          (2,3).
enum Shape { kRect = 0, kTriA = 1, kTriB = 2 };

template <int SHAPE>
struct Tiles;

template <>
struct Tiles<kRect> {
    static constexpr int NQ = 0, NO = 4, NT = 4, NXP = 1;
    __device__ static constexpr int qb(int) { return 0; }
    __device__ static constexpr int row(int) { return 0; }
    __device__ static constexpr int col(int t) { return t; }
    __device__ static constexpr int xpi(int) { return 0; }  // Xp index of a row
};

template <>
struct Tiles<kTriA> {
    static constexpr int NQ = 2, NO = 3, NT = 5, NXP = 1;
    __device__ static constexpr int qb(int k) { return k; }
    __device__ static constexpr int row(int) { return 0; }
    __device__ static constexpr int col(int t) { return t + 1; }
    __device__ static constexpr int xpi(int) { return 0; }
};

template <>
struct Tiles<kTriB> {
    static constexpr int NQ = 2, NO = 3, NT = 5, NXP = 2;
    __device__ static constexpr int qb(int k) { return 2 + k; }
    __device__ static constexpr int row(int t) { return t < 2 ? 1 : 2; }
    __device__ static constexpr int col(int t) { return t < 2 ? t + 2 : 3; }
    __device__ static constexpr int xpi(int i) { return i - 1; }
};

template <int SHAPE>
struct Acc {
    using T = Tiles<SHAPE>;
    v16i q[T::NQ > 0 ? T::NQ : 1];
    v16i re[T::NO], im[T::NO];
};

// Operand fragments of one 16-sample sub-step.  kRect: x[0] = the row
// block, y[j] = column block c0 + j.  kTriA/B: x[i] = block s0 + i (the
// ones the shape uses), xs[k] = Xs of its k-th diagonal block.
template <int SHAPE>
struct Ops {
    static constexpr bool kTri = SHAPE != kRect;
    v4i x[kTri ? 4 : 1];
    v4i y[kTri ? 1 : 4];
    v4i xs[kTri ? 2 : 1];
};

template <int SHAPE>
__device__ __forceinline__ void read_ops(const uint8_t *buf, int slot_bytes, int s0, int c0,
                                         int sub, Ops<SHAPE> &o) {
    const int lane = threadIdx.x & 63;
    auto frag = [&](int s, int op) {
        return *(const v4i *)(buf + chunk_off(slot_bytes, s, op, sub, lane));
    };
    if (SHAPE == kRect) {
        o.x[0] = frag(s0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) o.y[j] = frag(c0 + j, 0);
    } else {
#pragma unroll
        for (int i = SHAPE == kTriA ? 0 : 1; i < 4; ++i) o.x[i] = frag(s0 + i, 0);
#pragma unroll
        for (int k = 0; k < 2; ++k) o.xs[k] = frag(s0 + Tiles<SHAPE>::qb(k), 1);
    }
}

// One loop step: the 16 MFMAs of step s, with the decode of step s + 2
// woven into them and the operands of the next sub-steps read ahead
// (kMma = false: the decode only, for the rectangle waves of the halves
// geometry, whose tiles would pair different time steps).
//   * (s, sub 0) operands arrive in `o`, read during the previous step;
//     (s, sub 1) operands are read at the start; (s + 1, sub 0) operands
//     are read into `o` once the sub-0 MFMAs have taken theirs, so the next
//     step starts its MFMAs as soon as it passes the barrier.
//   * the decode of step s + 2 comes in small pieces (a 4x4 transpose, or
//     the decode and LDS write of one input) between MFMAs, spread over the
//     first 14 of them so the last LDS write lands before the barrier.  A
//     piece's VALU work issues while the MFMA before it occupies the matrix
//     core; scheduling barriers keep the order.
template <int SHAPE, bool kXs, int UPT, bool kMma, bool kSmall>
__device__ __forceinline__ void pipelined_step(const uint8_t *cur, const uint8_t *next,
                                               uint8_t *dec, int slot_bytes, int s0, int c0,
                                               Acc<SHAPE> &acc, const Unit (&u)[UPT],
                                               const Prefetch<UPT> &p, uint32_t vb0,
                                               uint32_t vb1, Ops<SHAPE> &o) {
    // 5 pieces: the transposes of all units, then input c of all units;
    // the units' chains are independent, so a piece has UPT-fold ILP
    constexpr int kPieces = 5;
    constexpr int kSpan = 14;
    using TL = Tiles<SHAPE>;
    Ops<SHAPE> o1;
    if (kMma) read_ops(cur, slot_bytes, s0, c0, 1, o1);
    // decode state
    uint32_t L[UPT][4];
    uint32_t msk[UPT];
    auto piece = [&](int k) {
        const int c = k - 1;
        if (c < 0) {
#pragma unroll
            for (int r = 0; r < UPT; ++r) {
                transpose4(p.d[r], L[r]);
                const uint32_t vbits = kSmall && u[r].hi ? vb1 : vb0;
                const uint32_t vq = u[r].act ? (vbits >> (4 * u[r].sq)) & 15u : 0u;
                msk[r] = bits_to_bytes(vq);
            }
        } else {
#pragma unroll
            for (int r = 0; r < UPT; ++r) {
                const int oo = u[r].sq >> 1, h = u[r].sq & 1;
                uint32_t Lm = (L[r][c] & msk[r]) | (0x88888888u & ~msk[r]);
                uint32_t an = (Lm >> 4) & 0x0f0f0f0fu, bn = Lm & 0x0f0f0f0fu;
                uint8_t *dst = dec + chunk_off(slot_bytes, u[r].s, 0, oo >> 1,
                                               (oo & 1) * 32 + 4 * u[r].q + c) + 8 * h;
                v2u xr = {nib_to_s8(an), nib_to_s8(bn)};
                *(v2u *)dst = xr;
                if (kXs) {
                    v2u v = {(an + bn + 0x70707070u) ^ 0x80808080u,
                             ((bn | 0x80808080u) - an) ^ 0x80808080u};
                    *(v2u *)(dst + kFragBytes) = v;
                }
            }
        }
    };
    v4i xp[TL::NXP];
    auto rows_xp = [&](const Ops<SHAPE> &q) {
        if (SHAPE == kRect) {
            xp[0] = make_xp(q.x[0]);
        } else {
#pragma unroll
            for (int i = 0; i < TL::NXP; ++i) xp[i] = make_xp(q.x[TL::row(2 * i)]);
        }
    };
    // MFMA k (0..7) of a sub-step
    auto mfma_op = [&](const Ops<SHAPE> &q, int k) {
        if (SHAPE == kRect) {
            const int t = k / 2;
            if (k % 2 == 0)
                acc.re[t] = mfma(q.x[0], q.y[t], acc.re[t]);
            else
                acc.im[t] = mfma(xp[0], q.y[t], acc.im[t]);
        } else if (k < 2) {
            acc.q[k] = mfma(q.xs[k], q.x[TL::qb(k)], acc.q[k]);
        } else {
            const int t = (k - 2) / 2;
            const int i = TL::row(t), j = TL::col(t);
            if (k % 2 == 0)
                acc.re[t] = mfma(q.x[i], q.x[j], acc.re[t]);
            else
                acc.im[t] = mfma(xp[TL::xpi(i)], q.x[j], acc.im[t]);
        }
    };

    if (kMma) rows_xp(o);
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        if (kMma) {
            if (m == 8) rows_xp(o1);
            if (m == 9) read_ops(next, slot_bytes, s0, c0, 0, o);
            if (m < 8)
                mfma_op(o, m);
            else
                mfma_op(o1, m - 8);
        }
#pragma unroll
        for (int q = 0; q < kPieces; ++q)
            if (q * kSpan / kPieces == m) piece(q);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Where the tiles of a wave lie: tile k < NQ is the diagonal tile of block
// qb(k), the others pair a row block with a column block.  Element v of a
// tile held by `lane` is (i, j) = (8 (v/4) + 4 (lane/32) + v%4, lane%32)
// within the tile (the output layout of v_mfma_i32_32x32x32_i8).
template <int SHAPE>
struct TileMap {
    Group g;
    int s0, c0, N;
    __device__ void rc(int k, int &rs, int &cs) const {
        using TL = Tiles<SHAPE>;
        if (k < TL::NQ) {
            rs = cs = s0 + TL::qb(k);
        } else if (SHAPE == kRect) {
            rs = s0;
            cs = c0 + TL::col(k - TL::NQ);
        } else {
            rs = s0 + TL::row(k - TL::NQ);
            cs = s0 + TL::col(k - TL::NQ);
        }
    }
    // index of the element in the packed triangle, or -1 when it lies below
    // the diagonal or past N
    __device__ int64_t elem(int k, int v, int lane) const {
        int rs, cs;
        rc(k, rs, cs);
        const int i = slot_block(g, rs) * kBlk + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int j = slot_block(g, cs) * kBlk + (lane & 31);
        if (i > j || j >= N) return -1;
        return (int64_t)i * N - (int64_t)i * (i - 1) / 2 + (j - i);
    }
};

// The role of wave `wave` in a tile group: its staging share, tile shape and
// first row / column slot.  Waves w and w + 4 share a SIMD: each SIMD gets
// one rectangle and (diagonal group) one half triangle.
template <int NSLOT_, int SHAPE_, int UPT_, bool kMma_ = true, bool kSmall_ = false>
struct Role {
    static constexpr int NSLOT = NSLOT_, SHAPE = SHAPE_, UPT = UPT_;
    static constexpr bool kMma = kMma_;     // runs MFMAs (else stages only)
    static constexpr bool kSmall = kSmall_;  // the halves geometry
};

// Which role sets a caller instantiates: kAllKinds (decides per group), or
// only the groups of one geometry (the two persistent batch kernels, so
// that each is register-allocated for its own roles).
enum Kinds { kAllKinds = 0, kSuperOnly = 1, kHalvesOnly = 2 };

template <int KINDS = kAllKinds, class Fn>
__device__ __forceinline__ void with_role(const Group &g, int wave, Fn &&fn) {
    if (KINDS == kHalvesOnly || (KINDS == kAllKinds && g.diag && g.small)) {
        // halves geometry: the rectangle waves stage only; waves 4, 5 take
        // the triangle of slots 0..3 (even steps), waves 6, 7 of 4..7 (odd)
        if (wave < 4)
            fn(Role<8, kRect, 1, false, true>{}, wave, 4);
        else if ((wave & 1) == 0)
            fn(Role<8, kTriA, 1, true, true>{}, 2 * (wave - 4), 0);
        else
            fn(Role<8, kTriB, 1, true, true>{}, 2 * (wave - 5), 0);
    } else if (g.diag) {
        if (wave < 4)  // row block `wave` x columns 4..7
            fn(Role<8, kRect, 1>{}, wave, 4);
        else if ((wave & 1) == 0)  // triangle of blocks 0..3 (wave 4) or 4..7 (wave 6)
            fn(Role<8, kTriA, 1>{}, 2 * (wave - 4), 0);
        else
            fn(Role<8, kTriB, 1>{}, 2 * (wave - 5), 0);
    } else {
        // row slot wave % 4 x column slots 4 + 4 (wave / 4) .. + 3
        if (wave < 4)
            fn(Role<12, kRect, 2>{}, wave, 4);
        else
            fn(Role<12, kRect, 1>{}, wave - 4, 8);
    }
}

// (Re, Im) partial tiles of chunk `split` (>= 1) of tile group `key`, wave
// `wave`: [tile k][re 0..3 | im 4..7][lane] x 4 int32
template <class T>
__device__ __forceinline__ T *partial_tiles(T *partials, int64_t key, int splits, int split,
                                            int wave) {
    return partials + (key * (splits - 1) + (split - 1)) * kGroupPartial +
           (int64_t)wave * kWavePartial;
}

// Valid samples of one channel (mask row m of nblk blocks of B samples, T
// samples), counted by one wave: lane l takes blocks l, l + 64, ..., four
// per pass with every load issued before the first is used (indices clamped
// in range), then the lanes' sums are added; every lane gets the total.
__device__ inline int64_t valid_count(const uint8_t *m, int nblk, int B, int T, int lane) {
    if (m == nullptr) return T;
    const int last = nblk - 1;
    int n = 0;  // <= T < 2^24
    for (int b0 = 0; b0 <= last; b0 += 64 * 4) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = m[min(b0 + 64 * u + lane, last)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + 64 * u + lane;
            const int64_t lo = (int64_t)b * B;
            const int64_t hi = lo + B < T ? lo + B : T;
            n += (b <= last && v[u] == 0u) ? (int)(hi - lo) : 0;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
    return n;
}

// Q of a diagonal tile -> (Re, Im) = ((Q + Q^T) / 2, (Q - Q^T) / 2), exact
// (Q + Q^T = 2 Re is even; int64 so the sum cannot wrap).  The transpose
// goes through LDS (32 x 33 int32 per wave, padded against bank conflicts).
__device__ __forceinline__ void split_q(const v16i &q, int32_t *tbuf, v16i &re, v16i &im) {
    const int lane = threadIdx.x & 63;
    const int col = lane & 31;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        tbuf[row * 33 + col] = q[v];
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS writes landed
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        int64_t qij = q[v], qji = tbuf[col * 33 + row];
        re[v] = (int32_t)((qij + qji) >> 1);
        im[v] = (int32_t)((qij - qji) >> 1);
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
}

// UPT = staging units per lane and step (wave-rounds of 64 units): the
// 16 (diagonal) or 24 (off-diagonal) wave-rounds of a step are dealt to the
// 8 waves as x = r * 8 + wave.
template <bool kAligned, bool kOverwrite, int NSLOT, int SHAPE, int UPT, bool kMma, bool kSmall>
__device__ __forceinline__ void run_wave(const CorrArgs &a, const Group &g, int f, int gid,
                                         int split, int s0, int c0, uint8_t *lds,
                                         uint32_t *mwords) {
    using TL = Tiles<SHAPE>;
    constexpr bool kDiagGroup = NSLOT == 8;
    constexpr int SLOT = kDiagGroup ? 2 * kFragBytes : kFragBytes;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;

    const int t_begin = split * a.steps_per_split * kStep;
    int t_end = t_begin + a.steps_per_split * kStep;
    if (t_end > a.T) t_end = a.T;
    // 32-sample steps of the chunk, and loop steps: one 32-sample step, or
    // a pair of them in the halves geometry
    const int nsteps32 = (t_end - t_begin + kStep - 1) / kStep;
    constexpr int pair = kSmall ? 2 : 1;
    const int nsteps = (nsteps32 + pair - 1) / pair;
    constexpr int step_samples = pair * kStep;

    const Chunk ch = make_chunk(a, f, t_begin, t_end);
    Unit u[UPT];
#pragma unroll
    for (int r = 0; r < UPT; ++r) {
        const int x = r * kWaves + wave;  // wave-round: 64 units
        const int o = x / (NSLOT / 4), sg = x % (NSLOT / 4);
        const int h = (lane >> 4) & 1;
        u[r].q = lane & 7;
        u[r].s = 4 * sg + ((lane >> 3) & 1) + 2 * ((lane >> 5) & 1);
        u[r].sq = 2 * o + h;
        int n0 = slot_block(g, u[r].s) * kBlk + 4 * u[r].q;
        u[r].act = n0 < a.N;
        u[r].hi = kSmall && u[r].s >= 4;
        u[r].voff = u[r].act ? (uint32_t)(4 * u[r].sq + (u[r].hi ? kStep : 0)) * ch.row_bytes +
                                   (uint32_t)n0
                             : 0x80000000u;
        u[r].inb = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) u[r].inb |= (n0 + c < a.N ? 1u : 0u) << c;
    }

    Acc<SHAPE> acc;
#pragma unroll
    for (int k = 0; k < TL::NO; ++k) {
        acc.re[k] = (v16i){0};
        acc.im[k] = (v16i){0};
    }
#pragma unroll
    for (int k = 0; k < TL::NQ; ++k) acc.q[k] = (v16i){0};

    // pipeline, per step s:
    //   raw bytes   loaded kDepth steps ahead into a ring of register sets
    //               (set k holds steps = k mod D), loop unrolled D times so
    //               each set has fixed registers;
    //   decode      two steps ahead, into the third of three LDS buffers;
    //   MFMA        from the buffer of step s, operands read ahead.
    // Steps past the chunk are staged as zeros (the last ring is padded).
    constexpr int D = kAligned ? kDepth : 3;
    static_assert(D >= 3, "the ring must hold the step being decoded and two in flight");
    // validity words: a window of kMaskWindow steps in LDS; each lane caches
    // the word of one of the next 64 steps, read out with readlane
    // (in 32-sample steps: loop step j uses word j, or words 2j and 2j + 1)
    fill_mask_window(a, f, ch, 0, nsteps32, mwords);
    Prefetch<UPT> pf[D];
#pragma unroll
    for (int k = 0; k < D; ++k) issue_loads<kAligned>(ch, t_begin + k * step_samples, u, pf[k]);
    __syncthreads();
    uint32_t mcache = mwords[lane];
    auto vbits_of = [&](int j32) -> uint32_t {
        return j32 < nsteps32 ? (uint32_t)__builtin_amdgcn_readlane((int)mcache, j32 & 63) : 0u;
    };
    commit<kDiagGroup, kSmall>(u, pf[0], vbits_of(0), vbits_of(pair - 1), lds, SLOT);
    commit<kDiagGroup, kSmall>(u, pf[1], vbits_of(pair), vbits_of(2 * pair - 1),
                               lds + kBufBytes, SLOT);
    __syncthreads();
    Ops<SHAPE> ops;
    if (kMma) read_ops(lds, SLOT, s0, c0, 0, ops);
    int b_cur = 0, b_next = kBufBytes, b_dec = 2 * kBufBytes;  // LDS byte offsets
    const int npad = (nsteps + D - 1) / D * D;
    for (int sb = 0; sb < npad; sb += D) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int s = sb + k;
            const int j = s + 2;   // step decoded now
            const int j32 = pair * j;
            if ((j32 & 63) == 0 && j32 < nsteps32) {
                if (j32 % kMaskWindow == 0) {
                    // next window of validity words (uniform branch, rare)
                    fill_mask_window(a, f, ch, j32, nsteps32, mwords);
                    __syncthreads();
                }
                mcache = mwords[(j32 % kMaskWindow) + lane];
            }
            const uint32_t vb0 = vbits_of(j32), vb1 = kSmall ? vbits_of(j32 + 1) : vb0;
            issue_loads<kAligned>(ch, t_begin + (s + D) * step_samples, u, pf[k]);
            pipelined_step<SHAPE, kDiagGroup, UPT, kMma, kSmall>(
                lds + b_cur, lds + b_next, lds + b_dec, SLOT, s0, c0, acc, u, pf[(k + 2) % D], vb0,
                vb1, ops);
            __syncthreads();
            const int t = b_cur;
            b_cur = b_next;
            b_next = b_dec;
            b_dec = t;
        }
    }

    // ---- epilogue, one tile at a time -----------------------------------
    // Chunk 0 (or the only chunk) writes the sums: plain stores (overwrite)
    // or read-add-write (accumulate).  Later chunks store their tiles in the
    // workspace and the merge kernel, launched next on the same stream, adds
    // them: the kernel boundary orders the two, so no fence or counter is
    // needed and the additions spread over the whole GPU.
    // Halves geometry: waves 6 and 7 (odd steps) hand their sums to waves 4
    // and 5 (even steps, the same tiles and layout) through LDS, which is
    // free after the loop's last barrier; only waves 4 and 5 write.
    if (kSmall) {
        int32_t *cb = (int32_t *)lds + (wave & 1) * (8 * 16 * 64);
        auto each = [&](auto fn) {
            int m = 0;
#pragma unroll
            for (int k = 0; k < TL::NQ; ++k) fn(acc.q[k], m++);
#pragma unroll
            for (int k = 0; k < TL::NO; ++k) {
                fn(acc.re[k], m++);
                fn(acc.im[k], m++);
            }
        };
        if (kMma && wave >= 6)
            each([&](v16i &x, int m) {
#pragma unroll
                for (int v = 0; v < 16; ++v) cb[(m * 16 + v) * 64 + lane] = x[v];
            });
        __syncthreads();
        if (kMma && (wave == 4 || wave == 5))
            each([&](v16i &x, int m) {
#pragma unroll
                for (int v = 0; v < 16; ++v) x[v] += cb[(m * 16 + v) * 64 + lane];
            });
        __syncthreads();
        if (!(kMma && (wave == 4 || wave == 5))) return;
    }
    constexpr int NT = TL::NT;
    int32_t *tbuf = (int32_t *)lds + wave * (32 * 33);  // staging buffers are free now
    const TileMap<SHAPE> map{g, s0, c0, a.N};
    auto tile = [&](int k, v16i &re, v16i &im) {
        if (k < TL::NQ) {
            split_q(acc.q[k < TL::NQ ? k : 0], tbuf, re, im);
        } else {
            re = acc.re[k - TL::NQ];
            im = acc.im[k - TL::NQ];
        }
    };
    if (split > 0) {
        const int64_t key = (int64_t)f * a.groups + gid;
        int32_t *mine = partial_tiles(a.partials, key, a.splits, split, wave);
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            v16i re, im;
            tile(k, re, im);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                v4i x = {re[4 * v], re[4 * v + 1], re[4 * v + 2], re[4 * v + 3]};
                v4i y = {im[4 * v], im[4 * v + 1], im[4 * v + 2], im[4 * v + 3]};
                *(v4i *)(mine + ((k * 8 + v) * 64 + lane) * 4) = x;
                *(v4i *)(mine + ((k * 8 + 4 + v) * 64 + lane) * 4) = y;
            }
        }
        return;
    }
    const int64_t P = (int64_t)a.N * (a.N + 1) / 2;
    int32_t *visf = a.vis + (int64_t)f * P * 2;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        // previous contents first (accumulate), all loads before any store
        v2i old[16];
        if (!kOverwrite) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t idx = map.elem(k, v, lane);
                old[v] = idx >= 0 ? *(const v2i *)(visf + 2 * idx) : (v2i){0, 0};
            }
        }
        v16i re, im;
        tile(k, re, im);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t idx = map.elem(k, v, lane);
            if (idx >= 0) {
                v2i val = {re[v], im[v]};
                *(v2i *)(visf + 2 * idx) = kOverwrite ? val : old[v] + val;
            }
        }
    }
}

// Workgroup b runs on XCD b % 8 (round-robin dispatch); number the work so
// that consecutive work items (the time chunks and groups of one channel)
// share an XCD and its L2.
__device__ __forceinline__ int64_t xcd_local_index(int64_t b, int64_t total) {
    const int64_t per = total / 8, rem = total % 8;
    const int64_t x = b % 8, idx = b / 8;
    return x * per + (x < rem ? x : rem) + idx;
}

// One work item: tile group gid of channel f over time chunk `split`.
// Every wave runs the same number of steps and barriers; the tile pattern is
// fixed per group kind (blocks past N are staged as zeros).
template <bool kAligned, bool kOverwrite, int KINDS = kAllKinds>
__device__ __forceinline__ void run_item(const CorrArgs &a, int f, int gid, int split,
                                         uint8_t *lds, uint32_t *mwords) {
    const Group g = make_group(a.nb, gid, a.halves);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    with_role<KINDS>(g, wave, [&](auto role, int s0, int c0) {
        using R = decltype(role);
        run_wave<kAligned, kOverwrite, R::NSLOT, R::SHAPE, R::UPT, R::kMma, R::kSmall>(
            a, g, f, gid, split, s0, c0, lds, mwords);
    });
}

// One frame: workgroup -> (channel, group, chunk), groups of a channel
// and chunks of a (channel, group) numbered next to each other.
template <bool kAligned, bool kOverwrite>
__global__ __launch_bounds__(kThreads, 1) void corr_kernel(CorrArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[3 * kBufBytes];
    __shared__ uint32_t mwords[kMaskWindow];

    const int G = a.groups;
    const int64_t total = (int64_t)a.F * G * a.splits;
    int64_t w = xcd_local_index(blockIdx.x, total);
    const int gid = (int)(w % G);
    w /= G;
    const int split = (int)(w % a.splits);
    const int f = (int)(w / a.splits);
    run_item<kAligned, kOverwrite>(a, f, gid, split, lds, mwords);
}

// ---------------------------------------------------------------------------
// batched persistent launch
// ---------------------------------------------------------------------------

// One correlator instance of a batch, as the kernel sees it.
struct BatchInstance {
    const uint8_t *packed;
    const uint8_t *mask;
    int32_t *vis;
    int64_t *count;
    int32_t N, F, T, B;
    int32_t nblk_mask, nb, groups, splits;
    int32_t steps_per_split, aligned;
    int32_t halves, pad_;
    int64_t partial_base;  // first int32 of its partial tiles
};

struct BatchItem {
    int32_t inst, f, gid, split;
};

// A grid of one workgroup per CU pulls work items from a queue until it is
// empty (every workgroup reaches the exit).  The last workgroup to finish
// resets the queue, so the next launch of the same plan starts clean and
// the launch can be replayed from a graph.  Items are accumulated into their
// instances' resident sums.  Instances must take the dword-load path
// (N % 4 == 0, 4-byte aligned frame); the host runs others on their own.
// A batch has one list of items per geometry, each drained by its own
// launch of this kernel (KINDS = kSuperOnly or kHalvesOnly).
template <int KINDS>
__global__ __launch_bounds__(kThreads, 1) void batch_kernel(const BatchInstance *inst,
                                                            const BatchItem *items, int n_items,
                                                            int *queue,
                                                            int32_t *partials) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[3 * kBufBytes];
    __shared__ uint32_t mwords[kMaskWindow];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();  // the previous item has released LDS
        if (threadIdx.x == 0) s_item = atomicAdd(&queue[0], 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);  // uniform: scalar loads below
        if (it >= n_items) break;
        // every field is wave-uniform: readfirstlane keeps them in scalar
        // registers (buffer resources and offsets must live there)
        auto u32 = [](int32_t v) { return (int32_t)__builtin_amdgcn_readfirstlane(v); };
        auto u64 = [](int64_t v) {
            uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
            uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
            return (int64_t)(((uint64_t)hi << 32) | lo);
        };
        auto ptr = [&](const void *p) { return (void *)(uintptr_t)u64((int64_t)(uintptr_t)p); };
        const BatchItem w = items[it];
        const int wi = u32(w.inst), wf = u32(w.f), wg = u32(w.gid), ws = u32(w.split);
        const BatchInstance &bi = inst[wi];
        CorrArgs a;
        a.packed = (const uint8_t *)ptr(bi.packed);
        a.mask = (const uint8_t *)ptr(bi.mask);
        a.vis = (int32_t *)ptr(bi.vis);
        a.count = (int64_t *)ptr(bi.count);
        a.partials = partials + u64(bi.partial_base);
        a.N = u32(bi.N);
        a.F = u32(bi.F);
        a.T = u32(bi.T);
        a.B = u32(bi.B);
        a.nblk_mask = u32(bi.nblk_mask);
        a.nb = u32(bi.nb);
        a.groups = u32(bi.groups);
        a.splits = u32(bi.splits);
        a.steps_per_split = u32(bi.steps_per_split);
        a.halves = u32(bi.halves);
        run_item<true, false, KINDS>(a, wf, wg, ws, lds, mwords);
    }
    if (threadIdx.x == 0) {
        int done = atomicAdd(&queue[1], 1);
        if (done == (int)gridDim.x - 1) {
            queue[0] = 0;
            queue[1] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// merge of time chunks
// ---------------------------------------------------------------------------

// An instance whose time chunks are merged: chunk 0 has written its sums to
// `vis`, chunks 1 .. splits-1 left their tiles in `partials`.
struct MergeInst {
    int32_t *vis;
    int32_t *partials;
    int N, nb, groups, splits;
    int halves, pad_;
    int64_t block_begin;  // first merge block of the instance (batch lists)
};

// One wave adds chunks 1.. of tile k of its role in group `key` into vis;
// the loads of three chunks and of the old sums are in flight together.
template <int SHAPE>
__device__ __forceinline__ void merge_tile(const MergeInst &m, const Group &g, int64_t key,
                                           int wave, int k, int s0, int c0) {
    using TL = Tiles<SHAPE>;
    if (k >= TL::NT) return;
    const int lane = threadIdx.x & 63;
    const TileMap<SHAPE> map{g, s0, c0, m.N};
    const int64_t f = key / m.groups;
    const int64_t P = (int64_t)m.N * (m.N + 1) / 2;
    int32_t *visf = m.vis + f * P * 2;
    {
        v2i old[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t idx = map.elem(k, v, lane);
            old[v] = idx >= 0 ? *(const v2i *)(visf + 2 * idx) : (v2i){0, 0};
        }
        v16i re = (v16i){0}, im = (v16i){0};
        for (int sp0 = 1; sp0 < m.splits; sp0 += 3) {
            v4i ld[3][8];
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
                const int sp = sp0 + jj < m.splits ? sp0 + jj : 1;
                const int32_t *src = partial_tiles(m.partials, key, m.splits, sp, wave) +
                                     (k * 8 * 64 + lane) * 4;
#pragma unroll
                for (int v = 0; v < 8; ++v) ld[jj][v] = *(const v4i *)(src + v * 256);
            }
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
                if (sp0 + jj < m.splits) {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            re[4 * v + c] += ld[jj][v][c];
                            im[4 * v + c] += ld[jj][4 + v][c];
                        }
                }
            }
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t idx = map.elem(k, v, lane);
            if (idx >= 0) *(v2i *)(visf + 2 * idx) = old[v] + (v2i){re[v], im[v]};
        }
    }
}

// merge block b of an instance = (group key, wave role, tile) =
// (b / (8 kTilesPerWave), b / kTilesPerWave % 8, b % kTilesPerWave)
constexpr int kMergeBlocksPerGroup = kWaves * kTilesPerWave;

__device__ __forceinline__ void merge_block(const MergeInst &m, int64_t b) {
    const int64_t key = b / kMergeBlocksPerGroup;
    const int wave = (int)(b / kTilesPerWave % kWaves);
    const int k = (int)(b % kTilesPerWave);
    const Group g = make_group(m.nb, (int)(key % m.groups), m.halves);
    if (g.small && wave != 4 && wave != 5) return;   // halves: waves 4 and 5 own the sums
    with_role(g, wave, [&](auto role, int s0, int c0) {
        merge_tile<decltype(role)::SHAPE>(m, g, key, wave, k, s0, c0);
    });
}

// one instance: F * groups * 8 * kTilesPerWave blocks of one wave
// Valid-sample counts of a frame, taken by extra blocks of its merge launch
// (block first_block + f counts channel f), so a chunked frame needs no
// launch of its own for them.
struct CountArgs {
    const uint8_t *mask;
    int64_t *count;
    int nblk, B, T, overwrite;
    int64_t first_block;
};

__global__ __launch_bounds__(64) void merge_kernel(MergeInst m, CountArgs c) {
    if ((int64_t)blockIdx.x >= c.first_block) {
        const int f = (int)(blockIdx.x - c.first_block);
        const int lane = threadIdx.x & 63;
        const int64_t n = valid_count(c.mask ? c.mask + (int64_t)f * c.nblk : nullptr, c.nblk,
                                      c.B, c.T, lane);
        if (lane == 0) c.count[f] = c.overwrite ? n : c.count[f] + n;
        return;
    }
    merge_block(m, blockIdx.x);
}

// a batch's chunked instances, sorted by block_begin; block b belongs to the
// last instance whose first block is <= b
__global__ __launch_bounds__(64) void merge_list_kernel(const MergeInst *list, int n) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (list[mid].block_begin <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    const MergeInst m = list[lo];
    merge_block(m, b - m.block_begin);
}

// ---------------------------------------------------------------------------
// valid-sample counts (the packet-loss counter, Sec. II-C)
// ---------------------------------------------------------------------------

// One wave per channel of one frame; a separate launch, so that the
// correlation kernel's registers stay with its main loop.
constexpr int kCountWaves = 4;

__global__ __launch_bounds__(64 * kCountWaves) void count_kernel(const uint8_t *mask, int nblk,
                                                                 int B, int T, int F,
                                                                 int64_t *count, int overwrite) {
    const int lane = threadIdx.x & 63;
    const int f = blockIdx.x * kCountWaves + (threadIdx.x >> 6);
    if (f >= F) return;
    const int64_t n = valid_count(mask ? mask + (int64_t)f * nblk : nullptr, nblk, B, T, lane);
    if (lane == 0) count[f] = overwrite ? n : count[f] + n;
}

// The same for every instance of a batch (block b = instance b, its waves
// take its channels in turn); batches accumulate.
__global__ __launch_bounds__(64 * kCountWaves) void count_list_kernel(const BatchInstance *inst,
                                                                      int n_inst) {
    const BatchInstance &x = inst[blockIdx.x];
    const int lane = threadIdx.x & 63;
    for (int f = threadIdx.x >> 6; f < x.F; f += kCountWaves) {
        const int64_t n = valid_count(x.mask ? x.mask + (int64_t)f * x.nblk_mask : nullptr,
                                      x.nblk_mask, x.B, x.T, lane);
        if (lane == 0) x.count[f] += n;
    }
}

// ---------------------------------------------------------------------------
// normalisation
// ---------------------------------------------------------------------------

// out = (float)((double)v / (double)n), 0 when n == 0; four values per
// thread and iteration (16-byte accesses when kVec: both pointers aligned)
template <bool kVec>
__global__ void normalize_kernel(const int32_t *vis, const int64_t *count, float *out,
                                 int64_t per_channel, int F) {
    const int64_t total = per_channel * F;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t k = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * 4; k < total;
         k += stride) {
        if (kVec && k + 4 <= total && (k / per_channel) == ((k + 3) / per_channel)) {
            int64_t n = count[k / per_channel];
            v4i v = *(const v4i *)(vis + k);
            double dn = (double)n;
            float4 o;
            o.x = n == 0 ? 0.0f : (float)((double)v.x / dn);
            o.y = n == 0 ? 0.0f : (float)((double)v.y / dn);
            o.z = n == 0 ? 0.0f : (float)((double)v.z / dn);
            o.w = n == 0 ? 0.0f : (float)((double)v.w / dn);
            *(float4 *)(out + k) = o;
        } else {
            for (int64_t e = k; e < k + 4 && e < total; ++e) {
                int64_t n = count[e / per_channel];
                out[e] = n == 0 ? 0.0f : (float)((double)vis[e] / (double)n);
            }
        }
    }
}

}  // namespace xe
