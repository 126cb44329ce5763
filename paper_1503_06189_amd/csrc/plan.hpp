// plan.hpp -- how one frame is split into workgroups (host and device).
//
// The triangle of 32x32 input-block tiles (I <= J) of each channel is cut
// into "super-blocks" of 8x8 tiles (256 x 256 inputs).  A workgroup of eight
// waves (two per SIMD, 128 accumulator registers each) takes one tile group:
//   * a diagonal super-block: a triangle of 36 tiles, 8 on the diagonal
//     and 28 off it.  A diagonal tile costs half (one MFMA chain, 16
//     accumulator registers).  Waves 0..3 take the 1 x 4 rectangles of
//     tiles (w, 4..7); waves 4..7 take the halves of the triangles of
//     blocks 0..3 and 4..7 (2 diagonal tiles and 3 off-diagonal ones each);
//   * half of an off-diagonal super-block: 4 tile rows x 8 tile columns.
//     Wave w takes row w % 4 and columns 4 (w / 4) .. + 3.
// Every wave thus runs 16 MFMAs per staged step, and the two waves of a
// SIMD (w and w + 4) together run 32.  Super-blocks at the edge of the
// triangle are padded: input blocks past ceil(N/32) are staged as zeros and
// their tiles are computed but never stored, so every wave has a fixed,
// compile-time tile pattern.  With ns = ceil(blocks / 8) super-rows there
// are ns diagonal groups and ns(ns-1)/2 off-diagonal super-blocks of two
// halves each: ns^2 groups.  Each workgroup integrates its tiles over one
// chunk of the frame's time samples; chunk 0 writes the output and a merge
// kernel adds the other chunks.
//
// Second geometry ("halves", for N <= 128, at most 4 input blocks): the
// padded super-block would compute 36 tiles for the 10 of the 4-block
// triangle.  Instead the 8 staged slots hold blocks 0..3 at two consecutive
// 32-sample steps (slots 4..7 one step later), so a loop step covers 64
// samples: waves 4 and 5 integrate the triangle over the even steps, waves
// 6 and 7 over the odd ones, and the rectangle waves only stage.  At the end
// waves 6 and 7 hand their sums to 4 and 5 through LDS, which write them.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define XE_HD __host__ __device__
#else
#define XE_HD
#endif

namespace xe {

constexpr int kBlk = 32;          // inputs per tile edge (one 32x32 MFMA)
constexpr int kStep = 32;         // samples staged per step
constexpr int kSuper = 8;         // tile blocks per super-block edge
constexpr int kMaxSlots = 12;     // input blocks staged per workgroup
constexpr int kTilesPerWave = 5;  // (Re, Im) tiles a wave writes out, at most
constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
// |Q| of a diagonal tile grows by at most 248 per sample: a chunk of at
// most 2^18 steps (8,388,608 samples) keeps it inside int32
constexpr int kMaxStepsPerChunk = 1 << 18;
// Raw bytes are loaded this many steps ahead of their use; a chunk is run
// in whole rings of kDepth steps (the last ring padded with zeros), so the
// byte offsets of a chunk plus 4 * kDepth 32-sample steps must stay below
// 2^31.
#ifndef XE_DEPTH
#define XE_DEPTH 4
#endif
constexpr int kDepth = XE_DEPTH;

// longest chunk (in steps) whose byte offsets, lookahead included (twice the
// ring in 32-sample steps: a halves loop step covers two), stay below 2^31
// for F channels of N inputs
inline int64_t max_steps_per_chunk(int64_t F, int64_t N) {
    int64_t m = (((int64_t)1 << 31) - 1) / (F * N * kStep) - 4 * kDepth;
    if (m > kMaxStepsPerChunk) m = kMaxStepsPerChunk;
    return m - m % kDepth;
}

// round a chunk length up to whole rings
inline int round_steps(int sps) { return (sps + kDepth - 1) / kDepth * kDepth; }

// One tile group, in scalars (no arrays: kept in scalar registers on the
// device).  Slot s of the staged blocks holds input block
//   diagonal:      rbase + s                       (s < nslots)
//   off-diagonal:  rbase + s for s < 4, cbase + s - 4 otherwise
//   halves:        s % 4 (slots 4..7 one step later)
struct Group {
    int diag;
    int small;   // the halves geometry
    int rbase, cbase;
    int nslots;
};

// the halves geometry applies to frames of at most 4 input blocks
XE_HD inline int use_halves(int halves, int nb) { return halves && nb <= 4 ? 1 : 0; }

XE_HD inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

XE_HD inline int super_rows(int nb) { return ceil_div(nb, kSuper); }

XE_HD inline int groups_per_channel(int nb) {
    int ns = super_rows(nb);
    return ns * ns;
}

// off-diagonal super-block number p (row-major over R < C) -> (R, C)
XE_HD inline void offdiag_pair(int ns, int p, int *R, int *C) {
    int r = 0;
    while (p >= ns - 1 - r) {
        p -= ns - 1 - r;
        ++r;
    }
    *R = r;
    *C = r + 1 + p;
}

XE_HD inline Group make_group(int nb, int gid, int halves) {
    Group g;
    int ns = super_rows(nb);
    g.small = 0;
    if (gid < ns) {
        g.diag = 1;
        g.small = use_halves(halves, nb);
        g.rbase = g.cbase = gid * kSuper;
        g.nslots = kSuper;  // blocks past the last one are staged as zeros
    } else {
        int q = gid - ns;
        int R, C;
        offdiag_pair(ns, q / 2, &R, &C);
        g.diag = 0;
        g.rbase = R * kSuper + 4 * (q % 2);  // R is never the last super-row
        g.cbase = C * kSuper;
        g.nslots = 4 + kSuper;
    }
    return g;
}

XE_HD inline int slot_block(const Group &g, int s) {
    if (g.small) return s & 3;
    return (g.diag || s < 4) ? g.rbase + s : g.cbase + (s - 4);
}

// 32x32 tiles computed per channel: 36 per diagonal group (8 x 9), 32 per
// off-diagonal half (4 x 8); padded tiles past N included.  The halves
// geometry computes the 10 tiles of the 4-block triangle.
inline int64_t tiles_per_channel(int nb, int halves) {
    if (use_halves(halves, nb)) return 10;
    int64_t ns = super_rows(nb);
    return ns * 36 + ns * (ns - 1) * 32;
}

// Time split: enough workgroups to cover `n_cu` compute units once, but
// at least `min_steps` staged steps per chunk.
inline void choose_split(int64_t units, int steps, int n_cu, int *splits,
                         int *steps_per_split) {
    const int min_steps = 8;
    int64_t want = (n_cu + units - 1) / units;
    int64_t cap = steps / min_steps;
    if (cap < 1) cap = 1;
    int64_t s = want < cap ? want : cap;
    if (s < 1) s = 1;
    int sps = round_steps(ceil_div(steps, (int)s));
    *steps_per_split = sps;
    *splits = ceil_div(steps, sps);
}

}  // namespace xe
