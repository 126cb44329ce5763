// shift_kernels.hpp -- per-input time shifting on gfx950.
//
// The GPU kernel stage of the method includes extra operations such as time
// shifting (caption of Fig. 4, Sec. II-B), with no algorithm given.  The
// reading here: input i of every channel is delayed by an integer d_i
// samples, out[t][f][i] = in[t - d_i][f][i].  A sample shifted in from
// outside the frame has no data: it is written as 0 + 0i (0x88) and marked
// as a flagged point, so the per-baseline normalisation counts it out;
// F-engine flags move with their data.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xe {
namespace shift {

// A workgroup takes channel f, output samples [t0, t0 + kRows) and inputs
// [i0, i0 + kCols).  When the tile's delays span at most kSpan samples, the
// source rows it needs (kRows + span rows of up to kCols bytes and kCols / 32
// flag words) are staged in LDS; every load of the stage is issued before
// the first is stored, so a workgroup waits for memory once.  A source row
// outside the frame is staged as 0x88 bytes and all-ones flag words, so the
// output needs no per-sample test: every output byte is one LDS read at a
// fixed offset from its input's column, and every output flag word one
// ballot over the 32 lanes of its inputs, gathered in LDS and stored row
// after row.  Wider spans, and frames whose rows are not 16-byte multiples,
// take direct gathers with the frame test per sample.  Every output element
// of the tile is written.
constexpr int kRows = 128;
constexpr int kCols = 256;
constexpr int kSpan = 32;
constexpr int kTileThreads = 256;
constexpr int kStageRows = kRows + kSpan;
constexpr int kWords = kCols / 32;
// per-thread loads of a full stage: 16-byte pieces of data, flag words
constexpr int kDataPer = kStageRows * (kCols / 16) / kTileThreads;
constexpr int kFlagPer = kStageRows * kWords / kTileThreads;
static_assert(kDataPer * kTileThreads == kStageRows * (kCols / 16), "whole data stage");
static_assert(kFlagPer * kTileThreads == kStageRows * kWords, "whole flag stage");
static_assert(kWords == 2 * (kTileThreads / 64), "one flag-word column per half-wave");

// v_writelane_b32 (the compiler's intrinsic, which has no builtin here):
// lane `lane` of `old` takes the wave-uniform value v
__device__ int llvm_writelane(int v, int lane, int old) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ uint32_t write_lane(uint32_t old, uint32_t v, int lane) {
    return (uint32_t)llvm_writelane((int)v, lane, (int)old);
}

struct Smem {
    uint8_t rows[kStageRows][kCols];
    uint32_t frows[kStageRows][kWords + 1];   // padded: rows 9 words apart
    uint32_t fout[kRows][kWords];
    int32_t dl[kCols];
    int32_t red[2][kTileThreads / 64];
};

// kVec: N % 16 == 0 and both frames 16-byte aligned: rows are staged with
// 16-byte loads and output bytes are written as dwords.
template <bool kVec>
__global__ __launch_bounds__(kTileThreads) void tile_kernel(const uint8_t *in,
                                                             const uint32_t *flags_in,
                                                             const int32_t *delays, uint8_t *out,
                                                             uint32_t *flags_out, int N, int F,
                                                             int T, int W) {
    __shared__ __attribute__((aligned(16))) Smem sm;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // channels vary fastest: workgroups that run together read and write
    // whole sample rows (F x N contiguous bytes) rather than pieces a row
    // apart
    const int i_tiles = (N + kCols - 1) / kCols;
    int64_t b = blockIdx.x;
    const int it = (int)(b % i_tiles);
    b /= i_tiles;
    const int f = (int)(b % F);
    const int tt = (int)(b / F);
    const int i0 = it * kCols, t0 = tt * kRows;
    const int ni = min(kCols, N - i0), nt = min(kRows, T - t0);

    // the tile's delays and their range
    int d = tid < ni ? delays[i0 + tid] : 0;
    sm.dl[tid] = d;
    int lo = tid < ni ? d : INT32_MAX, hi = tid < ni ? d : INT32_MIN;
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o));
        hi = max(hi, __shfl_xor(hi, o));
    }
    if (lane == 0) {
        sm.red[0][wave] = lo;
        sm.red[1][wave] = hi;
    }
    __syncthreads();
    lo = sm.red[0][0];
    hi = sm.red[1][0];
    for (int k = 1; k < kTileThreads / 64; ++k) {
        lo = min(lo, sm.red[0][k]);
        hi = max(hi, sm.red[1][k]);
    }
    const bool staged = (int64_t)hi - lo <= kSpan;
    // source rows t - d for t in [t0, t0 + nt) and d in [lo, hi]: [t0 - hi, t0 + nt - 1 - lo]
    const int64_t s0 = (int64_t)t0 - hi;
    const int nrows = staged ? nt + (hi - lo) : 0;
    const int wbase = i0 / 32, nw = (ni + 31) / 32;

    if (staged) {
        if (kVec) {
            // ni is a multiple of 16 here; all loads first, then the stores
            auto stage = [&](const int pieces) {
                const int total = nrows * pieces;
                uint4 v[kDataPer];
#pragma unroll
                for (int k = 0; k < kDataPer; ++k) {
                    const int e = tid + k * kTileThreads;
                    v[k] = (uint4){0x88888888u, 0x88888888u, 0x88888888u, 0x88888888u};
                    if (e < total) {
                        const int64_t src = s0 + e / pieces;
                        if (src >= 0 && src < T)
                            v[k] = *(const uint4 *)(in + (src * F + f) * N + i0 +
                                                    16 * (e % pieces));
                    }
                }
#pragma unroll
                for (int k = 0; k < kDataPer; ++k) {
                    const int e = tid + k * kTileThreads;
                    if (e < total) *(uint4 *)&sm.rows[e / pieces][16 * (e % pieces)] = v[k];
                }
            };
            // a full-width tile divides by a constant
            if (ni == kCols)
                stage(kCols / 16);
            else
                stage(ni / 16);
        } else {
            for (int e = tid; e < nrows * kCols; e += kTileThreads) {
                const int r = e / kCols, c = e % kCols;
                const int64_t src = s0 + r;
                sm.rows[r][c] = (c < ni && src >= 0 && src < T) ? in[(src * F + f) * N + i0 + c] : 0;
            }
        }
        if (flags_out) {
            const int total = nrows * kWords;
            uint32_t w[kFlagPer];
#pragma unroll
            for (int k = 0; k < kFlagPer; ++k) {
                const int e = tid + k * kTileThreads;
                const int r = e / kWords, c = e % kWords;
                const int64_t src = s0 + r;
                const bool in_frame = src >= 0 && src < T;
                w[k] = (flags_in && e < total && c < nw && in_frame)
                           ? flags_in[((int64_t)f * T + src) * W + wbase + c]
                           : in_frame ? 0u : 0xffffffffu;
            }
#pragma unroll
            for (int k = 0; k < kFlagPer; ++k) {
                const int e = tid + k * kTileThreads;
                if (e < total) sm.frows[e / kWords][e % kWords] = w[k];
            }
        }
        __syncthreads();
    }

    // data: thread tid keeps input quad tid % 64 and walks rows tid / 64, +4,
    // ...; one dword each (kVec), else bytes
    if (kVec && staged) {
        // output byte (r, c) is staged byte (r + hi - d_c, c)
        const int g = tid & 63, quads = ni / 4;
        if (g < quads) {
            const uint8_t *col[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                col[k] = &sm.rows[hi - sm.dl[4 * g + k] + wave][4 * g + k];
            uint8_t *dst = out + ((int64_t)(t0 + wave) * F + f) * N + i0 + 4 * g;
            const int64_t rstride = (int64_t)F * N;
            auto row = [&](int j) {   // row wave + 4 j
                const int o = 4 * j * kCols;
                const uint32_t v = (uint32_t)col[0][o] | ((uint32_t)col[1][o] << 8) |
                                   ((uint32_t)col[2][o] << 16) | ((uint32_t)col[3][o] << 24);
                *(uint32_t *)(dst + 4 * j * rstride) = v;
            };
            if (nt == kRows) {
#pragma unroll
                for (int j = 0; j < kRows / 4; ++j) row(j);
            } else {
                for (int j = 0; wave + 4 * j < nt; ++j) row(j);
            }
        }
    } else if (kVec) {
        const int g = tid & 63, quads = ni / 4;
        if (g < quads) {
            // per input: rows r of the tile whose source lies in the frame,
            // rlo <= r < rhi, and the staged row of r, r + base
            int dk[4], rlo[4], rhi[4], base[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                dk[k] = sm.dl[4 * g + k];
                const int64_t l = (int64_t)dk[k] - t0, u = (int64_t)T + dk[k] - t0;
                rlo[k] = (int)(l < 0 ? 0 : (l > nt ? nt : l));
                rhi[k] = (int)(u < 0 ? 0 : (u > nt ? nt : u));
                base[k] = staged ? hi - dk[k] : 0;   // in [0, kSpan] when staged
            }
#pragma unroll 4
            for (int r = tid >> 6; r < nt; r += kTileThreads / 64) {
                const int t = t0 + r;
                uint32_t v = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int c = 4 * g + k;
                    uint32_t byte = 0x88u;
                    if (r >= rlo[k] && r < rhi[k])
                        byte = staged ? sm.rows[r + base[k]][c]
                                      : in[((int64_t)(t - dk[k]) * F + f) * N + i0 + c];
                    v |= byte << (8 * k);
                }
                *(uint32_t *)(out + ((int64_t)t * F + f) * N + i0 + 4 * g) = v;
            }
        }
    } else {
        for (int c = tid; c < ni; c += kTileThreads) {
            const int dc = sm.dl[c];
            for (int r = 0; r < nt; ++r) {
                const int t = t0 + r;
                const int64_t src = (int64_t)t - dc;
                uint8_t v = 0x88;
                if (src >= 0 && src < T)
                    v = staged ? sm.rows[r + hi - dc][c] : in[(src * F + f) * N + i0 + c];
                out[((int64_t)t * F + f) * N + i0 + c] = v;
            }
        }
    }
    // flags: half-wave h (of 8) owns word column h of the tile; lane b holds
    // input 32 h + b and its delay, and each row's word is one ballot, kept
    // in LDS; then the tile's words go out row after row
    if (flags_out && staged) {
        // flag of output (r, c) = bit c % 32 of staged word (r + hi - d_c,
        // c / 32); lane 32 h + b of the gathered word holds row r0 + b of
        // word column 2 wave + h
        const int half = lane >> 5, bit = lane & 31;
        const int w = wave * 2 + half;
        const int c = 32 * w + bit;
        const bool inb = c < ni;
        const uint32_t *src = &sm.frows[inb ? hi - sm.dl[c] : 0][w];
        const uint32_t sel = inb ? 1u << bit : 0u;
        for (int r0 = 0; r0 < nt; r0 += 32) {
            // rows past nt read staged rows that are never stored
            uint32_t word[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) word[u] = src[(r0 + u) * (kWords + 1)];
            uint32_t mine = 0;
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                const unsigned long long m = __ballot((word[u] & sel) != 0u);
                mine = write_lane(mine, (uint32_t)m, u);
                mine = write_lane(mine, (uint32_t)(m >> 32), 32 + u);
            }
            if (w < nw && r0 + bit < nt) sm.fout[r0 + bit][w] = mine;
        }
    } else if (flags_out) {
        const int half = lane >> 5, bit = lane & 31;
        const int w = wave * 2 + half;
        if (w < nw) {
            const int c = 32 * w + bit;
            const bool inb = c < ni;
            const int dc = inb ? sm.dl[c] : 0;
            const int64_t l = (int64_t)dc - t0, u = (int64_t)T + dc - t0;
            const int rlo = (int)(l < 0 ? 0 : (l > nt ? nt : l));
            const int rhi = (int)(u < 0 ? 0 : (u > nt ? nt : u));
            const int base = staged ? hi - dc : 0;
            // four rows per pass: their reads are in flight together
            for (int r0 = 0; r0 < nt; r0 += 4) {
                bool set[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int r = r0 + u;
                    set[u] = false;
                    if (inb && r < nt) {
                        if (r < rlo || r >= rhi) {
                            set[u] = true;
                        } else if (flags_in) {
                            const uint32_t word =
                                staged ? sm.frows[r + base][w]
                                       : flags_in[((int64_t)f * T + (t0 + r - dc)) * W + wbase + w];
                            set[u] = (word >> bit) & 1u;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const unsigned long long m = __ballot(set[u]);
                    if (bit == 0 && r0 + u < nt) sm.fout[r0 + u][w] = (uint32_t)(m >> (32 * half));
                }
            }
        }
    }
    if (flags_out) {
        __syncthreads();
        for (int e = tid; e < nt * nw; e += kTileThreads) {
            const int r = e / nw, c = e % nw;
            flags_out[((int64_t)f * T + t0 + r) * W + wbase + c] = sm.fout[r][c];
        }
    }
}

}  // namespace shift
}  // namespace xe
