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

// A workgroup takes channel f, output samples [t0, t0 + 32) and
// inputs [i0, i0 + 256).  When the tile's delays span at most kSpan samples,
// the source rows it needs (32 + span rows of up to 256 bytes and 8 flag
// words) are staged in LDS with coalesced loads; every output byte is then
// a read from LDS, and every output flag word one ballot over the 32 lanes
// of its inputs.  Wider spans fall back to direct gathers in the same
// workgroup.  Every output element of the tile is written.
constexpr int kRows = 32;
constexpr int kCols = 256;
constexpr int kSpan = 32;
constexpr int kTileThreads = 256;
static_assert(kCols / 32 == 2 * (kTileThreads / 64), "one flag-word column per half-wave");

// kVec: N % 16 == 0 and both frames 16-byte aligned: rows are staged with
// 16-byte loads and output bytes are written as dwords.
template <bool kVec>
__global__ __launch_bounds__(kTileThreads) void tile_kernel(const uint8_t *in,
                                                             const uint32_t *flags_in,
                                                             const int32_t *delays, uint8_t *out,
                                                             uint32_t *flags_out, int N, int F,
                                                             int T, int W) {
    __shared__ __attribute__((aligned(16))) uint8_t rows[kRows + kSpan][kCols];
    __shared__ uint32_t frows[kRows + kSpan][kCols / 32 + 1];   // padded: rows 9 words apart
    __shared__ int32_t dl[kCols];
    __shared__ int32_t red[2][kTileThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // channels vary fastest: workgroups that run together read and write
    // whole sample rows (F x N contiguous bytes) rather than 256-byte pieces
    // a row apart
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
    dl[tid] = d;
    int lo = tid < ni ? d : INT32_MAX, hi = tid < ni ? d : INT32_MIN;
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o));
        hi = max(hi, __shfl_xor(hi, o));
    }
    if (lane == 0) {
        red[0][wave] = lo;
        red[1][wave] = hi;
    }
    __syncthreads();
    lo = red[0][0];
    hi = red[1][0];
    for (int k = 1; k < kTileThreads / 64; ++k) {
        lo = min(lo, red[0][k]);
        hi = max(hi, red[1][k]);
    }
    const bool staged = (int64_t)hi - lo <= kSpan;
    // source rows t - d for t in [t0, t0 + nt) and d in [lo, hi]: [t0 - hi, t0 + nt - 1 - lo]
    const int64_t s0 = (int64_t)t0 - hi;
    const int nrows = staged ? nt + (hi - lo) : 0;
    const int wbase = i0 / 32, nw = (ni + 31) / 32;

    if (staged) {
        if (kVec) {
            // ni is a multiple of 16 here
            const int pieces = ni / 16;
            for (int e = tid; e < nrows * pieces; e += kTileThreads) {
                const int r = e / pieces, q = e % pieces;
                const int64_t src = s0 + r;
                uint4 v = {0u, 0u, 0u, 0u};
                if (src >= 0 && src < T)
                    v = *(const uint4 *)(in + (src * F + f) * N + i0 + 16 * q);
                *(uint4 *)&rows[r][16 * q] = v;
            }
        } else {
            for (int e = tid; e < nrows * kCols; e += kTileThreads) {
                const int r = e / kCols, c = e % kCols;
                const int64_t src = s0 + r;
                rows[r][c] = (c < ni && src >= 0 && src < T) ? in[(src * F + f) * N + i0 + c] : 0;
            }
        }
        if (flags_out)
            for (int e = tid; e < nrows * (kCols / 32); e += kTileThreads) {
                const int r = e / (kCols / 32), w = e % (kCols / 32);
                const int64_t src = s0 + r;
                frows[r][w] = (flags_in && w < nw && src >= 0 && src < T)
                                  ? flags_in[((int64_t)f * T + src) * W + wbase + w]
                                  : 0u;
            }
        __syncthreads();
    }

    // data: thread tid keeps input quad tid % 64 (its 4 delays in registers)
    // and walks rows tid / 64, +4, ...; one dword each (kVec), else bytes
    if (kVec) {
        const int g = tid & 63, quads = ni / 4;
        if (g < quads) {
            // per input: rows r of the tile whose source lies in the frame,
            // rlo <= r < rhi, and the staged row of r, r + base
            int dk[4], rlo[4], rhi[4], base[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                dk[k] = dl[4 * g + k];
                const int64_t l = (int64_t)dk[k] - t0, u = (int64_t)T + dk[k] - t0;
                rlo[k] = (int)(l < 0 ? 0 : (l > nt ? nt : l));
                rhi[k] = (int)(u < 0 ? 0 : (u > nt ? nt : u));
                base[k] = staged ? hi - dk[k] : 0;   // in [0, kSpan] when staged
            }
            for (int r = tid >> 6; r < nt; r += kTileThreads / 64) {
                const int t = t0 + r;
                uint32_t v = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int c = 4 * g + k;
                    uint32_t byte = 0x88u;
                    if (r >= rlo[k] && r < rhi[k])
                        byte = staged ? rows[r + base[k]][c]
                                      : in[((int64_t)(t - dk[k]) * F + f) * N + i0 + c];
                    v |= byte << (8 * k);
                }
                *(uint32_t *)(out + ((int64_t)t * F + f) * N + i0 + 4 * g) = v;
            }
        }
    } else {
        for (int c = tid; c < ni; c += kTileThreads) {
            const int dc = dl[c];
            for (int r = 0; r < nt; ++r) {
                const int t = t0 + r;
                const int64_t src = (int64_t)t - dc;
                uint8_t v = 0x88;
                if (src >= 0 && src < T)
                    v = staged ? rows[r + hi - dc][c] : in[(src * F + f) * N + i0 + c];
                out[((int64_t)t * F + f) * N + i0 + c] = v;
            }
        }
    }
    // flags: half-wave h (of 8) owns word column h of the tile; lane b holds
    // input 32 h + b and its delay, and each row's word is one ballot
    if (flags_out) {
        const int half = lane >> 5, bit = lane & 31;
        const int w = wave * 2 + half;
        if (w < nw) {
            const int c = 32 * w + bit;
            const bool inb = c < ni;
            const int dc = inb ? dl[c] : 0;
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
                                staged ? frows[r + base][w]
                                       : flags_in[((int64_t)f * T + (t0 + r - dc)) * W + wbase + w];
                            set[u] = (word >> bit) & 1u;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const unsigned long long m = __ballot(set[u]);
                    if (bit == 0 && r0 + u < nt)
                        flags_out[((int64_t)f * T + t0 + r0 + u) * W + wbase + w] =
                            (uint32_t)(m >> (32 * half));
                }
            }
        }
    }
}

}  // namespace shift
}  // namespace xe
