// xcorr_kernels.hpp -- gfx950 kernels of the correlator.
//
// Correlation (Sec. II-B: cross-correlate every input pair of a channel and
// add into the previous output):
//   x = a + i b.  With the real K-vector of one input laid out as the pairs
//   (a_t, b_t) and the derived vector (b_t, -a_t),
//     Re V_ij = sum_k Xr_i[k] Xr_j[k]      Im V_ij = sum_k Xp_i[k] Xr_j[k]
//   with Xr = (a, b), Xp = (b, -a): two real int8 GEMMs with K = 2T on the
//   matrix cores, exact int32 accumulation.  Only tiles with I <= J run.
//
// Per staged step of 32 samples a workgroup
//   1. loads the packed bytes of its input blocks (coalesced dword loads
//      along the input axis), substitutes 0x88 (= 0) for lost samples and
//      for samples past the end of its time chunk, transposes 4x4 byte
//      blocks in registers so each dword holds 4 samples of one input, and
//      decodes nibbles to signed int8 with carry-free SWAR arithmetic;
//   2. writes them to LDS in the operand layout of
//      v_mfma_i32_32x32x32_i8: per block, per 16-sample sub-step, lane l
//      reads 16 bytes = 8 samples of input (l % 32), (a a a a a a a a
//      b b b b b b b b); both operands use the same K order, so the order of
//      samples inside K does not matter for the sum;
//   3. each wave runs its tiles: the A operand (rows) in Xr and Xp form,
//      the B operand (columns) in Xr form.
// At the end each lane adds its accumulators into the packed triangle with
// integer atomics (exact, any order), which also merges time chunks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.hpp"

namespace xe {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kSlotBytes = kBlk * kStep * 2;  // decoded bytes per block per step
constexpr int kBufBytes = kSlotBytes * kMaxSlots;

struct CorrArgs {
    const uint8_t *packed;
    const uint8_t *mask;  // may be null
    int32_t *vis;
    int64_t *count;
    int N, F, T, B;
    int nblk_mask;        // ceil(T / B)
    int nb;               // ceil(N / 32)
    int groups;           // groups per channel
    int splits;
    int steps_per_split;
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

// Xr fragment (a0..7 | b0..7) -> Xp fragment (b0..7 | -a0..7)
__device__ __forceinline__ v4i make_xp(v4i x) {
    v4i p;
    p.x = x.z;
    p.y = x.w;
    p.z = (int)neg_s8((uint32_t)x.x);
    p.w = (int)neg_s8((uint32_t)x.y);
    return p;
}

// ---------------------------------------------------------------------------
// staging: global packed bytes -> decoded int8 operand layout in LDS
// ---------------------------------------------------------------------------

// 4 consecutive input bytes of one sample; out-of-range or invalid bytes
// read a safe address and are replaced by 0x88 (= 0), without branches
template <bool kAligned>
__device__ __forceinline__ uint32_t load4(const uint8_t *packed, int64_t row_off, int n0,
                                          int N, bool ok) {
    if (kAligned) {
        // N % 4 == 0: the dword is either wholly inside [0, N) or wholly out
        bool in = ok && n0 < N;
        const uint32_t *p = (const uint32_t *)(packed + (in ? row_off + n0 : 0));
        uint32_t v = *p;
        return in ? v : 0x88888888u;
    } else {
        uint32_t v = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            bool in = ok && n0 + c < N;
            uint32_t b = packed[in ? row_off + n0 + c : 0];
            v |= (in ? b : 0x88u) << (8 * c);
        }
        return v;
    }
}

// validity of samples tb .. tb+31 of channel f within [.., t_end) as a
// wave-uniform bit mask
__device__ __forceinline__ uint32_t step_valid_bits(const CorrArgs &a, int f, int tb,
                                                    int t_end) {
    int lane = threadIdx.x & 63;
    int t = tb + (lane & 31);
    bool ok = lane < 32 && t < t_end;
    if (ok && a.mask) ok = a.mask[(int64_t)f * a.nblk_mask + t / a.B] == 0;
    return (uint32_t)__ballot(ok);
}

// One staging unit: 4 inputs (n0..n0+3) x 8 samples (octet o of the step)
// of slot s.  Loads 8 dwords, transposes to 4 inputs x 8 samples, decodes
// and writes four 16-byte operand chunks.
template <bool kAligned>
__device__ __forceinline__ void stage_unit(const CorrArgs &a, int f, int tb, uint32_t vbits,
                                           int s, int q, int o, int n0, bool active,
                                           uint8_t *buf) {
    uint32_t d[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int t = tb + 8 * o + e;
        bool ok = active && ((vbits >> (8 * o + e)) & 1u);
        int64_t row_off = ((int64_t)t * a.F + f) * a.N;
        d[e] = load4<kAligned>(a.packed, row_off, n0, a.N, ok);
    }
    uint32_t lo[4], hi[4];
    transpose4(d, lo);
    transpose4(d + 4, hi);
    if (active) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            v4i frag;
            frag.x = (int)nib_to_s8((lo[c] >> 4) & 0x0f0f0f0fu);
            frag.y = (int)nib_to_s8((hi[c] >> 4) & 0x0f0f0f0fu);
            frag.z = (int)nib_to_s8(lo[c] & 0x0f0f0f0fu);
            frag.w = (int)nib_to_s8(hi[c] & 0x0f0f0f0fu);
            int r = 4 * q + c;
            *(v4i *)(buf + s * kSlotBytes + (o * kBlk + r) * 16) = frag;
        }
    }
}

// ---------------------------------------------------------------------------
// the correlation kernel
// ---------------------------------------------------------------------------

// Main loop of one wave with NA tiles on row slot A and NB on row slot B
// (compile-time counts, so every accumulator index is static).
template <bool kAligned, int NA, int NB>
__device__ __forceinline__ void run_wave(const CorrArgs &a, const Group &g, int f,
                                         int t_begin, int t_end, int rowA, int colA0,
                                         int rowB, int colB0, uint8_t *lds) {
    constexpr int NT = NA + NB;
    const int lane = threadIdx.x & 63;

    // staging units of this thread (at most two per step)
    const int units = g.nslots * 32;
    int us[2], uq[2], uo[2], un0[2];
    bool uact[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        int u = threadIdx.x + r * kThreads;
        uact[r] = u < units;
        uq[r] = u & 7;
        us[r] = (u >> 3) % g.nslots;
        uo[r] = (u >> 3) / g.nslots;
        un0[r] = slot_block(g, us[r]) * kBlk + 4 * uq[r];
    }
    const bool two_rounds = units > kThreads;

    v16i acc_re[NT], acc_im[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        acc_re[k] = (v16i){0};
        acc_im[k] = (v16i){0};
    }

    for (int tb = t_begin; tb < t_end; tb += kStep) {
        uint32_t vbits = step_valid_bits(a, f, tb, t_end);
        stage_unit<kAligned>(a, f, tb, vbits, us[0], uq[0], uo[0], un0[0], uact[0], lds);
        if (two_rounds)
            stage_unit<kAligned>(a, f, tb, vbits, us[1], uq[1], uo[1], un0[1], uact[1], lds);
        __syncthreads();
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            const uint8_t *base = lds + sub * (kBlk * 2 * 16) + lane * 16;
            v4i xa = *(const v4i *)(base + rowA * kSlotBytes);
            v4i pa = make_xp(xa);
            v4i xb = xa, pb = pa;
            if (NB > 0) {
                xb = *(const v4i *)(base + rowB * kSlotBytes);
                pb = make_xp(xb);
            }
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                int cs = k < NA ? colA0 + k : colB0 + (k - NA);
                v4i y = *(const v4i *)(base + cs * kSlotBytes);
                if (k < NA) {
                    acc_re[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa, y, acc_re[k], 0, 0, 0);
                    acc_im[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(pa, y, acc_im[k], 0, 0, 0);
                } else {
                    acc_re[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xb, y, acc_re[k], 0, 0, 0);
                    acc_im[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(pb, y, acc_im[k], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    // epilogue: add the tiles into the packed upper triangle
    const int64_t P = (int64_t)a.N * (a.N + 1) / 2;
    int32_t *visf = a.vis + (int64_t)f * P * 2;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        int rs = k < NA ? rowA : rowB;
        int cs = k < NA ? colA0 + k : colB0 + (k - NA);
        int I = slot_block(g, rs), J = slot_block(g, cs);
        int j = J * kBlk + (lane & 31);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            int i = I * kBlk + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            if (i <= j && j < a.N) {
                int64_t idx = (int64_t)i * a.N - (int64_t)i * (i - 1) / 2 + (j - i);
                atomicAdd(&visf[2 * idx], acc_re[k][v]);
                atomicAdd(&visf[2 * idx + 1], acc_im[k][v]);
            }
        }
    }
}

template <bool kAligned>
__global__ __launch_bounds__(kThreads, 1) void corr_kernel(CorrArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kBufBytes];

    const int G = a.groups;
    int64_t wg = blockIdx.x;
    const int gid = (int)(wg % G);
    wg /= G;
    const int split = (int)(wg % a.splits);
    const int f = (int)(wg / a.splits);

    const Group g = make_group(a.nb, gid);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const int t_begin = split * a.steps_per_split * kStep;
    int t_end = t_begin + a.steps_per_split * kStep;
    if (t_end > a.T) t_end = a.T;

    // Every wave runs the same number of steps and barriers; the tile
    // pattern is fixed per group kind (blocks past N are staged as zeros).
    if (g.diag) {
        // rows w and 7-w of the 8-block triangle
        const int rA = wave, rB = 7 - wave;
        switch (wave) {
            case 0: run_wave<kAligned, 8, 1>(a, g, f, t_begin, t_end, rA, rA, rB, rB, lds); break;
            case 1: run_wave<kAligned, 7, 2>(a, g, f, t_begin, t_end, rA, rA, rB, rB, lds); break;
            case 2: run_wave<kAligned, 6, 3>(a, g, f, t_begin, t_end, rA, rA, rB, rB, lds); break;
            default: run_wave<kAligned, 5, 4>(a, g, f, t_begin, t_end, rA, rA, rB, rB, lds); break;
        }
    } else {
        // rows 2(w/2), 2(w/2)+1 x column slots 4 + 4(w%2) .. +3
        const int rA = 2 * (wave / 2), c0 = 4 + 4 * (wave % 2);
        run_wave<kAligned, 4, 4>(a, g, f, t_begin, t_end, rA, c0, rA + 1, c0, lds);
    }

    // valid samples of this chunk, once per (channel, chunk)
    if (gid == 0 && threadIdx.x == 0) {
        int64_t n = 0;
        if (a.mask == nullptr) {
            n = t_end - t_begin;
        } else {
            for (int b = t_begin / a.B; b * (int64_t)a.B < t_end; ++b) {
                int64_t lo = (int64_t)b * a.B, hi = lo + a.B;
                if (lo < t_begin) lo = t_begin;
                if (hi > t_end) hi = t_end;
                if (a.mask[(int64_t)f * a.nblk_mask + b] == 0) n += hi - lo;
            }
        }
        atomicAdd((unsigned long long *)&a.count[f], (unsigned long long)n);
    }
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

__global__ void zero_kernel(int32_t *vis, int64_t n_vis, int64_t *count, int F) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_vis; k += stride)
        vis[k] = 0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < F; k += stride)
        count[k] = 0;
}

// out = (float)((double)v / (double)n), 0 when n == 0
__global__ void normalize_kernel(const int32_t *vis, const int64_t *count, float *out,
                                 int64_t per_channel, int F) {
    int64_t total = per_channel * F;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total; k += stride) {
        int64_t n = count[k / per_channel];
        out[k] = n == 0 ? 0.0f : (float)((double)vis[k] / (double)n);
    }
}

}  // namespace xe
