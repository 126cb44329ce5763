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

// One thread per 4 inputs of one (sample, channel): four byte gathers, one
// dword store (kVec: N % 4 == 0 and both frames 4-byte aligned), else one
// byte per thread.
template <bool kVec>
__global__ void data_kernel(const uint8_t *in, const int32_t *delays, uint8_t *out, int N,
                            int F, int T) {
    const int per = kVec ? N / 4 : N;
    const int64_t total = (int64_t)T * F * per;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += stride) {
        const int g = (int)(e % per);
        const int64_t tf = e / per;
        const int f = (int)(tf % F);
        const int64_t t = tf / F;
        if (kVec) {
            uint32_t v = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int i = 4 * g + c;
                const int64_t src = t - delays[i];
                const uint32_t b = (src >= 0 && src < T) ? in[(src * F + f) * N + i] : 0x88u;
                v |= b << (8 * c);
            }
            *(uint32_t *)(out + (t * F + f) * N + 4 * g) = v;
        } else {
            const int64_t src = t - delays[g];
            out[(t * F + f) * N + g] = (src >= 0 && src < T) ? in[(src * F + f) * N + g]
                                                             : (uint8_t)0x88;
        }
    }
}

// One thread per flag word: bit b (input 32 w + b < N) is the source
// sample's F-engine flag, or 1 when the source lies outside the frame.
__global__ void flag_kernel(const uint32_t *flags_in, const int32_t *delays, uint32_t *flags_out,
                            int N, int F, int T, int W) {
    const int64_t total = (int64_t)F * T * W;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += stride) {
        const int w = (int)(e % W);
        const int64_t ft = e / W;
        const int64_t t = ft % T, f = ft / T;
        uint32_t v = 0;
        for (int b = 0; b < 32 && 32 * w + b < N; ++b) {
            const int64_t src = t - delays[32 * w + b];
            uint32_t bit = 1u;
            if (src >= 0 && src < T)
                bit = flags_in ? (flags_in[(f * T + src) * W + w] >> b) & 1u : 0u;
            v |= bit << b;
        }
        flags_out[e] = v;
    }
}

}  // namespace shift
}  // namespace xe
