// assemble_kernels.hpp -- gfx950 kernels that build a frame from F-engine
// UDP packets (Sec. II-A).
//
// The network thread of the method places every packet's data by its
// sequence number, writes zeros where a packet is missing, puts packets
// that arrive out of order in their own place and ignores duplicates.
// Here a batch of raw packets already in device memory (one host-to-device
// copy of the receive ring) is placed by four launches:
//   reset  owner[stream][slot] = "none", counters = 0;
//   claim  one thread per packet reads its header, checks stream, window
//          and input count, and takes its (stream, slot) with an atomic
//          minimum of its arrival index: the first arrival wins whatever
//          order the threads run in, so duplicates are ignored;
//   place  one workgroup per (stream, slot) copies the winner's 4 samples x
//          8 bands of data into the frame and its footer flag words into
//          the channel-major flag array, or, when no packet arrived, writes
//          0 + 0i (byte 0x88), no flags and a lost block in the mask;
//   count  places filled and left empty, from the owner table.
// Every output element is written, so buffers need no clearing between
// frames.  Packet layout: 16-byte header (uint64 sequence number, uint32
// stream id, uint32 input count N), data [4][8][N] bytes, footer
// [4][8][ceil(N/32)] uint32 flag words.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xe {
namespace pkt {

constexpr int kSamples = 4;
constexpr int kBands = 8;
constexpr int kHeader = 16;
constexpr int kPlaceThreads = 256;
constexpr int32_t kNone = 0x7fffffff;

struct Args {
    const uint8_t *packets;
    int64_t n_packets;
    int64_t pbytes;          // bytes per packet
    int N, W, n_streams, stream_base;
    int64_t seq0;
    int T, slots;            // slots = T / 4
    uint8_t *packed;         // [T][8 n_streams][N]
    uint8_t *mask;           // [8 n_streams][slots]
    uint32_t *flags;         // [8 n_streams][T][W], may be null
    int32_t *owner;          // [n_streams][slots]
    unsigned long long *stats;  // [6]
};

__global__ void reset_kernel(int32_t *owner, int64_t n, unsigned long long *stats) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += stride)
        owner[k] = kNone;
    if (blockIdx.x == 0 && threadIdx.x < 6) stats[threadIdx.x] = 0ull;
}

// Counters are summed per workgroup in LDS and added to the device counters
// once per workgroup: thousands of atomics on one address would serialise.
__device__ __forceinline__ void count_lds(unsigned int *c, bool pred) {
    const unsigned long long m = __ballot(pred);
    if (m != 0ull && (threadIdx.x & 63) == (unsigned)__ffsll((long long)m) - 1u)
        atomicAdd(c, (unsigned int)__popcll(m));
}

// a little-endian word at a 4-byte aligned address inside a packet (the
// batch is 4-byte aligned and a packet's size is a multiple of 4)
__device__ __forceinline__ uint32_t le32(const uint8_t *p) { return *(const uint32_t *)p; }

__global__ void claim_kernel(Args a) {
    __shared__ unsigned int c[4];
    if (threadIdx.x < 4) c[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool in_window = false, out_window = false, unknown = false, malformed = false;
    if (p < a.n_packets) {
        const uint8_t *h = a.packets + p * a.pbytes;
        const uint64_t seq = (uint64_t)le32(h) | ((uint64_t)le32(h + 4) << 32);
        const uint32_t sid = le32(h + 8), nin = le32(h + 12);
        const int64_t s = (int64_t)sid - a.stream_base;
        if (nin != (uint32_t)a.N) {
            malformed = true;
        } else if (s < 0 || s >= a.n_streams) {
            unknown = true;
        } else if (seq < (uint64_t)a.seq0 || seq - (uint64_t)a.seq0 >= (uint64_t)a.slots) {
            out_window = true;
        } else {
            in_window = true;
            atomicMin(a.owner + s * a.slots + (int64_t)(seq - (uint64_t)a.seq0), (int32_t)p);
        }
    }
    count_lds(c + 0, in_window);
    count_lds(c + 1, out_window);
    count_lds(c + 2, unknown);
    count_lds(c + 3, malformed);
    __syncthreads();
    if (threadIdx.x < 4 && c[threadIdx.x] != 0u)
        atomicAdd(a.stats + threadIdx.x, (unsigned long long)c[threadIdx.x]);
}

// places filled and left empty, from the owner table
__global__ void count_kernel(const int32_t *owner, int64_t n, unsigned long long *stats) {
    __shared__ unsigned int c[2];
    if (threadIdx.x < 2) c[threadIdx.x] = 0u;
    __syncthreads();
    unsigned int filled = 0, empty = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += stride) {
        const bool f = owner[k] != kNone;
        filled += f ? 1u : 0u;
        empty += f ? 0u : 1u;
    }
    atomicAdd(c + 0, filled);
    atomicAdd(c + 1, empty);
    __syncthreads();
    if (threadIdx.x < 2 && c[threadIdx.x] != 0u)
        atomicAdd(stats + 4 + threadIdx.x, (unsigned long long)c[threadIdx.x]);
}

// kVec: 16-byte copies (N even, frame and packets 16-byte aligned)
template <bool kVec>
__global__ __launch_bounds__(kPlaceThreads) void place_kernel(Args a) {
    // streams vary fastest: workgroups that run together read packets that
    // arrived side by side and write whole sample rows of the frame
    const int64_t q = blockIdx.x;
    const int s = (int)(q % a.n_streams), k = (int)(q / a.n_streams);
    const int32_t p = a.owner[(int64_t)s * a.slots + k];
    const bool lost = p == kNone;
    const int F = kBands * a.n_streams;
    const uint8_t *pkt = lost ? nullptr : a.packets + (int64_t)p * a.pbytes;
    const int run = kBands * a.N;   // bytes of one sample's 8 bands, contiguous in both
    if (kVec) {
        // all 4 samples as one index space of 16-byte pieces; kU loads in
        // flight per thread before their stores
        constexpr int kU = 4;
        const int per = run / 16, total = kSamples * per;
        const uint4 zero = {0x88888888u, 0x88888888u, 0x88888888u, 0x88888888u};
        for (int base = threadIdx.x; base < total; base += kPlaceThreads * kU) {
            uint4 v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int idx = base + u * kPlaceThreads;
                const int smp = idx / per, e = idx - smp * per;
                v[u] = (lost || idx >= total)
                           ? zero
                           : ((const uint4 *)(pkt + kHeader + (int64_t)smp * run))[e];
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int idx = base + u * kPlaceThreads;
                if (idx >= total) break;
                const int smp = idx / per, e = idx - smp * per;
                ((uint4 *)(a.packed + ((int64_t)(k * kSamples + smp) * F + kBands * s) * a.N))[e] =
                    v[u];
            }
        }
    } else {
        for (int smp = 0; smp < kSamples; ++smp) {
            uint8_t *dst = a.packed + ((int64_t)(k * kSamples + smp) * F + kBands * s) * a.N;
            const uint8_t *src = lost ? nullptr : pkt + kHeader + (int64_t)smp * run;
            for (int e = threadIdx.x; e < run; e += kPlaceThreads)
                dst[e] = lost ? (uint8_t)0x88 : src[e];
        }
    }
    if (a.flags) {
        const int words = kSamples * kBands * a.W;
        const uint8_t *foot = lost ? nullptr : pkt + kHeader + (int64_t)kSamples * run;
        for (int e = threadIdx.x; e < words; e += kPlaceThreads) {
            const int w = e % a.W, sb = e / a.W, b = sb % kBands, smp = sb / kBands;
            const uint32_t v = lost ? 0u : le32(foot + 4 * (int64_t)e);
            a.flags[((int64_t)(kBands * s + b) * a.T + k * kSamples + smp) * a.W + w] = v;
        }
    }
    if (threadIdx.x < kBands)
        a.mask[(int64_t)(kBands * s + threadIdx.x) * a.slots + k] = lost ? 1 : 0;
}

}  // namespace pkt
}  // namespace xe
