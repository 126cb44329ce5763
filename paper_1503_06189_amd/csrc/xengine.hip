// xengine.hip -- the C ABI of the correlator (declared in include/xengine.h):
// argument checks, launch planning and kernel launches on the caller's
// stream.  Nothing here allocates after xe_create.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

#include "../../include/xengine.h"
#include "plan.hpp"
#include "xcorr_kernels.hpp"

struct xe_handle_s {
    int device;          // XE_DEVICE_NONE for a validation-only handle
    int n_cu;
    void *workspace;
    size_t workspace_bytes;
    std::string last_error;
};

namespace {

xe_status fail(xe_handle h, xe_status s, const char *what) {
    if (h) h->last_error = what;
    return s;
}

xe_status hip_fail(xe_handle h, hipError_t e, const char *where) {
    if (h) {
        h->last_error = where;
        h->last_error += ": ";
        h->last_error += hipGetErrorString(e);
    }
    return XE_ERR_HIP;
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

xe_status check_shape(xe_handle h, int32_t N, int32_t F, int32_t T, int32_t B) {
    if (N < 1 || N > XE_MAX_N) return fail(h, XE_ERR_ARG, "N must be in [1, 4096]");
    if (F < 1) return fail(h, XE_ERR_ARG, "F must be >= 1");
    if (T < 1) return fail(h, XE_ERR_ARG, "T must be >= 1");
    if (B < 1) return fail(h, XE_ERR_ARG, "B must be >= 1");
    if (T > XE_MAX_SAMPLES) return fail(h, XE_ERR_OVERFLOW, "T exceeds XE_MAX_SAMPLES");
    int64_t P = (int64_t)N * (N + 1) / 2;
    if ((int64_t)F * P * 2 > ((int64_t)1 << 40)) return fail(h, XE_ERR_ARG, "F*P too large");
    if ((int64_t)T * F * N > ((int64_t)1 << 40)) return fail(h, XE_ERR_ARG, "frame too large");
    // a staged step of 32 samples must stay addressable with 32-bit offsets
    if ((int64_t)F * N * xe::kStep >= ((int64_t)1 << 30))
        return fail(h, XE_ERR_ARG, "F*N too large for one call");
    return XE_OK;
}

xe_status check_frame(xe_handle h, const uint8_t *packed, int32_t N, int32_t F, int32_t T,
                      int32_t B, const int32_t *vis, const int64_t *count) {
    if (!h) return XE_ERR_ARG;
    xe_status s = check_shape(h, N, F, T, B);
    if (s != XE_OK) return s;
    if (!packed || !vis || !count) return fail(h, XE_ERR_ARG, "null pointer");
    if (!aligned(vis, 8) || !aligned(count, 8)) return fail(h, XE_ERR_ALIGN, "vis/count not 8-byte aligned");
    return XE_OK;
}

// Workspace layout: [counters: kCounterBytes][partial accumulators ...]
constexpr size_t kCounterBytes = 1u << 20;
constexpr int64_t kMaxKeys = kCounterBytes / sizeof(int32_t);

size_t partial_bytes(int64_t keys, int splits) {
    return splits > 1 ? (size_t)keys * splits * xe::kGroupPartial * sizeof(int32_t) : 0;
}

// Returns false when time chunks are unavoidable but their partial sums do
// not fit the workspace.
bool fill_plan(int32_t N, int32_t F, int32_t T, int32_t n_cu, size_t ws_bytes,
               xe_plan_info *p) {
    int nb = xe::ceil_div(N, xe::kBlk);
    int G = xe::groups_per_channel(nb);
    int steps = xe::ceil_div(T, xe::kStep);
    int splits, sps;
    int64_t keys = (int64_t)F * G;
    xe::choose_split(keys, steps, n_cu, &splits, &sps);
    // Chunk limits: the byte offsets inside a chunk stay below 2^31, and a
    // diagonal tile's Q (at most 248 per sample) stays within int32.
    const int64_t step_bytes = (int64_t)F * N * xe::kStep;
    int64_t max_sps = (((int64_t)1 << 31) - 1) / step_bytes - 1;
    if (max_sps > xe::kMaxStepsPerChunk) max_sps = xe::kMaxStepsPerChunk;
    if (sps > max_sps) {
        sps = (int)max_sps;
        splits = xe::ceil_div(steps, sps);
    }
    // fewer chunks when their partial sums do not fit the workspace
    while (splits > 1 && (keys > kMaxKeys || kCounterBytes + partial_bytes(keys, splits) > ws_bytes)) {
        int want = splits - 1;
        int next = xe::ceil_div(steps, want);
        if (next > max_sps) break;  // cannot merge chunks any further
        sps = next;
        splits = xe::ceil_div(steps, sps);
    }
    p->blocks = nb;
    p->groups = G;
    p->splits = splits;
    p->steps_per_split = sps;
    p->workgroups = keys * splits;
    p->mfma_tiles = xe::tiles_per_channel(nb);
    return splits == 1 ||
           (keys <= kMaxKeys && kCounterBytes + partial_bytes(keys, splits) <= ws_bytes);
}

xe_status launch_corr(xe_handle h, const uint8_t *packed, const uint8_t *mask, int32_t N,
                      int32_t F, int32_t T, int32_t B, int32_t *vis, int64_t *count,
                      bool overwrite, hipStream_t stream) {
    xe_plan_info p;
    if (!fill_plan(N, F, T, h->n_cu, h->workspace_bytes, &p))
        return fail(h, XE_ERR_WORKSPACE, "time chunks do not fit the workspace");
    xe::CorrArgs a;
    a.packed = packed;
    a.mask = mask;
    a.vis = vis;
    a.count = count;
    a.counters = (int32_t *)h->workspace;
    a.partials = (int32_t *)((char *)h->workspace + kCounterBytes);
    a.N = N;
    a.F = F;
    a.T = T;
    a.B = B;
    a.nblk_mask = xe::ceil_div(T, B);
    a.nb = p.blocks;
    a.groups = p.groups;
    a.splits = p.splits;
    a.steps_per_split = p.steps_per_split;
    if (p.workgroups > 0x7fffffff) return fail(h, XE_ERR_ARG, "too many workgroups");
    dim3 grid((unsigned)p.workgroups), block(xe::kThreads);
    bool al = aligned(packed, 4) && (N % 4 == 0);
    if (al && overwrite)
        hipLaunchKernelGGL((xe::corr_kernel<true, true>), grid, block, 0, stream, a);
    else if (al)
        hipLaunchKernelGGL((xe::corr_kernel<true, false>), grid, block, 0, stream, a);
    else if (overwrite)
        hipLaunchKernelGGL((xe::corr_kernel<false, true>), grid, block, 0, stream, a);
    else
        hipLaunchKernelGGL((xe::corr_kernel<false, false>), grid, block, 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "correlation launch");
    return XE_OK;
}

}  // namespace

extern "C" {

xe_status xe_create(xe_handle *out, int32_t hip_device, size_t workspace_bytes) {
    if (!out) return XE_ERR_ARG;
    *out = nullptr;
    xe_handle h = new (std::nothrow) xe_handle_s();
    if (!h) return XE_ERR_ARG;
    h->device = hip_device;
    h->n_cu = 256;
    h->workspace = nullptr;
    h->workspace_bytes = 0;
    if (hip_device == XE_DEVICE_NONE) {
        *out = h;
        return XE_OK;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || hip_device < 0 || hip_device >= ndev) {
        delete h;
        return XE_ERR_HIP;
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, hip_device);
    if (e != hipSuccess) {
        delete h;
        return XE_ERR_HIP;
    }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        delete h;
        return XE_ERR_UNSUPPORTED;
    }
    h->n_cu = prop.multiProcessorCount;
    if (workspace_bytes == 0) workspace_bytes = (size_t)256 << 20;
    if (workspace_bytes < kCounterBytes) workspace_bytes = kCounterBytes;
    {
        DeviceGuard g(hip_device);
        if (!g.ok) {
            delete h;
            return XE_ERR_HIP;
        }
        e = hipMalloc(&h->workspace, workspace_bytes);
        if (e != hipSuccess) {
            delete h;
            return XE_ERR_HIP;
        }
        // arrival counters start at zero; every launch leaves them at zero
        e = hipMemset(h->workspace, 0, kCounterBytes);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            (void)hipFree(h->workspace);
            delete h;
            return XE_ERR_HIP;
        }
    }
    h->workspace_bytes = workspace_bytes;
    *out = h;
    return XE_OK;
}

xe_status xe_destroy(xe_handle h) {
    if (!h) return XE_OK;
    if (h->workspace) {
        DeviceGuard g(h->device);
        (void)hipFree(h->workspace);
    }
    delete h;
    return XE_OK;
}

const char *xe_status_string(xe_status s) {
    switch (s) {
        case XE_OK: return "ok";
        case XE_ERR_ARG: return "invalid argument";
        case XE_ERR_ALIGN: return "misaligned pointer";
        case XE_ERR_OVERFLOW: return "integration too long for int32 sums";
        case XE_ERR_WORKSPACE: return "workspace too small";
        case XE_ERR_HIP: return "HIP runtime error";
        case XE_ERR_UNSUPPORTED: return "device is not gfx950";
        case XE_ERR_NO_DEVICE: return "validation-only handle";
        default: return "unknown status";
    }
}

const char *xe_last_error(xe_handle h) { return h ? h->last_error.c_str() : ""; }

xe_status xe_plan_query(int32_t N, int32_t F, int32_t T, int32_t B, int32_t n_cu,
                        xe_plan_info *info) {
    if (!info) return XE_ERR_ARG;
    xe_status s = check_shape(nullptr, N, F, T, B);
    if (s != XE_OK) return s;
    if (n_cu < 1) return XE_ERR_ARG;
    if (!fill_plan(N, F, T, n_cu, (size_t)256 << 20, info)) return XE_ERR_WORKSPACE;
    return XE_OK;
}

xe_status xe_accumulate(xe_handle h, const uint8_t *packed, const uint8_t *loss_mask,
                        int32_t N, int32_t F, int32_t T, int32_t B, int32_t *vis,
                        int64_t *count, void *stream) {
    xe_status s = check_frame(h, packed, N, F, T, B, vis, count);
    if (s != XE_OK) return s;
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    return launch_corr(h, packed, loss_mask, N, F, T, B, vis, count, false,
                       (hipStream_t)stream);
}

xe_status xe_correlate_frame(xe_handle h, const uint8_t *packed, const uint8_t *loss_mask,
                             int32_t N, int32_t F, int32_t T, int32_t B, int32_t *vis,
                             int64_t *count, void *stream) {
    xe_status s = check_frame(h, packed, N, F, T, B, vis, count);
    if (s != XE_OK) return s;
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    return launch_corr(h, packed, loss_mask, N, F, T, B, vis, count, true,
                       (hipStream_t)stream);
}

xe_status xe_normalize(xe_handle h, const int32_t *vis, const int64_t *count, int32_t N,
                       int32_t F, float *out, void *stream) {
    if (!h) return XE_ERR_ARG;
    xe_status s = check_shape(h, N, F, 1, 1);
    if (s != XE_OK) return s;
    if (!vis || !count || !out) return fail(h, XE_ERR_ARG, "null pointer");
    if (!aligned(vis, 8) || !aligned(count, 8) || !aligned(out, 8))
        return fail(h, XE_ERR_ALIGN, "vis/count/out not 8-byte aligned");
    int64_t per = (int64_t)N * (N + 1);
    const char *vb = (const char *)vis, *ob = (const char *)out;
    if (ob < vb + per * F * 4 && vb < ob + per * F * 4)
        return fail(h, XE_ERR_ARG, "vis and out overlap");
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    int64_t total = per * F;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (aligned(vis, 16) && aligned(out, 16))
        hipLaunchKernelGGL(xe::normalize_kernel<true>, dim3((unsigned)blocks), dim3(256), 0,
                           (hipStream_t)stream, vis, count, out, per, F);
    else
        hipLaunchKernelGGL(xe::normalize_kernel<false>, dim3((unsigned)blocks), dim3(256), 0,
                           (hipStream_t)stream, vis, count, out, per, F);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "normalize launch");
    return XE_OK;
}

xe_status xe_accumulate_batch(xe_handle h, const xe_instance *inst, int32_t n_inst,
                              void *stream) {
    if (!h || !inst || n_inst < 0) return fail(h, XE_ERR_ARG, "bad batch arguments");
    for (int32_t k = 0; k < n_inst; ++k) {
        const xe_instance &x = inst[k];
        xe_status s = check_frame(h, x.packed, x.N, x.F, x.T, x.B, x.vis, x.count);
        if (s != XE_OK) return s;
    }
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    for (int32_t k = 0; k < n_inst; ++k) {
        const xe_instance &x = inst[k];
        xe_status s = xe_accumulate(h, x.packed, x.loss_mask, x.N, x.F, x.T, x.B, x.vis,
                                    x.count, stream);
        if (s != XE_OK) return s;
    }
    return XE_OK;
}

}  // extern "C"
