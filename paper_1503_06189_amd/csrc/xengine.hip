// xengine.hip -- the C ABI of the correlator (declared in include/xengine.h):
// argument checks, launch planning and kernel launches on the caller's
// stream.  Nothing here allocates after xe_create.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/xengine.h"
#include "plan.hpp"
#include "xcorr_kernels.hpp"
#include "flag_kernels.hpp"
#include "assemble_kernels.hpp"
#include "shift_kernels.hpp"

// Batch plans live in a device area allocated with the handle: kRingSlots
// slots that xe_accumulate_batch cycles through (each guarded by an event,
// with a pinned host staging copy) and kPlanSlots slots for plans made with
// xe_batch_plan and replayed with xe_batch_run.
constexpr int kRingSlots = 4;
constexpr int kPlanSlots = 4;
constexpr size_t kSlotBytes = (size_t)4 << 20;
constexpr size_t kQueueBytes = 256;  // queue head and done counters, padded

// sizes of a plan kept in a device slot
struct SlotShape {
    int n_inst = 0, n_items = 0, n_small = 0, n_merges = 0;  // n_small: halves items
    int64_t merge_blocks = 0;
};

struct PlanSlot {
    bool used = false;
    SlotShape shape;
    std::vector<xe_instance> unaligned;  // instances run as plain launches
};

struct xe_handle_s {
    int device;          // XE_DEVICE_NONE for a validation-only handle
    int n_cu;
    void *workspace;
    size_t workspace_bytes;
    void *plan_area;     // (kRingSlots + kPlanSlots) x kSlotBytes, device
    void *staging;       // kRingSlots x kSlotBytes, pinned host
    hipEvent_t ring_done[kRingSlots];
    int ring_next;
    PlanSlot slots[kRingSlots + kPlanSlots];
    int geometry;        // XE_GEOM_*: tile geometry of frames with N <= 128
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

// A loss block longer than the frame is one block covering all of it, as a
// block of exactly T samples is: the mask has ceil(T/B) = 1 entry per
// channel either way.  Kernels take the clamped length, so block indices
// and bounds (b * B, (b + 1) * B, T + B - 1) stay far inside int32.
int32_t eff_block(int32_t B, int32_t T) { return B < T ? B : T; }

xe_status check_shape(xe_handle h, int32_t N, int32_t F, int32_t T, int32_t B) {
    if (N < 1 || N > XE_MAX_N) return fail(h, XE_ERR_ARG, "N must be in [1, 4096]");
    if (F < 1) return fail(h, XE_ERR_ARG, "F must be >= 1");
    if (T < 1) return fail(h, XE_ERR_ARG, "T must be >= 1");
    if (B < 1) return fail(h, XE_ERR_ARG, "B must be >= 1");
    if (T > XE_MAX_SAMPLES) return fail(h, XE_ERR_OVERFLOW, "T exceeds XE_MAX_SAMPLES");
    int64_t P = (int64_t)N * (N + 1) / 2;
    if ((int64_t)F * P * 2 > ((int64_t)1 << 40)) return fail(h, XE_ERR_ARG, "F*P too large");
    if ((int64_t)T * F * N > ((int64_t)1 << 40)) return fail(h, XE_ERR_ARG, "frame too large");
    // a chunk with its lookahead must stay addressable with 31-bit offsets
    static_assert((int64_t)XE_MAX_FN * xe::kStep * (2 * xe::kDepth + 2) < ((int64_t)1 << 31),
                  "XE_MAX_FN too large for the prefetch depth");
    if ((int64_t)F * N > XE_MAX_FN) return fail(h, XE_ERR_ARG, "F*N exceeds XE_MAX_FN");
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

// Workspace: the tiles of time chunks 1 .. splits-1 of every chunked tile
// group (chunk 0 writes the output directly), 327,680 B per group and chunk.
// The default leaves room for large batches and is small next to 288 GB.
constexpr size_t kDefaultWorkspace = (size_t)1 << 30;

size_t partial_bytes(int64_t keys, int splits) {
    return splits > 1 ? (size_t)keys * (splits - 1) * xe::kGroupPartial * sizeof(int32_t) : 0;
}

// Returns false when time chunks are unavoidable but their partial sums do
// not fit the workspace.
// the halves geometry for frames of at most 4 input blocks, unless the
// caller asked for padded super-blocks
int halves_of(int geometry) { return geometry == XE_GEOM_SUPER ? 0 : 1; }

bool fill_plan(int32_t N, int32_t F, int32_t T, int32_t n_cu, size_t ws_bytes, int halves,
               xe_plan_info *p) {
    int nb = xe::ceil_div(N, xe::kBlk);
    int G = xe::groups_per_channel(nb);
    int steps = xe::ceil_div(T, xe::kStep);
    int splits, sps;
    int64_t keys = (int64_t)F * G;
    xe::choose_split(keys, steps, n_cu, &splits, &sps);
    // Chunk limits: the byte offsets inside a chunk stay below 2^31, and a
    // diagonal tile's Q (at most 248 per sample) stays within int32.
    const int64_t max_sps = xe::max_steps_per_chunk(F, N);
    if (sps > max_sps) {
        sps = (int)max_sps;
        splits = xe::ceil_div(steps, sps);
    }
    // fewer chunks when their partial sums do not fit the workspace
    while (splits > 1 && partial_bytes(keys, splits) > ws_bytes) {
        int want = splits - 1;
        int next = xe::round_steps(xe::ceil_div(steps, want));
        if (next > max_sps) break;  // cannot merge chunks any further
        sps = next;
        splits = xe::ceil_div(steps, sps);
    }
    p->blocks = nb;
    p->groups = G;
    p->splits = splits;
    p->steps_per_split = sps;
    p->workgroups = keys * splits;
    p->mfma_tiles = xe::tiles_per_channel(nb, halves);
    return splits == 1 || partial_bytes(keys, splits) <= ws_bytes;
}

// Where a correlation call keeps the partial sums of its time chunks: the
// handle's workspace, or the static scratch array of the allocation-free
// entry point.  `h` (may be null) receives the error text.
struct Scratch {
    void *ptr;
    size_t bytes;
    int n_cu;
};

xe_status launch_corr(xe_handle h, const Scratch &ws, const uint8_t *packed, const uint8_t *mask,
                      int32_t N, int32_t F, int32_t T, int32_t B, int32_t *vis, int64_t *count,
                      bool overwrite, hipStream_t stream) {
    xe_plan_info p;
    const int halves = halves_of(h ? h->geometry : XE_GEOM_AUTO);
    if (!fill_plan(N, F, T, ws.n_cu, ws.bytes, halves, &p))
        return fail(h, XE_ERR_WORKSPACE, "time chunks do not fit the workspace");
    xe::CorrArgs a;
    a.packed = packed;
    a.mask = mask;
    a.vis = vis;
    a.count = count;
    a.partials = (int32_t *)ws.ptr;
    a.N = N;
    a.F = F;
    a.T = T;
    B = eff_block(B, T);
    a.B = B;
    a.nblk_mask = xe::ceil_div(T, B);
    a.nb = p.blocks;
    a.groups = p.groups;
    a.splits = p.splits;
    a.steps_per_split = p.steps_per_split;
    a.halves = halves;
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
    // The valid-sample counts run outside the correlation kernel, so that
    // its registers stay with its main loop: in extra blocks of the merge
    // launch when the frame is chunked, else in a launch of their own.
    if (p.splits == 1)
        hipLaunchKernelGGL(xe::count_kernel,
                           dim3((unsigned)((F + xe::kCountWaves - 1) / xe::kCountWaves)),
                           dim3(64 * xe::kCountWaves), 0, stream, mask, a.nblk_mask, B, T, F,
                           count, overwrite ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "correlation launch");
    if (p.splits > 1) {
        // chunks 1.. into the output; stream order makes their tiles visible
        xe::MergeInst m;
        m.vis = vis;
        m.partials = a.partials;
        m.N = N;
        m.nb = p.blocks;
        m.groups = p.groups;
        m.splits = p.splits;
        m.halves = halves;
        m.block_begin = 0;
        const int64_t blocks = (int64_t)F * p.groups * xe::kMergeBlocksPerGroup;
        if (blocks + F > 0x7fffffff) return fail(h, XE_ERR_ARG, "too many merge blocks");
        xe::CountArgs c;
        c.mask = mask;
        c.count = count;
        c.nblk = a.nblk_mask;
        c.B = B;
        c.T = T;
        c.overwrite = overwrite ? 1 : 0;
        c.first_block = blocks;
        hipLaunchKernelGGL(xe::merge_kernel, dim3((unsigned)(blocks + F)), dim3(64), 0, stream, m,
                           c);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(h, e, "merge launch");
    }
    return XE_OK;
}

void release_device_memory(xe_handle h) {
    for (int k = 0; k < kRingSlots; ++k)
        if (h->ring_done[k]) (void)hipEventDestroy(h->ring_done[k]);
    if (h->staging) (void)hipHostFree(h->staging);
    if (h->plan_area) (void)hipFree(h->plan_area);
    if (h->workspace) (void)hipFree(h->workspace);
    h->staging = h->plan_area = h->workspace = nullptr;
}

// ---------------------------------------------------------------------------
// batch planning (host)
// ---------------------------------------------------------------------------

struct BatchPlan {
    std::vector<xe::BatchInstance> inst;
    std::vector<xe::BatchItem> items;        // super-block groups
    std::vector<xe::BatchItem> small_items;  // halves-geometry groups
    std::vector<xe_instance> unaligned;
    std::vector<xe::MergeInst> merges;  // chunked instances, for the merge pass
    std::vector<int64_t> merge_base;    // their first partial value in the workspace
    int chunk_steps = 0;
    int64_t partials = 0;      // int32 partial values used
    int64_t merge_blocks = 0;  // one-wave blocks of the merge pass
};

size_t plan_bytes(const BatchPlan &p) {
    return kQueueBytes + p.inst.size() * sizeof(xe::BatchInstance) +
           (p.items.size() + p.small_items.size()) * sizeof(xe::BatchItem) +
           p.merges.size() * sizeof(xe::MergeInst);
}

// Work items of a batch: every (instance, channel, group, time chunk), with
// time chunks of about `chunk_steps` 32-sample steps (0: enough items for
// about four per compute unit), longest first so the queue drains evenly.
// Fills `plan` with the items of the batch: time chunks of `chunk_steps`
// 32-sample steps, and of `small_chunk` steps for the halves-geometry
// instances, which run in a launch of their own.
xe_status fill_batch(xe_handle h, const xe_instance *inst, int32_t n_inst, int32_t chunk_steps,
                     int32_t small_chunk, int halves, size_t ws_bytes, BatchPlan *plan);

xe_status build_batch(xe_handle h, const xe_instance *inst, int32_t n_inst, int n_cu,
                      int32_t chunk_steps, size_t ws_bytes, BatchPlan *plan) {
    if (n_inst < 0 || (n_inst > 0 && !inst)) return fail(h, XE_ERR_ARG, "bad batch arguments");
    if (chunk_steps < 0) return fail(h, XE_ERR_ARG, "chunk_steps must be >= 0");
    const int halves = halves_of(h->geometry);
    int64_t work = 0, small_work = 0;
    for (int32_t k = 0; k < n_inst; ++k) {
        const xe_instance &x = inst[k];
        xe_status s = check_frame(h, x.packed, x.N, x.F, x.T, x.B, x.vis, x.count);
        if (s != XE_OK) return s;
        int nb = xe::ceil_div(x.N, xe::kBlk);
        const int64_t w = (int64_t)x.F * xe::groups_per_channel(nb) * xe::ceil_div(x.T, xe::kStep);
        work += w;
        if (xe::use_halves(halves, nb) && aligned(x.packed, 4) && x.N % 4 == 0) small_work += w;
    }
    // instances of one launch update their sums without atomics, so their
    // output ranges must be disjoint
    {
        struct Range {
            uintptr_t lo, hi;
        };
        std::vector<Range> r;
        for (int32_t k = 0; k < n_inst; ++k) {
            const xe_instance &x = inst[k];
            uintptr_t v = (uintptr_t)x.vis, c = (uintptr_t)x.count;
            r.push_back({v, v + (uintptr_t)x.F * ((uintptr_t)x.N * (x.N + 1) / 2) * 8});
            r.push_back({c, c + (uintptr_t)x.F * 8});
        }
        std::sort(r.begin(), r.end(), [](const Range &a, const Range &b) { return a.lo < b.lo; });
        for (size_t k = 1; k < r.size(); ++k)
            if (r[k].lo < r[k - 1].hi)
                return fail(h, XE_ERR_ARG, "batch instances share output memory");
    }
    if (chunk_steps == 0) {
        int64_t c = work / (4 * (int64_t)n_cu);
        chunk_steps = (int)std::max<int64_t>(32, std::min<int64_t>(c, xe::kMaxStepsPerChunk));
    }
    // The halves-geometry items drain in a launch of their own after the
    // others: with the common chunk length a few long items would hold it
    // while most compute units idle, so their chunks are cut to about one
    // item per compute unit (never longer than the common length, at least
    // 32 steps), unless the extra chunk sums would not fit the workspace.
    const int32_t small_chunk = (int32_t)std::max<int64_t>(
        32, std::min<int64_t>(chunk_steps, (small_work + n_cu - 1) / n_cu));
    if (small_chunk < chunk_steps) {
        xe_status s = fill_batch(h, inst, n_inst, chunk_steps, small_chunk, halves, ws_bytes, plan);
        if (s != XE_ERR_WORKSPACE) return s;
        *plan = BatchPlan();
    }
    return fill_batch(h, inst, n_inst, chunk_steps, chunk_steps, halves, ws_bytes, plan);
}

xe_status fill_batch(xe_handle h, const xe_instance *inst, int32_t n_inst, int32_t chunk_steps,
                     int32_t small_chunk, int halves, size_t ws_bytes, BatchPlan *plan) {
    plan->chunk_steps = chunk_steps;
    struct Cost {
        int64_t steps;
        xe::BatchItem item;
    };
    std::vector<Cost> costs, small_costs;
    for (int32_t k = 0; k < n_inst; ++k) {
        const xe_instance &x = inst[k];
        if (!aligned(x.packed, 4) || x.N % 4 != 0) {
            plan->unaligned.push_back(x);
            continue;
        }
        const int nb = xe::ceil_div(x.N, xe::kBlk);
        const int G = xe::groups_per_channel(nb);
        const int steps = xe::ceil_div(x.T, xe::kStep);
        const int64_t max_sps = xe::max_steps_per_chunk(x.F, x.N);
        const int32_t cs = xe::use_halves(halves, nb) ? small_chunk : chunk_steps;
        int sps = (int)std::min<int64_t>(std::min<int64_t>(cs, steps), max_sps);
        int splits = xe::ceil_div(steps, sps);
        sps = std::min<int>(xe::round_steps(xe::ceil_div(steps, splits)), (int)max_sps);
        splits = xe::ceil_div(steps, sps);
        xe::BatchInstance b;
        b.packed = x.packed;
        b.mask = x.loss_mask;
        b.vis = x.vis;
        b.count = x.count;
        b.N = x.N;
        b.F = x.F;
        b.T = x.T;
        b.B = eff_block(x.B, x.T);
        b.nblk_mask = xe::ceil_div(x.T, b.B);
        b.nb = nb;
        b.groups = G;
        b.splits = splits;
        b.steps_per_split = sps;
        b.aligned = 1;
        b.halves = halves;
        b.pad_ = 0;
        b.partial_base = plan->partials;
        if (splits > 1) {
            xe::MergeInst m;
            m.vis = x.vis;
            m.partials = nullptr;  // set from the workspace at launch
            m.N = x.N;
            m.nb = nb;
            m.groups = G;
            m.splits = splits;
            m.halves = halves;
            m.pad_ = 0;
            m.block_begin = plan->merge_blocks;
            plan->merges.push_back(m);
            plan->merge_base.push_back(plan->partials);
            plan->merge_blocks += (int64_t)x.F * G * xe::kMergeBlocksPerGroup;
            plan->partials += (int64_t)x.F * G * (splits - 1) * xe::kGroupPartial;
        }
        const int idx = (int)plan->inst.size();
        plan->inst.push_back(b);
        // halves-geometry items go to their own list and launch
        std::vector<Cost> &to = xe::use_halves(halves, nb) ? small_costs : costs;
        for (int f = 0; f < x.F; ++f)
            for (int gid = 0; gid < G; ++gid)
                for (int sp = 0; sp < splits; ++sp) {
                    int64_t len = std::min<int64_t>(sps, steps - (int64_t)sp * sps);
                    to.push_back({len, {idx, f, gid, sp}});
                }
    }
    auto longest_first = [](const Cost &a, const Cost &b) { return a.steps > b.steps; };
    std::stable_sort(costs.begin(), costs.end(), longest_first);
    std::stable_sort(small_costs.begin(), small_costs.end(), longest_first);
    plan->items.reserve(costs.size());
    for (const Cost &c : costs) plan->items.push_back(c.item);
    plan->small_items.reserve(small_costs.size());
    for (const Cost &c : small_costs) plan->small_items.push_back(c.item);
    if ((size_t)plan->partials * sizeof(int32_t) > ws_bytes)
        return fail(h, XE_ERR_WORKSPACE, "batch partial sums do not fit the workspace");
    if (plan->merge_blocks > 0x7fffffff) return fail(h, XE_ERR_ARG, "too many merge blocks");
    if (plan_bytes(*plan) > kSlotBytes) return fail(h, XE_ERR_WORKSPACE, "batch work list too large");
    return XE_OK;
}

// Slot layout: [queues][instances][items][halves items][merge list]; the
// queue area holds two (head, done) pairs, one per item list; the merge
// list's partial pointers are filled in from the handle's workspace.
void write_plan(const BatchPlan &p, int32_t *workspace, char *dst) {
    memset(dst, 0, kQueueBytes);
    char *q = dst + kQueueBytes;
    memcpy(q, p.inst.data(), p.inst.size() * sizeof(xe::BatchInstance));
    q += p.inst.size() * sizeof(xe::BatchInstance);
    memcpy(q, p.items.data(), p.items.size() * sizeof(xe::BatchItem));
    q += p.items.size() * sizeof(xe::BatchItem);
    memcpy(q, p.small_items.data(), p.small_items.size() * sizeof(xe::BatchItem));
    q += p.small_items.size() * sizeof(xe::BatchItem);
    for (size_t k = 0; k < p.merges.size(); ++k) {
        xe::MergeInst m = p.merges[k];
        m.partials = workspace + p.merge_base[k];
        memcpy(q, &m, sizeof m);
        q += sizeof m;
    }
}

SlotShape shape_of(const BatchPlan &p) {
    SlotShape sh;
    sh.n_inst = (int)p.inst.size();
    sh.n_items = (int)p.items.size();
    sh.n_small = (int)p.small_items.size();
    sh.n_merges = (int)p.merges.size();
    sh.merge_blocks = p.merge_blocks;
    return sh;
}

xe_status launch_batch(xe_handle h, int slot, const SlotShape &sh, hipStream_t stream) {
    if (sh.n_items + sh.n_small == 0) return XE_OK;
    char *base = (char *)h->plan_area + (size_t)slot * kSlotBytes;
    const xe::BatchInstance *bi = (const xe::BatchInstance *)(base + kQueueBytes);
    const xe::BatchItem *items = (const xe::BatchItem *)(base + kQueueBytes +
                                                           sh.n_inst * sizeof(xe::BatchInstance));
    const xe::BatchItem *small = items + sh.n_items;
    const xe::MergeInst *merges = (const xe::MergeInst *)(small + sh.n_small);
    int *queues = (int *)base;   // [0, 1]: super-block items, [2, 3]: halves items
    if (sh.n_items > 0)
        hipLaunchKernelGGL(xe::batch_kernel<xe::kSuperOnly>, dim3(std::min(h->n_cu, sh.n_items)),
                           dim3(xe::kThreads), 0, stream, bi, items, sh.n_items, queues,
                           (int32_t *)h->workspace);
    if (sh.n_small > 0)
        hipLaunchKernelGGL(xe::batch_kernel<xe::kHalvesOnly>,
                           dim3(std::min(h->n_cu, sh.n_small)), dim3(xe::kThreads), 0, stream, bi,
                           small, sh.n_small, queues + 2, (int32_t *)h->workspace);
    hipLaunchKernelGGL(xe::count_list_kernel, dim3((unsigned)sh.n_inst),
                       dim3(64 * xe::kCountWaves), 0, stream, bi, sh.n_inst);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "batch launch");
    if (sh.n_merges > 0) {
        hipLaunchKernelGGL(xe::merge_list_kernel, dim3((unsigned)sh.merge_blocks), dim3(64), 0,
                           stream, merges, sh.n_merges);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(h, e, "batch merge launch");
    }
    return XE_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// per-input flags
// ---------------------------------------------------------------------------

namespace {

// Work split of the flag Gram kernel: (channel, super-block pair, time
// chunk), about one workgroup per compute unit (a diagonal pair's
// workgroup holds 96 KB of LDS counts, an off-diagonal one 156 KB), chunks
// of at least 64 steps (four per wave), and at most the kernel's
// validity window of 32768 samples, whose counts also fit 16 bits.
xe::flag::Args flag_args(const uint32_t *flags, const uint8_t *mask, int32_t N, int32_t F,
                         int32_t T, int32_t B, int32_t *d, int n_cu) {
    using namespace xe::flag;
    Args a{};
    a.flags = flags;
    a.mask = mask;
    a.d = d;
    a.N = N;
    a.F = F;
    a.T = T;
    a.B = B;
    a.W = (N + 31) / 32;
    a.nblk = (T + B - 1) / B;
    a.ns = (N + 255) / 256;
    const int64_t units = (int64_t)F * (a.ns * (a.ns + 1) / 2);
    const int64_t steps = (T + 31) / 32;
    int64_t want = ((int64_t)std::max(n_cu, 1) + units - 1) / units;
    const int64_t most = std::max<int64_t>(1, steps / 64);
    want = std::min(std::max<int64_t>(want, 1), most);
    want = std::max(want, (steps + kWindow - 1) / kWindow);
    const int64_t per = (steps + want - 1) / want;
    a.chunks = (int)((steps + per - 1) / per);
    a.chunk_samples = (int)(per * 32);
    a.b_magic = B <= 65536 ? (((uint64_t)1 << 40) + (uint64_t)B - 1) / (uint64_t)B : 0;
    return a;
}

xe_status check_flags(xe_handle h, const uint32_t *flags, int32_t N, int32_t F, int32_t T,
                      int32_t B) {
    if (!h) return XE_ERR_ARG;
    xe_status s = check_shape(h, N, F, T, B);
    if (s != XE_OK) return s;
    if (!flags) return fail(h, XE_ERR_ARG, "null pointer");
    if (!aligned(flags, 4)) return fail(h, XE_ERR_ALIGN, "flags not 4-byte aligned");
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
    h->plan_area = nullptr;
    h->staging = nullptr;
    h->ring_next = 0;
    h->geometry = XE_GEOM_AUTO;
    for (int k = 0; k < kRingSlots; ++k) h->ring_done[k] = nullptr;
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
    if (workspace_bytes == 0) workspace_bytes = kDefaultWorkspace;
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
        // batch queues start at zero; every batch launch leaves them at zero
        e = hipMalloc(&h->plan_area, (kRingSlots + kPlanSlots) * kSlotBytes);
        if (e == hipSuccess)
            e = hipMemset(h->plan_area, 0, (kRingSlots + kPlanSlots) * kSlotBytes);
        if (e == hipSuccess) e = hipHostMalloc(&h->staging, kRingSlots * kSlotBytes, 0);
        for (int k = 0; k < kRingSlots && e == hipSuccess; ++k)
            e = hipEventCreateWithFlags(&h->ring_done[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            release_device_memory(h);
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
    if (h->device != XE_DEVICE_NONE) {
        DeviceGuard g(h->device);
        release_device_memory(h);
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

xe_status xe_set_geometry(xe_handle h, int32_t geometry) {
    if (!h) return XE_ERR_ARG;
    if (geometry != XE_GEOM_AUTO && geometry != XE_GEOM_SUPER && geometry != XE_GEOM_HALVES)
        return fail(h, XE_ERR_ARG, "unknown geometry");
    h->geometry = geometry;
    return XE_OK;
}

xe_status xe_plan_query(int32_t N, int32_t F, int32_t T, int32_t B, int32_t n_cu,
                        xe_plan_info *info) {
    if (!info) return XE_ERR_ARG;
    xe_status s = check_shape(nullptr, N, F, T, B);
    if (s != XE_OK) return s;
    if (n_cu < 1) return XE_ERR_ARG;
    if (!fill_plan(N, F, T, n_cu, kDefaultWorkspace, halves_of(XE_GEOM_AUTO), info))
        return XE_ERR_WORKSPACE;
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
    return launch_corr(h, Scratch{h->workspace, h->workspace_bytes, h->n_cu}, packed, loss_mask,
                       N, F, T, B, vis, count, false, (hipStream_t)stream);
}

xe_status xe_correlate_frame(xe_handle h, const uint8_t *packed, const uint8_t *loss_mask,
                             int32_t N, int32_t F, int32_t T, int32_t B, int32_t *vis,
                             int64_t *count, void *stream) {
    xe_status s = check_frame(h, packed, N, F, T, B, vis, count);
    if (s != XE_OK) return s;
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    return launch_corr(h, Scratch{h->workspace, h->workspace_bytes, h->n_cu}, packed, loss_mask,
                       N, F, T, B, vis, count, true, (hipStream_t)stream);
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

xe_status xe_flag_accumulate(xe_handle h, const uint32_t *flags, const uint8_t *loss_mask,
                             int32_t N, int32_t F, int32_t T, int32_t B, int32_t *dcount,
                             void *stream) {
    xe_status s = check_flags(h, flags, N, F, T, B);
    if (s != XE_OK) return s;
    if (!dcount) return fail(h, XE_ERR_ARG, "null pointer");
    if (!aligned(dcount, 4)) return fail(h, XE_ERR_ALIGN, "dcount not 4-byte aligned");
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    xe::flag::Args a = flag_args(flags, loss_mask, N, F, T, eff_block(B, T), dcount, h->n_cu);
    const int64_t diag_blocks = (int64_t)F * a.ns * a.chunks;
    const int64_t off_blocks = (int64_t)F * (a.ns * (a.ns - 1) / 2) * a.chunks;
    // 16-byte loads when a row is whole groups of four words, 16-byte aligned
    const bool vec = a.W % 4 == 0 && aligned(flags, 16);
    using xe::flag::Shape;
    if (vec)
        hipLaunchKernelGGL((xe::flag::gram_kernel<false, true>), dim3((unsigned)diag_blocks),
                           dim3(Shape<false>::kThreads), 0, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL((xe::flag::gram_kernel<false, false>), dim3((unsigned)diag_blocks),
                           dim3(Shape<false>::kThreads), 0, (hipStream_t)stream, a);
    if (off_blocks > 0 && vec)
        hipLaunchKernelGGL((xe::flag::gram_kernel<true, true>), dim3((unsigned)off_blocks),
                           dim3(Shape<true>::kThreads), 0, (hipStream_t)stream, a);
    else if (off_blocks > 0)
        hipLaunchKernelGGL((xe::flag::gram_kernel<true, false>), dim3((unsigned)off_blocks),
                           dim3(Shape<true>::kThreads), 0, (hipStream_t)stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "flag gram launch");
    return XE_OK;
}

xe_status xe_apply_flags(xe_handle h, uint8_t *packed, const uint32_t *flags, int32_t N,
                         int32_t F, int32_t T, void *stream) {
    xe_status s = check_flags(h, flags, N, F, T, 1);
    if (s != XE_OK) return s;
    if (!packed) return fail(h, XE_ERR_ARG, "null pointer");
    const int W = (N + 31) / 32;
    const char *pb = (const char *)packed, *fb = (const char *)flags;
    const int64_t pbytes = (int64_t)T * F * N, fbytes = (int64_t)F * T * W * 4;
    if (pb < fb + fbytes && fb < pb + pbytes) return fail(h, XE_ERR_ARG, "packed and flags overlap");
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    const int64_t total = (int64_t)F * T * W;
    int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
    if (N % 32 == 0 && aligned(packed, 16))
        hipLaunchKernelGGL(xe::flag::apply_kernel<true>, dim3((unsigned)blocks), dim3(256), 0,
                           (hipStream_t)stream, packed, flags, N, F, T, W);
    else
        hipLaunchKernelGGL(xe::flag::apply_kernel<false>, dim3((unsigned)blocks), dim3(256), 0,
                           (hipStream_t)stream, packed, flags, N, F, T, W);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "apply flags launch");
    return XE_OK;
}

xe_status xe_normalize_flagged(xe_handle h, const int32_t *vis, const int64_t *count,
                               const int32_t *dcount, int32_t N, int32_t F, float *out,
                               int32_t *n_out, void *stream) {
    if (!h) return XE_ERR_ARG;
    xe_status s = check_shape(h, N, F, 1, 1);
    if (s != XE_OK) return s;
    if (!vis || !count || !dcount || !out) return fail(h, XE_ERR_ARG, "null pointer");
    if (!aligned(vis, 8) || !aligned(count, 8) || !aligned(out, 8) || !aligned(dcount, 4) ||
        (n_out && !aligned(n_out, 4)))
        return fail(h, XE_ERR_ALIGN, "vis/count/out not 8-byte or dcount/n_out not 4-byte aligned");
    const int64_t P = (int64_t)N * (N + 1) / 2;
    auto overlap = [](const void *a, int64_t na, const void *b, int64_t nb) {
        const char *x = (const char *)a, *y = (const char *)b;
        return x < y + nb && y < x + na;
    };
    if (overlap(out, P * F * 8, vis, P * F * 8) || overlap(out, P * F * 8, dcount, P * F * 4) ||
        (n_out && (overlap(n_out, P * F * 4, vis, P * F * 8) ||
                   overlap(n_out, P * F * 4, dcount, P * F * 4) ||
                   overlap(n_out, P * F * 4, out, P * F * 8))))
        return fail(h, XE_ERR_ARG, "outputs overlap inputs");
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    const int64_t total = P * F;
    int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(xe::flag::normalize_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, vis, count, dcount, out, n_out, N, F);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "normalize flagged launch");
    return XE_OK;
}

xe_status xe_assemble_frame(xe_handle h, const uint8_t *packets, int64_t n_packets, int32_t N,
                            int32_t n_streams, int32_t stream_base, int64_t seq0, int32_t T,
                            uint8_t *packed, uint8_t *loss_mask, uint32_t *flags, int64_t *stats,
                            void *stream) {
    using namespace xe::pkt;
    if (!h) return XE_ERR_ARG;
    if (n_streams < 1) return fail(h, XE_ERR_ARG, "n_streams must be >= 1");
    if (T % kSamples != 0) return fail(h, XE_ERR_ARG, "T must be a multiple of 4");
    if (n_packets < 0 || n_packets >= (int64_t)kNone) return fail(h, XE_ERR_ARG, "bad n_packets");
    if ((int64_t)kBands * n_streams > INT32_MAX) return fail(h, XE_ERR_ARG, "n_streams too large");
    xe_status s = check_shape(h, N, kBands * n_streams, T, kSamples);
    if (s != XE_OK) return s;
    if ((n_packets > 0 && !packets) || !packed || !loss_mask || !stats)
        return fail(h, XE_ERR_ARG, "null pointer");
    if (!aligned(packets, 4) || !aligned(flags, 4) || !aligned(stats, 8))
        return fail(h, XE_ERR_ALIGN, "packets/flags not 4-byte or stats not 8-byte aligned");
    const int64_t slots = T / kSamples;
    if ((size_t)(n_streams * slots) * 4 > h->workspace_bytes && h->device != XE_DEVICE_NONE)
        return fail(h, XE_ERR_WORKSPACE, "owner table does not fit the workspace");
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    Args a{};
    a.packets = packets;
    a.n_packets = n_packets;
    a.pbytes = XE_PACKET_BYTES(N);
    a.N = N;
    a.W = (N + 31) / 32;
    a.n_streams = n_streams;
    a.stream_base = stream_base;
    a.seq0 = seq0;
    a.T = T;
    a.slots = (int)slots;
    a.packed = packed;
    a.mask = loss_mask;
    a.flags = flags;
    a.owner = (int32_t *)h->workspace;
    a.stats = (unsigned long long *)stats;
    hipStream_t st = (hipStream_t)stream;
    const int64_t places = (int64_t)n_streams * slots;
    hipLaunchKernelGGL(reset_kernel, dim3((unsigned)std::min<int64_t>((places + 255) / 256, 4096)),
                       dim3(256), 0, st, a.owner, places, a.stats);
    if (n_packets > 0)
        hipLaunchKernelGGL(claim_kernel, dim3((unsigned)((n_packets + 255) / 256)), dim3(256), 0,
                           st, a);
    if (N % 2 == 0 && aligned(packed, 16) && aligned(packets, 16))
        hipLaunchKernelGGL(place_kernel<true>, dim3((unsigned)places), dim3(kPlaceThreads), 0, st,
                           a);
    else
        hipLaunchKernelGGL(place_kernel<false>, dim3((unsigned)places), dim3(kPlaceThreads), 0,
                           st, a);
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)std::min<int64_t>((places + 255) / 256, 256)),
                       dim3(256), 0, st, a.owner, places, a.stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "assemble launch");
    return XE_OK;
}

xe_status xe_time_shift(xe_handle h, const uint8_t *packed_in, const uint32_t *flags_in,
                        const int32_t *delays, int32_t N, int32_t F, int32_t T,
                        uint8_t *packed_out, uint32_t *flags_out, void *stream) {
    if (!h) return XE_ERR_ARG;
    xe_status s = check_shape(h, N, F, T, 1);
    if (s != XE_OK) return s;
    if (!packed_in || !delays || !packed_out) return fail(h, XE_ERR_ARG, "null pointer");
    if (!aligned(delays, 4) || !aligned(flags_in, 4) || !aligned(flags_out, 4))
        return fail(h, XE_ERR_ALIGN, "delays/flags not 4-byte aligned");
    const int W = (N + 31) / 32;
    const int64_t fbytes = (int64_t)F * T * W * 4, pbytes = (int64_t)T * F * N;
    auto overlap = [](const void *a, int64_t na, const void *b, int64_t nb) {
        const char *x = (const char *)a, *y = (const char *)b;
        return a && b && x < y + nb && y < x + na;
    };
    if (overlap(packed_out, pbytes, packed_in, pbytes) ||
        overlap(flags_out, fbytes, flags_in, fbytes) ||
        overlap(flags_out, fbytes, packed_in, pbytes) ||
        overlap(packed_out, pbytes, flags_in, fbytes) ||
        overlap(packed_out, pbytes, flags_out, fbytes))
        return fail(h, XE_ERR_ARG, "outputs overlap inputs or each other");
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    using namespace xe::shift;
    const int64_t tiles =
        (int64_t)F * ((T + kRows - 1) / kRows) * ((N + kCols - 1) / kCols);
    if (N % 16 == 0 && aligned(packed_in, 16) && aligned(packed_out, 16))
        hipLaunchKernelGGL(tile_kernel<true>, dim3((unsigned)tiles), dim3(kTileThreads), 0,
                           (hipStream_t)stream, packed_in, flags_in, delays, packed_out,
                           flags_out, N, F, T, W);
    else
        hipLaunchKernelGGL(tile_kernel<false>, dim3((unsigned)tiles), dim3(kTileThreads), 0,
                           (hipStream_t)stream, packed_in, flags_in, delays, packed_out,
                           flags_out, N, F, T, W);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "time shift launch");
    return XE_OK;
}

xe_status xe_accumulate_batch(xe_handle h, const xe_instance *inst, int32_t n_inst,
                              void *stream) {
    if (!h) return XE_ERR_ARG;
    BatchPlan plan;
    xe_status s = build_batch(h, inst, n_inst, h->n_cu, 0,
                              h->device == XE_DEVICE_NONE ? kDefaultWorkspace
                                                          : h->workspace_bytes, &plan);
    if (s != XE_OK) return s;
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    if (!plan.items.empty() || !plan.small_items.empty()) {
        // the ring slot (and its pinned staging copy) is free once the
        // launch that last used it has finished
        const int slot = h->ring_next;
        h->ring_next = (h->ring_next + 1) % kRingSlots;
        hipError_t e = hipEventSynchronize(h->ring_done[slot]);
        if (e != hipSuccess) return hip_fail(h, e, "batch ring wait");
        char *stage = (char *)h->staging + (size_t)slot * kSlotBytes;
        write_plan(plan, (int32_t *)h->workspace, stage);
        e = hipMemcpyAsync((char *)h->plan_area + (size_t)slot * kSlotBytes, stage,
                           plan_bytes(plan), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(h, e, "batch upload");
        s = launch_batch(h, slot, shape_of(plan), st);
        if (s != XE_OK) return s;
        e = hipEventRecord(h->ring_done[slot], st);
        if (e != hipSuccess) return hip_fail(h, e, "batch ring record");
    }
    for (const xe_instance &x : plan.unaligned) {
        s = launch_corr(h, Scratch{h->workspace, h->workspace_bytes, h->n_cu}, x.packed,
                        x.loss_mask, x.N, x.F, x.T, x.B, x.vis, x.count, false, st);
        if (s != XE_OK) return s;
    }
    return XE_OK;
}

xe_status xe_batch_plan(xe_handle h, const xe_instance *inst, int32_t n_inst,
                        int32_t chunk_steps, int32_t *plan_id) {
    if (!h || !plan_id) return XE_ERR_ARG;
    BatchPlan plan;
    xe_status s = build_batch(h, inst, n_inst, h->n_cu, chunk_steps,
                              h->device == XE_DEVICE_NONE ? kDefaultWorkspace
                                                          : h->workspace_bytes, &plan);
    if (s != XE_OK) return s;
    if (h->device == XE_DEVICE_NONE) return XE_ERR_NO_DEVICE;
    int slot = -1;
    for (int k = kRingSlots; k < kRingSlots + kPlanSlots; ++k)
        if (!h->slots[k].used) {
            slot = k;
            break;
        }
    if (slot < 0) return fail(h, XE_ERR_WORKSPACE, "all plan slots in use");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    std::vector<char> host(plan_bytes(plan));
    write_plan(plan, (int32_t *)h->workspace, host.data());
    hipError_t e = hipMemcpy((char *)h->plan_area + (size_t)slot * kSlotBytes, host.data(),
                             host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(h, e, "plan upload");
    PlanSlot &ps = h->slots[slot];
    ps.used = true;
    ps.shape = shape_of(plan);
    ps.unaligned = plan.unaligned;
    *plan_id = slot;
    return XE_OK;
}

xe_status xe_batch_run(xe_handle h, int32_t plan_id, void *stream) {
    if (!h || plan_id < kRingSlots || plan_id >= kRingSlots + kPlanSlots ||
        !h->slots[plan_id].used)
        return fail(h, XE_ERR_ARG, "unknown plan");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, XE_ERR_HIP, "hipSetDevice failed");
    const PlanSlot &ps = h->slots[plan_id];
    hipStream_t st = (hipStream_t)stream;
    xe_status s = launch_batch(h, plan_id, ps.shape, st);
    if (s != XE_OK) return s;
    for (const xe_instance &x : ps.unaligned) {
        s = launch_corr(h, Scratch{h->workspace, h->workspace_bytes, h->n_cu}, x.packed,
                        x.loss_mask, x.N, x.F, x.T, x.B, x.vis, x.count, false, st);
        if (s != XE_OK) return s;
    }
    return XE_OK;
}

xe_status xe_batch_release(xe_handle h, int32_t plan_id) {
    if (!h || plan_id < kRingSlots || plan_id >= kRingSlots + kPlanSlots ||
        !h->slots[plan_id].used)
        return fail(h, XE_ERR_ARG, "unknown plan");
    h->slots[plan_id] = PlanSlot();
    return XE_OK;
}

xe_status xe_batch_query(const xe_instance *inst, int32_t n_inst, int32_t n_cu,
                         int32_t chunk_steps, xe_batch_info *info) {
    if (!info || n_cu < 1) return XE_ERR_ARG;
    BatchPlan plan;
    xe_handle_s probe{};  // validation only: never touches a device
    probe.device = XE_DEVICE_NONE;
    xe_status s = build_batch(&probe, inst, n_inst, n_cu, chunk_steps, kDefaultWorkspace, &plan);
    if (s != XE_OK) return s;
    info->items = (int64_t)(plan.items.size() + plan.small_items.size());
    info->instances = (int32_t)plan.inst.size();
    info->unaligned = (int32_t)plan.unaligned.size();
    info->chunk_steps = plan.chunk_steps;
    info->partial_bytes = plan.partials * (int64_t)sizeof(int32_t);
    return XE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// the allocation-free accumulate
// ---------------------------------------------------------------------------

// Partial sums of time chunks for xe_accumulate_noalloc: one static array
// per device, loaded with the code object and held until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host its name
// is a stand-in, not a device address): the address comes from
// hipGetSymbolAddress, once per device, and is kept in g_scratch.
static __device__ __align__(256) int32_t scratch[XE_NOALLOC_SCRATCH_BYTES / sizeof(int32_t)];

namespace {

constexpr int kMaxDevices = 64;

struct DeviceScratch {
    bool ready = false;
    void *ptr = nullptr;
    int n_cu = 0;
};

std::mutex g_scratch_lock;
DeviceScratch g_scratch[kMaxDevices];

// Address and CU count of the current device's scratch array, taken on the
// first call on that device (with the device current).
xe_status device_scratch(Scratch *out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return XE_ERR_HIP;
    if (dev >= kMaxDevices) return XE_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_lock);
    DeviceScratch &d = g_scratch[dev];
    if (!d.ready) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return XE_ERR_HIP;
        if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return XE_ERR_UNSUPPORTED;
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return XE_ERR_HIP;
        d.ptr = p;
        d.n_cu = prop.multiProcessorCount;
        d.ready = true;
    }
    *out = Scratch{d.ptr, (size_t)XE_NOALLOC_SCRATCH_BYTES, d.n_cu};
    return XE_OK;
}

}  // namespace

extern "C" xe_status xe_accumulate_noalloc(const uint8_t *packed, const uint8_t *loss_mask,
                                           int32_t N, int32_t F, int32_t T, int32_t B,
                                           int32_t *vis, int64_t *count, void *stream) {
    xe_status s = check_shape(nullptr, N, F, T, B);
    if (s != XE_OK) return s;
    if (!packed || !vis || !count) return XE_ERR_ARG;
    if (!aligned(vis, 8) || !aligned(count, 8)) return XE_ERR_ALIGN;
    // Sizes beyond the scratch array: even the fewest time chunks the
    // frame's byte offsets allow leave more partial sums than it holds.
    // Decided on the host before any device call.
    {
        const int nb = xe::ceil_div(N, xe::kBlk);
        const int64_t keys = (int64_t)F * xe::groups_per_channel(nb);
        const int steps = xe::ceil_div(T, xe::kStep);
        const int64_t max_sps = xe::max_steps_per_chunk(F, N);
        const int fewest = (int)((steps + max_sps - 1) / max_sps);
        if (partial_bytes(keys, fewest) > (size_t)XE_NOALLOC_SCRATCH_BYTES)
            return XE_ERR_WORKSPACE;
    }
    Scratch ws;
    s = device_scratch(&ws);
    if (s != XE_OK) return s;
    return launch_corr(nullptr, ws, packed, loss_mask, N, F, T, B, vis, count, false,
                       (hipStream_t)stream);
}
