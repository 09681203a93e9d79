// pcr_batch.hip -- batched multi-view rendering: many cameras and framebuffers
// of one resident cloud per launch.
//
// A launch is one hipGraph replay of four stages:
//   clear   all views' buffers
//   pass A  closest-point views (basic / dedup) and the depth pass of HQ views
//   pass B  the colour pass of HQ views (needs every HQ depth complete)
//   resolve all views
// In the grouped form, passes A and B are one kernel each: workgroups step
// over (group, tile) items in group-major order, load the tile's points once
// and render them into every view of the group in turn with the single-view
// kernels' tile body, so the point stream is read once per group instead of
// once per view.  A group holds up to tune group views (16 by default) and
// at most 2 GiB of framebuffers.  In the per-view form (tune group 1) every view slot runs the
// single-view passes instead, reading its view from the device table; slots a
// launch does not use are disabled in the graph.  Every update is an integer
// min or sum, so each view is bit-identical to rendering it alone.
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <vector>

#include "pcr_internal.h"

namespace pcr {
namespace {

// Framebuffer bytes per group.  Fewer, larger groups read the point stream
// fewer times; a group's framebuffers need not stay cache resident (the
// atomics execute at the memory side), so only the view count limits a group
// of ordinary images.
constexpr uint64_t kGroupBudget = 2048ull << 20;
constexpr uint32_t kMaxGroup = 32;                // views per group
constexpr uint32_t kPidMask = (1u << 27) - 1u;    // largest pixel count of a batched view

using DevView = BatchView;
using Group = BatchGroup;

// Device table: header, then groups and index lists of both passes, then views.
struct Header {
    uint32_t counter[2];  // work queues of pass A and B (zeroed by the clear kernel)
    uint32_t ngroups[2];
    uint32_t nviews;
    uint32_t pad[3];
};

struct TableLayout {
    size_t groups[2], index[2], views, bytes;
};

TableLayout layout(uint32_t cap) {
    TableLayout L;
    size_t off = sizeof(Header);
    for (int p = 0; p < 2; ++p) {
        L.groups[p] = off;
        off += sizeof(Group) * cap;
        L.index[p] = off;
        off += sizeof(uint32_t) * cap;
    }
    off = (off + 63) & ~(size_t)63;
    L.views = off;
    off += sizeof(DevView) * cap;
    L.bytes = (off + 255) & ~(size_t)255;
    return L;
}

struct Table {
    const Header *h;
    const Group *groups[2];
    const uint32_t *index[2];
    const DevView *views;
};

__device__ __forceinline__ Table table(const unsigned char *base, TableLayout L) {
    Table t;
    t.h = (const Header *)base;
    for (int p = 0; p < 2; ++p) {
        t.groups[p] = (const Group *)(base + L.groups[p]);
        t.index[p] = (const uint32_t *)(base + L.index[p]);
    }
    t.views = (const DevView *)(base + L.views);
    return t;
}

// ---------------------------------------------------------------------------
// Clear and resolve of all views (grid-stride over views x words)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_batch_clear(unsigned char *base, TableLayout L) {
    Table t = table(base, L);
    if (blockIdx.x == 0 && threadIdx.x < 2) ((Header *)base)->counter[threadIdx.x] = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t i = 0; i < t.h->nviews; ++i) {
        const DevView &dv = t.views[i];
        uint64_t px = (uint64_t)dv.v.W * dv.v.H;
        if (dv.variant == PCR_HQ) {
            for (uint64_t k = gid; k < px; k += stride) {
                dv.D[k] = 0xFFFFFFFFu;
                dv.S[2 * k] = 0;
                dv.S[2 * k + 1] = 0;
            }
        } else {
            for (uint64_t k = gid; k < px; k += stride) dv.fb[k] = kEmptyKey;
        }
    }
}

__global__ __launch_bounds__(256) void k_batch_resolve(const unsigned char *base, TableLayout L) {
    Table t = table(base, L);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t i = 0; i < t.h->nviews; ++i) {
        const DevView &dv = t.views[i];
        uint64_t px = (uint64_t)dv.v.W * dv.v.H;
        if (dv.variant == PCR_HQ) {
            const u32x4 *S = (const u32x4 *)dv.S;
            for (uint64_t k = gid; k < px; k += stride) {
                u32x4 s = S[k];  // {G sum, R sum, count, B sum}
                uint32_t c = s.z, o = 0;
                if (c != 0)
                    o = ((s.y / c) & 0xFFu) | ((s.x / c) & 0xFFu) << 8 | ((s.w / c) & 0xFFu) << 16 | 0xFF000000u;
                dv.out[k] = o;
            }
        } else {
            for (uint64_t k = gid; k < px; k += stride) {
                u64 key = dv.fb[k];
                dv.out[k] = key == kEmptyKey ? 0u : (uint32_t)key;
            }
        }
    }
}



}  // namespace

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
}  // namespace pcr

struct pcr_batch {
    const pcr::u32x4 *pts = nullptr;
    uint64_t n = 0;
    uint32_t capacity = 0;
    pcr::Shape sh{};
    pcr::TableLayout lay{};
    unsigned char *dtable = nullptr;
    static constexpr int kRing = 4;
    unsigned char *staging[kRing] = {};
    hipEvent_t done[kRing] = {};
    int next = 0;
    int last = -1;  // staging slot of the previous launch (its event marks its end)
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t grid_io = 0;
    // Per-view mode: the graph node of each (pass, slot) and whether it is
    // enabled in `exec`; slots a launch does not use are disabled, so they
    // cost no dispatch.
    std::vector<hipGraphNode_t> vnode[2];
    std::vector<uint8_t> von[2];
};

namespace pcr {
namespace {

// Grouped pass `pass` over the plan's table (pass < 0: only raise the
// kernels' LDS limits, done before graph capture).
int launch_pass(pcr_batch *b, int pass, hipStream_t s) {
    const BatchView *views = (const BatchView *)(b->dtable + b->lay.views);
    const int p = pass < 0 ? 0 : pass;
    const uint32_t *index = (const uint32_t *)(b->dtable + b->lay.index[p]);
    const BatchGroup *groups = (const BatchGroup *)(b->dtable + b->lay.groups[p]);
    const uint32_t *ng = (const uint32_t *)(b->dtable + offsetof(Header, ngroups) + sizeof(uint32_t) * p);
    return launch_group_pass(pass, b->pts, b->n, views, index, groups, ng, b->sh, s);
}

// Per-view mode (group 1): every view slot gets the single-view passes; a
// slot beyond the launch's view count ends at once.
int view_passes(pcr_batch *b, int pass, hipStream_t s) {
    const BatchView *views = (const BatchView *)(b->dtable + b->lay.views);
    const uint32_t *nv = (const uint32_t *)(b->dtable + offsetof(Header, nviews));
    if (pass < 0) return launch_view_pass(-1, b->pts, b->n, views, nv, 0, b->sh, s);
    b->vnode[pass].assign(b->capacity, nullptr);
    b->von[pass].assign(b->capacity, 1);
    for (uint32_t i = 0; i < b->capacity; ++i) {
        if (int rc = launch_view_pass(pass, b->pts, b->n, views, nv, i, b->sh, s)) return rc;
        // The kernel just captured is the stream's only dependency now.
        hipStreamCaptureStatus st;
        const hipGraphNode_t *deps = nullptr;
        size_t ndeps = 0;
        if (hipStreamGetCaptureInfo_v2(s, &st, nullptr, nullptr, &deps, &ndeps) != hipSuccess ||
            st != hipStreamCaptureStatusActive || ndeps != 1)
            return fail(PCR_EHIP, "could not identify the captured node of view slot %u", i);
        b->vnode[pass][i] = deps[0];
    }
    return PCR_OK;
}

// Enables the per-view nodes the launch needs (slot i < nviews; the colour
// pass only for HQ views) and disables the others.
int select_view_nodes(pcr_batch *b, const std::vector<BatchView> &dv) {
    for (int pass = 0; pass < 2; ++pass) {
        for (uint32_t i = 0; i < b->capacity; ++i) {
            const uint8_t want = i < dv.size() && (pass == 0 || dv[i].variant == PCR_HQ);
            if (b->von[pass][i] == want) continue;
            PCR_HIP(hipGraphNodeSetEnabled(b->exec, b->vnode[pass][i], want));
            b->von[pass][i] = want;
        }
    }
    return PCR_OK;
}

int record(pcr_batch *b, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_clear, dim3(b->grid_io), dim3(256), 0, s, b->dtable, b->lay);
    PCR_LAUNCHED();
    const bool per_view = b->sh.group == 1;
    int rc = per_view ? view_passes(b, 0, s) : launch_pass(b, 0, s);
    if (rc == PCR_OK) rc = per_view ? view_passes(b, 1, s) : launch_pass(b, 1, s);
    if (rc != PCR_OK) return rc;
    hipLaunchKernelGGL(k_batch_resolve, dim3(b->grid_io), dim3(256), 0, s, b->dtable, b->lay);
    PCR_LAUNCHED();
    return PCR_OK;
}

void destroy(pcr_batch *b) {
    if (!b) return;
    // Every launch of the plan ends with a record of one of its events: once
    // they have all completed, no replay of the graph reads its table.
    for (int i = 0; i < pcr_batch::kRing; ++i)
        if (b->done[i]) (void)hipEventSynchronize(b->done[i]);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int i = 0; i < pcr_batch::kRing; ++i) {
        if (b->done[i]) (void)hipEventDestroy(b->done[i]);
        if (b->staging[i]) (void)hipHostFree(b->staging[i]);
    }
    if (b->dtable) (void)hipFree(b->dtable);
    delete b;
}

}  // namespace
}  // namespace pcr

using namespace pcr;

extern "C" int pcr_batch_create(pcr_batch **plan, const pcr_point *pts, uint64_t n, uint32_t capacity,
                                const pcr_tune *tune, void *stream) {
    if (!plan) return fail(PCR_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (capacity == 0 || capacity > 4096) return fail(PCR_EINVAL, "capacity %u not in [1, 4096]", capacity);
    if (n == 0 || !pts || ((uintptr_t)pts & 15)) return fail(PCR_EINVAL, "points must be a non-empty 16-byte aligned device buffer");
    pcr_tune t{};
    if (tune) t = *tune;
    Shape sh;
    int rc = resolve_shape(&t, PCR_DEDUP, sh);
    if (rc != PCR_OK) return rc;
    pcr_batch *b = new pcr_batch();
    b->pts = (const u32x4 *)pts;
    b->n = n;
    b->capacity = capacity;
    b->sh = sh;
    b->lay = layout(capacity);
    b->grid_io = (uint32_t)device_cus() * 16;
    hipError_t e = hipMalloc((void **)&b->dtable, b->lay.bytes);
    if (e != hipSuccess) {
        destroy(b);
        return fail(PCR_ENOMEM, "view table: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < pcr_batch::kRing; ++i) {
        if (hipHostMalloc((void **)&b->staging[i], b->lay.bytes, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming) != hipSuccess) {
            destroy(b);
            return fail(PCR_ENOMEM, "staging buffers");
        }
        memset(b->staging[i], 0, b->lay.bytes);
    }
    // An empty table makes every kernel a no-op; upload it so a graph replay
    // before the first launch is harmless.
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(b->dtable, b->staging[0], b->lay.bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        destroy(b);
        return fail(PCR_EHIP, "plan set-up failed");
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        destroy(b);
        return fail(PCR_EHIP, "plan set-up failed");
    }
    rc = b->sh.group == 1 ? view_passes(b, -1, nullptr) : launch_pass(b, -1, nullptr);
    if (rc != PCR_OK) {
        destroy(b);
        return rc;
    }
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        destroy(b);
        return fail(PCR_EHIP, "graph capture failed to start");
    }
    rc = record(b, b->cap);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(b->cap, &g);
    b->graph = g;
    if (rc != PCR_OK || ee != hipSuccess) {
        destroy(b);
        return rc != PCR_OK ? rc : fail(PCR_EHIP, "graph capture failed: %s", hipGetErrorString(ee));
    }
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
        destroy(b);
        return fail(PCR_EHIP, "graph instantiation failed");
    }
    *plan = b;
    return PCR_OK;
}

extern "C" int pcr_batch_launch(pcr_batch *b, const pcr_view *views, uint32_t nviews, void *stream) {
    if (!b) return fail(PCR_EINVAL, "plan is NULL");
    if (nviews > b->capacity) return fail(PCR_EINVAL, "%u views exceed the plan's capacity %u", nviews, b->capacity);
    if (nviews > 0 && !views) return fail(PCR_EINVAL, "views is NULL");
    // Validate and sort views into groups on the host.
    std::vector<DevView> dv;
    dv.reserve(nviews);
    for (uint32_t i = 0; i < nviews; ++i) {
        const pcr_view &v = views[i];
        if (v.variant < 0) continue;
        int rc = check_image(v.w, v.h);
        if (rc == PCR_OK) rc = check_variant(v.variant & 0xFF);
        if (rc != PCR_OK) return rc;
        if (v.variant & (PCR_F_HQ_PACKED | PCR_F_HQ_ROBUST))
            return fail(PCR_EUNSUPPORTED,
                        "view %u: batches render the two-word HQ sums (no PCR_F_HQ_PACKED or PCR_F_HQ_ROBUST)", i);
        if ((uint64_t)v.w * v.h > kPidMask)
            return fail(PCR_EINVAL, "view %u: batched views hold at most 2^27 - 1 pixels", i);
        if (!v.fb || ((uintptr_t)v.fb & 15) || !v.rgba_out || ((uintptr_t)v.rgba_out & 3))
            return fail(PCR_EINVAL, "view %u: framebuffer must be 16-byte aligned, rgba_out 4-byte aligned", i);
        DevView d{};
        d.v = make_view(v.mvp, v.w, v.h);
        d.variant = v.variant & 0xFF;
        d.fb = (u64 *)v.fb;
        d.D = (uint32_t *)v.fb;
        d.S = (u64 *)((char *)v.fb + hq_depth_bytes(v.w, v.h));
        d.out = v.rgba_out;
        dv.push_back(d);
    }
    pcr_batch &B = *b;
    int slot = B.next;
    B.next = (B.next + 1) % pcr_batch::kRing;
    PCR_HIP(hipEventSynchronize(B.done[slot]));  // the staging slot's last upload has completed
    unsigned char *st = B.staging[slot];
    Header *h = (Header *)st;
    memset(h, 0, sizeof(Header));
    h->nviews = (uint32_t)dv.size();
    memcpy(st + B.lay.views, dv.data(), dv.size() * sizeof(DevView));
    const uint32_t maxg = std::min<uint32_t>(B.sh.group ? B.sh.group : 16, kMaxGroup);
    for (int pass = 0; pass < 2; ++pass) {
        Group *gs = (Group *)(st + B.lay.groups[pass]);
        uint32_t *ix = (uint32_t *)(st + B.lay.index[pass]);
        uint32_t ng = 0, ni = 0;
        uint64_t bytes = 0;
        for (uint32_t i = 0; i < dv.size(); ++i) {
            bool hq = dv[i].variant == PCR_HQ;
            if (pass == 1 && !hq) continue;
            uint64_t fbb = pcr_fb_bytes(dv[i].v.W, dv[i].v.H, dv[i].variant);
            bool open = ng > 0 && gs[ng - 1].count < maxg && bytes + fbb <= kGroupBudget;
            if (!open) {
                gs[ng].first = ni;
                gs[ng].count = 0;
                ++ng;
                bytes = 0;
            }
            ix[ni++] = i;
            gs[ng - 1].count++;
            bytes += fbb;
        }
        h->ngroups[pass] = ng;
    }
    if (B.sh.group == 1)
        if (int rc = select_view_nodes(b, dv)) return rc;
    hipStream_t s = (hipStream_t)stream;
    // The plan's device table is rewritten below: on another stream, wait for
    // the previous launch of this plan first (a no-op on the same stream).
    if (B.last >= 0) PCR_HIP(hipStreamWaitEvent(s, B.done[B.last], 0));
    PCR_HIP(hipMemcpyAsync(B.dtable, st, B.lay.bytes, hipMemcpyHostToDevice, s));
    PCR_HIP(hipGraphLaunch(B.exec, s));
    PCR_HIP(hipEventRecord(B.done[slot], s));
    B.last = slot;
    return PCR_OK;
}

// ---------------------------------------------------------------------------
// One-call batches over a small cache of plans
// ---------------------------------------------------------------------------
namespace {

struct CachedPlan {
    int device;
    const pcr_point *pts;
    uint64_t n;
    uint32_t capacity;
    pcr_tune tune;
    pcr_batch *plan;
    uint64_t used;
};

std::mutex g_cache_mu;
std::vector<CachedPlan> g_cache;
uint64_t g_cache_tick = 0;
constexpr size_t kCachedPlans = 8;

bool same_tune(const pcr_tune &a, const pcr_tune &b) {
    return a.ppt == b.ppt && a.wg == b.wg && a.grid == b.grid && a.group == b.group && a.slots == b.slots &&
           a.run == b.run;
}

}  // namespace

extern "C" int pcr_render_batch(const pcr_point *pts, uint64_t n, const pcr_view *views, uint32_t nviews,
                                const pcr_tune *tune, void *stream) {
    if (nviews == 0) return PCR_OK;
    if (!views) return fail(PCR_EINVAL, "views is NULL");
    if (nviews > 4096) return fail(PCR_EINVAL, "%u views exceed 4096", nviews);
    int dev = 0;
    PCR_HIP(hipGetDevice(&dev));
    pcr_tune t{};
    if (tune) t = *tune;
    uint32_t cap = 4;
    while (cap < nviews) cap *= 2;
    std::lock_guard<std::mutex> g(g_cache_mu);
    CachedPlan *hit = nullptr;
    for (auto &c : g_cache)
        if (c.device == dev && c.pts == pts && c.n == n && c.capacity == cap && same_tune(c.tune, t)) hit = &c;
    if (!hit) {
        if (g_cache.size() >= kCachedPlans) {  // drop the least recently used plan
            auto lru = std::min_element(g_cache.begin(), g_cache.end(),
                                        [](const CachedPlan &a, const CachedPlan &b) { return a.used < b.used; });
            pcr_batch_destroy(lru->plan);
            g_cache.erase(lru);
        }
        pcr_batch *plan = nullptr;
        if (int rc = pcr_batch_create(&plan, pts, n, cap, tune ? &t : nullptr, stream)) return rc;
        g_cache.push_back(CachedPlan{dev, pts, n, cap, t, plan, 0});
        hit = &g_cache.back();
    }
    hit->used = ++g_cache_tick;
    return pcr_batch_launch(hit->plan, views, nviews, stream);
}

extern "C" int pcr_release_batch_plans(void) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    for (auto &c : g_cache) pcr_batch_destroy(c.plan);
    g_cache.clear();
    return PCR_OK;
}

extern "C" int pcr_batch_destroy(pcr_batch *b) {
    destroy(b);
    return PCR_OK;
}
