// pcr_batch.hip -- batched multi-view rendering: many cameras and framebuffers
// of one resident cloud per launch.
//
// A launch is one hipGraph replay of four stages:
//   clear   all views' buffers
//   pass A  closest-point views (basic / dedup) and the depth pass of HQ views
//   pass B  the colour pass of HQ views (needs every HQ depth complete)
//   resolve all views
// In the batched form, passes A and B are one kernel each: workgroups step
// over (group, tile) items in group-major order, load the tile's points once
// and render them into every view of the group, deduplicating same-pixel
// updates in a shared LDS table.  Views are grouped so that a group's
// framebuffers fit the cache budget, which keeps the atomics of a pass inside
// a small, cache-resident working set while the point stream is read once per
// group.  In the per-view form (tune group 1) every view slot runs the
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

constexpr uint32_t kBatchWg = 256;
constexpr uint64_t kGroupBudget = 160ull << 20;  // framebuffer bytes per group

using DevView = BatchView;

struct Group {
    uint32_t first, count;  // range of the pass's view-index list
};

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

// ---------------------------------------------------------------------------
// Persistent multi-view passes
// ---------------------------------------------------------------------------
constexpr uint32_t kMaxProbeB = 8;

__device__ __forceinline__ void bar_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS: item | count | val[HS] (16 B: min key, or RG and BA sums) | tag[HS] | list[HS]
struct BLds {
    uint32_t *item, *count, *tag, *list;
    u64 *val;  // 2 words per slot
    uint32_t mask, shift;
    __device__ BLds(unsigned char *sm, uint32_t hbits) {
        item = (uint32_t *)sm;
        count = item + 1;
        val = (u64 *)(sm + 16);
        tag = (uint32_t *)(val + 2 * (1u << hbits));
        list = tag + (1u << hbits);
        mask = (1u << hbits) - 1u;
        shift = 24u - hbits;  // hbits <= 15: the top bits of a 24-bit product
    }
    // Home slot of a (view slot, pixel) tag: the view bits are folded into
    // the low 24 bits, then Fibonacci hashing in a 24-bit word (full-rate
    // 24-bit multiply; __umul24 returns a signed int: shifted as unsigned and
    // masked into the table).
    __device__ __forceinline__ uint32_t home(uint32_t key) const {
        const uint32_t k = (key ^ (key >> 20)) & 0xFFFFFFu;
        return ((uint32_t)__umul24(k, 0x9E3779u) >> shift) & mask;
    }
    __device__ __forceinline__ uint32_t slot(uint32_t pid) {
        uint32_t h = home(pid);
#pragma unroll 1
        for (uint32_t probe = 0; probe < kMaxProbeB; ++probe) {
            uint32_t t = __hip_atomic_load(tag + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (t == pid) return h;
            if (t == kEmptyPid) {
                uint32_t old = atomicCAS(tag + h, kEmptyPid, pid);
                if (old == kEmptyPid) {
                    list[atomicAdd(count, 1u)] = h;
                    return h;
                }
                if (old == pid) return h;
            }
            h = (h + 1u) & mask;
        }
        return 0xFFFFFFFFu;
    }
};

__device__ __forceinline__ void lmin64(u64 *p, u64 v) {
    u64 cur = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (v < cur) __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One LDS table serves all views of a group: its tag packs the view's slot in
// the group (5 bits) above the pixel index (27 bits).  A tile is projected into
// every view of its group in turn; the table is flushed to the framebuffers
// only when it is half full and at the end of the tile.
constexpr uint32_t kPidBits = 27;
constexpr uint32_t kPidMask = (1u << kPidBits) - 1u;
constexpr uint32_t kMaxGroup = 32;

// PASS = 0: closest-point views (64-bit keys) and HQ depth (depth bits);
// PASS = 1: HQ colour sums.
template <int PPT, int PASS>
__global__ __launch_bounds__(kBatchWg) void k_batch_pass(const u32x4 *__restrict__ pts, uint64_t n,
                                                         unsigned char *base, TableLayout L, uint32_t hbits) {
    extern __shared__ __align__(16) unsigned char smem[];
    // The group's views, staged once per item: camera and viewport, buffers.
    __shared__ View vpar[kMaxGroup];
    __shared__ u64 vbuf[kMaxGroup][2];  // per group slot: fb (or D) and S
    __shared__ uint32_t vhq[kMaxGroup];
    BLds S(smem, hbits);
    Table t = table(base, L);
    const uint32_t HS = 1u << hbits;
    const uint32_t wg = blockDim.x;  // 64, 128 or 256
    const uint32_t T = wg * PPT;
    const uint64_t ntiles = (n + T - 1) / T;
    for (uint32_t s = threadIdx.x; s < HS; s += wg) {
        S.tag[s] = kEmptyPid;
        S.val[2 * s] = PASS ? 0ull : kEmptyKey;
        S.val[2 * s + 1] = 0ull;
    }
    if (threadIdx.x == 0) *S.count = 0;
    bar_lds();

    // Writes the table's entries to their views' buffers and empties it.
    auto flush = [&]() {
        bar_lds();
        const uint32_t cnt = *S.count;
        bar_lds();
        if (threadIdx.x == 0) *S.count = 0;
        for (uint32_t k = threadIdx.x; k < cnt; k += wg) {
            uint32_t h = S.list[k];
            uint32_t tag = S.tag[h];
            uint32_t vs = tag >> kPidBits, pid = tag & kPidMask;
            u64 a = S.val[2 * h], b = S.val[2 * h + 1];
            S.tag[h] = kEmptyPid;
            S.val[2 * h] = PASS ? 0ull : kEmptyKey;
            S.val[2 * h + 1] = 0ull;
            if (PASS == 0) {
                if (vhq[vs]) {
                    // Early test: any value the word has held is >= its
                    // current one, so a stale read never skips a needed update.
                    uint32_t *D = (uint32_t *)vbuf[vs][0];
                    const uint32_t seen = __hip_atomic_load(D + pid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if ((uint32_t)a < seen) gmin_u32(D + pid, (uint32_t)a);
                } else {
                    gmin_u64((u64 *)vbuf[vs][0] + pid, a);
                }
            } else {
                u64 *Sm = (u64 *)vbuf[vs][1];
                gadd_u64(Sm + 2 * (u64)pid, a);
                gadd_u64(Sm + 2 * (u64)pid + 1, b);
            }
        }
        bar_lds();
    };

    // Grid-stride over the (group, tile) items in group-major order with the
    // tiles in their natural order (no shared queue: same-address atomics
    // serialise at the memory-side atomic unit): the workgroups resident at
    // one time work on one window of the point order, the schedule that the
    // single-view kernels measured fastest.  A workgroup's items stay in one
    // group for ntiles / grid items, so its views are restaged only when the
    // group changes.
    const uint32_t ngroups = t.h->ngroups[PASS];
    const uint64_t nitems = (uint64_t)ngroups * ntiles;
    uint32_t cur_g = 0xFFFFFFFFu, gcount = 0;
    for (uint64_t item = blockIdx.x; item < nitems; item += gridDim.x) {  // uniform exit for every workgroup
        const uint32_t g = (uint32_t)(item / ntiles);
        const uint64_t tile = item - (uint64_t)g * ntiles;
        const uint64_t first = tile * T;
        const uint64_t rem = n - first;
        u32x4 p[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            uint32_t k = (uint32_t)(j * wg + threadIdx.x);
            p[j] = load_point(pts + first + (k < rem ? k : (uint32_t)(rem - 1)));
        }
        if (g != cur_g) {
            const Group grp = t.groups[PASS][g];
            gcount = (uint32_t)__builtin_amdgcn_readfirstlane((int)grp.count);
            if (threadIdx.x < gcount) {
                const DevView &dv = t.views[t.index[PASS][grp.first + threadIdx.x]];
                vpar[threadIdx.x] = dv.v;
                vhq[threadIdx.x] = dv.variant == PCR_HQ;
                vbuf[threadIdx.x][0] = (u64)(dv.variant == PCR_HQ ? (void *)dv.D : (void *)dv.fb);
                vbuf[threadIdx.x][1] = (u64)dv.S;
            }
            cur_g = g;
            bar_lds();
        }
        for (uint32_t vs = 0; vs < gcount; ++vs) {
            const View v = vpar[vs];
            const bool hq = vhq[vs] != 0;
            u64 *const fbv = (u64 *)vbuf[vs][0];
            uint32_t *const Dv = (uint32_t *)vbuf[vs][0];
            u64 *const Sv = (u64 *)vbuf[vs][1];
            uint32_t pids[PPT], dbs[PPT];
#pragma unroll
            for (int j = 0; j < PPT; ++j)
                pids[j] = project_wave(v, p[j], (uint64_t)(j * wg + threadIdx.x) < rem, dbs[j]);
            if (PASS == 0) {
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    const uint32_t pid = pids[j];
                    if (pid == kEmptyPid) continue;
                    const uint32_t key = (vs << kPidBits) | pid;
                    u64 val = hq ? (u64)dbs[j] : make_key(dbs[j], p[j].w);
                    uint32_t h = S.slot(key);
                    if (h != 0xFFFFFFFFu) {
                        lmin64(S.val + 2 * h, val);
                    } else if (hq) {
                        gmin_u32(Dv + pid, dbs[j]);
                    } else {
                        gmin_u64(fbv + pid, val);
                    }
                }
            } else {
                // All closest-depth reads of the tile back to back, then the sums.
                uint32_t dref[PPT];
#pragma unroll
                for (int j = 0; j < PPT; ++j) dref[j] = Dv[pids[j] != kEmptyPid ? pids[j] : 0u];
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    const uint32_t pid = pids[j];
                    if (pid == kEmptyPid) continue;
                    if (!(__uint_as_float(dbs[j]) <= __uint_as_float(dref[j]) * 1.01f)) continue;
                    const uint32_t key = (vs << kPidBits) | pid;
                    u64 r = p[j].w & 0xFFu, gg = (p[j].w >> 8) & 0xFFu, bl = (p[j].w >> 16) & 0xFFu;
                    u64 rg = (r << 32) | gg, ba = (bl << 32) | 1u;
                    uint32_t h = S.slot(key);
                    if (h != 0xFFFFFFFFu) {
                        __hip_atomic_fetch_add(S.val + 2 * h, rg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        __hip_atomic_fetch_add(S.val + 2 * h + 1, ba, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    } else {
                        gadd_u64(Sv + 2 * (u64)pid, rg);
                        gadd_u64(Sv + 2 * (u64)pid + 1, ba);
                    }
                }
            }
            // Flush early when the table is half full.  The decision must be
            // the same in every wave: all waves read the count between two
            // barriers, so none inserts again before all have read it.
            if (vs + 1 < gcount) {
                bar_lds();
                const uint32_t fill = (uint32_t)__builtin_amdgcn_readfirstlane((int)*S.count);
                bar_lds();
                if (fill > HS / 2) flush();
            }
        }
        flush();
    }
}

inline size_t batch_lds(uint32_t hbits) { return 16 + 24ull * (1u << hbits); }

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
    uint32_t hbits = 10;
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
    uint32_t grid_pass[2] = {0, 0}, grid_io = 0;
    // Per-view mode: the graph node of each (pass, slot) and whether it is
    // enabled in `exec`; slots a launch does not use are disabled, so they
    // cost no dispatch.
    std::vector<hipGraphNode_t> vnode[2];
    std::vector<uint8_t> von[2];
};

namespace pcr {
namespace {

// Workgroups of a batched pass without a set grid: as many as are resident at
// once on the device, so that no workgroup waits for another to finish its
// whole share.
int resident_grid(const void *fn, uint32_t wg, size_t sm, uint32_t &grid) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)wg, sm);
    if (e != hipSuccess || per_cu <= 0) return fail(PCR_EHIP, "occupancy query failed: %s", hipGetErrorString(e));
    grid = (uint32_t)per_cu * (uint32_t)device_cus();
    return PCR_OK;
}

// Workgroups of a batched pass: the plan's grid, or as many as are resident.
int pass_grid(const void *fn, const pcr_batch *b, size_t sm, uint32_t &grid) {
    if (b->sh.grid) {
        grid = b->sh.grid;
        return PCR_OK;
    }
    return resident_grid(fn, b->sh.wg, sm, grid);
}

int launch_pass(pcr_batch *b, int pass, hipStream_t s) {
    // pass < 0: only raise the kernels' LDS limit (done before graph capture).
    size_t sm = batch_lds(b->hbits);
#define PCR_BP(P)                                                                                      \
    case P:                                                                                            \
        if (pass < 0) {                                                                                \
            int rc = allow_lds((const void *)&k_batch_pass<P, 0>, sm);                                 \
            if (rc == PCR_OK) rc = allow_lds((const void *)&k_batch_pass<P, 1>, sm);                   \
            if (rc == PCR_OK) rc = pass_grid((const void *)&k_batch_pass<P, 0>, b, sm, b->grid_pass[0]);     \
            if (rc == PCR_OK) rc = pass_grid((const void *)&k_batch_pass<P, 1>, b, sm, b->grid_pass[1]);     \
            return rc;                                                                                 \
        }                                                                                              \
        if (pass)                                                                                      \
            hipLaunchKernelGGL((k_batch_pass<P, 1>), dim3(b->grid_pass[1]), dim3(b->sh.wg), sm, s, b->pts, b->n, \
                               b->dtable, b->lay, b->hbits);                                           \
        else                                                                                           \
            hipLaunchKernelGGL((k_batch_pass<P, 0>), dim3(b->grid_pass[0]), dim3(b->sh.wg), sm, s, b->pts, b->n, \
                               b->dtable, b->lay, b->hbits);                                           \
        break;
    switch (b->sh.ppt) {
        PCR_BP(1) PCR_BP(2) PCR_BP(4) PCR_BP(8) PCR_BP(16)
        default: return fail(PCR_EINVAL, "points per thread %u", b->sh.ppt);
    }
#undef PCR_BP
    PCR_LAUNCHED();
    return PCR_OK;
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
    if (t.group != 1) {  // the batched pass runs 64-, 128- or 256-thread workgroups
        if (t.wg == 0) t.wg = kBatchWg;
        if (t.wg > kBatchWg) return fail(PCR_EINVAL, "batched passes take at most %u threads per workgroup", kBatchWg);
    }
    Shape sh;
    int rc = resolve_shape(&t, PCR_DEDUP, sh);
    if (rc != PCR_OK) return rc;
    pcr_batch *b = new pcr_batch();
    b->pts = (const u32x4 *)pts;
    b->n = n;
    b->capacity = capacity;
    b->sh = sh;
    uint32_t want = sh.slots ? sh.slots : sh.wg * sh.ppt / 2;
    b->hbits = 8;
    while ((1u << b->hbits) < want && b->hbits < 14) ++b->hbits;
    if (batch_lds(b->hbits) > max_lds()) {
        destroy(b);
        return fail(PCR_EINVAL, "%u LDS slots do not fit", 1u << b->hbits);
    }
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
    rc = launch_pass(b, -1, nullptr);
    if (rc == PCR_OK && b->sh.group == 1) rc = view_passes(b, -1, nullptr);
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
    return a.ppt == b.ppt && a.wg == b.wg && a.grid == b.grid && a.group == b.group && a.slots == b.slots;
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
