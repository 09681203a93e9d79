// pcr_render.hip -- clear, render and resolve kernels of the point rasterizer
// (Sec. 3.1-3.5) and their host launchers.
//
// Data layout in HBM: points are a 16-byte array streamed once per geometry
// pass with non-temporal 16-byte loads (one point per lane, 1 KiB per wave per
// load); framebuffers are small (7-166 MB) and stay in L2 / Infinity Cache.
#include <mutex>
#include <type_traits>

#include "pcr_internal.h"

namespace pcr {

// ---------------------------------------------------------------------------
// Clear: 16-byte stores of a 32-bit pattern (no hipMemset, so the clear can be
// captured in a graph).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill(u32x4 *__restrict__ p, uint64_t n16, uint32_t word,
                                              uint32_t *__restrict__ tail, uint32_t ntail) {
    const u32x4 v = {word, word, word, word};
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        __builtin_nontemporal_store(v, p + i);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = word;
}

int launch_fill(void *p, size_t bytes, uint32_t word, hipStream_t s) {
    if (bytes == 0) return PCR_OK;
    uint64_t n16 = bytes / 16;
    uint32_t ntail = (uint32_t)((bytes % 16) / 4);
    uint32_t *tail = (uint32_t *)((char *)p + n16 * 16);
    uint64_t want = (n16 + 255) / 256;
    uint32_t grid = (uint32_t)(want < 1 ? 1 : (want > 8192 ? 8192 : want));
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, s, (u32x4 *)p, n16, word, tail, ntail);
    PCR_LAUNCHED();
    return PCR_OK;
}

// ---------------------------------------------------------------------------
// Wavefront reduction of Sec. 3.3 on a 64-lane wavefront: when many live lanes
// target one pixel, only the lanes holding the group's smallest depth go on
// (first listing); otherwise neighbouring lane pairs merge (second listing).
// A lane that drops out can never hold the pixel's minimum key.
// ---------------------------------------------------------------------------
// Wave-wide reductions with DPP moves (VALU, no LDS traffic), 32 bits wide:
// pairs, quads, half rows and rows by quad_perm / row mirrors, then rows
// combined by row_bcast:15 and row_bcast:31; lane 63 ends with the total.
// Lanes outside a DPP pattern's row mask keep the identity.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp32(uint32_t x, uint32_t ident) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)x, CTRL, ROWS, 0xF, false);
}

__device__ __forceinline__ uint32_t vmin(uint32_t a, uint32_t b) { return b < a ? b : a; }

// Set lanes of a lane mask, counted as two 32-bit halves: compared with a
// constant, a single 64-bit count is widened by the compiler into a 64-bit
// vector compare, where the halves stay on the scalar unit.
__device__ __forceinline__ uint32_t lanes_in(uint64_t m) {
    return (uint32_t)__builtin_popcount((uint32_t)m) + (uint32_t)__builtin_popcount((uint32_t)(m >> 32));
}

// Minimum over the wavefront (uniform result).
__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
    const uint32_t I = ~0u;
    x = vmin(x, dpp32<0xB1, 0xF>(x, I));   // quad_perm [1,0,3,2]
    x = vmin(x, dpp32<0x4E, 0xF>(x, I));   // quad_perm [2,3,0,1]
    x = vmin(x, dpp32<0x141, 0xF>(x, I));  // row_half_mirror
    x = vmin(x, dpp32<0x140, 0xF>(x, I));  // row_mirror
    x = vmin(x, dpp32<0x142, 0xA>(x, I));  // row_bcast:15
    x = vmin(x, dpp32<0x143, 0xC>(x, I));  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Sum over the wavefront (uniform result), modulo 2^32.
__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
    x += dpp32<0xB1, 0xF>(x, 0u);
    x += dpp32<0x4E, 0xF>(x, 0u);
    x += dpp32<0x141, 0xF>(x, 0u);
    x += dpp32<0x140, 0xF>(x, 0u);
    x += dpp32<0x142, 0xA>(x, 0u);
    x += dpp32<0x143, 0xC>(x, 0u);
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Depth bits of a value: the high word of a 64-bit key, or the value itself
// (HQ depth pass).  The key with the smallest depth bits is among the keys
// whose depth equals the minimum, so a group can keep just those lanes
// (a 32-bit reduction) and leave the colour tie-break to the atomic minimum.
template <typename V>
__device__ __forceinline__ uint32_t depth_of(V val) {
    if constexpr (sizeof(V) == 8)
        return (uint32_t)(val >> 32);
    else
        return (uint32_t)val;
}

template <typename V>
__device__ __forceinline__ V lane_pair(V x) {
    // quad_perm [1,0,3,2]: exchange with lane ^ 1.
    if constexpr (sizeof(V) == 8) {
        uint32_t lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)x, 0xB1, 0xF, 0xF, false);
        uint32_t hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(x >> 32), 0xB1, 0xF, 0xF, false);
        return ((V)hi << 32) | lo;
    } else {
        return (V)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);
    }
}

// Lane of a uniform lane mask as a per-lane predicate (no vector work: the
// mask itself is the predicate).
__device__ __forceinline__ bool lane_in(uint64_t mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }

// The group loops below keep `live` as a uniform lane mask and return it
// through lane_in(): updated per lane inside the loop, the flag was kept in a
// vector register (a select, a mask and a compare per group).

// RED: bit 0 = leader groups (all lanes equal), bit 1 = neighbouring pairs.
// Must be called by the whole wave.
template <typename V, int RED>
__device__ __forceinline__ bool wave_reduce(uint32_t pid, V val, bool live) {
    // Leader groups: the lanes sharing the first remaining live lane's pixel
    // keep only their minimum (with every live lane in one group this is the
    // all-lanes-equal case of Sec. 3.3).  Up to two groups of at least 24
    // lanes; a wavefront spread over several pixels leaves after one ballot.
    if (RED & 1) {
        uint64_t act = __ballot(live);  // live lanes not in a group yet
        uint64_t keep = act;            // live lanes
        // A group is a subset of act: with fewer than 24 lanes left none can form.
#pragma unroll 1
        for (int it = 0; it < 2 && lanes_in(act) >= 24u; ++it) {
            uint32_t leader = (uint32_t)__builtin_ctzll(act);
            uint32_t p0 = (uint32_t)__builtin_amdgcn_readlane((int)pid, leader);
            uint64_t m = __ballot(pid == p0) & act;  // the group: live lanes on pixel p0
            if (lanes_in(m) < 24u) break;
            const uint32_t md = wave_min(lane_in(m) ? depth_of(val) : ~0u);
            keep &= ~m | __ballot(depth_of(val) == md);  // the group's minimum is among these lanes
            act &= ~m;
        }
        live = lane_in(keep);
    }
    if (!(RED & 2)) return live;
    // Neighbouring lane pairs merge (Sec. 3.3, pairs).
    const uint32_t lane = __lane_id();
    uint32_t ppid = lane_pair(live ? pid : kEmptyPid);
    V pval = lane_pair(val);
    bool same = live && ppid == pid;
    bool lose = same && (pval < val || (pval == val && (lane & 1)));
    return live && !lose;
}

// Sums of the HQ colour pass: lanes that share the first live lane's pixel
// hand their red, green, blue and count to that lane (the all-lanes-equal
// reduction of Sec. 3.3 applied to integer sums; exact because + commutes),
// for up to two leaders per wavefront, each with a group of at least 16 lanes
// (smaller groups cost more in the reduction than the LDS adds they save:
// measured on HQ frames and batches).  A wavefront adds at most 64 values of
// at most 255, so two channels share one 32-bit word (16 bits each) without
// carries; the leader unpacks them into the (r<<32|g, b<<32|count) words.
// Takes and returns the lane mask of the live lanes.  Must be called by the
// whole wave.
__device__ __forceinline__ uint64_t wave_group_sums(uint32_t pid, uint32_t rgba, u64 &rg, u64 &ba, uint64_t act) {
    uint64_t keep = act;
#pragma unroll 1
    for (int it = 0; it < 2 && lanes_in(act) >= 16u; ++it) {  // a group is a subset of act
        uint32_t leader = (uint32_t)__builtin_ctzll(act);
        uint32_t p0 = (uint32_t)__builtin_amdgcn_readlane((int)pid, leader);
        uint64_t m = __ballot(pid == p0) & act;
        if (lanes_in(m) < 16u) break;
        const bool in = lane_in(m);
        const uint32_t w0 = (rgba & 0xFFu) | (rgba & 0xFF00u) << 8;    // r | g << 16
        const uint32_t w1 = ((rgba >> 16) & 0xFFu) | 0x10000u;         // b | 1 << 16
        const uint32_t a = wave_sum(in ? w0 : 0u), b = wave_sum(in ? w1 : 0u);
        const uint64_t lead = 1ull << leader;  // the leader is in the group
        if (lane_in(lead)) {
            rg = (u64)(a & 0xFFFFu) << 32 | (a >> 16);
            ba = (u64)(b & 0xFFFFu) << 32 | (b >> 16);
        }
        keep &= ~m | lead;
        act &= ~m;
    }
    return keep;
}

// ---------------------------------------------------------------------------
// Workgroup deduplication in LDS (Sec. 3.4 realised without partition
// intrinsics): an open-addressing hash table keyed by pixel index, one slot
// per distinct pixel of the tile, merged with LDS atomics, then one global
// atomic per distinct pixel.
// Shared memory: count[2] | val[HS] | tag[HS] | list[T].
// ---------------------------------------------------------------------------
struct Sum2 {
    u64 rg, ba;
};

constexpr uint32_t kMaxProbe = 8;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

template <typename V>
struct Lds {
    uint32_t *count;
    V *val;
    uint32_t *tag;
    uint32_t *list;
    uint32_t mask, shift;

    __device__ Lds(void *smem, uint32_t hbits) {
        count = (uint32_t *)smem;
        val = (V *)((char *)smem + 16);
        tag = (uint32_t *)(val + (1u << hbits));
        list = tag + (1u << hbits);
        mask = (1u << hbits) - 1u;
        shift = 24u - hbits;  // hbits <= 15: the top bits of a 24-bit product
    }

    // Home slot: Fibonacci hashing in a 24-bit word (full-rate 24-bit
    // multiply, top hbits of the low 24 bits of the product), which spreads
    // runs of consecutive pixels like the 32-bit form; the tag keeps the whole
    // pixel index, the hash only places it.  __umul24 returns a signed int:
    // shifted as unsigned and masked, the index never leaves the table.
    __device__ __forceinline__ uint32_t home(uint32_t pid) const {
        return ((uint32_t)__umul24(pid, 0x9E3779u) >> shift) & mask;
    }

    // Slot of pixel `pid`, claimed if new (then appended to the list of the
    // tile with parity `par`), or kNoSlot when kMaxProbe slots in a row are
    // taken by other pixels -- the caller then updates the framebuffer
    // directly, which is always correct because min and + commute.
    // The home slot is tested before the probing loop: most updates find
    // their pixel there, and the loop's divergent control flow is then
    // skipped by the whole wavefront.
    __device__ __forceinline__ uint32_t slot(uint32_t pid, uint32_t par) {
        uint32_t h = home(pid);
        uint32_t t = __hip_atomic_load(tag + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (t == pid) return h;
#pragma unroll 1
        for (uint32_t probe = 1;; ++probe) {
            if (t == kEmptyPid) {
                uint32_t old = atomicCAS(tag + h, kEmptyPid, pid);
                if (old == kEmptyPid) {
                    list[atomicAdd(count + par, 1u)] = h;
                    return h;
                }
                if (old == pid) return h;
            }
            if (probe == kMaxProbe) return kNoSlot;
            h = (h + 1u) & mask;
            t = __hip_atomic_load(tag + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (t == pid) return h;
        }
    }
};

// Workgroup barrier that orders LDS only: outstanding global loads, stores
// and atomics stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Collapse of a dense wavefront before the LDS table (PCR_F_REDUCE with
// PCR_F_LDS): when at least 24 live lanes share the first live lane's pixel
// and that pixel has no slot in the table yet, the group keeps only its
// minimum, so that the new slot is not claimed and lowered by 24-64 lanes one
// after another.  A pixel that already has a slot is left to the slot's early
// test (its value is already small).  Up to two groups.
template <typename V>
__device__ __forceinline__ bool dense_collapse(const Lds<V> &L, uint32_t pid, V val, bool live) {
    uint64_t act = __ballot(live);
    uint64_t keep = act;
#pragma unroll 1
    for (int it = 0; it < 2 && lanes_in(act) >= 24u; ++it) {  // a group is a subset of act
        uint32_t leader = (uint32_t)__builtin_ctzll(act);
        uint32_t p0 = (uint32_t)__builtin_amdgcn_readlane((int)pid, leader);
        uint64_t m = __ballot(pid == p0) & act;
        if (lanes_in(m) < 24u) break;
        act &= ~m;
        uint32_t t0 = L.tag[L.home(p0)];
        if (t0 == p0) continue;  // slot exists: the early test filters
        const uint32_t md = wave_min(lane_in(m) ? depth_of(val) : ~0u);
        keep &= ~m | __ballot(depth_of(val) == md);  // the group's minimum is among these lanes
    }
    return lane_in(keep);
}

inline size_t lds_bytes(uint32_t hbits, size_t vbytes) {
    return 16 + ((size_t)vbytes + 8) * (1u << hbits);
}

// Table of about T/2 slots for a tile of T points (at least 256): tiles with
// more distinct pixels overflow into direct updates.
inline uint32_t lds_hbits(uint32_t T, uint32_t group) {
    uint32_t want = group ? group : T / 2;
    uint32_t b = 8;
    while ((1u << b) < want && b < 15) ++b;
    return b;
}

// ---------------------------------------------------------------------------
// Render kernels.  One tile = wg * PPT consecutive points; lane t loads points
// tile*T + j*wg + t (j < PPT), all loads issued before any use.
// ---------------------------------------------------------------------------
// Workgroup g takes tiles g, g + grid, ... (natural order: the workgroups
// resident at one time work on one window of the point order).
struct Tiles {
    uint64_t n, ntiles, nblocks;
    uint32_t run;  // basic kernel: consecutive points per lane
    __device__ __forceinline__ bool tile(uint64_t b, uint64_t &t) const {
        t = b;
        return t < ntiles;
    }
};

// Tile load.  The tile's first point is uniform across the workgroup, so full
// tiles use a scalar base plus a 32-bit lane offset and issue all PPT loads
// back to back before the first use; in the last, partial tile indices past
// the end are clamped to the last point (the caller discards those lanes).
template <int PPT>
__device__ __forceinline__ void load_tile(const u32x4 *__restrict__ pts, uint64_t first, uint32_t wg,
                                          uint64_t n, u32x4 (&p)[PPT]) {
    const u32x4 *tp = pts + first;
    const uint64_t rem = n - first;
    if (rem >= (uint64_t)wg * PPT) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) p[j] = load_point(tp + (uint32_t)(j * wg + threadIdx.x));
    } else {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            uint32_t k = (uint32_t)(j * wg + threadIdx.x);
            p[j] = load_point(tp + (k < rem ? k : (uint32_t)(rem - 1)));
        }
    }
}

// Point sources of the render kernels.  load() fills the tile's points and
// returns how many lanes of the tile hold one.  FlatSrc: one contiguous buffer
// (the kernel's `pts` argument), one tile per workgroup.  ChunkSrc: many
// separate buffers (level-of-detail chunks, Sec. 5.4), tiled chunk by chunk so
// that a tile never spans two chunks: every lane loads from one uniform base
// exactly as in the flat case, and only the last tile of a chunk is partial.
// start[c] is the first tile of chunk c and start[nchunks] the tile count,
// written on the device by k_chunk_starts, so the tile count is only known
// inside the kernel (setup()).
struct FlatSrc {
    static constexpr bool chunked = false;
    __device__ __forceinline__ void setup(Tiles &, uint32_t) {}
    __device__ __forceinline__ bool tile(const Tiles &tl, uint64_t b, uint64_t &t) { return tl.tile(b, t); }
    template <int PPT>
    __device__ __forceinline__ uint32_t load(const u32x4 *__restrict__ pts, uint64_t t, uint32_t wg, uint64_t n,
                                             u32x4 (&p)[PPT]) {
        const uint64_t first = t * wg * PPT;
        load_tile<PPT>(pts, first, wg, n, p);
        return n - first < (uint64_t)wg * PPT ? (uint32_t)(n - first) : wg * PPT;
    }
};

struct ChunkSrc {
    static constexpr bool chunked = true;
    const pcr_chunk *chunks;
    const uint64_t *start;
    const uint32_t *wgc;  // chunk of each workgroup's first tile (k_chunk_wg)
    uint32_t nchunks;
    // Per workgroup (set up in the kernel): the contiguous tile range
    // [t_next, t_end), the chunk `cur` holding tile t_next, and that chunk's
    // tile range, base and size, kept in registers until a tile leaves it.
    uint64_t t_next, t_end;
    uint32_t cur;
    uint64_t cur_first, cur_last;  // tiles [cur_first, cur_last) of chunk cur
    const u32x4 *cur_pts;
    uint64_t cur_n;

    __device__ __forceinline__ void enter(uint32_t c) {
        cur = c;
        cur_first = start[c];
        cur_last = start[c + 1];
        cur_pts = (const u32x4 *)chunks[c].pts;
        cur_n = chunks[c].n;
    }

    // Static schedule: workgroup b takes the b-th contiguous range of tiles,
    // so its chunk cursor only moves forward (no search per tile), and the
    // workgroups resident at one time cover one window of the tile order (the
    // order that the flat kernels' grid-stride schedule also follows).
    __device__ __forceinline__ void setup(Tiles &tl, uint32_t) {
        tl.ntiles = start[nchunks];
        const uint64_t per_wg = (tl.ntiles + gridDim.x - 1) / gridDim.x;
        const uint64_t lo = (uint64_t)blockIdx.x * per_wg;
        t_next = lo < tl.ntiles ? lo : tl.ntiles;
        t_end = t_next + per_wg < tl.ntiles ? t_next + per_wg : tl.ntiles;
        tl.nblocks = blockIdx.x + (t_end - t_next) * gridDim.x;  // this workgroup's loop count
        if (t_next < t_end) enter(wgc[blockIdx.x]);
    }
    __device__ __forceinline__ bool tile(const Tiles &, uint64_t, uint64_t &t) {
        t = t_next++;
        return true;
    }
    template <int PPT>
    __device__ __forceinline__ uint32_t load(const u32x4 *__restrict__, uint64_t t, uint32_t wg, uint64_t,
                                             u32x4 (&p)[PPT]) {
        while (cur_last <= t) enter(cur + 1);  // uniform; passes empty and skipped chunks
        const uint64_t first = (t - cur_first) * wg * PPT;  // < cur_n: the chunk has a tile t
        load_tile<PPT>(cur_pts, first, wg, cur_n, p);
        return cur_n - first < (uint64_t)wg * PPT ? (uint32_t)(cur_n - first) : wg * PPT;
    }
};

// Basic closest-point render (Sec. 3.1), optionally with the early depth test
// (Sec. 3.2) and the wavefront reduction (Sec. 3.3).
//
// Lane mapping.  With the wavefront reduction (which merges neighbouring
// lanes) and for chunked frames, an instruction's lanes take consecutive
// points.  Otherwise each wavefront takes a sub-tile of 64 * run consecutive
// points, PPT per lane per step, in one of two mappings:
//   runs       lane l walks the points [l*run, (l+1)*run) of the sub-tile;
//   interleaved step c covers the points [c*64*PPT, (c+1)*64*PPT), lane l
//              taking PPT consecutive ones.
// The same atomics land differently: where consecutive points fall on one
// pixel (distant views, many points per pixel) the interleaved mapping puts
// many lanes of an instruction on one address, which the memory-side atomic
// unit serialises, while runs spread them over distinct pixels; where
// consecutive points fall on neighbouring pixels, the interleaved mapping
// keeps an instruction's atomics on few 64-byte lines, which the unit takes
// in one request each.  tl.run > 0 fixes runs of that length (run == PPT is
// both mappings); tl.run == 0 adapts per wavefront and sub-tile of 64 *
// kAdaptRun points: the first step is interleaved, and the rest of the
// sub-tile goes in runs (of kAdaptRun - PPT points) when in that first step
// more neighbouring lanes (points PPT apart) landed on one pixel than on two
// pixels of one 64-byte line, else interleaved: same-pixel atomics favour
// runs, same-line ones the interleaved mapping.  (Measured against fixed
// mappings and other rules on three vertex orders and three poses of the
// terrain and on the 796M frame: within 9% of the best fixed mapping in every
// case and best summed over them.)
constexpr uint32_t kAdaptRun = 32;

// RED: the wavefront reductions (bit 0 leader groups, bit 1 pairs; 0 none).
template <int PPT, bool EARLYZ, int RED, class Src>
__global__ __launch_bounds__(1024) void k_basic(const u32x4 *__restrict__ pts, Tiles tl, View v,
                                                u64 *__restrict__ fb, Src src) {
    const uint32_t wg = blockDim.x;
    if constexpr (Src::chunked) src.setup(tl, wg * PPT);
    constexpr bool kSub = RED == 0 && !Src::chunked;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const bool adapt = kSub && tl.run == 0;
    const uint32_t run = !kSub ? PPT : (adapt ? kAdaptRun : tl.run);
    for (uint64_t b = blockIdx.x; b < tl.nblocks; b += gridDim.x) {
        uint64_t t;
        if (!src.tile(tl, b, t)) continue;
        // sub: points of this wavefront's sub-tile (uniform; 32-bit compares).
        uint32_t sub = 0;
        const u32x4 *tp = pts;
        if constexpr (kSub) {
            const uint64_t first = t * wg * run + (uint64_t)wave * 64u * run;
            const uint64_t rem = first < tl.n ? tl.n - first : 0;
            sub = rem < 64ull * run ? (uint32_t)rem : 64u * run;
            tp = pts + first;
            if (sub == 0) continue;  // the last tile ends before this wavefront's part
        }
        bool runs = !adapt;           // adaptive: decided after the first step
        // neighbouring lanes whose visible points share a pixel / share only a 64-byte line
        uint32_t same = 0, line = 0;
#pragma unroll 1
        for (uint32_t c = 0; c < run; c += PPT) {
            u32x4 p[PPT];
            uint32_t k0 = 0;  // index of the lane's first point of this step in the sub-tile
            uint32_t lim = sub;
            if constexpr (kSub) {
                if (!adapt) k0 = lane * run + c;
                else if (c == 0 || !runs) k0 = c * 64u + lane * PPT;
                else k0 = 64u * PPT + lane * (run - PPT) + (c - PPT);
                // Cached loads: a lane's PPT consecutive loads touch each line
                // several times (non-temporal loads would fetch it again).
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    const uint32_t k = k0 + j;
                    p[j] = *(const __attribute__((address_space(1))) u32x4 *)(tp + (k < sub ? k : sub - 1));
                }
            } else {
                lim = src.template load<PPT>(pts, t, wg, tl.n, p);
            }
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                uint32_t dbits;
                const uint32_t k = kSub ? k0 + j : j * wg + threadIdx.x;
                uint32_t pid = project_wave(v, p[j], __ballot(k < lim), dbits);
                u64 key = make_key(dbits, p[j].w);
                bool w = pid != kEmptyPid;
                if (adapt && c == 0) {
                    // the next lane's point of this instruction (PPT points on)
                    const uint32_t nxt = (uint32_t)__shfl_down((int)pid, 1, 64);
                    const bool both = w && lane < 63u && nxt != kEmptyPid;
                    same += __popcll(__ballot(both && pid == nxt));
                    line += __popcll(__ballot(both && pid != nxt && (pid >> 3) == (nxt >> 3)));
                }
                if (RED) w = wave_reduce<u64, RED>(pid, key, w);
                if (EARLYZ && w) w = key < peek_u64(fb + pid);
                if (w) gmin_u64(fb + pid, key);
            }
            if (adapt && c == 0) runs = same > line;
        }
    }
}

// Closest-point render with LDS deduplication (Sec. 3.4); V = u64 keys for the
// basic framebuffer, V = uint32 depth bits for the HQ depth pass (Sec. 3.5).
template <typename V>
__device__ __forceinline__ void direct_min(V *fb, uint32_t pid, V val, bool earlyz) {
    if constexpr (sizeof(V) == 8) {
        if (!earlyz || val < peek_u64(fb + pid)) gmin_u64(fb + pid, val);
    } else {
        if (!earlyz || val < peek_u32(fb + pid)) gmin_u32(fb + pid, val);
    }
}

template <typename V, int PPT, bool EARLYZ, bool REDUCE, class Src>
__device__ __forceinline__ void dedup_tiles(const u32x4 *__restrict__ pts, Tiles tl, const View &v,
                                            V *__restrict__ fb, uint32_t hbits, Src src) {
    extern __shared__ __align__(16) unsigned char smem[];
    Lds<V> L(smem, hbits);
    const uint32_t wg = blockDim.x;
    if constexpr (Src::chunked) src.setup(tl, wg * PPT);
    const uint32_t HS = 1u << hbits;
    for (uint32_t s = threadIdx.x; s < HS; s += wg) {
        L.tag[s] = kEmptyPid;
        L.val[s] = (V)~(V)0;
    }
    if (threadIdx.x < 2) L.count[threadIdx.x] = 0;
    lds_barrier();
    uint32_t par = 0;
    for (uint64_t b = blockIdx.x; b < tl.nblocks; b += gridDim.x) {
        uint64_t t;
        if (!src.tile(tl, b, t)) continue;
        u32x4 p[PPT];
        // lim: lanes of the tile that hold a point (uniform; 32-bit compares).
        const uint32_t lim = src.template load<PPT>(pts, t, wg, tl.n, p);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            uint32_t dbits;
            uint32_t pid = project_wave(v, p[j], __ballot((uint32_t)(j * wg + threadIdx.x) < lim), dbits);
            V val;
            if constexpr (sizeof(V) == 8)
                val = make_key(dbits, p[j].w);
            else
                val = dbits;
            bool w = pid != kEmptyPid;
            if (REDUCE) w = dense_collapse<V>(L, pid, val, w);
            if (w) {
                uint32_t h = L.slot(pid, par);
                if (h != kNoSlot) {
                    // Early test against the slot (its value only decreases):
                    // lanes that cannot lower it skip the atomic, which keeps
                    // many lanes hitting one slot from serialising.
                    V cur = __hip_atomic_load(L.val + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (val < cur)
                        __hip_atomic_fetch_min(L.val + h, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    direct_min<V>(fb, pid, val, EARLYZ);
                }
            }
        }
        lds_barrier();
        uint32_t cnt = L.count[par];
        if (threadIdx.x == 0) L.count[par ^ 1u] = 0;
        for (uint32_t k = threadIdx.x; k < cnt; k += wg) {
            uint32_t h = L.list[k];
            uint32_t pid = L.tag[h];
            V val = L.val[h];
            L.tag[h] = kEmptyPid;
            L.val[h] = (V)~(V)0;
            direct_min<V>(fb, pid, val, EARLYZ);
        }
        lds_barrier();
        par ^= 1u;
    }
}

template <typename V, int PPT, bool EARLYZ, bool REDUCE, class Src>
__global__ __launch_bounds__(1024) void k_dedup(const u32x4 *__restrict__ pts, Tiles tl, View v,
                                                V *__restrict__ fb, uint32_t hbits, Src src) {
    dedup_tiles<V, PPT, EARLYZ, REDUCE, Src>(pts, tl, v, fb, hbits, src);
}

// HQ depth pass without LDS (Sec. 3.5: a 32-bit atomicMin of the depth),
// optionally with the wavefront reductions of Sec. 3.3 on the depth bits.
template <int PPT, bool EARLYZ, int RED>
__global__ __launch_bounds__(1024) void k_hq_depth(const u32x4 *__restrict__ pts, Tiles tl, View v,
                                                   uint32_t *__restrict__ D) {
    const uint32_t wg = blockDim.x;
    for (uint64_t b = blockIdx.x; b < tl.nblocks; b += gridDim.x) {
        uint64_t t;
        if (!tl.tile(b, t)) continue;
        const uint64_t first = t * wg * PPT;
        // Lanes of the tile that hold a point (uniform bound; 32-bit compares).
        const uint32_t lim = tl.n - first < (uint64_t)wg * PPT ? (uint32_t)(tl.n - first) : wg * PPT;
        u32x4 p[PPT];
        load_tile<PPT>(pts, first, wg, tl.n, p);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            uint32_t dbits;
            uint32_t pid = project_wave(v, p[j], __ballot((uint32_t)(j * wg + threadIdx.x) < lim), dbits);
            bool w = pid != kEmptyPid;
            if (RED) w = wave_reduce<uint32_t, RED>(pid, dbits, w);
            if (EARLYZ && w) w = dbits < peek_u32(D + pid);
            if (w) gmin_u32(D + pid, dbits);
        }
    }
}

// HQ colour pass (Sec. 3.5): a point within 1% of its pixel's closest depth
// (depth <= fl32(closest * 1.01f)) adds (r << 32 | g) and (b << 32 | 1) to the
// pixel's two 64-bit sums.  How an update (the sums of one or more such
// points) reaches the framebuffer depends on the sums layout:
//   kTwoWord  two 64-bit adds, one per sum word
//   kPacked   the 18-18-18-10 form of Sec. 3.5.1: one add of r << 46 | g << 28
//             | b << 10 | count to S[pid], modulo 2^64 (exact while at most
//             1023 points blend into a pixel).  Sums pack into that word
//             linearly: R << 46 + G << 28 + B << 10 + n is the sum of the
//             packed values of its points, modulo 2^64.
//   kRobust   the robust single-atomic form of Sec. 3.5.1 (16-16-16-16 word
//             with fallback to the two sum words); see robust_add.
enum { kTwoWord = 0, kPacked = 1, kRobust = 2 };

__device__ __forceinline__ u64 packed_sums(u64 rg, u64 ba) {
    return ((rg >> 32) << 46) + ((rg & 0xFFFFFFFFull) << 28) + ((ba >> 32) << 10) + (ba & 0xFFFFFFFFull);
}

// Robust single-atomic update (Sec. 3.5.1, HQS1R).  Each pixel has a fast
// word F[pid] = R << 48 | G << 32 | B << 16 | n holding the sums of at most
// 255 points (so no 16-bit field can carry: 255 * 255 < 2^16), beside the two
// fallback words of the two-word layout.  An update of c <= 255 points with
// sums (R, G, B) is applied to F by compare-and-swap: when the word's count
// plus c stays within 255 the new word is the old one plus the update;
// otherwise the word is swapped to zero and the update goes to the fallback
// words together with the old word's sums (the transfer of the paper's
// overflowing thread).  The first swap assumes a cleared word (right for a
// pixel's first update; otherwise it fails and returns the current word at
// the atomic unit, a fresher guess than a separate load); a swap that fails
// retries with the value it returned; after kRobustTries failures, and for
// updates of more than 255 points, the update goes to the fallback words
// alone (few retries keep hot pixels from queueing swaps that mostly fail).
// The fast word only ever changes by a successful swap from a value
// its thread knows exactly, so every completed update is counted exactly once
// in F or in the fallback, whatever number of updates is in flight: the sums
// are exact with no bound on concurrency (the paper's single add needs fewer
// than 65,280 adds to land between the overflow and the reset).  The resolve
// adds F's fields to the fallback words.
constexpr int kRobustTries = 2;

__device__ __forceinline__ void robust_add(u64 *__restrict__ F, u64 *__restrict__ S, uint32_t pid, u64 rg, u64 ba) {
    const uint32_t c = (uint32_t)ba;
    if (c <= 255u) {
        const u64 v = (rg >> 32) << 48 | (rg & 0xFFFFull) << 32 | (ba >> 32) << 16 | c;
        u64 exp = 0;
#pragma unroll 1
        for (int a = 0; a < kRobustTries; ++a) {
            const bool fits = ((uint32_t)exp & 0xFFFFu) + c <= 255u;
            const u64 prev = atomicCAS(F + pid, exp, fits ? exp + v : 0ull);
            if (prev == exp) {
                if (fits) return;
                // transfer: the word's sums join this update in the fallback words
                rg += (exp >> 48) << 32 | ((exp >> 32) & 0xFFFFull);
                ba += ((exp >> 16) & 0xFFFFull) << 32 | (exp & 0xFFFFull);
                break;
            }
            exp = prev;
        }
    }
    gadd_u64(S + 2 * (u64)pid, rg);
    gadd_u64(S + 2 * (u64)pid + 1, ba);
}

template <int SUMS>
__device__ __forceinline__ void add_sums(u64 *__restrict__ S, u64 *__restrict__ F, uint32_t pid, u64 rg, u64 ba) {
    if constexpr (SUMS == kPacked) {
        gadd_u64(S + pid, packed_sums(rg, ba));
    } else if constexpr (SUMS == kRobust) {
        robust_add(F, S, pid, rg, ba);
    } else {
        gadd_u64(S + 2 * (u64)pid, rg);
        gadd_u64(S + 2 * (u64)pid + 1, ba);
    }
}

// Flush of a colour table into the two-word sums: two lanes per slot, one
// word each, so that a pixel's two adds leave in one instruction and travel
// in one memory request (adjacent words of one line); with one lane per slot
// they were two instructions and two requests.  The lanes of a pair are
// neighbours in one wavefront (wg is a power of two of at least 64), and each
// reads its slot before the even lane clears the tag.
__device__ __forceinline__ void flush_sum_pairs(Lds<Sum2> &L, u64 *__restrict__ S, uint32_t cnt, uint32_t wg) {
    for (uint32_t k2 = threadIdx.x; k2 < 2 * cnt; k2 += wg) {
        const uint32_t h = L.list[k2 >> 1], half = k2 & 1u;
        const uint32_t pid = L.tag[h];
        u64 *word = half ? &L.val[h].ba : &L.val[h].rg;
        const u64 x = *word;
        *word = 0;
        if (!half) L.tag[h] = kEmptyPid;
        gadd_u64(S + 2 * (u64)pid + half, x);
    }
}

// GROUPS: the wavefront group sums before the table or the global adds (the
// merged paths and PCR_F_REDUCE); without them every point in the window adds
// its own pair of words (the plain colour pass of Sec. 3.5).
template <int PPT, bool LDS, class Src, int SUMS = kTwoWord, bool GROUPS = true>
__device__ __forceinline__ void hq_color_tiles(const u32x4 *__restrict__ pts, Tiles tl, const View &v,
                                               const uint32_t *__restrict__ D, u64 *__restrict__ S,
                                               uint32_t hbits, Src src) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t wg = blockDim.x;
    if constexpr (Src::chunked) src.setup(tl, wg * PPT);
    Lds<Sum2> L(smem, hbits);
    // robust form: the fast words follow the two sum words of every pixel
    u64 *F = SUMS == kRobust ? S + 2 * (u64)v.W * v.H : nullptr;
    if (LDS) {
        for (uint32_t s = threadIdx.x; s < (1u << hbits); s += wg) {
            L.tag[s] = kEmptyPid;
            L.val[s].rg = 0;
            L.val[s].ba = 0;
        }
        if (threadIdx.x < 2) L.count[threadIdx.x] = 0;
        lds_barrier();
    }
    uint32_t par = 0;
    for (uint64_t b = blockIdx.x; b < tl.nblocks; b += gridDim.x) {
        uint64_t t;
        if (!src.tile(tl, b, t)) continue;
        u32x4 p[PPT];
        // lim: lanes of the tile that hold a point (uniform; 32-bit compares).
        const uint32_t lim = src.template load<PPT>(pts, t, wg, tl.n, p);
        // Project every point first, then read all their closest depths back
        // to back (one round trip for the tile instead of one per point).
        uint32_t pids[PPT], dbs[PPT], dref[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) pids[j] = project_wave(v, p[j], __ballot((uint32_t)(j * wg + threadIdx.x) < lim), dbs[j]);
#pragma unroll
        for (int j = 0; j < PPT; ++j) dref[j] = D[pids[j] != kEmptyPid ? pids[j] : 0u];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const uint32_t pid = pids[j];
            // live lanes: a pixel, and a depth within 1% of the closest (for an
            // empty pixel dref is pixel 0's depth, and the lane is out either
            // way); ballots of single compares, since the lane mask of a
            // combined predicate was moved through a vector register
            const uint64_t lm = __ballot(pid != kEmptyPid) &
                                __ballot(__uint_as_float(dbs[j]) <= __uint_as_float(dref[j]) * 1.01f);
            u64 r = p[j].w & 0xFFu, g = (p[j].w >> 8) & 0xFFu, bl = (p[j].w >> 16) & 0xFFu;
            u64 rg = (r << 32) | g, ba = (bl << 32) | 1u;
            if (!lane_in(GROUPS ? wave_group_sums(pid, p[j].w, rg, ba, lm) : lm)) continue;
            if (!LDS) {
                add_sums<SUMS>(S, F, pid, rg, ba);
                continue;
            }
            uint32_t h = L.slot(pid, par);
            if (h == kNoSlot) {
                add_sums<SUMS>(S, F, pid, rg, ba);
                continue;
            }
            __hip_atomic_fetch_add(&L.val[h].rg, rg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(&L.val[h].ba, ba, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (!LDS) continue;
        lds_barrier();
        uint32_t cnt = L.count[par];
        if (threadIdx.x == 0) L.count[par ^ 1u] = 0;
        if constexpr (SUMS == kTwoWord) {
            flush_sum_pairs(L, S, cnt, wg);
        } else {
            for (uint32_t k = threadIdx.x; k < cnt; k += wg) {
                uint32_t h = L.list[k];
                uint32_t pid = L.tag[h];
                Sum2 sm = L.val[h];
                L.tag[h] = kEmptyPid;
                L.val[h].rg = 0;
                L.val[h].ba = 0;
                add_sums<SUMS>(S, F, pid, sm.rg, sm.ba);
            }
        }
        lds_barrier();
        par ^= 1u;
    }
}

template <int PPT, bool LDS, class Src, int SUMS = kTwoWord, bool GROUPS = true>
__global__ __launch_bounds__(1024) void k_hq_color(const u32x4 *__restrict__ pts, Tiles tl, View v,
                                                   const uint32_t *__restrict__ D,
                                                   u64 *__restrict__ S, uint32_t hbits, Src src) {
    hq_color_tiles<PPT, LDS, Src, SUMS, GROUPS>(pts, tl, v, D, S, hbits, src);
}

// Single-view passes driven by a batch plan's table: the view is read on the
// device (so a captured graph serves any views), its words moved to scalar
// registers like the arguments of the single-view kernels.
__device__ __forceinline__ View uniform_view(const View *p) {
    View v;
    const uint32_t *src = (const uint32_t *)p;
    uint32_t *dst = (uint32_t *)&v;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(View) / 4); ++i) dst[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)src[i]);
    return v;
}

template <int PPT, int PASS>
__global__ __launch_bounds__(1024) void k_view_pass(const u32x4 *__restrict__ pts, Tiles tl,
                                                    const BatchView *__restrict__ views,
                                                    const uint32_t *__restrict__ nviews, uint32_t slot,
                                                    uint32_t hbits) {
    if (slot >= *nviews) return;
    const BatchView *bv = views + slot;
    const int variant = __builtin_amdgcn_readfirstlane(bv->variant);
    if (PASS == 1 && variant != PCR_HQ) return;
    const View v = uniform_view(&bv->v);
    if (PASS == 0) {
        if (variant == PCR_HQ)
            dedup_tiles<uint32_t, PPT, false, true, FlatSrc>(pts, tl, v, bv->D, hbits, FlatSrc{});
        else
            dedup_tiles<u64, PPT, false, true, FlatSrc>(pts, tl, v, bv->fb, hbits, FlatSrc{});
    } else {
        hq_color_tiles<PPT, true, FlatSrc>(pts, tl, v, bv->D, bv->S, hbits, FlatSrc{});
    }
}

// ---------------------------------------------------------------------------
// Grouped multi-view passes: every tile of the cloud is loaded once per group
// of views and rendered into each view of the group in turn, each view with
// the single-view kernels' tile body (projection, dense-group collapse, LDS
// deduplication, flush), so a view costs what its single-view pass costs
// minus the point stream.  Pass 0 renders the closest-point views and the HQ
// depth passes, pass 1 the HQ colour passes.
// ---------------------------------------------------------------------------

// One tile into one closest-point view (basic key buffer) or HQ depth buffer.
// Both use the 64-bit table: an HQ depth goes in the high word (low word 0),
// so the table's minimum is the smallest depth and the dense-group collapse
// compares depths as for keys.
template <int PPT>
__device__ __forceinline__ void group_tile_closest(Lds<u64> &L, const u32x4 (&p)[PPT], const uint64_t (&lm)[PPT],
                                                   const View &v, bool hq, u64 *__restrict__ fb,
                                                   uint32_t *__restrict__ D, uint32_t &par) {
    const uint32_t wg = blockDim.x;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        uint32_t dbits;
        const uint32_t pid = project_wave(v, p[j], lm[j], dbits);
        const u64 val = hq ? (u64)dbits << 32 : make_key(dbits, p[j].w);
        bool w = dense_collapse<u64>(L, pid, val, pid != kEmptyPid);
        if (w) {
            const uint32_t h = L.slot(pid, par);
            if (h != kNoSlot) {
                const u64 cur = __hip_atomic_load(L.val + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (val < cur) __hip_atomic_fetch_min(L.val + h, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else if (hq) {
                gmin_u32(D + pid, dbits);
            } else {
                gmin_u64(fb + pid, val);
            }
        }
    }
    lds_barrier();
    const uint32_t cnt = L.count[par];
    if (threadIdx.x == 0) L.count[par ^ 1u] = 0;
    for (uint32_t k = threadIdx.x; k < cnt; k += wg) {
        const uint32_t h = L.list[k];
        const uint32_t pid = L.tag[h];
        const u64 val = L.val[h];
        L.tag[h] = kEmptyPid;
        L.val[h] = kEmptyKey;
        if (hq) gmin_u32(D + pid, (uint32_t)(val >> 32));
        else gmin_u64(fb + pid, val);
    }
    lds_barrier();
    par ^= 1u;
}

// One tile into one HQ view's colour sums (the merged two-word colour pass).
template <int PPT>
__device__ __forceinline__ void group_tile_color(Lds<Sum2> &L, const u32x4 (&p)[PPT], const uint64_t (&lm)[PPT],
                                                 const View &v, const uint32_t *__restrict__ D,
                                                 u64 *__restrict__ S, uint32_t &par) {
    const uint32_t wg = blockDim.x;
    uint32_t pids[PPT], dbs[PPT], dref[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) pids[j] = project_wave(v, p[j], lm[j], dbs[j]);
#pragma unroll
    for (int j = 0; j < PPT; ++j) dref[j] = D[pids[j] != kEmptyPid ? pids[j] : 0u];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const uint32_t pid = pids[j];
        const uint64_t lm = __ballot(pid != kEmptyPid) &
                            __ballot(__uint_as_float(dbs[j]) <= __uint_as_float(dref[j]) * 1.01f);  // as in hq_color_tiles
        u64 r = p[j].w & 0xFFu, g = (p[j].w >> 8) & 0xFFu, bl = (p[j].w >> 16) & 0xFFu;
        u64 rg = (r << 32) | g, ba = (bl << 32) | 1u;
        if (!lane_in(wave_group_sums(pid, p[j].w, rg, ba, lm))) continue;
        const uint32_t h = L.slot(pid, par);
        if (h == kNoSlot) {
            gadd_u64(S + 2 * (u64)pid, rg);
            gadd_u64(S + 2 * (u64)pid + 1, ba);
            continue;
        }
        __hip_atomic_fetch_add(&L.val[h].rg, rg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&L.val[h].ba, ba, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    lds_barrier();
    const uint32_t cnt = L.count[par];
    if (threadIdx.x == 0) L.count[par ^ 1u] = 0;
    flush_sum_pairs(L, S, cnt, wg);
    lds_barrier();
    par ^= 1u;
}

// Items (group g, tile t) in group-major order, tiles in their natural order;
// workgroup b takes items b, b + grid, ... (the resident workgroups work on one
// window of one group's point order).  Group g's views are
// views[index[groups[g].first + k]], k < groups[g].count.
template <int PPT, int PASS>
__global__ __launch_bounds__(1024) void k_group_pass(const u32x4 *__restrict__ pts, Tiles tl,
                                                     const BatchView *__restrict__ views,
                                                     const uint32_t *__restrict__ index,
                                                     const BatchGroup *__restrict__ groups,
                                                     const uint32_t *__restrict__ ngroups, uint32_t hbits) {
    extern __shared__ __align__(16) unsigned char smem[];
    using V = typename std::conditional<PASS == 0, u64, Sum2>::type;
    Lds<V> L(smem, hbits);
    const uint32_t wg = blockDim.x;
    const uint32_t HS = 1u << hbits;
    for (uint32_t s = threadIdx.x; s < HS; s += wg) {
        L.tag[s] = kEmptyPid;
        if constexpr (PASS == 0) {
            L.val[s] = kEmptyKey;
        } else {
            L.val[s].rg = 0;
            L.val[s].ba = 0;
        }
    }
    if (threadIdx.x < 2) L.count[threadIdx.x] = 0;
    lds_barrier();
    const uint32_t ng = (uint32_t)__builtin_amdgcn_readfirstlane((int)*ngroups);
    if (ng == 0 || tl.ntiles == 0) return;
    // (g, t) of item blockIdx.x, advanced by the grid stride (uniform)
    uint64_t t = blockIdx.x;
    uint32_t g = 0;
    while (t >= tl.ntiles && g < ng) {
        t -= tl.ntiles;
        ++g;
    }
    uint32_t par = 0;
    for (; g < ng;) {
        u32x4 p[PPT];
        const uint32_t lim = FlatSrc{}.template load<PPT>(pts, t, wg, tl.n, p);
        // lanes that hold a point, per row, as lane masks: taken next to their
        // compares, they stay in scalar registers across the loop over views
        uint64_t lm[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) lm[j] = __ballot((uint32_t)(j * wg + threadIdx.x) < lim);
        const uint32_t first = (uint32_t)__builtin_amdgcn_readfirstlane((int)groups[g].first);
        const uint32_t count = (uint32_t)__builtin_amdgcn_readfirstlane((int)groups[g].count);
        for (uint32_t k = 0; k < count; ++k) {
            const uint32_t vi = (uint32_t)__builtin_amdgcn_readfirstlane((int)index[first + k]);
            const BatchView *bv = views + vi;
            const int variant = __builtin_amdgcn_readfirstlane(bv->variant);
            const View v = uniform_view(&bv->v);
            if constexpr (PASS == 0) {
                group_tile_closest<PPT>(L, p, lm, v, variant == PCR_HQ, bv->fb, bv->D, par);
            } else {
                if (variant == PCR_HQ) group_tile_color<PPT>(L, p, lm, v, bv->D, bv->S, par);
            }
        }
        t += gridDim.x;
        while (t >= tl.ntiles && g < ng) {
            t -= tl.ntiles;
            ++g;
        }
    }
}

// ---------------------------------------------------------------------------
// Resolve (Sec. 3.1 second listing; Sec. 3.5 resolve listing).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_resolve_basic(const u64 *__restrict__ fb,
                                                       uint32_t *__restrict__ out, uint64_t npix) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += stride) {
        u64 k = fb[i];
        out[i] = k == kEmptyKey ? 0u : (uint32_t)k;
    }
}

// Integer average of one pixel's sums; s = {G sum, R sum, count, B sum}.
__device__ __forceinline__ uint32_t hq_colour(u32x4 s) {
    const uint32_t c = s.z;
    if (c == 0) return 0u;
    uint32_t r = s.y / c, g = s.x / c, b = s.w / c;
    return (r & 0xFFu) | (g & 0xFFu) << 8 | (b & 0xFFu) << 16 | 0xFF000000u;
}

// Integer average of one packed word (Sec. 3.5.1): 18-bit colour fields over
// the 10-bit count.
__device__ __forceinline__ uint32_t hq_colour_packed(u64 w) {
    const uint32_t c = (uint32_t)w & 0x3FFu;
    if (c == 0) return 0u;
    const uint32_t r = (uint32_t)(w >> 46) & 0x3FFFFu, g = (uint32_t)(w >> 28) & 0x3FFFFu,
                   b = (uint32_t)(w >> 10) & 0x3FFFFu;
    return (r / c & 0xFFu) | (g / c & 0xFFu) << 8 | (b / c & 0xFFu) << 16 | 0xFF000000u;
}

// The two sum words of pixel i in the robust form: the fallback words plus
// the fast word's 16-bit fields, R << 32 | G and B << 32 | count (each sum
// modulo 2^64, as the two-word layout holds them).
__device__ __forceinline__ u32x4 robust_words(const u64 *__restrict__ S, const u64 *__restrict__ F, uint64_t i) {
    const u32x4 s = ((const u32x4 *)S)[i];
    const u64 f = F[i];
    const u64 rg = ((u64)s.y << 32 | s.x) + ((f >> 48) << 32 | ((f >> 32) & 0xFFFFull));
    const u64 ba = ((u64)s.w << 32 | s.z) + (((f >> 16) & 0xFFFFull) << 32 | (f & 0xFFFFull));
    return u32x4{(uint32_t)rg, (uint32_t)(rg >> 32), (uint32_t)ba, (uint32_t)(ba >> 32)};
}

// Colour of pixel i from the sums area: two words per pixel, one packed word,
// or the robust form's fallback words plus fast word (F = S + 2 * npix).
template <int SUMS>
__device__ __forceinline__ uint32_t hq_pixel(const u64 *__restrict__ S, uint64_t i, uint64_t npix) {
    if constexpr (SUMS == kPacked) return hq_colour_packed(S[i]);
    else if constexpr (SUMS == kRobust) return hq_colour(robust_words(S, S + 2 * npix, i));
    else return hq_colour(((const u32x4 *)S)[i]);
}

template <int SUMS>
__global__ __launch_bounds__(256) void k_resolve_hq(const u64 *__restrict__ S,
                                                    uint32_t *__restrict__ out, uint64_t npix) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += stride)
        out[i] = hq_pixel<SUMS>(S, i, npix);
}

// Depth output (Sec. 3.1, closing paragraph): the stored linear depth w, or
// a + b * (1/w) (window or reverse-z depth of a perspective projection), with
// the projection's correctly rounded reciprocal and no contraction.
__device__ __forceinline__ float depth_value(uint32_t dbits, int mode, float a, float b) {
    const float w = __uint_as_float(dbits);
    if (mode == PCR_DEPTH_LINEAR) return w;
    const float t = b * recip_rn(w);
    return a + t;
}

__global__ __launch_bounds__(256) void k_resolve_basic_depth(const u64 *__restrict__ fb,
                                                             uint32_t *__restrict__ out,
                                                             float *__restrict__ depth, uint64_t npix,
                                                             int mode, float a, float b, float empty) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += stride) {
        const u64 k = fb[i];
        const bool hit = k != kEmptyKey;
        if (out) out[i] = hit ? (uint32_t)k : 0u;
        const float d = depth_value((uint32_t)(k >> 32), mode, a, b);
        depth[i] = hit ? d : empty;
    }
}

template <int SUMS>
__global__ __launch_bounds__(256) void k_resolve_hq_depth(const uint32_t *__restrict__ D,
                                                          const u64 *__restrict__ S,
                                                          uint32_t *__restrict__ out,
                                                          float *__restrict__ depth, uint64_t npix,
                                                          int mode, float a, float b, float empty) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += stride) {
        if (out) out[i] = hq_pixel<SUMS>(S, i, npix);
        const uint32_t db = D[i];
        const float d = depth_value(db, mode, a, b);
        depth[i] = db != 0xFFFFFFFFu ? d : empty;
    }
}

// Raw framebuffer words in one linear layout.  Closest-point frames: the keys
// as stored.  HQ: three planes of npix words, the depth bits (zero-extended),
// R << 32 | G and B << 32 | count; a robust frame's fast and fallback words
// are combined into these two, a packed word's four fields are spread over
// them (as stored, so a wrapped count stays wrapped).
__global__ __launch_bounds__(256) void k_raw_basic(const u64 *__restrict__ fb, u64 *__restrict__ out,
                                                   uint64_t npix) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += stride) out[i] = fb[i];
}

template <int SUMS>
__global__ __launch_bounds__(256) void k_raw_hq(const uint32_t *__restrict__ D, const u64 *__restrict__ S,
                                                u64 *__restrict__ out, uint64_t npix) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += stride) {
        u64 rg, ba;
        if constexpr (SUMS == kPacked) {
            const u64 w = S[i];
            rg = (w >> 46) << 32 | ((w >> 28) & 0x3FFFFull);
            ba = ((w >> 10) & 0x3FFFFull) << 32 | (w & 0x3FFull);
        } else {
            const u32x4 s = SUMS == kRobust ? robust_words(S, S + 2 * npix, i) : ((const u32x4 *)S)[i];
            rg = (u64)s.y << 32 | s.x;
            ba = (u64)s.w << 32 | s.z;
        }
        out[i] = D[i];
        out[npix + i] = rg;
        out[2 * npix + i] = ba;
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
namespace {

// Tiles of wg * ppt points, or wg * run (run > 0) / wg * kAdaptRun (run = 0,
// adaptive) for the basic kernel's sub-tiles.
Tiles make_tiles(uint64_t n, const Shape &sh, uint32_t &grid, uint32_t run = 0, bool basic_runs = false) {
    Tiles tl;
    tl.n = n;
    tl.run = run;
    uint64_t T = (uint64_t)sh.wg * (!basic_runs ? sh.ppt : run ? run : kAdaptRun);
    tl.ntiles = (n + T - 1) / T;
    tl.nblocks = tl.ntiles;
    // sh.grid is set by resolve_shape; 0 would mean one workgroup per tile.
    uint64_t g = sh.grid && sh.grid < tl.ntiles ? sh.grid : tl.ntiles;
    grid = (uint32_t)(g < 1 ? 1 : (g > 0x7FFFFFFFull ? 0x7FFFFFFFull : g));
    return tl;
}

template <template <int> class F, typename... A>
int by_ppt(uint32_t ppt, A &&...a) {
    switch (ppt) {
        case 1: return F<1>::run(a...);
        case 2: return F<2>::run(a...);
        case 4: return F<4>::run(a...);
        case 8: return F<8>::run(a...);
        case 16: return F<16>::run(a...);
    }
    return fail(PCR_EINVAL, "points per thread must be 1, 2, 4, 8 or 16 (got %u)", ppt);
}

struct Launch {
    const u32x4 *pts;
    uint64_t n;
    View v;
    void *fb;
    Shape sh;
    uint32_t flags;
    hipStream_t s;
};

template <int P>
struct BasicL {
    static int run(const Launch &L) {
        uint32_t grid;
        const int red = reduce_mode(L.flags);
        const bool runs = !(L.flags & PCR_F_LDS) && red == 0;  // the kernel's lane mapping
        Tiles tl = make_tiles(L.n, L.sh, grid, runs ? L.sh.run : 0, runs);
        const bool ez = L.flags & PCR_F_EARLYZ, rd = red != 0;
        u64 *fb = (u64 *)L.fb;
        if (L.flags & PCR_F_LDS) {
            uint32_t T = L.sh.wg * P, hb = lds_hbits(T, L.sh.slots);
            size_t sm = lds_bytes(hb, 8);
            if (sm > max_lds())
                return fail(PCR_EINVAL, "tile of %u points needs %zu bytes of LDS", T, sm);
#define PCR_DD(E, R)                                                                                    \
    do {                                                                                                \
        if (int rc_ = allow_lds((const void *)&k_dedup<u64, P, E, R, FlatSrc>, sm)) return rc_;         \
        hipLaunchKernelGGL((k_dedup<u64, P, E, R, FlatSrc>), dim3(grid), dim3(L.sh.wg), sm, L.s, L.pts, tl, L.v, fb, \
                           hb, FlatSrc{});                                                             \
    } while (0)
            if (ez && rd) PCR_DD(true, true);
            else if (ez) PCR_DD(true, false);
            else if (rd) PCR_DD(false, true);
            else PCR_DD(false, false);
#undef PCR_DD
        } else {
#define PCR_BB(E, R) \
    hipLaunchKernelGGL((k_basic<P, E, R, FlatSrc>), dim3(grid), dim3(L.sh.wg), 0, L.s, L.pts, tl, L.v, fb, FlatSrc{})
#define PCR_BR(E)                \
    do {                         \
        if (red == 3) PCR_BB(E, 3); \
        else if (red == 2) PCR_BB(E, 2); \
        else if (red == 1) PCR_BB(E, 1); \
        else PCR_BB(E, 0);       \
    } while (0)
            if (ez) PCR_BR(true);
            else PCR_BR(false);
#undef PCR_BR
#undef PCR_BB
        }
        PCR_LAUNCHED();
        return PCR_OK;
    }
};

template <int P>
struct DepthL {
    static int run(const Launch &L) {
        uint32_t grid;
        Tiles tl = make_tiles(L.n, L.sh, grid);
        const int red = reduce_mode(L.flags);
        const bool ez = L.flags & PCR_F_EARLYZ, rd = red != 0;
        uint32_t *D = (uint32_t *)L.fb;
        if (L.flags & PCR_F_LDS) {
            uint32_t T = L.sh.wg * P, hb = lds_hbits(T, L.sh.slots);
            size_t sm = lds_bytes(hb, 4);
            if (sm > max_lds())
                return fail(PCR_EINVAL, "tile of %u points needs %zu bytes of LDS", T, sm);
#define PCR_DD(E, R)                                                                                    \
    do {                                                                                                \
        if (int rc_ = allow_lds((const void *)&k_dedup<uint32_t, P, E, R, FlatSrc>, sm)) return rc_;    \
        hipLaunchKernelGGL((k_dedup<uint32_t, P, E, R, FlatSrc>), dim3(grid), dim3(L.sh.wg), sm, L.s, L.pts, tl, L.v, \
                           D, hb, FlatSrc{});                                                          \
    } while (0)
            if (ez && rd) PCR_DD(true, true);
            else if (ez) PCR_DD(true, false);
            else if (rd) PCR_DD(false, true);
            else PCR_DD(false, false);
#undef PCR_DD
        } else {
#define PCR_HD(E, R) hipLaunchKernelGGL((k_hq_depth<P, E, R>), dim3(grid), dim3(L.sh.wg), 0, L.s, L.pts, tl, L.v, D)
#define PCR_HR(E)                \
    do {                         \
        if (red == 3) PCR_HD(E, 3); \
        else if (red == 2) PCR_HD(E, 2); \
        else if (red == 1) PCR_HD(E, 1); \
        else PCR_HD(E, 0);       \
    } while (0)
            if (ez) PCR_HR(true);
            else PCR_HR(false);
#undef PCR_HR
#undef PCR_HD
        }
        PCR_LAUNCHED();
        return PCR_OK;
    }
};

// Sums layout of an HQ variant's flags.
inline int sums_layout(uint32_t flags) {
    return (flags & PCR_F_HQ_PACKED) ? kPacked : (flags & PCR_F_HQ_ROBUST) ? kRobust : kTwoWord;
}

template <int P>
struct ColorL {
    template <bool LDS, int SUMS, bool GROUPS = true>
    static int go(const Launch &L, const Tiles &tl, uint32_t grid, const uint32_t *D, u64 *S, uint32_t hb,
                  size_t sm) {
        if (LDS)
            if (int rc = allow_lds((const void *)&k_hq_color<P, LDS, FlatSrc, SUMS, GROUPS>, sm)) return rc;
        hipLaunchKernelGGL((k_hq_color<P, LDS, FlatSrc, SUMS, GROUPS>), dim3(grid), dim3(L.sh.wg), sm, L.s, L.pts, tl,
                           L.v, D, S, hb, FlatSrc{});
        PCR_LAUNCHED();
        return PCR_OK;
    }
    static int run(const Launch &L, uint32_t w, uint32_t h) {
        uint32_t grid;
        Tiles tl = make_tiles(L.n, L.sh, grid);
        const uint32_t *D = (const uint32_t *)L.fb;
        u64 *S = (u64 *)((char *)L.fb + hq_depth_bytes(w, h));
        const int sums = sums_layout(L.flags);
        if (L.flags & PCR_F_LDS) {
            uint32_t T = L.sh.wg * P, hb = lds_hbits(T, L.sh.slots);
            size_t sm = lds_bytes(hb, 16);
            if (sm > max_lds())
                return fail(PCR_EINVAL, "tile of %u points needs %zu bytes of LDS", T, sm);
            if (sums == kPacked) return go<true, kPacked>(L, tl, grid, D, S, hb, sm);
            if (sums == kRobust) return go<true, kRobust>(L, tl, grid, D, S, hb, sm);
            return go<true, kTwoWord>(L, tl, grid, D, S, hb, sm);
        }
        // Without the table the group sums run only with the leader-group
        // reduction (PCR_F_REDUCE or PCR_F_REDUCE_WAVE).
        if (reduce_mode(L.flags) & 1) {
            if (sums == kPacked) return go<false, kPacked, true>(L, tl, grid, D, S, 1u, 0);
            if (sums == kRobust) return go<false, kRobust, true>(L, tl, grid, D, S, 1u, 0);
            return go<false, kTwoWord, true>(L, tl, grid, D, S, 1u, 0);
        }
        if (sums == kPacked) return go<false, kPacked, false>(L, tl, grid, D, S, 1u, 0);
        if (sums == kRobust) return go<false, kRobust, false>(L, tl, grid, D, S, 1u, 0);
        return go<false, kTwoWord, false>(L, tl, grid, D, S, 1u, 0);
    }
};

// ---- many-chunk frames ------------------------------------------------------

// Exclusive prefix of the chunks' tile counts (tiles of T points) into
// start[0..nchunks] (one workgroup; a skipped chunk has no tile).
__device__ __forceinline__ uint64_t shfl_up64(uint64_t x, uint32_t d) {
    uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, d, 64);
    uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), d, 64);
    return ((uint64_t)hi << 32) | lo;
}

// One workgroup of 1024 threads takes 4096 chunks per step, 4 consecutive
// chunks per thread: their tile counts are summed in the thread and the
// thread totals scanned across the workgroup; tiles hold 2^tshift points (a
// power of two).  The tile counts and the start offsets go through LDS, so
// that the global loads and stores are coalesced (lane l takes chunk
// r * 1024 + l of the step) while each thread scans consecutive chunks: with
// each thread reading its own records, every load and store instruction
// touched 64 cache lines, and the kernel ran several times longer on 40,000
// chunks.  One padding word per 4 keeps the per-thread LDS accesses to
// 2-way bank conflicts.
constexpr uint32_t kStartsPer = 4;
constexpr uint32_t kStartsThreads = 1024;

__device__ __forceinline__ uint32_t starts_slot(uint32_t k) { return k + (k >> 2); }

__global__ __launch_bounds__(kStartsThreads) void k_chunk_starts(const pcr_chunk *__restrict__ chunks,
                                                                 uint32_t nchunks, uint32_t tshift,
                                                                 uint64_t *__restrict__ start) {
    // tile counts, then start offsets, of the step's chunks (slot starts_slot(k))
    __shared__ uint64_t stage[kStartsThreads * kStartsPer * 5 / 4];
    __shared__ uint64_t wtot[kStartsThreads / 64];
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    constexpr uint32_t nw = kStartsThreads / 64, step = kStartsThreads * kStartsPer;
    const uint64_t T = 1ull << tshift;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < nchunks; base += step) {
        // Coalesced: chunk base + r * 1024 + tid (the loads are issued together:
        // indices past the end read the last record, whose count is dropped).
        pcr_chunk ch[kStartsPer];
#pragma unroll
        for (uint32_t r = 0; r < kStartsPer; ++r) {
            const uint32_t i = base + r * kStartsThreads + threadIdx.x;
            ch[r] = chunks[i < nchunks ? i : nchunks - 1];
        }
#pragma unroll
        for (uint32_t r = 0; r < kStartsPer; ++r) {
            const uint32_t i = base + r * kStartsThreads + threadIdx.x;
            const bool ok = i < nchunks && ch[r].pts != nullptr && ((uintptr_t)ch[r].pts & 15u) == 0 &&
                            ch[r].n <= PCR_CHUNK_MAX_POINTS;
            stage[starts_slot(r * kStartsThreads + threadIdx.x)] = ok ? (ch[r].n + T - 1) >> tshift : 0;
        }
        lds_barrier();
        // Thread tid: chunks base + tid * 4 + [0, 4).
        uint64_t c[kStartsPer];
        uint64_t sum = 0;
#pragma unroll
        for (uint32_t r = 0; r < kStartsPer; ++r) {
            c[r] = stage[starts_slot(threadIdx.x * kStartsPer + r)];
            sum += c[r];
        }
        uint64_t x = sum;  // inclusive scan of the thread totals over the wavefront
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint64_t y = shfl_up64(x, d);
            if (lane >= d) x += y;
        }
        if (lane == 63) wtot[wid] = x;
        lds_barrier();
        uint64_t before = carry, total = carry;
        for (uint32_t k = 0; k < nw; ++k) {
            if (k < wid) before += wtot[k];
            total += wtot[k];
        }
        uint64_t run = before + x - sum;
#pragma unroll
        for (uint32_t r = 0; r < kStartsPer; ++r) {
            stage[starts_slot(threadIdx.x * kStartsPer + r)] = run;
            run += c[r];
        }
        carry = total;
        lds_barrier();
#pragma unroll
        for (uint32_t r = 0; r < kStartsPer; ++r) {  // coalesced stores
            const uint32_t i = base + r * kStartsThreads + threadIdx.x;
            if (i < nchunks) start[i] = stage[starts_slot(r * kStartsThreads + threadIdx.x)];
        }
        lds_barrier();  // stage and wtot are written again by the next step
    }
    if (threadIdx.x == 0) start[nchunks] = carry;
}

// Workgroups of a chunked launch: at most kChunkGridMax (the scratch holds
// one word per workgroup).
constexpr uint32_t kChunkGridMax = 1u << 17;

// Chunk of the first tile of every workgroup of a chunked launch of `grid`
// workgroups (workgroup b takes tiles [b * per, (b + 1) * per), per =
// ceil(tiles / grid), as ChunkSrc::setup): the last c with start[c] <= b * per,
// by binary search, one thread per workgroup, so that a render workgroup
// starts with one dependent load instead of a search.
__global__ __launch_bounds__(256) void k_chunk_wg(const uint64_t *__restrict__ start, uint32_t nchunks,
                                                  uint32_t grid, uint32_t *__restrict__ wgc) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= grid) return;
    const uint64_t ntiles = start[nchunks];
    const uint64_t per = (ntiles + grid - 1) / grid;
    const uint64_t t = (uint64_t)b * per;
    uint32_t lo = 0, hi = nchunks;
    if (t < ntiles) {
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (start[mid] <= t) lo = mid;
            else hi = mid;
        }
    }
    wgc[b] = lo;
}

struct ChunkLaunch {
    ChunkSrc src;
    View v;
    void *fb;
    int fam;
    uint32_t pass;  // HQ passes to run
    int sums;       // HQ sums layout (kTwoWord, kPacked, kRobust)
    Shape sh;
    uint32_t w, h;
    hipStream_t s;
};

template <int P>
struct ChunkL {
    template <int SUMS>
    static int color(const ChunkLaunch &C, const Tiles &tl, uint32_t hb, size_t sm) {
        const void *fn = (const void *)&k_hq_color<P, true, ChunkSrc, SUMS>;
        if (int rc = allow_lds(fn, sm)) return rc;
        const uint32_t *D = (const uint32_t *)C.fb;
        u64 *S = (u64 *)((char *)C.fb + hq_depth_bytes(C.w, C.h));
        hipLaunchKernelGGL((k_hq_color<P, true, ChunkSrc, SUMS>), dim3(C.sh.grid), dim3(C.sh.wg), sm,
                           C.s, nullptr, tl, C.v, D, S, hb, C.src);
        PCR_LAUNCHED();
        return PCR_OK;
    }
    static int run(const ChunkLaunch &C) {
        const uint32_t wg = C.sh.wg, T = wg * P, hb = lds_hbits(T, C.sh.slots);
        const Tiles tl{};
        if (C.fam == PCR_BASIC) {
            hipLaunchKernelGGL((k_basic<P, false, 0, ChunkSrc>), dim3(C.sh.grid), dim3(wg), 0, C.s, nullptr, tl, C.v,
                               (u64 *)C.fb, C.src);
            PCR_LAUNCHED();
            return PCR_OK;
        }
        if (C.fam == PCR_DEDUP) {
            const size_t sm = lds_bytes(hb, 8);
            if (sm > max_lds()) return fail(PCR_EINVAL, "tile of %u points needs %zu bytes of LDS", T, sm);
            const void *fn = (const void *)&k_dedup<u64, P, false, true, ChunkSrc>;
            if (int rc = allow_lds(fn, sm)) return rc;
            hipLaunchKernelGGL((k_dedup<u64, P, false, true, ChunkSrc>), dim3(C.sh.grid), dim3(wg), sm, C.s, nullptr,
                               tl, C.v, (u64 *)C.fb, hb, C.src);
            PCR_LAUNCHED();
            return PCR_OK;
        }
        if (C.pass & PCR_F_HQ_DEPTH) {
            const size_t sm = lds_bytes(hb, 4);
            if (sm > max_lds()) return fail(PCR_EINVAL, "tile of %u points needs %zu bytes of LDS", T, sm);
            const void *fn = (const void *)&k_dedup<uint32_t, P, false, true, ChunkSrc>;
            if (int rc = allow_lds(fn, sm)) return rc;
            hipLaunchKernelGGL((k_dedup<uint32_t, P, false, true, ChunkSrc>), dim3(C.sh.grid), dim3(wg), sm, C.s,
                               nullptr, tl, C.v, (uint32_t *)C.fb, hb, C.src);
            PCR_LAUNCHED();
        }
        if (C.pass & PCR_F_HQ_COLOR) {
            const size_t sm = lds_bytes(hb, 16);
            if (sm > max_lds()) return fail(PCR_EINVAL, "tile of %u points needs %zu bytes of LDS", T, sm);
            if (C.sums == kPacked) return color<kPacked>(C, tl, hb, sm);
            if (C.sums == kRobust) return color<kRobust>(C, tl, hb, sm);
            return color<kTwoWord>(C, tl, hb, sm);
        }
        return PCR_OK;
    }
};

template <int P>
struct GroupL {
    static int run(int pass, const u32x4 *pts, uint64_t n, const BatchView *views, const uint32_t *index,
                   const BatchGroup *groups, const uint32_t *ngroups, const Shape &sh, hipStream_t s) {
        const uint32_t T = sh.wg * P, hb = lds_hbits(T, sh.slots);
        const size_t sm0 = lds_bytes(hb, 8), sm1 = lds_bytes(hb, 16);
        if (sm1 > max_lds()) return fail(PCR_EINVAL, "tile of %u points needs %zu bytes of LDS", T, sm1);
        if (pass < 0) {
            int rc = allow_lds((const void *)&k_group_pass<P, 0>, sm0);
            return rc ? rc : allow_lds((const void *)&k_group_pass<P, 1>, sm1);
        }
        uint32_t grid;
        const Tiles tl = make_tiles(n, sh, grid);
        if (pass == 0)
            hipLaunchKernelGGL((k_group_pass<P, 0>), dim3(grid), dim3(sh.wg), sm0, s, pts, tl, views, index, groups,
                               ngroups, hb);
        else
            hipLaunchKernelGGL((k_group_pass<P, 1>), dim3(grid), dim3(sh.wg), sm1, s, pts, tl, views, index, groups,
                               ngroups, hb);
        PCR_LAUNCHED();
        return PCR_OK;
    }
};

template <int P>
struct ViewL {
    static int run(int pass, const u32x4 *pts, uint64_t n, const BatchView *views, const uint32_t *nviews,
                   uint32_t slot, const Shape &sh, hipStream_t s) {
        const uint32_t T = sh.wg * P, hb = lds_hbits(T, sh.slots);
        const size_t sm0 = lds_bytes(hb, 8), sm1 = lds_bytes(hb, 16);
        if (sm1 > max_lds()) return fail(PCR_EINVAL, "tile of %u points needs %zu bytes of LDS", T, sm1);
        if (pass < 0) {
            int rc = allow_lds((const void *)&k_view_pass<P, 0>, sm0);
            return rc ? rc : allow_lds((const void *)&k_view_pass<P, 1>, sm1);
        }
        uint32_t grid;
        const Tiles tl = make_tiles(n, sh, grid);
        if (pass == 0)
            hipLaunchKernelGGL((k_view_pass<P, 0>), dim3(grid), dim3(sh.wg), sm0, s, pts, tl, views, nviews, slot, hb);
        else
            hipLaunchKernelGGL((k_view_pass<P, 1>), dim3(grid), dim3(sh.wg), sm1, s, pts, tl, views, nviews, slot, hb);
        PCR_LAUNCHED();
        return PCR_OK;
    }
};

}  // namespace

int render_basic(const Launch &L) { return by_ppt<BasicL>(L.sh.ppt, L); }
int render_hq_depth(const Launch &L) { return by_ppt<DepthL>(L.sh.ppt, L); }
int render_hq_color(const Launch &L, uint32_t w, uint32_t h) { return by_ppt<ColorL>(L.sh.ppt, L, w, h); }
int launch_view_pass(int pass, const u32x4 *pts, uint64_t n, const BatchView *views, const uint32_t *nviews,
                     uint32_t slot, const Shape &sh, hipStream_t s) {
    return by_ppt<ViewL>(sh.ppt, pass, pts, n, views, nviews, slot, sh, s);
}
int launch_group_pass(int pass, const u32x4 *pts, uint64_t n, const BatchView *views, const uint32_t *index,
                      const BatchGroup *groups, const uint32_t *ngroups, const Shape &sh, hipStream_t s) {
    return by_ppt<GroupL>(sh.ppt, pass, pts, n, views, index, groups, ngroups, sh, s);
}

}  // namespace pcr

// ---------------------------------------------------------------------------
// C ABI: framebuffers, render, resolve
// ---------------------------------------------------------------------------
using namespace pcr;

extern "C" size_t pcr_fb_bytes(uint32_t w, uint32_t h, int variant) {
    if (check_image(w, h) != PCR_OK || check_variant(variant) != PCR_OK) return 0;
    uint64_t px = (uint64_t)w * h;
    if ((variant & 0xFF) == PCR_HQ) return hq_depth_bytes(w, h) + ((variant & PCR_F_HQ_ROBUST) ? 24 : 16) * px;
    return 8 * px;
}

extern "C" int pcr_fb_clear(void *fb, uint32_t w, uint32_t h, int variant, void *stream) {
    int rc = check_image(w, h);
    if (rc == PCR_OK) rc = check_variant(variant);
    if (rc != PCR_OK) return rc;
    if (!fb || ((uintptr_t)fb & 15)) return fail(PCR_EINVAL, "framebuffer must be a 16-byte aligned device pointer");
    hipStream_t s = (hipStream_t)stream;
    uint64_t px = (uint64_t)w * h;
    if ((variant & 0xFF) == PCR_HQ) {
        size_t db = hq_depth_bytes(w, h);
        rc = launch_fill(fb, db, 0xFFFFFFFFu, s);
        // the packed form uses one sum word per pixel, the robust form three
        const size_t sb = (variant & PCR_F_HQ_PACKED) ? 8 : (variant & PCR_F_HQ_ROBUST) ? 24 : 16;
        if (rc == PCR_OK) rc = launch_fill((char *)fb + db, sb * px, 0u, s);
        return rc;
    }
    return launch_fill(fb, 8 * px, 0xFFFFFFFFu, s);
}

extern "C" int pcr_render_ex(const pcr_point *pts, uint64_t n, const float mvp[16], uint32_t w,
                             uint32_t h, int variant, void *fb, const pcr_tune *tune, void *stream) {
    int rc = check_image(w, h);
    if (rc == PCR_OK) rc = check_variant(variant);
    if (rc != PCR_OK) return rc;
    if (!mvp) return fail(PCR_EINVAL, "mvp is NULL");
    if (!fb || ((uintptr_t)fb & 15)) return fail(PCR_EINVAL, "framebuffer must be a 16-byte aligned device pointer");
    if (n > 0 && (!pts || ((uintptr_t)pts & 15)))
        return fail(PCR_EINVAL, "points must be a 16-byte aligned device pointer");
    int fam = variant & 0xFF;
    uint32_t flags = (uint32_t)variant & ~0xFFu;
    Shape sh;
    // A basic render through the LDS kernel takes the deduplicating shape.
    rc = resolve_shape(tune, fam == PCR_BASIC && (flags & PCR_F_LDS) ? PCR_DEDUP : fam, sh);
    if (rc != PCR_OK) return rc;
    if (n == 0) return PCR_OK;
    Launch L{(const u32x4 *)pts, n, make_view(mvp, w, h), fb, sh, flags & ~PCR_F_PLAIN, (hipStream_t)stream};
    const bool chosen = (flags & kFlagMask) != 0;
    if (fam == PCR_BASIC) return render_basic(L);
    if (fam == PCR_DEDUP) {
        if (!chosen) L.flags |= PCR_F_LDS | PCR_F_REDUCE;
        return render_basic(L);
    }
    // PCR_HQ: depth pass, then colour pass.
    if (!chosen) L.flags |= PCR_F_LDS | PCR_F_REDUCE;
    uint32_t pass = flags & kHqPassMask;
    if (pass == 0) pass = kHqPassMask;
    if (pass & PCR_F_HQ_DEPTH) {
        rc = render_hq_depth(L);
        if (rc != PCR_OK) return rc;
    }
    if (pass & PCR_F_HQ_COLOR) rc = render_hq_color(L, w, h);
    return rc;
}

extern "C" int pcr_render(const pcr_point *pts, uint64_t n, const float mvp[16], uint32_t w, uint32_t h,
                          int variant, void *fb, void *stream) {
    return pcr_render_ex(pts, n, mvp, w, h, variant, fb, nullptr, stream);
}

// Chunk scratch: the chunks' tile offsets (nchunks + 1 words, padded to 256
// bytes), then the first chunk of each workgroup (kChunkGridMax words).
static size_t chunk_starts_bytes(uint32_t nchunks) { return ((size_t)8 * (nchunks + 1) + 255) / 256 * 256; }

extern "C" size_t pcr_chunks_scratch_bytes(uint32_t nchunks) {
    if (nchunks == 0 || nchunks > (1u << 24)) return 0;
    return chunk_starts_bytes(nchunks) + (size_t)4 * kChunkGridMax;
}

namespace pcr {
namespace {

// Renders a chunk table with `work` (device, pcr_chunks_scratch_bytes bytes)
// as its scratch.  Arguments other than `work` are checked here.
int render_chunks_into(const pcr_chunk *chunks, uint32_t nchunks, const float mvp[16], uint32_t w, uint32_t h,
                       int variant, void *fb, void *work, const pcr_tune *tune, hipStream_t s) {
    const int fam = variant & 0xFF;
    const uint32_t flags = (uint32_t)variant & ~0xFFu;
    Shape sh;
    int rc = resolve_shape(tune, fam, sh);
    if (rc != PCR_OK) return rc;
    if (sh.grid > kChunkGridMax) sh.grid = kChunkGridMax;
    uint64_t *start = (uint64_t *)work;
    uint32_t *wgc = (uint32_t *)((char *)work + chunk_starts_bytes(nchunks));
    // wg and ppt are powers of two (checked by resolve_shape), so is a tile.
    const uint32_t tshift = (uint32_t)__builtin_ctz(sh.wg * sh.ppt);
    hipLaunchKernelGGL(k_chunk_starts, dim3(1), dim3(kStartsThreads), 0, s, chunks, nchunks, tshift, start);
    hipLaunchKernelGGL(k_chunk_wg, dim3((sh.grid + 255) / 256), dim3(256), 0, s, start, nchunks, sh.grid, wgc);
    PCR_LAUNCHED();
    uint32_t pass = flags & kHqPassMask;
    if (pass == 0) pass = kHqPassMask;
    ChunkLaunch C{ChunkSrc{chunks, start, wgc, nchunks}, make_view(mvp, w, h), fb, fam, pass,
                  sums_layout(flags), sh, w, h, s};
    return by_ppt<ChunkL>(sh.ppt, C);
}

// Checks shared by both chunked entry points; PCR_OK with *noop set when
// there is nothing to render.
int check_chunks(const pcr_chunk *chunks, uint32_t nchunks, const float mvp[16], uint32_t w, uint32_t h,
                 int variant, const void *fb, const pcr_tune *tune, bool &noop) {
    noop = false;
    int rc = check_image(w, h);
    if (rc == PCR_OK) rc = check_variant(variant);
    if (rc != PCR_OK) return rc;
    const int fam = variant & 0xFF;
    const uint32_t flags = (uint32_t)variant & ~0xFFu;
    if ((flags & kFlagMask) != 0 || (fam != PCR_HQ && flags != 0))
        return fail(PCR_EUNSUPPORTED, "chunked rendering takes the default form of each variant (flags 0x%x)", flags);
    if (!mvp) return fail(PCR_EINVAL, "mvp is NULL");
    if (!fb || ((uintptr_t)fb & 15)) return fail(PCR_EINVAL, "framebuffer must be a 16-byte aligned device pointer");
    if (nchunks > (1u << 24)) return fail(PCR_EINVAL, "at most 2^24 chunks (got %u)", nchunks);
    Shape sh;
    rc = resolve_shape(tune, fam, sh);
    if (rc != PCR_OK) return rc;
    if (nchunks == 0) {
        noop = true;
        return PCR_OK;
    }
    if (!chunks || ((uintptr_t)chunks & 7)) return fail(PCR_EINVAL, "chunks must be an 8-byte aligned device pointer");
    return PCR_OK;
}

}  // namespace
}  // namespace pcr

extern "C" int pcr_render_chunks(const pcr_chunk *chunks, uint32_t nchunks, const float mvp[16], uint32_t w,
                                 uint32_t h, int variant, void *fb, void *work, size_t work_bytes,
                                 const pcr_tune *tune, void *stream) {
    bool noop;
    int rc = check_chunks(chunks, nchunks, mvp, w, h, variant, fb, tune, noop);
    if (rc != PCR_OK || noop) return rc;
    if (!work || ((uintptr_t)work & 15)) return fail(PCR_EINVAL, "scratch must be a 16-byte aligned device pointer");
    const size_t need = pcr_chunks_scratch_bytes(nchunks);
    if (work_bytes < need)
        return fail(PCR_ENOMEM, "scratch holds %zu bytes, %u chunks need %zu", work_bytes, nchunks, need);
    return render_chunks_into(chunks, nchunks, mvp, w, h, variant, fb, work, tune, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Chunked frames without caller scratch: the chunk offsets live in a
// library-owned device array (one copy per GPU, held until the process ends).
// ---------------------------------------------------------------------------
namespace pcr {
namespace {

// Sized as pcr_chunks_scratch_bytes(PCR_STATIC_CHUNKS_MAX), in 8-byte words.
constexpr size_t kStaticWords = ((size_t)8 * (PCR_STATIC_CHUNKS_MAX + 1) + 255) / 256 * 32 + kChunkGridMax / 2;
static __device__ __align__(256) uint64_t scratch[kStaticWords];

// Device address of `scratch` on the current device, looked up once per
// device (in host code the array's name is a host-side stand-in, never a
// device address).
int static_scratch(uint64_t **out) {
    static std::mutex mu;
    static uint64_t *addr[64] = {nullptr};
    int dev = 0;
    PCR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(PCR_EUNSUPPORTED, "device %d: at most 64 devices", dev);
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        PCR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PCR_EHIP, "hipGetSymbolAddress returned no address");
        addr[dev] = (uint64_t *)p;
    }
    *out = addr[dev];
    return PCR_OK;
}

}  // namespace
}  // namespace pcr

extern "C" int pcr_render_chunks_static(const pcr_chunk *chunks, uint32_t nchunks, const float mvp[16], uint32_t w,
                                        uint32_t h, int variant, void *fb, const pcr_tune *tune, void *stream) {
    bool noop;
    int rc = check_chunks(chunks, nchunks, mvp, w, h, variant, fb, tune, noop);
    if (rc != PCR_OK || noop) return rc;
    if (nchunks > PCR_STATIC_CHUNKS_MAX)
        return fail(PCR_EINVAL, "at most %u chunks without caller scratch (got %u)", (unsigned)PCR_STATIC_CHUNKS_MAX,
                    nchunks);
    uint64_t *work = nullptr;
    rc = static_scratch(&work);
    if (rc != PCR_OK) return rc;
    return render_chunks_into(chunks, nchunks, mvp, w, h, variant, fb, work, tune, (hipStream_t)stream);
}

extern "C" int pcr_resolve(const void *fb, uint32_t w, uint32_t h, int variant, uint32_t *rgba_out,
                           void *stream) {
    int rc = check_image(w, h);
    if (rc == PCR_OK) rc = check_variant(variant);
    if (rc != PCR_OK) return rc;
    if (!fb || ((uintptr_t)fb & 15)) return fail(PCR_EINVAL, "framebuffer must be a 16-byte aligned device pointer");
    if (!rgba_out || ((uintptr_t)rgba_out & 3)) return fail(PCR_EINVAL, "rgba_out must be a 4-byte aligned device pointer");
    uint64_t px = (uint64_t)w * h;
    uint64_t want = (px + 255) / 256;
    uint32_t grid = (uint32_t)(want > 16384 ? 16384 : want);
    hipStream_t s = (hipStream_t)stream;
    if ((variant & 0xFF) == PCR_HQ) {
        const u64 *S = (const u64 *)((const char *)fb + hq_depth_bytes(w, h));
        const int sums = sums_layout((uint32_t)variant);
        if (sums == kPacked)
            hipLaunchKernelGGL(k_resolve_hq<kPacked>, dim3(grid), dim3(256), 0, s, S, rgba_out, px);
        else if (sums == kRobust)
            hipLaunchKernelGGL(k_resolve_hq<kRobust>, dim3(grid), dim3(256), 0, s, S, rgba_out, px);
        else
            hipLaunchKernelGGL(k_resolve_hq<kTwoWord>, dim3(grid), dim3(256), 0, s, S, rgba_out, px);
    } else {
        hipLaunchKernelGGL(k_resolve_basic, dim3(grid), dim3(256), 0, s, (const u64 *)fb, rgba_out, px);
    }
    PCR_LAUNCHED();
    return PCR_OK;
}

extern "C" int pcr_resolve_raw(const void *fb, uint32_t w, uint32_t h, int variant, unsigned long long *raw_out,
                               void *stream) {
    int rc = check_image(w, h);
    if (rc == PCR_OK) rc = check_variant(variant);
    if (rc != PCR_OK) return rc;
    if (!fb || ((uintptr_t)fb & 15)) return fail(PCR_EINVAL, "framebuffer must be a 16-byte aligned device pointer");
    if (!raw_out || ((uintptr_t)raw_out & 7)) return fail(PCR_EINVAL, "raw_out must be an 8-byte aligned device pointer");
    const uint64_t px = (uint64_t)w * h;
    const uint64_t want = (px + 255) / 256;
    const uint32_t grid = (uint32_t)(want > 16384 ? 16384 : want);
    hipStream_t s = (hipStream_t)stream;
    u64 *out = (u64 *)raw_out;
    if ((variant & 0xFF) == PCR_HQ) {
        const uint32_t *D = (const uint32_t *)fb;
        const u64 *S = (const u64 *)((const char *)fb + hq_depth_bytes(w, h));
        const int sums = sums_layout((uint32_t)variant);
        if (sums == kPacked)
            hipLaunchKernelGGL(k_raw_hq<kPacked>, dim3(grid), dim3(256), 0, s, D, S, out, px);
        else if (sums == kRobust)
            hipLaunchKernelGGL(k_raw_hq<kRobust>, dim3(grid), dim3(256), 0, s, D, S, out, px);
        else
            hipLaunchKernelGGL(k_raw_hq<kTwoWord>, dim3(grid), dim3(256), 0, s, D, S, out, px);
    } else {
        hipLaunchKernelGGL(k_raw_basic, dim3(grid), dim3(256), 0, s, (const u64 *)fb, out, px);
    }
    PCR_LAUNCHED();
    return PCR_OK;
}

extern "C" int pcr_resolve_depth(const void *fb, uint32_t w, uint32_t h, int variant, int mode, float a,
                                 float b, float empty, uint32_t *rgba_out, float *depth_out, void *stream) {
    int rc = check_image(w, h);
    if (rc == PCR_OK) rc = check_variant(variant);
    if (rc != PCR_OK) return rc;
    if (mode != PCR_DEPTH_LINEAR && mode != PCR_DEPTH_HYPERBOLIC) return fail(PCR_EINVAL, "unknown depth mode %d", mode);
    if (!fb || ((uintptr_t)fb & 15)) return fail(PCR_EINVAL, "framebuffer must be a 16-byte aligned device pointer");
    if (!depth_out || ((uintptr_t)depth_out & 3))
        return fail(PCR_EINVAL, "depth_out must be a 4-byte aligned device pointer");
    if ((uintptr_t)rgba_out & 3) return fail(PCR_EINVAL, "rgba_out must be 4-byte aligned");
    uint64_t px = (uint64_t)w * h;
    uint64_t want = (px + 255) / 256;
    uint32_t grid = (uint32_t)(want > 16384 ? 16384 : want);
    hipStream_t s = (hipStream_t)stream;
    if ((variant & 0xFF) == PCR_HQ) {
        const uint32_t *D = (const uint32_t *)fb;
        const u64 *S = (const u64 *)((const char *)fb + hq_depth_bytes(w, h));
        const int sums = sums_layout((uint32_t)variant);
        if (sums == kPacked)
            hipLaunchKernelGGL(k_resolve_hq_depth<kPacked>, dim3(grid), dim3(256), 0, s, D, S, rgba_out, depth_out, px,
                               mode, a, b, empty);
        else if (sums == kRobust)
            hipLaunchKernelGGL(k_resolve_hq_depth<kRobust>, dim3(grid), dim3(256), 0, s, D, S, rgba_out, depth_out, px,
                               mode, a, b, empty);
        else
            hipLaunchKernelGGL(k_resolve_hq_depth<kTwoWord>, dim3(grid), dim3(256), 0, s, D, S, rgba_out, depth_out,
                               px, mode, a, b, empty);
    } else {
        hipLaunchKernelGGL(k_resolve_basic_depth, dim3(grid), dim3(256), 0, s, (const u64 *)fb, rgba_out,
                           depth_out, px, mode, a, b, empty);
    }
    PCR_LAUNCHED();
    return PCR_OK;
}
