// pcr_reorder.hip -- vertex orders of Sec. 4 / Sec. 5: Morton order (a 21-level
// octree traversal = 63-bit Morton code), shuffled Morton order (batches of
// the Morton sequence moved to random places) and the shuffled order.
//
// Pipeline: bounding box (one pass, ordered-integer atomics) -> Morton codes
// and indices -> stable LSD radix sort of (64-bit key, 32-bit index), 8-bit
// digits, eight passes -> gather.  The shuffle keys are SplitMix64 outputs.
// All work runs on the caller's stream in caller-provided scratch.
#include "pcr_internal.h"

namespace pcr {
namespace {

// 8192-key tiles of 256 threads x 32 keys: each digit's run of a tile
// averages 32 keys (256 bytes), so the scatter's stores are mostly whole
// 128-byte lines, and the 64 KiB staging buffer leaves room for two
// workgroups per CU.  Measured Morton reorders: 100M points 9.6 ms, 796M 81 ms,
// against 11.0 and 83 ms with 4096-key tiles; 16384-key tiles (one workgroup
// per CU) took 9.5 and 87 ms.
constexpr uint32_t kSortWg = 256;                   // threads per tile (at least one per digit)
constexpr uint32_t kSortIpt = 32;                   // keys per thread
constexpr uint32_t kSortTile = kSortWg * kSortIpt;  // keys per tile
constexpr uint32_t kWaves = kSortWg / 64;
static_assert(kSortWg >= 256 && kSortWg % 64 == 0, "one thread per 8-bit digit");
constexpr uint32_t kScanChunk = 4096;               // entries per scan block

// ---------------------------------------------------------------------------
// Bounding box: floats mapped to unsigned integers whose order is the float
// order, so min and max are integer atomics.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ord(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__global__ __launch_bounds__(64) void k_bbox_init(uint32_t *bb) {
    if (threadIdx.x < 3) bb[threadIdx.x] = 0xFFFFFFFFu;       // min
    else if (threadIdx.x < 6) bb[threadIdx.x] = 0u;           // max
}

// Each step a thread has kBboxLoads points in flight (consecutive threads on
// consecutive points in each of them).
constexpr uint32_t kBboxLoads = 8;

__device__ __forceinline__ void bbox_add(const u32x4 &p, uint32_t (&lo)[3], uint32_t (&hi)[3]) {
    const uint32_t k[3] = {ord(__uint_as_float(p.x)), ord(__uint_as_float(p.y)), ord(__uint_as_float(p.z))};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = k[a] < lo[a] ? k[a] : lo[a];
        hi[a] = k[a] > hi[a] ? k[a] : hi[a];
    }
}

__global__ __launch_bounds__(256) void k_bbox(const u32x4 *__restrict__ pts, uint64_t n, uint32_t *bb) {
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kBboxLoads - 1) * stride < n; i += kBboxLoads * stride) {
        u32x4 p[kBboxLoads];
#pragma unroll
        for (uint32_t r = 0; r < kBboxLoads; ++r) p[r] = load_point(pts + i + r * stride);
#pragma unroll
        for (uint32_t r = 0; r < kBboxLoads; ++r) bbox_add(p[r], lo, hi);
    }
    for (; i < n; i += stride) bbox_add(load_point(pts + i), lo, hi);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            uint32_t l = __shfl_xor(lo[a], o, 64), h = __shfl_xor(hi[a], o, 64);
            lo[a] = l < lo[a] ? l : lo[a];
            hi[a] = h > hi[a] ? h : hi[a];
        }
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            atomicMin(bb + a, lo[a]);
            atomicMax(bb + 3 + a, hi[a]);
        }
    }
}

// ---------------------------------------------------------------------------
// Morton codes: cell = min(trunc(((v - lo) / size) * 2^21), 2^21 - 1) over the
// cube of edge `size` (the longest extent), interleaved x, y, z from bit 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint32_t cell21(float v, float lo, float size) {
    if (size == 0.0f) return 0u;
    float t = ((v - lo) / size) * 2097152.0f;
    uint32_t q = (uint32_t)t;
    return q > 2097151u ? 2097151u : q;
}

__global__ __launch_bounds__(256) void k_morton(const u32x4 *__restrict__ pts, uint64_t n,
                                                const uint32_t *__restrict__ bb, uint64_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals) {
    float lo[3], size;
    {
        float l0 = unord(bb[0]), l1 = unord(bb[1]), l2 = unord(bb[2]);
        float sx = unord(bb[3]) - l0, sy = unord(bb[4]) - l1, sz = unord(bb[5]) - l2;
        size = sx;
        if (sy > size) size = sy;
        if (sz > size) size = sz;
        lo[0] = l0;
        lo[1] = l1;
        lo[2] = l2;
    }
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        u32x4 p = load_point(pts + i);
        uint32_t qx = cell21(__uint_as_float(p.x), lo[0], size);
        uint32_t qy = cell21(__uint_as_float(p.y), lo[1], size);
        uint32_t qz = cell21(__uint_as_float(p.z), lo[2], size);
        keys[i] = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
        vals[i] = (uint32_t)i;
    }
}

// SplitMix64 (Steele, Lea, Flood 2014): output k of the stream seeded with
// `seed` is the mix of seed + (k + 1) * golden gamma.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_random_keys(uint64_t n, uint64_t seed, uint64_t *__restrict__ keys,
                                                     uint32_t *__restrict__ vals) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        keys[i] = splitmix64(seed, i);
        vals[i] = (uint32_t)i;
    }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort pass.  A tile is kSortTile keys; wave w of the tile
// owns keys [w * 64 * kSortIpt, (w + 1) * 64 * kSortIpt) of it and visits them
// in kSortIpt rounds of 64 consecutive keys, so (wave, round, lane) order is
// the tile order.
// ---------------------------------------------------------------------------

// Lanes of the wavefront whose digit equals this lane's digit.
__device__ __forceinline__ uint64_t peers(uint32_t d, bool live) {
    uint64_t m = __ballot(live);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        uint64_t vb = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? vb : ~vb;
    }
    return m;
}

__device__ __forceinline__ uint64_t lanes_below() {
    uint32_t l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// hist[d * ntiles + tile] = number of keys of the tile with digit d.
__global__ __launch_bounds__(kSortWg) void k_sort_hist(const uint64_t *__restrict__ keys, uint64_t n,
                                                       uint32_t shift, uint32_t ntiles, uint32_t *__restrict__ hist) {
    __shared__ uint32_t cnt[256];
    if (threadIdx.x < 256) cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t wave = threadIdx.x / 64, lane = __lane_id();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile + wave * (64 * kSortIpt);
    uint64_t k[kSortIpt];  // all loads issued before the first use
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; ++r) {
        const uint64_t i = base + r * 64 + lane;
        k[r] = i < n ? keys[i] : 0ull;
    }
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; ++r) {
        const bool live = base + r * 64 + lane < n;
        const uint32_t d = (uint32_t)(k[r] >> shift) & 0xFFu;
        const uint64_t pm = peers(d, live);
        if (live && (pm & lanes_below()) == 0) atomicAdd(&cnt[d], (uint32_t)__popcll(pm));
    }
    __syncthreads();
    if (threadIdx.x < 256) hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of `a` (len entries) in chunks of kScanChunk; chunk totals go
// to `sums`.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t *sh, uint32_t &total) {
    // inclusive scan across the wave
    uint32_t lane = __lane_id(), wave = threadIdx.x / 64;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (uint32_t w = 0; w < blockDim.x / 64; ++w) {
        uint32_t s = sh[w];
        if (w < wave) off += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

__global__ __launch_bounds__(256) void k_scan_chunks(uint32_t *__restrict__ a, uint64_t len,
                                                     uint32_t *__restrict__ sums) {
    __shared__ uint32_t sh[4];
    constexpr uint32_t per = kScanChunk / 256;
    uint64_t base = (uint64_t)blockIdx.x * kScanChunk + threadIdx.x * per;
    uint32_t v[per], s = 0;
#pragma unroll
    for (uint32_t k = 0; k < per; ++k) {
        v[k] = base + k < len ? a[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = block_scan_excl(s, sh, total);
#pragma unroll
    for (uint32_t k = 0; k < per; ++k) {
        if (base + k < len) a[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Single-workgroup exclusive scan of the chunk totals (any length).
__global__ __launch_bounds__(256) void k_scan_sums(uint32_t *__restrict__ sums, uint32_t len) {
    __shared__ uint32_t sh[4];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < len; base += 256) {
        uint32_t i = base + threadIdx.x;
        uint32_t v = i < len ? sums[i] : 0u;
        uint32_t total;
        uint32_t e = block_scan_excl(v, sh, total);
        if (i < len) sums[i] = carry + e;
        carry += total;
    }
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t *__restrict__ a, uint64_t len,
                                                  const uint32_t *__restrict__ sums) {
    uint32_t add = sums[blockIdx.x];
    uint64_t base = (uint64_t)blockIdx.x * kScanChunk;
    for (uint32_t k = threadIdx.x; k < kScanChunk; k += 256)
        if (base + k < len) a[base + k] += add;
}

// Stable scatter of one pass.  off = scanned histogram (global positions).
// The tile is first put in digit order in LDS (stably: within a digit, tile
// order), then stored from there, so that consecutive lanes store consecutive
// addresses of one digit's run; keys and values go through the same LDS
// buffer one after the other.
__global__ __launch_bounds__(kSortWg) void k_sort_scatter(const uint64_t *__restrict__ kin,
                                                          const uint32_t *__restrict__ vin, uint64_t n,
                                                          uint32_t shift, uint32_t ntiles,
                                                          const uint32_t *__restrict__ off,
                                                          uint64_t *__restrict__ kout, uint32_t *__restrict__ vout) {
    __shared__ uint32_t wcnt[kWaves][256];
    __shared__ uint32_t goff[256];
    __shared__ uint32_t tstart[256];
    __shared__ uint32_t scan_sh[kWaves];
    __shared__ uint64_t stage[kSortTile];
    const uint32_t wave = threadIdx.x / 64, lane = __lane_id();
    if (threadIdx.x < 256) {
        for (uint32_t w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
        goff[threadIdx.x] = off[(uint64_t)threadIdx.x * ntiles + blockIdx.x];
    }
    __syncthreads();
    const uint64_t tile0 = (uint64_t)blockIdx.x * kSortTile;
    const uint64_t base = tile0 + wave * (64 * kSortIpt);
    uint64_t k[kSortIpt];
    uint32_t v[kSortIpt], rank[kSortIpt];
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; ++r) {
        uint64_t i = base + r * 64 + lane;
        bool live = i < n;
        k[r] = live ? kin[i] : 0ull;
        v[r] = live ? vin[i] : 0u;
    }
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; ++r) {
        uint64_t i = base + r * 64 + lane;
        bool live = i < n;
        uint32_t d = (uint32_t)(k[r] >> shift) & 0xFFu;
        uint64_t pm = peers(d, live);
        uint32_t before = (uint32_t)__popcll(pm & lanes_below());
        uint32_t prior = live ? wcnt[wave][d] : 0u;
        rank[r] = prior + before;
        // The lowest lane of each digit group publishes the new count after
        // every lane of the group has read the old one: LDS operations of one
        // wave complete in order, and the wave barriers keep the compiler
        // from moving the read and the write across each other or across
        // rounds.
        __builtin_amdgcn_wave_barrier();
        if (live && before == 0) wcnt[wave][d] = prior + (uint32_t)__popcll(pm);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // Thread t = digit t: prefix of its count over the waves (wave order is
    // tile order), then the start of its run in the digit-ordered tile.
    uint32_t run = 0;
    if (threadIdx.x < 256) {
        for (uint32_t w = 0; w < kWaves; ++w) {
            uint32_t c = wcnt[w][threadIdx.x];
            wcnt[w][threadIdx.x] = run;
            run += c;
        }
    }
    uint32_t total;
    const uint32_t ts = block_scan_excl(run, scan_sh, total);
    if (threadIdx.x < 256) tstart[threadIdx.x] = ts;
    __syncthreads();
    const uint32_t cnt = (uint32_t)(n - tile0 < kSortTile ? n - tile0 : kSortTile);
    uint32_t lp[kSortIpt];
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; ++r) {
        uint32_t d = (uint32_t)(k[r] >> shift) & 0xFFu;
        lp[r] = tstart[d] + wcnt[wave][d] + rank[r];
        if (base + r * 64 + lane < n) stage[lp[r]] = k[r];
    }
    __syncthreads();
    uint32_t pos[kSortIpt];
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; ++r) {
        uint32_t j = threadIdx.x + r * kSortWg;
        pos[r] = 0xFFFFFFFFu;
        if (j < cnt) {
            uint64_t key = stage[j];
            uint32_t d = (uint32_t)(key >> shift) & 0xFFu;
            uint64_t p = (uint64_t)goff[d] + (j - tstart[d]);
            if (p < n) {  // always true for a consistent histogram
                pos[r] = (uint32_t)p;
                kout[p] = key;
            }
        }
    }
    __syncthreads();
    uint32_t *vstage = (uint32_t *)stage;
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; ++r)
        if (base + r * 64 + lane < n) vstage[lp[r]] = v[r];
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; ++r) {
        uint32_t j = threadIdx.x + r * kSortWg;
        if (pos[r] != 0xFFFFFFFFu) vout[pos[r]] = vstage[j];
    }
}

// ---------------------------------------------------------------------------
// Gathers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather(const u32x4 *__restrict__ in, const uint32_t *__restrict__ perm,
                                                uint64_t n, u32x4 *__restrict__ out, uint32_t *__restrict__ perm_out) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        uint32_t s = perm[j];
        if (s >= n) continue;  // never taken for a permutation
        out[j] = in[s];
        if (perm_out) perm_out[j] = s;
    }
}

// Rank (position in the shuffled batch order) of every batch: rank[order[r]] = r.
__global__ __launch_bounds__(256) void k_batch_rank(const uint32_t *__restrict__ order, uint64_t nb,
                                                    uint32_t *__restrict__ rank) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nb; r += stride) {
        const uint32_t b = order[r];
        if (b < nb) rank[b] = (uint32_t)r;  // always taken for a permutation
    }
}

// Batch b (Morton positions [b * batch, b * batch + len)) goes to rank r =
// rank[b]: output position start(r) + k, where batches before the partial
// last one start at r * batch and those after it `batch - len_last` earlier.
// Workgroups take batches in Morton order, so consecutive workgroups read
// neighbouring points of the source (its pages stay in the TLB) and write
// whole batches to scattered places.
__global__ __launch_bounds__(256) void k_gather_batches(const u32x4 *__restrict__ in,
                                                        const uint32_t *__restrict__ morton,
                                                        const uint32_t *__restrict__ rank, uint64_t n,
                                                        uint64_t nb, uint32_t batch,
                                                        u32x4 *__restrict__ out, uint32_t *__restrict__ perm_out) {
    const uint64_t len_last = n - (nb - 1) * batch;
    const uint64_t rl = rank[nb - 1];
    for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const uint64_t r = rank[b];
        const uint64_t len = b == nb - 1 ? len_last : batch;
        const uint64_t start = r * batch - (r > rl ? batch - len_last : 0);
        for (uint32_t k = threadIdx.x; k < len; k += blockDim.x) {
            const uint32_t src = morton[b * batch + k];
            if (start + k >= n || src >= n) continue;  // never taken for permutations
            out[start + k] = in[src];
            if (perm_out) perm_out[start + k] = src;
        }
    }
}

// ---------------------------------------------------------------------------
// Host
// ---------------------------------------------------------------------------
inline size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

struct SortBufs {
    uint64_t *k0, *k1;
    uint32_t *v0, *v1;
    uint32_t *hist, *sums;
};

size_t sort_bytes(uint64_t n) {
    uint64_t ntiles = (n + kSortTile - 1) / kSortTile;
    uint64_t hlen = 256 * ntiles;
    uint64_t nchunks = (hlen + kScanChunk - 1) / kScanChunk;
    return 2 * a256(8 * n) + 2 * a256(4 * n) + a256(4 * hlen) + a256(4 * (nchunks + 1));
}

char *carve_sort(char *p, uint64_t n, SortBufs &sb) {
    uint64_t ntiles = (n + kSortTile - 1) / kSortTile;
    uint64_t hlen = 256 * ntiles;
    uint64_t nchunks = (hlen + kScanChunk - 1) / kScanChunk;
    sb.k0 = (uint64_t *)p; p += a256(8 * n);
    sb.k1 = (uint64_t *)p; p += a256(8 * n);
    sb.v0 = (uint32_t *)p; p += a256(4 * n);
    sb.v1 = (uint32_t *)p; p += a256(4 * n);
    sb.hist = (uint32_t *)p; p += a256(4 * hlen);
    sb.sums = (uint32_t *)p; p += a256(4 * (nchunks + 1));
    return p;
}

uint32_t grid_for(uint64_t n, uint32_t cap = 65536) {
    uint64_t g = (n + 255) / 256;
    return (uint32_t)(g < 1 ? 1 : (g > cap ? cap : g));
}

// Sorts (sb.k0, sb.v0) by the low `bits` bits of the key, stably; the result
// ends in (sb.k0, sb.v0) (an even number of passes).
int radix_sort(SortBufs &sb, uint64_t n, uint32_t bits, hipStream_t s) {
    uint32_t ntiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
    uint64_t hlen = 256ull * ntiles;
    uint32_t nchunks = (uint32_t)((hlen + kScanChunk - 1) / kScanChunk);
    uint32_t passes = (bits + 7) / 8;
    passes += passes & 1u;
    uint64_t *ki = sb.k0, *ko = sb.k1;
    uint32_t *vi = sb.v0, *vo = sb.v1;
    for (uint32_t p = 0; p < passes; ++p) {
        uint32_t shift = 8 * p;
        hipLaunchKernelGGL(k_sort_hist, dim3(ntiles), dim3(kSortWg), 0, s, ki, n, shift, ntiles, sb.hist);
        hipLaunchKernelGGL(k_scan_chunks, dim3(nchunks), dim3(256), 0, s, sb.hist, hlen, sb.sums);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, sb.sums, nchunks);
        hipLaunchKernelGGL(k_scan_add, dim3(nchunks), dim3(256), 0, s, sb.hist, hlen, sb.sums);
        hipLaunchKernelGGL(k_sort_scatter, dim3(ntiles), dim3(kSortWg), 0, s, ki, vi, n, shift, ntiles, sb.hist,
                           ko, vo);
        PCR_LAUNCHED();
        uint64_t *tk = ki; ki = ko; ko = tk;
        uint32_t *tv = vi; vi = vo; vo = tv;
    }
    return PCR_OK;
}

size_t reorder_bytes(uint64_t n, int order, uint32_t batch) {
    if (n == 0) return 256;
    size_t b = sort_bytes(n) + 256;  // + bbox / rank word
    if (order == PCR_ORDER_MORTON_SHUFFLE) b += sort_bytes((n + batch - 1) / batch);
    return b;
}

}  // namespace
}  // namespace pcr

using namespace pcr;

extern "C" size_t pcr_reorder_scratch_bytes(uint64_t n, int order, uint32_t batch) {
    if (order < 0 || order > 2 || n >= (1ull << 32)) return 0;
    if (order == PCR_ORDER_MORTON_SHUFFLE && batch == 0) return 0;
    return reorder_bytes(n, order, batch);
}

extern "C" int pcr_reorder(const pcr_point *in, pcr_point *out, uint32_t *perm_out, uint64_t n, int order,
                           uint32_t batch, uint64_t seed, void *scratch, size_t scratch_bytes, void *stream) {
    if (order < 0 || order > 2) return fail(PCR_EINVAL, "unknown order %d", order);
    if (order == PCR_ORDER_MORTON_SHUFFLE && batch == 0) return fail(PCR_EINVAL, "batch size 0");
    if (n >= (1ull << 32)) return fail(PCR_EINVAL, "reorder needs n < 2^32 (got %llu)", (unsigned long long)n);
    if (n == 0) return PCR_OK;
    if (!in || !out || ((uintptr_t)in & 15) || ((uintptr_t)out & 15))
        return fail(PCR_EINVAL, "points must be 16-byte aligned device pointers");
    if ((uintptr_t)perm_out & 3) return fail(PCR_EINVAL, "perm_out must be 4-byte aligned");
    const char *ib = (const char *)in, *ob = (const char *)out;
    if (ib < ob + 16 * n && ob < ib + 16 * n) return fail(PCR_EINVAL, "in and out overlap");
    size_t need = reorder_bytes(n, order, batch);
    if (!scratch || ((uintptr_t)scratch & 255)) return fail(PCR_EINVAL, "scratch must be a 256-byte aligned device pointer");
    if (scratch_bytes < need) return fail(PCR_ENOMEM, "scratch has %zu bytes, %zu needed", scratch_bytes, need);

    hipStream_t s = (hipStream_t)stream;
    const u32x4 *pin = (const u32x4 *)in;
    u32x4 *pout = (u32x4 *)out;
    char *p = (char *)scratch;
    uint32_t *word = (uint32_t *)p;  // bbox[6]
    p += 256;
    SortBufs sb;
    p = carve_sort(p, n, sb);
    uint32_t g = grid_for(n);

    if (order == PCR_ORDER_SHUFFLE) {
        hipLaunchKernelGGL(k_random_keys, dim3(g), dim3(256), 0, s, n, seed, sb.k0, sb.v0);
        PCR_LAUNCHED();
        int rc = radix_sort(sb, n, 64, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_gather, dim3(g), dim3(256), 0, s, pin, sb.v0, n, pout, perm_out);
        PCR_LAUNCHED();
        return PCR_OK;
    }
    uint32_t gb = grid_for(n, 2048);
    hipLaunchKernelGGL(k_bbox_init, dim3(1), dim3(64), 0, s, word);
    hipLaunchKernelGGL(k_bbox, dim3(gb), dim3(256), 0, s, pin, n, word);
    hipLaunchKernelGGL(k_morton, dim3(g), dim3(256), 0, s, pin, n, word, sb.k0, sb.v0);
    PCR_LAUNCHED();
    int rc = radix_sort(sb, n, 63, s);
    if (rc) return rc;
    if (order == PCR_ORDER_MORTON) {
        hipLaunchKernelGGL(k_gather, dim3(g), dim3(256), 0, s, pin, sb.v0, n, pout, perm_out);
        PCR_LAUNCHED();
        return PCR_OK;
    }
    // Shuffled Morton (Sec. 4): the Morton permutation stays in sb.v0; the
    // batch indices are sorted by their SplitMix64 keys in a second sort whose
    // buffers follow sb in the scratch; the batches are emitted in that order.
    uint64_t nb = (n + batch - 1) / batch;
    SortBufs bs;
    carve_sort(p, nb, bs);
    uint32_t gn = grid_for(nb);
    hipLaunchKernelGGL(k_random_keys, dim3(gn), dim3(256), 0, s, nb, seed, bs.k0, bs.v0);
    PCR_LAUNCHED();
    rc = radix_sort(bs, nb, 64, s);
    if (rc) return rc;
    // bs.v1 is free after the sort (an even number of passes ends in bs.v0)
    hipLaunchKernelGGL(k_batch_rank, dim3(gn), dim3(256), 0, s, bs.v0, nb, bs.v1);
    const uint32_t gwg = (uint32_t)(nb < 65536 ? nb : 65536);
    hipLaunchKernelGGL(k_gather_batches, dim3(gwg), dim3(256), 0, s, pin, sb.v0, bs.v1, n, nb, batch, pout,
                       perm_out);
    PCR_LAUNCHED();
    return PCR_OK;
}
