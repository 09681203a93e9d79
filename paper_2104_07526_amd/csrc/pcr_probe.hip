// pcr_probe.hip -- measurement helpers: the number of points a view keeps
// (one global atomic each in the basic renderer of Sec. 3.1), a
// microbenchmark of device-wide 64-bit atomic minimum throughput, the rate
// that bounds that renderer on this chip, and a read-only stream of a point
// buffer, the practical floor of the deduplicating renderers' point stream.
#include "pcr_internal.h"

namespace pcr {

// Points of [0, n) that land in the image (not culled by the projection).
__global__ __launch_bounds__(256) void k_count_visible(const u32x4 *__restrict__ pts, uint64_t n, View v,
                                                       unsigned long long *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long cnt = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const u32x4 p = load_point(pts + i);
        uint32_t dbits;
        cnt += project(v, __uint_as_float(p.x), __uint_as_float(p.y), __uint_as_float(p.z), dbits) != kEmptyPid;
    }
    // one atomic per wavefront (a lane counts at most n / stride points, far below 2^32)
    uint32_t c = (uint32_t)cnt;
    for (int d = 32; d >= 1; d >>= 1) c += (uint32_t)__shfl_xor((int)c, d, 64);
    if (__lane_id() == 0 && c) atomicAdd(out, (unsigned long long)c);
}

// 32-bit integer mix (xorshift-multiply finaliser); addresses for the probe.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

// Uniform index in [0, range) from a 32-bit hash.
__device__ __forceinline__ uint32_t below(uint32_t h, uint32_t range) { return __umulhi(h, range); }

// Each lane issues `iters` 64-bit atomic minimums on buf[0, words) (words a
// multiple of 64, below 2^32):
//   PCR_PROBE_RANDOM      every lane its own random word
//   PCR_PROBE_LINE        8 lanes on the 8 words of one random 64-byte line
//   PCR_PROBE_ADDRESS     all 64 lanes of a wavefront on one random word
//   PCR_PROBE_CONTIGUOUS  a wavefront on 64 consecutive words (512 bytes)
// RET: the returning form (the old values are folded into a word written
// only if an impossible value turns up, so the atomics must complete).
template <int PATTERN, bool RET>
__global__ __launch_bounds__(256) void k_probe_atomics(u64 *__restrict__ buf, uint32_t words, uint32_t iters,
                                                       uint32_t seed, u64 *__restrict__ sink) {
    const uint32_t lane = __lane_id();
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t wave = gid >> 6;
    u64 acc = 0;
#pragma unroll 1
    for (uint32_t it = 0; it < iters; ++it) {
        const uint32_t hl = mix32(gid * 0x9E3779B9u + it * 0x85EBCA6Bu + seed);
        const uint32_t hw = mix32(wave * 0xC2B2AE35u + it * 0x27D4EB2Fu + seed);
        uint32_t idx;
        if constexpr (PATTERN == PCR_PROBE_RANDOM) {
            idx = below(hl, words);
        } else if constexpr (PATTERN == PCR_PROBE_LINE) {
            const uint32_t hg = mix32(hw ^ ((lane >> 3) * 0x165667B1u));
            idx = below(hg, words >> 3) * 8u + (lane & 7u);
        } else if constexpr (PATTERN == PCR_PROBE_ADDRESS) {
            idx = below(hw, words);
        } else {
            idx = below(hw, words >> 6) * 64u + lane;
        }
        const u64 val = ((u64)hl << 32) | gid;
        if constexpr (RET)
            acc ^= __hip_atomic_fetch_min(buf + idx, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            gmin_u64(buf + idx, val);
    }
    if (RET && acc == 0x5A5A5A5A5A5A5A5Aull) sink[0] = acc;
}

// Read-only stream of n 16-byte records in the render kernels' access
// pattern (workgroup tiles of U * 256 records, record j * 256 + thread of a
// tile in row j, non-temporal loads, grid-stride over the tiles): the rate at
// which this chip delivers a point buffer with no other work.  The records are
// folded into one word per lane, stored only if it takes one fixed value (the
// stored word means nothing), so every load must complete.
template <int U>
__global__ __launch_bounds__(256) void k_probe_read(const u32x4 *__restrict__ p, uint64_t n,
                                                    uint32_t *__restrict__ sink) {
    const uint64_t ntiles = (n + U * 256ull - 1) / (U * 256ull);
    uint32_t acc = 0;
#pragma unroll 1
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        u32x4 v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = t * (U * 256ull) + j * 256u + threadIdx.x;
            v[j] = load_point(p + (i < n ? i : n - 1));
        }
#pragma unroll
        for (int j = 0; j < U; ++j) acc ^= (v[j].x ^ v[j].y) ^ (v[j].z ^ v[j].w);
    }
    if (acc == 0x5A5A5A5Au) sink[0] = acc;
}

}  // namespace pcr

using namespace pcr;

extern "C" int pcr_count_visible(const pcr_point *pts, uint64_t n, const float mvp[16], uint32_t w, uint32_t h,
                                 unsigned long long *count, void *stream) {
    int rc = check_image(w, h);
    if (rc != PCR_OK) return rc;
    if (!mvp) return fail(PCR_EINVAL, "mvp is NULL");
    if (!count || ((uintptr_t)count & 7)) return fail(PCR_EINVAL, "count must be an 8-byte aligned device pointer");
    if (n > 0 && (!pts || ((uintptr_t)pts & 15)))
        return fail(PCR_EINVAL, "points must be a 16-byte aligned device pointer");
    if (n == 0) return PCR_OK;
    const uint64_t want = (n + 255) / 256;
    const uint32_t grid = (uint32_t)(want > 65536 ? 65536 : want);
    hipLaunchKernelGGL(k_count_visible, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const u32x4 *)pts, n,
                       make_view(mvp, w, h), count);
    PCR_LAUNCHED();
    return PCR_OK;
}

extern "C" int pcr_probe_atomics(unsigned long long *buf, uint64_t words, int pattern, int returning,
                                 uint32_t workgroups, uint32_t iters, uint32_t seed, unsigned long long *sink,
                                 void *stream) {
    if (!buf || ((uintptr_t)buf & 63)) return fail(PCR_EINVAL, "buf must be a 64-byte aligned device pointer");
    if (words < 64 || words >= (1ull << 32) || (words & 63))
        return fail(PCR_EINVAL, "words must be a multiple of 64 in [64, 2^32) (got %llu)", (unsigned long long)words);
    if (workgroups == 0 || workgroups > (1u << 22)) return fail(PCR_EINVAL, "workgroups must be in [1, 2^22]");
    if (returning && (!sink || ((uintptr_t)sink & 7)))
        return fail(PCR_EINVAL, "the returning form needs an 8-byte aligned sink word");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t wd = (uint32_t)words;
    u64 *b = (u64 *)buf, *k = (u64 *)sink;
#define PCR_PR(P)                                                                                          \
    do {                                                                                                   \
        if (returning)                                                                                     \
            hipLaunchKernelGGL((k_probe_atomics<P, true>), dim3(workgroups), dim3(256), 0, s, b, wd, iters, seed, k); \
        else                                                                                               \
            hipLaunchKernelGGL((k_probe_atomics<P, false>), dim3(workgroups), dim3(256), 0, s, b, wd, iters, seed, k); \
    } while (0)
    switch (pattern) {
        case PCR_PROBE_RANDOM: PCR_PR(PCR_PROBE_RANDOM); break;
        case PCR_PROBE_LINE: PCR_PR(PCR_PROBE_LINE); break;
        case PCR_PROBE_ADDRESS: PCR_PR(PCR_PROBE_ADDRESS); break;
        case PCR_PROBE_CONTIGUOUS: PCR_PR(PCR_PROBE_CONTIGUOUS); break;
        default: return fail(PCR_EINVAL, "unknown probe pattern %d", pattern);
    }
#undef PCR_PR
    PCR_LAUNCHED();
    return PCR_OK;
}

extern "C" int pcr_probe_read(const void *buf, uint64_t n16, uint32_t per_thread, uint32_t workgroups,
                              uint32_t *sink, void *stream) {
    if (n16 == 0) return PCR_OK;
    if (!buf || ((uintptr_t)buf & 15)) return fail(PCR_EINVAL, "buf must be a 16-byte aligned device pointer");
    if (per_thread != 4 && per_thread != 8) return fail(PCR_EINVAL, "per_thread must be 4 or 8 (got %u)", per_thread);
    if (workgroups == 0 || workgroups > (1u << 22)) return fail(PCR_EINVAL, "workgroups must be in [1, 2^22]");
    if (!sink || ((uintptr_t)sink & 3)) return fail(PCR_EINVAL, "sink must be a 4-byte aligned device pointer");
    hipStream_t s = (hipStream_t)stream;
    const u32x4 *p = (const u32x4 *)buf;
    if (per_thread == 4)
        hipLaunchKernelGGL(k_probe_read<4>, dim3(workgroups), dim3(256), 0, s, p, n16, sink);
    else
        hipLaunchKernelGGL(k_probe_read<8>, dim3(workgroups), dim3(256), 0, s, p, n16, sink);
    PCR_LAUNCHED();
    return PCR_OK;
}
