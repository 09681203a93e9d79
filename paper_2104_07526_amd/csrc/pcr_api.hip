// pcr_api.hip -- host-side plumbing of the C ABI: argument checks, launch
// shapes, error messages.
#include <mutex>
#include <string>

#include "pcr_internal.h"

namespace pcr {

namespace {
thread_local std::string g_error;
}

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int check_image(uint32_t w, uint32_t h) {
    if (w == 0 || h == 0) return fail(PCR_EINVAL, "image size %ux%u is empty", w, h);
    if (w >= (1u << 24) || h >= (1u << 24))
        return fail(PCR_EINVAL, "image size %ux%u: each side must be below 2^24", w, h);
    if ((uint64_t)w * h >= (1ull << 32))
        return fail(PCR_EINVAL, "image size %ux%u: at most 2^32 - 1 pixels", w, h);
    return PCR_OK;
}

int check_variant(int variant) {
    if (variant < 0) return fail(PCR_EINVAL, "unknown variant %d", variant);
    int fam = variant & 0xFF;
    uint32_t flags = (uint32_t)variant & ~0xFFu;
    if (fam != PCR_BASIC && fam != PCR_DEDUP && fam != PCR_HQ)
        return fail(PCR_EINVAL, "unknown variant %d", fam);
    uint32_t allowed = fam == PCR_HQ ? (kFlagMask | kHqPassMask | PCR_F_HQ_PACKED | PCR_F_HQ_ROBUST) : kFlagMask;
    if ((flags & PCR_F_PLAIN) && (flags & (PCR_F_EARLYZ | kReduceMask | PCR_F_LDS)))
        return fail(PCR_EINVAL, "PCR_F_PLAIN excludes the other path flags");
    if ((flags & PCR_F_REDUCE_PAIR) && (flags & PCR_F_LDS))
        return fail(PCR_EINVAL, "PCR_F_REDUCE_PAIR applies to the paths without PCR_F_LDS");
    if ((flags & PCR_F_HQ_PACKED) && (flags & PCR_F_HQ_ROBUST))
        return fail(PCR_EINVAL, "PCR_F_HQ_PACKED and PCR_F_HQ_ROBUST are two layouts of the sums: pick one");
    if (flags & ~allowed) return fail(PCR_EINVAL, "flag bits 0x%x do not apply to variant %d", flags & ~allowed, fam);
    return PCR_OK;
}

size_t hq_depth_bytes(uint32_t w, uint32_t h) {
    size_t b = 4ull * w * h;
    return (b + 255) & ~(size_t)255;
}

static bool pow2_in(uint32_t v, uint32_t lo, uint32_t hi) {
    return v >= lo && v <= hi && (v & (v - 1)) == 0;
}

int resolve_shape(const pcr_tune *tune, int family, Shape &s) {
    // Defaults (measured on MI355X), all with single-wavefront workgroups
    // stepping over the tiles in their natural order, which beat one
    // workgroup per tile in XCD-contiguous order on every measured order:
    // the basic kernel (family PCR_BASIC) runs of 4 points per lane and 64
    // workgroups per CU; the deduplicating and HQ kernels 256 LDS slots
    // (their barriers never wait for another wavefront), 512 workgroups per
    // CU and tiles of 256 points (dedup) or 512 points (HQ).
    const bool basic = family == PCR_BASIC;
    s.wg = 64;
    s.ppt = family == PCR_HQ ? 8 : 4;
    s.grid = (basic ? 64u : 512u) * (uint32_t)device_cus();
    s.group = 0;
    s.slots = 0;
    s.run = 0;
    if (tune) {
        if (tune->wg) s.wg = tune->wg;
        if (tune->ppt) s.ppt = tune->ppt;
        if (tune->grid) s.grid = tune->grid;
        s.group = tune->group;
        s.slots = tune->slots;
        s.run = tune->run;
    }
    if (s.run > 4096 || s.run % s.ppt) return fail(PCR_EINVAL, "run %u is not a multiple of ppt %u up to 4096", s.run, s.ppt);
    if (s.slots > 32768) return fail(PCR_EINVAL, "slots %u above 32768", s.slots);
    if (!pow2_in(s.wg, 64, 1024)) return fail(PCR_EINVAL, "workgroup size %u is not a power of two in [64, 1024]", s.wg);
    if (!pow2_in(s.ppt, 1, 16)) return fail(PCR_EINVAL, "points per thread %u is not 1, 2, 4, 8 or 16", s.ppt);
    return PCR_OK;
}

int device_cus() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> g(mu);
    if (cache[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cache[dev] = v;
    }
    return cache[dev];
}

size_t max_lds() {
    static std::mutex mu;
    static size_t cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
    std::lock_guard<std::mutex> g(mu);
    if (cache[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        cache[dev] = (size_t)v;
    }
    return cache[dev];
}

int allow_lds(const void *kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return PCR_OK;
    hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return fail(PCR_EHIP, "hipFuncSetAttribute(%zu bytes of LDS): %s", bytes, hipGetErrorString(e));
    return PCR_OK;
}

}  // namespace pcr

extern "C" const char *pcr_last_error(void) { return pcr::g_error.c_str(); }

extern "C" const char *pcr_version(void) { return "pcr 0.1 (gfx950)"; }

namespace pcr {
// For the floats w with bit patterns in [lo, lo + count): counts those whose
// projection reciprocal differs from the device division 1.0f / w, and adds
// the bit patterns of the reciprocals into a digest (their sum modulo 2^64 and
// their exclusive or), which the caller compares with the same digest of the
// IEEE quotients computed on the host.
__global__ __launch_bounds__(256) void k_check_recip(uint32_t lo, uint64_t count, unsigned long long *res) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long nbad = 0, sum = 0, x = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        float w = __uint_as_float(lo + (uint32_t)i);
        const uint32_t q = __float_as_uint(recip_rn(w));
        nbad += q != __float_as_uint(1.0f / w);
        sum += q;
        x ^= q;
    }
    if (nbad) atomicAdd(res, nbad);
    atomicAdd(res + 1, sum);
    atomicXor(res + 2, x);
}
}  // namespace pcr

extern "C" int pcr_check_reciprocal(uint32_t first_bits, uint32_t last_bits, unsigned long long *result,
                                    void *stream) {
    if (!result || ((uintptr_t)result & 7) || last_bits < first_bits)
        return pcr::fail(PCR_EINVAL, "bad reciprocal check arguments");
    uint64_t count = (uint64_t)last_bits - first_bits + 1;
    hipLaunchKernelGGL(pcr::k_check_recip, dim3(8192), dim3(256), 0, (hipStream_t)stream, first_bits, count,
                       result);
    PCR_LAUNCHED();
    return PCR_OK;
}
