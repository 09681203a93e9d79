// pcr_internal.h -- device helpers and host plumbing shared by the libpcr
// translation units (GPU library only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "pcr.h"

// Every float operation of the projection is one IEEE binary32 operation
// (no contraction into fused multiply-add), matching the fixed operation
// order documented in pcr.h.
#pragma clang fp contract(off)

namespace pcr {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned long long u64;

constexpr u64 kEmptyKey = ~0ull;
constexpr uint32_t kEmptyPid = 0xFFFFFFFFu;
constexpr uint32_t kReduceMask = PCR_F_REDUCE | PCR_F_REDUCE_WAVE | PCR_F_REDUCE_PAIR;
constexpr uint32_t kFlagMask = PCR_F_EARLYZ | kReduceMask | PCR_F_LDS | PCR_F_PLAIN;

// Wavefront reductions of a flag set: bit 0 leader groups, bit 1 neighbouring
// pairs (PCR_F_REDUCE = both).
inline int reduce_mode(uint32_t flags) {
    return ((flags & (PCR_F_REDUCE | PCR_F_REDUCE_WAVE)) ? 1 : 0) | ((flags & (PCR_F_REDUCE | PCR_F_REDUCE_PAIR)) ? 2 : 0);
}
constexpr uint32_t kHqPassMask = PCR_F_HQ_DEPTH | PCR_F_HQ_COLOR;

// Camera and viewport of one view, passed by value as a kernel argument (the
// matrix is read through scalar loads and used as SGPR operands).
struct View {
    float m[16];
    uint32_t W, H;
    float fW, fH, hw, hh;
};

inline View make_view(const float *mvp, uint32_t W, uint32_t H) {
    View v;
    for (int i = 0; i < 16; ++i) v.m[i] = mvp[i];
    v.W = W;
    v.H = H;
    v.fW = (float)W;
    v.fH = (float)H;
    v.hw = 0.5f * v.fW;
    v.hh = 0.5f * v.fH;
    return v;
}

// Projection (Sec. 3.1): clip = M * (x, y, z, 1); cull unless w > 0; one
// correctly rounded reciprocal; half-open viewport test in float; truncation.
// Split in two so that a whole wavefront of surely culled points can skip the
// division: clip() computes the clip coordinates, finish() the pixel index
// (kEmptyPid when culled) and the depth bits (the linear w) from them.
struct Clip {
    float cx, cy, cw;
};

__device__ __forceinline__ Clip clip(const View &v, float x, float y, float z) {
    Clip c;
    c.cx = ((v.m[0] * x + v.m[1] * y) + v.m[2] * z) + v.m[3];
    c.cy = ((v.m[4] * x + v.m[5] * y) + v.m[6] * z) + v.m[7];
    c.cw = ((v.m[12] * x + v.m[13] * y) + v.m[14] * z) + v.m[15];
    return c;
}

// Lanes of the wavefront whose points finish() culls for certain: behind the
// camera, or more than 0.1% outside the view cone in clip space (the rounding
// of the exact path is below 1e-6 relative).  NaN compares false: not certain.
// One ballot per compare: the lane mask of the combined predicate was moved
// through a vector register in some kernels.  Must be called by the whole wave.
__device__ __forceinline__ uint64_t surely_culled(const Clip &c) {
    const float lim = c.cw * 1.001f;  // >= 0 whenever the first test fails
    return __ballot(c.cw <= 0.0f) | __ballot(__builtin_fabsf(c.cx) > lim) | __ballot(__builtin_fabsf(c.cy) > lim);
}

// Correctly rounded 1/w by one Newton-Raphson step: r = v_rcp_f32(w) (the
// hardware reciprocal estimate, about 1 ulp), residual e = fma(-w, r, 1), then
// q = fma(e, r, r).  The fused residual is exact, so the corrected q equals the
// IEEE quotient 1.0f / w for every w in [2^-125, 2^126] (every float of that
// range is checked against the division by pcr_check_reciprocal); outside that
// range, where the estimate or the residual leaves the normal range, the full
// division is used.
// For w <= 0 or NaN the value is not used (the point is culled).
__device__ __forceinline__ float recip_rn(float w) {
    float r = __builtin_amdgcn_rcpf(w);
    float e = __builtin_fmaf(-w, r, 1.0f);
    float q = __builtin_fmaf(e, r, r);
    const bool slow = (w > 0.0f && w < 0x1p-125f) || w > 0x1p126f;
    if (__ballot(slow) != 0) {  // uniform branch: the division only runs when a lane needs it
        float d = 1.0f / w;
        q = slow ? d : q;
    }
    return q;
}

__device__ __forceinline__ uint32_t finish(const View &v, const Clip &c, uint32_t &dbits) {
    float rw = recip_rn(c.cw);
    float fx = (c.cx * rw + 1.0f) * v.hw;
    float fy = (c.cy * rw + 1.0f) * v.hh;
    // Bitwise '&' (the tests have no side effects): evaluated without
    // branches, where '&&' made the compiler diverge on every point.
    bool ok = (c.cw > 0.0f) & (fx >= 0.0f) & (fx < v.fW) & (fy >= 0.0f) & (fy < v.fH);
    dbits = __float_as_uint(c.cw);
    uint32_t px = (uint32_t)(ok ? fx : 0.0f);
    uint32_t py = (uint32_t)(ok ? fy : 0.0f);
    // py < H and W are below 2^24 and W*H below 2^32; __umul24 returns the
    // low 32 bits of the product as a signed int, taken back as unsigned.
    const uint32_t pid = (uint32_t)__umul24(py, v.W) + px;
    return ok ? pid : kEmptyPid;
}

__device__ __forceinline__ uint32_t project(const View &v, float x, float y, float z,
                                            uint32_t &dbits) {
    return finish(v, clip(v, x, y, z), dbits);
}

// Projection with the wavefront-level early out: returns kEmptyPid for every
// lane when no lane of the wavefront can be visible.  `live`: lane mask of the
// lanes that hold a point (the others are past the end of the buffer), passed
// as a mask so that it stays in scalar registers across the callers' loops.
// Must be called by the whole wavefront.
__device__ __forceinline__ uint32_t project_wave(const View &v, const u32x4 &p, uint64_t live, uint32_t &dbits) {
    Clip c = clip(v, __uint_as_float(p.x), __uint_as_float(p.y), __uint_as_float(p.z));
    dbits = __float_as_uint(c.cw);
    if ((live & ~surely_culled(c)) == 0) return kEmptyPid;
    uint32_t pid = finish(v, c, dbits);
    return __builtin_amdgcn_inverse_ballot_w64(live) ? pid : kEmptyPid;
}

// Non-temporal 16-byte point load, addressed as global memory (point
// buffers are device memory; a generic load would also wait on LDS traffic).
__device__ __forceinline__ u32x4 load_point(const u32x4 *p) {
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) u32x4 *)p);
}

__device__ __forceinline__ u64 make_key(uint32_t dbits, uint32_t rgba) {
    return ((u64)dbits << 32) | (u64)rgba;
}

// Relaxed (non-synchronising) read of a framebuffer word for the early depth
// test (Sec. 3.2), at workgroup scope: an ordinary cached load, served by the
// XCD's L2 when the line is there instead of by the memory side where the
// atomics execute.  Within a kernel a framebuffer word only decreases, so a
// stale value is >= the current one and a stale read only costs a superfluous
// atomic, never a wrong skip; values from before the frame's clear cannot be
// read, because the clear is an earlier kernel and every kernel starts with
// the device-scope acquire that invalidates the caches.  (Measured: 5-23%
// faster early-z frames on overviews than device-scope reads.)
__device__ __forceinline__ u64 peek_u64(const u64 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t peek_u32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void gmin_u64(u64 *p, u64 v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gmin_u32(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gadd_u64(u64 *p, u64 v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int device_cus();
size_t max_lds();
int allow_lds(const void *kernel, size_t bytes);

#define PCR_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::pcr::fail(PCR_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define PCR_LAUNCHED()                                                                 \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return ::pcr::fail(PCR_EHIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

int check_image(uint32_t w, uint32_t h);
int check_variant(int variant);
size_t hq_depth_bytes(uint32_t w, uint32_t h);

struct Shape {
    uint32_t ppt, wg, grid;
    uint32_t group;  // views per point pass (batches)
    uint32_t slots;  // LDS hash slots of the deduplicating kernels (0 = tile/2)
    uint32_t run;    // basic kernel: consecutive points per lane (a multiple of ppt)
};
int resolve_shape(const pcr_tune *tune, int family, Shape &s);

// Kernels launched by more than one translation unit.
int launch_fill(void *p, size_t bytes, uint32_t word, hipStream_t s);

// One view slot of a batch plan's device table.
struct BatchView {
    View v;
    int32_t variant;  // PCR_BASIC / PCR_DEDUP / PCR_HQ
    uint32_t pad;
    u64 *fb;          // basic key buffer
    uint32_t *D;      // HQ depth
    u64 *S;           // HQ sums
    uint32_t *out;
};

// A group of a batch pass: views index[first .. first + count) of the table.
struct BatchGroup {
    uint32_t first, count;
};

// Grouped pass of a batch (pass 0: closest-point views and HQ depth passes;
// pass 1: HQ colour passes): each tile of the points is loaded once per group
// and rendered into the group's views in turn.  *ngroups and the tables are
// read when the kernel runs.  pass < 0 only raises the kernels' LDS limits.
int launch_group_pass(int pass, const u32x4 *pts, uint64_t n, const BatchView *views, const uint32_t *index,
                      const BatchGroup *groups, const uint32_t *ngroups, const Shape &sh, hipStream_t s);

// Single-view render pass of batch slot `slot`, read from a plan's device
// table when the kernel runs (nothing happens if slot >= *nviews): pass 0 the
// closest-point render or the HQ depth pass, pass 1 the HQ colour pass, each
// with the single-view deduplicating kernels.  pass < 0 only raises the
// kernels' LDS limits (to be done before a graph capture).
int launch_view_pass(int pass, const u32x4 *pts, uint64_t n, const BatchView *views, const uint32_t *nviews,
                     uint32_t slot, const Shape &sh, hipStream_t s);

}  // namespace pcr
