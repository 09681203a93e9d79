/*
 * pcr.h -- C ABI of libpcr, a compute point-cloud rasterizer for AMD Instinct
 * MI355X (gfx950).
 *
 * The operations follow Schuetz, Kerbl and Wimmer, "Rendering Point Clouds
 * with Compute Shaders and Vertex Order Optimization" (EGSR 2021):
 *   - closest-point rendering with one 64-bit atomic minimum per point on a
 *     (depth, colour) key, and its resolve pass ............. Sec. 3.1
 *   - the early depth test ................................... Sec. 3.2
 *   - local reduction / deduplication of same-pixel updates .. Sec. 3.3, 3.4
 *   - high-quality blending: depth pass, epsilon colour pass,
 *     integer-average resolve ................................ Sec. 3.5
 *   - Morton, shuffled-Morton and shuffled vertex orders ..... Sec. 4, Sec. 5
 *
 * Conventions common to every call
 *   - Buffer pointers marked "device" are device (HBM) pointers owned by the
 *     caller; the library never frees or retains them beyond the call, except
 *     the point buffer held by a batch plan (see pcr_batch_create).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls only
 *     enqueue work on `stream` and return; they never synchronise.  Results are
 *     valid once the stream has reached the call.
 *   - Return value: PCR_OK (0) or a negative PCR_E* code.  pcr_last_error()
 *     then returns a message for the calling thread.  Argument errors are
 *     detected on the host before anything is enqueued.  A fault inside a
 *     kernel is reported by HIP on a later call or stream synchronisation.
 *   - Render-path calls (clear, render, resolve, reorder, batch launch)
 *     allocate no memory.
 *   - Images: row-major, W*H pixels, row 0 is the bottom row (NDC y = -1).
 *
 * Points
 *   16-byte records {float x, y, z; uint32 rgba}, 16-byte aligned, colour red
 *   in bits 0-7, green 8-15, blue 16-23, alpha 24-31 (Sec. 5 quotes 16 bytes
 *   per point for every data set).
 *
 * Projection (Sec. 3.1; the paper leaves the pixel mapping open, this is the
 * library's reading): clip = MVP * (x, y, z, 1) in float32, each row summed
 * left to right with one rounding per operation and no fused multiply-add; the
 * point is culled unless w > 0; rw = 1/w correctly rounded; fx = (cx*rw + 1) *
 * (W/2), fy = (cy*rw + 1) * (H/2); culled unless 0 <= fx < W and 0 <= fy < H;
 * pixel (trunc fx, trunc fy); the depth is the linear w (Sec. 3.1 closing
 * paragraph).  Clip z is not used (no near/far clipping).
 */
#ifndef PCR_H
#define PCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcr_point {
    float x, y, z;
    uint32_t rgba;
} pcr_point;

/* Status codes. */
enum {
    PCR_OK = 0,
    PCR_EINVAL = -1,      /* bad argument (nothing was enqueued) */
    PCR_EHIP = -2,        /* a HIP call failed */
    PCR_ENOMEM = -3,      /* scratch too small or allocation failed */
    PCR_EUNSUPPORTED = -4 /* valid request the build does not support */
};

/* Variants (low byte of `variant`).
 * PCR_BASIC  closest point per pixel by 64-bit atomicMin (Sec. 3.1).
 * PCR_DEDUP  the same image; same-pixel updates are merged inside each
 *            wavefront and workgroup before the global atomic (Sec. 3.3-3.4).
 *            Adding PCR_F_LDS | PCR_F_REDUCE | PCR_F_EARLYZ also skips the
 *            global atomic when the stored key is already smaller (Sec. 3.2):
 *            worth it on unordered clouds, whose tiles merge little, and a
 *            cost on ordered ones, so the default leaves it off.
 * PCR_HQ     blended colour of the points within 1% of the closest depth of
 *            each pixel: depth pass, colour pass, integer resolve (Sec. 3.5). */
enum { PCR_BASIC = 0, PCR_DEDUP = 1, PCR_HQ = 2 };

/* Flag bits OR-ed into `variant`.  They select the update path only: every
 * combination yields bit-identical framebuffers.  With none of EARLYZ,
 * REDUCE (or its two steps), LDS and PLAIN the variant's default path is
 * used: PCR_BASIC = one global atomic per point; PCR_DEDUP and PCR_HQ = the
 * tuned merging path.
 *   PCR_F_EARLYZ  read the stored value first, skip the atomic when it is not
 *                 larger (Sec. 3.2; safe because values only decrease)
 *   PCR_F_REDUCE  merge same-pixel updates inside a wavefront before the
 *                 atomic: the lanes sharing a leader lane's pixel keep their
 *                 minimum (the all-lanes-equal case of Sec. 3.3, for up to
 *                 two leaders with 24 or more lanes each); without PCR_F_LDS, neighbouring lane pairs
 *                 then merge as well (Sec. 3.3).  For PCR_HQ without
 *                 PCR_F_LDS it applies to the depth pass, and the leader
 *                 groups also pool their colour sums in the colour pass.
 *   PCR_F_REDUCE_WAVE / PCR_F_REDUCE_PAIR  one of PCR_F_REDUCE's two steps
 *                 alone: the leader groups, or the neighbouring pairs (the
 *                 latter only without PCR_F_LDS, else PCR_EINVAL).  Both
 *                 bits = PCR_F_REDUCE.
 *   PCR_F_LDS     merge all equal pixels of a workgroup's tile in an LDS hash
 *                 table before the atomics (Sec. 3.4's deduplication)
 *   PCR_F_PLAIN   none of the above (for PCR_HQ: every point within the
 *                 blend window adds its own two sum words by global atomics,
 *                 the paper's plain two-atomic colour pass)
 *   PCR_F_HQ_DEPTH / PCR_F_HQ_COLOR  (PCR_HQ) run only that pass; neither bit
 *                 = both passes in order.  Running the depth pass over several
 *                 point buffers and then the colour pass over the same buffers
 *                 renders their union.
 *   PCR_F_HQ_PACKED  (PCR_HQ) the single-atomic form of Sec. 3.5.1: the colour
 *                 sums of a pixel live in one 64-bit word,
 *                 r << 46 | g << 28 | b << 10 | count (18-bit colour sums, a
 *                 10-bit count; each contributing point adds its packed value
 *                 modulo 2^64, so a full field carries into the next one up).
 *                 Exact while at most 1023 points blend into one pixel; with
 *                 more, that pixel's colour is wrong (1024 points wrap the
 *                 count and the pixel resolves empty).  One global atomic per
 *                 merged update instead of two.  Pass the flag to
 *                 pcr_fb_clear, pcr_render, pcr_resolve and pcr_resolve_depth
 *                 alike (the word of pixel k is the k-th 64-bit word of the
 *                 sums area; the framebuffer size is unchanged).  Not
 *                 accepted in batch views.
 *   PCR_F_HQ_ROBUST  (PCR_HQ) the robust single-atomic form of Sec. 3.5.1:
 *                 each pixel also has a fast word r << 48 | g << 32 | b << 16
 *                 | count holding the sums of at most 255 points, updated by
 *                 one 64-bit compare-and-swap per merged update; an update
 *                 that would take the count past 255 moves the word's sums to
 *                 the two-word sums (the fallback buffers) and resets the word,
 *                 updates of more than 255 points go to the fallback directly,
 *                 and the resolve adds the fast word to the fallback.  Exact
 *                 for any number of points per pixel and any number of
 *                 concurrent updates (bit-identical images to PCR_HQ; the sum
 *                 words fast + fallback equal PCR_HQ's).  The framebuffer
 *                 grows by 8 bytes per pixel: pass the flag to pcr_fb_bytes,
 *                 pcr_fb_clear, pcr_render, pcr_resolve and pcr_resolve_depth
 *                 alike.  Excludes PCR_F_HQ_PACKED; not accepted in batch
 *                 views. */
enum {
    PCR_F_EARLYZ = 1 << 8,
    PCR_F_REDUCE = 1 << 9,
    PCR_F_LDS = 1 << 10,
    PCR_F_PLAIN = 1 << 11,
    PCR_F_HQ_DEPTH = 1 << 12,
    PCR_F_HQ_COLOR = 1 << 13,
    PCR_F_HQ_PACKED = 1 << 14,
    PCR_F_HQ_ROBUST = 1 << 15,
    PCR_F_REDUCE_WAVE = 1 << 16,
    PCR_F_REDUCE_PAIR = 1 << 17
};

/* Vertex orders (Sec. 4, Sec. 5). */
enum {
    PCR_ORDER_MORTON = 0,         /* stable sort by 63-bit Morton code */
    PCR_ORDER_MORTON_SHUFFLE = 1, /* Morton, then batches moved to random places */
    PCR_ORDER_SHUFFLE = 2         /* sort by one random key per point */
};

/* Launch shape for the render kernels.  Zero fields take the defaults
 * (measured on MI355X), all with 64-thread (one-wavefront) workgroups that
 * step over the tiles in their natural order: basic 4 points per thread per
 * step, adaptive lane mapping over 2,048-point sub-tiles and 64 workgroups
 * per compute unit; deduplicating 4 and HQ 8 points per thread, 256 LDS slots
 * and 512 workgroups per compute unit.
 *   ppt    points per thread (1, 2, 4, 8 or 16)
 *   wg     workgroup size (64, 128, 256, 512 or 1024)
 *   grid   workgroups per launch; each takes tiles g, g + grid, ... (0 = the
 *          default above)
 *   group  views per group of a batch's grouped passes (0 = 16, at most 32;
 *          a group also closes at 2 GiB of framebuffers; 1 = every view its
 *          own pass with the single-view kernels)
 *   slots  LDS hash-table slots per workgroup of the deduplicating kernels,
 *          rounded up to a power of two in [256, 32768] (0 = half a tile)
 *   run    basic kernel (PCR_BASIC without flags): consecutive points per lane,
 *          a multiple of ppt up to 4096, taken ppt at a time, so that one
 *          atomic instruction covers points `run` apart; 0 = adaptive: per
 *          wavefront and sub-tile of 2,048 points, lanes on neighbouring
 *          points while they fall on distinct pixels of shared cache lines,
 *          runs of 28 points (for 4 per step) while neighbouring points
 *          share pixels.  Any value gives the same framebuffer. */
typedef struct pcr_tune {
    uint32_t ppt;
    uint32_t wg;
    uint32_t grid;
    uint32_t group;
    uint32_t slots;
    uint32_t run;
} pcr_tune;

/* Framebuffer layout (device memory, size pcr_fb_bytes):
 *   PCR_BASIC / PCR_DEDUP: uint64 key[W*H]; key = (depth bits << 32) | rgba,
 *     cleared to all ones; the smallest key of a pixel is its closest point
 *     (ties in depth go to the smaller colour word).
 *   PCR_HQ: uint32 depth[W*H] (float bits, cleared to 0xFFFFFFFF), then at the
 *     next 256-byte boundary uint64 sum[2*W*H] with sum[2p] = (R sum << 32) |
 *     G sum and sum[2p+1] = (B sum << 32) | count, each word modulo 2^64
 *     (Sec. 3.5 packs the four 32-bit channels into two 64-bit integers);
 *     with PCR_F_HQ_PACKED, sum[p] is pixel p's packed word (see the flag);
 *     with PCR_F_HQ_ROBUST, sum[2p], sum[2p+1] are the fallback words and
 *     sum[2*W*H + p] is pixel p's fast word (see the flag).
 * Returns 0 for invalid sizes or variants. */
size_t pcr_fb_bytes(uint32_t w, uint32_t h, int variant);

/* Clears a framebuffer for a new frame.  fb: device, pcr_fb_bytes(w, h,
 * variant) bytes, 16-byte aligned.  w, h in [1, 2^24), w*h < 2^32. */
int pcr_fb_clear(void *fb, uint32_t w, uint32_t h, int variant, void *stream);

/* Renders n points into fb (Sec. 3.1-3.5).
 *   pts  device, n records, 16-byte aligned (ignored when n == 0)
 *   mvp  host, 16 floats, row-major (mvp[4*row + col]); copied by value, the
 *        array may be reused as soon as the call returns
 *   fb   device framebuffer of the variant, cleared by pcr_fb_clear
 * Basic and dedup accumulate: several calls on one framebuffer render the union
 * of their points.  PCR_HQ runs its depth pass and then its colour pass over
 * `pts` (or only the pass named by a PCR_F_HQ_* bit).  n == 0 is a no-op.
 * Errors: PCR_EINVAL for null or misaligned pointers, bad sizes, unknown
 * variant or flag bits. */
int pcr_render(const pcr_point *pts, uint64_t n, const float mvp[16], uint32_t w, uint32_t h,
               int variant, void *fb, void *stream);

/* pcr_render with an explicit launch shape (tune may be NULL). */
int pcr_render_ex(const pcr_point *pts, uint64_t n, const float mvp[16], uint32_t w, uint32_t h,
                  int variant, void *fb, const pcr_tune *tune, void *stream);

/* One chunk of a many-chunk frame: a separate point buffer (e.g. one node of a
 * level-of-detail octree).  16 bytes, as stored in a device array. */
typedef struct pcr_chunk {
    const pcr_point *pts; /* device, 16-byte aligned */
    uint64_t n;           /* points in the chunk */
} pcr_chunk;

/* Largest point count of one chunk; larger chunks are skipped. */
#define PCR_CHUNK_MAX_POINTS (1ull << 36)

/* Device scratch that pcr_render_chunks needs for nchunks chunks
 * (0 if nchunks is 0 or above 2^24). */
size_t pcr_chunks_scratch_bytes(uint32_t nchunks);

/* Renders many separate point buffers into one framebuffer with one
 * launch per geometry pass (Sec. 5.4: level-of-detail structures
 * draw thousands of small buffers per frame; per-buffer dispatches are what
 * makes them slow).  The result is the frame of the concatenation of the
 * chunks (basic, dedup and HQ alike; the order of points does not change a
 * closest-point image or an HQ sum).
 *   chunks     device array of nchunks pcr_chunk records, read on the device
 *              (so a GPU-side selection can write it).  A chunk with a NULL or
 *              misaligned pointer, or more than PCR_CHUNK_MAX_POINTS points,
 *              is skipped (contributes nothing); n == 0 is an empty chunk.
 *   nchunks    at most 2^24; 0 is a no-op.
 *   scratch    device, at least pcr_chunks_scratch_bytes(nchunks) bytes
 *              (8 bytes per chunk plus 512 KiB), 256-byte aligned;
 *              overwritten (chunk start offsets, each workgroup's first
 *              chunk).
 *   variant    PCR_BASIC, PCR_DEDUP or PCR_HQ; PCR_HQ optionally with one
 *              PCR_F_HQ_DEPTH / PCR_F_HQ_COLOR pass bit and PCR_F_HQ_PACKED;
 *              the other flag bits give PCR_EUNSUPPORTED.
 *   tune       as pcr_render_ex (may be NULL); the grid is at most 2^17
 *              workgroups (larger values are clamped), each taking one
 *              contiguous range of tiles.  Tiles of wg*ppt points never span
 *              two chunks (the last tile of a chunk is partial).
 * Errors: PCR_EINVAL (as pcr_render, plus NULL chunks with nchunks > 0,
 * nchunks > 2^24), PCR_ENOMEM (scratch too small). */
int pcr_render_chunks(const pcr_chunk *chunks, uint32_t nchunks, const float mvp[16], uint32_t w,
                      uint32_t h, int variant, void *fb, void *scratch, size_t scratch_bytes,
                      const pcr_tune *tune, void *stream);

/* Largest chunk count of pcr_render_chunks_static. */
#define PCR_STATIC_CHUNKS_MAX (1u << 20)

/* pcr_render_chunks without the scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The scratch lives in a device array
 * owned by the library, pcr_chunks_scratch_bytes(PCR_STATIC_CHUNKS_MAX) bytes
 * (8.5 MiB) per GPU, held from the first call on that GPU until the process
 * ends.  The call
 * allocates nothing.  Every call on one GPU shares that GPU's array, so calls
 * whose work overlaps on one GPU (e.g. on two streams) race and give wrong
 * frames: order them.  The array's old contents never matter (each call
 * rewrites what it reads before use).
 * Arguments and result as pcr_render_chunks; errors as pcr_render_chunks,
 * plus PCR_EINVAL for nchunks > PCR_STATIC_CHUNKS_MAX. */
int pcr_render_chunks_static(const pcr_chunk *chunks, uint32_t nchunks, const float mvp[16], uint32_t w,
                             uint32_t h, int variant, void *fb, const pcr_tune *tune, void *stream);

/* Resolve pass (Sec. 3.1 second listing, Sec. 3.5 resolve listing).
 *   rgba_out  device, uint32[W*H].
 * Basic/dedup: the colour word of the stored key, 0 where nothing landed.
 * HQ: per channel floor(sum / count) (integer division), alpha 255; 0 where
 * the count is 0. */
int pcr_resolve(const void *fb, uint32_t w, uint32_t h, int variant, uint32_t *rgba_out,
                void *stream);

/* The framebuffer's words in one linear layout, whatever the sum layout, for
 * tests and tools (the raw output the resolve of Sec. 3.1 and Sec. 3.5 reads).
 *   raw_out  device, 8-byte aligned:
 *            PCR_BASIC / PCR_DEDUP: uint64[W*H], the keys as stored;
 *            PCR_HQ: uint64[3*W*H], three planes: the depth bits (zero-
 *            extended; 0xFFFFFFFF where nothing landed), R << 32 | G sums,
 *            B << 32 | count.  With PCR_F_HQ_ROBUST the fast and fallback
 *            words are combined (the words equal PCR_HQ's); with
 *            PCR_F_HQ_PACKED the packed word's fields as stored (18-bit
 *            colour sums, 10-bit count).
 * Errors: as pcr_resolve. */
int pcr_resolve_raw(const void *fb, uint32_t w, uint32_t h, int variant, unsigned long long *raw_out,
                    void *stream);

/* Depth output modes of pcr_resolve_depth. */
enum { PCR_DEPTH_LINEAR = 0, PCR_DEPTH_HYPERBOLIC = 1 };

/* Resolve with a depth image (Sec. 3.1, closing paragraph: the stored depth is
 * the linear clip-space w, usable for depth buffering as it is; conventional
 * depth values, e.g. for hybrid rendering with triangles, are derived in the
 * resolve).
 *   mode       PCR_DEPTH_LINEAR: depth_out = w of the pixel's closest point.
 *              PCR_DEPTH_HYPERBOLIC: depth_out = a + b * (1/w) with a correctly
 *              rounded reciprocal, then one product and one sum, each rounded
 *              once (no fused multiply-add).  For a perspective projection with
 *              near n and far f: a = f/(f-n), b = -f*n/(f-n) gives the window
 *              depth in [0,1] (0 at the near plane); a = -n/(f-n), b = f*n/(f-n)
 *              gives reverse-z (1 at the near plane).
 *   empty      value written where nothing landed.
 *   rgba_out   device uint32[W*H] or NULL: when given, the pcr_resolve image,
 *              written in the same pass.
 *   depth_out  device float[W*H], 4-byte aligned.
 * HQ: the depth of a pixel is the closest depth kept by the depth pass.
 * Errors: as pcr_resolve; PCR_EINVAL for an unknown mode or a NULL depth_out. */
int pcr_resolve_depth(const void *fb, uint32_t w, uint32_t h, int variant, int mode, float a,
                      float b, float empty, uint32_t *rgba_out, float *depth_out, void *stream);

/* Device scratch needed by pcr_reorder for n points (0 if n is too large). */
size_t pcr_reorder_scratch_bytes(uint64_t n, int order, uint32_t batch);

/* Reorders a point buffer (Sec. 4: Morton order and shuffled Morton order;
 * Sec. 5: the shuffled order and the 21-level Morton code).
 *   in, out    device, n records each, must not overlap
 *   perm_out   device uint32[n] or NULL: perm_out[j] = input index of out[j]
 *   order      PCR_ORDER_*
 *   batch      batch size of PCR_ORDER_MORTON_SHUFFLE (the paper uses 128)
 *   seed       seed of the shuffle keys: batch b (or point i) gets the b-th
 *              (i-th) output of SplitMix64 seeded with `seed`, and batches are
 *              emitted in ascending (key, index) order
 *   scratch    device, scratch_bytes >= pcr_reorder_scratch_bytes(n, order, batch)
 * Morton codes interleave 21-bit cell indices of the cubic bounding box
 * (x in bit 3i, y in 3i+1, z in 3i+2); cell = min(trunc(((v - lo) / size) *
 * 2^21), 2^21 - 1) in float32.  Equal codes keep their input order.  n must be
 * below 2^32.  The Morton orders are defined for finite coordinates; with NaN
 * or infinite ones the order is unspecified, but out is still a permutation
 * of in (out[j] = in[perm_out[j]]). */
int pcr_reorder(const pcr_point *in, pcr_point *out, uint32_t *perm_out, uint64_t n, int order,
                uint32_t batch, uint64_t seed, void *scratch, size_t scratch_bytes, void *stream);

/* One view of a batch: camera, image size, variant and its buffers. */
typedef struct pcr_view {
    float mvp[16];      /* row-major */
    uint32_t w, h;
    int32_t variant;    /* PCR_BASIC, PCR_DEDUP or PCR_HQ (flag bits ignored); -1 = unused slot */
    uint32_t reserved;
    void *fb;           /* device framebuffer of the variant (cleared by the batch) */
    uint32_t *rgba_out; /* device uint32[w*h], resolved image */
} pcr_view;

/* A batch plan renders up to `capacity` views of one resident point buffer per
 * launch: the framebuffers are cleared, the views are rendered by grouped
 * passes that load each tile of points once per group of views and render it
 * into each view of the group in turn (or, with tune->group == 1, by one
 * single-view render pass per view slot), and every view is resolved.  The launch is a single hipGraph replay.  Each view's
 * image is bit-identical to pcr_fb_clear + pcr_render + pcr_resolve of that
 * view alone.  The plan allocates its device view table and graph at
 * creation; pcr_batch_launch allocates nothing.  A plan is not thread-safe;
 * a launch on another stream than the previous one waits for it on the
 * device (launches of one plan never overlap). */
typedef struct pcr_batch pcr_batch;

int pcr_batch_create(pcr_batch **plan, const pcr_point *pts, uint64_t n, uint32_t capacity,
                     const pcr_tune *tune, void *stream);

/* Enqueues one batch: views[0..nviews) (host array, copied before return),
 * nviews <= capacity. */
int pcr_batch_launch(pcr_batch *plan, const pcr_view *views, uint32_t nviews, void *stream);

/* Waits for the plan's enqueued launches to complete, then frees it (NULL is
 * a no-op).  Returns PCR_OK. */
int pcr_batch_destroy(pcr_batch *plan);

/* One-call form of a batch (the views of one launch, as pcr_batch_launch):
 * the library keeps up to 8 plans, keyed by device, point buffer, n, launch
 * shape and capacity (nviews rounded up to a power of two, at least 4), and
 * creates one on the first call with a new key (that call allocates; calls
 * that reuse a plan allocate nothing).  A cached plan refers to `pts`: call
 * pcr_release_batch_plans before freeing a point buffer that was batched.
 * Thread-safe; launches of one cached plan on different streams are ordered.
 * nviews == 0 is a no-op; errors as pcr_batch_create / pcr_batch_launch. */
int pcr_render_batch(const pcr_point *pts, uint64_t n, const pcr_view *views, uint32_t nviews,
                     const pcr_tune *tune, void *stream);

/* Destroys every cached plan of pcr_render_batch (waits for their launches). */
int pcr_release_batch_plans(void);

/* Self-check of the projection's reciprocal (see the Projection paragraph),
 * over the floats w with bit patterns in [first_bits, last_bits]:
 *   result  device uint64[3], 8-byte aligned, accumulated into (clear it first):
 *           result[0] += number of w whose reciprocal used by the render kernels
 *                        differs from the device's IEEE division 1.0f / w;
 *           result[1] += sum of the reciprocals' bit patterns (modulo 2^64);
 *           result[2] ^= exclusive or of the reciprocals' bit patterns.
 * The digest lets a caller compare the kernels' reciprocals with IEEE
 * quotients computed elsewhere (e.g. on the host), independently of the
 * device division.  result[0] == 0 over [0x00000001, 0x7F7FFFFF] means the
 * fast reciprocal agrees with the device division for every positive finite
 * float. */
int pcr_check_reciprocal(uint32_t first_bits, uint32_t last_bits, unsigned long long *result,
                         void *stream);

/* ---- Measurement helpers (not part of rendering) ---------------------- */

/* Adds to *count (device uint64, 8-byte aligned) the number of the n points
 * that the projection keeps for this camera and image (the points that are
 * not culled): the number of global atomics of a PCR_BASIC render of them
 * (Sec. 3.1: one atomicMin per visible point).  Errors as pcr_render. */
int pcr_count_visible(const pcr_point *pts, uint64_t n, const float mvp[16], uint32_t w, uint32_t h,
                      unsigned long long *count, void *stream);

/* Access patterns of pcr_probe_atomics. */
enum {
    PCR_PROBE_RANDOM = 0,    /* every lane its own random word */
    PCR_PROBE_LINE = 1,      /* 8 lanes on the 8 words of one random 64-byte line */
    PCR_PROBE_ADDRESS = 2,   /* all 64 lanes of a wavefront on one random word */
    PCR_PROBE_CONTIGUOUS = 3 /* a wavefront on 64 consecutive words */
};

/* Throughput probe of device-scope 64-bit unsigned atomic minimum, the
 * operation of the basic renderer (Sec. 3.1), on buf[0, words): workgroups x
 * 256 lanes each issue `iters` atomics with addresses drawn by `pattern` from
 * a hash of (seed, lane or wavefront, iteration).  returning != 0 uses the
 * value-returning form (sink: device uint64, written only in an impossible
 * case, so that the returned values are consumed).  Timing the call gives
 * atomics per second for the footprint 8 * words bytes.
 *   buf    device, 64-byte aligned, 8 * words bytes, overwritten
 *   words  a multiple of 64 in [64, 2^32)
 * Errors: PCR_EINVAL for bad pointers, sizes or pattern. */
int pcr_probe_atomics(unsigned long long *buf, uint64_t words, int pattern, int returning, uint32_t workgroups,
                      uint32_t iters, uint32_t seed, unsigned long long *sink, void *stream);

/* Read-rate probe: streams the n16 16-byte records of buf once, in the
 * access pattern of the render kernels' point loads (non-temporal 16-byte
 * loads, workgroup tiles of per_thread * 256 records, grid-stride over the
 * tiles), and does nothing else with them, so that timing the call gives the
 * rate at which the chip delivers a point buffer (the floor of a frame of the
 * deduplicating renderers, Sec. 3.4, whose point stream is their only HBM
 * traffic).
 *   buf         device, 16-byte aligned, 16 * n16 bytes, only read
 *   per_thread  4 or 8 records per lane and tile
 *   workgroups  in [1, 2^22], of 256 threads
 *   sink        device uint32, 4-byte aligned; a lane stores the XOR of its
 *               records there when it equals one fixed value (so that every
 *               loaded value is consumed): its content means nothing
 * n16 = 0 is a no-op.  Errors: PCR_EINVAL for bad pointers or sizes. */
int pcr_probe_read(const void *buf, uint64_t n16, uint32_t per_thread, uint32_t workgroups, uint32_t *sink,
                   void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *pcr_last_error(void);

/* Library version string. */
const char *pcr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PCR_H */
