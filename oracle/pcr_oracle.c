/*
 * pcr_oracle.c -- reference CPU implementation of the compute point rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares no
 * header, helper, table or constant with the GPU code.
 *
 * Source: Schuetz, Kerbl, Wimmer, "Rendering Point Clouds with Compute Shaders
 * and Vertex Order Optimization", EGSR 2021 (arXiv 2104.07526).
 *
 * Everything here is plain, single-threaded and in input order.  Floating point
 * is IEEE binary32 (the paper's shaders transform in float), one rounding per
 * operation, round to nearest even, no fused multiply-add (build with
 * -ffp-contract=off -fno-fast-math on x86-64 SSE), no flush-to-zero.
 *
 * Readings taken where the paper is silent (each also listed in the design
 * notes of the repository):
 *   - pixel mapping ("toPixelID" is left opaque in Sec. 3.1): cull unless
 *     w > 0; NDC->pixel by (c/w + 1) * (size/2) with one correctly rounded
 *     reciprocal 1/w; half-open viewport [0,W)x[0,H) tested in float; truncate;
 *     row 0 is the bottom row (NDC y = -1); no near/far clip on clip z.
 *   - key layout: Sec. 3.1 puts depth above colour in one 64-bit integer; here
 *     depth bits occupy the high 32 bits and the full 32-bit RGBA word the low
 *     32 bits, compared unsigned (w > 0 makes float order = bit order).
 *   - HQ threshold: depth <= fl32(closest * 1.01f) (Sec. 3.5, epsilon = 1%).
 *   - HQ output alpha 255 on covered pixels; empty pixels resolve to 0.
 *   - Morton code: 21 bits per axis over the cubic bounding box (Sec. 5, the
 *     21-level octree), bit 3i = x_i, 3i+1 = y_i, 3i+2 = z_i; stable sort.
 *   - shuffles (Sec. 4 and Sec. 5): each batch (or point) gets the b-th output
 *     of SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) seeded with `seed`; the
 *     batches are emitted in ascending (key, batch index).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <xmmintrin.h>

/* 16-byte point record: position in float, colour R in bits 0-7, G 8-15,
 * B 16-23, A 24-31. */
struct opoint {
    float x, y, z;
    uint32_t rgba;
};

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* Returns 1 when the x86 control register has neither flush-to-zero nor
 * denormals-are-zero set, so that the float results below are IEEE results. */
int oracle_fp_env_ok(void)
{
    unsigned csr = _mm_getcsr();
    return (csr & 0x8040u) == 0u; /* FTZ = bit 15, DAZ = bit 6 */
}

/* Projection of one point (Sec. 3.1: position times world-view-projection,
 * linear depth = clip w, Sec. 3.1 closing paragraph).  m is row-major,
 * m[4*r + c].  Returns 1 and writes the pixel index and the depth bits when the
 * point lands in the viewport, else 0. */
int oracle_project(const float *m, uint32_t W, uint32_t H,
                   float x, float y, float z,
                   uint32_t *pid_out, uint32_t *dbits_out)
{
    float cx = ((m[0] * x + m[1] * y) + m[2] * z) + m[3];
    float cy = ((m[4] * x + m[5] * y) + m[6] * z) + m[7];
    float cw = ((m[12] * x + m[13] * y) + m[14] * z) + m[15];
    if (!(cw > 0.0f))
        return 0;
    float rw = 1.0f / cw;
    float hw = 0.5f * (float)W;
    float hh = 0.5f * (float)H;
    float fx = (cx * rw + 1.0f) * hw;
    float fy = (cy * rw + 1.0f) * hh;
    if (!(fx >= 0.0f && fx < (float)W && fy >= 0.0f && fy < (float)H))
        return 0;
    uint32_t px = (uint32_t)fx;
    uint32_t py = (uint32_t)fy;
    *pid_out = py * W + px;
    *dbits_out = f2u(cw);
    return 1;
}

/* Projects every point; pid[i] = pixel or 0xFFFFFFFF when culled. */
void oracle_project_all(const struct opoint *pts, uint64_t n, const float *m,
                        uint32_t W, uint32_t H, uint32_t *pid, uint32_t *dbits)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t p, d;
        if (oracle_project(m, W, H, pts[i].x, pts[i].y, pts[i].z, &p, &d)) {
            pid[i] = p;
            dbits[i] = d;
        } else {
            pid[i] = 0xFFFFFFFFu;
            dbits[i] = 0xFFFFFFFFu;
        }
    }
}

/* ---- basic closest-point rendering (Sec. 3.1) -------------------------- */

void oracle_clear_basic(uint64_t *fb, uint32_t W, uint32_t H)
{
    for (uint64_t p = 0; p < (uint64_t)W * H; ++p)
        fb[p] = 0xFFFFFFFFFFFFFFFFull;
}

/* Accumulates the points into fb: each pixel keeps the smallest
 * (depth bits << 32 | rgba) among the points landing on it. */
void oracle_render_basic(const struct opoint *pts, uint64_t n, const float *m,
                         uint32_t W, uint32_t H, uint64_t *fb)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t pid, dbits;
        if (!oracle_project(m, W, H, pts[i].x, pts[i].y, pts[i].z, &pid, &dbits))
            continue;
        uint64_t key = ((uint64_t)dbits << 32) | (uint64_t)pts[i].rgba;
        if (key < fb[pid])
            fb[pid] = key;
    }
}

/* Resolve (Sec. 3.1, second listing): the colour word of the stored key;
 * a pixel nothing landed on resolves to 0. */
void oracle_resolve_basic(const uint64_t *fb, uint32_t W, uint32_t H, uint32_t *out)
{
    for (uint64_t p = 0; p < (uint64_t)W * H; ++p)
        out[p] = fb[p] == 0xFFFFFFFFFFFFFFFFull ? 0u : (uint32_t)fb[p];
}

/* ---- high-quality blended rendering (Sec. 3.5) ------------------------- */

void oracle_clear_hq(uint32_t *D, uint64_t *RG, uint64_t *BA, uint32_t W, uint32_t H)
{
    for (uint64_t p = 0; p < (uint64_t)W * H; ++p) {
        D[p] = 0xFFFFFFFFu;
        RG[p] = 0;
        BA[p] = 0;
    }
}

/* Depth pass: 32-bit minimum of the depth bits per pixel. */
void oracle_render_hq_depth(const struct opoint *pts, uint64_t n, const float *m,
                            uint32_t W, uint32_t H, uint32_t *D)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t pid, dbits;
        if (!oracle_project(m, W, H, pts[i].x, pts[i].y, pts[i].z, &pid, &dbits))
            continue;
        if (dbits < D[pid])
            D[pid] = dbits;
    }
}

/* Colour pass (Sec. 3.5): a point blends into its pixel when its depth is at
 * most the pixel's closest depth times 1.01.  Each pixel gathers four exact
 * sums over its blending points -- red, green, blue and their number -- and
 * the framebuffer stores them in the paper's two 64-bit words: the red sum in
 * the upper half of the first word over the green sum, the blue sum in the
 * upper half of the second over the count.  A call adds this call's sums to
 * the stored words as the 64-bit integer (sum_hi * 2^32 + sum_lo) modulo 2^64,
 * which is what adding every point's packed value modulo 2^64 amounts to (a
 * low sum past 32 bits carries into the high half). */
void oracle_render_hq_color(const struct opoint *pts, uint64_t n, const float *m,
                            uint32_t W, uint32_t H, const uint32_t *D,
                            uint64_t *RG, uint64_t *BA)
{
    uint64_t npix = (uint64_t)W * H;
    uint64_t *sum = calloc(4 * npix + 1, sizeof(uint64_t)); /* [channel][pixel]: r, g, b, count */
    if (!sum)
        abort();
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t pid, dbits;
        if (!oracle_project(m, W, H, pts[i].x, pts[i].y, pts[i].z, &pid, &dbits))
            continue;
        if (!(u2f(dbits) <= u2f(D[pid]) * 1.01f))
            continue;
        for (int c = 0; c < 3; ++c)
            sum[c * npix + pid] += (pts[i].rgba >> (8 * c)) & 0xFFu;
        sum[3 * npix + pid] += 1;
    }
    for (uint64_t p = 0; p < npix; ++p) {
        RG[p] += (sum[p] << 32) + sum[npix + p];
        BA[p] += (sum[2 * npix + p] << 32) + sum[3 * npix + p];
    }
    free(sum);
}

/* Both passes over one cloud, in the paper's order: depth, then colour. */
void oracle_render_hq(const struct opoint *pts, uint64_t n, const float *m,
                      uint32_t W, uint32_t H, uint32_t *D, uint64_t *RG, uint64_t *BA)
{
    oracle_render_hq_depth(pts, n, m, W, H, D);
    oracle_render_hq_color(pts, n, m, W, H, D, RG, BA);
}

/* Resolve (Sec. 3.5): each channel's sum divided by the count, truncating;
 * the four 32-bit fields are read back from the two words (red = upper half
 * of the first, green = its lower half, blue = upper half of the second,
 * count = its lower half); alpha 255; a pixel with count 0 resolves to 0. */
void oracle_resolve_hq(const uint64_t *RG, const uint64_t *BA, uint32_t W, uint32_t H,
                       uint32_t *out)
{
    for (uint64_t p = 0; p < (uint64_t)W * H; ++p) {
        uint64_t field[4] = {RG[p] >> 32, RG[p] & 0xFFFFFFFFull, BA[p] >> 32, BA[p] & 0xFFFFFFFFull};
        uint64_t count = field[3];
        if (count == 0) {
            out[p] = 0;
            continue;
        }
        uint32_t colour = 0xFF000000u;
        for (int c = 0; c < 3; ++c)
            colour |= (uint32_t)((field[c] / count) & 0xFFu) << (8 * c);
        out[p] = colour;
    }
}

/* ---- single-atomic HQ colour sums (Sec. 3.5.1, the 18-18-18-10 form) ---
 * Red, green and blue sums in 18 bits each and the count in 10 bits of one
 * 64-bit word per pixel.  Reading of the field order, which the paper leaves
 * open for this form: red highest, the count lowest, as in its 16-16-16-16
 * listing: word = r << 46 | g << 28 | b << 10 | count.  Every contributing
 * point adds its packed value modulo 2^64, so a field that passes its width
 * carries into the next one up; the sums are exact while at most 1023 points
 * blend into one pixel (255 * 1023 < 2^18).  Depth pass and threshold as in
 * oracle_render_hq_color. */
void oracle_render_hq_packed_color(const struct opoint *pts, uint64_t n, const float *m,
                                   uint32_t W, uint32_t H, const uint32_t *D, uint64_t *P)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t pid, dbits;
        if (!oracle_project(m, W, H, pts[i].x, pts[i].y, pts[i].z, &pid, &dbits))
            continue;
        float depth = u2f(dbits);
        float limit = u2f(D[pid]) * 1.01f;
        if (depth <= limit) {
            uint64_t r = pts[i].rgba & 0xFFu;
            uint64_t g = (pts[i].rgba >> 8) & 0xFFu;
            uint64_t b = (pts[i].rgba >> 16) & 0xFFu;
            P[pid] += (r << 46) | (g << 28) | (b << 10) | 1u;
        }
    }
}

/* Resolve of the packed word: the count is its low 10 bits; each channel its
 * 18-bit field divided by the count (truncating); alpha 255; count 0 -> 0. */
void oracle_resolve_hq_packed(const uint64_t *P, uint32_t W, uint32_t H, uint32_t *out)
{
    for (uint64_t p = 0; p < (uint64_t)W * H; ++p) {
        uint64_t a = P[p] & 0x3FFull;
        if (a == 0) {
            out[p] = 0;
            continue;
        }
        uint64_t r = ((P[p] >> 46) & 0x3FFFFull) / a;
        uint64_t g = ((P[p] >> 28) & 0x3FFFFull) / a;
        uint64_t b = ((P[p] >> 10) & 0x3FFFFull) / a;
        out[p] = (uint32_t)(r & 0xFFu) | (uint32_t)(g & 0xFFu) << 8 |
                 (uint32_t)(b & 0xFFu) << 16 | 0xFF000000u;
    }
}

/* ---- depth output of the resolve (Sec. 3.1, closing paragraph) --------- */

/* The stored depth is the linear depth w itself.  For hybrid rendering the
 * resolve may also emit a conventional depth value: for a perspective
 * projection that value is an affine function of 1/w, a + b * (1/w) (window
 * depth in [0,1] with a = f/(f-n), b = -f*n/(f-n); reverse-z with
 * a = -n/(f-n), b = f*n/(f-n)).  One correctly rounded reciprocal, then one
 * product and one sum, each rounded once.  mode 0 = linear, 1 = a + b/w.
 * A pixel nothing landed on gets `empty`. */
static float depth_value(float w, int mode, float a, float b)
{
    if (mode == 0)
        return w;
    float rw = 1.0f / w;
    float t = b * rw;
    return a + t;
}

void oracle_resolve_depth_basic(const uint64_t *fb, uint32_t W, uint32_t H, int mode,
                                float a, float b, float empty, float *out)
{
    for (uint64_t p = 0; p < (uint64_t)W * H; ++p) {
        if (fb[p] == 0xFFFFFFFFFFFFFFFFull) {
            out[p] = empty;
            continue;
        }
        out[p] = depth_value(u2f((uint32_t)(fb[p] >> 32)), mode, a, b);
    }
}

/* HQ: the depth of a pixel is the closest depth of its depth pass. */
void oracle_resolve_depth_hq(const uint32_t *D, uint32_t W, uint32_t H, int mode,
                             float a, float b, float empty, float *out)
{
    for (uint64_t p = 0; p < (uint64_t)W * H; ++p)
        out[p] = D[p] == 0xFFFFFFFFu ? empty : depth_value(u2f(D[p]), mode, a, b);
}

/* ---- vertex orders (Sec. 4, Sec. 5) ------------------------------------ */

/* SplitMix64: the k-th output (k = 0, 1, ...) of the generator seeded with
 * `seed` (state advanced by the golden-gamma increment, then mixed). */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Exact per-axis minimum and maximum of the positions. */
void oracle_bbox(const struct opoint *pts, uint64_t n, float *lo, float *hi)
{
    lo[0] = lo[1] = lo[2] = 0.0f;
    hi[0] = hi[1] = hi[2] = 0.0f;
    if (n == 0)
        return;
    lo[0] = hi[0] = pts[0].x;
    lo[1] = hi[1] = pts[0].y;
    lo[2] = hi[2] = pts[0].z;
    for (uint64_t i = 1; i < n; ++i) {
        const float v[3] = {pts[i].x, pts[i].y, pts[i].z};
        for (int a = 0; a < 3; ++a) {
            if (v[a] < lo[a]) lo[a] = v[a];
            if (v[a] > hi[a]) hi[a] = v[a];
        }
    }
}

/* 21-bit cell index of one coordinate inside the cube [lo, lo + size]. */
static uint32_t quantize21(float v, float lo, float size)
{
    if (size == 0.0f)
        return 0;
    float t = ((v - lo) / size) * 2097152.0f;
    uint32_t q = (uint32_t)t;
    return q > 2097151u ? 2097151u : q;
}

/* Interleaves three 21-bit cell indices into a 63-bit Morton code. */
uint64_t oracle_morton_interleave(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint64_t code = 0;
    for (int i = 0; i < 21; ++i) {
        code |= (uint64_t)((qx >> i) & 1u) << (3 * i);
        code |= (uint64_t)((qy >> i) & 1u) << (3 * i + 1);
        code |= (uint64_t)((qz >> i) & 1u) << (3 * i + 2);
    }
    return code;
}

/* Morton codes of all points over the cubic bounding box of the cloud. */
void oracle_morton_codes(const struct opoint *pts, uint64_t n, uint64_t *codes)
{
    float lo[3], hi[3];
    oracle_bbox(pts, n, lo, hi);
    float sx = hi[0] - lo[0], sy = hi[1] - lo[1], sz = hi[2] - lo[2];
    float size = sx;
    if (sy > size) size = sy;
    if (sz > size) size = sz;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t qx = quantize21(pts[i].x, lo[0], size);
        uint32_t qy = quantize21(pts[i].y, lo[1], size);
        uint32_t qz = quantize21(pts[i].z, lo[2], size);
        codes[i] = oracle_morton_interleave(qx, qy, qz);
    }
}

struct keyed { uint64_t key; uint64_t idx; };

static int cmp_keyed(const void *a, const void *b)
{
    const struct keyed *x = (const struct keyed *)a, *y = (const struct keyed *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

/* order: 0 = Morton, 1 = Morton then batches shuffled, 2 = shuffled points.
 * perm[j] = input index of the j-th output point.  Returns 0, or -1 on an
 * unknown order, a zero batch size or an allocation failure. */
int oracle_reorder(const struct opoint *pts, uint64_t n, int order, uint32_t batch,
                   uint64_t seed, uint32_t *perm)
{
    if (order < 0 || order > 2 || (order == 1 && batch == 0))
        return -1;
    if (n == 0)
        return 0;
    struct keyed *kv = (struct keyed *)malloc(n * sizeof(struct keyed));
    if (!kv)
        return -1;
    if (order == 2) {
        /* Shuffled: a random value per point, then sort by it (Sec. 5). */
        for (uint64_t i = 0; i < n; ++i) {
            kv[i].key = oracle_splitmix64(seed, i);
            kv[i].idx = i;
        }
        qsort(kv, n, sizeof(struct keyed), cmp_keyed);
        for (uint64_t j = 0; j < n; ++j)
            perm[j] = (uint32_t)kv[j].idx;
        free(kv);
        return 0;
    }
    /* Morton: stable sort by code (equal codes keep input order). */
    uint64_t *codes = (uint64_t *)malloc(n * sizeof(uint64_t));
    if (!codes) {
        free(kv);
        return -1;
    }
    oracle_morton_codes(pts, n, codes);
    for (uint64_t i = 0; i < n; ++i) {
        kv[i].key = codes[i];
        kv[i].idx = i;
    }
    free(codes);
    qsort(kv, n, sizeof(struct keyed), cmp_keyed);
    if (order == 0) {
        for (uint64_t j = 0; j < n; ++j)
            perm[j] = (uint32_t)kv[j].idx;
        free(kv);
        return 0;
    }
    /* Shuffled Morton (Sec. 4): cut the Morton sequence into batches of
     * `batch` points (the last may be shorter), move the batches to random
     * positions, keep the order inside each batch. */
    uint64_t nb = (n + batch - 1) / batch;
    struct keyed *bk = (struct keyed *)malloc(nb * sizeof(struct keyed));
    if (!bk) {
        free(kv);
        return -1;
    }
    for (uint64_t b = 0; b < nb; ++b) {
        bk[b].key = oracle_splitmix64(seed, b);
        bk[b].idx = b;
    }
    qsort(bk, nb, sizeof(struct keyed), cmp_keyed);
    uint64_t j = 0;
    for (uint64_t r = 0; r < nb; ++r) {
        uint64_t b = bk[r].idx;
        uint64_t s = b * batch, e = s + batch < n ? s + batch : n;
        for (uint64_t t = s; t < e; ++t)
            perm[j++] = (uint32_t)kv[t].idx;
    }
    free(bk);
    free(kv);
    return 0;
}
