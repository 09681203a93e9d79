/*
 * Host-side memory and undefined-behaviour check of the CPU oracle (test
 * infrastructure): built together with oracle/pcr_oracle.c under gcc's
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitize_cpu.py, it drives every oracle entry point over
 * ordinary, empty, one-pixel and hostile inputs (NaN, infinities, huge and
 * subnormal coordinates, points behind the camera), and the three vertex
 * orders over empty, single, degenerate and ragged clouds.  It checks no
 * rendering result (the pins and parity tests do); any sanitizer report ends
 * it with a non-zero status.  Inputs come from a xorshift generator of its
 * own; it holds none of the method's arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

struct opoint {
    float x, y, z;
    uint32_t rgba;
};

int oracle_fp_env_ok(void);
void oracle_project_all(const struct opoint *pts, uint64_t n, const float *m, uint32_t W, uint32_t H,
                        uint32_t *pid, uint32_t *dbits);
void oracle_clear_basic(uint64_t *fb, uint32_t W, uint32_t H);
void oracle_render_basic(const struct opoint *pts, uint64_t n, const float *m, uint32_t W, uint32_t H,
                         uint64_t *fb);
void oracle_resolve_basic(const uint64_t *fb, uint32_t W, uint32_t H, uint32_t *out);
void oracle_clear_hq(uint32_t *D, uint64_t *RG, uint64_t *BA, uint32_t W, uint32_t H);
void oracle_render_hq(const struct opoint *pts, uint64_t n, const float *m, uint32_t W, uint32_t H,
                      uint32_t *D, uint64_t *RG, uint64_t *BA);
void oracle_resolve_hq(const uint64_t *RG, const uint64_t *BA, uint32_t W, uint32_t H, uint32_t *out);
void oracle_render_hq_packed_color(const struct opoint *pts, uint64_t n, const float *m, uint32_t W,
                                   uint32_t H, const uint32_t *D, uint64_t *P);
void oracle_resolve_hq_packed(const uint64_t *P, uint32_t W, uint32_t H, uint32_t *out);
void oracle_resolve_depth_basic(const uint64_t *fb, uint32_t W, uint32_t H, int mode, float a, float b,
                                float empty, float *out);
void oracle_resolve_depth_hq(const uint32_t *D, uint32_t W, uint32_t H, int mode, float a, float b,
                             float empty, float *out);
void oracle_morton_codes(const struct opoint *pts, uint64_t n, uint64_t *codes);
int oracle_reorder(const struct opoint *pts, uint64_t n, int order, uint32_t batch, uint64_t seed,
                   uint32_t *perm);

static uint64_t rng = 0x9E3779B97F4A7C15ull;

static uint32_t next32(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (uint32_t)(rng >> 16);
}

static float unit(void) { return (float)(next32() & 0xFFFFFF) / 16777216.0f; }

/* Points in [-1, 1)^3 with random colours; `hostile` mixes in special floats. */
static void make_points(struct opoint *p, uint64_t n, int hostile) {
    static const float special[] = {NAN, INFINITY, -INFINITY, 3.0e38f, -3.0e38f, 1.0e-40f, -1.0e-40f, 0.0f, -0.0f};
    for (uint64_t i = 0; i < n; ++i) {
        p[i].x = 2.0f * unit() - 1.0f;
        p[i].y = 2.0f * unit() - 1.0f;
        p[i].z = 2.0f * unit() - 1.0f;
        p[i].rgba = next32();
        if (hostile && i % 7 == 0) {
            float *c = (i % 3 == 0) ? &p[i].x : (i % 3 == 1) ? &p[i].y : &p[i].z;
            *c = special[next32() % (sizeof(special) / sizeof(special[0]))];
        }
    }
}

static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static void frame(const struct opoint *p, uint64_t n, const float *m, uint32_t W, uint32_t H) {
    const uint64_t px = (uint64_t)W * H;
    uint32_t *pid = xcalloc(n, 4), *db = xcalloc(n, 4), *out = xcalloc(px, 4), *D = xcalloc(px, 4);
    uint64_t *fb = xcalloc(px, 8), *RG = xcalloc(px, 8), *BA = xcalloc(px, 8), *P = xcalloc(px, 8);
    float *depth = xcalloc(px, 4);
    oracle_project_all(p, n, m, W, H, pid, db);
    oracle_clear_basic(fb, W, H);
    oracle_render_basic(p, n, m, W, H, fb);
    oracle_resolve_basic(fb, W, H, out);
    oracle_resolve_depth_basic(fb, W, H, 0, 0.0f, 0.0f, INFINITY, depth);
    oracle_resolve_depth_basic(fb, W, H, 1, 1.001f, -0.1001f, 1.0f, depth);
    oracle_clear_hq(D, RG, BA, W, H);
    oracle_render_hq(p, n, m, W, H, D, RG, BA);
    oracle_resolve_hq(RG, BA, W, H, out);
    oracle_resolve_depth_hq(D, W, H, 1, 1.001f, -0.1001f, 1.0f, depth);
    oracle_render_hq_packed_color(p, n, m, W, H, D, P);
    oracle_resolve_hq_packed(P, W, H, out);
    free(pid), free(db), free(out), free(D), free(fb), free(RG), free(BA), free(P), free(depth);
}

static void orders(const struct opoint *p, uint64_t n) {
    uint32_t *perm = xcalloc(n, 4);
    uint64_t *codes = xcalloc(n, 8);
    static const uint32_t batches[] = {1, 2, 128, 1000003};
    oracle_morton_codes(p, n, codes);
    for (int order = 0; order < 3; ++order)
        for (size_t b = 0; b < sizeof(batches) / sizeof(batches[0]); ++b)
            if (oracle_reorder(p, n, order, batches[b], 3 + b, perm) != 0) {
                fprintf(stderr, "reorder failed: order %d batch %u n %llu\n", order, batches[b],
                        (unsigned long long)n);
                exit(3);
            }
    if (oracle_reorder(p, n, 1, 0, 1, perm) != -1 || oracle_reorder(p, n, 3, 1, 1, perm) != -1) {
        fprintf(stderr, "reorder accepted an invalid argument\n");
        exit(3);
    }
    free(perm), free(codes);
}

int main(void) {
    if (!oracle_fp_env_ok()) {
        fprintf(stderr, "flush-to-zero is set\n");
        return 4;
    }
    /* A perspective-like matrix (w = z + 2), one that puts every point behind
     * the camera, and one of zeros. */
    const float persp[16] = {1.2f, 0.1f, 0, 0.05f, -0.1f, 1.3f, 0, -0.02f, 0, 0, 1, 0, 0.01f, 0, 1, 2};
    const float behind[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, -1};
    const float zeros[16] = {0};
    const float *mats[] = {persp, behind, zeros};
    const uint32_t sizes[][2] = {{64, 48}, {1, 1}, {1000, 3}, {3, 700}};
    const uint64_t counts[] = {0, 1, 2, 257, 20000};
    for (size_t c = 0; c < sizeof(counts) / sizeof(counts[0]); ++c) {
        for (int hostile = 0; hostile < 2; ++hostile) {
            uint64_t n = counts[c];
            struct opoint *p = xcalloc(n, sizeof(struct opoint));
            make_points(p, n, hostile);
            for (size_t mi = 0; mi < 3; ++mi)
                for (size_t s = 0; s < sizeof(sizes) / sizeof(sizes[0]); ++s)
                    frame(p, n, mats[mi], sizes[s][0], sizes[s][1]);
            if (!hostile)
                orders(p, n);  /* the vertex orders take finite positions */
            free(p);
        }
    }
    /* Degenerate clouds for the orders: all points equal (an empty box), and
     * points equal in two coordinates (a flat box). */
    struct opoint q[300];
    for (int i = 0; i < 300; ++i) {
        q[i].x = 0.5f;
        q[i].y = 0.25f;
        q[i].z = 0.125f;
        q[i].rgba = (uint32_t)i;
    }
    orders(q, 300);
    for (int i = 0; i < 300; ++i)
        q[i].z = (float)i;
    orders(q, 300);
    puts("oracle sanitizer run: ok");
    return 0;
}
