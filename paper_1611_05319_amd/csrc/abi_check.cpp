// Host-side check of the C ABI (include/guidefill.h) for sanitizer builds:
// tests/test_sanitizers.py builds the library with AddressSanitizer and
// UndefinedBehaviorSanitizer on its host code and runs this program on the
// CPU.  It drives the validation, workspace-layout and
// tile-geometry code of guidefill.hip through every entry point, with
// arguments that are rejected before any kernel launch (so it is safe with
// or without a device), and checks the documented results.  Exit status 0
// when every check holds.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "guidefill.h"

static int failures = 0;

#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static gf_params defaults() {
    gf_params p;
    memset(&p, 0, sizeof p);
    p.eps = 3.0;
    p.mu = 50.0;
    p.c = -1.0;
    p.ghost = 1;
    p.tracking = 1;
    p.c2 = -1.0;
    return p;
}

static gf_status fill(const gf_params &p, int B, int H, int W, int C, int dt, void *ws,
                      size_t ws_bytes, void *ptr) {
    return gf_fill_batched(ptr, ptr, B, H, W, C, (gf_dtype)dt, (const uint8_t *)ptr,
                           (const float *)ptr, &p, (int32_t *)ptr, (int32_t *)ptr, nullptr, nullptr,
                           nullptr, 0, ws, ws_bytes, nullptr);
}

int main() {
    void *fake = reinterpret_cast<void *>(uintptr_t(1) << 20);
    CHECK(gf_version() == 2);
    for (int s = -4; s <= 1; ++s) CHECK(gf_status_string((gf_status)s) != nullptr);
    CHECK(gf_last_error() != nullptr);

    gf_params p = defaults();
    // workspace sizes: both engines, several shapes, binary32 and binary16
    for (int engine = 0; engine < 2; ++engine)
        for (int dt = 0; dt < 2; ++dt)
            for (int B = 1; B <= 3; ++B) {
                p.engine = engine;
                const size_t n = gf_workspace_size(B, 37, 53, 3, (gf_dtype)dt, &p);
                CHECK(n > 0 && n % 256 == 0);
                // the front lists grow with every frame; the per-tile words in 256-byte steps
                const size_t n2 = gf_workspace_size(B + 1, 37, 53, 3, (gf_dtype)dt, &p);
                CHECK(engine == GF_ENGINE_FRONT ? n2 > n : n2 >= n);
            }
    p = defaults();
    CHECK(gf_workspace_size(0, 10, 10, 3, GF_F32, &p) == 0);
    CHECK(gf_workspace_size(1, 10, 10, 3, GF_F32, nullptr) == 0);
    CHECK(gf_backward_workspace_size(2, 9, 11, 3, GF_F32, &p) >= 4096 + 2 * 9 * 11 * 4);
    CHECK(gf_backward_workspace_size(0, 9, 11, 3, GF_F32, &p) == 0);

    // tile geometry: defaults fit; a halo wider than the tile does not
    int32_t g6[6];
    for (int eps10 = 10; eps10 <= 90; eps10 += 7) {
        p = defaults();
        p.eps = eps10 / 10.0;
        const gf_status st = gf_tile_geometry(1080, 1920, 3, GF_F32, &p, g6);
        if (st == GF_OK) CHECK(g6[3] <= g6[0] && g6[3] <= g6[1] && g6[2] >= 1);
    }
    p = defaults();
    p.tile_w = 8;
    p.tile_h = 8;
    p.pass_shells = 4;
    CHECK(gf_tile_geometry(64, 64, 3, GF_F32, &p, g6) == GF_EINVAL);
    CHECK(gf_tile_geometry(64, 64, 3, GF_F32, nullptr, g6) == GF_EINVAL);

    // argument validation of the fill (every case is rejected before a launch)
    p = defaults();
    CHECK(fill(p, 0, 8, 8, 3, 0, fake, 1 << 20, fake) == GF_EINVAL);
    CHECK(fill(p, 1, 8, 8, 5, 0, fake, 1 << 20, fake) == GF_EINVAL);
    CHECK(fill(p, 1, 8, 8, 3, 7, fake, 1 << 20, fake) == GF_EINVAL);
    CHECK(fill(p, 1, 8, 8, 3, 0, fake, 16, fake) == GF_EINVAL);
    CHECK(fill(p, 1, 8, 8, 3, 0, (char *)fake + 8, 1 << 20, fake) == GF_EINVAL);
    CHECK(fill(p, 1, 8, 8, 3, 0, fake, 1 << 20, nullptr) == GF_EINVAL);
    CHECK(fill(p, 1 << 12, 1 << 10, 1 << 10, 3, 0, fake, (size_t)1 << 62, fake) == GF_EUNSUPPORTED);
    const double bad_eps[] = {0.0, 0.5, 9.5};
    for (double e : bad_eps) {
        p = defaults();
        p.eps = e;
        CHECK(fill(p, 1, 8, 8, 3, 0, fake, 1 << 20, fake) == GF_EINVAL);
    }
    p = defaults();
    p.mu = -1.0;
    CHECK(fill(p, 1, 8, 8, 3, 0, fake, 1 << 20, fake) == GF_EINVAL);
    p = defaults();
    p.group = 2;
    CHECK(fill(p, 1, 8, 8, 3, 0, fake, 1 << 20, fake) == GF_EINVAL);
    p = defaults();
    p.group = 8;
    p.eps = 5.0;  // 80 offsets do not fit 8 lanes
    CHECK(fill(p, 1, 8, 8, 3, 0, fake, 1 << 20, fake) == GF_EUNSUPPORTED);
    p = defaults();
    p.engine = GF_ENGINE_FRONT;
    p.tile_threads = 256;
    CHECK(fill(p, 1, 8, 8, 3, 0, fake, 1 << 20, fake) == GF_EINVAL);
    p = defaults();
    p.tile_threads = 640;
    CHECK(fill(p, 1, 8, 8, 3, 0, fake, 1 << 20, fake) == GF_EINVAL);
    p = defaults();
    p.c2 = 0.0;  // the data term's phase switch needs one frame
    CHECK(fill(p, 2, 8, 8, 3, 0, fake, 1 << 20, fake) == GF_EUNSUPPORTED);
    p.c2 = NAN;
    CHECK(fill(p, 1, 8, 8, 3, 0, fake, 1 << 20, fake) == GF_EINVAL);
    p = defaults();
    CHECK(gf_fill(fake, fake, 8, 8, 3, GF_F32, (const uint8_t *)fake, (const float *)fake, &p,
                  (int32_t *)fake, (int32_t *)fake, fake, 16, nullptr) == GF_EINVAL);

    // the no-allocation entry point: requests beyond its scratch
    p = defaults();
    p.engine = GF_ENGINE_FRONT;
    CHECK(gf_fill_batched_noalloc(fake, fake, 2, 1080, 1920, 3, GF_F32, (const uint8_t *)fake,
                                  (const float *)fake, &p, (int32_t *)fake, (int32_t *)fake, nullptr,
                                  nullptr, nullptr, 0, nullptr) == GF_EINVAL);
    CHECK(strstr(gf_last_error(), "scratch") != nullptr);

    // the adjoint
    p = defaults();
    const size_t nb = gf_backward_workspace_size(1, 8, 8, 3, GF_F32, &p);
    const float *fg = (const float *)fake;
    CHECK(gf_fill_backward(fg, fake, 1, 8, 8, 3, GF_F32, nullptr, fg, nullptr, 2, &p, (float *)fake,
                           (float *)fake, fake, nb, nullptr) == GF_EINVAL);
    CHECK(gf_fill_backward(fg, fake, 1, 8, 8, 3, GF_F32, nullptr, fg, (const int32_t *)fake, -2, &p,
                           (float *)fake, (float *)fake, fake, nb, nullptr) == GF_EINVAL);
    CHECK(gf_fill_backward(fg, fake, 1, 8, 8, 3, GF_F32, nullptr, fg, (const int32_t *)fake, 65, &p,
                           (float *)fake, (float *)fake, fake, nb, nullptr) == GF_EINVAL);
    CHECK(gf_fill_backward(fg, fake, 1, 8, 8, 3, GF_F32, nullptr, fg, (const int32_t *)fake, 2, &p,
                           (float *)fake, (float *)fake, fake, nb - 256, nullptr) == GF_EINVAL);

    // the comparison fill
    p = defaults();
    p.ghost = 0;
    const size_t nc = gf_coherence_workspace_size(2, 40, 50, 3, GF_F32, &p);
    CHECK(nc > 0 && nc % 256 == 0);
    CHECK(gf_coherence_workspace_size(0, 40, 50, 3, GF_F32, &p) == 0);
    int32_t *fi = (int32_t *)fake;
    CHECK(gf_fill_coherence(fake, fake, 2, 40, 50, 3, GF_F32, (const uint8_t *)fake, &p, 0.0, 4.0,
                            1e-5, fi, fi, nullptr, fake, nc, nullptr) == GF_EINVAL);
    CHECK(gf_fill_coherence(fake, fake, 2, 40, 50, 3, GF_F32, (const uint8_t *)fake, &p, 2.0, 17.0,
                            1e-5, fi, fi, nullptr, fake, nc, nullptr) == GF_EUNSUPPORTED);
    CHECK(gf_fill_coherence(fake, fake, 2, 40, 50, 3, GF_F32, (const uint8_t *)fake, &p, 2.0, 4.0,
                            1e-5, fi, fi, nullptr, fake, nc - 256, nullptr) == GF_EINVAL);
    p.c2 = 0.5;
    CHECK(gf_fill_coherence(fake, fake, 1, 40, 50, 3, GF_F32, (const uint8_t *)fake, &p, 2.0, 4.0,
                            1e-5, fi, fi, nullptr, fake, nc, nullptr) == GF_EUNSUPPORTED);

    // the guide field
    const uint8_t *fl = (const uint8_t *)fake;
    const float *fs = (const float *)fake;
    const int32_t *fo = (const int32_t *)fake;
    CHECK(gf_guide_field(0, 8, 8, fl, fs, fo, 3.0, 9.0, (float *)fake, nullptr) == GF_EINVAL);
    CHECK(gf_guide_field(1, 8, 8, fl, fs, fo, 0.0, 9.0, (float *)fake, nullptr) == GF_EINVAL);
    CHECK(gf_guide_field(1, 8, 8, fl, fs, fo, 3.0, -1.0, (float *)fake, nullptr) == GF_EINVAL);
    CHECK(gf_guide_field(1, 8, 8, fl, fs, nullptr, 3.0, 9.0, (float *)fake, nullptr) == GF_EINVAL);

    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("abi sanitize check ok\n");
    return 0;
}
