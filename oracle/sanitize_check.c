/*
 * Sanitizer driver for the FP64 oracle (gf_oracle.c).  TEST INFRASTRUCTURE
 * ONLY: built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py and run on the CPU.
 *
 * Runs the forward fill (Algorithm 1 in every mode the oracle has: rotated
 * and lattice ball, onion and smart order, binary64/32/16 storage, resumed
 * fills) and its adjoint on seeded random tiny problems, including the
 * degenerate shapes (1 x 1, single rows and columns, all-hole and no-hole
 * frames, bystander-enclosed holes), and checks the invariants that need no
 * second implementation: return codes, the shell map's codes, the fill
 * counts against the map, and that unfilled pixels keep their input.
 * Exit status 0 when every check holds; the sanitizers abort on any memory
 * or undefined-behaviour error.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int gfo_offsets(double eps, int *on, int *om, int cap);
int gfo_fill(int B, int H, int W, int C, const double *img_in, const uint8_t *label,
             const double *guide, double eps, double mu, double c, double c2, int ghost,
             int max_shells, int storage, double *img_out, int32_t *shell_out, int64_t *stats,
             int64_t *front_hist, int64_t *fill_hist, int hist_cap, int nthreads);
int gfo_adjoint(int B, int H, int W, int C, const uint8_t *label, const double *guide,
                double eps, double mu, int ghost, const double *u_out, const int32_t *shell,
                const double *grad_out, double *grad_in, double *grad_g);

int gfo_mod_structure_tensor(int H, int W, int C, const double *u, const uint8_t *known,
                             const uint8_t *want, double sigma, double rho, double *J);
int gfo_coherence_guide(int B, int H, int W, int C, const double *u, const uint8_t *label,
                        double sigma, double rho, double Lambda, double *guide);
int gfo_guide_field(int B, int H, int W, const uint8_t *label, const double *seg,
                    const int32_t *seg_off, double eta, double cutoff, double *guide);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static uint64_t next_u64(void)
{
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double uniform(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

static int failures = 0;

#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            fprintf(stderr, "check failed: " __VA_ARGS__); \
            fprintf(stderr, "\n");                         \
            ++failures;                                    \
        }                                                  \
    } while (0)

static void run_case(int B, int H, int W, int C, double p_hole, double p_bys, double eps, double mu,
                     double c, int ghost, int storage, int max_shells, double c2)
{
    const size_t np = (size_t)B * H * W;
    double *img = malloc(np * C * sizeof(double));
    double *out = malloc(np * C * sizeof(double));
    double *guide = malloc(np * 2 * sizeof(double));
    uint8_t *label = malloc(np);
    int32_t *shell = malloc(np * sizeof(int32_t));
    int64_t *stats = malloc((size_t)B * 8 * sizeof(int64_t));
    const int hist_cap = 64;
    int64_t *front = malloc((size_t)B * hist_cap * sizeof(int64_t));
    int64_t *fills = malloc((size_t)B * hist_cap * sizeof(int64_t));
    double *gout = malloc(np * C * sizeof(double));
    double *gin = malloc(np * C * sizeof(double));
    double *gg = malloc(np * 2 * sizeof(double));
    for (size_t i = 0; i < np; ++i) {
        const double r = uniform();
        label[i] = r < p_hole ? 1 : (r < p_hole + p_bys ? 2 : 0);
        const double th = 6.283185307179586 * uniform();
        const int zero = uniform() < 0.05;  /* some g = 0 pixels: lattice ball */
        guide[2 * i] = zero ? 0.0 : cos(th) * (0.5 + uniform());
        guide[2 * i + 1] = zero ? 0.0 : sin(th) * (0.5 + uniform());
        for (int ch = 0; ch < C; ++ch) {
            img[i * C + ch] = uniform();
            gout[i * C + ch] = uniform() - 0.5;
        }
    }
    int rc = gfo_fill(B, H, W, C, img, label, guide, eps, mu, c, c2, ghost, max_shells, storage,
                      out, shell, stats, front, fills, hist_cap, 1);
    CHECK(rc == 0, "gfo_fill returned %d (%dx%dx%dx%d)", rc, B, H, W, C);
    for (int b = 0; b < B && rc == 0; ++b) {
        long long filled = 0, unfilled = 0;
        for (size_t i = (size_t)b * H * W; i < (size_t)(b + 1) * H * W; ++i) {
            const int32_t s = shell[i];
            if (label[i] == 0) CHECK(s == -1, "readable pixel with shell %d", s);
            if (label[i] == 2) CHECK(s == -2, "bystander pixel with shell %d", s);
            if (label[i] == 1) {
                CHECK(s == -3 || (s >= 0 && s < stats[b * 8]), "hole pixel with shell %d", s);
                filled += s >= 0;
                unfilled += s == -3;
            }
            if (s < 0)
                for (int ch = 0; ch < C; ++ch)
                    CHECK(out[i * C + ch] == img[i * C + ch] || storage != 0,
                          "unfilled pixel changed");
        }
        CHECK(filled == stats[b * 8 + 1], "filled count %lld vs %lld", filled, (long long)stats[b * 8 + 1]);
        CHECK(unfilled == stats[b * 8 + 2], "unfilled count");
    }
    if (rc == 0 && storage == 0) {
        rc = gfo_adjoint(B, H, W, C, label, guide, eps, mu, ghost, out, shell, gout, gin, gg);
        CHECK(rc == 0, "gfo_adjoint returned %d", rc);
        for (size_t i = 0; i < np && rc == 0; ++i) {
            if (shell[i] >= 0)
                for (int ch = 0; ch < C; ++ch) CHECK(gin[i * C + ch] == 0.0, "filled pixel gradient");
            else
                CHECK(gg[2 * i] == 0.0 && gg[2 * i + 1] == 0.0, "guide gradient off the fill");
            for (int ch = 0; ch < C; ++ch) CHECK(isfinite(gin[i * C + ch]), "gradient not finite");
        }
    }
    free(img); free(out); free(guide); free(label); free(shell); free(stats); free(front);
    free(fills); free(gout); free(gin); free(gg);
}

int main(void)
{
    int on[256], om[256];
    CHECK(gfo_offsets(3.0, on, om, 256) == 28, "28 offsets for eps = 3");
    CHECK(gfo_offsets(5.0, on, om, 256) == 80, "80 offsets for eps = 5");
    const double eps_list[] = {1.0, 2.0, 3.0, 3.6, 5.0};
    for (int e = 0; e < 5; ++e)
        for (int ghost = 0; ghost < 2; ++ghost)
            for (int storage = 0; storage < 3; ++storage) {
                const double eps = eps_list[e];
                const double mu = 10.0 + 40.0 * uniform();
                run_case(2, 17, 23, 3, 0.4, 0.1, eps, mu, -1.0, ghost, storage, 0, -1.0);
                run_case(1, 12, 9, 1, 0.5, 0.0, eps, mu, 0.05, ghost, storage, 0, -1.0);
                run_case(1, 20, 20, 4, 0.6, 0.05, eps, mu, 0.3, ghost, storage, 2, -1.0);
                run_case(2, 19, 21, 3, 0.5, 0.05, eps, mu, 0.05, ghost, storage, 0, 0.0);
                run_case(1, 15, 17, 2, 0.5, 0.05, eps, mu, -1.0, ghost, storage, 0, 0.7);
            }
    /* degenerate shapes: single pixel, single row and column, all hole, no hole */
    run_case(1, 1, 1, 3, 0.5, 0.0, 3.0, 50.0, -1.0, 1, 0, 0, -1.0);
    run_case(1, 1, 31, 3, 0.5, 0.1, 3.0, 50.0, -1.0, 1, 0, 0, 0.0);
    run_case(1, 29, 1, 2, 0.5, 0.1, 3.0, 50.0, -1.0, 0, 0, 0, -1.0);
    run_case(1, 8, 8, 3, 1.0, 0.0, 3.0, 50.0, -1.0, 1, 0, 0, 0.0);
    run_case(3, 8, 8, 3, 0.0, 0.2, 3.0, 50.0, -1.0, 1, 0, 0, -1.0);
    /* a hole enclosed by bystanders stalls */
    run_case(1, 16, 16, 3, 0.3, 0.6, 3.0, 50.0, -1.0, 1, 0, 0, 0.0);
    /* the modified structure tensor, the comparison mode's guide and the
       guide field, on frames of several shapes including 1 x n and n x 1 */
    const int shapes[][3] = {{1, 1, 1}, {1, 17, 3}, {9, 1, 2}, {13, 19, 3}, {24, 20, 4}};
    for (int e = 0; e < 5; ++e) {
        const int H = shapes[e][0], W = shapes[e][1], C = shapes[e][2];
        const size_t HW = (size_t)H * W;
        double *u = (double *)malloc(2 * HW * C * sizeof(double));
        uint8_t *lab = (uint8_t *)malloc(2 * HW);
        double *J = (double *)malloc(HW * 3 * sizeof(double));
        double *g = (double *)malloc(2 * HW * 2 * sizeof(double));
        for (size_t i = 0; i < 2 * HW * C; ++i) u[i] = uniform();
        for (size_t i = 0; i < 2 * HW; ++i) {
            const double r = uniform();
            lab[i] = (uint8_t)(r < 0.4 ? 1 : (r < 0.5 ? 2 : 0));
        }
        uint8_t *known = (uint8_t *)malloc(HW);
        for (size_t i = 0; i < HW; ++i) known[i] = lab[i] == 0;
        CHECK(gfo_mod_structure_tensor(H, W, C, u, known, lab, 2.0, 4.0, J) == 0, "tensor %dx%d", H, W);
        CHECK(gfo_mod_structure_tensor(H, W, C, u, known, NULL, 0.3, 1.0, J) == 0, "tensor %dx%d", H, W);
        CHECK(gfo_coherence_guide(2, H, W, C, u, lab, 1.5, 3.0, 1e-5, g) == 0, "coherence %dx%d", H, W);
        const double seg[12] = {0.0, 0.0, W - 1.0, H - 1.0, 0.6, 0.8, 2.0, 2.0, 2.0, 2.0, 1.0, 0.0};
        const int32_t off[3] = {0, 2, 2};
        CHECK(gfo_guide_field(2, H, W, lab, seg, off, 3.0, 9.0, g) == 0, "guide field %dx%d", H, W);
        free(u); free(lab); free(J); free(g); free(known);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitize check ok\n");
    return 0;
}
