/*
 * Plain FP64 CPU reference of the Guidefill shell fill (Hocking, MacKenzie and
 * Schoenlieb, "Guidefill: GPU accelerated, artist guided geometric inpainting
 * for 3D conversion of film", arXiv 1611.05319).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP path is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it; the product never calls it.  It shares no code with
 * the HIP path.
 *
 * What it computes, step by step (pixel units, h = 1, x = column, y = row):
 *
 *  - Algorithm 1 ("Shell based geometric inpainting", Sec. 3): for k = 0, 1, ...
 *    every pixel of the active boundary of D^(k) that is ready gets the
 *    normalised weighted average of the readable points of its neighbourhood;
 *    F = ready pixels; D^(k+1) = D^(k) \ F.  The shells use the state at the
 *    start of shell k only (pixels filled during shell k are not read in
 *    shell k: the sum runs over the complement of D^(k), and F is removed
 *    from D only after the loop over the boundary).  This is done here in two
 *    phases per shell: compute every candidate from the frozen state, then
 *    commit.
 *  - Active boundary (Notation): pixels of D^(k) with at least one readable
 *    pixel among their in-image 8-neighbours.  Readable = not in D^(k) and
 *    not a bystander (Sec. 2.1).
 *  - Neighbourhood: the lattice ball B_eps(x) = {y : 0 < |y - x| <= eps}
 *    (coherence transport), or the rotated ball R(B_eps(x)) with R the
 *    rotation taking (0,1) to g(x)/|g(x)| (Guidefill, Sec. 3.1); if g = 0 the
 *    rotated ball is the lattice ball (remark after Theorem 4.1).
 *  - Ghost pixels (Sec. 3.3, bilinear extension eqn:bilinearDef): u is
 *    extended off the lattice by bilinear interpolation to Omega minus the
 *    continuous sets D^(k) and B, which contain every point within L-infinity
 *    distance < 1 of a pixel of D^(k)_h or B_h.  So a ghost point p is
 *    readable iff p lies in the image rectangle and every pixel with a nonzero
 *    bilinear basis value at p (|q - p|_inf < 1) is readable.
 *  - Weights (eqn:weight): w = exp(-mu^2/(2 eps^2) (g_perp . (y - x))^2) / |y - x|
 *    with g_perp = (-gy, gx) and g the (unnormalised) guide vector.
 *  - Ready (Sec. 3.4): onion order (c < 0) fills every active pixel that has
 *    at least one readable point; smart order uses the confidence
 *    C = sum_readable w / sum_all w (eqn:confidence, denominator over the
 *    whole rotated ball) and ready = 1(C > c) (eqn:ready).  The data-term
 *    variant (eqn:ready2) multiplies ready by 1(|g(x)| > c2) while the guided
 *    region can still advance; the paper reverts to eqn:ready once the region
 *    |g| > 0 has been filled.  Reading: the revert happens at the first shell
 *    in which the data term leaves nothing ready (which is the shell after the
 *    region's last pixel, or an earlier one if the rest of the region cannot
 *    be reached), and that shell is then evaluated with eqn:ready.
 *
 *  - Guide field (Sec. 3.2): g = g_Gamma exp(-d^2 / (2 eta^2)) from the
 *    nearest polyline spline, 0 beyond the cutoff (gfo_guide_field).
 *  - Comparison mode (Sec. 3.2, eqn:modStructureTensor): the modified
 *    structure tensor of the current known set and the coherence direction
 *    it gives (gfo_mod_structure_tensor, gfo_coherence_guide).
 *
 * Readings where the paper is silent (the same list is kept with the design
 * notes): (0,0) is not in the ball; R acts with the unit vector g/|g|; the
 * ball boundary n^2+m^2 <= eps^2 is inclusive; ghost points outside the image
 * are unreadable; a pixel with no readable point waits; when a shell fills
 * nothing while D is not empty the fill stops and the rest is reported
 * unfilled (shell -3, input colour kept); the weights are evaluated relative
 * to the largest readable weight (the quotient is unchanged, FP64 underflow is
 * avoided); the rotated offset is evaluated as ox = n*s + m*c,
 * oy = m*s - n*c with (c, s) = g/|g| in that order with no fused operations,
 * and the bilinear support comes from floor(ox), floor(oy) of the offset
 * alone, so that points landing on lattice lines are decided identically for
 * every pixel.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GFO_MAX_OFFSETS 1024

enum { GFO_OK = 0, GFO_EINVAL = 1, GFO_ELABEL = 2, GFO_ENOMEM = 3 };

/* Shell-map codes. */
enum { S_READABLE = -1, S_BYSTANDER = -2, S_UNFILLED = -3, S_INHOLE = -4 };

/* binary16 round-to-nearest-even of a double (IEEE 754 binary16: 10 fraction
 * bits, exponent bias 15, subnormal spacing 2^-24, largest finite 65504). */
double gfo_round_f16(double v)
{
    if (v != v) return v;
    double a = fabs(v);
    if (a >= 65520.0) return copysign(INFINITY, v);
    if (a == 0.0) return v;
    int e;
    frexp(a, &e);           /* a = f * 2^e, f in [0.5, 1) */
    int ue = e - 11;        /* spacing of binary16 numbers around a */
    if (ue < -24) ue = -24; /* subnormal range */
    double q = ldexp(a, -ue);
    double r = nearbyint(q); /* default rounding mode: to nearest, ties to even */
    return copysign(ldexp(r, ue), v);
}

static double round_storage(double v, int storage)
{
    if (storage == 1) return (double)(float)v;
    if (storage == 2) return gfo_round_f16(v);
    return v;
}

/* The lattice ball I_eps = {(n, m) : 0 < n^2 + m^2 <= eps^2}, m ascending then n. */
int gfo_offsets(double eps, int *on, int *om, int cap)
{
    int R = (int)floor(eps);
    int cnt = 0;
    for (int m = -R; m <= R; ++m)
        for (int n = -R; n <= R; ++n) {
            int r2 = n * n + m * m;
            if (r2 == 0 || (double)r2 > eps * eps) continue;
            if (cnt >= cap) return -1;
            on[cnt] = n;
            om[cnt] = m;
            ++cnt;
        }
    return cnt;
}

typedef struct {
    int H, W, C;
    const uint8_t *label;
    const double *g; /* H*W*2 */
    double eps, mu, c;
    int ghost;
    int T;
    const int *on, *om;
} prob_t;

/* One ghost point of pixel (i, j): offset o, bilinear support and basis values. */
typedef struct {
    double ox, oy;
    int nsx, nsy;        /* support size per axis (1 or 2) */
    int dx, dy;          /* floor of the offset */
    double bx[2], by[2]; /* 1-D basis values of the support columns / rows */
    double t;            /* g_perp . o */
    double rho;          /* |o| */
} ghost_t;

static void ghost_geometry(const prob_t *P, double gx, double gy, int n, int m, ghost_t *G)
{
    if (P->ghost && (gx != 0.0 || gy != 0.0)) {
        double L = sqrt(gx * gx + gy * gy);
        double c = gx / L, s = gy / L;
        double a = (double)n * s, b = (double)m * c;
        double d = (double)m * s, e = (double)n * c;
        G->ox = a + b;
        G->oy = d - e;
    } else {
        G->ox = (double)n;
        G->oy = (double)m;
    }
    double fx = floor(G->ox), fy = floor(G->oy);
    G->dx = (int)fx;
    G->dy = (int)fy;
    if (G->ox == fx) {
        G->nsx = 1;
        G->bx[0] = 1.0;
        G->bx[1] = 0.0;
    } else {
        double f = G->ox - fx;
        G->nsx = 2;
        G->bx[0] = 1.0 - f;
        G->bx[1] = f;
    }
    if (G->oy == fy) {
        G->nsy = 1;
        G->by[0] = 1.0;
        G->by[1] = 0.0;
    } else {
        double f = G->oy - fy;
        G->nsy = 2;
        G->by[0] = 1.0 - f;
        G->by[1] = f;
    }
    G->t = (-gy) * G->ox + gx * G->oy;
    G->rho = sqrt(G->ox * G->ox + G->oy * G->oy);
}

static inline int readable_px(const int32_t *s, int q, int k)
{
    int32_t v = s[q];
    return v == S_READABLE || (v >= 0 && v < k);
}

static int ghost_readable(const prob_t *P, const int32_t *s, int i, int j, const ghost_t *G, int k)
{
    for (int b = 0; b < G->nsy; ++b) {
        int y = j + G->dy + b;
        if (y < 0 || y >= P->H) return 0;
        for (int a = 0; a < G->nsx; ++a) {
            int x = i + G->dx + a;
            if (x < 0 || x >= P->W) return 0;
            if (!readable_px(s, y * P->W + x, k)) return 0;
        }
    }
    return 1;
}

static double ghost_value(const prob_t *P, const double *u, int i, int j, const ghost_t *G, int ch)
{
    double v = 0.0;
    for (int b = 0; b < G->nsy; ++b)
        for (int a = 0; a < G->nsx; ++a) {
            int q = (j + G->dy + b) * P->W + (i + G->dx + a);
            v += G->bx[a] * G->by[b] * u[(size_t)q * P->C + ch];
        }
    return v;
}

static int is_active(const prob_t *P, const int32_t *s, int i, int j, int k)
{
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
            if (!di && !dj) continue;
            int x = i + di, y = j + dj;
            if (x < 0 || x >= P->W || y < 0 || y >= P->H) continue;
            if (readable_px(s, y * P->W + x, k)) return 1;
        }
    return 0;
}

/* Evaluate pixel (i, j) at shell k from the frozen state (u, s).
 * Returns 1 if ready and writes the channel values to val; *conf gets C(x). */
static int eval_pixel(const prob_t *P, const double *u, const int32_t *s, int i, int j, int k,
                      double *val, double *conf, ghost_t *Gbuf, unsigned char *rd)
{
    int p = j * P->W + i;
    double gx = P->g[2 * (size_t)p], gy = P->g[2 * (size_t)p + 1];
    double a = P->mu * P->mu / (2.0 * P->eps * P->eps);
    int any = 0;
    double qmin_r = INFINITY, qmin_all = INFINITY;
    for (int t = 0; t < P->T; ++t) {
        ghost_geometry(P, gx, gy, P->on[t], P->om[t], &Gbuf[t]);
        rd[t] = (unsigned char)ghost_readable(P, s, i, j, &Gbuf[t], k);
        double q = a * Gbuf[t].t * Gbuf[t].t;
        if (q < qmin_all) qmin_all = q;
        if (rd[t]) {
            any = 1;
            if (q < qmin_r) qmin_r = q;
        }
    }
    *conf = 0.0;
    if (!any) return 0;
    int ready = 1;
    if (P->c >= 0.0) {
        double num = 0.0, den = 0.0;
        for (int t = 0; t < P->T; ++t) {
            double w = exp(-(a * Gbuf[t].t * Gbuf[t].t - qmin_all)) / Gbuf[t].rho;
            den += w;
            if (rd[t]) num += w;
        }
        *conf = num / den;
        ready = (*conf > P->c);
    }
    if (!ready) return 0;
    double S = 0.0;
    for (int ch = 0; ch < P->C; ++ch) val[ch] = 0.0;
    for (int t = 0; t < P->T; ++t) {
        if (!rd[t]) continue;
        double w = exp(-(a * Gbuf[t].t * Gbuf[t].t - qmin_r)) / Gbuf[t].rho;
        S += w;
        for (int ch = 0; ch < P->C; ++ch) val[ch] += w * ghost_value(P, u, i, j, &Gbuf[t], ch);
    }
    for (int ch = 0; ch < P->C; ++ch) val[ch] /= S;
    return 1;
}

/*
 * Fill B independent frames.
 *   img_in    B*H*W*C   input colours (hole colours are kept only where a
 *                       pixel is never filled)
 *   label     B*H*W     0 readable, 1 inpaint (D_h), 2 bystander (B_h)
 *   guide     B*H*W*2   (gx, gy), read on the hole only
 *   c         < 0: onion order; >= 0: smart order threshold (eqn:ready)
 *   c2        < 0: no data term; >= 0: eqn:ready2's data term |g(x)| > c2
 *             gates ready until a shell fills nothing; from that shell on
 *             (taken again) eqn:ready alone decides
 *   storage   0: keep FP64; 1: round every stored value to binary32;
 *             2: round to binary16 (inputs and each filled value)
 *   img_out   B*H*W*C, shell_out B*H*W (-1 readable, -2 bystander, k >= 0
 *             filled at shell k, -3 never filled)
 *   stats     B*8 int64: K, filled, unfilled, max active front, n_hole,
 *             smart-order tie count (|C - c| <= 1e-9 max(c, 1e-300)), 0, 0
 *   front_hist, fill_hist (nullable, B*hist_cap int64): per-shell active
 *             front size and number of filled pixels
 * Returns GFO_OK, or GFO_EINVAL / GFO_ELABEL / GFO_ENOMEM.
 */
int gfo_fill(int B, int H, int W, int C, const double *img_in, const uint8_t *label,
             const double *guide, double eps, double mu, double c, double c2, int ghost,
             int max_shells, int storage, double *img_out, int32_t *shell_out, int64_t *stats,
             int64_t *front_hist, int64_t *fill_hist, int hist_cap, int nthreads)
{
    if (B < 0 || H <= 0 || W <= 0 || C <= 0 || !(eps > 0) || !(mu > 0)) return GFO_EINVAL;
    int on[GFO_MAX_OFFSETS], om[GFO_MAX_OFFSETS];
    int T = gfo_offsets(eps, on, om, GFO_MAX_OFFSETS);
    if (T <= 0) return GFO_EINVAL;
    if (nthreads <= 0) nthreads = 1;
    size_t HW = (size_t)H * W;
    int *Dlist = (int *)malloc(HW * sizeof(int));
    int *Dnext = (int *)malloc(HW * sizeof(int));
    double *vals = (double *)malloc(HW * C * sizeof(double));
    unsigned char *ready = (unsigned char *)malloc(HW);
    unsigned char *active = (unsigned char *)malloc(HW);
    double *confs = (double *)malloc(HW * sizeof(double));
    if (!Dlist || !Dnext || !vals || !ready || !active || !confs) {
        free(Dlist); free(Dnext); free(vals); free(ready); free(active); free(confs);
        return GFO_ENOMEM;
    }
    int rc = GFO_OK;
    for (int b = 0; b < B && rc == GFO_OK; ++b) {
        const double *uin = img_in + (size_t)b * HW * C;
        const uint8_t *lab = label + (size_t)b * HW;
        double *u = img_out + (size_t)b * HW * C;
        int32_t *s = shell_out + (size_t)b * HW;
        int64_t *st = stats + (size_t)b * 8;
        prob_t P = {H, W, C, lab, guide + (size_t)b * HW * 2, eps, mu, c, ghost, T, on, om};
        int nD = 0;
        for (size_t q = 0; q < HW; ++q) {
            for (int ch = 0; ch < C; ++ch) u[q * C + ch] = round_storage(uin[q * C + ch], storage);
            if (lab[q] == 0) s[q] = S_READABLE;
            else if (lab[q] == 2) s[q] = S_BYSTANDER;
            else if (lab[q] == 1) { s[q] = S_INHOLE; Dlist[nD++] = (int)q; }
            else { rc = GFO_ELABEL; break; }
        }
        if (rc != GFO_OK) break;
        int64_t n_hole = nD, filled_total = 0, max_front = 0, ties = 0;
        int K = 0;
        int data_phase = c2 >= 0.0; /* eqn:ready2 gates ready until a shell fills nothing */
        for (int k = 0;; ++k) {
            if (nD == 0) break;                           /* D^(k) empty */
            if (max_shells > 0 && k >= max_shells) break; /* caller's stop */
            int64_t n_active = 0, n_ties = 0;
            /* phase 1: evaluate every pixel of D^(k) from the frozen state */
#pragma omp parallel num_threads(nthreads) reduction(+ : n_active, n_ties)
            {
                ghost_t Gbuf[GFO_MAX_OFFSETS];
                unsigned char rd[GFO_MAX_OFFSETS];
#pragma omp for schedule(static)
                for (int e = 0; e < nD; ++e) {
                    int q = Dlist[e];
                    int i = q % W, j = q / W;
                    active[e] = (unsigned char)is_active(&P, s, i, j, k);
                    ready[e] = 0;
                    if (!active[e]) continue;
                    ++n_active;
                    if (data_phase) { /* data term D(x) = |g(x)| of eqn:ready2 */
                        double gx = P.g[2 * (size_t)q], gy = P.g[2 * (size_t)q + 1];
                        if (!(sqrt(gx * gx + gy * gy) > c2)) continue;
                    }
                    double conf;
                    ready[e] = (unsigned char)eval_pixel(&P, u, s, i, j, k, vals + (size_t)e * C,
                                                         &conf, Gbuf, rd);
                    confs[e] = conf;
                    if (c >= 0.0 && fabs(conf - c) <= 1e-9 * fmax(c, 1e-300)) ++n_ties;
                }
            }
            /* phase 2: commit F, D^(k+1) = D^(k) \ F */
            int nF = 0, nN = 0;
            for (int e = 0; e < nD; ++e) {
                int q = Dlist[e];
                if (ready[e]) {
                    for (int ch = 0; ch < C; ++ch)
                        u[(size_t)q * C + ch] = round_storage(vals[(size_t)e * C + ch], storage);
                    s[q] = k;
                    ++nF;
                } else {
                    Dnext[nN++] = q;
                }
            }
            if (front_hist && k < hist_cap) front_hist[(size_t)b * hist_cap + k] = n_active;
            if (fill_hist && k < hist_cap) fill_hist[(size_t)b * hist_cap + k] = nF;
            if (n_active > max_front) max_front = n_active;
            if (nF == 0 && data_phase) {
                /* the data term holds every front pixel back: from this shell on
                   eqn:ready alone decides, and shell k is taken again (nothing
                   was committed, D^(k) is unchanged) */
                data_phase = 0;
                --k;
                continue;
            }
            ties += n_ties;
            if (nF == 0) break; /* nothing ready: the state can no longer change */
            K = k + 1;
            filled_total += nF;
            int *tmp = Dlist; Dlist = Dnext; Dnext = tmp;
            nD = nN;
        }
        for (int e = 0; e < nD; ++e) s[Dlist[e]] = S_UNFILLED;
        st[0] = K;
        st[1] = filled_total;
        st[2] = nD;
        st[3] = max_front;
        st[4] = n_hole;
        st[5] = ties;
        st[6] = 0;
        st[7] = 0;
    }
    free(Dlist); free(Dnext); free(vals); free(ready); free(active); free(confs);
    return rc;
}

/*
 * Reverse-mode derivative of the fill (an extension beyond the paper: the fill is
 * linear in the known colours with coefficients fixed by labels and guide,
 * Algorithm 1).  Given dL/du_out, returns dL/du_in and dL/dg, with the
 * readable sets and ready decisions held fixed (they are piecewise constant in
 * g).  Shells are visited from last to first; pixel x of shell k passes its
 * adjoint to the bilinear support of each readable ghost point with the
 * normalised weight times the basis value, and its guide gets
 *   sum_ch ubar_ch(x) * sum_j lambda_j [ (v_j - u)(d log w_j / dg) + grad v_j . d o_j / dg ].
 * At a lattice line (zero fraction) the support is the reduced one and the
 * derivative across it is taken as 0.  Frames are independent.
 *   u_out, shell: the forward's outputs (FP64 colours of the forward)
 *   grad_out: B*H*W*C; grad_in: B*H*W*C; grad_g: B*H*W*2
 */
int gfo_adjoint(int B, int H, int W, int C, const uint8_t *label, const double *guide,
                double eps, double mu, int ghost, const double *u_out, const int32_t *shell,
                const double *grad_out, double *grad_in, double *grad_g)
{
    if (B < 0 || H <= 0 || W <= 0 || C <= 0 || !(eps > 0) || !(mu > 0)) return GFO_EINVAL;
    int on[GFO_MAX_OFFSETS], om[GFO_MAX_OFFSETS];
    int T = gfo_offsets(eps, on, om, GFO_MAX_OFFSETS);
    if (T <= 0) return GFO_EINVAL;
    size_t HW = (size_t)H * W;
    double a = mu * mu / (2.0 * eps * eps);
    ghost_t *G = (ghost_t *)malloc(sizeof(ghost_t) * T);
    unsigned char *rd = (unsigned char *)malloc(T);
    double *lam = (double *)malloc(sizeof(double) * T);
    double *v = (double *)malloc(sizeof(double) * T * C);
    double *u = (double *)malloc(sizeof(double) * C);
    if (!G || !rd || !lam || !v || !u) {
        free(G); free(rd); free(lam); free(v); free(u);
        return GFO_ENOMEM;
    }
    for (int b = 0; b < B; ++b) {
        const uint8_t *lab = label + (size_t)b * HW;
        const int32_t *s = shell + (size_t)b * HW;
        const double *uo = u_out + (size_t)b * HW * C;
        double *ub = grad_in + (size_t)b * HW * C;
        double *gg = grad_g + (size_t)b * HW * 2;
        prob_t P = {H, W, C, lab, guide + (size_t)b * HW * 2, eps, mu, -1.0, ghost, T, on, om};
        memcpy(ub, grad_out + (size_t)b * HW * C, sizeof(double) * HW * C);
        memset(gg, 0, sizeof(double) * HW * 2);
        int K = 0;
        for (size_t q = 0; q < HW; ++q)
            if (s[q] + 1 > K) K = s[q] + 1;
        for (int k = K - 1; k >= 0; --k) {
            for (size_t q = 0; q < HW; ++q) {
                if (s[q] != k) continue;
                int i = (int)(q % W), j = (int)(q / W);
                double gx = P.g[2 * q], gy = P.g[2 * q + 1];
                int rot = ghost && (gx != 0.0 || gy != 0.0);
                double L = rot ? sqrt(gx * gx + gy * gy) : 1.0;
                double cc = rot ? gx / L : 0.0, ss = rot ? gy / L : 0.0;
                double qmin = INFINITY;
                for (int t = 0; t < T; ++t) {
                    ghost_geometry(&P, gx, gy, on[t], om[t], &G[t]);
                    rd[t] = (unsigned char)ghost_readable(&P, s, i, j, &G[t], k);
                    double qq = a * G[t].t * G[t].t;
                    if (rd[t] && qq < qmin) qmin = qq;
                }
                double S = 0.0;
                for (int t = 0; t < T; ++t) {
                    lam[t] = 0.0;
                    if (!rd[t]) continue;
                    lam[t] = exp(-(a * G[t].t * G[t].t - qmin)) / G[t].rho;
                    S += lam[t];
                }
                if (!(S > 0)) continue; /* cannot happen for a filled pixel */
                for (int ch = 0; ch < C; ++ch) u[ch] = 0.0;
                for (int t = 0; t < T; ++t) {
                    if (!rd[t]) continue;
                    lam[t] /= S;
                    for (int ch = 0; ch < C; ++ch) {
                        v[t * C + ch] = ghost_value(&P, uo, i, j, &G[t], ch);
                        u[ch] += lam[t] * v[t * C + ch];
                    }
                }
                double dgx = 0.0, dgy = 0.0;
                for (int t = 0; t < T; ++t) {
                    if (!rd[t]) continue;
                    const ghost_t *Gt = &G[t];
                    /* d o / d g: rotation of o about x by d(theta) = (c dgy - s dgx)/L */
                    double dox_dgx = 0, dox_dgy = 0, doy_dgx = 0, doy_dgy = 0;
                    if (rot) {
                        dox_dgx = ss * Gt->oy / L;
                        dox_dgy = -cc * Gt->oy / L;
                        doy_dgx = -ss * Gt->ox / L;
                        doy_dgy = cc * Gt->ox / L;
                    }
                    /* t = g_perp . o = -gy ox + gx oy */
                    double dt_dgx = Gt->oy + (-gy) * dox_dgx + gx * doy_dgx;
                    double dt_dgy = -Gt->ox + (-gy) * dox_dgy + gx * doy_dgy;
                    /* log w = -a t^2 - log rho */
                    double r2 = Gt->rho * Gt->rho;
                    double dlw_dgx = -2.0 * a * Gt->t * dt_dgx - (Gt->ox * dox_dgx + Gt->oy * doy_dgx) / r2;
                    double dlw_dgy = -2.0 * a * Gt->t * dt_dgy - (Gt->ox * dox_dgy + Gt->oy * doy_dgy) / r2;
                    for (int ch = 0; ch < C; ++ch) {
                        /* gradient of the bilinear interpolant in the cell of p */
                        double vpx = 0.0, vpy = 0.0;
                        for (int bb = 0; bb < Gt->nsy; ++bb)
                            for (int aa = 0; aa < Gt->nsx; ++aa) {
                                size_t qq = (size_t)((j + Gt->dy + bb) * W + (i + Gt->dx + aa));
                                double uv = uo[qq * C + ch];
                                if (Gt->nsx == 2) vpx += (aa ? 1.0 : -1.0) * Gt->by[bb] * uv;
                                if (Gt->nsy == 2) vpy += (bb ? 1.0 : -1.0) * Gt->bx[aa] * uv;
                            }
                        double dv_dgx = vpx * dox_dgx + vpy * doy_dgx;
                        double dv_dgy = vpx * dox_dgy + vpy * doy_dgy;
                        double du_dgx = lam[t] * ((v[t * C + ch] - u[ch]) * dlw_dgx + dv_dgx);
                        double du_dgy = lam[t] * ((v[t * C + ch] - u[ch]) * dlw_dgy + dv_dgy);
                        dgx += ub[q * C + ch] * du_dgx;
                        dgy += ub[q * C + ch] * du_dgy;
                    }
                    /* pass the adjoint to the support pixels */
                    for (int bb = 0; bb < Gt->nsy; ++bb)
                        for (int aa = 0; aa < Gt->nsx; ++aa) {
                            size_t qq = (size_t)((j + Gt->dy + bb) * W + (i + Gt->dx + aa));
                            double beta = Gt->bx[aa] * Gt->by[bb];
                            for (int ch = 0; ch < C; ++ch)
                                ub[qq * C + ch] += ub[q * C + ch] * lam[t] * beta;
                        }
                }
                gg[2 * q] = dgx;
                gg[2 * q + 1] = dgy;
            }
        }
        /* a filled hole pixel's input colour does not reach the output */
        for (size_t q = 0; q < HW; ++q)
            if (s[q] >= 0)
                for (int ch = 0; ch < C; ++ch) ub[q * C + ch] = 0.0;
    }
    free(G); free(rd); free(lam); free(v); free(u);
    return GFO_OK;
}

/*
 * Guide field (Sec. 3.2): for every inpaint pixel x (label 1) of a frame,
 * the spline Gamma_x nearest to x and
 *     g(x) = g_Gamma_x exp(-d(x, Gamma_x)^2 / (2 eta^2)),
 * set to 0 where d(x, Gamma_x) > cutoff (the paper cuts off at 3 eta); 0 on
 * every other pixel and where the frame has no spline.  A spline is given as
 * a polyline of segments, each segment carrying the direction g_Gamma of its
 * spline (a straight spline has one segment; a sampled curve may give its
 * segments the local tangent), so the spline nearest to x is the one holding
 * the nearest segment.  Pixel (i, j) sits at the point (i, j): i the column,
 * j the row.
 *   seg      nseg*6: x0, y0, x1, y1, gx, gy of each segment
 *   seg_off  B+1: the segments of frame b are seg_off[b] .. seg_off[b+1]-1
 *   guide    B*H*W*2 output
 * Distance to a segment: the foot of the perpendicular, clamped to the
 * segment (the nearer end when it falls outside; the point itself for a
 * segment of zero length).  Equal distances keep the first segment.
 * Returns GFO_OK or GFO_EINVAL.
 */
int gfo_guide_field(int B, int H, int W, const uint8_t *label, const double *seg,
                    const int32_t *seg_off, double eta, double cutoff, double *guide)
{
    if (B < 0 || H <= 0 || W <= 0 || !(eta > 0) || !(cutoff >= 0)) return GFO_EINVAL;
    for (int b = 0; b < B; ++b) {
        const int s0 = seg_off[b], s1 = seg_off[b + 1];
        if (s0 < 0 || s1 < s0) return GFO_EINVAL;
        for (int j = 0; j < H; ++j)
            for (int i = 0; i < W; ++i) {
                const size_t q = ((size_t)b * H + j) * W + i;
                guide[2 * q] = 0.0;
                guide[2 * q + 1] = 0.0;
                if (label[q] != 1) continue;
                double best = INFINITY;
                int arg = -1;
                for (int e = s0; e < s1; ++e) {
                    const double *S = seg + 6 * (size_t)e;
                    const double dx = S[2] - S[0], dy = S[3] - S[1];
                    const double qx = (double)i - S[0], qy = (double)j - S[1];
                    const double len2 = dx * dx + dy * dy;
                    double t = 0.0;
                    if (len2 > 0.0) {
                        t = (qx * dx + qy * dy) / len2;
                        if (t < 0.0) t = 0.0;
                        if (t > 1.0) t = 1.0;
                    }
                    const double ex = qx - t * dx, ey = qy - t * dy;
                    const double d2 = ex * ex + ey * ey;
                    if (d2 < best) {
                        best = d2;
                        arg = e;
                    }
                }
                if (arg < 0 || best > cutoff * cutoff) continue;
                const double f = exp(-best / (2.0 * eta * eta));
                guide[2 * q] = seg[6 * (size_t)arg + 4] * f;
                guide[2 * q + 1] = seg[6 * (size_t)arg + 5] * f;
            }
    }
    return GFO_OK;
}


/* ------------------------------------------------------------------------
 * Modified structure tensor of coherence transport (Sec. 3.2,
 * eqn:modStructureTensor) and the guide it gives, for the comparison mode in
 * which g is re-estimated on the current known set at every shell.
 *
 * With K = the known set (Omega minus D^(k) and B), g_s the Gaussian of
 * variance s^2 truncated to |dx|, |dy| <= floor(2 s) (the (4 s + 1)^2 window
 * of Sec. 3.2; its normalisation cancels in both quotients):
 *   v(p)  = sum_q g_sigma(q - p) 1_K(q) u(q) / sum_q g_sigma(q - p) 1_K(q),
 *           defined where the denominator is positive;
 *   T(p)  = sum over channels of grad v (x) grad v, at p in K, with grad v by
 *           central differences (one-sided where a neighbour is outside the
 *           image or v is undefined there, 0 if both are);
 *   J(x)  = sum_p g_rho(p - x) 1_K(p) T(p) / sum_p g_rho(p - x) 1_K(p),
 *           NaN where the denominator is 0 (and, when `want` is given, at
 *           the pixels it does not ask for).
 * Sums run over in-image pixels, rows outer, columns inner.
 */
static double gauss2(int dx, int dy, double s)
{
    return exp(-(double)(dx * dx + dy * dy) / (2.0 * s * s));
}

int gfo_mod_structure_tensor(int H, int W, int C, const double *u, const uint8_t *known,
                             const uint8_t *want, double sigma, double rho, double *J)
{
    if (H <= 0 || W <= 0 || C <= 0 || !(sigma > 0) || !(rho > 0)) return GFO_EINVAL;
    const int rs = (int)floor(2.0 * sigma), rr = (int)floor(2.0 * rho);
    const size_t HW = (size_t)H * W;
    double *v = (double *)malloc(HW * C * sizeof(double));
    unsigned char *vok = (unsigned char *)malloc(HW);
    double *T = (double *)malloc(HW * 3 * sizeof(double));
    if (!v || !vok || !T) {
        free(v); free(vok); free(T);
        return GFO_ENOMEM;
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            const size_t p = (size_t)j * W + i;
            double den = 0.0;
            for (int c = 0; c < C; ++c) v[p * C + c] = 0.0;
            for (int dy = -rs; dy <= rs; ++dy)
                for (int dx = -rs; dx <= rs; ++dx) {
                    const int qi = i + dx, qj = j + dy;
                    if (qi < 0 || qi >= W || qj < 0 || qj >= H) continue;
                    const size_t q = (size_t)qj * W + qi;
                    if (!known[q]) continue;
                    const double w = gauss2(dx, dy, sigma);
                    den += w;
                    for (int c = 0; c < C; ++c) v[p * C + c] += w * u[q * C + c];
                }
            vok[p] = den > 0.0;
            for (int c = 0; c < C; ++c) v[p * C + c] = den > 0.0 ? v[p * C + c] / den : 0.0;
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            const size_t p = (size_t)j * W + i;
            T[3 * p] = T[3 * p + 1] = T[3 * p + 2] = 0.0;
            if (!known[p]) continue;
            const int l = i > 0 && vok[p - 1], r = i < W - 1 && vok[p + 1];
            const int t = j > 0 && vok[p - W], b = j < H - 1 && vok[p + W];
            for (int c = 0; c < C; ++c) {
                double gx = 0.0, gy = 0.0;
                if (l && r) gx = (v[(p + 1) * C + c] - v[(p - 1) * C + c]) / 2.0;
                else if (r) gx = v[(p + 1) * C + c] - v[p * C + c];
                else if (l) gx = v[p * C + c] - v[(p - 1) * C + c];
                if (t && b) gy = (v[(p + W) * C + c] - v[(p - W) * C + c]) / 2.0;
                else if (b) gy = v[(p + W) * C + c] - v[p * C + c];
                else if (t) gy = v[p * C + c] - v[(p - W) * C + c];
                T[3 * p] += gx * gx;
                T[3 * p + 1] += gx * gy;
                T[3 * p + 2] += gy * gy;
            }
        }
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            const size_t x = (size_t)j * W + i;
            if (want && !want[x]) {
                J[3 * x] = J[3 * x + 1] = J[3 * x + 2] = NAN;
                continue;
            }
            double den = 0.0, a = 0.0, b = 0.0, c = 0.0;
            for (int dy = -rr; dy <= rr; ++dy)
                for (int dx = -rr; dx <= rr; ++dx) {
                    const int qi = i + dx, qj = j + dy;
                    if (qi < 0 || qi >= W || qj < 0 || qj >= H) continue;
                    const size_t q = (size_t)qj * W + qi;
                    if (!known[q]) continue;
                    const double w = gauss2(dx, dy, rho);
                    den += w;
                    a += w * T[3 * q];
                    b += w * T[3 * q + 1];
                    c += w * T[3 * q + 2];
                }
            if (den > 0.0) {
                J[3 * x] = a / den;
                J[3 * x + 1] = b / den;
                J[3 * x + 2] = c / den;
            } else {
                J[3 * x] = J[3 * x + 1] = J[3 * x + 2] = NAN;
            }
        }
    free(v); free(vok); free(T);
    return GFO_OK;
}

/* The coherence direction of a structure tensor (a, b; b, c) as a guide:
 * g = tanh((lambda+ - lambda-) / Lambda) v-, v- the unit eigenvector of the
 * smaller eigenvalue (Sec. 3.2, with the tensor in place of J at x_base).
 * With h = (a - c)/2 and r = sqrt(h^2 + b^2), lambda+ - lambda- = 2 r and v-
 * is along (b, -(h + r)) when h >= 0, else along (h - r, b).  Its sign (which
 * the fill does not see) is fixed so that gx > 0, or gx == 0 and gy > 0.  A
 * NaN tensor (no known pixel within reach) gives g = 0. */
void gfo_tensor_guide(const double *J, double Lambda, double *g)
{
    g[0] = g[1] = 0.0;
    const double a = J[0], b = J[1], c = J[2];
    if (isnan(a) || isnan(b) || isnan(c)) return;
    const double h = (a - c) / 2.0;
    const double r = sqrt(h * h + b * b);
    if (!(r > 0.0)) return;
    double vx, vy;
    if (h >= 0.0) {
        vx = b;
        vy = -(h + r);
    } else {
        vx = h - r;
        vy = b;
    }
    const double n = sqrt(vx * vx + vy * vy);
    vx /= n;
    vy /= n;
    if (vx < 0.0 || (vx == 0.0 && vy < 0.0)) {
        vx = -vx;
        vy = -vy;
    }
    const double m = tanh(2.0 * r / Lambda);
    g[0] = m * vx;
    g[1] = m * vy;
}

/* The comparison mode's guide at shell k for B frames: for every inpaint
 * pixel (label 1) of each frame, the coherence direction of the modified
 * structure tensor over the known set label == 0; 0 on every other pixel. */
int gfo_coherence_guide(int B, int H, int W, int C, const double *u, const uint8_t *label,
                        double sigma, double rho, double Lambda, double *guide)
{
    if (B < 0 || H <= 0 || W <= 0 || C <= 0 || !(Lambda > 0)) return GFO_EINVAL;
    const size_t HW = (size_t)H * W;
    unsigned char *known = (unsigned char *)malloc(HW);
    unsigned char *want = (unsigned char *)malloc(HW);
    double *J = (double *)malloc(HW * 3 * sizeof(double));
    if (!known || !want || !J) {
        free(known); free(want); free(J);
        return GFO_ENOMEM;
    }
    for (int f = 0; f < B; ++f) {
        const uint8_t *lab = label + (size_t)f * HW;
        for (size_t p = 0; p < HW; ++p) {
            known[p] = lab[p] == 0;
            want[p] = lab[p] == 1;
        }
        const int rc =
            gfo_mod_structure_tensor(H, W, C, u + (size_t)f * HW * C, known, want, sigma, rho, J);
        if (rc != GFO_OK) {
            free(known); free(want); free(J);
            return rc;
        }
        double *gf = guide + (size_t)f * HW * 2;
        for (size_t p = 0; p < HW; ++p) {
            gf[2 * p] = gf[2 * p + 1] = 0.0;
            if (lab[p] == 1) gfo_tensor_guide(J + 3 * p, Lambda, gf + 2 * p);
        }
    }
    free(known); free(want); free(J);
    return GFO_OK;
}
