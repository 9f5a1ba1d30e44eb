/*
 * FP64 CPU oracle for tile-based front-to-back blending of projected 2D Gaussians.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously-correct definition that the
 * GPU library is checked against. It shares no code, header, table or constant generator with the
 * GPU library, and nothing in the product path may link or call it: only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg do.
 *
 * What it computes (GEMM-GS, DAC'26, arXiv 2604.02120):
 *   - orc_bin_*      duplication with tile|depth keys and depth sort (§2.1(b)-(c)), tile ranges.
 *   - orc_forward    volume rendering, Eq. (volume-render), with the per-pixel loop of Alg. 1:
 *                    exponent of Eq. (power), alpha of Eq. (alpha), 1/255 alpha-skipping and
 *                    early termination.
 *   - orc_backward   gradient of L = sum_p g_p . C_p with respect to the stored 2D means,
 *                    conic scalars (A, B, C), opacities and colours, derived by the product rule
 *                    from Eq. (volume-render) and Eq. (alpha) (the paper has no backward pass).
 *
 * The GEMM form of the paper (Eq. (power rewritten)) is an exact algebraic identity, so the plain
 * definition above is also the oracle of the GEMM path; it is deliberately not used here.
 *
 * Readings of points where the paper is silent or self-contradictory (each also listed in the
 * design notes of the repository):
 *   - alpha-skip is "alpha < 1/255" (Alg. 1 writes "<="), thresholds are the FP32 constants
 *     1/255, 1e-4 and 0.99 promoted exactly to FP64;
 *   - early termination tests T' = T (1 - alpha) < 1e-4 BEFORE blending; the Gaussian that trips
 *     it is not blended and T keeps its previous value (Alg. 1 updates T before the test and
 *     checks "T <= 0", which contradicts Eq. (volume-render));
 *   - alpha = min(0.99, o exp(min(power, 0)));
 *   - pixel (px, py) sits at integer coordinates;
 *   - a Gaussian with radius r > 0 covers tiles tx in [floor((x - r)/16), floor((x + r + 15)/16))
 *     (same for y), clamped to the grid; r = 0 means "not rendered";
 *   - the list of a tile is ordered by depth, ties broken by the Gaussian's index;
 *   - last_contrib is the 1-based position, within the tile's list, of the last blended
 *     Gaussian (0 = none);
 *   - derivatives are taken with respect to the stored scalars (A, B, C) (full -dx dy for B) and
 *     pixel-space means; a clamp that is active (o G >= 0.99, or power > 0) passes no gradient.
 *
 * Numerics: plain double arithmetic, built with -ffp-contract=off and without fast-math.
 * Threads: OpenMP over tiles (results do not depend on the thread count, except the summation
 * order of the backward's atomic FP64 adds).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TILE 16

/* FP32 thresholds promoted exactly to FP64. */
static double tau_cull(void) { return (double)(1.0f / 255.0f); }
static double t_stop(void) { return (double)1e-4f; }
static double alpha_max(void) { return (double)0.99f; }

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int64_t clamp_i64(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Tiles covered by Gaussian i: [tx0, tx1) x [ty0, ty1); empty when r <= 0.
 * The arithmetic is exact in FP64 for the FP32 means and integer radii this library accepts. */
static void tile_rect(double x, double y, int32_t r, int64_t gx, int64_t gy,
                      int64_t *tx0, int64_t *tx1, int64_t *ty0, int64_t *ty1) {
    if (r <= 0) { *tx0 = *tx1 = *ty0 = *ty1 = 0; return; }
    *tx0 = clamp_i64((int64_t)floor((x - r) / ORC_TILE), 0, gx);
    *tx1 = clamp_i64((int64_t)floor((x + r + ORC_TILE - 1) / ORC_TILE), 0, gx);
    *ty0 = clamp_i64((int64_t)floor((y - r) / ORC_TILE), 0, gy);
    *ty1 = clamp_i64((int64_t)floor((y + r + ORC_TILE - 1) / ORC_TILE), 0, gy);
}

/* ---- Binning mode 1: tiles on which the Gaussian can be visible (the opacity-aware extent of
 * a tighter binning; the paper's method is unchanged by it, see below).
 *
 * alpha = o exp(-Q/2) with Q = d^T Sigma^-1 d reaches 1/255 only where Q <= 2 ln(255 o). A pair
 * (tile, Gaussian) of the 3-sigma rectangle is kept iff o >= fp32(1/255) and the minimum of Q over
 * the rectangle spanned by the tile's pixels inside the image is <= theta, where theta is an upper
 * bound of 2 ln(255 o) that needs no logarithm, plus a margin:
 *     255 o = m 2^e (m in [1, 2)),  ln(255 o) <= e ln2 + (m - 1),
 *     theta = 2 (e * LN2_UP + (m - 1)) + 0.1   (LN2_UP: the double just above ln 2).
 * A dropped pair has alpha < (1/255) e^-0.05 on every pixel of its tile, so any evaluation whose
 * exponent error is far below 0.05 (every path here) skips it anyway: images and final T are
 * unchanged; only positions within the lists (last_contrib) move.
 * Q's minimum over a rectangle of d = (x - px, y - py) is 0 when the rectangle contains d = 0,
 * else it lies on an edge that faces d = 0 (an edge whose line separates the rectangle from 0: at
 * a minimiser p on an edge with outward normal n, -grad Q(p) = -2 Sigma^-1 p is a non-negative
 * multiple of n, so n.p = -c n^T Sigma n < 0), each a 1D quadratic minimised at an interior point
 * or at an end. Only those (at most two) edges are tested. Every test is written without
 * division, with this fixed sequence of IEEE double operations (no contraction), so the decision
 * is reproducible bit for bit. */
#define ORC_LN2_UP 0x1.62e42fefa39fp-1
#define ORC_PI 3.14159265358979323846
#define ORC_CULL_MARGIN 0.1

static double vis_theta(double o) {
    const double z = 255.0 * o;                 /* exact: o is an fp32 value */
    uint64_t bits;
    memcpy(&bits, &z, sizeof bits);
    const int64_t e = (int64_t)((bits >> 52) & 0x7ff) - 1023;
    const uint64_t mb = (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    double m;
    memcpy(&m, &mb, sizeof m);
    const double t1 = (double)e * ORC_LN2_UP;
    const double t2 = m - 1.0;
    return 2.0 * (t1 + t2) + ORC_CULL_MARGIN;
}

/* one edge: u fixed at a, v in [c, d]; Q = P a^2 + 2 B a v + R v^2 (P, R = A, C or C, A) */
static int vis_edge(double P, double R, double B, double det, double theta, double a, double c,
                    double d) {
    const double ba = B * a;
    const double nba = -ba;
    if (c * R <= nba && nba <= d * R) {           /* interior minimum a^2 det / R */
        const double lhs = (a * a) * det;
        const double rhs = theta * R;
        return lhs <= rhs;
    }
    const double pa2 = P * (a * a);
    const double qc = (pa2 + (2.0 * ba) * c) + R * (c * c);
    const double qd = (pa2 + (2.0 * ba) * d) + R * (d * d);
    return qc <= theta || qd <= theta;
}

static int tile_visible(double x, double y, const double *conic, double o, int64_t tx, int64_t ty,
                        int32_t W, int32_t H) {
    if (o < (double)(1.0f / 255.0f)) return 0;
    const double A = conic[0], B = conic[1], C = conic[2];
    const double x0 = (double)(tx * ORC_TILE), y0 = (double)(ty * ORC_TILE);
    const double x1 = (double)(tx * ORC_TILE + ORC_TILE - 1 < W - 1 ? tx * ORC_TILE + ORC_TILE - 1 : W - 1);
    const double y1 = (double)(ty * ORC_TILE + ORC_TILE - 1 < H - 1 ? ty * ORC_TILE + ORC_TILE - 1 : H - 1);
    const double dxl = x - x1, dxh = x - x0, dyl = y - y1, dyh = y - y0;
    if (dxl <= 0.0 && 0.0 <= dxh && dyl <= 0.0 && 0.0 <= dyh) return 1;
    const double theta = vis_theta(o);
    const double det = A * C - B * B;
    /* the x-edge facing 0 (if 0 is left or right of the rectangle), then the y-edge */
    if (dxl > 0.0 && vis_edge(A, C, B, det, theta, dxl, dyl, dyh)) return 1;
    if (dxh < 0.0 && vis_edge(A, C, B, det, theta, dxh, dyl, dyh)) return 1;
    if (dyl > 0.0 && vis_edge(C, A, B, det, theta, dyl, dxl, dxh)) return 1;
    if (dyh < 0.0 && vis_edge(C, A, B, det, theta, dyh, dxl, dxh)) return 1;
    return 0;
}

/* whether pair (tile (tx, ty), Gaussian i) is emitted under `mode` (0: the 3-sigma rectangle alone) */
static int pair_kept(int mode, const double *means2d, const double *conics, const double *opacity,
                     int64_t i, int64_t tx, int64_t ty, int32_t W, int32_t H) {
    if (mode == 0) return 1;
    return tile_visible(means2d[2 * i], means2d[2 * i + 1], conics + 3 * i, opacity[i], tx, ty, W, H);
}

/* Number of (tile, Gaussian) pairs. conics/opacity are read in mode 1 only. */
int64_t orc_bin_count(const double *means2d, const int32_t *radii, const double *conics,
                      const double *opacity, int32_t mode, int64_t n, int32_t W, int32_t H) {
    int64_t gx = (W + ORC_TILE - 1) / ORC_TILE, gy = (H + ORC_TILE - 1) / ORC_TILE, total = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t tx0, tx1, ty0, ty1;
        tile_rect(means2d[2 * i], means2d[2 * i + 1], radii[i], gx, gy, &tx0, &tx1, &ty0, &ty1);
        for (int64_t ty = ty0; ty < ty1; ++ty)
            for (int64_t tx = tx0; tx < tx1; ++tx)
                total += pair_kept(mode, means2d, conics, opacity, i, tx, ty, W, H);
    }
    return total;
}

typedef struct { int64_t tile; double depth; int64_t idx; } orc_pair;

static int pair_less(const void *pa, const void *pb) {
    const orc_pair *a = (const orc_pair *)pa, *b = (const orc_pair *)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->depth != b->depth) return a->depth < b->depth ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* Duplicate, sort by (tile, depth, index), extract ranges.
 * point_list: u32[capacity]; ranges: u32[gx*gy][2] as [start, end), [0, 0) when empty.
 * Returns the pair count, or -1 if it exceeds capacity (nothing written then). */
int64_t orc_bin(const double *means2d, const int32_t *radii, const double *conics,
                const double *opacity, int32_t mode, const double *depths, int64_t n, int32_t W,
                int32_t H, int64_t capacity, uint32_t *point_list, uint32_t *ranges) {
    int64_t gx = (W + ORC_TILE - 1) / ORC_TILE, gy = (H + ORC_TILE - 1) / ORC_TILE;
    int64_t total = orc_bin_count(means2d, radii, conics, opacity, mode, n, W, H);
    if (total > capacity) return -1;
    orc_pair *pairs = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(total > 0 ? total : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t tx0, tx1, ty0, ty1;
        tile_rect(means2d[2 * i], means2d[2 * i + 1], radii[i], gx, gy, &tx0, &tx1, &ty0, &ty1);
        for (int64_t ty = ty0; ty < ty1; ++ty)
            for (int64_t tx = tx0; tx < tx1; ++tx) {
                if (!pair_kept(mode, means2d, conics, opacity, i, tx, ty, W, H)) continue;
                pairs[k].tile = ty * gx + tx;
                pairs[k].depth = depths[i];
                pairs[k].idx = i;
                ++k;
            }
    }
    qsort(pairs, (size_t)total, sizeof(orc_pair), pair_less);
    memset(ranges, 0, sizeof(uint32_t) * 2 * (size_t)(gx * gy));
    for (int64_t p = 0; p < total; ++p) {
        point_list[p] = (uint32_t)pairs[p].idx;
        int64_t t = pairs[p].tile;
        if (p == 0 || pairs[p - 1].tile != t) ranges[2 * t] = (uint32_t)p;
        if (p == total - 1 || pairs[p + 1].tile != t) ranges[2 * t + 1] = (uint32_t)(p + 1);
    }
    free(pairs);
    return total;
}

/* The sorted list of one tile alone: every Gaussian whose rectangle covers tile t, ordered by
 * (depth, index). Writes up to cap indices; returns the full count. (Used to check single tiles of
 * frames too large to bin whole on the CPU.) */
int64_t orc_bin_tile(const double *means2d, const int32_t *radii, const double *conics,
                     const double *opacity, int32_t mode, const double *depths, int64_t n,
                     int32_t W, int32_t H, int64_t t, int64_t cap, uint32_t *out) {
    int64_t gx = (W + ORC_TILE - 1) / ORC_TILE, gy = (H + ORC_TILE - 1) / ORC_TILE;
    const int64_t tx = t % gx, ty = t / gx;
    int64_t k = 0;
    orc_pair *pairs = (orc_pair *)malloc(sizeof(orc_pair) * 1024);
    int64_t room = 1024;
    for (int64_t i = 0; i < n; ++i) {
        int64_t tx0, tx1, ty0, ty1;
        tile_rect(means2d[2 * i], means2d[2 * i + 1], radii[i], gx, gy, &tx0, &tx1, &ty0, &ty1);
        if (tx < tx0 || tx >= tx1 || ty < ty0 || ty >= ty1) continue;
        if (!pair_kept(mode, means2d, conics, opacity, i, tx, ty, W, H)) continue;
        if (k == room) {
            room *= 2;
            pairs = (orc_pair *)realloc(pairs, sizeof(orc_pair) * (size_t)room);
        }
        pairs[k].tile = t;
        pairs[k].depth = depths[i];
        pairs[k].idx = i;
        ++k;
    }
    qsort(pairs, (size_t)k, sizeof(orc_pair), pair_less);
    for (int64_t p = 0; p < k && p < cap; ++p) out[p] = (uint32_t)pairs[p].idx;
    free(pairs);
    return k;
}

/* Exponent of Eq. (power): -1/2 A dx^2 - B dx dy - 1/2 C dy^2, dx = x_g - x_p, dy = y_g - y_p. */
static double gauss_power(const double *conic, double dx, double dy) {
    return -0.5 * (conic[0] * dx * dx + conic[2] * dy * dy) - conic[1] * dx * dy;
}

static double rel_margin(double v, double thr) { return fabs(v - thr) / thr; }

/* Forward blend of every pixel. image is planar [3][H][W]; final_T and last_contrib are [H][W].
 * n_eval (optional): list entries examined per pixel, including the one that stops it.
 * n_contrib (optional): Gaussians blended into the pixel.
 * margin (optional): smallest relative distance of any alpha-skip or stop decision to its
 * threshold, per pixel (decisions this close can flip under rounding). */
void orc_forward(int32_t W, int32_t H, const uint32_t *ranges, const uint32_t *point_list,
                 const double *means2d, const double *conics, const double *opacity,
                 const double *colors, const double *bg, double *image, double *final_T,
                 int32_t *last_contrib, int32_t *n_eval, int32_t *n_contrib, double *margin) {
    const int64_t gx = (W + ORC_TILE - 1) / ORC_TILE, gy = (H + ORC_TILE - 1) / ORC_TILE;
    const int64_t HW = (int64_t)H * W;
    const double tau = tau_cull(), tstop = t_stop(), amax = alpha_max();
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < gx * gy; ++t) {
        const int64_t tx = t % gx, ty = t / gx;
        const uint32_t start = ranges[2 * t], end = ranges[2 * t + 1];
        for (int64_t py = ty * ORC_TILE; py < (ty + 1) * ORC_TILE && py < H; ++py) {
            for (int64_t px = tx * ORC_TILE; px < (tx + 1) * ORC_TILE && px < W; ++px) {
                double T = 1.0, acc[3] = {0.0, 0.0, 0.0}, mmin = INFINITY;
                int32_t last = 0, evals = 0, contrib = 0;
                for (uint32_t n = start; n < end; ++n) {
                    const int64_t i = point_list[n];
                    ++evals;
                    const double dx = means2d[2 * i] - (double)px, dy = means2d[2 * i + 1] - (double)py;
                    const double power = gauss_power(&conics[3 * i], dx, dy);
                    double alpha = opacity[i] * exp(power < 0.0 ? power : 0.0);
                    if (alpha > amax) alpha = amax;
                    const double m1 = rel_margin(alpha, tau);
                    if (m1 < mmin) mmin = m1;
                    if (alpha < tau) continue;
                    const double Tn = T * (1.0 - alpha);
                    const double m2 = rel_margin(Tn, tstop);
                    if (m2 < mmin) mmin = m2;
                    if (Tn < tstop) break;
                    for (int c = 0; c < 3; ++c) acc[c] += alpha * T * colors[3 * i + c];
                    T = Tn;
                    last = (int32_t)(n - start + 1);
                    ++contrib;
                }
                const int64_t p = py * W + px;
                for (int c = 0; c < 3; ++c) image[c * HW + p] = acc[c] + T * bg[c];
                final_T[p] = T;
                last_contrib[p] = last;
                if (n_eval) n_eval[p] = evals;
                if (n_contrib) n_contrib[p] = contrib;
                if (margin) margin[p] = mmin;
            }
        }
    }
}

/* Largest tile list length (scratch size for the backward). */
static int64_t max_list(const uint32_t *ranges, int64_t n_tiles) {
    int64_t m = 0;
    for (int64_t t = 0; t < n_tiles; ++t)
        if ((int64_t)ranges[2 * t + 1] - ranges[2 * t] > m) m = (int64_t)ranges[2 * t + 1] - ranges[2 * t];
    return m;
}

/* Gradient of L = sum over pixels and channels of dL_dimage * image.
 * Outputs are overwritten: dmeans2d [N][2], dconics [N][3] (d/dA, d/dB, d/dC), dopacity [N],
 * dcolors [N][3]. The forward is recomputed in order, keeping every contributor's T. */
void orc_backward(int32_t W, int32_t H, const uint32_t *ranges, const uint32_t *point_list,
                  const double *means2d, const double *conics, const double *opacity,
                  const double *colors, const double *bg, int64_t n, const double *dL_dimage,
                  double *dmeans2d, double *dconics, double *dopacity, double *dcolors) {
    const int64_t gx = (W + ORC_TILE - 1) / ORC_TILE, gy = (H + ORC_TILE - 1) / ORC_TILE;
    const int64_t HW = (int64_t)H * W;
    const double tau = tau_cull(), tstop = t_stop(), amax = alpha_max();
    memset(dmeans2d, 0, sizeof(double) * 2 * (size_t)n);
    memset(dconics, 0, sizeof(double) * 3 * (size_t)n);
    memset(dopacity, 0, sizeof(double) * (size_t)n);
    memset(dcolors, 0, sizeof(double) * 3 * (size_t)n);
    const int64_t cap = max_list(ranges, gx * gy) + 1;
#pragma omp parallel
    {
        /* per-contributor record of the in-order pass */
        int64_t *c_idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        double *c_alpha = (double *)malloc(sizeof(double) * (size_t)cap);
        double *c_T = (double *)malloc(sizeof(double) * (size_t)cap);
        double *c_G = (double *)malloc(sizeof(double) * (size_t)cap);
        double *c_dx = (double *)malloc(sizeof(double) * (size_t)cap);
        double *c_dy = (double *)malloc(sizeof(double) * (size_t)cap);
        int *c_aclamp = (int *)malloc(sizeof(int) * (size_t)cap);
        int *c_pclamp = (int *)malloc(sizeof(int) * (size_t)cap);
#pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < gx * gy; ++t) {
            const int64_t tx = t % gx, ty = t / gx;
            const uint32_t start = ranges[2 * t], end = ranges[2 * t + 1];
            for (int64_t py = ty * ORC_TILE; py < (ty + 1) * ORC_TILE && py < H; ++py) {
                for (int64_t px = tx * ORC_TILE; px < (tx + 1) * ORC_TILE && px < W; ++px) {
                    const int64_t p = py * W + px;
                    double g[3];
                    for (int c = 0; c < 3; ++c) g[c] = dL_dimage[c * HW + p];
                    /* in-order pass: the contributors and the T in front of each */
                    double T = 1.0;
                    int64_t k = 0;
                    for (uint32_t m = start; m < end; ++m) {
                        const int64_t i = point_list[m];
                        const double dx = means2d[2 * i] - (double)px, dy = means2d[2 * i + 1] - (double)py;
                        const double power = gauss_power(&conics[3 * i], dx, dy);
                        const int pclamp = power > 0.0;
                        const double G = exp(pclamp ? 0.0 : power);
                        double alpha = opacity[i] * G;
                        const int aclamp = alpha >= amax;
                        if (aclamp) alpha = amax;
                        if (alpha < tau) continue;
                        const double Tn = T * (1.0 - alpha);
                        if (Tn < tstop) break;
                        c_idx[k] = i; c_alpha[k] = alpha; c_T[k] = T; c_G[k] = G;
                        c_dx[k] = dx; c_dy[k] = dy; c_aclamp[k] = aclamp; c_pclamp[k] = pclamp;
                        ++k;
                        T = Tn;
                    }
                    const double T_final = T;
                    double bg_g = 0.0;
                    for (int c = 0; c < 3; ++c) bg_g += bg[c] * g[c];
                    /* reverse pass: behind[c] = sum over later contributors of alpha_k T_k c_k */
                    double behind[3] = {0.0, 0.0, 0.0};
                    for (int64_t j = k - 1; j >= 0; --j) {
                        const int64_t i = c_idx[j];
                        const double a = c_alpha[j], Tj = c_T[j];
                        /* dC/dalpha_j = T_j c_j - (behind_j + T_final bg) / (1 - alpha_j) */
                        double dL_da = 0.0;
                        for (int c = 0; c < 3; ++c)
                            dL_da += g[c] * (Tj * colors[3 * i + c] - behind[c] / (1.0 - a));
                        dL_da -= T_final * bg_g / (1.0 - a);
                        for (int c = 0; c < 3; ++c) {
                            const double dc = a * Tj * g[c];
#pragma omp atomic
                            dcolors[3 * i + c] += dc;
                        }
                        if (!c_aclamp[j]) {
                            const double G = c_G[j];
                            const double d_o = G * dL_da;
#pragma omp atomic
                            dopacity[i] += d_o;
                            if (!c_pclamp[j]) {
                                const double dP = opacity[i] * G * dL_da;
                                const double dx = c_dx[j], dy = c_dy[j];
                                const double A = conics[3 * i], B = conics[3 * i + 1], C = conics[3 * i + 2];
                                const double gA = -0.5 * dx * dx * dP, gB = -dx * dy * dP, gC = -0.5 * dy * dy * dP;
                                const double gx_ = -(A * dx + B * dy) * dP, gy_ = -(B * dx + C * dy) * dP;
#pragma omp atomic
                                dconics[3 * i] += gA;
#pragma omp atomic
                                dconics[3 * i + 1] += gB;
#pragma omp atomic
                                dconics[3 * i + 2] += gC;
#pragma omp atomic
                                dmeans2d[2 * i] += gx_;
#pragma omp atomic
                                dmeans2d[2 * i + 1] += gy_;
                            }
                        }
                        for (int c = 0; c < 3; ++c) behind[c] += a * Tj * colors[3 * i + c];
                    }
                }
            }
        }
        free(c_idx); free(c_alpha); free(c_T); free(c_G); free(c_dx); free(c_dy);
        free(c_aclamp); free(c_pclamp);
    }
}


/* ---- Preprocessing (Sec. 2.1(a)): 3D Gaussians seen by a pinhole camera become the 2D
 * Gaussians the blend consumes (mean, conic, depth, extent radius) and get their colour for this
 * view. The paper names the step and its outputs without formulas; this is the EWA splatting
 * projection of 3D Gaussian splatting, the method the paper accelerates.
 *
 * Real spherical harmonics of degree l <= 3 at a unit direction (x, y, z), polar axis z, in the
 * usual order (l, m = -l..l), with the Condon-Shortley phase kept:
 *   Y_l^m = sqrt(2) K_l^m cos(m phi) P_l^m(cos theta)     (m > 0)
 *   Y_l^0 = K_l^0 P_l^0(cos theta)
 *   Y_l^m = sqrt(2) K_l^|m| sin(|m| phi) P_l^|m|(cos theta) (m < 0)
 *   K_l^m = sqrt((2l + 1) / (4 pi) (l - m)! / (l + m)!),
 * P_l^m the associated Legendre functions (with the (-1)^m phase) from the textbook recurrences
 *   P_m^m = (-1)^m (2m - 1)!! (1 - t^2)^(m/2),  P_{m+1}^m = t (2m + 1) P_m^m,
 *   P_l^m = ((2l - 1) t P_{l-1}^m - (l + m - 1) P_{l-2}^m) / (l - m).
 * out receives (deg + 1)^2 values per direction. */
static double orc_fact(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

static void sh_basis_one(const double *d, int deg, double *out) {
    const double nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double x = d[0] / nrm, y = d[1] / nrm, t = d[2] / nrm;
    const double st = sqrt(fmax(0.0, 1.0 - t * t));
    const double phi = atan2(y, x);
    double P[4][4] = {{0}};                          /* P[l][m], m >= 0 */
    for (int m = 0; m <= deg; ++m) {
        double pmm = 1.0;
        for (int k = 1; k <= m; ++k) pmm *= -(2.0 * k - 1.0) * st;
        P[m][m] = pmm;
        if (m + 1 <= deg) P[m + 1][m] = t * (2.0 * m + 1.0) * pmm;
        for (int l = m + 2; l <= deg; ++l)
            P[l][m] = ((2.0 * l - 1.0) * t * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (l - m);
    }
    for (int l = 0; l <= deg; ++l)
        for (int m = -l; m <= l; ++m) {
            const int am = m < 0 ? -m : m;
            const double K = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI) * orc_fact(l - am) / orc_fact(l + am));
            double v;
            if (m > 0) v = sqrt(2.0) * K * cos(m * phi) * P[l][am];
            else if (m == 0) v = K * P[l][0];
            else v = sqrt(2.0) * K * sin(am * phi) * P[l][am];
            out[l * l + l + m] = v;
        }
}

void orc_sh_basis(const double *dirs, int64_t n, int32_t deg, double *out) {
    const int64_t k = (int64_t)(deg + 1) * (deg + 1);
    for (int64_t i = 0; i < n; ++i) sh_basis_one(dirs + 3 * i, deg, out + k * i);
}

/* Projection. Camera cam = [R (9, row-major, world to camera), t (3), fx, fy, cx, cy, W, H,
 * near]. Per Gaussian i (mean m, per-axis scale s, quaternion q = (w, x, y, z), SH coefficients
 * sh[i][k][c] for k < sh_coeffs of which the first (deg + 1)^2 are used):
 *   p = R m + t; culled if p.z <= near;
 *   means2d = (fx p.x / p.z + cx, fy p.y / p.z + cy), depth = p.z;
 *   Sigma3 = Rq diag(s^2) Rq^T, Rq the rotation of q / |q|;
 *   J = d(means2d)/dp = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]], evaluated with x/z and y/z
 *       clamped to 1.3 times the half field of view (W / (2 fx), H / (2 fy));
 *   Sigma2 = J R Sigma3 R^T J^T + 0.3 I (a low-pass filter); culled unless det Sigma2 > 0;
 *   conic = Sigma2^-1 = (c, -b, a) / det for Sigma2 = [[a, b], [b, c]];
 *   radius = ceil(3 sqrt(lmax)), lmax = mid + sqrt(max(0.1, mid^2 - det)), mid = (a + c) / 2;
 *   culled if the radius-square's tile rectangle (the binning rule above) is empty;
 *   colour_c = max(0, 0.5 + sum_k Y_k(dir) sh[i][k][c]), dir = (m - o) / |m - o| with the
 *       camera centre o = -R^T t.
 * A culled Gaussian has radius 0 and every other output 0.
 * rad_real receives 3 sqrt(lmax) (before the ceiling) and margin[i][3] the distance of each
 * culling decision from its threshold: |z - near| / near, det / (a c), and the distance in pixels
 * of the means2d from the nearest edge of the rectangle test, so a caller can tell which integers
 * rounding may flip (a decision not reached has margin +inf). */
void orc_project(const double *means3d, const double *scales, const double *quats,
                 const double *sh, int32_t sh_coeffs, int32_t deg, int64_t n, const double *cam,
                 double *means2d, double *conics, double *depths, int32_t *radii,
                 double *colors, double *rad_real, double *margin) {
    const double *R = cam, *t = cam + 9;
    const double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    const int64_t W = (int64_t)cam[16], H = (int64_t)cam[17];
    const double near = cam[18];
    const double limx = 1.3 * ((double)W / (2.0 * fx)), limy = 1.3 * ((double)H / (2.0 * fy));
    const int64_t gx = (W + ORC_TILE - 1) / ORC_TILE, gy = (H + ORC_TILE - 1) / ORC_TILE;
    double o[3];
    for (int c = 0; c < 3; ++c) o[c] = -(R[c] * t[0] + R[3 + c] * t[1] + R[6 + c] * t[2]);
    const int nb = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double *m = means3d + 3 * i, *sc = scales + 3 * i, *q0 = quats + 4 * i;
        means2d[2 * i] = means2d[2 * i + 1] = 0.0;
        conics[3 * i] = conics[3 * i + 1] = conics[3 * i + 2] = 0.0;
        colors[3 * i] = colors[3 * i + 1] = colors[3 * i + 2] = 0.0;
        depths[i] = 0.0;
        radii[i] = 0;
        rad_real[i] = 0.0;
        margin[3 * i] = margin[3 * i + 1] = margin[3 * i + 2] = HUGE_VAL;
        double p[3];
        for (int r = 0; r < 3; ++r) p[r] = R[3 * r] * m[0] + R[3 * r + 1] * m[1] + R[3 * r + 2] * m[2] + t[r];
        margin[3 * i] = fabs(p[2] - near) / fmax(fabs(near), 1e-30);
        if (!(p[2] > near)) continue;
        const double u = fx * p[0] / p[2] + cx, v = fy * p[1] / p[2] + cy;
        /* Sigma3 */
        const double qn = sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3]);
        const double w = q0[0] / qn, x = q0[1] / qn, y = q0[2] / qn, z = q0[3] / qn;
        const double Rq[3][3] = {
            {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
        double S3[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += Rq[r][k] * sc[k] * sc[k] * Rq[c][k];
                S3[r][c] = acc;
            }
        /* J R, then Sigma2 */
        const double zc = p[2];
        const double xz = fmin(limx, fmax(-limx, p[0] / zc)), yz = fmin(limy, fmax(-limy, p[1] / zc));
        const double J[2][3] = {{fx / zc, 0.0, -fx * xz / zc}, {0.0, fy / zc, -fy * yz / zc}};
        double T[2][3];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c) T[r][c] = J[r][0] * R[c] + J[r][1] * R[3 + c] + J[r][2] * R[6 + c];
        double S2[2][2];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) acc += T[r][k] * S3[k][l] * T[c][l];
                S2[r][c] = acc;
            }
        const double a = S2[0][0] + 0.3, b = S2[0][1], c = S2[1][1] + 0.3;
        const double det = a * c - b * b;
        margin[3 * i + 1] = fabs(det) / fmax(a * c, 1e-300);
        if (!(det > 0.0)) continue;
        const double mid = 0.5 * (a + c);
        const double lmax = mid + sqrt(fmax(0.1, mid * mid - det));
        const double rr = 3.0 * sqrt(lmax);
        const int32_t r = (int32_t)ceil(rr);
        /* empty tile rectangle: x + r + 15 < 16 or x - r >= 16 gx (and in y) */
        int64_t tx0, tx1, ty0, ty1;
        tile_rect(u, v, r, gx, gy, &tx0, &tx1, &ty0, &ty1);
        const double em = fmin(fmin(fabs(u + r - 1.0), fabs(u - r - (double)(ORC_TILE * gx))),
                               fmin(fabs(v + r - 1.0), fabs(v - r - (double)(ORC_TILE * gy))));
        margin[3 * i + 2] = em;
        rad_real[i] = rr;
        if (tx1 <= tx0 || ty1 <= ty0) continue;
        means2d[2 * i] = u;
        means2d[2 * i + 1] = v;
        depths[i] = zc;
        conics[3 * i] = c / det;
        conics[3 * i + 1] = -b / det;
        conics[3 * i + 2] = a / det;
        radii[i] = r;
        /* colour */
        double dir[3] = {m[0] - o[0], m[1] - o[1], m[2] - o[2]};
        double Y[16];
        sh_basis_one(dir, deg, Y);
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.5;
            for (int k = 0; k < nb; ++k) acc += Y[k] * sh[(i * sh_coeffs + k) * 3 + ch];
            colors[3 * i + ch] = fmax(0.0, acc);
        }
    }
}
