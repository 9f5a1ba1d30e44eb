/* Test driver: runs every entry point of the FP64 oracle on inputs read from a directory, so that
 * the oracle can be built and exercised under AddressSanitizer and UndefinedBehaviorSanitizer.
 * Usage: oracle_sanitize DIR W H N N3 K DEG. DIR holds raw little-endian arrays written by the
 * test (means2d, conics, opacity, colors, depths f64; radii i32; dloss f64 [3][H][W]; means3d,
 * scales, quats, sh, cam f64). Prints one checksum line per stage. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t orc_bin_count(const double *, const int32_t *, const double *, const double *, int32_t,
                      int64_t, int32_t, int32_t);
int64_t orc_bin(const double *, const int32_t *, const double *, const double *, int32_t,
                const double *, int64_t, int32_t, int32_t, int64_t, uint32_t *, uint32_t *);
void orc_forward(int32_t, int32_t, const uint32_t *, const uint32_t *, const double *,
                 const double *, const double *, const double *, const double *, double *,
                 double *, int32_t *, int32_t *, int32_t *, double *);
void orc_backward(int32_t, int32_t, const uint32_t *, const uint32_t *, const double *,
                  const double *, const double *, const double *, const double *, int64_t,
                  const double *, double *, double *, double *, double *);
void orc_project(const double *, const double *, const double *, const double *, int32_t, int32_t,
                 int64_t, const double *, double *, double *, double *, int32_t *, double *,
                 double *, double *);

static void *load(const char *dir, const char *name, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
    void *p = malloc(bytes ? bytes : 1);
    if (bytes && fread(p, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
    fclose(f);
    return p;
}

static double sum_d(const double *a, int64_t m) {
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += a[i];
    return s;
}

int main(int argc, char **argv) {
    if (argc != 8) { fprintf(stderr, "usage: %s DIR W H N N3 K DEG\n", argv[0]); return 2; }
    const char *dir = argv[1];
    const int32_t W = atoi(argv[2]), H = atoi(argv[3]);
    const int64_t n = atoll(argv[4]), n3 = atoll(argv[5]);
    const int32_t K = atoi(argv[6]), deg = atoi(argv[7]);
    const int64_t gx = (W + 15) / 16, gy = (H + 15) / 16, HW = (int64_t)W * H;
    double *m2 = load(dir, "means2d", 16 * n), *con = load(dir, "conics", 24 * n);
    double *op = load(dir, "opacity", 8 * n), *col = load(dir, "colors", 24 * n);
    double *dep = load(dir, "depths", 8 * n), *g = load(dir, "dloss", 8 * 3 * HW);
    int32_t *rad = load(dir, "radii", 4 * n);
    const double bg[3] = {0.1, 0.2, 0.3};
    for (int32_t mode = 0; mode <= 1; ++mode) {
        const int64_t P = orc_bin_count(m2, rad, con, op, mode, n, W, H);
        uint32_t *pl = malloc(4 * (P ? P : 1)), *rg = malloc(8 * gx * gy);
        const int64_t got = orc_bin(m2, rad, con, op, mode, dep, n, W, H, P, pl, rg);
        double *img = malloc(8 * 3 * HW), *T = malloc(8 * HW), *mg = malloc(8 * HW);
        int32_t *last = malloc(4 * HW), *ne = malloc(4 * HW), *nc = malloc(4 * HW);
        orc_forward(W, H, rg, pl, m2, con, op, col, bg, img, T, last, ne, nc, mg);
        double *dm = malloc(16 * n), *dc = malloc(24 * n), *dop = malloc(8 * n), *dcol = malloc(24 * n);
        orc_backward(W, H, rg, pl, m2, con, op, col, bg, n, g, dm, dc, dop, dcol);
        printf("mode %d pairs %lld %lld image %.17g T %.17g dm %.17g dc %.17g do %.17g dcol %.17g\n",
               (int)mode, (long long)P, (long long)got, sum_d(img, 3 * HW), sum_d(T, HW),
               sum_d(dm, 2 * n), sum_d(dc, 3 * n), sum_d(dop, n), sum_d(dcol, 3 * n));
        free(pl); free(rg); free(img); free(T); free(mg); free(last); free(ne); free(nc);
        free(dm); free(dc); free(dop); free(dcol);
    }
    double *m3 = load(dir, "means3d", 24 * n3), *sc = load(dir, "scales", 24 * n3);
    double *q = load(dir, "quats", 32 * n3), *sh = load(dir, "sh", 8 * 3 * K * n3);
    double *cam = load(dir, "cam", 8 * 19);
    double *pm = malloc(16 * n3), *pc = malloc(24 * n3), *pd = malloc(8 * n3), *pcol = malloc(24 * n3);
    double *rr = malloc(8 * n3), *pmg = malloc(24 * n3);
    int32_t *prad = malloc(4 * n3);
    orc_project(m3, sc, q, sh, K, deg, n3, cam, pm, pc, pd, prad, pcol, rr, pmg);
    int64_t rsum = 0;
    for (int64_t i = 0; i < n3; ++i) rsum += prad[i];
    printf("project means %.17g conics %.17g colors %.17g radii %lld\n", sum_d(pm, 2 * n3),
           sum_d(pc, 3 * n3), sum_d(pcol, 3 * n3), (long long)rsum);
    free(m2); free(con); free(op); free(col); free(dep); free(g); free(rad);
    free(m3); free(sc); free(q); free(sh); free(cam);
    free(pm); free(pc); free(pd); free(pcol); free(rr); free(pmg); free(prad);
    return 0;
}
