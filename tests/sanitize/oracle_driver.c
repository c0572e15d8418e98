/* The oracle's entry points on a small refined tree, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure; the
 * CPU tests build and run it).  argv[1]: a grid file written by the test
 * (box f64, n0 i32, max_level i32, periodic i32, n_cells i64, then level u8
 * [n], ijk i32 [n][3], phi f64 [n], grad f64 [n][3]).  Exits 0 when every
 * call returns as expected; the sanitizers abort on a memory or UB error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            fprintf(stderr, "oracle driver: check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                        \
        }                                                                    \
    } while (0)

static int read_all(FILE* f, void* p, size_t n) { return fread(p, 1, n, f) == n; }

int main(int argc, char** argv)
{
    if (argc < 2) return 2;
    FILE* fp = fopen(argv[1], "rb");
    CHECK(fp != NULL);
    double box;
    int32_t n0, max_level, periodic;
    int64_t n;
    CHECK(read_all(fp, &box, 8) && read_all(fp, &n0, 4) && read_all(fp, &max_level, 4) &&
          read_all(fp, &periodic, 4) && read_all(fp, &n, 8));
    uint8_t* level = malloc((size_t)n);
    int32_t* ijk = malloc((size_t)n * 12);
    double* phi = malloc((size_t)n * 8);
    double* grad = malloc((size_t)n * 24);
    double* tdot = malloc((size_t)n * 8);
    CHECK(level && ijk && phi && grad && tdot);
    CHECK(read_all(fp, level, (size_t)n) && read_all(fp, ijk, (size_t)n * 12) && read_all(fp, phi, (size_t)n * 8) &&
          read_all(fp, grad, (size_t)n * 24));
    fclose(fp);
    char err[256];
    or_field* f = or_field_grid(box, n0, max_level, periodic, n, level, ijk, phi, grad, err, sizeof err);
    CHECK(f != NULL);
    const or_cosmo c = {0.3, 0.7, 0.7};
    const int nr = 48;
    double* dirs = malloc(sizeof(double) * 3 * nr);
    for (int r = 0; r < nr; ++r) or_pix2vec_nest(2, r, dirs + 3 * r);
    or_ray_out* out = calloc(nr, sizeof(or_ray_out));
    or_ray_tan* tan = calloc(nr, sizeof(or_ray_tan));
    double* A = calloc(4 * nr, sizeof(double));
    double* dth = calloc(2 * nr, sizeof(double));
    double* dphi = calloc((size_t)n, sizeof(double));
    double* dgrad = calloc((size_t)n * 3, sizeof(double));
    CHECK(out && tan && A && dth && dphi && dgrad);
    for (int r = 0; r < nr; ++r) dth[2 * r] = 1.0;
    for (int64_t i = 0; i < n; ++i) { dphi[i] = 1e-6 * (double)(i % 7); tdot[i] = 1e-9 * (double)(i % 5); }
    or_cast_params p;
    memset(&p, 0, sizeof p);
    p.obs[0] = 0.37 * box; p.obs[1] = 0.52 * box; p.obs[2] = 0.61 * box;
    p.stop_kind = OR_STOP_REDSHIFT;
    p.stop_value = 0.05;
    p.steps_per_cell = 4;
    p.adaptive = 1;
    p.max_steps = 1 << 20;
    p.surface = OR_SURF_ETA;
    p.dphidl = OR_DPHIDL_CHAIN;
    const int threads = 2;
    int rc = 0;
    for (int order = 0; order <= 2 && !rc; ++order) {
        CHECK(or_field_set_order(f, order) == 0);
        rc = or_cast(f, &c, &p, nr, dirs, out, threads);
        CHECK(rc == 0);
        /* a non-periodic box is left before the source (LEFT_DOMAIN) */
        CHECK(out[0].n_steps > 0 && (out[0].status == OR_REACHED || out[0].status == OR_LEFT_DOMAIN));
    }
    CHECK(or_field_set_order(f, 1) == 0);
    CHECK(or_cast_cs(f, &c, &p, nr, dirs, dth, dphi, dgrad, out, tan, threads) == 0);
    CHECK(or_infinitesimal(f, &c, &p, nr, dirs, 0.0, A, out, threads) == 0);
    CHECK(or_born(f, &c, &p, nr, dirs, 0.0, A, out, threads) == 0);
    const double stops[2] = {0.02, 0.035};
    or_ray_out* out3 = calloc(3 * nr, sizeof(or_ray_out));
    CHECK(out3 && or_cast_surfaces(f, &c, &p, 2, stops, nr, dirs, out3, threads) == 0);
    for (int s = OR_SURF_CHI; s <= OR_SURF_Z; ++s) {
        p.surface = s;
        CHECK(or_cast(f, &c, &p, nr, dirs, out, threads) == 0);
    }
    p.surface = OR_SURF_ETA;
    p.dphidl = OR_DPHIDL_DIFF;
    CHECK(or_cast(f, &c, &p, nr, dirs, out, threads) == 0);
    p.dphidl = OR_DPHIDL_CHAIN;
    CHECK(or_field_set_tdot(f, tdot) == 0);
    CHECK(or_cast(f, &c, &p, nr, dirs, out, threads) == 0);
    or_field_free(f);
    /* a tree whose refined cell lacks a child is rejected */
    if (n > (int64_t)n0 * n0 * n0) {
        or_field* bad = or_field_grid(box, n0, max_level, periodic, n - 1, level, ijk, phi, grad, err, sizeof err);
        CHECK(bad == NULL);
    }
    free(level); free(ijk); free(phi); free(grad); free(tdot); free(dirs); free(out); free(tan); free(A);
    free(dth); free(dphi); free(dgrad); free(out3);
    printf("oracle driver ok\n");
    return 0;
}
