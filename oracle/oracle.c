/*
 * oracle.c -- plain FP64 CPU oracle (see oracle.h).  TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the CPU-baseline leg of the bench,
 * never by the GPU library.
 *
 * Octree lookups use one dense array for the coarse level and a hash table
 * keyed by (level, i, j, k) for the refined levels: a cell "exists" when its
 * key is present, which is all the interpolation procedure of Sect. 2.2 needs.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* H0 in h/Mpc with c = 1 (100 h km/s/Mpc divided by c in km/s). */
#define OR_H0 (1.0 / 2997.92458)
#define FNV_OFFSET 2166136261u
#define FNV_PRIME 16777619u
#define CS_H 1e-20

struct or_field {
    int kind;
    int order;            /* grid interpolation: 0 NGP, 1 CIC, 2 TSC (Sect. 2.2) */
    /* grid */
    double box, h0;
    int n0, max_level, periodic;
    int64_t n_cells;
    double* phi;
    double* grad;
    double* tdot;         /* dPhi/deta per cell, or NULL (static potential) */
    int64_t* coarse;      /* [n0^3] cell index of coarse cell (i + n0 (j + n0 k)) */
    uint64_t* hkeys;      /* open-addressing table for levels >= 1 */
    int64_t* hvals;
    uint64_t hmask;
    /* closed form */
    double par[16];
};

typedef struct { const double* dphi; const double* dgrad; } cs_ctx;

/* eta_s, a_s: the FLRW stop; p_s: the value of the stop surface's parameter
 * there (ln(1 + z) for the redshift surface) */
typedef struct { double eta0, eta_s, a_s, p_s; } derived_t;

static inline uint32_t fnv_step(uint32_t h, uint32_t v) { return (h ^ v) * FNV_PRIME; }

/* ------------------------------------------------------------------------- */
/* octree                                                                     */
/* ------------------------------------------------------------------------- */
static uint64_t mix64(uint64_t x)
{
    x ^= x >> 30; x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27; x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

static uint64_t cell_key(int l, int64_t i, int64_t j, int64_t k, int64_t m)
{
    return ((uint64_t)l << 56) | (uint64_t)(i + m * (j + m * k));
}

static int64_t hash_find(const or_field* f, uint64_t key)
{
    uint64_t s = mix64(key) & f->hmask;
    for (;;) {
        if (f->hkeys[s] == key) return f->hvals[s];
        if (f->hkeys[s] == UINT64_MAX) return -1;
        s = (s + 1) & f->hmask;
    }
}

static int hash_insert(or_field* f, uint64_t key, int64_t val)
{
    uint64_t s = mix64(key) & f->hmask;
    for (;;) {
        if (f->hkeys[s] == key) return 0;           /* duplicate */
        if (f->hkeys[s] == UINT64_MAX) { f->hkeys[s] = key; f->hvals[s] = val; return 1; }
        s = (s + 1) & f->hmask;
    }
}

/* Index of cell (l, I) or -1 when it does not exist.  Periodic grids wrap the
 * indices; non-periodic grids have no cells outside the box. */
static int64_t find_cell(const or_field* f, int l, const int64_t cidx[3])
{
    const int64_t m = (int64_t)f->n0 << l;
    int64_t J[3];
    for (int d = 0; d < 3; ++d) {
        if (f->periodic) J[d] = ((cidx[d] % m) + m) % m;
        else if (cidx[d] < 0 || cidx[d] >= m) return -1;
        else J[d] = cidx[d];
    }
    if (l == 0) return f->coarse[J[0] + (int64_t)f->n0 * (J[1] + (int64_t)f->n0 * J[2])];
    return hash_find(f, cell_key(l, J[0], J[1], J[2], m));
}

/* Level of the deepest existing cell containing the point with coarse-grid
 * coordinates u (cells are half-open: index = floor), or -1 outside. */
static int leaf_level(const or_field* f, const double u[3])
{
    int leaf = -1;
    for (int l = 0; l <= f->max_level; ++l) {
        const double s = ldexp(1.0, l);
        int64_t cidx[3];
        for (int d = 0; d < 3; ++d) cidx[d] = (int64_t)floor(u[d] * s);
        if (find_cell(f, l, cidx) < 0) break;
        leaf = l;
    }
    return leaf;
}

/* The 8 cells b + {0,1}^3 at level l (octant o = ox + 2 oy + 4 oz); returns 0
 * if any of them is missing. */
static int stencil_cells(const or_field* f, int l, const int64_t b[3], int64_t ids[8])
{
    for (int o = 0; o < 8; ++o) {
        const int64_t cidx[3] = {b[0] + (o & 1), b[1] + ((o >> 1) & 1), b[2] + ((o >> 2) & 1)};
        ids[o] = find_cell(f, l, cidx);
        if (ids[o] < 0) return 0;
    }
    return 1;
}

/* The 27 cells c + {-1,0,1}^3 at level l (index (ox+1) + 3 (oy+1) + 9 (oz+1));
 * returns 0 if any of them is missing. */
static int tsc_cells(const or_field* f, int l, const int64_t c[3], int64_t ids[27])
{
    for (int q = 0; q < 27; ++q) {
        const int64_t cidx[3] = {c[0] + q % 3 - 1, c[1] + (q / 3) % 3 - 1, c[2] + q / 9 - 1};
        ids[q] = find_cell(f, l, cidx);
        if (ids[q] < 0) return 0;
    }
    return 1;
}

int or_field_set_order(or_field* f, int order)
{
    if (!f || f->kind != OR_FIELD_GRID || order < 0 || order > 2) return -1;
    f->order = order;
    return 0;
}

static void set_err(char* err, int errlen, const char* msg)
{
    if (err && errlen > 0) { strncpy(err, msg, (size_t)errlen - 1); err[errlen - 1] = 0; }
}

or_field* or_field_grid(double box, int n0, int max_level, int periodic, int64_t n_cells,
                        const uint8_t* level, const int32_t* ijk, const double* phi,
                        const double* grad, char* err, int errlen)
{
    if (!(box > 0) || n0 <= 0 || max_level < 0 || max_level > 12 || n_cells <= 0) {
        set_err(err, errlen, "invalid grid parameters");
        return NULL;
    }
    or_field* f = (or_field*)calloc(1, sizeof(or_field));
    f->kind = OR_FIELD_GRID;
    f->order = 1;
    f->box = box; f->n0 = n0; f->max_level = max_level; f->periodic = periodic;
    f->h0 = box / n0;
    f->n_cells = n_cells;
    f->phi = (double*)malloc(sizeof(double) * (size_t)n_cells);
    f->grad = (double*)malloc(sizeof(double) * 3 * (size_t)n_cells);
    memcpy(f->phi, phi, sizeof(double) * (size_t)n_cells);
    memcpy(f->grad, grad, sizeof(double) * 3 * (size_t)n_cells);
    const int64_t nc = (int64_t)n0 * n0 * n0;
    f->coarse = (int64_t*)malloc(sizeof(int64_t) * (size_t)nc);
    for (int64_t i = 0; i < nc; ++i) f->coarse[i] = -1;
    uint64_t cap = 16;
    while (cap < 2 * (uint64_t)n_cells) cap <<= 1;
    f->hmask = cap - 1;
    f->hkeys = (uint64_t*)malloc(sizeof(uint64_t) * cap);
    f->hvals = (int64_t*)malloc(sizeof(int64_t) * cap);
    memset(f->hkeys, 0xff, sizeof(uint64_t) * cap);
    char msg[256];
    const int progress = n_cells >= ((int64_t)1 << 26);   /* very large grids report their progress */
    for (int64_t c = 0; c < n_cells; ++c) {
        if (progress && (c & (((int64_t)1 << 25) - 1)) == 0)
            fprintf(stderr, "oracle grid: indexed %lld of %lld cells\n", (long long)c, (long long)n_cells);
        const int l = level[c];
        const int64_t m = (int64_t)n0 << l;
        const int64_t i = ijk[3 * c], j = ijk[3 * c + 1], k = ijk[3 * c + 2];
        if (l > max_level || i < 0 || j < 0 || k < 0 || i >= m || j >= m || k >= m) {
            snprintf(msg, sizeof msg, "cell %lld out of range", (long long)c);
            set_err(err, errlen, msg); or_field_free(f); return NULL;
        }
        if (l == 0) {
            int64_t* slot = &f->coarse[i + n0 * (j + n0 * k)];
            if (*slot >= 0) { set_err(err, errlen, "duplicate coarse cell"); or_field_free(f); return NULL; }
            *slot = c;
        } else if (!hash_insert(f, cell_key(l, i, j, k, m), c)) {
            set_err(err, errlen, "duplicate cell"); or_field_free(f); return NULL;
        }
    }
    for (int64_t i = 0; i < nc; ++i)
        if (f->coarse[i] < 0) { set_err(err, errlen, "missing coarse cell"); or_field_free(f); return NULL; }
    /* full tree: every refined cell's parent exists and has all 8 children.
     * A family is checked in full once, through its first child (octant 0);
     * any other child only checks that the first child exists. */
    for (int64_t c = 0; c < n_cells; ++c) {
        if (progress && (c & (((int64_t)1 << 25) - 1)) == 0)
            fprintf(stderr, "oracle grid: checked %lld of %lld cells\n", (long long)c, (long long)n_cells);
        const int l = level[c];
        if (l == 0) continue;
        const int64_t P[3] = {ijk[3 * c] >> 1, ijk[3 * c + 1] >> 1, ijk[3 * c + 2] >> 1};
        if (find_cell(f, l - 1, P) < 0) { set_err(err, errlen, "orphan cell (parent missing)"); or_field_free(f); return NULL; }
        int64_t b[3] = {2 * P[0], 2 * P[1], 2 * P[2]}, ids[8];
        const int first = ijk[3 * c] == b[0] && ijk[3 * c + 1] == b[1] && ijk[3 * c + 2] == b[2];
        if (first ? !stencil_cells(f, l, b, ids) : find_cell(f, l, b) < 0) {
            set_err(err, errlen, "not a full tree (a parent has 1-7 children)"); or_field_free(f); return NULL;
        }
    }
    return f;
}

or_field* or_field_analytic(int kind, const double* params)
{
    if (kind != OR_FIELD_LINEAR && kind != OR_FIELD_QUADRATIC && kind != OR_FIELD_POINT) return NULL;
    or_field* f = (or_field*)calloc(1, sizeof(or_field));
    f->kind = kind;
    const int np = kind == OR_FIELD_LINEAR ? 4 : kind == OR_FIELD_QUADRATIC ? 10 : 5;
    memcpy(f->par, params, sizeof(double) * (size_t)np);
    return f;
}

void or_field_free(or_field* f)
{
    if (!f) return;
    free(f->phi); free(f->grad); free(f->tdot); free(f->coarse); free(f->hkeys); free(f->hvals);
    free(f);
}

int or_field_set_tdot(or_field* f, const double* tdot)
{
    if (!f || f->kind != OR_FIELD_GRID) return -1;
    free(f->tdot);
    f->tdot = NULL;
    if (!tdot) return 0;
    f->tdot = (double*)malloc(sizeof(double) * (size_t)f->n_cells);
    memcpy(f->tdot, tdot, sizeof(double) * (size_t)f->n_cells);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* cosmology: flat LCDM, Omega_r = 0, conformal time from the closed form     */
/* ------------------------------------------------------------------------- */
static int is_static(const or_cosmo* c) { return c->omega_m == 0.0 && c->omega_l == 0.0; }

int or_cosmo_check(const or_cosmo* c)
{
    if (is_static(c)) return 0;
    if (c->omega_m > 0.0 && c->omega_l >= 0.0 && fabs(c->omega_m + c->omega_l - 1.0) < 1e-12) return 0;
    return -1;
}

/* Gauss hypergeometric series 2F1(2/3, 1/6; 7/6; w), 0 <= w < 1, with the
 * series coefficients (2/3)_n (1/6)_n / ((7/6)_n n!) tabulated once. */
#define HYP_NCOEF 4096
static double hyp_coef[HYP_NCOEF];
static pthread_once_t hyp_once = PTHREAD_ONCE_INIT;

static void hyp_init(void)
{
    const double A = 2.0 / 3.0, B = 1.0 / 6.0, Cc = 7.0 / 6.0;
    double t = 1.0;
    for (int n = 0; n < HYP_NCOEF; ++n) {
        hyp_coef[n] = t;
        t *= (A + n) * (B + n) / ((Cc + n) * (n + 1.0));
    }
}

static double hyp2f1_eta(double w)
{
    pthread_once(&hyp_once, hyp_init);
    double sum = 0.0, wn = 1.0;
    for (int n = 0; n < HYP_NCOEF; ++n) {
        const double term = hyp_coef[n] * wn;
        sum += term;
        if (term < 1e-18 * sum) break;
        wn *= w;
    }
    return sum;
}

/* eta(a) = int_0^a da' / (a'^2 H(a')), H = H0 sqrt(Om a^-3 + OL).  With
 * q = OL/Om this is 2 sqrt(a)/(H0 sqrt(Om)) 2F1(1/2, 1/6; 7/6; -q a^3); the
 * series is evaluated after Pfaff's transformation
 * 2F1(a, b; c; x) = (1-x)^-b 2F1(c-a, b; c; x/(x-1)), whose argument
 * q a^3/(1 + q a^3) lies in [0, 1). */
double or_eta_of_a(const or_cosmo* c, double a)
{
    if (is_static(c)) return NAN;
    const double om = c->omega_m, q = c->omega_l / om;
    const double qa3 = q * a * a * a;
    const double w = qa3 / (1.0 + qa3);
    return 2.0 * sqrt(a) / (OR_H0 * sqrt(om)) * pow(1.0 + qa3, -1.0 / 6.0) * hyp2f1_eta(w);
}

static double hubble_of_a(const or_cosmo* c, double a)
{
    return OR_H0 * sqrt(c->omega_m / (a * a * a) + c->omega_l);
}

double or_eta0(const or_cosmo* c) { return is_static(c) ? 0.0 : or_eta_of_a(c, 1.0); }

/* composite Simpson rule on 20000 intervals of 1/H(a) = a / (a'/a)(a) */
double or_lambda_of_a(const or_cosmo* c, double a)
{
    if (is_static(c)) return NAN;
    const int n = 20000;
    const double h = (1.0 - a) / n;
    double sum = 0.0;
    for (int i = 0; i <= n; ++i) {
        const double x = a + i * h;
        const double f = 1.0 / (OR_H0 * sqrt(c->omega_m / (x * x * x) + c->omega_l));
        sum += (i == 0 || i == n) ? f : (i % 2 ? 4.0 * f : 2.0 * f);
    }
    return sum * h / 3.0;
}

/* a(eta) by Newton iteration on eta as a function of y = sqrt(a), in which
 * eta is exactly linear during matter domination (d eta/dy = 2 / (y^3 H)),
 * started from the matter-dominated value and safeguarded by a bisection
 * bracket. */
double or_a_of_eta(const or_cosmo* c, double eta)
{
    if (is_static(c)) return 1.0;
    if (eta <= 0.0) return 0.0;
    double lo = 0.0, hi = 1.0;
    while (or_eta_of_a(c, hi * hi) < eta) hi *= 2.0;
    double y = 0.5 * OR_H0 * sqrt(c->omega_m) * eta;
    if (!(y > lo && y < hi)) y = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        const double a = y * y;
        const double e = or_eta_of_a(c, a) - eta;
        if (e > 0) hi = y; else lo = y;
        double yn = y - e * 0.5 * y * a * hubble_of_a(c, a);
        if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);
        /* quadratic convergence: stop once the update is a few ulp */
        if (fabs(yn - y) <= 4e-16 * y) { y = yn; break; }
        y = yn;
    }
    return y * y;
}

/* a'/a = a H(a) = H0 sqrt(Om/a + OL a^2) */
double or_conformal_hubble(const or_cosmo* c, double eta)
{
    if (is_static(c)) return 0.0;
    const double a = or_a_of_eta(c, eta);
    return OR_H0 * sqrt(c->omega_m / a + c->omega_l * a * a);
}

/* d(a'/a)/d eta = d(aH)/da * da/d eta, da/d eta = a (a'/a) */
static double conformal_hubble_deriv(const or_cosmo* c, double eta)
{
    if (is_static(c)) return 0.0;
    const double a = or_a_of_eta(c, eta);
    const double s = sqrt(c->omega_m / a + c->omega_l * a * a);
    const double dHda = OR_H0 * (-c->omega_m / (a * a) + 2.0 * c->omega_l * a) / (2.0 * s);
    return dHda * a * (OR_H0 * s);
}

/* ------------------------------------------------------------------------- */
/* HEALPix NESTED pixel centres (Gorski et al. 2005)                          */
/* ------------------------------------------------------------------------- */
/* Within base face f the nested index interleaves the bits of the face
 * coordinates: x in the even bits, y in the odd bits.  The ring index counted
 * from the north pole is jrll[f] nside - x - y - 1; rings 1..nside-1 form the
 * north polar cap (z = 1 - i^2/(3 nside^2)), rings 3 nside+1 .. 4 nside-1 the
 * south cap, and the rest the equatorial belt (z = 4/3 - 2 i/(3 nside)).  The
 * azimuth of the centre is pi/4 (jpll[f] + (x - y)/nr) with nr = pixels per
 * ring quadrant. */
static const int jrll[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
static const int jpll[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};

static int64_t compact_bits(int64_t v)
{
    int64_t r = 0;
    for (int b = 0; b < 31; ++b) r |= ((v >> (2 * b)) & 1) << b;
    return r;
}

void or_pix2vec_nest(int64_t nside, int64_t pix, double vec[3])
{
    const int64_t npface = nside * nside;
    const int face = (int)(pix / npface);
    const int64_t ip = pix % npface;
    const int64_t ix = compact_bits(ip), iy = compact_bits(ip >> 1);
    const int64_t jr = jrll[face] * nside - ix - iy - 1;
    int64_t nr;
    double z, sth;
    const double fns2 = 3.0 * (double)nside * (double)nside;
    if (jr < nside) {
        nr = jr;
        const double omz = (double)(nr * nr) / fns2;       /* 1 - z */
        z = 1.0 - omz;
        sth = sqrt(omz * (2.0 - omz));
    } else if (jr > 3 * nside) {
        nr = 4 * nside - jr;
        const double opz = (double)(nr * nr) / fns2;       /* 1 + z */
        z = opz - 1.0;
        sth = sqrt(opz * (2.0 - opz));
    } else {
        nr = nside;
        z = (double)(2 * nside - jr) * 2.0 / (3.0 * (double)nside);
        sth = sqrt((1.0 - z) * (1.0 + z));
    }
    const double ph = 0.25 * M_PI * ((double)jpll[face] + (double)(ix - iy) / (double)nr);
    vec[0] = sth * cos(ph);
    vec[1] = sth * sin(ph);
    vec[2] = z;
}

/* e1 = e_phi, e2 = -e_theta at the direction n (screen basis of Sect. 2.3.2) */
static void tangent_basis(const double n[3], double e1[3], double e2[3])
{
    const double ph = atan2(n[1], n[0]);
    const double th = atan2(hypot(n[0], n[1]), n[2]);
    e1[0] = -sin(ph); e1[1] = cos(ph); e1[2] = 0.0;
    e2[0] = -cos(ph) * cos(th); e2[1] = -sin(ph) * cos(th); e2[2] = sin(th);
}

/* ------------------------------------------------------------------------- */
/* the two instantiations of the integrator                                  */
/* ------------------------------------------------------------------------- */
#define SC double
#define FN(name) name##_r
#define RE(z) (z)
#define CSQRT sqrt
#define CASIN asin
#define CLOG log
#define EXT1(f, df, z) (f)
#define CELLV(v, dv) (v)
#define SIGMA(st, c) atan2((st), (c))
#define TAN(z) 0.0
#include "oracle_core.inc"
#undef SC
#undef FN
#undef RE
#undef CSQRT
#undef CASIN
#undef CLOG
#undef EXT1
#undef CELLV
#undef SIGMA
#undef TAN

#define SC double complex
#define FN(name) name##_c
#define RE(z) creal(z)
#define CSQRT csqrt
#define CASIN casin
#define CLOG clog
#define EXT1(f, df, z) ((f) + I * cimag(z) * (df))
#define CELLV(v, dv) ((v) + I * (CS_H * (dv)))
#define SIGMA(st, c) casin(st)
#define TAN(z) (cimag(z) / CS_H)
#include "oracle_core.inc"

/* ------------------------------------------------------------------------- */
/* drivers                                                                    */
/* ------------------------------------------------------------------------- */
int or_field_probe(const or_field* f, const double x[3], double* phi, double grad[3],
                   int* leaf_level_out, int* stencil_level)
{
    cs_ctx ctx = {NULL, NULL};
    return eval_r(f, &ctx, x, phi, grad, NULL, leaf_level_out, stencil_level);
}

static int derive(const or_cosmo* c, const or_cast_params* p, derived_t* dv)
{
    if (or_cosmo_check(c)) return -1;
    dv->eta0 = or_eta0(c);
    if (p->stop_kind == OR_STOP_REDSHIFT) {
        if (is_static(c)) return -1;
        dv->a_s = 1.0 / (1.0 + p->stop_value);
        dv->eta_s = or_eta_of_a(c, dv->a_s);
    } else if (p->stop_kind == OR_STOP_CHI) {
        dv->eta_s = dv->eta0 - p->stop_value;
        dv->a_s = or_a_of_eta(c, dv->eta_s);
    } else {
        return -1;
    }
    if (p->dphidl != OR_DPHIDL_CHAIN && p->dphidl != OR_DPHIDL_DIFF) return -1;
    switch (p->surface) {
        case OR_SURF_ETA: dv->p_s = dv->eta_s; break;
        case OR_SURF_CHI: dv->p_s = dv->eta0 - dv->eta_s; break;
        case OR_SURF_LAMBDA:
            dv->p_s = is_static(c) ? dv->eta0 - dv->eta_s : or_lambda_of_a(c, dv->a_s);
            break;
        case OR_SURF_Z:
            if (is_static(c)) return -1;
            dv->p_s = -log(dv->a_s);
            break;
        default: return -1;
    }
    return 0;
}

typedef struct {
    const or_field* f;
    const or_cosmo* c;
    const or_cast_params* p;
    derived_t dv;
    int64_t n_rays;
    const double* dirs;
    const double* dtheta;
    cs_ctx ctx;
    or_ray_out* out;
    or_ray_tan* tan;
    double* A;            /* infinitesimal-beam output */
    double h_deriv;
    int mode;             /* 0 values, 1 complex step, 2 infinitesimal beam, 3 Born beam, 4 surfaces */
    int n_surf;           /* mode 4: stop surfaces, nearest first, and their outputs [n_surf][n_rays] */
    const derived_t* dvs;
    int64_t next;
    pthread_mutex_t lock;
} job_t;

static int64_t grab(job_t* J, int64_t* end)
{
    pthread_mutex_lock(&J->lock);
    const int64_t b = J->next;
    J->next = b + 8 < J->n_rays ? b + 8 : J->n_rays;
    *end = J->next;
    pthread_mutex_unlock(&J->lock);
    return b;
}

/* ---- infinitesimal beam sampler (Sect. 2.3.1) ---- */
typedef struct {
    const or_field* f;
    const double* obs;
    const double* n;
    double h_deriv;
    int64_t len, cap;
    double* s;            /* [len][4]: chi, T11, T12, T22 */
    int bad;
} inf_acc;

static void inf_sample(void* user, const double* y)
{
    inf_acc* A = (inf_acc*)user;
    const double* x = y + 1;
    double r[3] = {x[0] - A->obs[0], x[1] - A->obs[1], x[2] - A->obs[2]};
    const double chi = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double* dir = chi > 0 ? r : A->n;
    double e1[3], e2[3];
    tangent_basis(dir, e1, e2);
    /* derivation step: the size of the deepest cell containing the photon */
    double h = A->h_deriv;
    if (A->f->kind == OR_FIELD_GRID) {
        double u[3] = {x[0] / A->f->h0, x[1] / A->f->h0, x[2] / A->f->h0};
        const int L = leaf_level(A->f, u);
        h = A->f->h0 / ldexp(1.0, L < 0 ? 0 : L);
    }
    /* Hessian from centred differences of the interpolated force, Eq. (FD) */
    double H[3][3];
    for (int i = 0; i < 3; ++i) {
        double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
        xp[i] += h; xm[i] -= h;
        double pp, pm, gp[3], gm[3];
        if (or_field_probe(A->f, xp, &pp, gp, NULL, NULL) || or_field_probe(A->f, xm, &pm, gm, NULL, NULL)) {
            A->bad = 1;
            for (int j = 0; j < 3; ++j) H[i][j] = 0.0;
            continue;
        }
        for (int j = 0; j < 3; ++j) H[i][j] = (gp[j] - gm[j]) / (2.0 * h);
    }
    /* mixed derivatives taken as equal: symmetrise */
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j) { const double m = 0.5 * (H[i][j] + H[j][i]); H[i][j] = H[j][i] = m; }
    double T[2][2];
    const double* E[2] = {e1, e2};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) s += E[a][i] * H[i][j] * E[b][j];
            T[a][b] = s;
        }
    if (A->len == A->cap) {
        A->cap = A->cap ? 2 * A->cap : 1024;
        A->s = (double*)realloc(A->s, sizeof(double) * 4 * (size_t)A->cap);
    }
    double* s = A->s + 4 * A->len++;
    s[0] = chi; s[1] = T[0][0]; s[2] = T[0][1]; s[3] = T[1][1];
}

static void* worker(void* arg)
{
    job_t* J = (job_t*)arg;
    inf_acc acc = {0};
    for (;;) {
        int64_t end;
        const int64_t b = grab(J, &end);
        if (b >= J->n_rays) break;
        for (int64_t r = b; r < end; ++r) {
            const double* n = J->dirs + 3 * r;
            if (J->mode == 1) {
                double complex nc[3] = {n[0], n[1], n[2]};
                if (J->dtheta) {
                    double e1[3], e2[3];
                    tangent_basis(n, e1, e2);
                    for (int i = 0; i < 3; ++i)
                        nc[i] += I * CS_H * (J->dtheta[2 * r] * e1[i] + J->dtheta[2 * r + 1] * e2[i]);
                }
                trace_t_c R;
                trace_c(J->f, &J->ctx, J->c, J->p, &J->dv, nc, &R, NULL, NULL);
                observe_c(J->c, J->p, &J->dv, n, &R, J->out ? J->out + r : NULL, J->tan ? J->tan + r : NULL);
            } else if (J->mode == 2) {
                acc.f = J->f; acc.obs = J->p->obs; acc.n = n; acc.h_deriv = J->h_deriv;
                acc.len = 0; acc.bad = 0;
                trace_t_r R;
                trace_r(J->f, &J->ctx, J->c, J->p, &J->dv, n, &R, inf_sample, &acc);
                observe_r(J->c, J->p, &J->dv, n, &R, J->out ? J->out + r : NULL, NULL);
                double* A = J->A + 4 * r;
                A[0] = 1.0; A[1] = 0.0; A[2] = 0.0; A[3] = 1.0;
                if (R.status != OR_REACHED || acc.len < 2) continue;
                /* A_ab = delta_ab - 2 int_0^chi_s (chi_s - chi) chi / chi_s T_ab dchi  (trapezoid) */
                const double chis = acc.s[4 * (acc.len - 1)];
                double I11 = 0.0, I12 = 0.0, I22 = 0.0;
                for (int64_t i = 0; i + 1 < acc.len; ++i) {
                    const double* s0 = acc.s + 4 * i;
                    const double* s1 = acc.s + 4 * (i + 1);
                    const double w0 = (chis - s0[0]) * s0[0] / chis, w1 = (chis - s1[0]) * s1[0] / chis;
                    const double dc = 0.5 * (s1[0] - s0[0]);
                    I11 += dc * (w0 * s0[1] + w1 * s1[1]);
                    I12 += dc * (w0 * s0[2] + w1 * s1[2]);
                    I22 += dc * (w0 * s0[3] + w1 * s1[3]);
                }
                A[0] = 1.0 - 2.0 * I11; A[1] = -2.0 * I12; A[2] = -2.0 * I12; A[3] = 1.0 - 2.0 * I22;
            } else if (J->mode == 4) {
                /* one photon through several stop surfaces: land on each in turn
                 * (the landing step ends exactly on it), record the observables
                 * there, and continue from the landed state to the next */
                trace_t_r R;
                const int bad = trace_start_r(J->f, &J->ctx, J->c, J->p, &J->dvs[0], n, &R);
                for (int k = 0; k < J->n_surf; ++k) {
                    if (!bad && (k == 0 || R.status == OR_REACHED)) {
                        R.status = -1;
                        trace_run_r(J->f, &J->ctx, J->c, J->p, &J->dvs[k], &R, NULL, NULL);
                        trace_end_r(J->f, &J->ctx, &R, NULL, NULL);
                    }
                    observe_r(J->c, J->p, &J->dvs[k], n, &R, J->out + (int64_t)k * J->n_rays + r, NULL);
                }
            } else if (J->mode == 3) {
                /* Born approximation: the same line-of-sight integral along the
                 * straight line x = x_obs + chi n, sampled with the step rule of
                 * the integration (h_leaf / N, or ds for closed-form fields) from
                 * chi = 0 to the stop surface's comoving distance */
                acc.f = J->f; acc.obs = J->p->obs; acc.n = n; acc.h_deriv = J->h_deriv;
                acc.len = 0; acc.bad = 0;
                const double chis = J->dv.eta0 - J->dv.eta_s;
                double chi = 0.0;
                int status = OR_MAX_STEPS;
                int64_t steps = 0;
                for (;;) {
                    double y[S_N] = {0};
                    for (int i = 0; i < 3; ++i) y[S_X + i] = J->p->obs[i] + chi * n[i];
                    double ds = J->p->ds_analytic;
                    if (J->f->kind == OR_FIELD_GRID) {
                        double u[3] = {y[S_X] / J->f->h0, y[S_X + 1] / J->f->h0, y[S_X + 2] / J->f->h0};
                        const int leaf = leaf_level(J->f, u);
                        if (leaf < 0) { status = OR_LEFT_DOMAIN; break; }
                        const int lstep = J->p->adaptive ? leaf : 0;
                        ds = J->f->h0 / ldexp(1.0, lstep) / (double)J->p->steps_per_cell;
                    }
                    inf_sample(&acc, y);
                    if (chi >= chis) { status = OR_REACHED; break; }
                    if (steps >= J->p->max_steps) break;
                    chi = chi + ds < chis ? chi + ds : chis;
                    ++steps;
                }
                if (J->out) { memset(J->out + r, 0, sizeof(or_ray_out)); J->out[r].status = status; J->out[r].n_steps = steps; }
                double* A = J->A + 4 * r;
                A[0] = 1.0; A[1] = 0.0; A[2] = 0.0; A[3] = 1.0;
                if (status != OR_REACHED || acc.len < 2) continue;
                const double cs = acc.s[4 * (acc.len - 1)];
                double I11 = 0.0, I12 = 0.0, I22 = 0.0;
                for (int64_t i = 0; i + 1 < acc.len; ++i) {
                    const double* s0 = acc.s + 4 * i;
                    const double* s1 = acc.s + 4 * (i + 1);
                    const double w0 = (cs - s0[0]) * s0[0] / cs, w1 = (cs - s1[0]) * s1[0] / cs;
                    const double dc = 0.5 * (s1[0] - s0[0]);
                    I11 += dc * (w0 * s0[1] + w1 * s1[1]);
                    I12 += dc * (w0 * s0[2] + w1 * s1[2]);
                    I22 += dc * (w0 * s0[3] + w1 * s1[3]);
                }
                A[0] = 1.0 - 2.0 * I11; A[1] = -2.0 * I12; A[2] = -2.0 * I12; A[3] = 1.0 - 2.0 * I22;
            } else {
                trace_t_r R;
                trace_r(J->f, &J->ctx, J->c, J->p, &J->dv, n, &R, NULL, NULL);
                observe_r(J->c, J->p, &J->dv, n, &R, J->out + r, NULL);
            }
        }
    }
    free(acc.s);
    return NULL;
}

static int run_job(job_t* J, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    J->next = 0;
    pthread_mutex_init(&J->lock, NULL);
    pthread_t th[256];
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, worker, J);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J->lock);
    return 0;
}

static int setup(job_t* J, const or_field* f, const or_cosmo* c, const or_cast_params* p,
                 int64_t n_rays, const double* dirs)
{
    memset(J, 0, sizeof *J);
    if (!f || !c || !p || !dirs || n_rays < 0) return -1;
    if (f->kind == OR_FIELD_GRID && p->steps_per_cell < 1) return -1;
    if (f->kind != OR_FIELD_GRID && !(p->ds_analytic > 0)) return -1;
    if (derive(c, p, &J->dv)) return -1;
    J->f = f; J->c = c; J->p = p; J->n_rays = n_rays; J->dirs = dirs;
    return 0;
}

int or_cast(const or_field* f, const or_cosmo* c, const or_cast_params* p, int64_t n_rays,
            const double* dirs, or_ray_out* out, int n_threads)
{
    job_t J;
    if (setup(&J, f, c, p, n_rays, dirs) || !out) return -1;
    J.out = out;
    J.mode = 0;
    return run_job(&J, n_threads);
}

int or_cast_cs(const or_field* f, const or_cosmo* c, const or_cast_params* p, int64_t n_rays,
               const double* dirs, const double* dtheta, const double* dphi, const double* dgrad,
               or_ray_out* out, or_ray_tan* tan, int n_threads)
{
    job_t J;
    if (setup(&J, f, c, p, n_rays, dirs) || !tan) return -1;
    J.out = out; J.tan = tan; J.dtheta = dtheta;
    J.ctx.dphi = dphi; J.ctx.dgrad = dgrad;
    J.mode = 1;
    return run_job(&J, n_threads);
}

int or_infinitesimal(const or_field* f, const or_cosmo* c, const or_cast_params* p, int64_t n_rays,
                     const double* dirs, double h_deriv, double* A, or_ray_out* out, int n_threads)
{
    job_t J;
    if (setup(&J, f, c, p, n_rays, dirs) || !A) return -1;
    J.A = A; J.out = out; J.h_deriv = h_deriv;
    J.mode = 2;
    return run_job(&J, n_threads);
}

int or_cast_surfaces(const or_field* f, const or_cosmo* c, const or_cast_params* p, int n_surf,
                     const double* stops, int64_t n_rays, const double* dirs, or_ray_out* out, int n_threads)
{
    job_t J;
    if (n_surf < 1 || n_surf > 64 || !stops || p->surface != OR_SURF_ETA || setup(&J, f, c, p, n_rays, dirs) ||
        !out)
        return -1;
    derived_t dvs[64];
    for (int k = 0; k < n_surf; ++k) {
        or_cast_params q = *p;
        q.stop_value = stops[k];
        if (derive(c, &q, &dvs[k])) return -1;
        if (k > 0 && !(dvs[k].eta_s < dvs[k - 1].eta_s)) return -1;   /* nearest first */
    }
    J.out = out;
    J.n_surf = n_surf;
    J.dvs = dvs;
    J.mode = 4;
    return run_job(&J, n_threads);
}

int or_born(const or_field* f, const or_cosmo* c, const or_cast_params* p, int64_t n_rays,
            const double* dirs, double h_deriv, double* A, or_ray_out* out, int n_threads)
{
    job_t J;
    if (p->surface != OR_SURF_ETA || setup(&J, f, c, p, n_rays, dirs) || !A) return -1;
    J.A = A; J.out = out; J.h_deriv = h_deriv;
    J.mode = 3;
    return run_job(&J, n_threads);
}

int or_integrate_steps(const or_field* f, const or_cosmo* c, double* y, int64_t n, const double* dl)
{
    cs_ctx ctx = {NULL, NULL};
    double s[S_N] = {0}, out[S_N];
    memcpy(s, y, 8 * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        const int st = rk4_r(f, &ctx, c, s, dl[i], out, NULL, NULL, NULL);
        if (st) return st;
        memcpy(s, out, sizeof out);
    }
    memcpy(y, s, 8 * sizeof(double));
    return 0;
}
