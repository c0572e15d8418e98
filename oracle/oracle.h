/*
 * oracle.h -- plain FP64 CPU oracle for backward null-geodesic ray tracing
 * through an AMR octree of the gravitational potential (Breton & Reverdy,
 * "Magrathea-Pathfinder", Sect. 2.2-2.4).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU library and is written for readability, not speed: one photon
 * per thread, scalar double precision, hash-table octree lookups.
 *
 * Units: c = 1, lengths and conformal time in Mpc/h, Phi = Phi/c^2.
 */
#ifndef MPATH_ORACLE_H
#define MPATH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Cosmology: flat LCDM with Omega_r = 0 (omega_m + omega_l == 1), or the
 * static case omega_m == omega_l == 0 (a == 1, conformal Hubble rate 0,
 * eta_0 = 0).  h only sets the unit convention (lengths in Mpc/h). */
typedef struct { double omega_m, omega_l, h; } or_cosmo;

/* Field kinds. GRID is an octree of cells; the others are closed-form fields
 * used by the pins. */
enum { OR_FIELD_GRID = 0, OR_FIELD_LINEAR = 1, OR_FIELD_QUADRATIC = 2, OR_FIELD_POINT = 3 };

typedef struct or_field or_field;

/* Build a grid field from a cell list of a full octree.  level[i], ijk[i][3]
 * (coordinates at the cell's own level), phi[i], grad[i][3].  Arrays are
 * copied.  Returns NULL and writes a message into err on invalid trees. */
or_field* or_field_grid(double box, int n0, int max_level, int periodic, int64_t n_cells,
                        const uint8_t* level, const int32_t* ijk, const double* phi,
                        const double* grad, char* err, int errlen);
/* Closed-form fields:
 *   LINEAR    params = {phi0, gx, gy, gz}                       Phi = phi0 + g.x
 *   QUADRATIC params = {phi0, cx,cy,cz, Hxx,Hxy,Hxz,Hyy,Hyz,Hzz} Phi = phi0 + (x-c)^T H (x-c)/2
 *   POINT     params = {m, cx,cy,cz, soft}                      Phi = -m / sqrt(|x-c|^2 + soft^2) */
or_field* or_field_analytic(int kind, const double* params);
void or_field_free(or_field* f);
/* Interpolation scheme of a grid field (Sect. 2.2, weights W_NGP, W_CIC,
 * W_TSC): 0 NGP (the deepest cell containing x), 1 CIC (default, 8 cells),
 * 2 TSC (27 cells centred on the cell containing x), CIC and TSC with the
 * level fallback.  Returns 0, or -1 for a bad order or a closed-form field. */
int or_field_set_order(or_field* f, int order);
/* Time derivative of the potential per cell (a grid field; NULL: static).
 * With it the geodesic equations take their dPhi/deta terms and each ray
 * carries the ISW integral (Sect. 2.2, Sect. 2.5 z4).  The values are
 * copied; they are interpolated with the weights of the potential. */
int or_field_set_tdot(or_field* f, const double* tdot);

/* Interpolation probe at a point: Phi, grad Phi, the leaf level (deepest
 * existing cell containing x) and the level the stencil was taken at.
 * Returns 0, or 1 when no complete stencil exists even at the coarse level. */
int or_field_probe(const or_field* f, const double x[3], double* phi, double grad[3],
                   int* leaf_level, int* stencil_level);

/* ---- cosmology ---- */
int    or_cosmo_check(const or_cosmo* c);
double or_eta_of_a(const or_cosmo* c, double a);
double or_a_of_eta(const or_cosmo* c, double eta);
double or_conformal_hubble(const or_cosmo* c, double eta);   /* a'/a */
double or_eta0(const or_cosmo* c);
/* Affine parameter of the FLRW photon (k0 = -1 at a = 1) from the observer
 * to scale factor a: int_a^1 da' / H(a') (a^2 d eta = da / H). */
double or_lambda_of_a(const or_cosmo* c, double a);

/* ---- HEALPix (NESTED scheme) pixel centre as a unit vector ---- */
void or_pix2vec_nest(int64_t nside, int64_t pix, double vec[3]);

/* ---- ray casting ---- */
enum { OR_STOP_REDSHIFT = 0, OR_STOP_CHI = 1 };
/* The surface a photon stops on (Sect. 2.4: maps on iso-p surfaces): the
 * parameter p of the photon takes the value an FLRW photon has on the stop
 * of stop_kind / stop_value.  ETA: eta = eta_s (iso-a too); CHI: comoving
 * distance |x - x_obs| = eta_0 - eta_s; LAMBDA: affine parameter
 * lambda = int a^2 d eta (k0 = -1 at the observer) of the FLRW photon;
 * Z: observed redshift z5 = 1/a_s - 1. */
enum { OR_SURF_ETA = 0, OR_SURF_CHI = 1, OR_SURF_LAMBDA = 2, OR_SURF_Z = 3 };
/* dPhi/dlambda in the geodesic equations (Sect. 2.2): CHAIN the chain rule
 * grad Phi . k + (dPhi/deta) k0 (Eq. dPhi/dl, first form); DIFF the
 * equations written with dPhi/dl only, which is estimated per step as the
 * difference of Phi between the last two step starts over the affine
 * length between them (Eq. dPhi/dl, second form; the first step takes
 * grad Phi . k at the observer). */
enum { OR_DPHIDL_CHAIN = 0, OR_DPHIDL_DIFF = 1 };
enum { OR_REACHED = 0, OR_LEFT_DOMAIN = 1, OR_MAX_STEPS = 2, OR_NONFINITE = 3 };

typedef struct {
    double obs[3];        /* observer position */
    int    stop_kind;     /* OR_STOP_REDSHIFT: stop_value = z_src; OR_STOP_CHI: eta_s = eta_0 - stop_value */
    double stop_value;
    int    steps_per_cell;/* N: comoving step length = h / N */
    int    adaptive;      /* 1: h of the leaf cell at the step start; 0: coarse h */
    double ds_analytic;   /* step length for closed-form fields */
    int64_t max_steps;
    int    surface;       /* OR_SURF_*: the stop surface */
    int    dphidl;        /* OR_DPHIDL_* */
} or_cast_params;

typedef struct {
    double theta[2];      /* (polar, azimuth) of the initial direction */
    double beta[2];       /* (polar, azimuth) of x_s - x_obs */
    double alpha[2];      /* deflection theta - beta, components on e1 = e_phi(theta), e2 = -e_theta(theta) */
    double sep2;          /* squared great-circle angle between theta and beta */
    double z5, z0, z1;    /* observed redshift (Eq. z5, v = 0), FLRW redshift, FLRW + potential */
    double z4;            /* z1 + ISW term (Eq. z4 with v = 0) */
    double isw;           /* integral of dPhi/deta d eta from eta_s to eta_0 along the ray */
    double phi_o, phi_s;  /* potential at the observer and at the end point */
    double chi;           /* |x_s - x_obs| */
    double r[3];          /* x_s - x_obs (unwrapped) */
    double k[4];          /* final (k^0, k^1, k^2, k^3) */
    double eta;           /* final conformal time */
    double lam;           /* final affine parameter */
    double max_null;      /* max over step starts of |null condition| */
    int64_t n_steps;
    int32_t status;
    uint32_t hash;        /* FNV-1a over the discrete decisions (levels) taken along the ray */
} or_ray_out;

/* Directional derivative of the outputs (complex-step, exact to rounding). */
typedef struct {
    double r[3], k[4], z5, phi_s, alpha[2], sep2, eta;
} or_ray_tan;

int or_cast(const or_field* f, const or_cosmo* c, const or_cast_params* p, int64_t n_rays,
            const double* dirs, or_ray_out* out, int n_threads);

/* Derivative along one direction of the inputs: dtheta[n][2] perturbs each
 * initial direction along (e1, e2); dphi[n_cells], dgrad[n_cells][3] perturb
 * the cell values (grid fields).  Any of them may be NULL. */
int or_cast_cs(const or_field* f, const or_cosmo* c, const or_cast_params* p, int64_t n_rays,
               const double* dirs, const double* dtheta, const double* dphi, const double* dgrad,
               or_ray_out* out, or_ray_tan* tan, int n_threads);

/* Infinitesimal-beam distortion matrix (Sect. 2.3.1) along each ray:
 * A[n][2][2] on the basis e1 = e_phi, e2 = -e_theta.  h_deriv is the
 * derivation step for closed-form fields (grid fields use the leaf cell size). */
int or_infinitesimal(const or_field* f, const or_cosmo* c, const or_cast_params* p, int64_t n_rays,
                     const double* dirs, double h_deriv, double* A, or_ray_out* out, int n_threads);

/* Plain RK4 over given affine steps from state y[8] = (eta, x, k0, k); used
 * by the time-reversal pin.  Returns 0 or the status of a failed stage. */
/* One cast through several stop surfaces (stops[k], nearest first, of
 * p->stop_kind; p->stop_value is not used): each photon lands on every
 * surface in turn and continues from there.  out[k * n_rays + r] holds the
 * observables of ray r on surface k (steps and hash cumulative). */
int or_cast_surfaces(const or_field* f, const or_cosmo* c, const or_cast_params* p, int n_surf,
                     const double* stops, int64_t n_rays, const double* dirs, or_ray_out* out, int n_threads);
/* Born approximation of the same matrix: the line-of-sight integral of
 * or_infinitesimal taken along the straight line x_obs + chi n (n = dirs[r])
 * from chi = 0 to the stop surface's comoving distance eta_0 - eta_s, sampled
 * at chi_{i+1} = min(chi_i + ds_i, chi_s) with ds_i the integration's step
 * rule at x(chi_i).  out (optional) receives status and the sample count. */
int or_born(const or_field* f, const or_cosmo* c, const or_cast_params* p, int64_t n_rays,
            const double* dirs, double h_deriv, double* A, or_ray_out* out, int n_threads);
int or_integrate_steps(const or_field* f, const or_cosmo* c, double* y, int64_t n, const double* dl);

#ifdef __cplusplus
}
#endif
#endif
