/*
 * mpath.h -- C ABI of the MI355X (gfx950) weak-field null-geodesic ray tracer.
 *
 * The method is the backward ray tracing of Breton & Reverdy,
 * "Magrathea-Pathfinder: A 3D adaptive-mesh code for geodesic ray tracing in
 * N-body simulations" (Sect. 2): photons leave an observer along HEALPix pixel
 * centres (Sect. 2.4), follow the null geodesic equations of the perturbed
 * FLRW metric in Newtonian gauge (Sect. 2.2, metric and geodesic equations),
 * integrated by RK4 with N steps per AMR cell, with Phi and grad Phi
 * interpolated at every RK4 sub-step by cloud-in-cell weights on an octree,
 * falling back to coarser levels where a finer stencil is incomplete
 * (Sect. 2.2, the five-step procedure), and stop on the source's iso-eta
 * surface, returning the lens-equation deflection (Sect. 2.3) and the
 * redshifts of Sect. 2.5.
 *
 * Conventions
 *   c = 1; lengths and conformal time eta in Mpc/h; phi = Phi/c^2;
 *   angles in radians; H0 = 100 h km/s/Mpc = 1/2997.92458 h/Mpc.
 *   Backward tracing starts with k^0 = -1 at the observer (a0 = 1).
 *
 * Memory ownership
 *   The library never allocates device memory.  Every call that needs device
 *   storage first reports its size (..._workspace_bytes); the caller
 *   allocates it (e.g. a torch tensor) and passes a raw device pointer.  All
 *   *_desc input arrays documented as HOST are read during the call only.
 *   Output arrays are caller-allocated DEVICE arrays.
 *
 * Streams and errors
 *   Every entry point takes a hipStream_t (as void*; NULL = the null stream)
 *   and returns an int status: MPATH_OK (0) or a negative MPATH_ERR_* code;
 *   no C++ exception crosses the ABI.  mpath_last_error() gives a
 *   human-readable message for the calling thread's last failure.  Kernel
 *   work is asynchronous on the stream; per-ray conditions (a ray that leaves
 *   a non-periodic domain, exceeds max_steps or becomes non-finite) are
 *   reported in the status[] output, not as call errors.
 */
#ifndef MPATH_H
#define MPATH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- call status ---- */
#define MPATH_OK 0
#define MPATH_ERR_INVALID_ARG (-1)          /* a NULL/negative/out-of-range argument  */
#define MPATH_ERR_NOT_FULL_TREE (-2)        /* the cell list is not a full octree      */
#define MPATH_ERR_WORKSPACE_TOO_SMALL (-3)  /* ws_bytes below the reported size        */
#define MPATH_ERR_DEVICE (-4)               /* a HIP runtime error (text in last_error) */
#define MPATH_ERR_UNSUPPORTED (-5)          /* a valid but not implemented option      */

/* ---- per-ray status (status[] output) ---- */
#define MPATH_RAY_REACHED 0      /* stopped on the source surface                          */
#define MPATH_RAY_LEFT_DOMAIN 1  /* no complete stencil even at the coarse level (Sect. 2.2,
                                    fifth step): only on non-periodic grids               */
#define MPATH_RAY_MAX_STEPS 2    /* max_steps reached before the source                   */
#define MPATH_RAY_NONFINITE 3    /* the state became NaN/Inf                              */

/* ---- value types of the input cell data ---- */
#define MPATH_F64 0
#define MPATH_F32 1

/* Background cosmology: flat LCDM with Omega_r = 0 (omega_m + omega_l == 1,
 * omega_m > 0), or the static case omega_m == omega_l == 0 (a == 1, a'/a = 0,
 * eta_0 = 0; only usable with stop_kind == MPATH_STOP_CHI).  The conformal
 * Hubble rate a'/a (Sect. 2.2 reads a(eta), a'(eta) from precomputed tables)
 * is tabulated by the library in double precision. */
typedef struct {
    double omega_m, omega_l, h;
} mpath_cosmo;

/* The octree of the gravitational potential (Sect. 2.1): a flat list of every
 * cell, internal and leaf, of a FULL tree (each cell has 0 or 8 children;
 * every coarse cell present).  All arrays are HOST arrays of length n_cells:
 *   level[i]    refinement level (0 = coarse, <= max_level)
 *   ijk[i][3]   integer coordinates at the cell's own level, in [0, n0 2^level)
 *   phi[i]      potential at the cell centre (each cell, internal or leaf,
 *               carries its own value: used when interpolating at its level)
 *   grad[i][3]  gradient of the potential at the cell centre, or grad == NULL:
 *               the library takes second-order central differences of phi
 *               between the two neighbours of the cell at its own level
 *               (periodic wrap on periodic grids), (phi[+] - phi[-]) / (2 h_l)
 *               in double precision, h_l = box / (n0 2^l); where only one
 *               neighbour exists at that level (the edge of a refined region
 *               or of a non-periodic box) the one-sided difference with it,
 *               and 0 where neither does.  Sect. 2.1 stores the force with
 *               the potential; this is the gradient such grids carry.
 *   dphi_deta[i] optional (NULL: a static potential): the time derivative of
 *               the potential at the cell centre (Sect. 2.2; from two light
 *               cones shifted in time, see mpath_double_layer).  A grid that
 *               carries it is integrated with the dPhi/deta terms of the
 *               geodesic equations and yields the ISW integral and z4.
 * value_dtype says whether phi, grad and dphi_deta are double or float.  Cell (l, i)
 * covers [i h_l, (i+1) h_l) per axis with h_l = box / (n0 2^l); n0 must be a
 * power of two (<= 1024) and max_level <= 10.  periodic != 0 replicates the
 * box (rays may travel further than the box size); otherwise cells outside
 * the box do not exist. */
typedef struct {
    double box;
    int32_t n0;
    int32_t max_level;
    int32_t periodic;
    int32_t value_dtype;
    int64_t n_cells;
    const uint8_t* level;
    const int32_t* ijk;
    const void* phi;
    const void* grad;
    const void* dphi_deta;
} mpath_grid_desc;

typedef struct mpath_grid mpath_grid;   /* opaque host handle */

/* Device workspace needed by mpath_grid_build for this tree: the image every
 * cast reads, 148 B per cell (payload 16 B, child link 4 B, stencil record
 * 128 B) plus 32 B per refined cell (level >= 1: the stencil of each
 * half-cell), 36 B more per cell with dphi_deta, the background tables and a
 * 64 MB staging area used during the build. */
int mpath_grid_workspace_bytes(const mpath_grid_desc* desc, size_t* bytes);

/* Device workspace of the grid's auxiliary tables, 40 B per cell: the
 * caller's index of every library cell and the 8 cell ids of every stencil.
 * Only mpath_grid_set_values and the cell cotangents of mpath_adjoint
 * (dL_dvalues, dL_dphi_total) read them; a grid built without them casts,
 * differentiates per ray (distortion matrix, dz/dtheta) and runs every
 * product the same. */
int mpath_grid_aux_bytes(const mpath_grid_desc* desc, size_t* bytes);

/* Validate the tree (MPATH_ERR_NOT_FULL_TREE if a cell's parent is missing, a
 * refined cell has 1-7 children, a coarse cell is missing or a cell repeats),
 * order it (coarse cells in Morton order, then blocks of 8 siblings level by
 * level), pack (phi, grad) to float32 and upload into dev_ws on the stream.
 * Synchronises the stream before returning, also when the upload or the
 * build fails part way; the host arrays may be freed afterwards.  *out receives a handle that refers to dev_ws: dev_ws must
 * outlive the handle. */
int mpath_grid_build(const mpath_grid_desc* desc, const mpath_cosmo* cosmo, void* dev_ws,
                     size_t ws_bytes, void* stream, mpath_grid** out);

/* mpath_grid_build plus the auxiliary tables in aux_ws (aux_bytes >=
 * mpath_grid_aux_bytes; a DEVICE buffer the caller owns and keeps alive with
 * dev_ws).  aux_ws == NULL is mpath_grid_build.  Errors as mpath_grid_build,
 * and WORKSPACE_TOO_SMALL for aux_bytes. */
int mpath_grid_build_with_aux(const mpath_grid_desc* desc, const mpath_cosmo* cosmo, void* dev_ws,
                              size_t ws_bytes, void* aux_ws, size_t aux_bytes, void* stream, mpath_grid** out);

/* dPhi/deta of every cell from a double-layer light cone (Sect. 2.2, the
 * equation for dPhi/deta from two light cones slightly shifted in time):
 *   dphi_deta[i] = (phi2[i] - phi1[i]) / (a2[i] - a1[i]) * a'(a_m),
 * where phi1, phi2 are the potential of cell i on the two cones, a1, a2 the
 * scale factors of the cell on them, and the conformal-time derivative
 * a' = da/deta = a (a'/a) of the background is taken at a_m = (a1 + a2)/2
 * (the centre of the difference quotient).  All arrays are HOST arrays of n
 * doubles; dphi_deta may alias neither input.  MPATH_ERR_INVALID_ARG when a
 * cell has a1 == a2 or a non-positive scale factor; MPATH_ERR_UNSUPPORTED
 * for the static background.  Runs on the host (grid ingest). */
int mpath_double_layer(int64_t n, const double* phi1, const double* phi2, const double* a1, const double* a2,
                       const mpath_cosmo* cosmo, double* dphi_deta);

/* Pixel-centre directions of the NESTED HEALPix pixels pix_first ..
 * pix_first + count - 1 at resolution nside (Sect. 2.4: the initial
 * directions of the maps), the unit vectors the casts start along when
 * mpath_cast_desc.dirs is NULL.  dirs: DEVICE double[count][3], written
 * asynchronously on the stream.  Errors: INVALID_ARG (nside outside
 * [1, 8192], a range outside the 12 nside^2 pixels, dirs NULL with
 * count > 0), DEVICE. */
int mpath_healpix_dirs(int32_t nside, int64_t pix_first, int64_t count, double* dirs, void* stream);

/* Release the handle (not dev_ws, which the caller owns). */
int mpath_grid_free(mpath_grid* grid);

typedef struct {
    int64_t n_cells;
    int32_t n0, max_level, periodic;
    double box;
    double eta0;              /* conformal time today */
    int64_t cells_per_level[16];
    float* payload;           /* DEVICE [n_cells][4] (phi, gx, gy, gz), library order */
    const int64_t* perm;      /* DEVICE [n_cells]: user index of library cell i (NULL
                                 without the auxiliary tables) */
} mpath_grid_info;

int mpath_grid_get_info(const mpath_grid* grid, mpath_grid_info* info);

/* Replace the cell values from a DEVICE array values[n_cells][4] = (phi, gx,
 * gy, gz) float32 in the caller's original cell order (asynchronous).
 * MPATH_ERR_UNSUPPORTED for a grid without its auxiliary tables. */
int mpath_grid_set_values(mpath_grid* grid, const float* values, void* stream);

/* ---- casting rays ---- */
#define MPATH_STOP_REDSHIFT 0   /* stop_value[j] = z_src: eta_s = eta(a = 1/(1+z_src))         */
#define MPATH_STOP_CHI 1        /* stop_value[j] = comoving distance: eta_s = eta_0 - value    */

#define MPATH_SURFACE_ETA 0     /* stop surfaces (mpath_cast_desc.stop_surface)                  */
#define MPATH_SURFACE_CHI 1
#define MPATH_SURFACE_LAMBDA 2
#define MPATH_SURFACE_Z 3

#define MPATH_DPHIDL_CHAIN 0    /* dPhi/dlambda (mpath_cast_desc.dphidl)                         */
#define MPATH_DPHIDL_DIFF 1

#define MPATH_SCHED_AUTO 0      /* library choice (persistent when many observers/uneven rays) */
#define MPATH_SCHED_STATIC 1    /* one lane per ray, one launch                                 */
#define MPATH_SCHED_PERSISTENT 2/* resident waves pull ray batches from a global queue          */

typedef struct {
    /* observers: HOST arrays */
    int32_t n_obs;
    const double* obs_pos;      /* [n_obs][3] observer positions */
    const double* stop_value;   /* [n_obs] per stop_kind */
    int32_t stop_kind;
    /* sky pixels (Sect. 2.4): NESTED HEALPix at nside; observer j casts the
       pixel range [pix_first[j], pix_first[j] + pix_count[j]); rays are
       numbered observer by observer, in pixel order.  pix_first/pix_count
       NULL = the full sky for every observer. */
    int32_t nside;
    const int64_t* pix_first;
    const int64_t* pix_count;
    /* integration (Sect. 2.2) */
    int32_t order;              /* interpolation (Sect. 2.2): 0 NGP, 1 CIC, 2 TSC; NGP and
                                   TSC run the static schedule and support neither
                                   checkpoints (the adjoint) nor the infinitesimal beam */
    int32_t steps_per_cell;     /* N >= 1: comoving step length h / N                   */
    int32_t adaptive;           /* 1: h of the leaf cell at the step start; 0: coarse h */
    int64_t max_steps;          /* per ray, including the landing step (at most 2^31-1)  */
    /* launch shape; 0 = library default (mpath_autotune picks them by timing) */
    int32_t schedule;
    int32_t block_size;         /* threads per block: 0 or 256                          */
    int32_t waves_per_cu;       /* persistent schedule: resident waves per CU            */
    int32_t batch;              /* persistent schedule: rays per queue pop per wave (64k)*/
    /* adjoint support: 0 = forward only; K > 0 = store every ray's state
       before steps 0, K, 2K, ... for mpath_adjoint.  A checkpointed cast runs
       the static schedule (schedule, waves_per_cu and batch are ignored) and
       sizes its checkpoints for at most
       min(max_steps, 1.02 (eta_0 - eta_s) / ds_min + 16) steps per ray
       (ds_min the smallest comoving step length), rounded up to a multiple
       of K; a ray that would need more ends with MPATH_RAY_MAX_STEPS. */
    int32_t checkpoint_every;
    /* initial directions: NULL = the NESTED pixel centres above; else a
       DEVICE array [n_rays][3] of unit vectors (norm 1 to rounding), ray r
       starting along dirs[r].  With dirs, pix_first is ignored (may be NULL)
       and pix_count[j] (NULL: 12 nside^2 each) is the number of rays of
       observer j.  The array is read during the call (copied to the
       workspace before the integration starts). */
    const double* dirs;
    /* intermediate stop surfaces (the maps at several source redshifts of one
       run): 0 = none; else n_surfaces (<= 64) more surfaces per observer,
       HOST surface_stops[n_obs][n_surfaces] of stop_kind, nearest first and
       each nearer than stop_value[j].  Every photon lands exactly on each
       surface in turn (as on its final stop) and continues from there; the
       outputs then hold n_surfaces + 1 blocks of n_rays entries, block k
       for surface k and the last block for stop_value (steps and hash
       cumulative).  Static schedule; order 1 and checkpoint_every 0 only. */
    int32_t n_surfaces;
    const double* surface_stops;
    /* the parameter the stop surface holds (Sect. 2.4: maps on iso-p
       surfaces, p in {a, eta, chi, z, lambda}, at the value p_n an FLRW
       photon takes on the stop of stop_kind / stop_value):
         MPATH_SURFACE_ETA     conformal time eta_s (iso-a too; the default)
         MPATH_SURFACE_CHI     comoving distance |x - x_obs| = eta_0 - eta_s
         MPATH_SURFACE_LAMBDA  affine parameter (k0 = -1 at the observer) of
                               the FLRW photon, int_{a_s}^1 da / H(a)
         MPATH_SURFACE_Z       observed redshift z5 = 1/a_s - 1
       A photon stops where its own parameter reaches that value: on the
       iso-eta surface the step that would cross it is solved by Newton
       iterations; on the others the step that reaches the surface is taken
       again from its start with the length that Newton iterations on
       p(RK4(dl)) - p_n give (two iterations from the linear prediction, then
       the step; iso-lambda: the remaining length exactly).  The observables
       then refer to the end point's own scale factor a(eta) (z0 = 1/a - 1).
       Non-eta surfaces: order 1, static potential, n_surfaces 0,
       checkpoint_every 0 (no adjoint), static schedule; MPATH_SURFACE_Z
       needs an expanding background. */
    int32_t stop_surface;
    /* dPhi/dlambda in the geodesic equations (Sect. 2.2):
         MPATH_DPHIDL_CHAIN  the chain rule grad Phi . k + (dPhi/deta) k0 at
                             every RK4 stage (Eq. dPhi/dl, first form; the default)
         MPATH_DPHIDL_DIFF   the equations written with dPhi/dlambda only
                             (dPhi/deta eliminated through the chain rule, so
                             the time equation takes grad Phi . k), with
                             dPhi/dlambda estimated once per step as the
                             difference of Phi between the last two step
                             starts over the affine length between them
                             (Eq. dPhi/dl, second form); the first step takes
                             grad Phi . k at the observer.  On a light cone it
                             carries the time variation of Phi without a
                             dPhi/deta field.
       MPATH_DPHIDL_DIFF: order 1, static grid (no dphi_deta), iso-eta stop,
       n_surfaces 0, checkpoint_every 0, static schedule. */
    int32_t dphidl;
} mpath_cast_desc;

/* Per-ray outputs: caller-allocated DEVICE arrays of length n_rays
 * (= sum pix_count; (n_surfaces + 1) n_rays with intermediate surfaces).
 * Any pointer may be NULL (not written).
 *   beta[2]     (polar, azimuth) of x_s - x_obs (lens equation, Sect. 2.3)
 *   alpha[2]    deflection theta - beta as a tangent vector at theta of length
 *               the great-circle angle, on e1 = e_phi(theta), e2 = -e_theta(theta)
 *   z5          observed redshift (ratio of g_mu nu k^mu u^nu, v = 0, Sect. 2.5)
 *   z0          FLRW redshift of the stop surface
 *   phi_src     Phi at the end point
 *   n_steps     RK4 steps taken, the landing step included
 *   status      MPATH_RAY_*
 *   hash        FNV-1a over the discrete decisions (leaf level of every step,
 *               stencil level of every sub-step) for comparing with a reference
 *   chi         |x_s - x_obs|
 *   z1          FLRW redshift plus the potential term, z0 + (1 + z0)(Phi_o - Phi_s)
 *               (Sect. 2.5; with v = 0 the Doppler and transverse Doppler
 *               terms vanish, so z2 = z3 = z1)
 *   z4          z1 plus the ISW term, z1 - 2 (1 + z0) isw (Sect. 2.5; equal to
 *               z1 for a static potential)
 *   isw         integral of dPhi/deta over conformal time from the stop surface
 *               to the observer along the ray (0 for a static potential) */
typedef struct {
    double* beta;
    float* alpha;
    double* z5;
    double* z0;
    float* phi_src;
    int32_t* n_steps;
    int32_t* status;
    uint32_t* hash;
    double* chi;
    double* z1;
    double* z4;
    double* isw;
} mpath_observables;

/* Device workspace for a cast (observer table, queue counter, end states,
 * directions and, when checkpoint_every > 0, the checkpoints of every ray
 * for mpath_adjoint: 40 bytes per ray and checkpoint). */
int mpath_cast_workspace_bytes(const mpath_grid* grid, const mpath_cast_desc* desc, size_t* bytes);

/* Cast all rays; asynchronous on the stream except for the upload of the
 * observer table (a few bytes per observer), which completes before return.
 * A grid with dphi_deta is cast with order 1, one stop surface and
 * checkpoint_every 0 (MPATH_ERR_UNSUPPORTED otherwise); the reverse mode,
 * the infinitesimal and Born beams and the finder take static potentials
 * only. */
int mpath_cast(const mpath_grid* grid, const mpath_cast_desc* desc, mpath_observables* out,
               void* dev_ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * mpath_cast with its workspace taken from a static device buffer of
 * MPATH_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, which the library holds until
 * the process ends; the caller still passes the grid, the desc and the
 * output arrays.  Plain casts only: checkpoint_every must be 0
 * (MPATH_ERR_UNSUPPORTED otherwise), and the workspace that
 * mpath_cast_workspace_bytes reports for the desc must fit the buffer (about
 * 48 B per ray and surface plus 80 B per observer: up to about 1.3 million
 * rays with one surface), else MPATH_ERR_WORKSPACE_TOO_SMALL before any
 * device work.  Calls no allocating routine.  Every call on one GPU uses
 * the same buffer: calls that overlap in time on one GPU (several streams
 * or host threads) race and must be serialised by the caller; a call's
 * outputs do not depend on what an earlier call left in the buffer. */
#define MPATH_NOALLOC_SCRATCH_BYTES (64u << 20)
int mpath_cast_noalloc(const mpath_grid* grid, const mpath_cast_desc* desc, mpath_observables* out, void* stream);

/* ---- forward mode ----
 * The distortion matrix of the lens equation (Sect. 2.3) and dz5/dtheta by
 * forward-mode differentiation of the same discrete map that mpath_cast
 * computes (RK4 on the geodesic equations of Sect. 2.2 with CIC
 * interpolation and the AMR level fallback, step length h_leaf / N through
 * |k0|, landing on the iso-eta surface): one pass carries, with every ray,
 * the tangents of its state for the two directions e1 = e_phi, e2 =
 * -e_theta in which the initial direction theta can move; the discrete
 * decisions (leaf levels, stencils) carry no derivative.  No checkpoints and
 * no reverse sweep: the cost is one cast with about twice the arithmetic.
 * Outputs as mpath_cast (bit for bit the same) plus, DEVICE, length n_rays:
 *   jac[2][2]     A_ab = d beta_a / d theta_b, beta_a on the screen basis
 *                 e~1 = e_phi, e~2 = -e_theta at the end direction, theta_b
 *                 on the basis at the initial direction (row-major: a, then
 *                 b); NaN for rays that did not reach the source
 *   dz_dtheta[2]  d z5 / d theta_b (NaN likewise)
 * either may be NULL.  CIC casts (order 1) to an iso-eta surface with the
 * chain-rule dPhi/dlambda, n_surfaces 0 and a static potential
 * (MPATH_ERR_UNSUPPORTED otherwise), checkpoint_every 0 (INVALID_ARG);
 * static schedule (the launch-shape fields are ignored).  Workspace:
 * mpath_cast_jacobian_workspace_bytes (the cast's plus 80 B per ray). */
int mpath_cast_jacobian_workspace_bytes(const mpath_grid* grid, const mpath_cast_desc* desc, size_t* bytes);
int mpath_cast_jacobian(const mpath_grid* grid, const mpath_cast_desc* desc, mpath_observables* out, float* jac,
                        float* dz_dtheta, void* dev_ws, size_t ws_bytes, void* stream);

/* ---- reverse mode ----
 * The derivative of the discrete map that mpath_cast computes (RK4 on the
 * geodesic equations of Sect. 2.2 with CIC interpolation and the AMR level
 * fallback, step length h_leaf / N, landing on the iso-eta surface), by one
 * reverse sweep per ray over the checkpointed forward path: each segment of
 * K steps is recomputed from its checkpoint, then traversed backwards.  The
 * discrete decisions (leaf levels, stencils, landing) are those of the
 * forward cast and carry no derivative.
 *
 * Per-ray outputs (DEVICE, length n_rays; NaN for rays whose status is not
 * MPATH_RAY_REACHED):
 *   jac[2][2]     distortion matrix A_ab = d beta_a / d theta_b of the lens
 *                 equation (Sect. 2.3), beta_a measured on e1 = e_phi,
 *                 e2 = -e_theta at the end point's direction, theta_b on the
 *                 same basis at the initial direction (row-major: a, then b)
 *   dz_dtheta[2]  d z5 / d theta_b
 * Cell outputs (DEVICE, caller order, overwritten) for the scalar loss L
 * whose per-ray cotangents are dL_dalpha[n_rays][2] (of alpha) and
 * dL_dz[n_rays] (of z5), either may be NULL (= 0):
 *   dL_dvalues[n_cells][4]  dL / d (phi, gx, gy, gz) of every cell
 *   dL_dphi_total[n_cells]  uniform periodic grids whose gradient is the
 *                           central difference (phi[i+1] - phi[i-1]) / 2h:
 *                           dL/dphi + (difference operator)^T dL/dgrad
 * Per-ray check (DEVICE int32 [n_rays]): ray_status[r] = 0 when the
 * derivative was computed, 1 when the ray did not reach the source (no
 * derivative), 2 when the recomputation did not retrace the forward path bit
 * for bit (only possible if the cell values changed after the cast; the
 * ray's outputs are then NaN and its cell terms incomplete).
 * Any output pointer may be NULL; the cell cotangents are float32 sums
 * accumulated with atomics, so their last bits depend on the order of the
 * additions, and need the grid's auxiliary tables (mpath_grid_build_with_aux;
 * MPATH_ERR_UNSUPPORTED without them). */
typedef struct {
    const float* dL_dalpha;
    const double* dL_dz;
    float* jac;
    float* dz_dtheta;
    float* dL_dvalues;
    float* dL_dphi_total;
    int32_t* ray_status;
} mpath_adjoint_desc;

/* Device workspace of mpath_adjoint for this desc (which needs
 * checkpoint_every > 0): K states per ray (40 B each) and 16 B per cell
 * (rounded up to a multiple of 8 cells). */
int mpath_adjoint_workspace_bytes(const mpath_grid* grid, const mpath_cast_desc* desc, size_t* bytes);

/* Reverse sweep after a checkpointed mpath_cast with the same grid (whose
 * values must not have changed since), the same desc and its workspace
 * cast_ws; fwd gives that cast's n_steps and status arrays (the other
 * fields are not read).  Asynchronous on the stream; cast_ws and the forward
 * outputs must stay untouched until it has run.  MPATH_ERR_UNSUPPORTED when
 * dL_dphi_total is requested on an AMR or non-periodic grid. */
int mpath_adjoint(const mpath_grid* grid, const mpath_cast_desc* desc, const mpath_observables* fwd,
                  const void* cast_ws, size_t cast_ws_bytes, const mpath_adjoint_desc* adj, void* dev_ws,
                  size_t ws_bytes, void* stream);

/* ---- launch autotuner ----
 * Times candidate launch shapes on a sample of the rays of desc (the first
 * ceil(count / sample_div) pixels of every observer, keeping the observers'
 * mix of source distances) and returns in *tuned a copy of desc with the
 * fastest schedule, waves_per_cu and batch.  Candidates: the static schedule
 * and the persistent one at the resident occupancy, half and twice that,
 * with queue refills every 8, 16, 32, 64 or 128 steps.  The launch shape
 * does not change any result.  Synchronises the stream; dev_ws (size from
 * mpath_autotune_workspace_bytes) is scratch for the sample casts; best_ms
 * (may be NULL) receives the sample's time with the chosen shape. */
int mpath_autotune_workspace_bytes(const mpath_grid* grid, const mpath_cast_desc* desc, int32_t sample_div,
                                   size_t* bytes);
int mpath_autotune(const mpath_grid* grid, const mpath_cast_desc* desc, int32_t sample_div, void* dev_ws,
                   size_t ws_bytes, void* stream, mpath_cast_desc* tuned, float* best_ms);

/* Number of rays a desc describes. */
int mpath_cast_count_rays(const mpath_cast_desc* desc, int64_t* n_rays);

/* ---- weak-lensing products (Sect. 2.3) ----
 *
 * Distortion matrices A (2x2, row-major A[a][b] = A_ab, screen basis
 * e1 = e_phi, e2 = -e_theta: at the initial direction on the theta side, at
 * the end point on the beta side) are those of mpath_adjoint (jac), of
 * mpath_finite_beam, or any other source. */

/* mpath_lensing_maps: convergence, shear, rotation and magnification of n
 * distortion matrices, inverting the decomposition of Sect. 2.3,
 *   A = R(omega) [[1 - kappa - g1, -g2], [-g2, 1 - kappa + g1]]:
 *   tan omega = (A21 - A12) / (A11 + A22),
 *   1 - kappa = |(A11 + A22, A21 - A12)| / 2,
 *   S = R(-omega) A, g1 = (S22 - S11) / 2, g2 = -(S12 + S21) / 2,
 *   mu = 1 / det A  (computed in FP64).
 *   A:   DEVICE float[n][2][2];  out: DEVICE float[n][5] =
 *        (kappa, gamma1, gamma2, omega, mu), written.
 * Asynchronous on the stream.  Errors: INVALID_ARG (n < 0, NULL pointers
 * with n > 0), DEVICE. */
int mpath_lensing_maps(const float* A, int64_t n, float* out, void* stream);

/* mpath_finite_beam: finite-beam distortion matrix (Sect. 2.3.2) of every ray
 * of desc.  Around each reference direction n four more rays start along
 * n + tan(eps) e1 (A), n - tan(eps) e1 (B), n - tan(eps) e2 (C) and
 * n + tan(eps) e2 (D), normalised, with (e1, e2) the screen basis at n; all
 * five are cast in one launch to the reference ray's stop surface, and
 *   A-hat = [[(r_A - r_B).f1, (r_D - r_C).f1], [(r_A - r_B).f2, (r_D - r_C).f2]]
 *           / (2 chi_0 tan(eps)),
 * with r = x_s - x_obs, chi_0 = |r_ref| and (f1, f2) the screen basis at
 * r_ref.  The second column is taken as (r_D - r_C), the sign that makes
 * A-hat the identity without lensing (the printed formula's opposite sign
 * gives -1 there).
 *   desc:   as for mpath_cast (checkpoint_every ignored); eps in (0, 0.1] rad.
 *   A:      DEVICE float[n_rays][2][2], written (NaN where a ray of the beam
 *           did not reach the source).
 *   status: DEVICE int32[n_rays] or NULL: first non-zero MPATH_RAY_* of the
 *           reference, A, B, C, D rays (0 when all five reached the source).
 *   dev_ws: mpath_finite_beam_workspace_bytes bytes (the five-ray cast).
 * Synchronises the stream once (table upload); the rest is asynchronous.
 * Errors: as mpath_cast, INVALID_ARG for eps. */
int mpath_finite_beam_workspace_bytes(const mpath_grid* grid, const mpath_cast_desc* desc, size_t* bytes);
int mpath_finite_beam(const mpath_grid* grid, const mpath_cast_desc* desc, double eps, float* A, int32_t* status,
                      void* dev_ws, size_t ws_bytes, void* stream);

/* mpath_infinitesimal_beam: a cast (as mpath_cast, same outputs, static
 * schedule, no checkpoints) that also integrates the infinitesimal-beam
 * distortion matrix of every ray (Sect. 2.3.1):
 *   A_ab = delta_ab - 2 int_0^chi_s (chi_s - chi) chi / chi_s T_ab dchi,
 *   T_ab = e_a . H e_b, H_ij = (G_j(x + h e_i) - G_j(x - h e_i)) / (2 h)
 * (the finite-difference Hessian of the interpolated force, mixed terms
 * symmetrised, derivation step h = the size of the leaf cell holding x),
 * (e_1, e_2) = (e_phi, -e_theta) at the direction of x - x_obs, sampled at
 * every step start and at the end point, trapezoid rule in chi.  A probe
 * outside a non-periodic box contributes a zero row of H.
 *   A: DEVICE float[n_rays][2][2] (symmetric), written; NaN for rays that
 *      did not reach the source.
 *   dev_ws: mpath_cast_workspace_bytes of desc.
 * Errors: as mpath_cast; INVALID_ARG when checkpoint_every != 0. */
int mpath_infinitesimal_beam(const mpath_grid* grid, const mpath_cast_desc* desc, mpath_observables* out, float* A,
                             void* dev_ws, size_t ws_bytes, void* stream);

/* ---- geodesic finder and relativistic catalogues (Sect. 2.5) ----
 *
 * For a source at comoving position x_src the comoving angular position
 * beta is the direction of x_src - x_obs and chi = |x_src - x_obs| its
 * distance (unwrapped: on a periodic grid the box is replicated).  The
 * finder seeks the initial direction theta whose photon, stopped on the
 * source's light-cone surface eta_s = eta_0 - chi, arrives in the direction
 * beta, by the Newton iteration theta_{i+1} = theta_i - A^-1 (beta_i - beta):
 * residual d_a = f_a(beta_i) . beta on the screen basis (f1, f2) at beta_i,
 * A dtheta = d solved, theta moved by dtheta along its own screen basis
 * (e1, e2) = (e_phi, -e_theta) and normalised.  The first identity_iters
 * iterations take A = I (plain casts, as the paper does), later ones the
 * exact distortion matrix of mpath_adjoint (a checkpointed cast and a
 * Jacobian sweep).  A source stops iterating when the angle between beta_i
 * and beta is below tol.  At the end every source is cast once more along
 * its theta (checkpointed) and, when requested, its exact A and dz5/dtheta
 * are computed there. */
typedef struct {
    const double* obs_pos;      /* HOST [3] observer position                            */
    int64_t n_src;
    const double* src_pos;      /* HOST [n_src][3] comoving source positions             */
    int32_t order;              /* 1 = CIC                                               */
    int32_t steps_per_cell;     /* as mpath_cast_desc                                     */
    int32_t adaptive;
    int64_t max_steps;
    double tol;                 /* convergence angle (rad), > 0                           */
    int32_t max_iter;           /* Newton iterations, >= 1                                */
    int32_t identity_iters;     /* iterations with A = I before the exact Jacobian, >= 0 */
    int32_t checkpoint_every;   /* K of the Jacobian sweeps, >= 1                         */
    /* the last-resort root finder (Sect. 2.5) for sources still unconverged
       after max_iter: grid_rounds (>= 0; 0 = none) rounds of grid_n x grid_n
       candidate directions (grid_n odd, 3..15) on the screen plane of theta,
       theta + a D e1 + b D e2 normalised, D = 2 w / (grid_n - 1), a and b in
       -(grid_n-1)/2 .. (grid_n-1)/2 (candidate (b + h) grid_n + (a + h)); the
       half-width w starts at twice the last Newton separation and becomes
       the previous spacing D after every round.  All candidates are cast to
       the source's surface in one launch; theta moves to the candidate that
       lands nearest beta (the first of equal ones).  A source converging in
       round r reports n_iter = max_iter + r.  At most grid_max sources
       (0: all), the first by index, take part (it sizes the workspace). */
    int32_t grid_rounds;
    int32_t grid_n;
    int64_t grid_max;
} mpath_finder_desc;

/* DEVICE outputs, arrays of n_src; theta is required, the others may be NULL. */
typedef struct {
    double* theta;              /* [n][3] initial direction found (unit)                           */
    float* A;                   /* [n][2][2] exact distortion matrix d beta / d theta at theta     */
    float* dz_dtheta;           /* [n][2] d z5 / d theta on (e1, e2) at theta                       */
    double* z5;                 /* observed redshift (Sect. 2.5, v = 0)                             */
    double* z0;                 /* FLRW redshift of the source's surface                            */
    float* phi_src;             /* Phi at the end point                                             */
    double* sep;                /* angle between the final end direction and beta (rad)             */
    int32_t* n_iter;            /* iteration of convergence (0: the first cast; >= max_iter: in
                                   round n_iter - max_iter of the grid search); -1 not converged;
                                   -2 a cast did not reach the source                               */
    int32_t* status;            /* MPATH_RAY_* of the final cast                                    */
    double* z1;                 /* z0 + (1 + z0)(Phi_o - Phi_s)                                      */
} mpath_finder_out;

/* Workspace: the checkpointed cast and Jacobian sweep of n_src rays plus
 * per-source tables (88 bytes per source). */
int mpath_find_geodesics_workspace_bytes(const mpath_grid* grid, const mpath_finder_desc* desc, size_t* bytes);
/* Synchronises the stream once per iteration and grid round (the count of
 * sources still iterating decides whether to continue).  Errors:
 * INVALID_ARG (NULL arrays, tol <= 0, max_iter < 1, identity_iters < 0,
 * checkpoint_every < 1, a source at the observer, grid_rounds < 0, grid_n
 * not odd in 3..15 with grid_rounds > 0, grid_max < 0), UNSUPPORTED
 * (order != 1, a source beyond the background table, z > 20),
 * WORKSPACE_TOO_SMALL, DEVICE. */
int mpath_find_geodesics(const mpath_grid* grid, const mpath_finder_desc* desc, mpath_finder_out* out,
                         void* dev_ws, size_t ws_bytes, void* stream);

/* mpath_born_beam: the Born approximation of the infinitesimal-beam matrix
 * (Sect. 2.3.1 and the comparison of Sect. 3.6): the same line-of-sight
 * integral taken along the straight line x_obs + chi n from the observer to
 * the stop surface's comoving distance chi_s = eta_0 - eta_s, with n the
 * ray's initial direction (pixel centre or desc->dirs: pass the source
 * directions beta there for the Born approximation in the direction of the
 * sources).  Samples at chi_{i+1} = min(chi_i + ds_i, chi_s), ds_i the
 * integration's step length (h / N) at x(chi_i); trapezoid rule in chi.
 *   A:      DEVICE float[n_rays][2][2], written (NaN if the line leaves a
 *           non-periodic box or exceeds max_steps samples).
 *   status: DEVICE int32[n_rays] or NULL (MPATH_RAY_*).
 *   dev_ws: mpath_cast_workspace_bytes of desc (checkpoint_every 0).
 * Errors: as mpath_cast; UNSUPPORTED for order != 1. */
int mpath_born_beam(const mpath_grid* grid, const mpath_cast_desc* desc, float* A, int32_t* status, void* dev_ws,
                    size_t ws_bytes, void* stream);

/* ---- measurement utility (not a step of the method) ----
 *
 * mpath_gather_probe: random-record gather throughput, the ceiling that the
 * integration kernel's data-dependent table lookups are measured against.
 * Launches n_waves one-wave workgroups; each of the n_waves * 64 lanes reads
 * `iters * in_flight` records of `record_bytes` (16, 64 or 128) bytes at
 * indices drawn uniformly in [0, table_bytes / record_bytes) from its own
 * xorshift64 sequence (seeded by `seed` and the lane number), with
 * `in_flight` (1, 2 or 4) independent reads outstanding per lane, and writes
 * the float sum of what it read to out[lane].
 *   table: DEVICE, 16-byte aligned, table_bytes readable bytes (any content).
 *   out:   DEVICE float[n_waves * 64], written.
 *   n_waves in [1, 2^24], iters >= 1.
 * Bytes gathered = n_waves * 64 * iters * in_flight * record_bytes.  The call
 * is asynchronous on the stream (time it with events on that stream).
 * Errors: INVALID_ARG for the ranges above, DEVICE for a launch failure. */
int mpath_gather_probe(const void* table, size_t table_bytes, int32_t record_bytes, int32_t in_flight,
                       int64_t n_waves, int32_t iters, uint32_t seed, float* out, void* stream);

const char* mpath_status_string(int status);
const char* mpath_last_error(void);
const char* mpath_version(void);

#ifdef __cplusplus
}
#endif
#endif
