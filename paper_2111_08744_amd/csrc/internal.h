// internal.h -- types shared by the host part and the kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpath.h"

namespace mpath {

// Per-observer table, uploaded by mpath_cast.  eta_s is the conformal time of
// the stop surface, a_s = a(eta_s), z0 = 1/a_s - 1.
struct ObsDev {
    double x[3];
    double eta_s;
    double a_s;
    double z0;
    double p_s;          // value of the stop surface's parameter (eta, chi, lambda or ln(1 + z))
    int64_t pix_first;
    int64_t ray_first;   // index of the observer's first ray in the outputs
    int64_t count;
};

// Octree on the device.  Cells are numbered level by level: coarse cell
// (i, j, k) has id morton3(i, j, k); the children of a refined cell c are the
// 8 consecutive ids child[c] + octant, octant = ox + 2 oy + 4 oz, and blocks
// of one level follow the order of their parents, so the ids of level l are
// the contiguous range [level_start[l], level_start[l + 1]).
//
// Two derived tables make a stencil one 128-byte read:
//   dual[c]      the trilinear coefficients c0..c7 (see device.h) of the
//                payloads of the 8 cells (l, ijk(c) + {0,1}^3) of c's level
//                (zeros where such a cell does not exist);
//   leafinfo[c - level_start[1]]  for a leaf c of level L >= 1 and each
//                half-cell q of it (the
//                8 sub-octants, q = qx + 2 qy + 4 qz), the id of the lowest
//                corner cell of the CIC stencil that the AMR fallback
//                procedure selects for points in that half-cell, or -1 when
//                no level has a complete stencil there.
constexpr int kMaxLevels = 11;

struct GridDev {
    const float4* payload;    // (phi, gx, gy, gz) per cell
    const int32_t* child;     // first child id, -1 for a leaf
    const float4* dual;       // [n][8]
    const int32_t* leafinfo;  // [n - level_start[1]][8]: rows of the refined cells only
    const int32_t* dual_ids;  // [n][8] ids of the 8 cells of dual[c] (-1: missing); null
                              // unless the grid has its auxiliary tables
    const float4* tdual;      // [n][2]: 8 trilinear coefficients of dPhi/deta, or null (static potential)
    double h0;                // coarse cell size
    double inv_h0;
    double inv_hf;            // 2^(max_level + 1) / h0: fine-grid coordinates
    double eta0;              // conformal time at the observers (a = 1)
    float phi_max;            // largest cell value of phi (+inf when unknown)
    int32_t n0;               // coarse cells per side (power of two)
    int32_t max_level;
    int32_t periodic;
    int32_t level_start[kMaxLevels + 1];
};

// Conformal Hubble rate a'/a tabulated with its eta-derivative on a uniform
// eta grid, for cubic Hermite interpolation.
struct CosmoDev {
    const double2* table;     // (H, dH/deta) at eta_lo + i * deta
    const double2* atable;    // (a, da/deta) at the same nodes
    double eta_lo;
    double inv_deta;
    double deta;
    int32_t n;
    int32_t is_static;
};

// Geodesic state in the split representation (see device.h).
struct GeoState {
    double eta, K;
    float d[3], dx[3];
};

// End state of a ray kept between the integration and the observables kernel.
struct RayEnd {
    double eta;
    float dx[3];
    int32_t obs;
};

// End state of the two forward-mode tangents of a ray (mpath_cast_jacobian):
// per tangent b the tangents of eta and K = |k0| and dX = dx - s e_b
// (x = x_obs + s n, s the path length, e_b the direction the initial n moves
// along) at the end point before the landing step's length is
// differentiated; the end state's d and K, Phi at the observer, and the
// stencil (lowest corner, level) of the end point.
struct TanEnd {
    float deta[2], dK[2], dX[2][3];
    float d[3];
    float phi_o;
    double K;
    int32_t base, lvl;
    int32_t status;
    int32_t pad;
};

struct OutDev {
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
};

struct CastArgs {
    GridDev grid;
    CosmoDev cosmo;
    double cosmo_eta0;           // conformal time at the observers (a = 1)
    const ObsDev* obs;
    int32_t n_obs;
    int32_t nside;
    int32_t steps_per_cell;
    int32_t adaptive;
    double ds_level[kMaxLevels + 1];  // comoving step length h_l / N (h_0 / N on every level if not adaptive);
                                      // kernels read it through step_length()
    int64_t max_steps;
    int64_t n_rays;
    OutDev out;
    unsigned long long* queue;   // persistent schedule: next ray to hand out
    int32_t batch;               // steps between queue refills
    RayEnd* ends;                // [n_rays] end states for the observables kernel
    double* dirs;                // [n_rays][3] initial directions (HEALPix pixel centres)
    GeoState* ckpt;              // [slots][n_rays] state before steps 0, K, 2K, ... (adjoint)
    int32_t ckpt_every;          // K (0: no checkpoints)
    int32_t ckpt_slots;
    const double2* ray_stop;     // [n_rays] (eta_s, a_s) of each ray's own stop surface, or
                                 // NULL: the observer's (geodesic finder: one source per ray)
    int32_t surface;             // MPATH_SURFACE_*: the parameter the stop surface holds
};

// Reverse-mode (adjoint) arguments.
struct AdjointArgs {
    CastArgs c;                  // the cast that stored the checkpoints
    GeoState* tape;              // [ckpt_every][n_rays] step states of one segment
    const int32_t* n_steps;      // forward outputs
    const int32_t* status;
    const float* dL_dalpha;      // [n_rays][2] or NULL
    const double* dL_dz;         // [n_rays] or NULL
    float* jac;                  // [n_rays][2][2] or NULL
    float* dz_dtheta;            // [n_rays][2] or NULL
    int32_t* ray_status;         // [n_rays] or NULL: 0 ok, 1 not reached, 2 replay mismatch
    float* grad;                 // cotangents of (phi, grad) per cell (see grad_slot) or NULL
    int64_t n_cells;
};

// Floats of the cell-cotangent accumulator of the adjoint for n cells.
inline int64_t grad_accumulator_floats(int64_t n) { return 4 * (((n + 7) >> 3) << 3); }

// Kernel launchers (defined in cast.hip).
hipError_t launch_cast_stop(const CastArgs& a, hipStream_t s);
hipError_t launch_cast_diff(const CastArgs& a, hipStream_t s);
hipError_t launch_cast_static(const CastArgs& a, int block, hipStream_t s);
hipError_t launch_cast_persistent(const CastArgs& a, int block, int blocks, hipStream_t s);
hipError_t launch_observables(const CastArgs& a, hipStream_t s);
hipError_t launch_ray_dirs(const CastArgs& a, hipStream_t s);
hipError_t launch_cast_infbeam(const CastArgs& a, float* A, hipStream_t s);
hipError_t launch_cast_tangent(const CastArgs& a, TanEnd* te, hipStream_t s);
hipError_t launch_tangent_observables(const CastArgs& a, const TanEnd* te, float* jac, float* dz_dtheta,
                                      hipStream_t s);
hipError_t launch_cast_order(const CastArgs& a, int order, hipStream_t s);
hipError_t launch_born_beam(const CastArgs& a, float* A, int32_t* status, hipStream_t s);
hipError_t launch_cast_surfaces(const CastArgs& a, const double2* surf, int n_extra, hipStream_t s);
hipError_t launch_permute_values(float4* payload, const int64_t* perm, const float4* values,
                                 int64_t n, hipStream_t s);
// Derived tables (defined in grid.hip), built for the cells [c0, c0 + m)
// from their positions pos[0 .. m) = (i, j, k, level) (a staged chunk).
hipError_t launch_build_dual(const GridDev& g, const int4* pos, int64_t c0, int64_t m, float4* dual, hipStream_t s);
hipError_t launch_rebuild_dual(const GridDev& g, const int32_t* ids, float4* dual, int64_t n, hipStream_t s);
hipError_t launch_build_tdual(const GridDev& g, const int4* pos, int64_t c0, int64_t m, const float* tpay,
                              float4* tdual, hipStream_t s);
hipError_t launch_build_leafinfo(const GridDev& g, const int4* pos, int64_t c0, int64_t m, int32_t* leafinfo,
                                 hipStream_t s);
hipError_t launch_build_dual_ids(const GridDev& g, const int4* pos, int64_t c0, int64_t m, int32_t* ids,
                                 hipStream_t s);
// Adjoint (defined in adjoint.hip).
hipError_t launch_cast_checkpointed(const CastArgs& a, hipStream_t s);
hipError_t launch_adjoint(const AdjointArgs& a, int columns, hipStream_t s);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);
hipError_t launch_scatter_grad(const float* grad_lib, const int64_t* perm, float4* out_user, int64_t n,
                               hipStream_t s);
hipError_t launch_central_transpose(const float* g_lib, const int64_t* perm, float* out, int n0, double h0,
                                    int64_t n, hipStream_t s);
int cast_occupancy_blocks_per_cu(int block, bool amr, bool time_dep);
// Reference rays of one observer for the finite-beam casts.
struct BeamObs {
    int64_t ray_first;   // first reference ray of the observer
    int64_t pix_first;   // first NESTED pixel (pixel-centre directions)
    int64_t count;       // reference rays of the observer
};
hipError_t launch_lensing_maps(const float* A, int64_t n, float* out, hipStream_t s);
hipError_t launch_healpix_dirs(int nside, int64_t pix_first, int64_t count, double* dirs, hipStream_t s);
hipError_t launch_beam_dirs(const BeamObs* obs, int n_obs, int nside, const double* user_dirs, double tan_eps,
                            int64_t n_rays, double* dirs5, hipStream_t s);
hipError_t launch_finite_beam(const BeamObs* obs, int n_obs, const RayEnd* ends, const double* dirs5,
                              const int32_t* status5, double eta0, double tan_eps, int64_t n_rays, float* A,
                              int32_t* status, hipStream_t s);
hipError_t launch_finder_update(int64_t n, const RayEnd* ends, const double* target, const int32_t* status,
                                const float* jac, double eta0, double tol, int it, double* theta, int32_t* n_iter,
                                double* sep, unsigned int* active, hipStream_t s);
hipError_t launch_finder_sep(int64_t n, const RayEnd* ends, const double* target, const double* theta,
                             const int32_t* status, double eta0, double* sep, hipStream_t s);
hipError_t launch_grid_init(int64_t m, const int64_t* idx, const double* sep, double* w, hipStream_t s);
hipError_t launch_grid_dirs(int64_t m, int g, const int64_t* idx, const double* theta, const double* w,
                            const double2* stop, double* dirs, double2* gstop, hipStream_t s);
hipError_t launch_grid_pick(int64_t m, int g, const int64_t* idx, const RayEnd* ends, const double* dirs,
                            const int32_t* status, const double* target, double eta0, double tol, int it,
                            double* theta, double* sep, int32_t* n_iter, double* w, unsigned int* active,
                            hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_gather_probe(const void* table, size_t table_bytes, int record_bytes, int in_flight,
                               int64_t n_waves, int iters, uint32_t seed, float* out, hipStream_t s);

// Morton interleave of three 10-bit coordinates (host and device).
__host__ __device__ inline uint32_t part1by2(uint32_t x)
{
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__host__ __device__ inline uint32_t morton3(uint32_t i, uint32_t j, uint32_t k)
{
    return part1by2(i) | (part1by2(j) << 1) | (part1by2(k) << 2);
}

// Inverse of part1by2: every third bit of x, compacted.
__host__ __device__ inline uint32_t compact1by2(uint32_t x)
{
    x &= 0x09249249u;
    x = (x | (x >> 2)) & 0x030C30C3u;
    x = (x | (x >> 4)) & 0x0300F00Fu;
    x = (x | (x >> 8)) & 0x030000FFu;
    x = (x | (x >> 16)) & 0x000003FFu;
    return x;
}

}  // namespace mpath
