// finder.hip -- geodesic finder (Sect. 2.5): the Newton iteration on the
// initial direction theta that brings the photon, stopped on the source's
// light-cone surface, to the source's comoving angular position beta:
//   theta_{i+1} = theta_i - A^-1 (beta_i - beta).
// 2-vectors live on the screen bases e1 = e_phi, e2 = -e_theta (at theta_i
// on the theta side, at beta_i on the beta side), the bases of A.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mpath {
namespace {

__device__ inline void basis_at(const double v[3], double e1[3], double e2[3])
{
    const double rho = hypot(v[0], v[1]);
    const double r = sqrt(rho * rho + v[2] * v[2]);
    const double cp = rho > 0.0 ? v[0] / rho : 1.0, sp = rho > 0.0 ? v[1] / rho : 0.0;
    const double ct = v[2] / r, st = rho / r;
    e1[0] = -sp; e1[1] = cp; e1[2] = 0.0;
    e2[0] = -cp * ct; e2[1] = -sp * ct; e2[2] = st;
}

__device__ inline double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Direction of the end point r = x_s - x_obs of ray i (the cast along theta)
// and its angle to the target direction t.
__device__ inline double end_direction(const RayEnd& e, const double th[3], double eta0, const double t[3],
                                       double b[3])
{
    const double s = eta0 - e.eta;
#pragma unroll
    for (int k = 0; k < 3; ++k) b[k] = s * th[k] + (double)e.dx[k];
    const double inv = 1.0 / sqrt(dot3(b, b));
#pragma unroll
    for (int k = 0; k < 3; ++k) b[k] *= inv;
    const double c[3] = {b[1] * t[2] - b[2] * t[1], b[2] * t[0] - b[0] * t[2], b[0] * t[1] - b[1] * t[0]};
    return atan2(sqrt(dot3(c, c)), dot3(b, t));
}

// One Newton step for every source still iterating (n_iter == -1): a ray
// that did not reach its source stops the iteration (-2); a ray within tol
// of its target converges at iteration it; the others move theta and are
// counted in *active.  jac NULL: A = I.
__global__ __launch_bounds__(256) void finder_update_kernel(int64_t n, const RayEnd* __restrict__ ends,
                                                            const double* __restrict__ target,
                                                            const int32_t* __restrict__ status,
                                                            const float* __restrict__ jac, double eta0, double tol,
                                                            int it, double* __restrict__ theta,
                                                            int32_t* __restrict__ n_iter, double* __restrict__ sep,
                                                            unsigned int* __restrict__ active)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || n_iter[i] != -1) return;
    if (status[i] != MPATH_RAY_REACHED) {
        n_iter[i] = -2;
        return;
    }
    const double t[3] = {target[3 * i], target[3 * i + 1], target[3 * i + 2]};
    double th[3] = {theta[3 * i], theta[3 * i + 1], theta[3 * i + 2]};
    double b[3];
    const double s = end_direction(ends[i], th, eta0, t, b);
    sep[i] = s;
    if (s < tol) {
        n_iter[i] = it;
        return;
    }
    // residual beta - beta_i as screen components at beta_i (zero exactly at the root)
    double f1[3], f2[3];
    basis_at(b, f1, f2);
    const double d0 = dot3(f1, t), d1 = dot3(f2, t);
    double a00 = 1.0, a01 = 0.0, a10 = 0.0, a11 = 1.0;
    if (jac) {
        a00 = jac[4 * i]; a01 = jac[4 * i + 1]; a10 = jac[4 * i + 2]; a11 = jac[4 * i + 3];
    }
    const double det = a00 * a11 - a01 * a10;
    const double x0 = (a11 * d0 - a01 * d1) / det, x1 = (a00 * d1 - a10 * d0) / det;
    double e1[3], e2[3];
    basis_at(th, e1, e2);
#pragma unroll
    for (int k = 0; k < 3; ++k) th[k] += x0 * e1[k] + x1 * e2[k];
    const double inv = 1.0 / sqrt(dot3(th, th));
#pragma unroll
    for (int k = 0; k < 3; ++k) theta[3 * i + k] = th[k] * inv;
    atomicAdd(active, 1u);
}

// Angle between the end direction of the final cast and the target.
__global__ __launch_bounds__(256) void finder_sep_kernel(int64_t n, const RayEnd* __restrict__ ends,
                                                         const double* __restrict__ target,
                                                         const double* __restrict__ theta,
                                                         const int32_t* __restrict__ status, double eta0,
                                                         double* __restrict__ sep)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t[3] = {target[3 * i], target[3 * i + 1], target[3 * i + 2]};
    const double th[3] = {theta[3 * i], theta[3 * i + 1], theta[3 * i + 2]};
    double b[3];
    sep[i] = status[i] == MPATH_RAY_REACHED ? end_direction(ends[i], th, eta0, t, b) : __builtin_nan("");
}

// Grid search (the last-resort root finder): half-width of each refined
// source's first grid, twice its last Newton separation.
__global__ __launch_bounds__(256) void grid_init_kernel(int64_t m, const int64_t* __restrict__ idx,
                                                        const double* __restrict__ sep, double* __restrict__ w)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) w[k] = 2.0 * sep[idx[k]];
}

// Candidate t = k g^2 + c of refined source k: theta + a D e1 + b D e2,
// normalised, a = c mod g - h, b = c / g - h, D = 2 w / (g - 1), with the
// source's stop surface.
__global__ __launch_bounds__(256) void grid_dirs_kernel(int64_t m, int g, const int64_t* __restrict__ idx,
                                                        const double* __restrict__ theta,
                                                        const double* __restrict__ w,
                                                        const double2* __restrict__ stop, double* __restrict__ dirs,
                                                        double2* __restrict__ gstop)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gg = (int64_t)g * g;
    if (t >= m * gg) return;
    const int64_t k = t / gg;
    const int c = (int)(t - k * gg);
    const int h = (g - 1) / 2;
    const int a = c % g - h, b = c / g - h;
    const int64_t i = idx[k];
    const double th[3] = {theta[3 * i], theta[3 * i + 1], theta[3 * i + 2]};
    double e1[3], e2[3];
    basis_at(th, e1, e2);
    const double D = 2.0 * w[k] / (double)(g - 1);
    double v[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) v[q] = th[q] + (double)a * D * e1[q] + (double)b * D * e2[q];
    const double inv = 1.0 / sqrt(dot3(v, v));
#pragma unroll
    for (int q = 0; q < 3; ++q) dirs[3 * t + q] = v[q] * inv;
    gstop[t] = stop[i];
}

// One round's choice for every refined source still iterating: the
// candidate whose end direction is nearest beta (the first of equal ones)
// becomes theta; below tol the source converges at iteration it, else its
// half-width shrinks to the spacing and it is counted in *active.
__global__ __launch_bounds__(256) void grid_pick_kernel(int64_t m, int g, const int64_t* __restrict__ idx,
                                                        const RayEnd* __restrict__ ends,
                                                        const double* __restrict__ dirs,
                                                        const int32_t* __restrict__ status,
                                                        const double* __restrict__ target, double eta0, double tol,
                                                        int it, double* __restrict__ theta, double* __restrict__ sep,
                                                        int32_t* __restrict__ n_iter, double* __restrict__ w,
                                                        unsigned int* __restrict__ active)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int64_t i = idx[k];
    if (n_iter[i] != -1) return;
    const double t[3] = {target[3 * i], target[3 * i + 1], target[3 * i + 2]};
    const int64_t gg = (int64_t)g * g;
    double best = __builtin_inf();
    int64_t bc = -1;
    for (int64_t c = 0; c < gg; ++c) {
        const int64_t r = k * gg + c;
        if (status[r] != MPATH_RAY_REACHED) continue;
        const double d[3] = {dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2]};
        double bdir[3];
        const double s = end_direction(ends[r], d, eta0, t, bdir);
        if (s < best) {
            best = s;
            bc = c;
        }
    }
    if (bc < 0) return;          // no candidate reached the source: the search ends here
    const int64_t r = k * gg + bc;
#pragma unroll
    for (int q = 0; q < 3; ++q) theta[3 * i + q] = dirs[3 * r + q];
    sep[i] = best;
    if (best < tol) {
        n_iter[i] = it;
    } else {
        w[k] = 2.0 * w[k] / (double)(g - 1);
        atomicAdd(active, 1u);
    }
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void zero_u32_kernel(unsigned int* p) { *p = 0u; }

inline dim3 blocks_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

hipError_t launch_finder_update(int64_t n, const RayEnd* ends, const double* target, const int32_t* status,
                                const float* jac, double eta0, double tol, int it, double* theta, int32_t* n_iter,
                                double* sep, unsigned int* active, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, active);
    if (n > 0)
        hipLaunchKernelGGL(finder_update_kernel, blocks_for(n), dim3(256), 0, s, n, ends, target, status, jac, eta0,
                           tol, it, theta, n_iter, sep, active);
    return hipGetLastError();
}

hipError_t launch_finder_sep(int64_t n, const RayEnd* ends, const double* target, const double* theta,
                             const int32_t* status, double eta0, double* sep, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(finder_sep_kernel, blocks_for(n), dim3(256), 0, s, n, ends, target, theta, status, eta0, sep);
    return hipGetLastError();
}

hipError_t launch_grid_init(int64_t m, const int64_t* idx, const double* sep, double* w, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(grid_init_kernel, blocks_for(m), dim3(256), 0, s, m, idx, sep, w);
    return hipGetLastError();
}

hipError_t launch_grid_dirs(int64_t m, int g, const int64_t* idx, const double* theta, const double* w,
                            const double2* stop, double* dirs, double2* gstop, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(grid_dirs_kernel, blocks_for(m * g * g), dim3(256), 0, s, m, g, idx, theta, w, stop, dirs,
                       gstop);
    return hipGetLastError();
}

hipError_t launch_grid_pick(int64_t m, int g, const int64_t* idx, const RayEnd* ends, const double* dirs,
                            const int32_t* status, const double* target, double eta0, double tol, int it,
                            double* theta, double* sep, int32_t* n_iter, double* w, unsigned int* active,
                            hipStream_t s)
{
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, active);
    if (m > 0)
        hipLaunchKernelGGL(grid_pick_kernel, blocks_for(m), dim3(256), 0, s, m, g, idx, ends, dirs, status, target,
                           eta0, tol, it, theta, sep, n_iter, w, active);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, blocks_for(n), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace mpath
