// lensing.hip -- weak-lensing products of the distortion matrix (Sect. 2.3):
// its decomposition into convergence, shear, rotation and magnification, and
// the finite-beam matrix of Sect. 2.3.2 from four rays around each reference
// ray.
#include <hip/hip_runtime.h>

#include "device.h"

namespace mpath {
namespace {

// Screen basis at a direction v (any non-zero length): e1 = e_phi,
// e2 = -e_theta, with phi = atan2(v_y, v_x) (0 on the polar axis) and
// theta the polar angle.
__device__ inline void screen_basis(const double v[3], double e1[3], double e2[3])
{
    const double rho = hypot(v[0], v[1]);
    const double r = sqrt(rho * rho + v[2] * v[2]);
    const double cp = rho > 0.0 ? v[0] / rho : 1.0, sp = rho > 0.0 ? v[1] / rho : 0.0;
    const double ct = v[2] / r, st = rho / r;
    e1[0] = -sp; e1[1] = cp; e1[2] = 0.0;
    e2[0] = -cp * ct; e2[1] = -sp * ct; e2[2] = st;
}

// Inversion of the decomposition A = R(omega) [[1 - kappa - g1, -g2],
// [-g2, 1 - kappa + g1]] (Sect. 2.3): A11 + A22 = 2 (1 - kappa) cos omega and
// A21 - A12 = 2 (1 - kappa) sin omega give omega and 1 - kappa; the symmetric
// factor S = R(-omega) A gives g1 = (S22 - S11) / 2 and g2 = -(S12 + S21) / 2;
// mu = 1 / det A.  FP64 internally.
__global__ __launch_bounds__(256) void lensing_maps_kernel(const float* __restrict__ A, int64_t n,
                                                           float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a11 = A[4 * i], a12 = A[4 * i + 1], a21 = A[4 * i + 2], a22 = A[4 * i + 3];
    const double tr = a11 + a22, rot = a21 - a12;
    const double omega = atan2(rot, tr);
    const double one_k = 0.5 * hypot(tr, rot);
    double s, c;
    sincos(omega, &s, &c);
    const double s11 = c * a11 + s * a21, s12 = c * a12 + s * a22;
    const double s21 = -s * a11 + c * a21, s22 = -s * a12 + c * a22;
    out[5 * i] = (float)(1.0 - one_k);
    out[5 * i + 1] = (float)(0.5 * (s22 - s11));
    out[5 * i + 2] = (float)(-0.5 * (s12 + s21));
    out[5 * i + 3] = (float)omega;
    out[5 * i + 4] = (float)(1.0 / (a11 * a22 - a12 * a21));
}

// Observer j of reference ray r (observers are few: scan from the end).
__device__ inline int beam_observer(const BeamObs* obs, int n_obs, int64_t r)
{
    int j = n_obs - 1;
    while (j > 0 && obs[j].ray_first > r) --j;
    return j;
}

// Directions of the five rays of every beam (Sect. 2.3.2): the reference
// direction n (pixel centre or caller's direction) and n +- tan(eps) e1,
// n -+ tan(eps) e2 normalised (rays A, B, C, D).  Observer j's block of 5 c_j
// rays holds the reference rays, then the A, B, C and D rays, each in the
// order of the reference rays.
// Pixel centres of NESTED pixels pix_first .. pix_first + count - 1.
__global__ __launch_bounds__(256) void healpix_dirs_kernel(int nside, int64_t pix_first, int64_t count,
                                                           double* __restrict__ dirs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double v[3];
    healpix_nest_dir(nside, pix_first + i, v);
    dirs[3 * i] = v[0];
    dirs[3 * i + 1] = v[1];
    dirs[3 * i + 2] = v[2];
}

__global__ __launch_bounds__(256) void beam_dirs_kernel(const BeamObs* __restrict__ obs, int n_obs, int nside,
                                                        const double* __restrict__ user_dirs, double tan_eps,
                                                        int64_t n_rays, double* __restrict__ dirs5)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rays) return;
    const int j = beam_observer(obs, n_obs, r);
    const BeamObs& o = obs[j];
    const int64_t loc = r - o.ray_first, c = o.count, b5 = 5 * o.ray_first;
    double n[3];
    if (user_dirs) {
        n[0] = user_dirs[3 * r]; n[1] = user_dirs[3 * r + 1]; n[2] = user_dirs[3 * r + 2];
    } else {
        healpix_nest_dir(nside, o.pix_first + loc, n);
    }
    double e1[3], e2[3];
    screen_basis(n, e1, e2);
    const double sgn1[4] = {1.0, -1.0, 0.0, 0.0}, sgn2[4] = {0.0, 0.0, -1.0, 1.0};
#pragma unroll
    for (int i = 0; i < 3; ++i) dirs5[3 * (b5 + loc) + i] = n[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) v[i] = n[i] + tan_eps * (sgn1[k] * e1[i] + sgn2[k] * e2[i]);
        const double inv = 1.0 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const int64_t q = b5 + (k + 1) * c + loc;
#pragma unroll
        for (int i = 0; i < 3; ++i) dirs5[3 * q + i] = v[i] * inv;
    }
}

// Finite-beam distortion matrix of every reference ray (Sect. 2.3.2): end
// points r = x_s - x_obs of the five rays (all stopped on the reference
// ray's source surface), differences of the A, B and D, C end points
// projected on the screen basis at the reference end point, divided by
// 2 chi_0 tan(eps).  The second column is taken as (r_D - r_C) so that the
// matrix is the identity without lensing.  A ray of the beam that did not
// reach the source makes the matrix NaN; status gets the first non-zero
// status of the reference, A, B, C, D rays.
__global__ __launch_bounds__(256) void finite_beam_kernel(const BeamObs* __restrict__ obs, int n_obs,
                                                          const RayEnd* __restrict__ ends,
                                                          const double* __restrict__ dirs5,
                                                          const int32_t* __restrict__ status5, double eta0,
                                                          double tan_eps, int64_t n_rays, float* __restrict__ A,
                                                          int32_t* __restrict__ status)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rays) return;
    const int j = beam_observer(obs, n_obs, r);
    const BeamObs& o = obs[j];
    const int64_t loc = r - o.ray_first, c = o.count, b5 = 5 * o.ray_first;
    double x[5][3];
    int32_t st = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int64_t q = b5 + k * c + loc;
        const RayEnd e = ends[q];
        const double s = eta0 - e.eta;
#pragma unroll
        for (int i = 0; i < 3; ++i) x[k][i] = s * dirs5[3 * q + i] + (double)e.dx[i];
        const int32_t sk = status5[q];
        if (st == 0) st = sk;
    }
    if (status) status[r] = st;
    float* a = A + 4 * r;
    if (st != 0) {
        a[0] = a[1] = a[2] = a[3] = __builtin_nanf("");
        return;
    }
    double f1[3], f2[3];
    screen_basis(x[0], f1, f2);
    const double chi0 = sqrt(x[0][0] * x[0][0] + x[0][1] * x[0][1] + x[0][2] * x[0][2]);
    const double den = 2.0 * chi0 * tan_eps;
    double dab[3], ddc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        dab[i] = x[1][i] - x[2][i];
        ddc[i] = x[4][i] - x[3][i];
    }
    a[0] = (float)((dab[0] * f1[0] + dab[1] * f1[1] + dab[2] * f1[2]) / den);
    a[1] = (float)((ddc[0] * f1[0] + ddc[1] * f1[1] + ddc[2] * f1[2]) / den);
    a[2] = (float)((dab[0] * f2[0] + dab[1] * f2[1] + dab[2] * f2[2]) / den);
    a[3] = (float)((ddc[0] * f2[0] + ddc[1] * f2[1] + ddc[2] * f2[2]) / den);
}

inline dim3 blocks_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

hipError_t launch_lensing_maps(const float* A, int64_t n, float* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(lensing_maps_kernel, blocks_for(n), dim3(256), 0, s, A, n, out);
    return hipGetLastError();
}

hipError_t launch_healpix_dirs(int nside, int64_t pix_first, int64_t count, double* dirs, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(healpix_dirs_kernel, blocks_for(count), dim3(256), 0, s, nside, pix_first, count, dirs);
    return hipGetLastError();
}

hipError_t launch_beam_dirs(const BeamObs* obs, int n_obs, int nside, const double* user_dirs, double tan_eps,
                            int64_t n_rays, double* dirs5, hipStream_t s)
{
    if (n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(beam_dirs_kernel, blocks_for(n_rays), dim3(256), 0, s, obs, n_obs, nside, user_dirs,
                       tan_eps, n_rays, dirs5);
    return hipGetLastError();
}

hipError_t launch_finite_beam(const BeamObs* obs, int n_obs, const RayEnd* ends, const double* dirs5,
                              const int32_t* status5, double eta0, double tan_eps, int64_t n_rays, float* A,
                              int32_t* status, hipStream_t s)
{
    if (n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(finite_beam_kernel, blocks_for(n_rays), dim3(256), 0, s, obs, n_obs, ends, dirs5, status5,
                       eta0, tan_eps, n_rays, A, status);
    return hipGetLastError();
}

}  // namespace mpath
