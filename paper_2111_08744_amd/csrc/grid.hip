// grid.hip -- derived octree tables built on the GPU after the upload:
// the 8-cell stencil record of every cell (stored as the trilinear
// coefficients of the 8 payloads), and the stencil that the AMR
// level-fallback procedure (Sect. 2.2: try the leaf level, go one level
// coarser while any of the 8 cells is missing) selects for each half-cell of
// every leaf.
#include <hip/hip_runtime.h>

#include "device.h"

namespace mpath {
namespace {

__global__ void build_dual_kernel(GridDev g, const int4* __restrict__ cellpos, float4* __restrict__ dual, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int4 p = cellpos[c];
    float4 v[8], coef[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const int id = lookup_cell(g, p.w, p.x + (o & 1), p.y + ((o >> 1) & 1), p.z + (o >> 2));
        v[o] = id >= 0 ? g.payload[id] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    trilinear_coefficients(v, coef);
#pragma unroll
    for (int o = 0; o < 8; ++o) dual[8 * c + o] = coef[o];
}

// The same record for dPhi/deta (a time-dependent potential): the 8
// trilinear coefficients of the stencil based at cell c, two float4.
__global__ void build_tdual_kernel(GridDev g, const int4* __restrict__ cellpos, const float* __restrict__ tpay,
                                   float4* __restrict__ tdual, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int4 p = cellpos[c];
    float4 v[8], coef[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const int id = lookup_cell(g, p.w, p.x + (o & 1), p.y + ((o >> 1) & 1), p.z + (o >> 2));
        v[o] = make_float4(id >= 0 ? tpay[id] : 0.f, 0.f, 0.f, 0.f);
    }
    trilinear_coefficients(v, coef);
    tdual[2 * c] = make_float4(coef[0].x, coef[1].x, coef[2].x, coef[3].x);
    tdual[2 * c + 1] = make_float4(coef[4].x, coef[5].x, coef[6].x, coef[7].x);
}

__global__ void build_leafinfo_kernel(GridDev g, const int4* __restrict__ cellpos, int32_t* __restrict__ info,
                                      int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    if (g.child[c] >= 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) info[8 * c + q] = -1;
        return;
    }
    const int4 p = cellpos[c];
    const int L = p.w;
    for (int q = 0; q < 8; ++q) {
        // coordinates of the half-cell q at level L + 1
        const int I0 = 2 * p.x + (q & 1), I1 = 2 * p.y + ((q >> 1) & 1), I2 = 2 * p.z + (q >> 2);
        int base = -1;
        for (int l = L; l >= 0 && base < 0; --l) {
            const int s = L - l;
            const int b0 = ((I0 >> s) - 1) >> 1, b1 = ((I1 >> s) - 1) >> 1, b2 = ((I2 >> s) - 1) >> 1;
            bool ok = true;
            for (int o = 0; o < 8 && ok; ++o)
                ok = lookup_cell(g, l, b0 + (o & 1), b1 + ((o >> 1) & 1), b2 + (o >> 2)) >= 0;
            if (ok) base = lookup_cell(g, l, b0, b1, b2);
        }
        info[8 * c + q] = base;
    }
}

__global__ void build_dual_ids_kernel(GridDev g, const int4* __restrict__ cellpos, int32_t* __restrict__ ids,
                                      int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int4 p = cellpos[c];
#pragma unroll
    for (int o = 0; o < 8; ++o)
        ids[8 * c + o] = lookup_cell(g, p.w, p.x + (o & 1), p.y + ((o >> 1) & 1), p.z + (o >> 2));
}

}  // namespace

hipError_t launch_build_dual_ids(const GridDev& g, const int4* cellpos, int32_t* ids, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(build_dual_ids_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, cellpos, ids, n);
    return hipGetLastError();
}

hipError_t launch_build_dual(const GridDev& g, const int4* cellpos, float4* dual, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(build_dual_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, cellpos, dual, n);
    return hipGetLastError();
}

hipError_t launch_build_tdual(const GridDev& g, const int4* cellpos, const float* tpay, float4* tdual, int64_t n,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(build_tdual_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, cellpos, tpay,
                       tdual, n);
    return hipGetLastError();
}

hipError_t launch_build_leafinfo(const GridDev& g, const int4* cellpos, int32_t* leafinfo, int64_t n,
                                 hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(build_leafinfo_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, cellpos,
                       leafinfo, n);
    return hipGetLastError();
}

}  // namespace mpath
