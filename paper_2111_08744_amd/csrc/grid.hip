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

// The build kernels take the positions of the cells [c0, c0 + m) as a chunk
// pos[0 .. m) = (i, j, k, level) staged by the host.

__device__ __forceinline__ void dual_record(const GridDev& g, int l, int i, int j, int k, float4* __restrict__ out)
{
    float4 v[8], coef[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const int id = lookup_cell(g, l, i + (o & 1), j + ((o >> 1) & 1), k + (o >> 2));
        v[o] = id >= 0 ? g.payload[id] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    trilinear_coefficients(v, coef);
#pragma unroll
    for (int o = 0; o < 8; ++o) out[o] = coef[o];
}

__global__ void build_dual_kernel(GridDev g, const int4* __restrict__ pos, int64_t c0, int64_t m,
                                  float4* __restrict__ dual)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int4 p = pos[t];
    dual_record(g, p.w, p.x, p.y, p.z, dual + 8 * (c0 + t));
}

// The same record from the stored cell ids of each stencil (ids[8 c + o],
// -1 where the cell does not exist): bit-identical to build_dual_kernel,
// which looks the ids up; used when the values change (set_values).
__global__ void rebuild_dual_kernel(GridDev g, const int32_t* __restrict__ ids, float4* __restrict__ dual, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    float4 v[8], coef[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const int id = ids[8 * c + o];
        v[o] = id >= 0 ? g.payload[id] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    trilinear_coefficients(v, coef);
#pragma unroll
    for (int o = 0; o < 8; ++o) dual[8 * c + o] = coef[o];
}

// The same record for dPhi/deta (a time-dependent potential): the 8
// trilinear coefficients of the stencil based at cell c, two float4.
__global__ void build_tdual_kernel(GridDev g, const int4* __restrict__ pos, int64_t c0, int64_t m,
                                   const float* __restrict__ tpay, float4* __restrict__ tdual)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int64_t c = c0 + t;
    const int4 p = pos[t];
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

// Stencil of every half-cell of the refined cells (level >= 1; row
// c - level_start[1]).  Internal cells get -1 rows (never read: a point is
// always located in a leaf).  Leaves of level 0 need no row: their stencil
// is the level-0 one, whose base follows from the Morton order.
__global__ void build_leafinfo_kernel(GridDev g, const int4* __restrict__ pos, int64_t c0, int64_t m,
                                      int32_t* __restrict__ info)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int64_t c = c0 + t;
    int32_t* row = info + 8 * (c - g.level_start[1]);
    if (g.child[c] >= 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) row[q] = -1;
        return;
    }
    const int4 p = pos[t];
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
        row[q] = base;
    }
}

__global__ void build_dual_ids_kernel(GridDev g, const int4* __restrict__ pos, int64_t c0, int64_t m,
                                      int32_t* __restrict__ ids)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int4 p = pos[t];
    int32_t* row = ids + 8 * (c0 + t);
#pragma unroll
    for (int o = 0; o < 8; ++o) row[o] = lookup_cell(g, p.w, p.x + (o & 1), p.y + ((o >> 1) & 1), p.z + (o >> 2));
}

dim3 blocks_for(int64_t m) { return dim3((unsigned)((m + 255) / 256)); }

}  // namespace

hipError_t launch_build_dual_ids(const GridDev& g, const int4* pos, int64_t c0, int64_t m, int32_t* ids,
                                 hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(build_dual_ids_kernel, blocks_for(m), dim3(256), 0, s, g, pos, c0, m, ids);
    return hipGetLastError();
}

hipError_t launch_build_dual(const GridDev& g, const int4* pos, int64_t c0, int64_t m, float4* dual, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(build_dual_kernel, blocks_for(m), dim3(256), 0, s, g, pos, c0, m, dual);
    return hipGetLastError();
}

hipError_t launch_rebuild_dual(const GridDev& g, const int32_t* ids, float4* dual, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(rebuild_dual_kernel, blocks_for(n), dim3(256), 0, s, g, ids, dual, n);
    return hipGetLastError();
}

hipError_t launch_build_tdual(const GridDev& g, const int4* pos, int64_t c0, int64_t m, const float* tpay,
                              float4* tdual, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(build_tdual_kernel, blocks_for(m), dim3(256), 0, s, g, pos, c0, m, tpay, tdual);
    return hipGetLastError();
}

hipError_t launch_build_leafinfo(const GridDev& g, const int4* pos, int64_t c0, int64_t m, int32_t* leafinfo,
                                 hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(build_leafinfo_kernel, blocks_for(m), dim3(256), 0, s, g, pos, c0, m, leafinfo);
    return hipGetLastError();
}

}  // namespace mpath
