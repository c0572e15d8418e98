// Random-record gather probe: the throughput ceiling of data-dependent
// lookups into a table of a given size, against which the integration
// kernel's table reads (stencil coefficients, stencil-table entries, child
// links) are measured.  Not a step of the method.
//
// Every lane draws record indices uniformly over the table from its own
// xorshift64 sequence (Marsaglia 2003, shifts 13, 7, 17; the index is the high
// half of the 128-bit product of the draw and the record count) and reads
// whole records (16, 64 or 128 bytes,
// 16-byte aligned) with `in_flight` independent gathers outstanding per
// lane; the loaded words are summed into one float per lane so that no load
// is dead.  Waves are one-per-workgroup, so the grid size sets the number of
// resident waves directly.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mpath {
namespace {

__device__ __forceinline__ uint64_t xorshift64(uint64_t s)
{
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return s;
}

template <int R16, int U>
__global__ __launch_bounds__(64) void gather_probe_kernel(const float4* __restrict__ table, uint64_t n_records,
                                                          int iters, uint32_t seed, float* __restrict__ out)
{
    const uint32_t lane = blockIdx.x * 64u + threadIdx.x;
    // distinct non-zero start per lane (the multiplier is odd, so the map is a bijection)
    uint64_t s = ((uint64_t)lane + 1u) * 0x9E3779B97F4A7C15ull ^ ((uint64_t)seed << 17);
    if (s == 0u) s = 0x6D2B79F5ull;
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
        float4 v[U][R16];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s = xorshift64(s);
            const uint64_t r = __umul64hi(s, n_records);          // uniform in [0, n_records)
            const float4* p = table + r * R16;
#pragma unroll
            for (int j = 0; j < R16; ++j) v[u][j] = p[j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < R16; ++j) acc += (v[u][j].x + v[u][j].y) + (v[u][j].z + v[u][j].w);
    }
    out[lane] = acc;
}

template <int R16>
hipError_t launch_r(const float4* t, uint64_t nrec, int in_flight, int64_t n_waves, int iters, uint32_t seed,
                    float* out, hipStream_t s)
{
    const dim3 grid((unsigned)n_waves), block(64);
    switch (in_flight) {
        case 1: hipLaunchKernelGGL((gather_probe_kernel<R16, 1>), grid, block, 0, s, t, nrec, iters, seed, out); break;
        case 2: hipLaunchKernelGGL((gather_probe_kernel<R16, 2>), grid, block, 0, s, t, nrec, iters, seed, out); break;
        default: hipLaunchKernelGGL((gather_probe_kernel<R16, 4>), grid, block, 0, s, t, nrec, iters, seed, out); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gather_probe(const void* table, size_t table_bytes, int record_bytes, int in_flight,
                               int64_t n_waves, int iters, uint32_t seed, float* out, hipStream_t s)
{
    const float4* t = static_cast<const float4*>(table);
    const uint64_t nrec = table_bytes / (uint64_t)record_bytes;
    switch (record_bytes) {
        case 16: return launch_r<1>(t, nrec, in_flight, n_waves, iters, seed, out, s);
        case 64: return launch_r<4>(t, nrec, in_flight, n_waves, iters, seed, out, s);
        default: return launch_r<8>(t, nrec, in_flight, n_waves, iters, seed, out, s);
    }
}

}  // namespace mpath
