// adjoint.hip -- reverse-mode derivative of the ray-casting map on gfx950.
//
// The forward cast (with checkpoints) stores every ray's state before steps
// 0, K, 2K, ...  The adjoint kernel then runs, per ray, one reverse sweep:
// segment by segment from the source back to the observer it recomputes the
// steps of the segment from its checkpoint (the same code as the forward, so
// every leaf level, stencil and landing decision is replayed exactly) into a
// per-ray tape, and for every step in reverse order re-records the four RK4
// stages and applies the transposed Jacobian of the step.
//
// The derivative is that of the discrete map: classical RK4 on the null
// geodesic equations of Sect. 2.2 with CIC interpolation (piecewise
// trilinear, so grad Phi has a piecewise-constant spatial derivative), step
// length h_leaf / N with affine step ds / |k0| (differentiated through k0),
// and the landing step on the source iso-eta surface (implicit step length).
// It is taken on the physical variables (eta, x, k0, k), whose RK4 map equals
// the split one of the forward kernels.  Precision follows the forward: the
// cotangent of the state is accumulated in double precision, while the
// per-stage products (stage Jacobians applied to small cotangent increments)
// run in single precision, like the stage arithmetic of the forward.
//
// Cotangent columns (one reverse sweep carries all of them):
//   beta_1, beta_2   e~_a(beta) . x / |x_s - x_obs|: their values at the
//                    observer, contracted with d k / d theta_b, give the
//                    distortion matrix A_ab = d beta_a / d theta_b (Sect. 2.3)
//   z                the observed redshift z5 (Sect. 2.5): d z5 / d theta_b
//   L                a scalar loss through the per-ray cotangents
//                    (dL/dalpha, dL/dz5); its cotangents of the interpolated
//                    (Phi, grad Phi) at every sub-step are scattered to the
//                    cells with the CIC weights (dL/d cell values).
#include <hip/hip_runtime.h>

#include "device.h"

namespace mpath {
namespace {

// Physical state (eta, x, k0, k) or a cotangent of it, in precision T.
template <class T>
struct PhysT {
    T eta, x[3], k0, k[3];
};
using Phys = PhysT<double>;
using Phys32 = PhysT<float>;

template <class T>
__device__ __forceinline__ void phys_zero(PhysT<T>& a)
{
    a.eta = T(0); a.k0 = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) { a.x[i] = T(0); a.k[i] = T(0); }
}

template <class T, class U>
__device__ __forceinline__ void phys_axpy(PhysT<T>& a, T s, const PhysT<U>& b)
{
    a.eta += s * (T)b.eta; a.k0 += s * (T)b.k0;
#pragma unroll
    for (int i = 0; i < 3; ++i) { a.x[i] += s * (T)b.x[i]; a.k[i] += s * (T)b.k[i]; }
}

template <class T>
__device__ __forceinline__ T phys_dot(const PhysT<T>& a, const PhysT<T>& b)
{
    T s = a.eta * b.eta + a.k0 * b.k0;
#pragma unroll
    for (int i = 0; i < 3; ++i) s += a.x[i] * b.x[i] + a.k[i] * b.k[i];
    return s;
}

__device__ __forceinline__ Phys32 to32(const Phys& a)
{
    Phys32 r;
    r.eta = (float)a.eta; r.k0 = (float)a.k0;
#pragma unroll
    for (int i = 0; i < 3; ++i) { r.x[i] = (float)a.x[i]; r.k[i] = (float)a.k[i]; }
    return r;
}

// What the forward computed at one RK4 stage: the state, the interpolated
// gradient and the stencil (lowest-corner id, level, offsets of the point).
struct StageData {
    GeoState y;
    float G[3], t[3];
    int base, lvl;
};

// The four stages of one RK4 step, kept in this lane's LDS slots (the
// forward's stage loop is not unrolled, so the stage index is a run-time
// value, and the replay must run that same loop to reproduce the forward's
// rounding bit for bit).  Word w of stage i is at p[(i * kWords + w) kBlock].
struct StageRecord {
    static constexpr int kWords = 18;
    float* p;

    __device__ __forceinline__ void put(float* q, int w, float v) const { q[w * kBlock] = v; }
    __device__ __forceinline__ void put64(float* q, int w, double v) const
    {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        q[w * kBlock] = __uint_as_float((unsigned)b);
        q[(w + 1) * kBlock] = __uint_as_float((unsigned)(b >> 32));
    }
    __device__ __forceinline__ double get64(const float* q, int w) const
    {
        const unsigned long long lo = __float_as_uint(q[w * kBlock]);
        const unsigned long long hi = __float_as_uint(q[(w + 1) * kBlock]);
        return __longlong_as_double((long long)(lo | (hi << 32)));
    }

    template <class FC>
    __device__ __forceinline__ void stage(int i, const GeoState&, const GeoState& yi, const FC& F, const float* G,
                                          const HubbleCubic&, const CosmoDev&)
    {
        float* q = p + i * kWords * kBlock;
        put64(q, 0, yi.eta);
        put64(q, 2, yi.K);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            put(q, 4 + k, yi.d[k]);
            put(q, 7 + k, yi.dx[k]);
            put(q, 10 + k, G[k]);
            put(q, 13 + k, F.t[k]);
        }
        put(q, 16, __int_as_float(F.base));
        put(q, 17, __int_as_float(F.lvl));
    }

    // After a stage's transposed Jacobian its gradient words are free: they
    // take the loss cotangent of the interpolated gradient at that stage.
    template <int I>
    __device__ __forceinline__ void put_gbar(const float g[3]) const
    {
        float* q = p + I * kWords * kBlock;
        put(q, 10, g[0]);
        put(q, 11, g[1]);
        put(q, 12, g[2]);
    }
    // stage i (run-time index): stencil base, offsets and the loss cotangent
    __device__ __forceinline__ void scatter_data(int i, int& base, float t[3], float g[3]) const
    {
        const float* q = p + i * kWords * kBlock;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            g[k] = q[(10 + k) * kBlock];
            t[k] = q[(13 + k) * kBlock];
        }
        base = __float_as_int(q[16 * kBlock]);
    }

    template <int I>
    __device__ __forceinline__ StageData get() const
    {
        const float* q = p + I * kWords * kBlock;
        StageData d;
        d.y.eta = get64(q, 0);
        d.y.K = get64(q, 2);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            d.y.d[k] = q[(4 + k) * kBlock];
            d.y.dx[k] = q[(7 + k) * kBlock];
            d.G[k] = q[(10 + k) * kBlock];
            d.t[k] = q[(13 + k) * kBlock];
        }
        d.base = __float_as_int(q[16 * kBlock]);
        d.lvl = __float_as_int(q[17 * kBlock]);
        return d;
    }
};

struct RayCtx {
    RayGeom geo;
    double xobs[3];
};

// Trilinear coefficients (component-major: c[8 q + k]) of a stencil, read
// from the dual table.  (The lane's LDS copy holds only the stencil of the
// replay's last stage; choosing between the two per lane made a wave wait
// for the table whenever any of its lanes missed, and the records of a
// step's stencils are in the caches after its replay.)
__device__ __forceinline__ void stencil_coefs(const GridDev& g, int base, float c[32])
{
    const float4* rec = g.dual + 8 * (int64_t)base;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const float4 q = rec[o];
        c[o] = q.x; c[8 + o] = q.y; c[16 + o] = q.z; c[24 + o] = q.w;
    }
}

// Offsets of a stage position from its stencil's lowest corner, at the
// stencil level (as the forward interpolation computes them).
__device__ __forceinline__ void stage_offsets(const GridDev& g, const RayCtx& R, const GeoState& ys, int lvl,
                                              double t[3])
{
    double v[3];
    grid_coords(g, R.geo, ys.eta, ys.dx, v);
    const double sl = ldexp(1.0, lvl - g.max_level - 1);    // v sl = x 2^lvl / h0 exactly
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double q = v[d] * sl - 0.5;
        t[d] = q - floor(q);
    }
}

// Value and t-derivatives of one trilinear component
// f = c0 + tx (c1 + ty (c4 + tz c7) + tz c5) + ty (c2 + tz c6) + tz c3.
template <class T>
__device__ __forceinline__ void trilinear_jet(const T c[8], T tx, T ty, T tz, T& f, T& fx, T& fy, T& fz)
{
    f = c[0] + tx * (c[1] + ty * (c[4] + tz * c[7]) + tz * c[5]) + ty * (c[2] + tz * c[6]) + tz * c[3];
    fx = c[1] + ty * c[4] + tz * c[5] + ty * tz * c[7];
    fy = c[2] + tx * c[4] + tz * c[6] + tx * tz * c[7];
    fz = c[3] + tx * c[5] + ty * c[6] + tx * ty * c[7];
}

// What the transposed stage Jacobian needs at one stage (single precision).
struct Jet32 {
    float k0, k[3];
    float G[3];
    float JG[3][3];     // dG_j / dx_l of the trilinear interpolant
    float H, dH;        // a'/a and its eta-derivative
    float t[3];         // CIC offsets (weights) at the stencil level
    int base;
};

// Stage quantities that need no stencil coefficients.
__device__ __forceinline__ void jet_from_stage(const AdjointArgs& A, const RayCtx& R, const StageData& d,
                                               const HubbleCubic& Hc, Jet32& J)
{
    const float K = (float)d.y.K;
    J.k0 = -K;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        J.k[i] = K * ((float)R.geo.n[i] + d.y.d[i]);
        J.G[i] = d.G[i];
        J.t[i] = d.t[i];
    }
    J.H = (float)Hc(A.c.cosmo, d.y.eta);
    J.dH = (float)Hc.deriv(A.c.cosmo, d.y.eta);
    J.base = d.base;
}

// Spatial derivatives of the interpolated gradient at the stage: the
// t-derivatives of the trilinear interpolant (Eq. W_CIC) times 2^lvl / h0.
__device__ __forceinline__ void jet_gradient(const GridDev& g, const StageData& d, Jet32& J)
{
    float c[32];
    stencil_coefs(g, d.base, c);
    const float tx = d.t[0], ty = d.t[1], tz = d.t[2];
    const float scale = (float)((double)(1 << d.lvl) * g.inv_h0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float* k = c + 8 * (j + 1);
        J.JG[j][0] = (k[1] + ty * k[4] + tz * k[5] + ty * tz * k[7]) * scale;
        J.JG[j][1] = (k[2] + tx * k[4] + tz * k[6] + tx * tz * k[7]) * scale;
        J.JG[j][2] = (k[3] + tx * k[5] + ty * k[6] + tx * ty * k[7]) * scale;
    }
}

// Right-hand side of the geodesic equations (Sect. 2.2) at a stage.
__device__ __forceinline__ Phys32 rhs32(const Jet32& J)
{
    Phys32 F;
    const float k0 = J.k0;
    const float psi = J.G[0] * J.k[0] + J.G[1] * J.k[1] + J.G[2] * J.k[2];
    F.eta = k0;
    F.k0 = -2.0f * J.H * k0 * k0 - 2.0f * psi * k0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F.x[j] = J.k[j];
        F.k[j] = -2.0f * J.H * k0 * J.k[j] + 2.0f * psi * J.k[j] - 2.0f * J.G[j] * k0 * k0;
    }
    return F;
}

// Transposed Jacobian of the right-hand side at a stage applied to v:
// Yb = (dF/dY)^T v and the cotangent Gb of the interpolated grad Phi.
//   F = (k0, k, -2 H k0^2 - 2 psi k0, -2 H k0 k + 2 psi k - 2 G k0^2), psi = G.k
__device__ __forceinline__ void rhs_vjp32(const Jet32& J, const Phys32& v, Phys32& Yb, float Gb[3])
{
    const float k0 = J.k0;
    const float a = v.k0;
    const float bk = v.k[0] * J.k[0] + v.k[1] * J.k[1] + v.k[2] * J.k[2];
    const float bG = v.k[0] * J.G[0] + v.k[1] * J.G[1] + v.k[2] * J.G[2];
    const float psi = J.G[0] * J.k[0] + J.G[1] * J.k[1] + J.G[2] * J.k[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) Gb[j] = -2.0f * k0 * a * J.k[j] + 2.0f * bk * J.k[j] - 2.0f * k0 * k0 * v.k[j];
    Yb.eta = -2.0f * J.dH * k0 * (a * k0 + bk);
    Yb.k0 = v.eta + a * (-4.0f * J.H * k0 - 2.0f * psi) - 2.0f * J.H * bk - 4.0f * k0 * bG;
#pragma unroll
    for (int j = 0; j < 3; ++j)
        Yb.k[j] = v.x[j] - 2.0f * k0 * a * J.G[j] + (-2.0f * J.H * k0 + 2.0f * psi) * v.k[j] + 2.0f * J.G[j] * bk;
#pragma unroll
    for (int l = 0; l < 3; ++l) Yb.x[l] = J.JG[0][l] * Gb[0] + J.JG[1][l] * Gb[1] + J.JG[2][l] * Gb[2];
}

__device__ __forceinline__ void cic_weights(const float t[3], float w[8])
{
#pragma unroll
    for (int o = 0; o < 8; ++o)
        w[o] = ((o & 1) ? t[0] : 1.0f - t[0]) * ((o & 2) ? t[1] : 1.0f - t[1]) * ((o & 4) ? t[2] : 1.0f - t[2]);
}

// Cell cotangents in the adjoint workspace: component-major (phi, gx, gy,
// gz), and within a component the ids of every aligned group of 8
// consecutive cells (a Morton 2x2x2 block) spread over 8 regions, so that
// the atomics of one stencil flush land in different cache lines instead of
// serialising on one.
__device__ __forceinline__ int64_t grad_slot(int64_t id, int q, int64_t n)
{
    const int64_t m = (n + 7) >> 3;
    return (int64_t)q * (m << 3) + (id & 7) * m + (id >> 3);
}

// Per-wave table in LDS aggregating the gradient cotangents of recently
// touched cells: direct-mapped on a hash of the cell id, filled with LDS
// atomics by the lanes of one wave and evicted to the cell array with device
// atomics when a quarter full (a fuller table sends more colliding cells
// straight to the cell array, which costs more than the extra evictions).
// The 64 rays of a wave start from
// neighbouring sky pixels and cross the same cells many times, so the table
// absorbs most additions and the device atomics (which resolve beyond the
// per-XCD L2) drop by that reuse factor.
constexpr int kTab = 256;               // entries per wave (power of two)
constexpr int kTabWords = 4 * kTab + 4; // keys, 3 value planes, fill counter (padded)

struct WaveTable {
    int* keys;
    float* vals;        // [3][kTab]
    int* count;

    __device__ __forceinline__ void bind(float* base)
    {
        keys = reinterpret_cast<int*>(base);
        vals = base + kTab;
        count = reinterpret_cast<int*>(base + 4 * kTab);
    }

    // every lane of the (full) wave clears a share of the table
    __device__ __forceinline__ void clear(int lane)
    {
        for (int e = lane; e < kTab; e += 64) {
            keys[e] = -1;
            vals[e] = 0.0f;
            vals[kTab + e] = 0.0f;
            vals[2 * kTab + e] = 0.0f;
        }
        if (lane == 0) *count = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }

    // Move every entry to the cell array; the currently active lanes share
    // the work.
    __device__ __forceinline__ void evict(const AdjointArgs& A)
    {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int lane = threadIdx.x & 63;
        const uint64_t act = __ballot(1);
        const int nact = __popcll(act);
        const int rank = __popcll(act & ((1ull << lane) - 1ull));
        for (int e = rank; e < kTab; e += nact) {
            const int key = keys[e];
            if (key >= 0) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const float v = vals[q * kTab + e];
                    if (v != 0.0f) unsafeAtomicAdd(A.grad + grad_slot(key, 1 + q, A.n_cells), v);
                    vals[q * kTab + e] = 0.0f;
                }
                keys[e] = -1;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (rank == 0) *count = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }

    // Add the cotangents acc[o] of the 8 stencil cells ids[o] (-1: no cell).
    // The table is direct-mapped on a hash of the cell id: a cell whose slot
    // is free or already its own is added in LDS; one whose slot holds
    // another cell goes straight to the cell array.  The 8 slot claims are
    // issued together and the LDS additions carry a zero where the slot is
    // not the cell's, so that the common path has no branches.
    __device__ __forceinline__ void add8(const AdjointArgs& A, const int ids[8], const float (&acc)[8][3])
    {
        int h[8], old[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            h[o] = (int)(((uint32_t)ids[o] * 2654435761u) >> (32 - 8));
            old[o] = ids[o] >= 0 ? atomicCAS(&keys[h[o]], -1, ids[o]) : ids[o];
        }
        int claimed = 0;
        uint32_t conflict = 0;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const bool cell = ids[o] >= 0;
            const bool mine = cell && (old[o] == -1 || old[o] == ids[o]);
            claimed += (cell && old[o] == -1) ? 1 : 0;
            conflict |= (cell && !mine) ? (1u << o) : 0u;
            const float m = mine ? 1.0f : 0.0f;
            atomicAdd(&vals[h[o]], m * acc[o][0]);
            atomicAdd(&vals[kTab + h[o]], m * acc[o][1]);
            atomicAdd(&vals[2 * kTab + h[o]], m * acc[o][2]);
        }
        if (claimed) atomicAdd(count, claimed);
        if (conflict) {
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                if (conflict & (1u << o)) {
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        unsafeAtomicAdd(A.grad + grad_slot(ids[o], 1 + q, A.n_cells), acc[o][q]);
                }
            }
        }
    }
};
static_assert(kTab == 256, "the slot hash takes the top 8 bits");

// Per-lane accumulator (registers) of the gradient cotangents of the 8 cells
// of the current stencil.  When the stencil changes the sums move to a
// pending slot in LDS, and pending slots enter the wave's table once per
// step, so that a wave runs the table insertion about once per step rather
// than at every stage where one of its lanes changes stencil.  The cell ids
// of a stencil are loaded when it becomes current, long before they are
// needed.
constexpr int kPendWords = 33;          // 24 sums, 8 cell ids, spare

template <bool AMR>
struct Scatter {
    float acc[8][3];
    int ids[8];
    int cur;
    bool pending;
    float* pend;        // this lane's pending slot: word w at pend[w * kBlock]

    __device__ __forceinline__ void init(float* slot)
    {
        pend = slot;
        pending = false;
        cur = -1;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            ids[o] = -1;
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[o][q] = 0.0f;
        }
    }

    __device__ __forceinline__ void flush_pending(const AdjointArgs& A, WaveTable& T)
    {
        float pa[8][3];
        int pi[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
#pragma unroll
            for (int q = 0; q < 3; ++q) pa[o][q] = pend[(3 * o + q) * kBlock];
            pi[o] = __float_as_int(pend[(24 + o) * kBlock]);
        }
        T.add8(A, pi, pa);
        pending = false;
    }

    // move the current sums to the pending slot (inserting an older pending
    // slot first)
    __device__ __forceinline__ void stash(const AdjointArgs& A, WaveTable& T)
    {
        if (cur < 0) return;
        if (pending) flush_pending(A, T);
#pragma unroll
        for (int o = 0; o < 8; ++o) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                pend[(3 * o + q) * kBlock] = acc[o][q];
                acc[o][q] = 0.0f;
            }
            pend[(24 + o) * kBlock] = __int_as_float(ids[o]);
        }
        pending = true;
        cur = -1;
    }

    __device__ __forceinline__ void end_step(const AdjointArgs& A, WaveTable& T)
    {
        if (pending) flush_pending(A, T);
    }

    __device__ __forceinline__ void flush(const AdjointArgs& A, WaveTable& T)
    {
        stash(A, T);
        end_step(A, T);
    }

    __device__ __forceinline__ void add(const AdjointArgs& A, WaveTable& T, int base, const float t[3],
                                        const float Gb[3])
    {
        if (base != cur) {
            stash(A, T);
            cur = base;
            const int4* p = reinterpret_cast<const int4*>(A.c.grid.dual_ids + 8 * (int64_t)base);
            const int4 a = p[0], b = p[1];
            ids[0] = a.x; ids[1] = a.y; ids[2] = a.z; ids[3] = a.w;
            ids[4] = b.x; ids[5] = b.y; ids[6] = b.z; ids[7] = b.w;
        }
        float w[8];
        cic_weights(t, w);
#pragma unroll
        for (int o = 0; o < 8; ++o)
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[o][q] += w[o] * Gb[q];
    }
};

// Direct atomics of a Phi cotangent onto the 8 cells of a stencil.
__device__ __forceinline__ void scatter_phi(const AdjointArgs& A, int base, const double t[3], double v)
{
    if (v == 0.0) return;
    const int32_t* ids = A.c.grid.dual_ids + 8 * (int64_t)base;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const double w = ((o & 1) ? t[0] : 1.0 - t[0]) * ((o & 2) ? t[1] : 1.0 - t[1]) *
                         ((o & 4) ? t[2] : 1.0 - t[2]);
        const int id = ids[o];
        if (id >= 0) unsafeAtomicAdd(A.grad + grad_slot(id, 0, A.n_cells), (float)(w * v));
    }
}

// Step length and landing decision at the start of a step, exactly as the
// forward kernels take them; the field there (stage 0 of the step) into s0.
template <bool AMR>
__device__ __forceinline__ bool plan_step(const CastArgs& a, FieldCache<AMR>& F, const RayGeom& geo,
                                          const GeoState& y, double eta_s, double& ds, double& dl, bool& landing,
                                          Stage0& s0)
{
    const GridDev& g = a.grid;
    double v[3];
    grid_coords(g, geo, y.eta, y.dx, v);
    int L;
    s0.phi = s0.G[0] = s0.G[1] = s0.G[2] = s0.tv = 0.0f;
    s0.l = 0;
    s0.bad = F.eval(g, v, s0.phi, s0.G, L, s0.l);
    if (L < 0) return false;
    ds = step_length(a, L);
    dl = ds / y.K;
    landing = fma(-y.K, dl, y.eta) < eta_s;
    return true;
}

// One forward step (regular or landing) from y, as in the forward kernels;
// records the stages of the final RK4 pass into rec when record is set.  Returns the
// affine length of the step taken through dl_taken.
template <bool AMR, class Rec>
__device__ __forceinline__ bool forward_step(const CastArgs& a, FieldCache<AMR>& F, const RayGeom& geo,
                                             const GeoState& y, double eta_s, GeoState& yn, Rec& rec, bool record,
                                             double& dl_taken, double& ds_out, bool& landing)
{
    double ds, dl;
    Stage0 s0;
    if (!plan_step<AMR>(a, F, geo, y, eta_s, ds, dl, landing, s0)) return false;
    uint32_t h = 0;
    ds_out = ds;
    if (__builtin_expect(!landing, 1)) {
        // the recorder of stage 0 sees the lane's cache as plan_step left it
        if (rk4_step<FieldCache<AMR>, Rec, true>(a.grid, a.cosmo, F, geo, y, dl, yn, h, rec, record, &s0))
            return false;
        dl_taken = dl;
        return true;
    }
    // landing: two Newton passes for the step length, then the step (a
    // recorded pass evaluates its stage 0 again, since the passes before it
    // moved the lane's cache)
    double dlx = (y.eta - eta_s) / y.K;
    for (int k = 0; k < 3; ++k) {
        const bool rec_pass = record && k == 2;
        if (rk4_step<FieldCache<AMR>, Rec, true>(a.grid, a.cosmo, F, geo, y, dlx, yn, h, rec, rec_pass,
                                                 rec_pass ? nullptr : &s0))
            return false;
        if (k < 2) dlx = dlx + (yn.eta - eta_s) / yn.K;
    }
    dl_taken = dlx;
    return true;
}

// Reverse of one RK4 step for all W cotangent columns: the four stages are
// visited last to first; the jet of a stage is formed once and applied to
// every column.  For y' = y + dl/6 (F1 + 2 F2 + 2 F3 + F4) with
// Y_i = y + c_i dl F_{i-1} (c = 1/2, 1/2, 1):
//   Fbar_4 = dl/6 v,  Ybar_i = J_i^T Fbar_i,
//   Fbar_{i-1} = w_{i-1}/6 dl v + c_i dl Ybar_i,  ybar = v + sum_i Ybar_i,
//   dlbar = sum_i (w_i/6) v.F_i + sum_{i>1} c_i Ybar_i.F_{i-1}.
// Stage I (0-based) is handled with J holding its jet; the recursion moves
// to stage I - 1.
template <int I, bool AMR, int W, bool SCATTER>
__device__ __forceinline__ void reverse_stage(const AdjointArgs& A, const RayCtx& R, const StageRecord& rec,
                                              const HubbleCubic& Hc, float dlf, Jet32& J,
                                              const Phys32 (&v)[W], Phys32 (&Fb)[W], float (&dlbar)[W],
                                              Phys32 (&dy)[W], const float (&lc)[W], Scatter<AMR>& S, WaveTable& T)
{
    Jet32 P;
    Phys32 FP;
    if constexpr (I > 0) {
        jet_from_stage(A, R, rec.template get<I - 1>(), Hc, P);
        FP = rhs32(P);
    }
    constexpr float ci = (I == 3) ? 1.0f : 0.5f;
    constexpr float wprev = (I == 1) ? 1.0f : 2.0f;
    float gL[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < W; ++c) {
        Phys32 Yb;
        float Gb[3];
        rhs_vjp32(J, Fb[c], Yb, Gb);
        phys_axpy(dy[c], 1.0f, Yb);
        if (SCATTER) {
#pragma unroll
            for (int q = 0; q < 3; ++q) gL[q] = fmaf(lc[c], Gb[q], gL[q]);
        }
        if constexpr (I > 0) {
            dlbar[c] += ci * phys_dot(Yb, FP) + (wprev * (1.0f / 6.0f)) * phys_dot(v[c], FP);
            phys_zero(Fb[c]);
            phys_axpy(Fb[c], wprev * (1.0f / 6.0f) * dlf, v[c]);
            phys_axpy(Fb[c], ci * dlf, Yb);
        }
    }
    if (SCATTER) rec.template put_gbar<I>(gL);
    if constexpr (I > 0) {
        J = P;
        jet_gradient(A.c.grid, rec.template get<I - 1>(), J);
        reverse_stage<I - 1, AMR, W, SCATTER>(A, R, rec, Hc, dlf, J, v, Fb, dlbar, dy, lc, S, T);
    }
}

// The loss column is a fixed linear combination of the others when the
// Jacobian columns are carried (its end-point cotangent is
// lc_0 beta_1 + lc_1 beta_2 + lc_2 z, and the sweep is linear), so it is
// not propagated separately: its gradient cotangents are that combination of
// the columns' ones.  Alone (W = 1) it is the only column, with lc_0 = 1.
template <bool AMR, int W, bool SCATTER>
__device__ __forceinline__ void reverse_step(const AdjointArgs& A, const RayCtx& R, const StageRecord& rec,
                                             const HubbleCubic& Hc, double dl,
                                             double ds_reg, double k0_step, Phys (&yb)[W], const float (&lc)[W],
                                             Scatter<AMR>& S, WaveTable& T)
{
    const float dlf = (float)dl;
    Phys32 v[W], Fb[W], dy[W];
    float dlbar[W];
    Jet32 J;
    const StageData d3 = rec.template get<3>();
    jet_from_stage(A, R, d3, Hc, J);
    jet_gradient(A.c.grid, d3, J);
    {
        const Phys32 F4 = rhs32(J);
#pragma unroll
        for (int c = 0; c < W; ++c) {
            v[c] = to32(yb[c]);
            dlbar[c] = phys_dot(v[c], F4) * (1.0f / 6.0f);
            phys_zero(Fb[c]);
            phys_axpy(Fb[c], dlf * (1.0f / 6.0f), v[c]);
            phys_zero(dy[c]);
        }
    }
    reverse_stage<3, AMR, W, SCATTER>(A, R, rec, Hc, dlf, J, v, Fb, dlbar, dy, lc, S, T);
    if (SCATTER) {
        // the stages' gradient cotangents to the cells, last stage first (one
        // copy of the accumulate-and-flush code)
#pragma unroll 1
        for (int i = 3; i >= 0; --i) {
            int base;
            float t[3], g[3];
            rec.scatter_data(i, base, t, g);
            S.add(A, T, base, t, g);
        }
        S.end_step(A, T);
    }
    // the four stage increments, summed in single precision, enter the
    // double-precision cotangent once per step
#pragma unroll
    for (int c = 0; c < W; ++c) phys_axpy(yb[c], 1.0, dy[c]);
    // a regular step has dl = ds / |k0| with ds fixed by the leaf level
    if (ds_reg > 0.0) {
        const double f = ds_reg / (k0_step * k0_step);
#pragma unroll
        for (int c = 0; c < W; ++c) yb[c].k0 += (double)dlbar[c] * f;
    }
}

// Rays without a derivative (not stopped on the source surface, or a replay
// that did not retrace the forward path, which only happens when the cell
// values changed after the cast) get NaN in the per-ray derivative outputs.
__device__ __forceinline__ void write_nan_jacobian(const AdjointArgs& A, int64_t ray)
{
    const float q = __builtin_nanf("");
    if (A.jac) {
#pragma unroll
        for (int i = 0; i < 4; ++i) A.jac[4 * ray + i] = q;
    }
    if (A.dz_dtheta) {
        A.dz_dtheta[2 * ray] = q;
        A.dz_dtheta[2 * ray + 1] = q;
    }
}

// e1 = e_phi, e2 = -e_theta at the direction v
__device__ __forceinline__ void screen_basis(const double v[3], double e1[3], double e2[3])
{
    const double ph = atan2(v[1], v[0]);
    const double th = atan2(hypot(v[0], v[1]), v[2]);
    double sp, cp, st, ct;
    sincos(ph, &sp, &cp);
    sincos(th, &st, &ct);
    e1[0] = -sp; e1[1] = cp; e1[2] = 0.0;
    e2[0] = -cp * ct; e2[1] = -sp * ct; e2[2] = st;
}

// Double-precision interpolation jet at one point (end point and observer):
// Phi, its gradient, grad Phi and the right-hand side there.
struct PointJet {
    double phi, gphi[3], G[3], t[3];
    Phys F;
};

__device__ __forceinline__ void point_jet(const AdjointArgs& A, const RayCtx& R, const GeoState& ys, int base,
                                          int lvl, const HubbleCubic& Hc, PointJet& P)
{
    const GridDev& g = A.c.grid;
    stage_offsets(g, R, ys, lvl, P.t);
    const float4* rec = g.dual + 8 * (int64_t)base;
    double c[4][8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const float4 q = rec[o];
        c[0][o] = q.x; c[1][o] = q.y; c[2][o] = q.z; c[3][o] = q.w;
    }
    const double scale = (double)(1 << lvl) * g.inv_h0;
    double fx, fy, fz;
    trilinear_jet<double>(c[0], P.t[0], P.t[1], P.t[2], P.phi, fx, fy, fz);
    P.gphi[0] = fx * scale; P.gphi[1] = fy * scale; P.gphi[2] = fz * scale;
#pragma unroll
    for (int j = 0; j < 3; ++j) trilinear_jet<double>(c[j + 1], P.t[0], P.t[1], P.t[2], P.G[j], fx, fy, fz);
    const double H = Hc(A.c.cosmo, ys.eta);
    const double k0 = -ys.K;
    double k[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) k[i] = ys.K * (R.geo.n[i] + (double)ys.d[i]);
    const double psi = P.G[0] * k[0] + P.G[1] * k[1] + P.G[2] * k[2];
    P.F.eta = k0;
    P.F.k0 = -2.0 * H * k0 * k0 - 2.0 * psi * k0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        P.F.x[j] = k[j];
        P.F.k[j] = -2.0 * H * k0 * k[j] + 2.0 * psi * k[j] - 2.0 * P.G[j] * k0 * k0;
    }
}

// Cotangents of the state at the end point yf (on the source surface):
// beta_a and z columns, and the loss column from dL/dalpha and dL/dz5; the
// direct Phi_s term of the loss is scattered to the end point's stencil and
// the Phi_o term returned.  The landing step has its length set by
// eta(y_f) = eta_s, so the cotangent along the flow F(y_f) is removed.
template <bool AMR, int W, bool SCATTER>
__device__ __forceinline__ void end_cotangents(const AdjointArgs& A, const RayCtx& R, FieldCache<AMR>& F,
                                               const ObsDev& ob, int64_t ray, const GeoState& yf, double phio,
                                               const double e1[3], const double e2[3], Phys (&yb)[W],
                                               float (&lc)[W], double& phio_bar)
{
    constexpr bool HAS_JAC = W >= 3;
    const GridDev& g = A.c.grid;
    float ph_f, Gt[3];
    int ll, lv;
    double vf[3];
    grid_coords(g, R.geo, yf.eta, yf.dx, vf);
    F.eval(g, vf, ph_f, Gt, ll, lv);
    HubbleCubic Hf;
    Hf.init(A.c.cosmo, yf.eta);
    PointJet Jf;
    point_jet(A, R, yf, F.base, F.lvl, Hf, Jf);
    const int end_base = F.base;
    const double* n = R.geo.n;
    double r[3];
    const double sf = g.eta0 - yf.eta;
#pragma unroll
    for (int i = 0; i < 3; ++i) r[i] = sf * n[i] + (double)yf.dx[i];
    const double chi = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double rh[3] = {r[0] / chi, r[1] / chi, r[2] / chi};
    double f1[3], f2[3];
    screen_basis(rh, f1, f2);
    const double phis = Jf.phi;
    const double a_s = A.c.ray_stop ? A.c.ray_stop[ray].y : ob.a_s;
    const double dz_dK = a_s * (1.0 + phis) / (1.0 + phio);
    const double dz_dphis = a_s * yf.K / (1.0 + phio);
    const double dz_dphio = -a_s * yf.K * (1.0 + phis) / ((1.0 + phio) * (1.0 + phio));
#pragma unroll
    for (int c = 0; c < W; ++c) phys_zero(yb[c]);
    if (HAS_JAC) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            yb[0].x[i] = f1[i] / chi;
            yb[1].x[i] = f2[i] / chi;
            yb[2].x[i] = dz_dphis * Jf.gphi[i];
        }
        yb[2].k0 = -dz_dK;
    }
    phio_bar = 0.0;
    if (SCATTER) {
        const float ga0 = A.dL_dalpha ? A.dL_dalpha[2 * ray] : 0.0f;
        const float ga1 = A.dL_dalpha ? A.dL_dalpha[2 * ray + 1] : 0.0f;
        const double gz = A.dL_dz ? A.dL_dz[ray] : 0.0;
        // alpha = -f(sigma) t, t = r^ - (r^.n) n, sin sigma = |t|, f = sigma / sin sigma;
        // d alpha_a / d r^ . e~_b = -f e_a.e~_b + (f'/sin sigma)(e_a.t)(n.e~_b)
        const double cth = rh[0] * n[0] + rh[1] * n[1] + rh[2] * n[2];
        double t[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) t[i] = rh[i] - cth * n[i];
        const double st = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        const double sig = atan2(st, cth);
        double fs, fps;           // f and f'/sin sigma (series below 1e-3 rad)
        if (sig < 1e-3) {
            fs = 1.0 + sig * sig / 6.0;
            fps = 1.0 / 3.0 + sig * sig * (2.0 / 15.0);
        } else {
            fs = sig / st;
            fps = (st - sig * cth) / (st * st * st);
        }
        const double ga[2] = {ga0, ga1};
        const double* ea[2] = {e1, e2};
        const double* fb[2] = {f1, f2};
        double cb[2] = {0.0, 0.0};
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) {
            const double et = ea[aa][0] * t[0] + ea[aa][1] * t[1] + ea[aa][2] * t[2];
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) {
                const double ee = ea[aa][0] * fb[bb][0] + ea[aa][1] * fb[bb][1] + ea[aa][2] * fb[bb][2];
                const double ne = n[0] * fb[bb][0] + n[1] * fb[bb][1] + n[2] * fb[bb][2];
                cb[bb] += ga[aa] * (-fs * ee + fps * et * ne);
            }
        }
        if constexpr (W == 1) {
            Phys& L = yb[0];
#pragma unroll
            for (int i = 0; i < 3; ++i) L.x[i] = (cb[0] * f1[i] + cb[1] * f2[i]) / chi + gz * dz_dphis * Jf.gphi[i];
            L.k0 = -gz * dz_dK;
            lc[0] = 1.0f;
        } else {
            lc[0] = (float)cb[0];
            lc[1] = (float)cb[1];
            lc[2] = (float)gz;
        }
        scatter_phi(A, end_base, Jf.t, gz * dz_dphis);
        phio_bar = gz * dz_dphio;
    }
#pragma unroll
    for (int c = 0; c < W; ++c) yb[c].eta -= phys_dot(yb[c], Jf.F) / Jf.F.eta;
}

// W cotangent columns: W = 3 (beta_1, beta_2, z) or 1 (the loss L).
// SCATTER: the cell cotangents of L are kept (with W = 3, L is the
// combination lc of the three columns).
template <bool AMR, int W, bool SCATTER>
__global__ __launch_bounds__(kBlock, 1) void adjoint_kernel(AdjointArgs A)
{
    // LDS: [32][kBlock] stencil coefficients, [4 * 18][kBlock] stage records,
    // [33][kBlock] pending scatter sums, then one table per wave
    extern __shared__ float lds[];
    WaveTable T;
    if (SCATTER) {
        T.bind(lds + (32 + 4 * StageRecord::kWords + kPendWords) * kBlock + (threadIdx.x >> 6) * kTabWords);
        T.clear(threadIdx.x & 63);
    }
    const int64_t ray = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const CastArgs& a = A.c;
    if (ray >= a.n_rays) return;
    constexpr bool HAS_JAC = W >= 3;
    const int N = A.n_steps[ray];
    if (A.status[ray] != MPATH_RAY_REACHED || N <= 0) {
        if (HAS_JAC) write_nan_jacobian(A, ray);
        if (A.ray_status) A.ray_status[ray] = 1;
        return;
    }
    const GridDev& g = a.grid;
    int j = a.n_obs - 1;
    while (j > 0 && a.obs[j].ray_first > ray) --j;
    const ObsDev& ob = a.obs[j];
    RayCtx R;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        R.xobs[i] = ob.x[i];
        R.geo.vo[i] = ldexp(ob.x[i] / g.h0, g.max_level + 1);
        R.geo.n[i] = a.dirs[3 * ray + i];
    }
    const double eta_s = a.ray_stop ? a.ray_stop[ray].x : ob.eta_s;
    FieldCache<AMR> F;
    F.bind(lds + threadIdx.x);
    F.reset();

    // potential at the observer and the initial |k| (as in the forward)
    float phio_f, Gt[3];
    int ll, lv;
    F.eval(g, R.geo.vo, phio_f, Gt, ll, lv);
    const int obs_base = F.base, obs_lvl = F.lvl;
    const double phio = (double)phio_f;
    const double kmag = sqrt((1.0 + 2.0 * phio) / (1.0 - 2.0 * phio));

    const int K = a.ckpt_every;
    const int nseg = (N + K - 1) / K;
    const double* n = R.geo.n;
    double e1[3], e2[3];
    screen_basis(n, e1, e2);
    Phys yb[W];
    float lc[W];
#pragma unroll
    for (int c = 0; c < W; ++c) lc[c] = 0.0f;
    double phio_bar = 0.0;
    Scatter<AMR> S;
    S.init(lds + (32 + 4 * StageRecord::kWords) * kBlock + threadIdx.x);

    // Segments from the source back to the observer.  Each is traversed
    // forwards from its checkpoint (storing the state before every step in
    // the tape; the last step of a segment other than the final one is not
    // needed, its result being the next checkpoint), then backwards with the
    // stages of every step re-recorded and reversed.  One loop with a single
    // step call site serves both directions.
    bool ok = true;
    // the tape entry of the next reverse step and the next segment's
    // checkpoint are loaded one iteration ahead of their use
    GeoState pre, ck = a.ckpt[(int64_t)(nseg - 1) * a.n_rays + ray];
    for (int seg = nseg - 1; seg >= 0 && ok; --seg) {
        const bool last = seg == nseg - 1;
        const int j0 = seg * K;
        const int len = min(N, j0 + K) - j0;
        const int nf = last ? len : len - 1;
        GeoState y = ck, yin = ck;
        for (int it = 0; it < nf + len; ++it) {
            const bool fwd = it < nf;
            // the lanes still iterating empty the table when it is a quarter full
            if (SCATTER && *T.count > kTab / 4) T.evict(A);
            if (it == nf) {
                // the state before the segment's last step is in registers
                pre = last ? yin : y;
                if (seg > 0) ck = a.ckpt[(int64_t)(seg - 1) * a.n_rays + ray];
                if (last) {
                    // the replay must end where the forward cast ended, bit for bit
                    const RayEnd e = a.ends[ray];
                    if (y.eta != e.eta || y.dx[0] != e.dx[0] || y.dx[1] != e.dx[1] || y.dx[2] != e.dx[2]) {
                        ok = false;
                        break;
                    }
                    end_cotangents<AMR, W, SCATTER>(A, R, F, ob, ray, y, phio, e1, e2, yb, lc, phio_bar);
                }
            }
            const int jl = fwd ? it : len - 1 - (it - nf);
            GeoState ys;
            if (fwd) {
                A.tape[(int64_t)jl * a.n_rays + ray] = y;
                ys = y;
                yin = y;
            } else {
                ys = pre;
                if (jl > 0) pre = A.tape[(int64_t)(jl - 1) * a.n_rays + ray];
            }
            StageRecord rec;
            rec.p = lds + 32 * kBlock + threadIdx.x;
            GeoState yn;
            double dl, ds;
            bool landing;
            if (!forward_step<AMR, StageRecord>(a, F, R.geo, ys, eta_s, yn, rec, !fwd, dl, ds, landing)) {
                ok = false;
                break;
            }
            if (fwd) {
                y = yn;
            } else {
                HubbleCubic Hc;
                Hc.init(a.cosmo, ys.eta);
                const double ds_reg = landing ? 0.0 : ds;
                reverse_step<AMR, W, SCATTER>(A, R, rec, Hc, dl, ds_reg, -ys.K, yb, lc, S, T);
            }
        }
    }

    // ---- the initial state: k = kmag(Phi_o) n (theta), k0 = -1 ----
    if (HAS_JAC && !ok) write_nan_jacobian(A, ray);
    if (A.ray_status) A.ray_status[ray] = ok ? 0 : 2;
    if (HAS_JAC && ok) {
        const double* eb[2] = {e1, e2};
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
            const double db0 = kmag * (yb[0].k[0] * eb[bb][0] + yb[0].k[1] * eb[bb][1] + yb[0].k[2] * eb[bb][2]);
            const double db1 = kmag * (yb[1].k[0] * eb[bb][0] + yb[1].k[1] * eb[bb][1] + yb[1].k[2] * eb[bb][2]);
            const double dz = kmag * (yb[2].k[0] * eb[bb][0] + yb[2].k[1] * eb[bb][1] + yb[2].k[2] * eb[bb][2]);
            if (A.jac) {
                A.jac[4 * ray + bb] = (float)db0;          // row beta_1
                A.jac[4 * ray + 2 + bb] = (float)db1;      // row beta_2
            }
            if (A.dz_dtheta) A.dz_dtheta[2 * ray + bb] = (float)dz;
        }
    }
    if (SCATTER) {
        if (ok) {
            S.flush(A, T);
            double Lk[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < W; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) Lk[i] += (double)lc[c] * yb[c].k[i];
            const double dkmag = kmag * 2.0 / (1.0 - 4.0 * phio * phio);
            phio_bar += (Lk[0] * n[0] + Lk[1] * n[1] + Lk[2] * n[2]) * dkmag;
            GeoState y0;
            y0.eta = g.eta0;
            y0.K = 1.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) { y0.d[i] = 0.0f; y0.dx[i] = 0.0f; }
            double t0[3];
            stage_offsets(g, R, y0, obs_lvl, t0);
            scatter_phi(A, obs_base, t0, phio_bar);
        }
        // every lane that took a ray arrives here together: empty the table
        T.evict(A);
    }
}

__global__ void fill_zero_kernel(float* __restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Cell cotangents from the workspace layout to the caller's order and
// layout [n][4] (overwrites).
__global__ void scatter_grad_kernel(const float* __restrict__ g_lib, const int64_t* __restrict__ perm,
                                    float4* __restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[perm[i]] = make_float4(g_lib[grad_slot(i, 0, n)], g_lib[grad_slot(i, 1, n)], g_lib[grad_slot(i, 2, n)],
                               g_lib[grad_slot(i, 3, n)]);
}

// On a uniform periodic grid whose gradient is the central difference of the
// potential, g_d[c] = (Phi[c + e_d] - Phi[c - e_d]) / (2 h0), the total
// cotangent of Phi is the direct one plus the transposed difference operator
// applied to the cotangents of g:
//   dL/dPhi[c] += sum_d (gbar_d[c - e_d] - gbar_d[c + e_d]) / (2 h0).
__global__ void central_transpose_kernel(const float* __restrict__ g_lib, const int64_t* __restrict__ perm,
                                         float* __restrict__ out, int n0, double inv_2h, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    // the id of a coarse cell is its Morton index
    const int3 p = make_int3((int)compact1by2((uint32_t)c), (int)compact1by2((uint32_t)c >> 1),
                             (int)compact1by2((uint32_t)c >> 2));
    const uint32_t m = (uint32_t)n0 - 1u;
    auto id = [m](int i, int j, int k) { return (int64_t)morton3((uint32_t)i & m, (uint32_t)j & m, (uint32_t)k & m); };
    auto gq = [&](int64_t cell, int q) { return (double)g_lib[grad_slot(cell, q, n)]; };
    double acc = gq(c, 0);
    acc += (gq(id(p.x - 1, p.y, p.z), 1) - gq(id(p.x + 1, p.y, p.z), 1)) * inv_2h;
    acc += (gq(id(p.x, p.y - 1, p.z), 2) - gq(id(p.x, p.y + 1, p.z), 2)) * inv_2h;
    acc += (gq(id(p.x, p.y, p.z - 1), 3) - gq(id(p.x, p.y, p.z + 1), 3)) * inv_2h;
    out[perm[c]] = (float)acc;
}

}  // namespace

hipError_t launch_adjoint(const AdjointArgs& A, int columns, hipStream_t s)
{
    const int64_t n = A.c.n_rays;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    const size_t lds_cache = (size_t)(32 + 4 * StageRecord::kWords) * kBlock * sizeof(float);
    const size_t lds = lds_cache + (columns == 3 ? 0 : ((size_t)kPendWords * kBlock + (size_t)(kBlock / 64) * kTabWords) *
                                                          sizeof(float));
    const bool amr = A.c.grid.max_level > 0;
    if (columns == 4) {
        if (amr) hipLaunchKernelGGL((adjoint_kernel<true, 3, true>), grid, block, lds, s, A);
        else hipLaunchKernelGGL((adjoint_kernel<false, 3, true>), grid, block, lds, s, A);
    } else if (columns == 3) {
        if (amr) hipLaunchKernelGGL((adjoint_kernel<true, 3, false>), grid, block, lds, s, A);
        else hipLaunchKernelGGL((adjoint_kernel<false, 3, false>), grid, block, lds, s, A);
    } else {
        if (amr) hipLaunchKernelGGL((adjoint_kernel<true, 1, true>), grid, block, lds, s, A);
        else hipLaunchKernelGGL((adjoint_kernel<false, 1, true>), grid, block, lds, s, A);
    }
    return hipGetLastError();
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_scatter_grad(const float* grad_lib, const int64_t* perm, float4* out_user, int64_t n,
                               hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, grad_lib, perm,
                       out_user, n);
    return hipGetLastError();
}

hipError_t launch_central_transpose(const float* g_lib, const int64_t* perm, float* out, int n0, double h0,
                                    int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(central_transpose_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g_lib, perm,
                       out, n0, 0.5 / h0, n);
    return hipGetLastError();
}

}  // namespace mpath
