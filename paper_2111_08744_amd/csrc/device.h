// device.h -- device-side building blocks of the ray tracer: HEALPix
// directions, the tabulated conformal Hubble rate, octree lookups with the
// AMR level fallback and a lane-resident stencil cache, and one RK4 step of
// the null geodesic equations in the split FP64/FP32 representation.
#pragma once

#include "internal.h"

namespace mpath {

constexpr uint32_t kFnvOffset = 2166136261u;
constexpr int kBlock = 256;       // threads per block of the integration kernels
constexpr uint32_t kFnvPrime = 16777619u;

__device__ __forceinline__ uint32_t fnv(uint32_t h, uint32_t v) { return (h ^ v) * kFnvPrime; }

// The GPU hands consecutive workgroups to its 8 XCDs in turn, and each XCD
// has its own L2.  Renumber workgroups so that each XCD runs a contiguous
// range of them (consecutive rays are neighbouring sky pixels whose paths
// share cells): XCD x = b mod 8 takes logical blocks
// [start(x), start(x) + count(x)) in the order it receives them.
constexpr int kNumXcd = 8;

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks)
{
    const int64_t q = nblocks / kNumXcd, r = nblocks % kNumXcd;
    const int64_t x = b % kNumXcd, idx = b / kNumXcd;
    return x < r ? x * (q + 1) + idx : r * (q + 1) + (x - r) * q + idx;
}

// ---------------------------------------------------------------------------
// HEALPix NESTED pixel centre (Gorski et al. 2005; Sect. 2.4 starts one photon
// at every pixel centre).  Within base face f the nested index interleaves
// the face coordinates (x in the even bits, y in the odd bits); the ring
// counted from the north pole is jr = (2 + f/4) nside - x - y - 1; the
// azimuth is pi/4 (jpll + (x - y)/nr) with jpll = 2 (f mod 4) + 1 on the
// polar faces and 2 (f mod 4) on the equatorial ones.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t compact1by1(uint32_t x)
{
    x &= 0x55555555u;
    x = (x ^ (x >> 1)) & 0x33333333u;
    x = (x ^ (x >> 2)) & 0x0f0f0f0fu;
    x = (x ^ (x >> 4)) & 0x00ff00ffu;
    x = (x ^ (x >> 8)) & 0x0000ffffu;
    return x;
}

__device__ inline void healpix_nest_dir(int64_t nside, int64_t pix, double v[3])
{
    const int64_t npface = nside * nside;
    const int face = (int)(pix / npface);
    const uint32_t ip = (uint32_t)(pix - (int64_t)face * npface);
    const int64_t x = compact1by1(ip), y = compact1by1(ip >> 1);
    const int64_t jr = (int64_t)(2 + face / 4) * nside - x - y - 1;
    const int jpll = 2 * (face & 3) + ((face >> 2) != 1 ? 1 : 0);
    const double three_ns2 = 3.0 * (double)nside * (double)nside;
    int64_t nr;
    double z, st;
    if (jr < nside) {
        nr = jr;
        const double one_minus_z = (double)(nr * nr) / three_ns2;
        z = 1.0 - one_minus_z;
        st = sqrt(one_minus_z * (2.0 - one_minus_z));
    } else if (jr > 3 * nside) {
        nr = 4 * nside - jr;
        const double one_plus_z = (double)(nr * nr) / three_ns2;
        z = one_plus_z - 1.0;
        st = sqrt(one_plus_z * (2.0 - one_plus_z));
    } else {
        nr = nside;
        z = (double)(2 * nside - jr) * 2.0 / (3.0 * (double)nside);
        st = sqrt((1.0 - z) * (1.0 + z));
    }
    const double ph = 0.25 * M_PI * ((double)jpll + (double)(x - y) / (double)nr);
    double sp, cp;
    sincos(ph, &sp, &cp);
    v[0] = st * cp;
    v[1] = st * sp;
    v[2] = z;
}

// Conformal Hubble rate a'/a near a conformal time eta_n: the cubic Hermite
// interpolant of the uniform table on the interval holding eta_n, re-expanded
// about eta_n, so that the sub-steps of one RK4 step (|eta - eta_n| <= one
// step, less than the table spacing) evaluate it with three FMAs.  Outside
// its interval the cubic deviates from the Hermite interpolant of the
// neighbouring interval by O(h^4 H'''') ~ 1e-18.
struct HubbleCubic {
    double b0, b1, b2, b3;   // H(eta_n + tau h) = b0 + tau (b1 + tau (b2 + tau b3))
    double eta_n;

    __device__ __forceinline__ void init(const CosmoDev& c, double eta)
    {
        #pragma clang fp contract(off)
        eta_n = eta;
        if (c.is_static) { b0 = b1 = b2 = b3 = 0.0; return; }
        const double u = (eta - c.eta_lo) * c.inv_deta;
        int i = (int)floor(u);
        i = i < 0 ? 0 : (i > c.n - 2 ? c.n - 2 : i);
        const double t = u - (double)i;
        const double2 p0 = c.table[i];
        const double2 p1 = c.table[i + 1];
        // Hermite cubic in t: a0 + a1 t + a2 t^2 + a3 t^3
        const double a0 = p0.x, a1 = c.deta * p0.y;
        const double a2 = fma(-c.deta, fma(2.0, p0.y, p1.y), 3.0 * (p1.x - p0.x));
        const double a3 = fma(c.deta, p0.y + p1.y, 2.0 * (p0.x - p1.x));
        // Taylor coefficients about t
        const double t3 = 3.0 * t;
        b0 = fma(t, fma(t, fma(t, a3, a2), a1), a0);
        b1 = fma(t, fma(t3, a3, 2.0 * a2), a1);
        b2 = fma(t3, a3, a2);
        b3 = a3;
    }

    __device__ __forceinline__ double operator()(const CosmoDev& c, double eta) const
    {
        #pragma clang fp contract(off)
        const double tau = (eta - eta_n) * c.inv_deta;
        return fma(tau, fma(tau, fma(tau, b3, b2), b1), b0);
    }

    // d(a'/a)/d eta of the same cubic
    __device__ __forceinline__ double deriv(const CosmoDev& c, double eta) const
    {
        const double tau = (eta - eta_n) * c.inv_deta;
        return (b1 + tau * (2.0 * b2 + 3.0 * tau * b3)) * c.inv_deta;
    }
};

// Scale factor a(eta): cubic Hermite interpolation of the (a, da/deta) table
// on the nodes of the a'/a table (1 on a static background).
__device__ inline double scale_factor(const CosmoDev& c, double eta)
{
    if (c.is_static) return 1.0;
    const double u = (eta - c.eta_lo) * c.inv_deta;
    int i = (int)floor(u);
    i = i < 0 ? 0 : (i > c.n - 2 ? c.n - 2 : i);
    const double t = u - (double)i;
    const double2 p0 = c.atable[i];
    const double2 p1 = c.atable[i + 1];
    const double a0 = p0.x, a1 = c.deta * p0.y;
    const double a2 = fma(-c.deta, fma(2.0, p0.y, p1.y), 3.0 * (p1.x - p0.x));
    const double a3 = fma(c.deta, p0.y + p1.y, 2.0 * (p0.x - p1.x));
    return fma(t, fma(t, fma(t, a3, a2), a1), a0);
}

// ---------------------------------------------------------------------------
// Octree lookups.  Integer cell coordinates are kept unwrapped (a periodic
// ray may leave the box) and wrapped only to address memory.
// ---------------------------------------------------------------------------

// Id of cell (l, J) or -1 if it does not exist: coarse ancestor by Morton
// index, then one child link per level.
__host__ __device__ __forceinline__ int lookup_cell(const GridDev& g, int l, int J0, int J1, int J2)
{
    const int M = g.n0 << l;
    if (g.periodic) {
        J0 &= M - 1; J1 &= M - 1; J2 &= M - 1;
    } else if ((unsigned)J0 >= (unsigned)M || (unsigned)J1 >= (unsigned)M || (unsigned)J2 >= (unsigned)M) {
        return -1;
    }
    int id = (int)morton3((uint32_t)(J0 >> l), (uint32_t)(J1 >> l), (uint32_t)(J2 >> l));
    for (int m = l - 1; m >= 0; --m) {
        const int ch = g.child[id];
        if (ch < 0) return -1;
        id = ch + (((J0 >> m) & 1) | (((J1 >> m) & 1) << 1) | (((J2 >> m) & 1) << 2));
    }
    return id;
}

// Level of a cell id (ids are level-major).  The scan stops at the grid's
// deepest level (a uniform branch), and the unrolled comparisons keep the
// level table in scalar registers (a dynamically indexed array would be
// copied to vector registers).
__device__ __forceinline__ int level_of(const GridDev& g, int id)
{
    int l = 0;
#pragma unroll
    for (int k = 1; k < kMaxLevels; ++k) {
        if (k > g.max_level) break;
        l += (id >= g.level_start[k]) ? 1 : 0;
    }
    return l;
}

// Trilinear coefficients of the 8 corner payloads v[o] (o = ox + 2 oy + 4 oz):
// f(t) = c0 + c1 tx + c2 ty + c3 tz + c4 tx ty + c5 tx tz + c6 ty tz + c7 tx ty tz,
// which equals sum_o prod_d W_CIC(t_d - o_d) v[o] for t in [0, 1]^3.
__device__ __forceinline__ void trilinear_coefficients(const float4 v[8], float4 c[8])
{
#define MPATH_TRI(f)                                                       \
    {                                                                      \
        const float c1 = v[1].f - v[0].f, c2 = v[2].f - v[0].f;            \
        const float c4 = v[3].f - v[2].f - c1;                             \
        c[0].f = v[0].f;                                                   \
        c[1].f = c1;                                                       \
        c[2].f = c2;                                                       \
        c[3].f = v[4].f - v[0].f;                                          \
        c[4].f = c4;                                                       \
        c[5].f = v[5].f - v[4].f - c1;                                     \
        c[6].f = v[6].f - v[4].f - c2;                                     \
        c[7].f = v[7].f - v[6].f - v[5].f + v[4].f - c4;                   \
    }
    MPATH_TRI(x) MPATH_TRI(y) MPATH_TRI(z) MPATH_TRI(w)
#undef MPATH_TRI
}

__device__ __forceinline__ float trilinear_eval(float c0, float c1, float c2, float c3, float c4, float c5,
                                                float c6, float c7, float tx, float ty, float tz)
{
    #pragma clang fp contract(off)
    const float a = fmaf(tz, c5, fmaf(ty, fmaf(tz, c7, c4), c1));
    const float b = fmaf(tz, c6, c2);
    return fmaf(tz, c3, fmaf(ty, b, fmaf(tx, a, c0)));
}

// Field value interpolated at one point, with the lane's cache of the leaf
// cell and of the last resolved 8-cell stencil (as trilinear coefficients).
//
// Reuse is exact: the leaf level of x only changes when x leaves the cached
// leaf cell, and for x inside a leaf cell of level L the CIC base at every
// level l <= L is a function of floor(x / h_{L+1}) alone (the half of the
// leaf cell x lies in per axis), so the resolved stencil is a function of
// (leaf cell, floor(x / h_{L+1})); the build precomputes it per half-cell.
//
// TIME: the grid also carries dPhi/deta (Sect. 2.2, from a double-layer
// light cone); its 8 coefficients follow the 32 of (phi, grad) in LDS and
// eval leaves the interpolated value in tv.  ONE_EXIT: eval without early
// returns (measured faster inside the RK4 stage loop on the uniform grid;
// the refined grid and the field probes of the beams keep the returns).
template <bool AMR, bool TIME = false, bool ONE_EXIT = !AMR>
struct FieldCache {
    static constexpr bool kTime = TIME;
    int leafId;         // id of the leaf cell containing the cached half-cell
    int keyL;           // level of that leaf (-1: nothing cached)
    int key[3];         // unwrapped coordinates of the half-cell at level keyL + 1
    int lvl;            // level of the resolved stencil
    int base;           // id of its lowest corner cell
    float t[3];         // offsets of the last evaluated point in that stencil
    float* c;           // trilinear coefficients in LDS: coefficient k of
                        // component f (phi, gx, gy, gz[, dphi/deta]) at c[(8 f + k) * kBlock]
    float tv;           // TIME: dPhi/deta at the last evaluated point
    float isw_step;     // TIME: ISW increment of the last RK4 step (set by rk4_step)
    static constexpr int cstride = kBlock;
    static constexpr int kFloats = TIME ? 40 : 32;   // LDS words per lane

    // lds: this lane's first slot; lanes of a block are kBlock words apart
    // per coefficient, so the 64 lanes of a wave touch 64 consecutive words
    // for every (f, k) (no bank conflicts) at compile-time offsets
    __device__ __forceinline__ void bind(float* lds) { c = lds; }

    __device__ __forceinline__ void reset()
    {
        keyL = -1;
        lvl = 0;
    }

    // Leaf level at the point with unwrapped coordinates I at level
    // max_level + 1; -1 outside a non-periodic box.  The cached leaf is the
    // one holding the cached half-cell; a walk to another leaf drops the
    // cached stencil, so that leafId always belongs to key.
    __device__ __forceinline__ int leaf(const GridDev& g, const int I[3])
    {
        if (!AMR) {
            if (!g.periodic) {
                const int M = g.n0;
                if ((unsigned)(I[0] >> 1) >= (unsigned)M || (unsigned)(I[1] >> 1) >= (unsigned)M ||
                    (unsigned)(I[2] >> 1) >= (unsigned)M)
                    return -1;
            }
            return 0;
        }
        const int Lm = g.max_level;
        {
            // the cached leaf (comparisons combined without branches; with
            // nothing cached, keyL = -1 and the shift stays below 32)
            const int sh = Lm + 1 - keyL;
            if ((keyL >= 0) & ((I[0] >> sh) == (key[0] >> 1)) & ((I[1] >> sh) == (key[1] >> 1)) &
                ((I[2] >> sh) == (key[2] >> 1)))
                return keyL;
        }
        int J0 = I[0] >> 1, J1 = I[1] >> 1, J2 = I[2] >> 1;   // level max_level
        const int M = g.n0 << Lm;
        if (g.periodic) {
            J0 &= M - 1; J1 &= M - 1; J2 &= M - 1;
        } else if ((unsigned)J0 >= (unsigned)M || (unsigned)J1 >= (unsigned)M || (unsigned)J2 >= (unsigned)M) {
            return -1;
        }
        int id = (int)morton3((uint32_t)(J0 >> Lm), (uint32_t)(J1 >> Lm), (uint32_t)(J2 >> Lm));
        int L = 0;
        for (int m = Lm - 1; m >= 0; --m) {
            const int ch = g.child[id];
            if (ch < 0) break;
            id = ch + (((J0 >> m) & 1) | (((J1 >> m) & 1) << 1) | (((J2 >> m) & 1) << 2));
            ++L;
        }
        leafId = id;
        keyL = -1;
        return L;
    }

    // Resolve (or reuse) the stencil for a point in a leaf cell of level L.
    // Returns false when no complete stencil exists even at level 0.
    __device__ __forceinline__ bool stencil(const GridDev& g, int L, const int I[3])
    {
        const int Lm = AMR ? g.max_level : 0;
        const int sh = Lm - L;                   // I is at level Lm + 1
        const int k0 = I[0] >> sh, k1 = I[1] >> sh, k2 = I[2] >> sh;
        if ((keyL == L) & (k0 == key[0]) & (k1 == key[1]) & (k2 == key[2])) return true;
        int base, l;
        // a point in a leaf of level 0 takes the level-0 stencil (or none at
        // the edge of a non-periodic box), whose base follows from the Morton
        // order without the per-half-cell table
        if (AMR && L > 0) {
            base = g.leafinfo[8 * (int64_t)(leafId - g.level_start[1]) + ((k0 & 1) | ((k1 & 1) << 1) | ((k2 & 1) << 2))];
            if (base < 0) return false;
            l = level_of(g, base);
        } else {
            l = 0;
            int b0 = (k0 - 1) >> 1, b1 = (k1 - 1) >> 1, b2 = (k2 - 1) >> 1;
            const int M = g.n0;
            if (g.periodic) {
                b0 &= M - 1; b1 &= M - 1; b2 &= M - 1;
            } else if ((unsigned)b0 >= (unsigned)(M - 1) || (unsigned)b1 >= (unsigned)(M - 1) ||
                       (unsigned)b2 >= (unsigned)(M - 1)) {
                return false;                     // b + 1 must exist too
            }
            if constexpr (AMR) {
                // the leaf is the coarse cell J = k >> 1, whose id leafId is
                // its Morton index, and b = J - 1 + (k & 1): the base id is
                // leafId with the dilated coordinate of every axis of even k
                // decremented, masked to the grid's bits (which wraps a
                // periodic grid like b & (M - 1))
                const uint32_t bits = (1u << (3 * __builtin_ctz((unsigned)M))) - 1u;
                const int kk[3] = {k0, k1, k2};
                uint32_t m = (uint32_t)leafId;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const uint32_t md = (0x49249249u << d) & bits;
                    const uint32_t dec = (m & ~md) | (((m & md) - (1u << d)) & md);
                    m = (kk[d] & 1) ? m : dec;
                }
                base = (int)m;
            } else {
                base = (int)morton3((uint32_t)b0, (uint32_t)b1, (uint32_t)b2);
            }
        }
        this->base = base;
        const float4* rec = g.dual + 8 * (int64_t)base;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const float4 q = rec[o];
            c[(0 + o) * cstride] = q.x;
            c[(8 + o) * cstride] = q.y;
            c[(16 + o) * cstride] = q.z;
            c[(24 + o) * cstride] = q.w;
        }
        if constexpr (TIME) {
            const float4 t0 = g.tdual[2 * (int64_t)base], t1 = g.tdual[2 * (int64_t)base + 1];
            c[32 * cstride] = t0.x; c[33 * cstride] = t0.y; c[34 * cstride] = t0.z; c[35 * cstride] = t0.w;
            c[36 * cstride] = t1.x; c[37 * cstride] = t1.y; c[38 * cstride] = t1.z; c[39 * cstride] = t1.w;
        }
        lvl = l;
        keyL = L;
        key[0] = k0; key[1] = k1; key[2] = k2;
        return true;
    }

    // Phi and grad Phi at the point with fine-grid coordinates v = x / h_f,
    // h_f = h0 / 2^(max_level + 1) (CIC,
    // Eq. W_CIC, with the level fallback).  Returns 0, or 1 when no complete
    // stencil exists.  leaf_level and stencil_level receive the levels of the
    // deepest cell containing the point and of the stencil used.
    __device__ __forceinline__ int eval(const GridDev& g, const double v[3], float& phi, float G[3],
                                        int& leaf_level, int& stencil_level)
    {
        #pragma clang fp contract(off)
        const int Lm = AMR ? g.max_level : 0;
        int I[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) I[d] = (int)floor(v[d]);
        int L;
        bool bad = false;
        const int shk = Lm - keyL;   // keyL = -1 (nothing cached): Lm + 1, below 32
        if (AMR && ((keyL >= 0) & ((I[0] >> shk) == key[0]) & ((I[1] >> shk) == key[1]) & ((I[2] >> shk) == key[2]))) {
            // same half-cell of the same leaf as the cached stencil
            L = keyL;
        } else if constexpr (!ONE_EXIT) {
            L = leaf(g, I);
            if (L < 0) {
                leaf_level = L;
                return 1;
            }
            if (!stencil(g, L, I)) {
                leaf_level = L;
                return 1;
            }
        } else {
            // a single exit: the cached coefficients are evaluated all the
            // same without a stencil and the values replaced by zeros
            L = leaf(g, I);
            bad = L < 0 || !stencil(g, L, I);
        }
        leaf_level = L;
        stencil_level = lvl;
        // offsets from the stencil base (lowest corner) at level lvl;
        // v 2^(lvl - Lm - 1) is exact
        const int s = Lm - lvl;
        const double sl = ldexp(1.0, -s - 1);
        const float tx = (float)(v[0] * sl - 0.5 - (double)(((I[0] >> s) - 1) >> 1));
        const float ty = (float)(v[1] * sl - 0.5 - (double)(((I[1] >> s) - 1) >> 1));
        const float tz = (float)(v[2] * sl - 0.5 - (double)(((I[2] >> s) - 1) >> 1));
        t[0] = tx; t[1] = ty; t[2] = tz;
        // f = c0 + tx (c1 + ty (c4 + tz c7) + tz c5) + ty (c2 + tz c6) + tz c3
        float f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float* k = c + 8 * q * cstride;
            const float k0 = k[0], k1 = k[cstride], k2 = k[2 * cstride], k3 = k[3 * cstride];
            const float k4 = k[4 * cstride], k5 = k[5 * cstride], k6 = k[6 * cstride], k7 = k[7 * cstride];
            f[q] = trilinear_eval(k0, k1, k2, k3, k4, k5, k6, k7, tx, ty, tz);
        }
        phi = bad ? 0.0f : f[0];
        G[0] = bad ? 0.0f : f[1];
        G[1] = bad ? 0.0f : f[2];
        G[2] = bad ? 0.0f : f[3];
        if constexpr (TIME) {
            const float* k = c + 32 * cstride;
            tv = trilinear_eval(k[0], k[cstride], k[2 * cstride], k[3 * cstride], k[4 * cstride], k[5 * cstride],
                                k[6 * cstride], k[7 * cstride], tx, ty, tz);
            if (bad) tv = 0.0f;
        }
        return bad ? 1 : 0;
    }
};

// Leaf containing the point with unwrapped coordinates I at level
// max_level + 1 (a walk from its coarse cell); its id in id.  Returns its
// level, or -1 outside a non-periodic box.
template <bool AMR>
__device__ __forceinline__ int walk_to_leaf(const GridDev& g, const int I[3], int& id)
{
    const int Lm = AMR ? g.max_level : 0;
    int J0 = I[0] >> 1, J1 = I[1] >> 1, J2 = I[2] >> 1;   // level max_level
    const int M = g.n0 << Lm;
    if (g.periodic) {
        J0 &= M - 1; J1 &= M - 1; J2 &= M - 1;
    } else if ((unsigned)J0 >= (unsigned)M || (unsigned)J1 >= (unsigned)M || (unsigned)J2 >= (unsigned)M) {
        return -1;
    }
    id = (int)morton3((uint32_t)(J0 >> Lm), (uint32_t)(J1 >> Lm), (uint32_t)(J2 >> Lm));
    int L = 0;
    if (AMR) {
        for (int m = Lm - 1; m >= 0; --m) {
            const int ch = g.child[id];
            if (ch < 0) break;
            id = ch + (((J0 >> m) & 1) | (((J1 >> m) & 1) << 1) | (((J2 >> m) & 1) << 2));
            ++L;
        }
    }
    return L;
}

// Field by nearest grid point (Sect. 2.2, W_NGP): the values of the deepest
// cell containing the point.  The lane keeps the last leaf and its values.
template <bool AMR>
struct NgpCache {
    static constexpr bool kTime = false;
    static constexpr int kNoKey = 0x40000000;
    int keyL;           // level of the cached leaf
    int key[3];         // its unwrapped coordinates at that level
    float val[4];       // its (phi, gx, gy, gz)

    __device__ __forceinline__ void bind(float*) {}
    __device__ __forceinline__ void reset()
    {
        keyL = 0;
        key[0] = key[1] = key[2] = kNoKey;
    }

    // Leaf level at the point with fine coordinates I (-1 outside a
    // non-periodic box); loads the leaf's values when it changes.
    __device__ __forceinline__ int leaf(const GridDev& g, const int I[3])
    {
        const int Lm = AMR ? g.max_level : 0;
        const int sh = Lm + 1 - keyL;
        if ((I[0] >> sh) == key[0] && (I[1] >> sh) == key[1] && (I[2] >> sh) == key[2]) return keyL;
        int id;
        const int L = walk_to_leaf<AMR>(g, I, id);
        if (L < 0) return -1;
        const float4 q = g.payload[id];
        val[0] = q.x; val[1] = q.y; val[2] = q.z; val[3] = q.w;
        const int s2 = Lm + 1 - L;
        keyL = L;
        key[0] = I[0] >> s2; key[1] = I[1] >> s2; key[2] = I[2] >> s2;
        return L;
    }

    __device__ __forceinline__ int eval(const GridDev& g, const double v[3], float& phi, float G[3],
                                        int& leaf_level, int& stencil_level)
    {
        int I[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) I[d] = (int)floor(v[d]);
        const int L = leaf(g, I);
        leaf_level = L;
        if (L < 0) return 1;
        stencil_level = L;
        phi = val[0];
        G[0] = val[1]; G[1] = val[2]; G[2] = val[3];
        return 0;
    }
};

// Field by triangular-shaped cloud (Sect. 2.2, W_TSC): the 27 cells around
// the cell containing the point at the leaf level, falling back one level at
// a time while any of them is missing.  The stencil depends only on the leaf
// cell (the cell containing the point at every coarser level is its
// ancestor), so the lane resolves it only when the leaf changes and keeps
// the 27 payloads in registers: a stage then costs its
// weights and 108 multiply-adds, with no memory access.  Per axis, with f
// the position in the centre cell (in [0, 1)), the weights of the cells at
// -1, 0, +1 are (1 - f)^2 / 2, 3/4 - (f - 1/2)^2 and f^2 / 2.
template <bool AMR>
struct TscCache {
    static constexpr bool kTime = false;
    static constexpr int kNoKey = 0x40000000;
    int keyL;           // level of the leaf whose stencil is cached
    int key[3];         // its unwrapped coordinates at that level
    int lvl;            // level of the stencil (-1: not resolved for this leaf)
    int c[3];           // centre cell of the stencil, unwrapped, at level lvl
    float4 p[27];       // payloads of stencil cell q = (x + 1) + 3 (y + 1) + 9 (z + 1)

    __device__ __forceinline__ void bind(float*) {}
    __device__ __forceinline__ void reset()
    {
        keyL = 0;
        key[0] = key[1] = key[2] = kNoKey;
        lvl = -1;
    }

    __device__ __forceinline__ int leaf(const GridDev& g, const int I[3])
    {
        const int Lm = AMR ? g.max_level : 0;
        const int sh = Lm + 1 - keyL;
        if ((I[0] >> sh) == key[0] && (I[1] >> sh) == key[1] && (I[2] >> sh) == key[2]) return keyL;
        int id;
        const int L = walk_to_leaf<AMR>(g, I, id);
        if (L < 0) return -1;
        const int s2 = Lm + 1 - L;
        keyL = L;
        key[0] = I[0] >> s2; key[1] = I[1] >> s2; key[2] = I[2] >> s2;
        lvl = -1;
        return L;
    }

    // Load the payloads of the 27 cells cc + {-1, 0, 1}^3 at level l when
    // all of them exist; false otherwise (nothing is loaded).  Level 0: the
    // Morton id is the OR of one bit spread per axis, so 9 spreads give the
    // 27 ids.  Refined level: the 27 cells have 2 x 2 x 2 parents (two per
    // axis, the parents of cc - 1 and cc + 1); each cell is its parent's
    // first child plus its octant, so 8 walks to level l - 1 replace 27
    // walks to level l.
    __host__ __device__ __forceinline__ bool gather(const GridDev& g, int l, const int cc[3])
    {
        if (!AMR || l == 0) {
            const int M = g.n0;
            uint32_t sp[3][3];
            bool all = true;
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int J = cc[d] + a - 1;
                    all &= g.periodic || (unsigned)J < (unsigned)M;
                    sp[d][a] = part1by2((uint32_t)(J & (M - 1))) << d;
                }
            if (!all) return false;
#pragma unroll
            for (int q = 0; q < 27; ++q) p[q] = g.payload[sp[0][q % 3] | sp[1][(q / 3) % 3] | sp[2][q / 9]];
            return true;
        }
        // per axis: the two parents, which of them holds the middle cell, and
        // the octant bit of the outer cells (cc -+ 1) and of the middle one
        int P[3][2], mid[3], bo[3], bm[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            P[d][0] = (cc[d] - 1) >> 1;
            P[d][1] = (cc[d] + 1) >> 1;
            mid[d] = (cc[d] >> 1) - P[d][0];
            bo[d] = (cc[d] + 1) & 1;
            bm[d] = cc[d] & 1;
        }
        int ch[8];
        bool all = true;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int par = lookup_cell(g, l - 1, P[0][s & 1], P[1][(s >> 1) & 1], P[2][s >> 2]);
            const int k = g.child[par >= 0 ? par : 0];
            ch[s] = par >= 0 ? k : -1;
            all &= ch[s] >= 0;
        }
        if (!all) return false;
        // first child of the parent of every cell, selected along z, y, x
        int t[2][2][3], u[2][3][3];
#pragma unroll
        for (int sx = 0; sx < 2; ++sx)
#pragma unroll
            for (int sy = 0; sy < 2; ++sy) {
                t[sx][sy][0] = ch[sx + 2 * sy];
                t[sx][sy][2] = ch[sx + 2 * sy + 4];
                t[sx][sy][1] = mid[2] ? t[sx][sy][2] : t[sx][sy][0];
            }
#pragma unroll
        for (int sx = 0; sx < 2; ++sx)
#pragma unroll
            for (int z = 0; z < 3; ++z) {
                u[sx][0][z] = t[sx][0][z];
                u[sx][2][z] = t[sx][1][z];
                u[sx][1][z] = mid[1] ? u[sx][2][z] : u[sx][0][z];
            }
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            const int x = q % 3, y = (q / 3) % 3, z = q / 9;
            const int first = x == 0 ? u[0][y][z] : x == 2 ? u[1][y][z] : (mid[0] ? u[1][y][z] : u[0][y][z]);
            const int oct = (x == 1 ? bm[0] : bo[0]) | ((y == 1 ? bm[1] : bo[1]) << 1) | ((z == 1 ? bm[2] : bo[2]) << 2);
            p[q] = g.payload[first + oct];
        }
        return true;
    }

    __device__ __forceinline__ bool resolve(const GridDev& g, int L, const int I[3])
    {
        const int Lm = AMR ? g.max_level : 0;
        for (int l = L; l >= 0; --l) {
            const int s = Lm + 1 - l;
            const int cc[3] = {I[0] >> s, I[1] >> s, I[2] >> s};
            if (gather(g, l, cc)) {
                lvl = l;
                c[0] = cc[0]; c[1] = cc[1]; c[2] = cc[2];
                return true;
            }
        }
        // no stencil (the ray stops): the payloads are cleared so that every
        // path writes them, and the old ones need no registers during the search
#pragma unroll
        for (int q = 0; q < 27; ++q) p[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        return false;
    }

    __device__ __forceinline__ int eval(const GridDev& g, const double v[3], float& phi, float G[3],
                                        int& leaf_level, int& stencil_level)
    {
        const int Lm = AMR ? g.max_level : 0;
        int I[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) I[d] = (int)floor(v[d]);
        const int L = leaf(g, I);
        leaf_level = L;
        if (L < 0) return 1;
        if (lvl < 0 && !resolve(g, L, I)) return 1;
        stencil_level = lvl;
        // position in the centre cell: v 2^(lvl - Lm - 1) - c, exact in FP64
        const double sc = ldexp(1.0, lvl - Lm - 1);
        float w[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float f = (float)(v[d] * sc - (double)c[d]);
            const float h = f - 0.5f;
            w[d][0] = 0.5f * (1.0f - f) * (1.0f - f);
            w[d][1] = 0.75f - h * h;
            w[d][2] = 0.5f * f * f;
        }
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int z = 0; z < 3; ++z)
#pragma unroll
            for (int y = 0; y < 3; ++y) {
                const float wyz = w[1][y] * w[2][z];
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    const float wq = w[0][x] * wyz;
                    const float4 q = p[x + 3 * y + 9 * z];
                    acc[0] = fmaf(wq, q.x, acc[0]);
                    acc[1] = fmaf(wq, q.y, acc[1]);
                    acc[2] = fmaf(wq, q.z, acc[2]);
                    acc[3] = fmaf(wq, q.w, acc[3]);
                }
            }
        phi = acc[0];
        G[0] = acc[1]; G[1] = acc[2]; G[2] = acc[3];
        return 0;
    }
};

// ---------------------------------------------------------------------------
// Geodesic state in the split representation.  With K = -k0 > 0,
// k = K (n + d) and x = x_obs + s n + dx, the null geodesic equations of
// Sect. 2.2 (dPhi/dlambda = grad Phi . k, dPhi/deta = 0) become
//   d eta/dl = -K,  ds/dl = K,  d dx/dl = K d,
//   dK/dl = 2 H K^2 - 2 K^2 (m.G),                          m = n + d, G = grad Phi
//   d(K d)/dl - n dK/dl = K^2 [4 (m.G) m - 2 G + 2 (H - m.G) d]   (=: P)
// RK4 is applied to (eta, K, dx, K d): d at a stage or at the step end is
// (K_n d_n + c dl P)/K.  This is the same RK4 as on (eta, x, k0, k), since
// the map between the two is linear given K, and it keeps only small
// quantities (d ~ deflection, dx ~ transverse displacement) in FP32.  The
// path coordinate s has the same increments as -eta, so s = eta_0 - eta
// exactly and is not carried.
// ---------------------------------------------------------------------------
struct RayGeom {
    double vo[3];       // observer in fine-grid coordinates (x_obs / h_f)
    double n[3];        // initial direction (unit)
};

// Comoving step length in a leaf of level L: h_L / N = ds_level[L], which
// equals ds_level[0] 2^-L exactly (h0 / 2^L / N rounds like h0 / N, and the
// power of two scales exactly); computed so, since indexing the argument
// array by a per-lane level would be a memory load at every step.
__device__ __forceinline__ double step_length(const CastArgs& a, int L)
{
    return a.adaptive ? ldexp(a.ds_level[0], -L) : a.ds_level[0];
}

// Fine-grid coordinates v = x / h_f, h_f = h0 / 2^(max_level + 1), of
// x = x_obs + s n + dx, s = eta0 - eta.  The observer term is the exact
// quotient; the displacement is scaled by 1/h_f (at the observer both agree
// exactly with x / h_f, elsewhere to one rounding).  Scaling by the power of
// two is exact, so v is 2^(max_level + 1) times the coarse-grid coordinates
// computed the same way.
__device__ __forceinline__ void grid_coords(const GridDev& g, const RayGeom& r, double eta, const float dx[3],
                                            double v[3])
{
    #pragma clang fp contract(off)
    const double s = g.eta0 - eta;
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i] = fma(fma(s, r.n[i], (double)dx[i]), g.inv_hf, r.vo[i]);
}

// dPhi/dl in the spatial geodesic equation.  ChainRule: grad Phi . k
// (+ dPhi/deta k0 on a time-dependent grid) at every RK4 stage (Eq. dPhi/dl,
// first form).  StepDifference: the equations written with dPhi/dl only
// (dPhi/deta eliminated, so the time equation takes grad Phi . k) and
// dPhi/dl estimated once per step as the difference of Phi between the last
// two step starts over the affine length between them (Eq. dPhi/dl, second
// form; the first step takes grad Phi . k at the observer).
struct ChainRule {
    static constexpr bool kDiff = false;
};

struct StepDifference {
    static constexpr bool kDiff = true;
    float phi_prev;     // Phi at the previous step start
    double dl_prev;     // affine length of the previous step (0: no step yet)
    float phi0;         // Phi at the start of the step being taken
    float D;            // its dPhi/dl
};

// No-op stage recorder of the forward kernels.  A recorder's stage hook
// sees the stage index, the step-start state y, the stage state yi, the
// field evaluator (its stencil and offsets at the stage), the interpolated
// gradient and the background cubic of the step.
struct NoRecord {
    template <class FC>
    __device__ __forceinline__ void stage(int, const GeoState&, const GeoState&, const FC&, const float*,
                                          const HubbleCubic&, const CosmoDev&)
    {
    }
};

// The field at a step's start point, evaluated by the caller (which needs
// the leaf level there for the step length): with PEEL, stage 0 of the step
// runs before the stage loop and takes it instead of evaluating the same
// point again.  (Peeling lengthens the code; kernels whose registers are
// tight keep the plain loop.)
struct Stage0 {
    float phi, G[3], tv;   // tv: dPhi/deta (time-dependent potential)
    int l;                 // stencil level
    int bad;               // no complete stencil
};

// One RK4 step of affine length dl from y into out (F: the lane's field
// evaluator, any interpolation order).  With a time-dependent potential
// (FC::kTime) the spatial equation takes dPhi/dl = grad Phi . k + T k0 with
// T = dPhi/deta (in the time equation the two T terms cancel: 2 T k0^2 -
// 2 T k0 k0), and the step's ISW increment int T K dl (= int T |d eta|) is
// left in F.isw_step.  The four stencil levels
// are appended to hash only when all four stages succeed (return 0).  When
// record is set, the recorder receives every stage's state and stencil (base
// id, level); the reverse sweep uses it to replay the forward stages exactly.
template <class FC, class Rec, class DP, bool PEEL = false>
__device__ __forceinline__ int rk4_core(const GridDev& g, const CosmoDev& cz, FC& F,
                                        const RayGeom& r, const GeoState& y, double dl, GeoState& out,
                                        uint32_t& hash, Rec& rec, bool record, DP& dp,
                                        const Stage0* s0 = nullptr)
{
    #pragma clang fp contract(off)
    const float nf[3] = {(float)r.n[0], (float)r.n[1], (float)r.n[2]};
    double acc_eta = 0.0, acc_K = 0.0;
    float acc_dx[3] = {0.f, 0.f, 0.f}, acc_P[3] = {0.f, 0.f, 0.f};
    double f_K = 0.0, Kprev = y.K;
    float f_dx[3] = {0.f, 0.f, 0.f}, f_P[3] = {0.f, 0.f, 0.f};
    float acc_I = 0.f;
    uint32_t h = hash;
    HubbleCubic Hc;
    Hc.init(cz, y.eta);
    // one stage; true when no complete stencil exists at its position (the
    // remaining stages then run on meaningless values, every lookup staying
    // in bounds, and the step is rejected after the loop, so that the loop
    // has a single exit)
    auto stage = [&](const int st, const Stage0* z) -> bool {
        #pragma clang fp contract(off)
        GeoState yi;
        if (st == 0) {
            yi = y;
        } else {
            const double c = (st == 3 ? 1.0 : 0.5) * dl;
            yi.eta = fma(-c, Kprev, y.eta);        // f_eta = -K of the previous stage
            yi.K = fma(c, f_K, y.K);
            // d_stage = (K d + c P) / K_stage = d + (K / K_stage - 1) d + (c / K_stage) P:
            // d is carried exactly and only the small corrections are rounded
            const float cf = (float)c;
            const float inv = __builtin_amdgcn_rcpf((float)yi.K);   // 1 ulp
            const float rm1 = (float)(y.K - yi.K) * inv;
            const float cK = cf * inv;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                yi.dx[i] = fmaf(cf, f_dx[i], y.dx[i]);
                yi.d[i] = fmaf(cK, f_P[i], fmaf(rm1, y.d[i], y.d[i]));
            }
        }
        float phi = 0.0f, G[3] = {0.0f, 0.0f, 0.0f};
        int l = 0;
        bool bad;
        if (z) {
            // stage 0 at the step start, evaluated by the caller
            phi = z->phi;
            G[0] = z->G[0]; G[1] = z->G[1]; G[2] = z->G[2];
            l = z->l;
            bad = z->bad != 0;
            if constexpr (FC::kTime) F.tv = z->tv;
        } else {
            double u[3];
            grid_coords(g, r, yi.eta, yi.dx, u);
            int leafl;
            bad = F.eval(g, u, phi, G, leafl, l) != 0;
        }
        h = fnv(h, (uint32_t)l);
        if (record) rec.stage(st, y, yi, F, G, Hc, cz);
        const double H = Hc(cz, yi.eta);
        const float m[3] = {nf[0] + yi.d[0], nf[1] + yi.d[1], nf[2] + yi.d[2]};
        const float mG = fmaf(m[2], G[2], fmaf(m[1], G[1], m[0] * G[0]));
        Kprev = yi.K;
        f_K = yi.K * yi.K * (2.0 * H - 2.0 * (double)mG);
        const float Kf = (float)yi.K;
        const float K2 = Kf * Kf;
        const float hm = 2.0f * ((float)H - mG);
        // dk/dl with k = K m: K^2 (2 H m + 2 (m.G - T) m - 2 G); the P form
        // subtracts n dK/dl, dK/dl = K^2 (2 H - 2 m.G)
        float cm = 4.0f * mG;
        if constexpr (FC::kTime) cm = fmaf(-2.0f, F.tv, cm);
        if constexpr (DP::kDiff) {
            // 2 m.G (from -n dK/dl) + 2 D / K (the spatial equation's dPhi/dl)
            if (st == 0) {
                dp.phi0 = phi;
                dp.D = dp.dl_prev > 0.0 ? (float)(((double)phi - (double)dp.phi_prev) / dp.dl_prev) : Kf * mG;
            }
            cm = fmaf(2.0f, dp.D / Kf, 2.0f * mG);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            f_dx[i] = Kf * yi.d[i];
            f_P[i] = K2 * fmaf(hm, yi.d[i], fmaf(cm, m[i], -2.0f * G[i]));
        }
        const double w = (st == 0 || st == 3) ? 1.0 : 2.0;
        const float wf = (float)w;
        if constexpr (FC::kTime) acc_I = fmaf(wf, F.tv * Kf, acc_I);
        acc_eta = fma(-w, yi.K, acc_eta);
        acc_K = fma(w, f_K, acc_K);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            acc_dx[i] = fmaf(wf, f_dx[i], acc_dx[i]);
            acc_P[i] = fmaf(wf, f_P[i], acc_P[i]);
        }
        return bad;
    };
    bool failed = false;
    if constexpr (PEEL) {
        failed = stage(0, s0);
#pragma unroll 1
        for (int st = 1; st < 4; ++st) failed |= stage(st, nullptr);
    } else {
#pragma unroll 1
        for (int st = 0; st < 4; ++st) failed |= stage(st, nullptr);
    }
    if (failed) return 1;
    const double h6 = dl * (1.0 / 6.0);
    out.eta = fma(h6, acc_eta, y.eta);
    out.K = fma(h6, acc_K, y.K);
    const float h6f = (float)h6;
    const float inv = __builtin_amdgcn_rcpf((float)out.K);
    const float rm1 = (float)(y.K - out.K) * inv;
    const float cK = h6f * inv;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        out.dx[i] = fmaf(h6f, acc_dx[i], y.dx[i]);
        out.d[i] = fmaf(cK, acc_P[i], fmaf(rm1, y.d[i], y.d[i]));
    }
    if constexpr (FC::kTime) F.isw_step = h6f * acc_I;
    hash = h;
    return 0;
}

template <class FC, class Rec, bool PEEL = false>
__device__ __forceinline__ int rk4_step(const GridDev& g, const CosmoDev& cz, FC& F,
                                        const RayGeom& r, const GeoState& y, double dl, GeoState& out,
                                        uint32_t& hash, Rec& rec, bool record, const Stage0* s0 = nullptr)
{
    ChainRule cr;
    return rk4_core<FC, Rec, ChainRule, PEEL>(g, cz, F, r, y, dl, out, hash, rec, record, cr, s0);
}

template <class FC>
__device__ __forceinline__ int rk4_step(const GridDev& g, const CosmoDev& cz, FC& F,
                                        const RayGeom& r, const GeoState& y, double dl, GeoState& out,
                                        uint32_t& hash)
{
    NoRecord none;
    return rk4_step<FC, NoRecord>(g, cz, F, r, y, dl, out, hash, none, false);
}

// The forward step with a choice of dPhi/dl (ChainRule or StepDifference).
template <class FC, class DP, bool PEEL = false>
__device__ __forceinline__ int rk4_step_dp(const GridDev& g, const CosmoDev& cz, FC& F,
                                           const RayGeom& r, const GeoState& y, double dl, GeoState& out,
                                           uint32_t& hash, DP& dp, const Stage0* s0 = nullptr)
{
    NoRecord none;
    return rk4_core<FC, NoRecord, DP, PEEL>(g, cz, F, r, y, dl, out, hash, none, false, dp, s0);
}

// NaN or infinity anywhere in the state (a sum of the small FP32 parts is
// non-finite exactly when one of them is; they cannot overflow together).
__device__ __forceinline__ bool finite_state(const GeoState& y)
{
    const float s = ((y.d[0] + y.d[1]) + (y.d[2] + y.dx[0])) + (y.dx[1] + y.dx[2]);
    return isfinite(y.eta) && isfinite(y.K) && isfinite(s);
}

}  // namespace mpath
