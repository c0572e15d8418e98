// device.h -- device-side building blocks of the ray tracer: HEALPix
// directions, the tabulated conformal Hubble rate, octree lookups with the
// AMR level fallback and a lane-resident stencil cache, and one RK4 step of
// the null geodesic equations in the split FP64/FP32 representation.
#pragma once

#include "internal.h"

namespace mpath {

constexpr uint32_t kFnvOffset = 2166136261u;
constexpr uint32_t kFnvPrime = 16777619u;

__device__ __forceinline__ uint32_t fnv(uint32_t h, uint32_t v) { return (h ^ v) * kFnvPrime; }

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

// Conformal Hubble rate a'/a at eta: cubic Hermite on the uniform table.
__device__ __forceinline__ double conformal_hubble(const CosmoDev& c, double eta)
{
    if (c.is_static) return 0.0;
    const double u = (eta - c.eta_lo) * c.inv_deta;
    int i = (int)floor(u);
    i = i < 0 ? 0 : (i > c.n - 2 ? c.n - 2 : i);
    const double t = u - (double)i;
    const double2 p0 = c.table[i];
    const double2 p1 = c.table[i + 1];
    const double t2 = t * t, t3 = t2 * t;
    const double h00 = 2.0 * t3 - 3.0 * t2 + 1.0;
    const double h10 = t3 - 2.0 * t2 + t;
    const double h01 = 3.0 * t2 - 2.0 * t3;
    const double h11 = t3 - t2;
    return h00 * p0.x + h01 * p1.x + c.deta * (h10 * p0.y + h11 * p1.y);
}

// ---------------------------------------------------------------------------
// Octree lookups.  Integer cell coordinates are kept unwrapped (a periodic
// ray may leave the box) and wrapped only to address memory.
// ---------------------------------------------------------------------------

// Id of cell (l, J) or -1 if it does not exist: coarse ancestor by Morton
// index, then one child link per level.
__device__ __forceinline__ int lookup_cell(const GridDev& g, int l, int J0, int J1, int J2)
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

// Field value interpolated at one point, with the lane's cache of the leaf
// cell and of the last resolved 8-cell stencil (with its payload).
//
// Reuse is exact: the leaf level of x only changes when x leaves the cached
// leaf cell, and for x inside a leaf cell of level L the CIC base at every
// level l <= L is a function of floor(x / h_{L+1}) alone (the half of the
// leaf cell x lies in per axis), so the resolved stencil is a function of
// (L, floor(x / h_{L+1})).
template <bool AMR>
struct FieldCache {
    int leafL;          // level of the cached leaf cell (-1: none)
    int leafI[3];       // its unwrapped coordinates at level leafL
    int keyL;           // leaf level the stencil was resolved for (-1: none)
    int key[3];         // unwrapped coordinates at level keyL + 1
    int lvl;            // level of the resolved stencil
    int b[3];           // its unwrapped base (lowest corner) at level lvl
    float4 v[8];        // payload of the 8 cells, octant o = ox + 2 oy + 4 oz

    __device__ __forceinline__ void reset()
    {
        leafL = -1;
        keyL = -1;
    }

    // Leaf level at the point with unwrapped finest+1 coordinates I (level
    // max_level + 1); -1 outside a non-periodic box.
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
        if (leafL >= 0) {
            const int sh = Lm + 1 - leafL;
            if ((I[0] >> sh) == leafI[0] && (I[1] >> sh) == leafI[1] && (I[2] >> sh) == leafI[2]) return leafL;
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
        leafL = L;
        const int sh = Lm + 1 - L;
        leafI[0] = I[0] >> sh; leafI[1] = I[1] >> sh; leafI[2] = I[2] >> sh;
        return L;
    }

    // Resolve (or reuse) the stencil for a point in a leaf cell of level L.
    // Returns false when no complete stencil exists even at level 0.
    __device__ __forceinline__ bool stencil(const GridDev& g, int L, const int I[3])
    {
        const int Lm = AMR ? g.max_level : 0;
        const int sh = Lm - L;                   // I is at level Lm + 1
        const int k0 = I[0] >> sh, k1 = I[1] >> sh, k2 = I[2] >> sh;
        if (keyL == L && k0 == key[0] && k1 == key[1] && k2 == key[2]) return true;
        for (int l = L; l >= 0; --l) {
            const int s = Lm - l;
            const int b0 = ((I[0] >> s) - 1) >> 1;
            const int b1 = ((I[1] >> s) - 1) >> 1;
            const int b2 = ((I[2] >> s) - 1) >> 1;
            int ids[8];
            bool ok = true;
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                ids[o] = lookup_cell(g, l, b0 + (o & 1), b1 + ((o >> 1) & 1), b2 + (o >> 2));
                ok = ok && ids[o] >= 0;
            }
            if (!ok) continue;
#pragma unroll
            for (int o = 0; o < 8; ++o) v[o] = g.payload[ids[o]];
            lvl = l;
            b[0] = b0; b[1] = b1; b[2] = b2;
            keyL = L;
            key[0] = k0; key[1] = k1; key[2] = k2;
            return true;
        }
        return false;
    }

    // Phi and grad Phi at x (CIC, Eq. W_CIC, with the level fallback).
    // Returns 0, or 1 when no complete stencil exists.  *leaf_level and
    // *stencil_level receive the levels of the deepest cell containing x and
    // of the stencil used.
    __device__ __forceinline__ int eval(const GridDev& g, const double x[3], float& phi, float G[3],
                                        int& leaf_level, int& stencil_level)
    {
        const int Lm = AMR ? g.max_level : 0;
        const double scale = (double)(2 << Lm);      // 2^(Lm+1)
        double u[3];
        int I[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            u[d] = x[d] / g.h0;                      // coarse-grid coordinates
            I[d] = (int)floor(u[d] * scale);
        }
        const int L = leaf(g, I);
        leaf_level = L;
        if (L < 0) return 1;
        if (!stencil(g, L, I)) return 1;
        stencil_level = lvl;
        const double sl = (double)(1 << lvl);
        const float tx = (float)(u[0] * sl - 0.5 - (double)b[0]);
        const float ty = (float)(u[1] * sl - 0.5 - (double)b[1]);
        const float tz = (float)(u[2] * sl - 0.5 - (double)b[2]);
        // trilinear interpolation of the 8 payloads (weights (1-t) or t per axis)
        const float4 c00 = lerp4(v[0], v[1], tx), c10 = lerp4(v[2], v[3], tx);
        const float4 c01 = lerp4(v[4], v[5], tx), c11 = lerp4(v[6], v[7], tx);
        const float4 c0 = lerp4(c00, c10, ty), c1 = lerp4(c01, c11, ty);
        const float4 r = lerp4(c0, c1, tz);
        phi = r.x;
        G[0] = r.y; G[1] = r.z; G[2] = r.w;
        return 0;
    }

    static __device__ __forceinline__ float4 lerp4(const float4 a, const float4 b, float t)
    {
        const float s = 1.0f - t;
        return make_float4(s * a.x + t * b.x, s * a.y + t * b.y, s * a.z + t * b.z, s * a.w + t * b.w);
    }
};

// ---------------------------------------------------------------------------
// Geodesic state in the split representation.  With K = -k0 > 0 and
// k = K (n + d), x = x_obs + s n + dx, the null geodesic equations of
// Sect. 2.2 (dPhi/dlambda = grad Phi . k, dPhi/deta = 0) become
//   d eta/dl = -K,  ds/dl = K,  d dx/dl = K d,
//   dK/dl = 2 H K^2 - 2 K^2 (m.G),                          m = n + d, G = grad Phi
//   d(K d)/dl - n dK/dl = K^2 [4 (m.G) m - 2 G + 2 (H - m.G) d]   (=: P)
// RK4 is applied to (eta, K, s, dx, K d): d at a stage or at the step end is
// (K_n d_n + c dl P)/K.  This is the same RK4 as on (eta, x, k0, k), since
// the map between the two is linear given K, and it keeps only small
// quantities (d ~ deflection, dx ~ transverse displacement) in FP32.
// ---------------------------------------------------------------------------
struct GeoState {
    double eta, K, s;
    float d[3], dx[3];
};

struct RayGeom {
    double o[3];        // observer
    double n[3];        // initial direction (unit)
};

__device__ __forceinline__ void position(const RayGeom& r, double s, const float dx[3], double x[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i) x[i] = r.o[i] + (s * r.n[i] + (double)dx[i]);
}

// One RK4 step of affine length dl from y into out.  The four stencil levels
// are appended to *hash only when all four stages succeed (return 0).
template <bool AMR>
__device__ __forceinline__ int rk4_step(const GridDev& g, const CosmoDev& cz, FieldCache<AMR>& F,
                                        const RayGeom& r, const GeoState& y, double dl, GeoState& out,
                                        uint32_t& hash)
{
    const float nf[3] = {(float)r.n[0], (float)r.n[1], (float)r.n[2]};
    double acc_eta = 0.0, acc_K = 0.0, acc_s = 0.0;
    float acc_dx[3] = {0.f, 0.f, 0.f}, acc_P[3] = {0.f, 0.f, 0.f};
    double f_eta = 0.0, f_K = 0.0, f_s = 0.0;
    float f_dx[3] = {0.f, 0.f, 0.f}, f_P[3] = {0.f, 0.f, 0.f};
    uint32_t h = hash;
#pragma unroll 1
    for (int st = 0; st < 4; ++st) {
        GeoState yi;
        if (st == 0) {
            yi = y;
        } else {
            const double c = (st == 3 ? 1.0 : 0.5) * dl;
            yi.eta = y.eta + c * f_eta;
            yi.K = y.K + c * f_K;
            yi.s = y.s + c * f_s;
            const float cf = (float)c;
            const float ratio = (float)(y.K / yi.K);
            const float cK = (float)(c / yi.K);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                yi.dx[i] = y.dx[i] + cf * f_dx[i];
                yi.d[i] = ratio * y.d[i] + cK * f_P[i];
            }
        }
        double x[3];
        position(r, yi.s, yi.dx, x);
        float phi, G[3];
        int leafl, l;
        if (F.eval(g, x, phi, G, leafl, l)) return 1;
        h = fnv(h, (uint32_t)l);
        const double H = conformal_hubble(cz, yi.eta);
        const float m[3] = {nf[0] + yi.d[0], nf[1] + yi.d[1], nf[2] + yi.d[2]};
        const float mG = m[0] * G[0] + m[1] * G[1] + m[2] * G[2];
        f_eta = -yi.K;
        f_K = yi.K * yi.K * (2.0 * H - 2.0 * (double)mG);
        f_s = yi.K;
        const float Kf = (float)yi.K;
        const float K2 = Kf * Kf;
        const float hm = 2.0f * ((float)H - mG);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            f_dx[i] = Kf * yi.d[i];
            f_P[i] = K2 * (4.0f * mG * m[i] - 2.0f * G[i] + hm * yi.d[i]);
        }
        const double w = (st == 0 || st == 3) ? 1.0 : 2.0;
        const float wf = (float)w;
        acc_eta += w * f_eta;
        acc_K += w * f_K;
        acc_s += w * f_s;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            acc_dx[i] += wf * f_dx[i];
            acc_P[i] += wf * f_P[i];
        }
    }
    const double h6 = dl / 6.0;
    out.eta = y.eta + h6 * acc_eta;
    out.K = y.K + h6 * acc_K;
    out.s = y.s + h6 * acc_s;
    const float h6f = (float)h6;
    const float ratio = (float)(y.K / out.K);
    const float cK = (float)(h6 / out.K);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        out.dx[i] = y.dx[i] + h6f * acc_dx[i];
        out.d[i] = ratio * y.d[i] + cK * acc_P[i];
    }
    hash = h;
    return 0;
}

__device__ __forceinline__ bool finite_state(const GeoState& y)
{
    bool ok = isfinite(y.eta) && isfinite(y.K) && isfinite(y.s);
#pragma unroll
    for (int i = 0; i < 3; ++i) ok = ok && isfinite(y.d[i]) && isfinite(y.dx[i]);
    return ok;
}

}  // namespace mpath
