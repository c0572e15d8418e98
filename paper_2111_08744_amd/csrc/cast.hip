// cast.hip -- forward ray-casting kernels for gfx950.
//
// One lane integrates one photon (Sect. 2.2: photons are independent).  Two
// schedules share the per-ray code:
//   static      one launch with one lane per ray; rays of a wave are
//               neighbouring NESTED pixels of one observer, so their
//               stencil gathers hit the same cache lines near the observer;
//   persistent  a grid sized to the resident capacity of the GPU; every lane
//               that finishes its ray takes the next one from a global
//               queue (one atomic per wave per refill, ballot-aggregated), so
//               rays of uneven length (many observers, many source
//               redshifts, AMR) do not leave lanes idle.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"

namespace mpath {
namespace {

constexpr int kWave = 64;
// Occupancy target of the integration kernels: 4 waves per SIMD (128
// registers).  A wave stalls on every stage where one of its lanes enters a
// new stencil (a dependent stencil-table and coefficient gather), so latency
// hiding pays more than the few values the bound spills (measured on the AMR
// workload: 3 waves 102.6 ms, 4 waves 89.5 ms per cast).
constexpr int kMinWavesPerSimd = 4;

// Step-start hook of RayRun::advance that does nothing (plain casts).
struct NoSample {
    __device__ __forceinline__ void at_step(const CastArgs&, const RayGeom&, const GeoState&, int) {}
    template <class Run>
    __device__ __forceinline__ bool at_surface(const CastArgs&, Run&) { return false; }
};

// Everything one lane carries for its current ray (DP: the form of dPhi/dl).
template <bool AMR, class FC = FieldCache<AMR>, class DP = ChainRule>
struct RayRun {
    int64_t ray;          // -1: no ray
    RayGeom geo;
    double eta_s;
    float phi_o;
    GeoState y;
    int32_t n_steps;
    uint32_t hash;
    int status;           // -1 while running
    double isw;           // int dPhi/deta |d eta| so far (time-dependent potential; else 0)
    double lam;           // affine parameter (iso-lambda stops)
    double p_cur, dp_cur; // stop parameter and its lambda-derivative at y (iso-chi, iso-z stops)
    DP dp;
    FC F;

    template <bool CKPT = false>
    __device__ __forceinline__ bool advance(const CastArgs& a, int max_iter)
    {
        NoSample none;
        return advance<CKPT, NoSample>(a, max_iter, none);
    }

    __device__ __forceinline__ void start(const CastArgs& a, int64_t r)
    {
        ray = r;
        // observer owning the ray (observers are few; linear scan from the end)
        int j = a.n_obs - 1;
        while (j > 0 && a.obs[j].ray_first > r) --j;
        const ObsDev& ob = a.obs[j];
#pragma unroll
        for (int i = 0; i < 3; ++i) geo.vo[i] = ldexp(ob.x[i] / a.grid.h0, a.grid.max_level + 1);
        geo.n[0] = a.dirs[3 * r];
        geo.n[1] = a.dirs[3 * r + 1];
        geo.n[2] = a.dirs[3 * r + 2];
        eta_s = a.ray_stop ? a.ray_stop[r].x : ob.eta_s;
        F.reset();
        n_steps = 0;
        hash = kFnvOffset;
        status = -1;
        isw = 0.0;
        if constexpr (DP::kDiff) dp.dl_prev = 0.0;
        float G[3];
        int leafl, l;
        if (F.eval(a.grid, geo.vo, phi_o, G, leafl, l)) {
            status = MPATH_RAY_LEFT_DOMAIN;
            phi_o = __builtin_nanf("");
        }
        // k0 = -1 (backward in time); |k| from the null condition
        const double po = (double)phi_o;
        const double kmag = sqrt((1.0 + 2.0 * po) / (1.0 - 2.0 * po));
        y.eta = a.cosmo_eta0;
        y.K = 1.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            y.d[i] = (float)(geo.n[i] * (kmag - 1.0));
            y.dx[i] = 0.0f;
        }
    }

    // Advance by at most max_iter steps; returns true when the ray is done.
    // With CKPT the state before every K-th step is stored for the adjoint.
    // smp.at_step(y, L) sees the state at every step start (after the leaf
    // level L there is known, before the step is taken).
    template <bool CKPT = false, class Smp = NoSample>
    __device__ __forceinline__ bool advance(const CastArgs& a, int max_iter, Smp& smp)
    {
        if (status >= 0) return true;
        const GridDev& g = a.grid;
        // plain casts peel stage 0 (the step start's field evaluation serves
        // it); the sampling casts keep the shorter code of the plain loop
        constexpr bool kPeel = std::is_same<Smp, NoSample>::value;
        int it = 0;
        for (;;) {
            // the field at the step start (stage 0 of the step, and of every
            // landing pass, which all start there)
            Stage0 s0;
            // regular steps up to the one that would cross the stop surface
            for (;; ++it) {
                if (it >= max_iter) return false;
                if (n_steps >= a.max_steps) { status = MPATH_RAY_MAX_STEPS; return true; }
                if (CKPT && n_steps % a.ckpt_every == 0)
                    a.ckpt[(n_steps / a.ckpt_every) * a.n_rays + ray] = y;
                // leaf level at the step start sets the step length (N steps
                // per cell); the same evaluation gives stage 0's field
                double v[3];
                grid_coords(g, geo, y.eta, y.dx, v);
                int L;
                if constexpr (kPeel) {
                    s0.phi = s0.G[0] = s0.G[1] = s0.G[2] = 0.0f;
                    s0.l = 0;
                    s0.bad = F.eval(g, v, s0.phi, s0.G, L, s0.l);
                    if constexpr (FC::kTime) s0.tv = F.tv;
                } else {
                    int I[3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) I[d] = (int)floor(v[d]);
                    L = F.leaf(g, I);
                }
                if (L < 0) { status = MPATH_RAY_LEFT_DOMAIN; return true; }
                hash = fnv(hash, (uint32_t)L);
                smp.at_step(a, geo, y, L);
                const double dl = step_length(a, L) / y.K;
                if (fma(-y.K, dl, y.eta) < eta_s) break;
                GeoState yn;
                if (rk4_step_dp<FC, DP, kPeel>(g, a.cosmo, F, geo, y, dl, yn, hash, dp, &s0)) {
                    status = MPATH_RAY_LEFT_DOMAIN;
                    return true;
                }
                if constexpr (FC::kTime) isw += (double)F.isw_step;
                if (!finite_state(yn)) { status = MPATH_RAY_NONFINITE; return true; }
                y = yn;
                ++n_steps;
                if constexpr (DP::kDiff) {
                    dp.phi_prev = dp.phi0;
                    dp.dl_prev = dl;
                }
            }
            ++it;
            // landing on the iso-eta surface: Newton on eta_RK4(dl) = eta_s
            // with derivative -K at the trial end, two iterations, then the step
            double dlx = (y.eta - eta_s) / y.K;
            GeoState yn;
            for (int k = 0; k < 3; ++k) {
                if (rk4_step_dp<FC, DP, kPeel>(g, a.cosmo, F, geo, y, dlx, yn, hash, dp, &s0)) {
                    status = MPATH_RAY_LEFT_DOMAIN;
                    return true;
                }
                if (k < 2) dlx = dlx + (yn.eta - eta_s) / yn.K;
            }
            const bool fin = finite_state(yn);
            if constexpr (FC::kTime) isw += (double)F.isw_step;
            y = yn;
            ++n_steps;
            if constexpr (!std::is_same<Smp, NoSample>::value)
                if (fin && smp.at_surface(a, *this)) continue;   // on to the next stop surface
            status = fin ? MPATH_RAY_REACHED : MPATH_RAY_NONFINITE;
            return true;
        }
    }

    // Stop parameter of state s and its lambda-derivative (iso-chi: the
    // comoving distance r from the observer, d/dl = K r.m / r; iso-z:
    // ln(1 + z5) with z5 of the end-point formula at s, d/dl =
    // K (a'/a - m.G), the first-order rate of a K (1 + Phi)).  Returns false
    // when the field has no stencil there.
    template <int SURF>
    __device__ __forceinline__ bool stop_param(const CastArgs& a, const GeoState& s, double& p, double& dp)
    {
        const double sp = a.grid.eta0 - s.eta;
        double r[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) r[i] = fma(sp, geo.n[i], (double)s.dx[i]);
        if constexpr (SURF == MPATH_SURFACE_CHI) {
            const double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            double rm = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) rm += r[i] * (geo.n[i] + (double)s.d[i]);
            p = rr;
            dp = s.K * rm / rr;
            return true;
        } else {
            double v[3];
            grid_coords(a.grid, geo, s.eta, s.dx, v);
            float phi, G[3];
            int leafl, l;
            if (F.eval(a.grid, v, phi, G, leafl, l)) return false;
            const double sa = scale_factor(a.cosmo, s.eta);
            p = log(sa * s.K * (1.0 + (double)phi) / (1.0 + (double)phi_o));
            HubbleCubic Hc;
            Hc.init(a.cosmo, s.eta);
            double mG = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) mG += (geo.n[i] + (double)s.d[i]) * (double)G[i];
            dp = s.K * (Hc(a.cosmo, s.eta) - mG);
            return true;
        }
    }

    // The integration to an iso-chi, iso-lambda or iso-z surface (SURF): the
    // regular steps of advance; the step that reaches the surface is taken
    // again from its start with the length from two Newton iterations on
    // p(RK4(dl)) - p_s (iso-lambda: the remaining length exactly).
    template <int SURF>
    __device__ __forceinline__ void advance_stop(const CastArgs& a, double p_s)
    {
        if (status >= 0) return;
        const GridDev& g = a.grid;
        lam = 0.0;
        if constexpr (SURF == MPATH_SURFACE_CHI) {
            // at the observer: chi = 0, rising at |k| = K |n + d|
            p_cur = 0.0;
            dp_cur = 1.0 + (geo.n[0] * y.d[0] + geo.n[1] * y.d[1] + geo.n[2] * y.d[2]);
        }
        for (;;) {
            if (n_steps >= a.max_steps) { status = MPATH_RAY_MAX_STEPS; return; }
            double v[3];
            grid_coords(g, geo, y.eta, y.dx, v);
            int I[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) I[d] = (int)floor(v[d]);
            const int L = F.leaf(g, I);
            if (L < 0) { status = MPATH_RAY_LEFT_DOMAIN; return; }
            hash = fnv(hash, (uint32_t)L);
            const double dl = step_length(a, L) / y.K;
            GeoState yn;
            if constexpr (SURF == MPATH_SURFACE_LAMBDA) {
                if (lam + dl >= p_s) {
                    const double dlx = p_s - lam;
                    if (rk4_step<FC>(g, a.cosmo, F, geo, y, dlx, yn, hash)) { status = MPATH_RAY_LEFT_DOMAIN; return; }
                    y = yn;
                    lam += dlx;
                    ++n_steps;
                    status = finite_state(y) ? MPATH_RAY_REACHED : MPATH_RAY_NONFINITE;
                    return;
                }
            }
            if (rk4_step<FC>(g, a.cosmo, F, geo, y, dl, yn, hash)) { status = MPATH_RAY_LEFT_DOMAIN; return; }
            if (!finite_state(yn)) { status = MPATH_RAY_NONFINITE; return; }
            if constexpr (SURF != MPATH_SURFACE_LAMBDA) {
                bool check = true;
                if constexpr (SURF == MPATH_SURFACE_Z) {
                    // interpolation weights are convex, so Phi <= phi_max anywhere (up
                    // to float32 rounding) and 1 + z5 <= a K (1 + phi_max) / (1 + Phi_o):
                    // below 1 + z_s (with a relative margin of 1e-9) the surface is not
                    // reached and the field need not be evaluated
                    const double bound = scale_factor(a.cosmo, yn.eta) * yn.K * (1.0 + (double)g.phi_max) /
                                         (1.0 + (double)phi_o);
                    check = bound >= exp(p_s) * (1.0 - 1e-9);
                }
                double pn = 0.0, dpn = 0.0;
                if (check && !stop_param<SURF>(a, yn, pn, dpn)) { status = MPATH_RAY_LEFT_DOMAIN; return; }
                if (check && pn >= p_s) {
                    if constexpr (SURF == MPATH_SURFACE_Z) {
                        // the parameter and its rate at the step start (the previous
                        // step's end), skipped while far from the surface
                        if (!stop_param<SURF>(a, y, p_cur, dp_cur)) { status = MPATH_RAY_LEFT_DOMAIN; return; }
                    }
                    // two Newton passes, then the step
                    double dlx = (p_s - p_cur) / dp_cur;
#pragma unroll 1
                    for (int it = 0; it < 3; ++it) {
                        if (rk4_step<FC>(g, a.cosmo, F, geo, y, dlx, yn, hash)) { status = MPATH_RAY_LEFT_DOMAIN; return; }
                        if (it < 2) {
                            double pt, dpt;
                            if (!stop_param<SURF>(a, yn, pt, dpt)) { status = MPATH_RAY_LEFT_DOMAIN; return; }
                            dlx = dlx - (pt - p_s) / dpt;
                        }
                    }
                    y = yn;
                    lam += dlx;
                    ++n_steps;
                    status = finite_state(y) ? MPATH_RAY_REACHED : MPATH_RAY_NONFINITE;
                    return;
                }
                if constexpr (SURF == MPATH_SURFACE_CHI) {
                    p_cur = pn;
                    dp_cur = dpn;
                }
            }
            y = yn;
            lam += dl;
            ++n_steps;
        }
    }

    // Outputs at the end of advance_stop: the end point's own scale factor.
    // advance() for a plain cast (iso-eta stop, chain rule, static
    // potential) with a stage recorder T that also sees every step's start
    // and end: T.begin_step(y, dl, regular) before the RK4 pass it records
    // (every regular step; of the landing only the final pass) and
    // T.end_step(y, yn) after it.  The steps, their decisions and the
    // primal arithmetic are those of advance(), bit for bit.
    template <class Tan>
    __device__ __forceinline__ void advance_recorded(const CastArgs& a, Tan& T)
    {
        if (status >= 0) return;
        const GridDev& g = a.grid;
        ChainRule cr;
        for (;;) {
            if (n_steps >= a.max_steps) { status = MPATH_RAY_MAX_STEPS; return; }
            double v[3];
            grid_coords(g, geo, y.eta, y.dx, v);
            int I[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) I[d] = (int)floor(v[d]);
            const int L = F.leaf(g, I);
            if (L < 0) { status = MPATH_RAY_LEFT_DOMAIN; return; }
            hash = fnv(hash, (uint32_t)L);
            const double dl = step_length(a, L) / y.K;
            if (fma(-y.K, dl, y.eta) < eta_s) break;
            GeoState yn;
            T.begin_step(y, dl, true);
            if (rk4_core<FC, Tan, ChainRule, true>(g, a.cosmo, F, geo, y, dl, yn, hash, T, true, cr)) {
                status = MPATH_RAY_LEFT_DOMAIN;
                return;
            }
            if (!finite_state(yn)) { status = MPATH_RAY_NONFINITE; return; }
            T.end_step(y, yn);
            y = yn;
            ++n_steps;
        }
        // landing on the iso-eta surface (as advance())
        double dlx = (y.eta - eta_s) / y.K;
        GeoState yn;
        for (int k = 0; k < 3; ++k) {
            if (k == 2) T.begin_step(y, dlx, false);
            if (rk4_core<FC, Tan, ChainRule, true>(g, a.cosmo, F, geo, y, dlx, yn, hash, T, k == 2, cr)) {
                status = MPATH_RAY_LEFT_DOMAIN;
                return;
            }
            if (k < 2) dlx = dlx + (yn.eta - eta_s) / yn.K;
        }
        const bool fin = finite_state(yn);
        T.end_step(y, yn);
        y = yn;
        ++n_steps;
        status = fin ? MPATH_RAY_REACHED : MPATH_RAY_NONFINITE;
    }

    __device__ __forceinline__ void finish_stop(const CastArgs& a)
    {
        int j = a.n_obs - 1;
        while (j > 0 && a.obs[j].ray_first > ray) --j;
        const double ae = scale_factor(a.cosmo, y.eta);
        write_outputs(a, ray, j, ae, 1.0 / ae - 1.0, status);
    }

    // Redshift observables (Sect. 2.5) and the end state; the angular
    // observables follow in observables_kernel, which keeps the FP64
    // transcendental functions out of the integration kernel's registers.
    __device__ __forceinline__ void finish(const CastArgs& a)
    {
        int j = a.n_obs - 1;
        while (j > 0 && a.obs[j].ray_first > ray) --j;
        const ObsDev& ob = a.obs[j];
        const double a_s = a.ray_stop ? a.ray_stop[ray].y : ob.a_s;
        write_outputs(a, ray, j, a_s, a.ray_stop ? 1.0 / a_s - 1.0 : ob.z0, status);
    }

    // Outputs of the current state at output slot `slot` (observer j, stop
    // surface with scale factor a_s and FLRW redshift z0) with ray status st
    // (MPATH_RAY_REACHED: the ray is on that surface).
    __device__ __forceinline__ void write_outputs(const CastArgs& a, int64_t slot, int j, double a_s, double z0,
                                                  int st)
    {
        const bool ok = st == MPATH_RAY_REACHED;
        double v[3];
        grid_coords(a.grid, geo, y.eta, y.dx, v);
        float phi_s = __builtin_nanf(""), G[3];
        int leafl, l;
        if (F.eval(a.grid, v, phi_s, G, leafl, l)) phi_s = __builtin_nanf("");
        const OutDev& o = a.out;
        if (o.z5)
            o.z5[slot] = ok ? a_s * y.K * (1.0 + (double)phi_s) / (1.0 + (double)phi_o) - 1.0 : __builtin_nan("");
        if (o.z0) o.z0[slot] = ok ? z0 : __builtin_nan("");
        const double z1 = z0 + (1.0 + z0) * ((double)phi_o - (double)phi_s);
        if (o.z1) o.z1[slot] = ok ? z1 : __builtin_nan("");
        // z4 = z1 - 2 (a0 / a_s) int_{eta_s}^{eta_0} dPhi/deta d eta (Sect. 2.5, v = 0)
        if (o.z4) o.z4[slot] = ok ? z1 - 2.0 * (1.0 + z0) * isw : __builtin_nan("");
        if (o.isw) o.isw[slot] = ok ? isw : __builtin_nan("");
        if (o.phi_src) o.phi_src[slot] = phi_s;
        if (o.n_steps) o.n_steps[slot] = (int32_t)n_steps;
        if (o.status) o.status[slot] = st;
        if (o.hash) o.hash[slot] = hash;
        RayEnd e;
        e.eta = y.eta;
        e.dx[0] = y.dx[0]; e.dx[1] = y.dx[1]; e.dx[2] = y.dx[2];
        e.obs = j;
        a.ends[slot] = e;
    }
};

// Initial directions: HEALPix NESTED pixel centres (Sect. 2.4), computed once
// per cast so that the integration kernel does not carry the FP64 sincos.
__global__ __launch_bounds__(256) void ray_dirs_kernel(CastArgs a)
{
    const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ray >= a.n_rays) return;
    int j = a.n_obs - 1;
    while (j > 0 && a.obs[j].ray_first > ray) --j;
    const ObsDev& ob = a.obs[j];
    double n[3];
    healpix_nest_dir(a.nside, ob.pix_first + (ray - ob.ray_first), n);
    a.dirs[3 * ray] = n[0];
    a.dirs[3 * ray + 1] = n[1];
    a.dirs[3 * ray + 2] = n[2];
}

// Lens equation (Sect. 2.3): beta from the end point r = x_s - x_obs, and the
// deflection alpha = theta - beta as the tangent vector at theta pointing
// away from beta with the great-circle angle as length, on e1 = e_phi,
// e2 = -e_theta.
__global__ __launch_bounds__(256) void observables_kernel(CastArgs a)
{
    const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ray >= a.n_rays) return;
    const RayEnd e = a.ends[ray];
    const double n[3] = {a.dirs[3 * ray], a.dirs[3 * ray + 1], a.dirs[3 * ray + 2]};
    const double s = a.cosmo_eta0 - e.eta;
    double r[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) r[i] = s * n[i] + (double)e.dx[i];
    const double chi = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const OutDev& o = a.out;
    if (o.chi) o.chi[ray] = chi;
    if (o.beta) {
        o.beta[2 * ray] = atan2(hypot(r[0], r[1]), r[2]);
        o.beta[2 * ray + 1] = atan2(r[1], r[0]);
    }
    if (o.alpha) {
        const double rh[3] = {r[0] / chi, r[1] / chi, r[2] / chi};
        const double c = rh[0] * n[0] + rh[1] * n[1] + rh[2] * n[2];
        double t[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) t[i] = rh[i] - c * n[i];
        const double st2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
        double fac = 0.0;
        if (st2 > 0.0) {
            const double st = sqrt(st2);
            fac = -atan2(st, c) / st;
        }
        const double ph = atan2(n[1], n[0]);
        const double th = atan2(hypot(n[0], n[1]), n[2]);
        double sp, cp, stt, ctt;
        sincos(ph, &sp, &cp);
        sincos(th, &stt, &ctt);
        const double e1[3] = {-sp, cp, 0.0};
        const double e2[3] = {-cp * ctt, -sp * ctt, stt};
        o.alpha[2 * ray] = (float)(fac * (t[0] * e1[0] + t[1] * e1[1] + t[2] * e1[2]));
        o.alpha[2 * ray + 1] = (float)(fac * (t[0] * e2[0] + t[1] * e2[1] + t[2] * e2[2]));
    }
}

// TIME: the grid carries dPhi/deta (time-dependent potential).
template <bool AMR, bool TIME>
__global__ __launch_bounds__(kBlock, kMinWavesPerSimd) void cast_static_kernel(CastArgs a)
{
    extern __shared__ float coef_lds[];
    const int64_t r = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_rays) return;
    RayRun<AMR, FieldCache<AMR, TIME>> R;
    R.F.bind(coef_lds + threadIdx.x);
    R.start(a, r);
    R.advance(a, 0x7fffffff);
    R.finish(a);
}

// Static schedule storing checkpoints for the adjoint.
template <bool AMR>
__global__ __launch_bounds__(kBlock, kMinWavesPerSimd) void cast_ckpt_kernel(CastArgs a)
{
    extern __shared__ float coef_lds[];
    const int64_t r = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_rays) return;
    RayRun<AMR> R;
    R.F.bind(coef_lds + threadIdx.x);
    R.start(a, r);
    R.template advance<true>(a, 0x7fffffff);
    R.finish(a);
}

template <bool AMR, bool TIME>
__global__ __launch_bounds__(kBlock, kMinWavesPerSimd) void cast_persistent_kernel(CastArgs a)
{
    extern __shared__ float coef_lds[];
    const int lane = threadIdx.x & (kWave - 1);
    RayRun<AMR, FieldCache<AMR, TIME>> R;
    R.F.bind(coef_lds + threadIdx.x);
    R.ray = -1;
    bool exhausted = false;
    for (;;) {
        // refill every lane without a ray (one atomic per wave)
        const bool need = R.ray < 0 && !exhausted;
        const unsigned long long want = __ballot(need);
        if (want) {
            const int cnt = __popcll(want);
            const int leader = __ffsll((long long)want) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)cnt);
            base = __shfl(base, leader);
            if (base + (unsigned long long)cnt >= (unsigned long long)a.n_rays) exhausted = true;
            if (need) {
                const unsigned long long mine = base + __popcll(want & ((1ull << lane) - 1ull));
                if (mine < (unsigned long long)a.n_rays) R.start(a, (int64_t)mine);
            }
        }
        if (!__ballot(R.ray >= 0)) break;          // queue drained and every lane idle
        if (R.ray >= 0 && R.advance(a, a.batch)) {
            R.finish(a);
            R.ray = -1;
        }
    }
}

// Infinitesimal-beam distortion matrix (Sect. 2.3.1): along the path,
//   A_ab = delta_ab - 2 int_0^chi_s (chi_s - chi) chi / chi_s T_ab dchi,
// T_ab = e_a . H e_b with H the Hessian of Phi from centred differences of
// the interpolated gradient, H_ij = (G_j(x + h e_i) - G_j(x - h e_i)) / 2h
// (mixed derivatives symmetrised), h the size of the leaf cell holding x,
// and (e_1, e_2) = (e_phi, -e_theta) at the direction of x - x_obs.  The
// integrand is sampled at every step start and at the end point and
// integrated by the trapezoid rule in chi; with w = chi - chi^2 / chi_s the
// two sums int chi T and int chi^2 T are carried so that chi_s is needed only
// at the end.  The field at the probe points comes from a second stencil
// cache so that the integration's own cache is left in place.
template <bool AMR>
struct InfBeam {
    FieldCache<AMR, false, false> P;
    double chi_p, Tp[3];         // previous sample (T11, T12, T22)
    double J1[3], J2[3];         // trapezoid sums of chi T and chi^2 T
    int n;

    __device__ __forceinline__ void init(float* lds)
    {
        P.bind(lds);
        P.reset();
        n = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) J1[k] = J2[k] = 0.0;
    }

    __device__ __forceinline__ void at_step(const CastArgs& a, const RayGeom& geo, const GeoState& y, int L)
    {
        const GridDev& g = a.grid;
        double v[3];
        grid_coords(g, geo, y.eta, y.dx, v);
        const double s = g.eta0 - y.eta;
        double r[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) r[i] = s * geo.n[i] + (double)y.dx[i];
        const double chi = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        const double* dir = chi > 0.0 ? r : geo.n;
        const double rho = hypot(dir[0], dir[1]);
        const double rr = sqrt(rho * rho + dir[2] * dir[2]);
        const double cp = rho > 0.0 ? dir[0] / rho : 1.0, sp = rho > 0.0 ? dir[1] / rho : 0.0;
        const double ct = dir[2] / rr, st = rho / rr;
        const double e[2][3] = {{-sp, cp, 0.0}, {-cp * ct, -sp * ct, st}};
        // h = h0 / 2^L; in fine-grid units 2^(max_level + 1 - L), exact
        const double h = ldexp(g.h0, -L);
        const double hf = ldexp(1.0, g.max_level + 1 - L);
        double H[3][3];
#pragma unroll 1
        for (int i = 0; i < 3; ++i) {
            double vp[3] = {v[0], v[1], v[2]}, vm[3] = {v[0], v[1], v[2]};
            vp[i] += hf;
            vm[i] -= hf;
            float php, phm, gp[3], gm[3];
            int l0, l1;
            const bool bad = P.eval(g, vp, php, gp, l0, l1) != 0 || P.eval(g, vm, phm, gm, l0, l1) != 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) H[i][j] = bad ? 0.0 : ((double)gp[j] - (double)gm[j]) / (2.0 * h);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i + 1; j < 3; ++j) {
                const double m = 0.5 * (H[i][j] + H[j][i]);
                H[i][j] = H[j][i] = m;
            }
        double T[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int a0 = k == 2 ? 1 : 0, b0 = k == 0 ? 0 : 1;
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) acc += e[a0][i] * H[i][j] * e[b0][j];
            T[k] = acc;
        }
        if (n > 0) {
            const double dc = 0.5 * (chi - chi_p);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                J1[k] += dc * (chi_p * Tp[k] + chi * T[k]);
                J2[k] += dc * (chi_p * chi_p * Tp[k] + chi * chi * T[k]);
            }
        }
        chi_p = chi;
#pragma unroll
        for (int k = 0; k < 3; ++k) Tp[k] = T[k];
        ++n;
    }

    template <class Run>
    __device__ __forceinline__ bool at_surface(const CastArgs&, Run&) { return false; }

    // A at the end of a ray that reached the source (after the end-point
    // sample); NaN otherwise or without two samples.
    __device__ __forceinline__ void write(float* A, bool reached) const
    {
        if (!reached || n < 2) {
            A[0] = A[1] = A[2] = A[3] = __builtin_nanf("");
            return;
        }
        const double cs = chi_p;
        const double I11 = J1[0] - J2[0] / cs, I12 = J1[1] - J2[1] / cs, I22 = J1[2] - J2[2] / cs;
        A[0] = (float)(1.0 - 2.0 * I11);
        A[1] = (float)(-2.0 * I12);
        A[2] = (float)(-2.0 * I12);
        A[3] = (float)(1.0 - 2.0 * I22);
    }
};

// One lane per ray: the static cast with the infinitesimal-beam samples
// (two stencil caches in LDS, so fewer resident waves than the plain cast).
template <bool AMR>
__global__ __launch_bounds__(kBlock, 2) void cast_infbeam_kernel(CastArgs a, float* A)
{
    extern __shared__ float coef_lds[];
    const int64_t r = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_rays) return;
    RayRun<AMR> R;
    R.F.bind(coef_lds + threadIdx.x);
    InfBeam<AMR> B;
    B.init(coef_lds + 32 * kBlock + threadIdx.x);
    R.start(a, r);
    R.template advance<false, InfBeam<AMR>>(a, 0x7fffffff, B);
    const bool reached = R.status == MPATH_RAY_REACHED;
    if (reached) {
        // end-point sample: leaf level of the end point
        double v[3];
        grid_coords(a.grid, R.geo, R.y.eta, R.y.dx, v);
        float ph, G[3];
        int L, l;
        B.P.eval(a.grid, v, ph, G, L, l);       // sets L (-1 outside a non-periodic box)
        B.at_step(a, R.geo, R.y, L < 0 ? 0 : L);
    }
    B.write(A + 4 * r, reached);
    R.finish(a);
}

// One lane per ray with dPhi/dl from the difference of Phi between step
// starts (the second form of the geodesic equations).
template <bool AMR>
__global__ __launch_bounds__(kBlock, kMinWavesPerSimd) void cast_diff_kernel(CastArgs a)
{
    extern __shared__ float coef_lds[];
    const int64_t r = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_rays) return;
    RayRun<AMR, FieldCache<AMR>, StepDifference> R;
    R.F.bind(coef_lds + threadIdx.x);
    R.start(a, r);
    R.advance(a, 0x7fffffff);
    R.finish(a);
}

// One lane per ray to an iso-chi, iso-lambda or iso-z surface (SURF).
template <bool AMR, int SURF>
__global__ __launch_bounds__(kBlock, kMinWavesPerSimd) void cast_stop_kernel(CastArgs a)
{
    extern __shared__ float coef_lds[];
    const int64_t r = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_rays) return;
    RayRun<AMR> R;
    R.F.bind(coef_lds + threadIdx.x);
    R.start(a, r);
    int j = a.n_obs - 1;
    while (j > 0 && a.obs[j].ray_first > r) --j;
    R.template advance_stop<SURF>(a, a.obs[j].p_s);
    R.finish_stop(a);
}

// Intermediate stop surfaces of a cast (the paper's maps at several source
// redshifts from one run): landing on surface k < n_extra writes the ray's
// observables there to output block k and sends the ray on to surface k + 1;
// the observer's own stop is the last surface (block n_extra).
struct Surfaces {
    const double2* surf;    // [n_obs][n_extra] (eta_s, a_s), nearest first
    int n_extra;
    int k;

    __device__ __forceinline__ void at_step(const CastArgs&, const RayGeom&, const GeoState&, int) {}

    template <class Run>
    __device__ __forceinline__ bool at_surface(const CastArgs& a, Run& R)
    {
        if (k >= n_extra) return false;
        int j = a.n_obs - 1;
        while (j > 0 && a.obs[j].ray_first > R.ray) --j;
        const double a_s = surf[j * n_extra + k].y;
        R.write_outputs(a, (int64_t)k * a.n_rays + R.ray, j, a_s, 1.0 / a_s - 1.0, MPATH_RAY_REACHED);
        ++k;
        R.eta_s = k < n_extra ? surf[j * n_extra + k].x : a.obs[j].eta_s;
        return true;
    }
};

template <bool AMR>
__global__ __launch_bounds__(kBlock, 2) void cast_surfaces_kernel(CastArgs a, Surfaces S)
{
    extern __shared__ float coef_lds[];
    const int64_t r = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_rays) return;
    RayRun<AMR> R;
    R.F.bind(coef_lds + threadIdx.x);
    R.start(a, r);
    int j = a.n_obs - 1;
    while (j > 0 && a.obs[j].ray_first > r) --j;
    R.eta_s = S.surf[j * S.n_extra].x;
    S.k = 0;
    R.template advance<false, Surfaces>(a, 0x7fffffff, S);
    // a ray that stopped before some surface: those slots get its status
    for (int k = S.k; k < S.n_extra; ++k) {
        const double a_s = S.surf[j * S.n_extra + k].y;
        R.write_outputs(a, (int64_t)k * a.n_rays + r, j, a_s, 1.0 / a_s - 1.0, R.status);
    }
    const ObsDev& ob = a.obs[j];
    R.write_outputs(a, (int64_t)S.n_extra * a.n_rays + r, j, ob.a_s, ob.z0, R.status);
}

// Born approximation of the infinitesimal-beam matrix: the same
// line-of-sight integral taken along the straight line x_obs + chi n from the
// observer to the stop surface's comoving distance chi_s = eta_0 - eta_s,
// sampled at chi_{i+1} = min(chi_i + ds_i, chi_s), ds_i the integration's
// step length at x(chi_i) (N steps per leaf or coarse cell).
template <bool AMR>
__global__ __launch_bounds__(kBlock, 2) void born_beam_kernel(CastArgs a, float* A, int32_t* status_out)
{
    extern __shared__ float born_lds[];
    const int64_t r = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_rays) return;
    const GridDev& g = a.grid;
    int j = a.n_obs - 1;
    while (j > 0 && a.obs[j].ray_first > r) --j;
    const ObsDev& ob = a.obs[j];
    RayGeom geo;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        geo.vo[i] = ldexp(ob.x[i] / g.h0, g.max_level + 1);
        geo.n[i] = a.dirs[3 * r + i];
    }
    const double eta_s = a.ray_stop ? a.ray_stop[r].x : ob.eta_s;
    const double chis = a.cosmo_eta0 - eta_s;
    InfBeam<AMR> B;
    B.init(born_lds + threadIdx.x);
    FieldCache<AMR> F;          // leaf lookups only (no stencil, no LDS)
    F.reset();
    GeoState y;
    y.K = 1.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) { y.d[i] = 0.0f; y.dx[i] = 0.0f; }
    double chi = 0.0;
    int status = MPATH_RAY_MAX_STEPS;
    for (int64_t steps = 0;; ++steps) {
        y.eta = a.cosmo_eta0 - chi;
        double v[3];
        grid_coords(g, geo, y.eta, y.dx, v);
        int I[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) I[d] = (int)floor(v[d]);
        const int L = F.leaf(g, I);
        if (L < 0) { status = MPATH_RAY_LEFT_DOMAIN; break; }
        B.at_step(a, geo, y, L);
        if (chi >= chis) { status = MPATH_RAY_REACHED; break; }
        if (steps >= a.max_steps) break;
        const double ds = step_length(a, L);
        chi = chi + ds < chis ? chi + ds : chis;
    }
    B.write(A + 4 * r, status == MPATH_RAY_REACHED);
    if (status_out) status_out[r] = status;
}

// Static schedule with the NGP (ORDER 0) or TSC (ORDER 2) field evaluator.
template <bool AMR, int ORDER>
__global__ __launch_bounds__(kBlock, 2) void cast_order_kernel(CastArgs a)
{
    extern __shared__ float order_lds[];
    const int64_t r = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_rays) return;
    using FC = typename std::conditional<ORDER == 0, NgpCache<AMR>, TscCache<AMR>>::type;
    RayRun<AMR, FC> R;
    R.F.bind(order_lds + threadIdx.x);
    R.start(a, r);
    R.advance(a, 0x7fffffff);
    R.finish(a);
}

__global__ void zero_u64(unsigned long long* p) { *p = 0ull; }

__global__ void permute_values_kernel(float4* payload, const int64_t* perm, const float4* values, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) payload[i] = values[perm[i]];
}

// ---------------------------------------------------------------------------
// Forward-mode derivative of the cast with respect to the initial direction
// theta: two tangents, b = 1, 2, moving the initial unit vector n along
// e1 = e_phi, e2 = -e_theta (the screen basis at theta).  Written in the
// physical variables (eta, x, k0 = -K, k) of the geodesic equations
// (Sect. 2.2), whose RK4 map equals the split one of the kernels; the
// tangent of a state is kept as
//   (deta, dK, dX = dx - s e_b, dQ = dk - K e_b),   s = eta_0 - eta,
// so that the parts of order one (the unlensed change s e_b of the position
// and K e_b of the wave vector, carried exactly by the primal s and K) never
// enter float32 arithmetic, and only lensing-sized quantities do.  With
// F = dy/dl, psi = G.k and G, JG the interpolated gradient and its spatial
// derivative (the trilinear interpolant of the stencil),
//   deta' = -dK
//   dK'   = 2 H' K^2 deta + (4 H K - 2 psi) dK - 2 K dpsi
//   dX'   = dQ
//   dQ'   = 2 H' deta K k + 2 H dK k + (2 H K + 2 psi) dQ + 2 dpsi k
//           - 2 dG K^2 - 4 G K dK + 4 psi K e_b,
//   dG = JG (s e_b + dX),  dpsi = dG.k + K G.e_b + G.dQ,
// and RK4 is differentiated stage by stage, including the step length
// dl = ds / K (d(dl) = -dl dK / K: the term rho (Y_i - y), rho = -dK/K,
// with Y_i - y = c_i dl F_{i-1}).  The landing step's length is set by the
// source surface; its pass is differentiated at fixed length and the end
// tangent projected along the flow afterwards (tangent_observables_kernel).
// ---------------------------------------------------------------------------
struct TangentPair {
    float n[3];                                   // initial direction
    float e[2][3];                                // e_b
    float dEta[2], dK[2], dX[2][3], dQ[2][3];     // tangents at the step start
    float fEta[2], fK[2], fX[2][3], fQ[2][3];     // their derivative at the previous stage
    float aEta[2], aK[2], aX[2][3], aQ[2][3];     // sum of w_i times it over the stages
    float rho[2];                                  // d(dl)/dl of the recorded pass
    float dlf;                                     // its affine length
    double eta0;
    float inv_h0;

    __device__ __forceinline__ void init(const CastArgs& a, const RayGeom& geo, float phi_o)
    {
        eta0 = a.cosmo_eta0;
        inv_h0 = (float)a.grid.inv_h0;
        const double* v = geo.n;
        const double rh = hypot(v[0], v[1]);
        const double cp = rh > 0.0 ? v[0] / rh : 1.0, sp = rh > 0.0 ? v[1] / rh : 0.0;
        const double ct = v[2], st = rh;
        const double eb[2][3] = {{-sp, cp, 0.0}, {-cp * ct, -sp * ct, st}};
        // k = kmag n at the observer, so dk = kmag e_b there and dQ = (kmag - 1) e_b
        const double po = (double)phi_o;
        const float km1 = (float)(sqrt((1.0 + 2.0 * po) / (1.0 - 2.0 * po)) - 1.0);
#pragma unroll
        for (int i = 0; i < 3; ++i) n[i] = (float)v[i];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            dEta[b] = 0.0f;
            dK[b] = 0.0f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                e[b][i] = (float)eb[b][i];
                dX[b][i] = 0.0f;
                dQ[b][i] = km1 * e[b][i];
            }
        }
    }

    __device__ __forceinline__ void begin_step(const GeoState& y, double dl, bool regular)
    {
        dlf = (float)dl;
        const float invK = 1.0f / (float)y.K;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            rho[b] = regular ? -dK[b] * invK : 0.0f;
            aEta[b] = 0.0f;
            aK[b] = 0.0f;
#pragma unroll
            for (int i = 0; i < 3; ++i) { aX[b][i] = 0.0f; aQ[b][i] = 0.0f; }
        }
    }

    // Y - y in the physical variables: (eta, K, x, k) differences
    __device__ __forceinline__ void diff(const GeoState& y, const GeoState& Y, float& De, float& DK, float Dx[3],
                                         float Dk[3]) const
    {
        De = (float)(Y.eta - y.eta);
        DK = (float)(Y.K - y.K);
        const float KY = (float)Y.K, Ky = (float)y.K;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Dx[i] = fmaf(-De, n[i], Y.dx[i] - y.dx[i]);
            Dk[i] = fmaf(DK, n[i], fmaf(KY, Y.d[i], -Ky * y.d[i]));
        }
    }

    template <class FC>
    __device__ __forceinline__ void stage(int st, const GeoState& y, const GeoState& yi, const FC& F,
                                          const float* G, const HubbleCubic& Hc, const CosmoDev& cz)
    {
        const float c = st == 0 ? 0.0f : (st == 3 ? 1.0f : 0.5f);
        const float cdl = c * dlf;
        const float w = (st == 0 || st == 3) ? 1.0f : 2.0f;
        const float Kf = (float)yi.K;
        float k[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) k[i] = Kf * (n[i] + yi.d[i]);
        const float s = (float)(eta0 - yi.eta);
        const float H = (float)Hc(cz, yi.eta), dH = (float)Hc.deriv(cz, yi.eta);
        const float psi = G[0] * k[0] + G[1] * k[1] + G[2] * k[2];
        float De, DK, Dx[3], Dk[3];
        diff(y, yi, De, DK, Dx, Dk);
        // spatial derivative of the interpolated gradient: the t-derivatives
        // of the stencil's trilinear interpolant times 2^lvl / h0
        const float tx = F.t[0], ty = F.t[1], tz = F.t[2];
        const float sc = ldexpf(inv_h0, F.lvl);
        float JG[3][3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float* q = F.c + 8 * (j + 1) * FC::cstride;
            const float c1 = q[FC::cstride], c2 = q[2 * FC::cstride], c3 = q[3 * FC::cstride];
            const float c4 = q[4 * FC::cstride], c5 = q[5 * FC::cstride], c6 = q[6 * FC::cstride];
            const float c7 = q[7 * FC::cstride];
            JG[j][0] = (c1 + ty * c4 + tz * c5 + ty * tz * c7) * sc;
            JG[j][1] = (c2 + tx * c4 + tz * c6 + tx * tz * c7) * sc;
            JG[j][2] = (c3 + tx * c5 + ty * c6 + tx * ty * c7) * sc;
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            float te = dEta[b], tK = dK[b], tX[3], tQ[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) { tX[i] = dX[b][i]; tQ[i] = dQ[b][i]; }
            if (st > 0) {
                te += cdl * fEta[b] + rho[b] * De;
                tK += cdl * fK[b] + rho[b] * DK;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    tX[i] += cdl * fX[b][i] + rho[b] * Dx[i];
                    tQ[i] += cdl * fQ[b][i] + rho[b] * Dk[i];
                }
            }
            float dxf[3], dG[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) dxf[i] = s * e[b][i] + tX[i];
#pragma unroll
            for (int j = 0; j < 3; ++j) dG[j] = JG[j][0] * dxf[0] + JG[j][1] * dxf[1] + JG[j][2] * dxf[2];
            const float dpsi = (dG[0] * k[0] + dG[1] * k[1] + dG[2] * k[2]) +
                               Kf * (G[0] * e[b][0] + G[1] * e[b][1] + G[2] * e[b][2]) +
                               (G[0] * tQ[0] + G[1] * tQ[1] + G[2] * tQ[2]);
            fEta[b] = -tK;
            fK[b] = 2.0f * dH * Kf * Kf * te + (4.0f * H * Kf - 2.0f * psi) * tK - 2.0f * Kf * dpsi;
            const float ck = 2.0f * dH * te * Kf + 2.0f * H * tK + 2.0f * dpsi;
            const float cq = 2.0f * H * Kf + 2.0f * psi;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                fX[b][i] = tQ[i];
                fQ[b][i] = ck * k[i] + cq * tQ[i] - 2.0f * Kf * Kf * dG[i] - 4.0f * Kf * tK * G[i] +
                           4.0f * psi * Kf * e[b][i];
            }
            aEta[b] += w * fEta[b];
            aK[b] += w * fK[b];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                aX[b][i] += w * fX[b][i];
                aQ[b][i] += w * fQ[b][i];
            }
        }
    }

    __device__ __forceinline__ void end_step(const GeoState& y, const GeoState& yn)
    {
        float De, DK, Dx[3], Dk[3];
        diff(y, yn, De, DK, Dx, Dk);
        const float h6 = dlf * (1.0f / 6.0f);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            dEta[b] += h6 * aEta[b] + rho[b] * De;
            dK[b] += h6 * aK[b] + rho[b] * DK;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                dX[b][i] += h6 * aX[b][i] + rho[b] * Dx[i];
                dQ[b][i] += h6 * aQ[b][i] + rho[b] * Dk[i];
            }
        }
    }
};

// The cast with the two tangents: the primal outputs of the plain cast (bit
// for bit) and the tangent end states for tangent_observables_kernel.
// The tangents take registers the plain cast has not: two waves per SIMD.
template <bool AMR>
__global__ __launch_bounds__(kBlock, 2) void cast_tangent_kernel(CastArgs a, TanEnd* te)
{
    extern __shared__ float coef_lds[];
    const int64_t r = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_rays) return;
    RayRun<AMR> R;
    R.F.bind(coef_lds + threadIdx.x);
    R.start(a, r);
    TangentPair T;
    T.init(a, R.geo, R.phi_o);
    R.advance_recorded(a, T);
    R.finish(a);           // leaves the end point's stencil in R.F
    TanEnd e;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        e.deta[b] = T.dEta[b];
        e.dK[b] = T.dK[b];
#pragma unroll
        for (int i = 0; i < 3; ++i) e.dX[b][i] = T.dX[b][i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) e.d[i] = R.y.d[i];
    e.phi_o = R.phi_o;
    e.K = R.y.K;
    e.base = R.F.base;
    e.lvl = R.F.lvl;
    e.status = R.status;
    e.pad = 0;
    te[r] = e;
}

// Distortion matrix and dz5/dtheta from the tangent end states (double
// precision).  The landing step ends on eta = eta_s whatever theta is, so
// the end tangent is projected along the flow F(y_f) until deta = 0:
// dy_f += F(y_f) deta / K_f.  Then, with r = x_f - x_obs,
//   A_ab = e~_a(beta) . (s_f e_b + dX_b) / |r|     (Sect. 2.3, rows on the
//          screen basis at the end direction, columns on the one at theta)
//   dz5_b = a_s / (1 + Phi_o) [dK_b (1 + Phi_s) + K_f dPhi_s_b],
// dPhi_s_b the derivative of the interpolated Phi along the end tangent
// (Sect. 2.5, z5 with v = 0).
__global__ __launch_bounds__(256) void tangent_observables_kernel(CastArgs a, const TanEnd* te, float* jac,
                                                                  float* dz)
{
    const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ray >= a.n_rays) return;
    const float q = __builtin_nanf("");
    const TanEnd T = te[ray];
    if (T.status != MPATH_RAY_REACHED) {
        if (jac) {
#pragma unroll
            for (int i = 0; i < 4; ++i) jac[4 * ray + i] = q;
        }
        if (dz) { dz[2 * ray] = q; dz[2 * ray + 1] = q; }
        return;
    }
    const GridDev& g = a.grid;
    const RayEnd e = a.ends[ray];
    const ObsDev& ob = a.obs[e.obs];
    const double n[3] = {a.dirs[3 * ray], a.dirs[3 * ray + 1], a.dirs[3 * ray + 2]};
    const double s = a.cosmo_eta0 - e.eta;
    double r[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) r[i] = s * n[i] + (double)e.dx[i];
    const double chi = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    // bases: e_b at theta, e~_a at the end direction
    auto basis = [](const double v[3], double e1[3], double e2[3]) {
        const double rh = hypot(v[0], v[1]), rr = sqrt(rh * rh + v[2] * v[2]);
        const double cp = rh > 0.0 ? v[0] / rh : 1.0, sp = rh > 0.0 ? v[1] / rh : 0.0;
        const double ct = v[2] / rr, st = rh / rr;
        e1[0] = -sp; e1[1] = cp; e1[2] = 0.0;
        e2[0] = -cp * ct; e2[1] = -sp * ct; e2[2] = st;
    };
    double eb[2][3], ea[2][3];
    basis(n, eb[0], eb[1]);
    basis(r, ea[0], ea[1]);
    // the interpolant at the end point: Phi, its gradient and grad Phi
    double v[3];
    {
        RayGeom geo;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            geo.vo[i] = ldexp(ob.x[i] / g.h0, g.max_level + 1);
            geo.n[i] = n[i];
        }
        grid_coords(g, geo, e.eta, e.dx, v);
    }
    const double sl = ldexp(1.0, T.lvl - g.max_level - 1);
    double t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double u = v[d] * sl - 0.5;
        t[d] = u - floor(u);
    }
    const float4* rec = g.dual + 8 * (int64_t)T.base;
    double cf[4][8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const float4 c4 = rec[o];
        cf[0][o] = c4.x; cf[1][o] = c4.y; cf[2][o] = c4.z; cf[3][o] = c4.w;
    }
    auto tri = [&](const double* c, double& f, double& fx, double& fy, double& fz) {
        const double tx = t[0], ty = t[1], tz = t[2];
        f = c[0] + tx * (c[1] + ty * (c[4] + tz * c[7]) + tz * c[5]) + ty * (c[2] + tz * c[6]) + tz * c[3];
        fx = c[1] + ty * c[4] + tz * c[5] + ty * tz * c[7];
        fy = c[2] + tx * c[4] + tz * c[6] + tx * tz * c[7];
        fz = c[3] + tx * c[5] + ty * c[6] + tx * ty * c[7];
    };
    const double scale = ldexp(g.inv_h0, T.lvl);
    double phis, gp[3], G[3], dum[3];
    tri(cf[0], phis, gp[0], gp[1], gp[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) gp[i] *= scale;
#pragma unroll
    for (int j = 0; j < 3; ++j) tri(cf[j + 1], G[j], dum[0], dum[1], dum[2]);
    HubbleCubic Hc;
    Hc.init(a.cosmo, e.eta);
    const double H = Hc(a.cosmo, e.eta);
    const double K = T.K;
    double k[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) k[i] = K * (n[i] + (double)T.d[i]);
    const double psi = G[0] * k[0] + G[1] * k[1] + G[2] * k[2];
    const double FK = 2.0 * H * K * K - 2.0 * psi * K;
    const double a_s = a.ray_stop ? a.ray_stop[ray].y : ob.a_s;
    const double pref = a_s / (1.0 + (double)T.phi_o);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const double tau = (double)T.deta[b] / K;
        double dr[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) dr[i] = s * eb[b][i] + ((double)T.dX[b][i] + tau * k[i]);
        const double dKb = (double)T.dK[b] + tau * FK;
        if (jac) {
#pragma unroll
            for (int aa = 0; aa < 2; ++aa)
                jac[4 * ray + 2 * aa + b] = (float)((ea[aa][0] * dr[0] + ea[aa][1] * dr[1] + ea[aa][2] * dr[2]) / chi);
        }
        if (dz) {
            const double dphi = gp[0] * dr[0] + gp[1] * dr[1] + gp[2] * dr[2];
            dz[2 * ray + b] = (float)(pref * (dKb * (1.0 + phis) + K * dphi));
        }
    }
}

}  // namespace

hipError_t launch_cast_static(const CastArgs& a, int block, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    const int64_t blocks = (a.n_rays + block - 1) / block;
    const bool amr = a.grid.max_level > 0, td = a.grid.tdual != nullptr;
    const size_t lds = (size_t)(td ? FieldCache<true, true>::kFloats : FieldCache<true>::kFloats) * block *
                       sizeof(float);
    const dim3 grid((unsigned)blocks), blk(block);
    if (td) {
        if (amr) hipLaunchKernelGGL((cast_static_kernel<true, true>), grid, blk, lds, s, a);
        else hipLaunchKernelGGL((cast_static_kernel<false, true>), grid, blk, lds, s, a);
    } else {
        if (amr) hipLaunchKernelGGL((cast_static_kernel<true, false>), grid, blk, lds, s, a);
        else hipLaunchKernelGGL((cast_static_kernel<false, false>), grid, blk, lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_cast_checkpointed(const CastArgs& a, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    const int64_t blocks = (a.n_rays + kBlock - 1) / kBlock;
    const size_t lds = (size_t)32 * kBlock * sizeof(float);
    if (a.grid.max_level > 0)
        hipLaunchKernelGGL(cast_ckpt_kernel<true>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
    else
        hipLaunchKernelGGL(cast_ckpt_kernel<false>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_cast_infbeam(const CastArgs& a, float* A, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    const int64_t blocks = (a.n_rays + kBlock - 1) / kBlock;
    const size_t lds = (size_t)64 * kBlock * sizeof(float);
    if (a.grid.max_level > 0)
        hipLaunchKernelGGL(cast_infbeam_kernel<true>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a, A);
    else
        hipLaunchKernelGGL(cast_infbeam_kernel<false>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a, A);
    return hipGetLastError();
}

hipError_t launch_cast_tangent(const CastArgs& a, TanEnd* te, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    const int64_t blocks = (a.n_rays + kBlock - 1) / kBlock;
    const size_t lds = (size_t)32 * kBlock * sizeof(float);
    if (a.grid.max_level > 0)
        hipLaunchKernelGGL(cast_tangent_kernel<true>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a, te);
    else
        hipLaunchKernelGGL(cast_tangent_kernel<false>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a, te);
    return hipGetLastError();
}

hipError_t launch_tangent_observables(const CastArgs& a, const TanEnd* te, float* jac, float* dz_dtheta,
                                      hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(tangent_observables_kernel, dim3((unsigned)((a.n_rays + 255) / 256)), dim3(256), 0, s, a, te,
                       jac, dz_dtheta);
    return hipGetLastError();
}

hipError_t launch_cast_order(const CastArgs& a, int order, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    const int64_t blocks = (a.n_rays + kBlock - 1) / kBlock;
    const size_t lds = 0;
    const dim3 grid((unsigned)blocks), block(kBlock);
    const bool amr = a.grid.max_level > 0;
    if (order == 0) {
        if (amr) hipLaunchKernelGGL((cast_order_kernel<true, 0>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((cast_order_kernel<false, 0>), grid, block, lds, s, a);
    } else {
        if (amr) hipLaunchKernelGGL((cast_order_kernel<true, 2>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((cast_order_kernel<false, 2>), grid, block, lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_born_beam(const CastArgs& a, float* A, int32_t* status, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    const int64_t blocks = (a.n_rays + kBlock - 1) / kBlock;
    const size_t lds = (size_t)32 * kBlock * sizeof(float);
    if (a.grid.max_level > 0)
        hipLaunchKernelGGL(born_beam_kernel<true>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a, A, status);
    else
        hipLaunchKernelGGL(born_beam_kernel<false>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a, A, status);
    return hipGetLastError();
}

hipError_t launch_cast_surfaces(const CastArgs& a, const double2* surf, int n_extra, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    const int64_t blocks = (a.n_rays + kBlock - 1) / kBlock;
    const size_t lds = (size_t)32 * kBlock * sizeof(float);
    Surfaces S;
    S.surf = surf;
    S.n_extra = n_extra;
    S.k = 0;
    if (a.grid.max_level > 0)
        hipLaunchKernelGGL(cast_surfaces_kernel<true>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a, S);
    else
        hipLaunchKernelGGL(cast_surfaces_kernel<false>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a, S);
    return hipGetLastError();
}

hipError_t launch_cast_stop(const CastArgs& a, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n_rays + kBlock - 1) / kBlock)), blk(kBlock);
    const size_t lds = (size_t)FieldCache<true>::kFloats * kBlock * sizeof(float);
    const bool amr = a.grid.max_level > 0;
    switch (a.surface) {
        case MPATH_SURFACE_CHI:
            if (amr) hipLaunchKernelGGL((cast_stop_kernel<true, MPATH_SURFACE_CHI>), grid, blk, lds, s, a);
            else hipLaunchKernelGGL((cast_stop_kernel<false, MPATH_SURFACE_CHI>), grid, blk, lds, s, a);
            break;
        case MPATH_SURFACE_LAMBDA:
            if (amr) hipLaunchKernelGGL((cast_stop_kernel<true, MPATH_SURFACE_LAMBDA>), grid, blk, lds, s, a);
            else hipLaunchKernelGGL((cast_stop_kernel<false, MPATH_SURFACE_LAMBDA>), grid, blk, lds, s, a);
            break;
        case MPATH_SURFACE_Z:
            if (amr) hipLaunchKernelGGL((cast_stop_kernel<true, MPATH_SURFACE_Z>), grid, blk, lds, s, a);
            else hipLaunchKernelGGL((cast_stop_kernel<false, MPATH_SURFACE_Z>), grid, blk, lds, s, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cast_diff(const CastArgs& a, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n_rays + kBlock - 1) / kBlock)), blk(kBlock);
    const size_t lds = (size_t)FieldCache<true>::kFloats * kBlock * sizeof(float);
    if (a.grid.max_level > 0) hipLaunchKernelGGL(cast_diff_kernel<true>, grid, blk, lds, s, a);
    else hipLaunchKernelGGL(cast_diff_kernel<false>, grid, blk, lds, s, a);
    return hipGetLastError();
}

hipError_t launch_ray_dirs(const CastArgs& a, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(ray_dirs_kernel, dim3((unsigned)((a.n_rays + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_observables(const CastArgs& a, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(observables_kernel, dim3((unsigned)((a.n_rays + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cast_persistent(const CastArgs& a, int block, int blocks, hipStream_t s)
{
    if (a.n_rays == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, s, a.queue);
    const bool amr = a.grid.max_level > 0, td = a.grid.tdual != nullptr;
    const size_t lds = (size_t)(td ? FieldCache<true, true>::kFloats : FieldCache<true>::kFloats) * block *
                       sizeof(float);
    const dim3 grid(blocks), blk(block);
    if (td) {
        if (amr) hipLaunchKernelGGL((cast_persistent_kernel<true, true>), grid, blk, lds, s, a);
        else hipLaunchKernelGGL((cast_persistent_kernel<false, true>), grid, blk, lds, s, a);
    } else {
        if (amr) hipLaunchKernelGGL((cast_persistent_kernel<true, false>), grid, blk, lds, s, a);
        else hipLaunchKernelGGL((cast_persistent_kernel<false, false>), grid, blk, lds, s, a);
    }
    return hipGetLastError();
}

int cast_occupancy_blocks_per_cu(int block, bool amr, bool time_dep)
{
    int nb = 0;
    const size_t lds = (size_t)(time_dep ? FieldCache<true, true>::kFloats : FieldCache<true>::kFloats) * block *
                       sizeof(float);
    hipError_t e;
    if (time_dep)
        e = amr ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cast_persistent_kernel<true, true>, block, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cast_persistent_kernel<false, true>, block, lds);
    else
        e = amr ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cast_persistent_kernel<true, false>, block, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cast_persistent_kernel<false, false>, block, lds);
    return e == hipSuccess ? nb : 0;
}

hipError_t launch_permute_values(float4* payload, const int64_t* perm, const float4* values, int64_t n,
                                 hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(permute_values_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, payload, perm,
                       values, n);
    return hipGetLastError();
}

}  // namespace mpath
