// adjoint.hip -- reverse-mode derivative of the ray-casting map on gfx950.
//
// The forward cast (with checkpoints) stores every ray's state before steps
// 0, K, 2K, ...  The adjoint kernel then runs, per ray, one reverse sweep:
// segment by segment from the source back to the observer it recomputes the
// K steps of the segment from its checkpoint (the same code as the forward,
// so every leaf level, stencil and landing decision is replayed exactly) into
// a per-ray tape, and for every step in reverse order re-records the four
// RK4 stages and applies the transposed Jacobian of the step.
//
// The derivative is that of the discrete map: classical RK4 on the null
// geodesic equations of Sect. 2.2 with CIC interpolation (piecewise
// trilinear, so grad Phi has a piecewise-constant spatial derivative), step
// length h_leaf / N with affine step ds / |k0| (differentiated through k0),
// and the landing step on the source iso-eta surface (implicit step length).
// It is computed in double precision on the physical variables
// (eta, x, k0, k), whose RK4 map equals the split one of the forward kernels.
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

constexpr int kMinWavesAdj = 1;

// Physical state (eta, x, k0, k) or a cotangent of it.
struct Phys {
    double eta, x[3], k0, k[3];
};

__device__ __forceinline__ void phys_zero(Phys& a)
{
    a.eta = 0.0; a.k0 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) { a.x[i] = 0.0; a.k[i] = 0.0; }
}

__device__ __forceinline__ void phys_axpy(Phys& a, double s, const Phys& b)
{
    a.eta += s * b.eta; a.k0 += s * b.k0;
#pragma unroll
    for (int i = 0; i < 3; ++i) { a.x[i] += s * b.x[i]; a.k[i] += s * b.k[i]; }
}

__device__ __forceinline__ double phys_dot(const Phys& a, const Phys& b)
{
    double s = a.eta * b.eta + a.k0 * b.k0;
#pragma unroll
    for (int i = 0; i < 3; ++i) s += a.x[i] * b.x[i] + a.k[i] * b.k[i];
    return s;
}

// The four stages of one RK4 step as the forward computed them.
struct StageRecord {
    GeoState y[4];
    int base[4];
    int lvl[4];
    __device__ __forceinline__ void stage(int i, const GeoState& yi, int b, int l)
    {
        y[i] = yi;
        base[i] = b;
        lvl[i] = l;
    }
};

// Everything the transposed stage Jacobian needs at one stage.
struct Jet {
    Phys Y;             // stage state
    Phys F;             // right-hand side at Y
    double G[3];        // interpolated grad Phi
    double JG[3][3];    // dG_j / dx_l of the trilinear interpolant
    double phi, gphi[3];// interpolated Phi and the gradient of its interpolant
    double H, dH;       // a'/a and its eta-derivative
    float w[8];         // CIC weights of the 8 stencil cells
    int base;
};

struct RayCtx {
    RayGeom geo;
    double xobs[3];
};

__device__ __forceinline__ void make_jet(const AdjointArgs& A, const RayCtx& R, const GeoState& ys, int base,
                                         int lvl, const HubbleCubic& Hc, Jet& J)
{
    const GridDev& g = A.c.grid;
    const double s = g.eta0 - ys.eta;
    double u[3];
    J.Y.eta = ys.eta;
    J.Y.k0 = -ys.K;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double disp = s * R.geo.n[i] + (double)ys.dx[i];
        J.Y.x[i] = R.xobs[i] + disp;
        u[i] = R.geo.uo[i] + disp * g.inv_h0;
        J.Y.k[i] = ys.K * (R.geo.n[i] + (double)ys.d[i]);
    }
    const double sl = (double)(1 << lvl);
    double t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double q = u[d] * sl - 0.5;
        t[d] = q - floor(q);
    }
    const float4* rec = g.dual + 8 * (int64_t)base;
    float4 c[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) c[o] = rec[o];
    const double tx = t[0], ty = t[1], tz = t[2];
    const double scale = sl * g.inv_h0;      // d t / d x
    double f[4], fx[4], fy[4], fz[4];
#define MPATH_JET(q, m)                                                                       \
    {                                                                                         \
        const double c0 = c[0].m, c1 = c[1].m, c2 = c[2].m, c3 = c[3].m;                       \
        const double c4 = c[4].m, c5 = c[5].m, c6 = c[6].m, c7 = c[7].m;                       \
        f[q] = c0 + tx * (c1 + ty * (c4 + tz * c7) + tz * c5) + ty * (c2 + tz * c6) + tz * c3; \
        fx[q] = c1 + ty * c4 + tz * c5 + ty * tz * c7;                                        \
        fy[q] = c2 + tx * c4 + tz * c6 + tx * tz * c7;                                        \
        fz[q] = c3 + tx * c5 + ty * c6 + tx * ty * c7;                                        \
    }
    MPATH_JET(0, x) MPATH_JET(1, y) MPATH_JET(2, z) MPATH_JET(3, w)
#undef MPATH_JET
    J.phi = f[0];
    J.gphi[0] = fx[0] * scale; J.gphi[1] = fy[0] * scale; J.gphi[2] = fz[0] * scale;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        J.G[j] = f[j + 1];
        J.JG[j][0] = fx[j + 1] * scale;
        J.JG[j][1] = fy[j + 1] * scale;
        J.JG[j][2] = fz[j + 1] * scale;
    }
    const CosmoDev& cz = A.c.cosmo;
    J.H = Hc(cz, ys.eta);
    J.dH = Hc.deriv(cz, ys.eta);
    // right-hand side of the geodesic equations (Sect. 2.2) at the stage
    const double k0 = J.Y.k0;
    const double psi = J.G[0] * J.Y.k[0] + J.G[1] * J.Y.k[1] + J.G[2] * J.Y.k[2];
    J.F.eta = k0;
    J.F.k0 = -2.0 * J.H * k0 * k0 - 2.0 * psi * k0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        J.F.x[j] = J.Y.k[j];
        J.F.k[j] = -2.0 * J.H * k0 * J.Y.k[j] + 2.0 * psi * J.Y.k[j] - 2.0 * J.G[j] * k0 * k0;
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const double wx = (o & 1) ? tx : 1.0 - tx;
        const double wy = (o & 2) ? ty : 1.0 - ty;
        const double wz = (o & 4) ? tz : 1.0 - tz;
        J.w[o] = (float)(wx * wy * wz);
    }
    J.base = base;
}

// Transposed Jacobian of the right-hand side at a stage applied to v:
// Yb = (dF/dY)^T v and the cotangent Gb of the interpolated grad Phi.
__device__ __forceinline__ void rhs_vjp(const Jet& J, const Phys& v, Phys& Yb, double Gb[3])
{
    const double k0 = J.Y.k0;
    const double a = v.k0;
    const double bk = v.k[0] * J.Y.k[0] + v.k[1] * J.Y.k[1] + v.k[2] * J.Y.k[2];
    const double bG = v.k[0] * J.G[0] + v.k[1] * J.G[1] + v.k[2] * J.G[2];
    const double psi = J.G[0] * J.Y.k[0] + J.G[1] * J.Y.k[1] + J.G[2] * J.Y.k[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) Gb[j] = -2.0 * k0 * a * J.Y.k[j] + 2.0 * bk * J.Y.k[j] - 2.0 * k0 * k0 * v.k[j];
    Yb.eta = -2.0 * J.dH * k0 * (a * k0 + bk);
    Yb.k0 = v.eta + a * (-4.0 * J.H * k0 - 2.0 * psi) - 2.0 * J.H * bk - 4.0 * k0 * bG;
#pragma unroll
    for (int j = 0; j < 3; ++j)
        Yb.k[j] = v.x[j] - 2.0 * k0 * a * J.G[j] + (-2.0 * J.H * k0 + 2.0 * psi) * v.k[j] + 2.0 * J.G[j] * bk;
#pragma unroll
    for (int l = 0; l < 3; ++l) Yb.x[l] = J.JG[0][l] * Gb[0] + J.JG[1][l] * Gb[1] + J.JG[2][l] * Gb[2];
}

// Per-lane accumulator of cell cotangents for the current stencil (in LDS),
// flushed to global memory with atomics when the stencil changes.
struct Scatter {
    float* acc;         // 32 slots, stride kBlock: (corner o, component q) at (4 o + q) * kBlock
    int cur;

    __device__ __forceinline__ void init(float* lds)
    {
        acc = lds;
        cur = -1;
#pragma unroll
        for (int i = 0; i < 32; ++i) acc[i * kBlock] = 0.0f;
    }

    __device__ __forceinline__ void flush(const AdjointArgs& A)
    {
        if (cur < 0) return;
        const int32_t* ids = A.c.grid.dual_ids + 8 * (int64_t)cur;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int id = ids[o];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float v = acc[(4 * o + q) * kBlock];
                if (v != 0.0f && id >= 0) unsafeAtomicAdd(A.grad + 4 * (int64_t)id + q, v);
                acc[(4 * o + q) * kBlock] = 0.0f;
            }
        }
        cur = -1;
    }

    // add w_o * vals[q] to component q0 + q of corner o
    __device__ __forceinline__ void add(const AdjointArgs& A, int base, const float w[8], int q0, int nq,
                                        const double* vals)
    {
        if (base != cur) {
            flush(A);
            cur = base;
        }
#pragma unroll
        for (int o = 0; o < 8; ++o)
            for (int q = 0; q < nq; ++q) acc[(4 * o + q0 + q) * kBlock] += w[o] * (float)vals[q];
    }
};

// Step length and landing decision at the start of a step, exactly as the
// forward kernels take them.
template <bool AMR>
__device__ __forceinline__ bool plan_step(const CastArgs& a, FieldCache<AMR>& F, const RayGeom& geo,
                                          const GeoState& y, double eta_s, double& ds, double& dl, bool& landing)
{
    const GridDev& g = a.grid;
    double u[3];
    grid_coords(g, geo, y.eta, y.dx, u);
    const int Lm = AMR ? g.max_level : 0;
    const double scale = (double)(2 << Lm);
    int I[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) I[d] = (int)floor(u[d] * scale);
    const int L = F.leaf(g, I);
    if (L < 0) return false;
    const int lstep = a.adaptive ? L : 0;
    ds = g.h0 / (double)(1 << lstep) / (double)a.steps_per_cell;
    dl = ds / y.K;
    landing = y.eta - y.K * dl < eta_s;
    return true;
}

// One forward step (regular or landing) from y, as in the forward kernels;
// records the stages of the final RK4 pass when rec is given.  Returns the
// affine length of the step taken through *dl_taken.
template <bool AMR, class Rec>
__device__ __forceinline__ bool forward_step(const CastArgs& a, FieldCache<AMR>& F, const RayGeom& geo,
                                             const GeoState& y, double eta_s, GeoState& yn, Rec* rec,
                                             double& dl_taken, double& ds_out, bool& landing)
{
    double ds, dl;
    if (!plan_step<AMR>(a, F, geo, y, eta_s, ds, dl, landing)) return false;
    double dlx = landing ? (y.eta - eta_s) / y.K : dl;
    uint32_t h = 0;
    if (landing) {
        for (int k = 0; k < 2; ++k) {
            if (rk4_step<AMR>(a.grid, a.cosmo, F, geo, y, dlx, yn, h)) return false;
            dlx = dlx + (yn.eta - eta_s) / yn.K;
        }
    }
    if (rk4_step<AMR, Rec>(a.grid, a.cosmo, F, geo, y, dlx, yn, h, rec)) return false;
    dl_taken = dlx;
    ds_out = ds;
    return true;
}

// Recompute segment seg (steps [seg K, min(N, (seg + 1) K))) from its
// checkpoint, storing the state before each step in the tape; returns the
// state after the segment.
template <bool AMR>
__device__ __forceinline__ bool recompute_segment(const AdjointArgs& A, FieldCache<AMR>& F, const RayGeom& geo,
                                                  double eta_s, int64_t ray, int seg, int N, GeoState& yend)
{
    const CastArgs& a = A.c;
    const int K = a.ckpt_every;
    GeoState y = a.ckpt[(int64_t)seg * a.n_rays + ray];
    const int j1 = min(N, (seg + 1) * K);
    for (int j = seg * K; j < j1; ++j) {
        A.tape[(int64_t)(j - seg * K) * a.n_rays + ray] = y;
        GeoState yn;
        double dl, ds;
        bool landing;
        if (!forward_step<AMR, NoRecord>(a, F, geo, y, eta_s, yn, (NoRecord*)nullptr, dl, ds, landing))
            return false;
        y = yn;
    }
    yend = y;
    return true;
}

// Reverse of one RK4 step for all W cotangent columns: the four stages are
// visited last to first; the jet of a stage is formed once and applied to
// every column.  For y' = y + dl/6 (F1 + 2 F2 + 2 F3 + F4) with
// Y_i = y + c_i dl F_{i-1} (c = 1/2, 1/2, 1):
//   Fbar_4 = dl/6 v,  Ybar_i = J_i^T Fbar_i,
//   Fbar_{i-1} = w_{i-1}/6 dl v + c_i dl Ybar_i,  ybar = v + sum_i Ybar_i,
//   dlbar = sum_i (w_i/6) v.F_i + sum_{i>1} c_i Ybar_i.F_{i-1}.
template <bool AMR, int W, bool SCATTER>
__device__ __forceinline__ void reverse_step(const AdjointArgs& A, const RayCtx& R, const StageRecord& rec,
                                             const HubbleCubic& Hc, double dl, double ds_reg, double k0_step,
                                             Phys (&yb)[W], Scatter& S)
{
    Phys v[W], Fb[W];
    double dlbar[W];
    Jet J;
    make_jet(A, R, rec.y[3], rec.base[3], rec.lvl[3], Hc, J);
#pragma unroll
    for (int c = 0; c < W; ++c) {
        v[c] = yb[c];
        dlbar[c] = phys_dot(v[c], J.F) / 6.0;
        phys_zero(Fb[c]);
        phys_axpy(Fb[c], dl / 6.0, v[c]);
    }
#pragma unroll 1
    for (int i = 3; i >= 0; --i) {
        Jet P;
        if (i > 0) make_jet(A, R, rec.y[i - 1], rec.base[i - 1], rec.lvl[i - 1], Hc, P);
        const double ci = (i == 3) ? 1.0 : 0.5;
        const double wprev = (i == 1) ? 1.0 : 2.0;
#pragma unroll
        for (int c = 0; c < W; ++c) {
            Phys Yb;
            double Gb[3];
            rhs_vjp(J, Fb[c], Yb, Gb);
            phys_axpy(yb[c], 1.0, Yb);
            if (SCATTER && c == W - 1) S.add(A, J.base, J.w, 1, 3, Gb);
            if (i > 0) {
                dlbar[c] += ci * phys_dot(Yb, P.F) + (wprev / 6.0) * phys_dot(v[c], P.F);
                phys_zero(Fb[c]);
                phys_axpy(Fb[c], wprev / 6.0 * dl, v[c]);
                phys_axpy(Fb[c], ci * dl, Yb);
            }
        }
        if (i > 0) J = P;
    }
    // a regular step has dl = ds / |k0| with ds fixed by the leaf level
    if (ds_reg > 0.0) {
#pragma unroll
        for (int c = 0; c < W; ++c) yb[c].k0 += dlbar[c] * ds_reg / (k0_step * k0_step);
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

// W cotangent columns: W = 4 (beta_1, beta_2, z, L), 3 (beta_1, beta_2, z)
// or 1 (L).  SCATTER: the last column is L and its cell cotangents are kept.
template <bool AMR, int W, bool SCATTER>
__global__ __launch_bounds__(kBlock, kMinWavesAdj) void adjoint_kernel(AdjointArgs A)
{
    extern __shared__ float lds[];      // [32][kBlock] stencil coefficients, [32][kBlock] scatter
    const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const CastArgs& a = A.c;
    if (ray >= a.n_rays) return;
    constexpr bool HAS_JAC = W >= 3;
    const int N = A.n_steps[ray];
    if (A.status[ray] != MPATH_RAY_REACHED || N <= 0) {
        if (HAS_JAC) write_nan_jacobian(A, ray);
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
        R.geo.uo[i] = ob.x[i] / g.h0;
        R.geo.n[i] = a.dirs[3 * ray + i];
    }
    const double eta_s = ob.eta_s;
    FieldCache<AMR> F;
    F.bind(lds + threadIdx.x);
    F.reset();
    Scatter S;
    S.init(lds + 32 * kBlock + threadIdx.x);

    // potential at the observer and the initial |k| (as in the forward)
    float phio_f, Gt[3];
    int ll, lv;
    F.eval(g, R.geo.uo, phio_f, Gt, ll, lv);
    const int obs_base = F.base, obs_lvl = F.lvl;
    const double phio = (double)phio_f;
    const double kmag = sqrt((1.0 + 2.0 * phio) / (1.0 - 2.0 * phio));

    const int K = a.ckpt_every;
    const int nseg = (N + K - 1) / K;
    GeoState yf;
    if (!recompute_segment<AMR>(A, F, R.geo, eta_s, ray, nseg - 1, N, yf)) {
        if (HAS_JAC) write_nan_jacobian(A, ray);
        return;
    }

    // ---- cotangents at the end point ----
    float ph_f;
    double uf[3];
    grid_coords(g, R.geo, yf.eta, yf.dx, uf);
    F.eval(g, uf, ph_f, Gt, ll, lv);
    HubbleCubic Hf;
    Hf.init(a.cosmo, yf.eta);
    Jet Jf;
    make_jet(A, R, yf, F.base, F.lvl, Hf, Jf);
    const double* n = R.geo.n;
    double r[3];
    const double sf = g.eta0 - yf.eta;
#pragma unroll
    for (int i = 0; i < 3; ++i) r[i] = sf * n[i] + (double)yf.dx[i];
    const double chi = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double rh[3] = {r[0] / chi, r[1] / chi, r[2] / chi};
    double f1[3], f2[3], e1[3], e2[3];
    screen_basis(rh, f1, f2);
    screen_basis(n, e1, e2);
    const double phis = Jf.phi;
    const double dz_dK = ob.a_s * (1.0 + phis) / (1.0 + phio);
    const double dz_dphis = ob.a_s * yf.K / (1.0 + phio);
    const double dz_dphio = -ob.a_s * yf.K * (1.0 + phis) / ((1.0 + phio) * (1.0 + phio));

    Phys yb[W];
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
    double phio_bar = 0.0;
    if (SCATTER) {
        // loss column: dL/dalpha through alpha(r^) and dL/dz5
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
        double fs, fps;           // f and f'/sin sigma
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
        Phys& L = yb[W - 1];
#pragma unroll
        for (int i = 0; i < 3; ++i) L.x[i] = (cb[0] * f1[i] + cb[1] * f2[i]) / chi + gz * dz_dphis * Jf.gphi[i];
        L.k0 = -gz * dz_dK;
        const double phis_bar = gz * dz_dphis;
        S.add(A, Jf.base, Jf.w, 0, 1, &phis_bar);
        phio_bar = gz * dz_dphio;
    }
    // landing: eta_s fixed, so the last affine step depends on the state;
    // remove the cotangent along the flow (d y_f / d dl ~ F(y_f), d eta_f / d dl = k0)
#pragma unroll
    for (int c = 0; c < W; ++c) yb[c].eta -= phys_dot(yb[c], Jf.F) / Jf.F.eta;

    // ---- reverse sweep ----
    for (int seg = nseg - 1; seg >= 0; --seg) {
        GeoState ytmp;
        if (seg != nseg - 1)
            if (!recompute_segment<AMR>(A, F, R.geo, eta_s, ray, seg, N, ytmp)) {
                if (HAS_JAC) write_nan_jacobian(A, ray);
                return;
            }
        const int j0 = seg * K;
        const int j1 = min(N, (seg + 1) * K) - 1;
        for (int jj = j1; jj >= j0; --jj) {
            const GeoState y = A.tape[(int64_t)(jj - j0) * a.n_rays + ray];
            StageRecord rec;
            GeoState yn;
            double dl, ds;
            bool landing;
            if (!forward_step<AMR, StageRecord>(a, F, R.geo, y, eta_s, yn, &rec, dl, ds, landing)) {
                if (HAS_JAC) write_nan_jacobian(A, ray);
                return;
            }
            HubbleCubic Hc;
            Hc.init(a.cosmo, y.eta);
            const double ds_reg = landing ? 0.0 : ds;
            reverse_step<AMR, W, SCATTER>(A, R, rec, Hc, dl, ds_reg, -y.K, yb, S);
        }
    }

    // ---- the initial state: k = kmag(Phi_o) n (theta), k0 = -1 ----
    if (HAS_JAC) {
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
        const Phys& L = yb[W - 1];
        const double dkmag = kmag * 2.0 / (1.0 - 4.0 * phio * phio);
        phio_bar += (L.k[0] * n[0] + L.k[1] * n[1] + L.k[2] * n[2]) * dkmag;
        // CIC weights at the observer
        GeoState y0;
        y0.eta = g.eta0;
        y0.K = 1.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) { y0.d[i] = 0.0f; y0.dx[i] = 0.0f; }
        Jet J0;
        make_jet(A, R, y0, obs_base, obs_lvl, Hf, J0);
        S.add(A, obs_base, J0.w, 0, 1, &phio_bar);
        S.flush(A);
    }
}

__global__ void fill_zero_kernel(float* __restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Cell cotangents from library order to the caller's order (overwrites).
__global__ void scatter_grad_kernel(const float4* __restrict__ g_lib, const int64_t* __restrict__ perm,
                                    float4* __restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[perm[i]] = g_lib[i];
}

// On a uniform periodic grid whose gradient is the central difference of the
// potential, g_d[c] = (Phi[c + e_d] - Phi[c - e_d]) / (2 h0), the total
// cotangent of Phi is the direct one plus the transposed difference operator
// applied to the cotangents of g:
//   dL/dPhi[c] += sum_d (gbar_d[c - e_d] - gbar_d[c + e_d]) / (2 h0).
__global__ void central_transpose_kernel(const float4* __restrict__ g_lib, const int4* __restrict__ cellpos,
                                         const int64_t* __restrict__ perm, float* __restrict__ out, int n0,
                                         double inv_2h, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int4 p = cellpos[c];
    const uint32_t m = (uint32_t)n0 - 1u;
    auto id = [m](int i, int j, int k) { return (int64_t)morton3((uint32_t)i & m, (uint32_t)j & m, (uint32_t)k & m); };
    double acc = (double)g_lib[c].x;
    acc += ((double)g_lib[id(p.x - 1, p.y, p.z)].y - (double)g_lib[id(p.x + 1, p.y, p.z)].y) * inv_2h;
    acc += ((double)g_lib[id(p.x, p.y - 1, p.z)].z - (double)g_lib[id(p.x, p.y + 1, p.z)].z) * inv_2h;
    acc += ((double)g_lib[id(p.x, p.y, p.z - 1)].w - (double)g_lib[id(p.x, p.y, p.z + 1)].w) * inv_2h;
    out[perm[c]] = (float)acc;
}

}  // namespace

hipError_t launch_adjoint(const AdjointArgs& A, int columns, hipStream_t s)
{
    const int64_t n = A.c.n_rays;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    const size_t lds = (size_t)64 * kBlock * sizeof(float);
    const bool amr = A.c.grid.max_level > 0;
    if (columns == 4) {
        if (amr) hipLaunchKernelGGL((adjoint_kernel<true, 4, true>), grid, block, lds, s, A);
        else hipLaunchKernelGGL((adjoint_kernel<false, 4, true>), grid, block, lds, s, A);
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

hipError_t launch_scatter_grad(const float4* grad_lib, const int64_t* perm, float4* out_user, int64_t n,
                               hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, grad_lib, perm,
                       out_user, n);
    return hipGetLastError();
}

hipError_t launch_central_transpose(const float4* g_lib, const int4* cellpos, const int64_t* perm, float* out,
                                    int n0, double h0, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(central_transpose_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g_lib, cellpos,
                       perm, out, n0, 0.5 / h0, n);
    return hipGetLastError();
}

}  // namespace mpath
