// mpath_host.cpp -- host side of the C ABI: argument checks, octree build
// (validation, ordering, packing), background cosmology table, observer
// table and kernel launches.  See include/mpath.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace mpath;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(MPATH_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// A failed enqueue after others on the stream: wait for what was queued
// before it (which may still read host buffers released on return), then
// report the failure.
int hip_fail_drain(hipError_t e, hipStream_t s, const char* what)
{
    (void)hipStreamSynchronize(s);
    return hip_fail(e, what);
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr double kH0 = 1.0 / 2997.92458;   // h/Mpc with c = 1
constexpr int kTableN = 4096;
constexpr double kZMaxTable = 20.0;          // rays may be traced up to this redshift

// ---------------------------------------------------------------------------
// Background: flat LCDM, Omega_r = 0.  With y = sqrt(a), d eta = da/(a^2 H)
// becomes d eta = 2 dy / (H0 sqrt(Om + OL y^6)), a smooth integrand; eta(a)
// is evaluated by composite Gauss-Legendre quadrature and a(eta) by Newton's
// method in y.
// ---------------------------------------------------------------------------
struct Background {
    double om = 0.3, ol = 0.7;
    bool is_static = false;
    double gl_x[20], gl_w[20];

    void init(double omega_m, double omega_l)
    {
        om = omega_m;
        ol = omega_l;
        is_static = (om == 0.0 && ol == 0.0);
        // Gauss-Legendre nodes on [-1, 1]: Newton on P_20 from the
        // Chebyshev-like initial guesses
        const int n = 20;
        for (int i = 0; i < n; ++i) {
            double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
            double dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = x;
                for (int k = 2; k <= n; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (x * p1 - p0) / (x * x - 1.0);
                const double dx = p1 / dp;
                x -= dx;
                if (std::fabs(dx) < 1e-16) break;
            }
            gl_x[i] = x;
            gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
        }
    }

    double deta_dy(double y) const { return 2.0 / (kH0 * std::sqrt(om + ol * y * y * y * y * y * y)); }

    double eta_of_y(double y) const
    {
        const int panels = 8;
        const double w = y / panels;
        double sum = 0.0;
        for (int p = 0; p < panels; ++p) {
            const double c = (p + 0.5) * w;
            double s = 0.0;
            for (int i = 0; i < 20; ++i) s += gl_w[i] * deta_dy(c + 0.5 * w * gl_x[i]);
            sum += 0.5 * w * s;
        }
        return sum;
    }

    double eta_of_a(double a) const { return is_static ? 0.0 : eta_of_y(std::sqrt(a)); }

    // affine parameter of the FLRW photon (k0 = -1 at a = 1) from the
    // observer to a: int_a^1 da' / H(a'), H = H0 sqrt(Om / a^3 + OL)
    double lambda_of_a(double a) const
    {
        const int panels = 16;
        const double w = (1.0 - a) / panels;
        double sum = 0.0;
        for (int p = 0; p < panels; ++p) {
            const double c = a + (p + 0.5) * w;
            double s = 0.0;
            for (int i = 0; i < 20; ++i) {
                const double x = c + 0.5 * w * gl_x[i];
                s += gl_w[i] / (kH0 * std::sqrt(om / (x * x * x) + ol));
            }
            sum += 0.5 * w * s;
        }
        return sum;
    }
    double eta0() const { return eta_of_a(1.0); }

    double a_of_eta(double eta) const
    {
        if (is_static) return 1.0;
        // matter-dominated start: eta = 2 y / (H0 sqrt(Om))
        double y = 0.5 * kH0 * std::sqrt(om) * eta;
        for (int it = 0; it < 60; ++it) {
            const double dy = (eta_of_y(y) - eta) / deta_dy(y);
            y -= dy;
            if (std::fabs(dy) <= 1e-16 * y) break;
        }
        return y * y;
    }

    // a'/a = a H = H0 sqrt(Om/a + OL a^2) and its eta-derivative
    // d(a'/a)/d eta = d(aH)/da * a (a'/a)
    void hubble(double a, double& H, double& dH) const
    {
        const double s = std::sqrt(om / a + ol * a * a);
        H = kH0 * s;
        const double dHda = kH0 * (-om / (a * a) + 2.0 * ol * a) / (2.0 * s);
        dH = dHda * a * H;
    }
};

}  // namespace

struct mpath_grid {
    int64_t n_cells = 0;
    int32_t n0 = 0, max_level = 0, periodic = 0;
    double box = 0.0;
    int64_t cells_per_level[16] = {0};
    Background bg;
    double eta0 = 0.0;
    double table_eta_lo = 0.0, table_deta = 0.0;
    char* ws = nullptr;
    float4* payload = nullptr;
    int32_t* child = nullptr;
    float4* dual = nullptr;
    int32_t* leafinfo = nullptr;  // rows of the refined cells (ids >= level_start[1])
    int64_t* perm = nullptr;      // auxiliary tables (null without them)
    int32_t* dual_ids = nullptr;
    double2* table = nullptr;
    double2* atable = nullptr;    // (a, da/deta) on the nodes of table
    float phi_max = INFINITY;     // largest payload phi (+inf after set_values)
    float* tpay = nullptr;        // dPhi/deta per cell (time-dependent potential), else null
    float4* tdual = nullptr;      // its 8 trilinear coefficients per stencil base
    int32_t level_start[kMaxLevels + 1] = {0};
    int num_cus = 0;
};

namespace {

struct GridLayout {
    size_t off_payload, off_child, off_dual, off_leafinfo, off_table, off_atable, off_tpay, off_tdual, off_stage;
    size_t total;
    int64_t stage_cells;
};

// Cells whose positions one staging chunk of the build holds (64 MB).
constexpr int64_t kStageCells = (int64_t)1 << 22;

// Device image of a grid, everything a cast reads: payload (16 B), child
// link (4 B) and stencil record (128 B) per cell, the per-half-cell stencil
// table (32 B) per refined cell (level >= 1), the background tables, and for
// a time-dependent potential 36 B more per cell (dPhi/deta and its stencil
// coefficients); plus a staging area for cell positions during the build.
GridLayout grid_layout(int64_t n, int64_t n_coarse, bool time_dep)
{
    GridLayout L;
    const int64_t n_ref = n - n_coarse;
    L.stage_cells = std::min<int64_t>(n, kStageCells);
    L.off_payload = 0;
    L.off_child = align_up(L.off_payload + (size_t)n * 16, 256);
    L.off_dual = align_up(L.off_child + (size_t)n * 4, 256);
    L.off_leafinfo = align_up(L.off_dual + (size_t)n * 128, 256);
    L.off_table = align_up(L.off_leafinfo + (size_t)n_ref * 32, 256);
    L.off_atable = align_up(L.off_table + (size_t)kTableN * 16, 256);
    L.off_tpay = align_up(L.off_atable + (size_t)kTableN * 16, 256);
    L.off_tdual = align_up(L.off_tpay + (time_dep ? (size_t)n * 4 : 0), 256);
    L.off_stage = align_up(L.off_tdual + (time_dep ? (size_t)n * 32 : 0), 256);
    L.total = align_up(L.off_stage + (size_t)L.stage_cells * 16, 256);
    return L;
}

// Auxiliary tables: the caller's index of every library cell (8 B) and the
// ids of the 8 cells of every stencil record (32 B).
struct AuxLayout {
    size_t off_perm, off_dual_ids, total;
};

AuxLayout aux_layout(int64_t n)
{
    AuxLayout L;
    L.off_perm = 0;
    L.off_dual_ids = align_up((size_t)n * 8, 256);
    L.total = align_up(L.off_dual_ids + (size_t)n * 32, 256);
    return L;
}

int host_threads()
{
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h, 32u));
}

// fn(a, b) over consecutive ranges of [0, n) on up to host_threads()
// threads; each range writes only its own outputs.
template <class F>
void parallel_ranges(int64_t n, F fn, int64_t min_per_thread = (int64_t)1 << 16)
{
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / min_per_thread));
    if (T <= 1) {
        fn((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) {
        const int64_t a = n * t / T, b = n * (t + 1) / T;
        th.emplace_back([=, &fn] { fn(a, b); });
    }
    for (auto& x : th) x.join();
}

// Sort (key, cell) pairs by key: sorted runs on threads, then pairwise merges.
void parallel_sort(std::vector<std::pair<uint64_t, int64_t>>& v)
{
    const int64_t n = (int64_t)v.size();
    int T = 1;
    while (T * 2 <= host_threads() && n / (T * 2) >= ((int64_t)1 << 18)) T *= 2;
    if (T == 1) {
        std::sort(v.begin(), v.end());
        return;
    }
    std::vector<int64_t> cut(T + 1);
    for (int t = 0; t <= T; ++t) cut[t] = n * t / T;
    {
        std::vector<std::thread> th;
        for (int t = 0; t < T; ++t) th.emplace_back([&, t] { std::sort(v.begin() + cut[t], v.begin() + cut[t + 1]); });
        for (auto& x : th) x.join();
    }
    std::vector<std::pair<uint64_t, int64_t>> tmp(n);
    auto* src = &v;
    auto* dst = &tmp;
    for (int w = 1; w < T; w *= 2) {
        std::vector<std::thread> th;
        for (int t = 0; t < T; t += 2 * w) {
            th.emplace_back([&, t] {
                const int64_t a = cut[t], m = cut[std::min(t + w, T)], b = cut[std::min(t + 2 * w, T)];
                std::merge(src->begin() + a, src->begin() + m, src->begin() + m, src->begin() + b, dst->begin() + a);
            });
        }
        for (auto& x : th) x.join();
        std::swap(src, dst);
    }
    if (src != &v) v.swap(tmp);
}

GridDev make_griddev(const mpath_grid* g)
{
    GridDev d;
    std::memset(&d, 0, sizeof d);
    d.payload = g->payload;
    d.child = g->child;
    d.dual = g->dual;
    d.leafinfo = g->leafinfo;
    d.dual_ids = g->dual_ids;
    d.tdual = g->tdual;
    d.h0 = g->box / g->n0;
    d.inv_h0 = g->n0 / g->box;
    d.inv_hf = std::ldexp(d.inv_h0, g->max_level + 1);
    d.eta0 = g->eta0;
    d.phi_max = g->phi_max;
    d.n0 = g->n0;
    d.max_level = g->max_level;
    d.periodic = g->periodic;
    for (int l = 0; l <= kMaxLevels; ++l) d.level_start[l] = g->level_start[l];
    return d;
}

int check_grid_desc(const mpath_grid_desc* d)
{
    if (!d) return fail(MPATH_ERR_INVALID_ARG, "grid desc is NULL");
    if (!(d->box > 0.0) || !std::isfinite(d->box)) return fail(MPATH_ERR_INVALID_ARG, "box must be > 0");
    if (d->n0 < 1 || d->n0 > 1024 || (d->n0 & (d->n0 - 1)))
        return fail(MPATH_ERR_INVALID_ARG, "n0 must be a power of two in [1, 1024]");
    if (d->max_level < 0 || d->max_level >= kMaxLevels)
        return fail(MPATH_ERR_INVALID_ARG, "max_level must be in [0, 10]");
    if ((int64_t)d->n0 << d->max_level > (1 << 20))
        return fail(MPATH_ERR_INVALID_ARG, "n0 * 2^max_level must be <= 2^20");
    if (d->value_dtype != MPATH_F64 && d->value_dtype != MPATH_F32)
        return fail(MPATH_ERR_INVALID_ARG, "value_dtype must be MPATH_F64 or MPATH_F32");
    const int64_t nc = (int64_t)d->n0 * d->n0 * d->n0;
    if (d->n_cells < nc) return fail(MPATH_ERR_NOT_FULL_TREE, "fewer cells than the coarse grid");
    if (d->n_cells > ((int64_t)1 << 31) - 8) return fail(MPATH_ERR_INVALID_ARG, "n_cells must be < 2^31");
    if (!d->level || !d->ijk || !d->phi) return fail(MPATH_ERR_INVALID_ARG, "a cell array is NULL");
    return MPATH_OK;
}

uint64_t morton_key(uint32_t i, uint32_t j, uint32_t k)
{
    // 21 bits per axis
    auto spread = [](uint64_t x) {
        x &= 0x1fffffull;
        x = (x | (x << 32)) & 0x1f00000000ffffull;
        x = (x | (x << 16)) & 0x1f0000ff0000ffull;
        x = (x | (x << 8)) & 0x100f00f00f00f00full;
        x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
        x = (x | (x << 2)) & 0x1249249249249249ull;
        return x;
    };
    return spread(i) | (spread(j) << 1) | (spread(k) << 2);
}

}  // namespace

extern "C" {

const char* mpath_last_error(void) { return g_last_error.c_str(); }

const char* mpath_version(void) { return "mpath 0.1 (gfx950)"; }

const char* mpath_status_string(int s)
{
    switch (s) {
        case MPATH_OK: return "ok";
        case MPATH_ERR_INVALID_ARG: return "invalid argument";
        case MPATH_ERR_NOT_FULL_TREE: return "not a full octree";
        case MPATH_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case MPATH_ERR_DEVICE: return "device error";
        case MPATH_ERR_UNSUPPORTED: return "unsupported option";
        default: return "unknown status";
    }
}

int mpath_grid_workspace_bytes(const mpath_grid_desc* desc, size_t* bytes)
{
    if (!bytes) return fail(MPATH_ERR_INVALID_ARG, "bytes is NULL");
    const int rc = check_grid_desc(desc);
    if (rc) return rc;
    const int64_t nc = (int64_t)desc->n0 * desc->n0 * desc->n0;
    *bytes = grid_layout(desc->n_cells, nc, desc->dphi_deta != nullptr).total;
    return MPATH_OK;
}

int mpath_grid_aux_bytes(const mpath_grid_desc* desc, size_t* bytes)
{
    if (!bytes) return fail(MPATH_ERR_INVALID_ARG, "bytes is NULL");
    const int rc = check_grid_desc(desc);
    if (rc) return rc;
    *bytes = aux_layout(desc->n_cells).total;
    return MPATH_OK;
}

int mpath_grid_build_with_aux(const mpath_grid_desc* d, const mpath_cosmo* cosmo, void* dev_ws, size_t ws_bytes,
                              void* aux_ws, size_t aux_bytes, void* stream, mpath_grid** out)
{
    if (!out) return fail(MPATH_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_grid_desc(d);
    if (rc) return rc;
    if (!cosmo) return fail(MPATH_ERR_INVALID_ARG, "cosmo is NULL");
    const bool stat = cosmo->omega_m == 0.0 && cosmo->omega_l == 0.0;
    if (!stat && !(cosmo->omega_m > 0.0 && cosmo->omega_l >= 0.0 &&
                   std::fabs(cosmo->omega_m + cosmo->omega_l - 1.0) < 1e-12))
        return fail(MPATH_ERR_UNSUPPORTED, "only flat LCDM (omega_m + omega_l = 1) or a static background");
    const bool time_dep = d->dphi_deta != nullptr;
    const int64_t n = d->n_cells;
    const int L = d->max_level;
    const uint32_t n0 = (uint32_t)d->n0;
    const int64_t nc = (int64_t)n0 * n0 * n0;
    const GridLayout lay = grid_layout(n, nc, time_dep);
    if (!dev_ws) return fail(MPATH_ERR_INVALID_ARG, "dev_ws is NULL");
    if (ws_bytes < lay.total) return fail(MPATH_ERR_WORKSPACE_TOO_SMALL, "grid workspace too small");
    const bool aux = aux_ws != nullptr;
    const AuxLayout alay = aux_layout(n);
    if (aux && aux_bytes < alay.total) return fail(MPATH_ERR_WORKSPACE_TOO_SMALL, "grid auxiliary workspace too small");

    // ---- bucket cells by level, keyed by Morton order at their level ----
    for (int64_t c = 0; c < n; ++c)
        if (d->level[c] > L) return fail(MPATH_ERR_INVALID_ARG, "cell " + std::to_string(c) + " level above max_level");
    std::vector<int64_t> per_level(L + 1, 0);
    for (int64_t c = 0; c < n; ++c) ++per_level[d->level[c]];
    if (per_level[0] != nc) return fail(MPATH_ERR_NOT_FULL_TREE, "the coarse level must hold n0^3 cells");
    // keys of the coarse level are 0 .. nc-1 when every coarse cell is
    // present once: they go straight to their slot
    std::vector<int64_t> coarse(nc, -1);
    std::vector<std::vector<std::pair<uint64_t, int64_t>>> lev(L + 1);
    for (int l = 1; l <= L; ++l) lev[l].reserve(per_level[l]);
    for (int64_t c = 0; c < n; ++c) {
        const int l = d->level[c];
        const int64_t m = (int64_t)n0 << l;
        const int32_t* q = d->ijk + 3 * c;
        if (q[0] < 0 || q[1] < 0 || q[2] < 0 || q[0] >= m || q[1] >= m || q[2] >= m)
            return fail(MPATH_ERR_INVALID_ARG, "cell " + std::to_string(c) + " coordinates out of range");
        const uint64_t key = morton_key((uint32_t)q[0], (uint32_t)q[1], (uint32_t)q[2]);
        if (l == 0) {
            if (coarse[key] >= 0) return fail(MPATH_ERR_NOT_FULL_TREE, "missing or repeated coarse cell");
            coarse[key] = c;
        } else {
            lev[l].push_back({key, c});
        }
    }
    for (int l = 1; l <= L; ++l) parallel_sort(lev[l]);
    // refined levels: complete sibling groups whose parent exists
    std::vector<int32_t> child(n, -1);
    std::vector<int64_t> perm(n);
    for (int64_t i = 0; i < nc; ++i) perm[i] = coarse[i];
    int64_t base_prev = 0, base = nc;
    for (int l = 1; l <= L; ++l) {
        const auto& cur = lev[l];
        if (cur.size() % 8) return fail(MPATH_ERR_NOT_FULL_TREE, "a refined cell has 1-7 children (level " + std::to_string(l) + ")");
        // keys of the parent level in library order
        auto parent_key = [&](int64_t j) -> uint64_t {
            return l == 1 ? (uint64_t)j : lev[l - 1][(size_t)j].first;
        };
        const int64_t n_par = l == 1 ? nc : (int64_t)lev[l - 1].size();
        int64_t pj = 0;
        for (size_t g = 0; g < cur.size(); g += 8) {
            const uint64_t pk = cur[g].first >> 3;
            for (int o = 0; o < 8; ++o)
                if (cur[g + o].first != (pk << 3) + (uint64_t)o)
                    return fail(MPATH_ERR_NOT_FULL_TREE, "a refined cell has 1-7 children or a repeated child (level " + std::to_string(l) + ")");
            while (pj < n_par && parent_key(pj) < pk) ++pj;
            if (pj == n_par || parent_key(pj) != pk)
                return fail(MPATH_ERR_NOT_FULL_TREE, "a cell's parent is missing (level " + std::to_string(l) + ")");
            const int64_t id = base + (int64_t)g;
            child[base_prev + pj] = (int32_t)id;
            for (int o = 0; o < 8; ++o) perm[id + o] = cur[g + o].second;
        }
        base_prev = base;
        base += (int64_t)cur.size();
    }
    // ---- caller index of cell (l, i, j, k), -1 if absent (gradients) ----
    auto find_cell = [&](int l, int64_t i, int64_t j, int64_t k) -> int64_t {
        const int64_t m = (int64_t)n0 << l;
        if (d->periodic) {
            i = ((i % m) + m) % m; j = ((j % m) + m) % m; k = ((k % m) + m) % m;
        } else if (i < 0 || j < 0 || k < 0 || i >= m || j >= m || k >= m) {
            return -1;
        }
        const uint64_t key = morton_key((uint32_t)i, (uint32_t)j, (uint32_t)k);
        if (l == 0) return coarse[key];
        const auto& v = lev[l];
        auto it = std::lower_bound(v.begin(), v.end(), std::make_pair(key, (int64_t)-1));
        return (it != v.end() && it->first == key) ? it->second : -1;
    };
    auto phi_at = [&](int64_t c) -> double {
        return d->value_dtype == MPATH_F64 ? ((const double*)d->phi)[c] : (double)((const float*)d->phi)[c];
    };
    // ---- pack (phi, grad) as float32 and the cell positions in library order ----
    std::vector<float4> payload(n);
    std::vector<int4> cellpos(n);
    std::vector<float> tpay(time_dep ? n : 0);
    parallel_ranges(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            const int64_t c = perm[i];
            const int l = d->level[c];
            const int32_t* q = d->ijk + 3 * c;
            if (time_dep)
                tpay[i] = d->value_dtype == MPATH_F64 ? (float)((const double*)d->dphi_deta)[c]
                                                      : ((const float*)d->dphi_deta)[c];
            cellpos[i] = make_int4(q[0], q[1], q[2], l);
            float gr[3];
            if (d->grad) {
                for (int a = 0; a < 3; ++a)
                    gr[a] = d->value_dtype == MPATH_F64 ? (float)((const double*)d->grad)[3 * c + a]
                                                        : ((const float*)d->grad)[3 * c + a];
            } else {
                // second-order central differences of phi between the two
                // neighbours at the cell's own level; where one of them does
                // not exist (the edge of a refined region or of a
                // non-periodic box), the one-sided difference with the other
                const double h = d->box / (double)((int64_t)n0 << l);
                const double p0 = phi_at(c);
                for (int a = 0; a < 3; ++a) {
                    const int e0 = a == 0, e1 = a == 1, e2 = a == 2;
                    const int64_t cp = find_cell(l, (int64_t)q[0] + e0, (int64_t)q[1] + e1, (int64_t)q[2] + e2);
                    const int64_t cm = find_cell(l, (int64_t)q[0] - e0, (int64_t)q[1] - e1, (int64_t)q[2] - e2);
                    double g = 0.0;
                    if (cp >= 0 && cm >= 0) g = (phi_at(cp) - phi_at(cm)) / (2.0 * h);
                    else if (cp >= 0) g = (phi_at(cp) - p0) / h;
                    else if (cm >= 0) g = (p0 - phi_at(cm)) / h;
                    gr[a] = (float)g;
                }
            }
            payload[i] = make_float4((float)phi_at(c), gr[0], gr[1], gr[2]);
        }
    });
    lev.clear();
    lev.shrink_to_fit();
    std::vector<int64_t>().swap(coarse);
    // ---- background table of a'/a ----
    mpath_grid* G = new mpath_grid();
    G->phi_max = -INFINITY;
    for (int64_t i = 0; i < n; ++i) G->phi_max = std::max(G->phi_max, payload[i].x);
    G->bg.init(cosmo->omega_m, cosmo->omega_l);
    G->eta0 = G->bg.is_static ? 0.0 : G->bg.eta0();
    std::vector<double2> table(kTableN, make_double2(0.0, 0.0));
    std::vector<double2> atable(kTableN, make_double2(1.0, 0.0));
    if (!G->bg.is_static) {
        const double lo = G->bg.eta_of_a(1.0 / (1.0 + kZMaxTable)) - 50.0;
        const double hi = G->eta0 + 50.0;
        G->table_eta_lo = lo;
        G->table_deta = (hi - lo) / (kTableN - 1);
        for (int i = 0; i < kTableN; ++i) {
            const double a = G->bg.a_of_eta(lo + i * G->table_deta);
            double H, dH;
            G->bg.hubble(a, H, dH);
            table[i] = make_double2(H, dH);
            atable[i] = make_double2(a, a * H);
        }
    }
    // ---- upload ----
    G->n_cells = n;
    G->n0 = d->n0;
    G->max_level = L;
    G->periodic = d->periodic ? 1 : 0;
    G->box = d->box;
    int64_t start = 0;
    for (int l = 0; l <= kMaxLevels; ++l) {
        G->level_start[l] = (int32_t)start;
        if (l <= L) {
            G->cells_per_level[l] = per_level[l];
            start += per_level[l];
        }
    }
    G->ws = (char*)dev_ws;
    G->payload = (float4*)(G->ws + lay.off_payload);
    G->child = (int32_t*)(G->ws + lay.off_child);
    G->dual = (float4*)(G->ws + lay.off_dual);
    G->leafinfo = (int32_t*)(G->ws + lay.off_leafinfo);
    G->table = (double2*)(G->ws + lay.off_table);
    G->atable = (double2*)(G->ws + lay.off_atable);
    if (time_dep) {
        G->tpay = (float*)(G->ws + lay.off_tpay);
        G->tdual = (float4*)(G->ws + lay.off_tdual);
    }
    if (aux) {
        G->perm = (int64_t*)((char*)aux_ws + alay.off_perm);
        G->dual_ids = (int32_t*)((char*)aux_ws + alay.off_dual_ids);
    }
    int4* stage = (int4*)(G->ws + lay.off_stage);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    const GridDev gd = make_griddev(G);
    if ((e = hipMemcpyAsync(G->payload, payload.data(), (size_t)n * 16, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(G->child, child.data(), (size_t)n * 4, hipMemcpyHostToDevice, s)) ||
        (aux && (e = hipMemcpyAsync(G->perm, perm.data(), (size_t)n * 8, hipMemcpyHostToDevice, s))) ||
        (e = hipMemcpyAsync(G->table, table.data(), (size_t)kTableN * 16, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(G->atable, atable.data(), (size_t)kTableN * 16, hipMemcpyHostToDevice, s)) ||
        (time_dep && (e = hipMemcpyAsync(G->tpay, tpay.data(), (size_t)n * 4, hipMemcpyHostToDevice, s)))) {
        delete G;
        return hip_fail_drain(e, s, "grid upload");
    }
    // derived tables, chunk by chunk through the staging area (stream order
    // keeps each chunk's positions until its kernels have read them)
    for (int64_t c0 = 0; c0 < n && !e; c0 += lay.stage_cells) {
        const int64_t m = std::min(lay.stage_cells, n - c0);
        const int64_t r0 = std::max(c0, nc);      // first refined cell of the chunk
        (void)((e = hipMemcpyAsync(stage, cellpos.data() + c0, (size_t)m * 16, hipMemcpyHostToDevice, s)) ||
               (e = launch_build_dual(gd, stage, c0, m, G->dual, s)) ||
               (r0 < c0 + m && (e = launch_build_leafinfo(gd, stage + (r0 - c0), r0, c0 + m - r0, G->leafinfo, s))) ||
               (aux && (e = launch_build_dual_ids(gd, stage, c0, m, G->dual_ids, s))) ||
               (time_dep && (e = launch_build_tdual(gd, stage, c0, m, G->tpay, G->tdual, s))));
    }
    if (e || (e = hipStreamSynchronize(s))) {
        delete G;
        return hip_fail_drain(e, s, "grid build");
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&G->num_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        G->num_cus = 0;
    *out = G;
    return MPATH_OK;
}

int mpath_grid_build(const mpath_grid_desc* d, const mpath_cosmo* cosmo, void* dev_ws, size_t ws_bytes,
                     void* stream, mpath_grid** out)
{
    return mpath_grid_build_with_aux(d, cosmo, dev_ws, ws_bytes, nullptr, 0, stream, out);
}

int mpath_double_layer(int64_t n, const double* phi1, const double* phi2, const double* a1, const double* a2,
                       const mpath_cosmo* cosmo, double* dphi_deta)
{
    if (n < 0) return fail(MPATH_ERR_INVALID_ARG, "n must be >= 0");
    if (!cosmo) return fail(MPATH_ERR_INVALID_ARG, "cosmo is NULL");
    if (n > 0 && (!phi1 || !phi2 || !a1 || !a2 || !dphi_deta)) return fail(MPATH_ERR_INVALID_ARG, "an array is NULL");
    if (!(cosmo->omega_m > 0.0 && cosmo->omega_l >= 0.0 && std::fabs(cosmo->omega_m + cosmo->omega_l - 1.0) < 1e-12))
        return fail(MPATH_ERR_UNSUPPORTED, "the double layer needs an expanding flat LCDM background");
    Background bg;
    bg.init(cosmo->omega_m, cosmo->omega_l);
    for (int64_t i = 0; i < n; ++i) {
        if (!(a1[i] > 0.0 && a2[i] > 0.0 && a1[i] != a2[i]) || !std::isfinite(a1[i]) || !std::isfinite(a2[i]))
            return fail(MPATH_ERR_INVALID_ARG, "cell " + std::to_string(i) + ": layers need 0 < a1 != a2");
        // dPhi/da from the two layers, times da/deta = a (a'/a) at the midpoint
        const double am = 0.5 * (a1[i] + a2[i]);
        double H, dH;
        bg.hubble(am, H, dH);
        dphi_deta[i] = (phi2[i] - phi1[i]) / (a2[i] - a1[i]) * (am * H);
    }
    return MPATH_OK;
}

int mpath_healpix_dirs(int32_t nside, int64_t pix_first, int64_t count, double* dirs, void* stream)
{
    if (nside < 1 || nside > 8192) return fail(MPATH_ERR_INVALID_ARG, "nside must be in [1, 8192]");
    if (pix_first < 0 || count < 0 || pix_first + count > 12ll * nside * nside)
        return fail(MPATH_ERR_INVALID_ARG, "pixel range outside the sky");
    if (count > 0 && !dirs) return fail(MPATH_ERR_INVALID_ARG, "dirs is NULL");
    const hipError_t e = launch_healpix_dirs(nside, pix_first, count, dirs, (hipStream_t)stream);
    return e ? hip_fail(e, "healpix directions launch") : MPATH_OK;
}

int mpath_grid_free(mpath_grid* grid)
{
    delete grid;
    return MPATH_OK;
}

int mpath_grid_get_info(const mpath_grid* g, mpath_grid_info* info)
{
    if (!g || !info) return fail(MPATH_ERR_INVALID_ARG, "NULL argument");
    std::memset(info, 0, sizeof *info);
    info->n_cells = g->n_cells;
    info->n0 = g->n0;
    info->max_level = g->max_level;
    info->periodic = g->periodic;
    info->box = g->box;
    info->eta0 = g->eta0;
    for (int l = 0; l < 16; ++l) info->cells_per_level[l] = g->cells_per_level[l];
    info->payload = (float*)g->payload;
    info->perm = g->perm;
    return MPATH_OK;
}

int mpath_grid_set_values(mpath_grid* g, const float* values, void* stream)
{
    if (!g || !values) return fail(MPATH_ERR_INVALID_ARG, "NULL argument");
    if (!g->perm) return fail(MPATH_ERR_UNSUPPORTED, "set_values needs the grid's auxiliary tables (mpath_grid_build_with_aux)");
    g->phi_max = INFINITY;   // the new values stay on the device: no bound
    hipError_t e = launch_permute_values(g->payload, g->perm, (const float4*)values, g->n_cells,
                                         (hipStream_t)stream);
    if (!e) e = launch_rebuild_dual(make_griddev(g), g->dual_ids, g->dual, g->n_cells, (hipStream_t)stream);
    return e ? hip_fail(e, "set_values launch") : MPATH_OK;
}

}  // extern "C"

namespace {

struct CastLayout {
    size_t off_obs, off_surf, off_queue, off_ends, off_dirs, off_ckpt, total;
    int64_t ckpt_slots;
};

// Cast workspace: observer table, queue counter, per-ray end states, initial
// directions and, for a checkpointed cast, ckpt_slots states per ray.
CastLayout cast_layout(int64_t n_obs, int64_t n_rays, int64_t ckpt_slots, int n_surf = 0)
{
    CastLayout L;
    L.off_obs = 0;
    L.off_surf = align_up((size_t)n_obs * sizeof(ObsDev), 256);
    L.off_queue = align_up(L.off_surf + (size_t)n_obs * n_surf * sizeof(double2), 256);
    L.off_ends = align_up(L.off_queue + 256, 256);
    L.off_dirs = align_up(L.off_ends + (size_t)(n_surf + 1) * n_rays * sizeof(RayEnd), 256);
    L.off_ckpt = align_up(L.off_dirs + (size_t)n_rays * 24, 256);
    L.ckpt_slots = ckpt_slots;
    L.total = align_up(L.off_ckpt + (size_t)ckpt_slots * (size_t)n_rays * sizeof(GeoState), 256);
    return L;
}

int check_cast_desc(const mpath_grid* g, const mpath_cast_desc* d, int64_t* n_rays)
{
    if (!g) return fail(MPATH_ERR_INVALID_ARG, "grid is NULL");
    if (!d) return fail(MPATH_ERR_INVALID_ARG, "cast desc is NULL");
    if (d->n_obs < 1) return fail(MPATH_ERR_INVALID_ARG, "n_obs must be >= 1");
    if (!d->obs_pos || !d->stop_value) return fail(MPATH_ERR_INVALID_ARG, "obs_pos or stop_value is NULL");
    if (d->nside < 1 || d->nside > 8192) return fail(MPATH_ERR_INVALID_ARG, "nside must be in [1, 8192]");
    if (!d->dirs && (d->pix_first == nullptr) != (d->pix_count == nullptr))
        return fail(MPATH_ERR_INVALID_ARG, "pix_first and pix_count must both be given or both NULL");
    if (d->order < 0 || d->order > 2) return fail(MPATH_ERR_INVALID_ARG, "order must be 0 (NGP), 1 (CIC) or 2 (TSC)");
    if (d->order != 1 && d->checkpoint_every > 0)
        return fail(MPATH_ERR_UNSUPPORTED, "checkpoints (the adjoint) need order = 1 (CIC)");
    if (d->n_surfaces < 0 || d->n_surfaces > 64) return fail(MPATH_ERR_INVALID_ARG, "n_surfaces must be in [0, 64]");
    if (d->n_surfaces > 0) {
        if (!d->surface_stops) return fail(MPATH_ERR_INVALID_ARG, "surface_stops is NULL");
        if (d->checkpoint_every > 0 || d->order != 1)
            return fail(MPATH_ERR_UNSUPPORTED, "several stop surfaces need order = 1 and no checkpoints");
    }
    if (d->steps_per_cell < 1) return fail(MPATH_ERR_INVALID_ARG, "steps_per_cell must be >= 1");
    if (d->max_steps < 1) return fail(MPATH_ERR_INVALID_ARG, "max_steps must be >= 1");
    if (d->stop_kind != MPATH_STOP_REDSHIFT && d->stop_kind != MPATH_STOP_CHI)
        return fail(MPATH_ERR_INVALID_ARG, "unknown stop_kind");
    if (d->stop_kind == MPATH_STOP_REDSHIFT && g->bg.is_static)
        return fail(MPATH_ERR_INVALID_ARG, "a static background has no redshift stop");
    if (d->schedule < 0 || d->schedule > 2) return fail(MPATH_ERR_INVALID_ARG, "unknown schedule");
    if (d->block_size && d->block_size != 256)
        return fail(MPATH_ERR_UNSUPPORTED, "the integration kernels run 256 threads per block (block_size 0 or 256)");
    if (d->checkpoint_every < 0) return fail(MPATH_ERR_INVALID_ARG, "checkpoint_every must be >= 0");
    if (d->stop_surface < MPATH_SURFACE_ETA || d->stop_surface > MPATH_SURFACE_Z)
        return fail(MPATH_ERR_INVALID_ARG, "unknown stop_surface");
    if (d->stop_surface != MPATH_SURFACE_ETA &&
        (d->order != 1 || d->checkpoint_every > 0 || d->n_surfaces > 0 || g->tdual))
        return fail(MPATH_ERR_UNSUPPORTED,
                    "iso-chi, iso-lambda and iso-z stops take order 1, a static potential, one surface and no "
                    "checkpoints");
    if (d->stop_surface == MPATH_SURFACE_Z && g->bg.is_static)
        return fail(MPATH_ERR_UNSUPPORTED, "a static background has no redshift surface");
    if (d->dphidl != MPATH_DPHIDL_CHAIN && d->dphidl != MPATH_DPHIDL_DIFF)
        return fail(MPATH_ERR_INVALID_ARG, "unknown dphidl");
    if (d->dphidl == MPATH_DPHIDL_DIFF &&
        (d->order != 1 || d->checkpoint_every > 0 || d->n_surfaces > 0 || g->tdual ||
         d->stop_surface != MPATH_SURFACE_ETA))
        return fail(MPATH_ERR_UNSUPPORTED,
                    "the step-difference dPhi/dlambda takes order 1, a static grid, the iso-eta stop, one surface "
                    "and no checkpoints");
    const int64_t npix = 12ll * d->nside * d->nside;
    int64_t total = 0;
    for (int j = 0; j < d->n_obs; ++j) {
        const int64_t f = (d->pix_first && !d->dirs) ? d->pix_first[j] : 0;
        const int64_t c = d->pix_count ? d->pix_count[j] : npix;
        if (d->dirs ? c < 0 : (f < 0 || c < 0 || f + c > npix))
            return fail(MPATH_ERR_INVALID_ARG, d->dirs ? "negative ray count" : "pixel range outside the sky");
        total += c;
    }
    *n_rays = total;
    return MPATH_OK;
}

// Observer table: stop surface per observer (conformal time eta_s, a_s, z0)
// and the first ray of each observer.
int make_obs_table(const mpath_grid* g, const mpath_cast_desc* d, std::vector<ObsDev>& obs)
{
    obs.assign(d->n_obs, ObsDev{});
    const double amin = 1.0 / (1.0 + kZMaxTable);
    const int Lm = g->max_level;
    const double h0 = g->box / g->n0;
    int64_t first = 0;
    for (int j = 0; j < d->n_obs; ++j) {
        ObsDev& o = obs[j];
        for (int i = 0; i < 3; ++i) {
            o.x[i] = d->obs_pos[3 * j + i];
            if (!std::isfinite(o.x[i])) return fail(MPATH_ERR_INVALID_ARG, "observer position not finite");
        }
        const double v = d->stop_value[j];
        if (d->stop_kind == MPATH_STOP_REDSHIFT) {
            if (!(v >= 0.0)) return fail(MPATH_ERR_INVALID_ARG, "z_src must be >= 0");
            if (v > kZMaxTable) return fail(MPATH_ERR_UNSUPPORTED, "z_src above 20 is outside the background table");
            o.a_s = 1.0 / (1.0 + v);
            o.eta_s = g->bg.eta_of_a(o.a_s);
        } else {
            if (!(v >= 0.0)) return fail(MPATH_ERR_INVALID_ARG, "comoving distance must be >= 0");
            o.eta_s = g->eta0 - v;
            if (!g->bg.is_static && o.eta_s < g->bg.eta_of_a(amin))
                return fail(MPATH_ERR_UNSUPPORTED, "stop surface beyond z = 20 is outside the background table");
            o.a_s = g->bg.a_of_eta(o.eta_s);
        }
        o.z0 = 1.0 / o.a_s - 1.0;
        // the stop surface's parameter at the FLRW photon's stop
        switch (d->stop_surface) {
            case MPATH_SURFACE_CHI: o.p_s = g->eta0 - o.eta_s; break;
            case MPATH_SURFACE_LAMBDA: o.p_s = g->bg.is_static ? g->eta0 - o.eta_s : g->bg.lambda_of_a(o.a_s); break;
            case MPATH_SURFACE_Z: o.p_s = -std::log(o.a_s); break;
            default: o.p_s = o.eta_s; break;
        }
        o.pix_first = d->pix_first ? d->pix_first[j] : 0;
        o.count = d->pix_count ? d->pix_count[j] : 12ll * d->nside * d->nside;
        o.ray_first = first;
        first += o.count;
        // integer cell coordinates at level max_level + 1 must stay inside int32
        const double reach = (std::fabs(o.x[0]) + std::fabs(o.x[1]) + std::fabs(o.x[2]) +
                              1.01 * (g->eta0 - o.eta_s) + 4.0 * h0) / h0 * std::ldexp(1.0, Lm + 1);
        if (reach > 1.0e9) return fail(MPATH_ERR_UNSUPPORTED, "ray path too long for 32-bit cell coordinates");
    }
    return MPATH_OK;
}

// Checkpoint slots per ray: every step advances eta by at least the comoving
// step length ds >= ds_min (|k0| grows along a backward path), so a ray
// takes at most (eta_0 - eta_s) / ds_min + 1 steps; 2 % and 16 steps of
// margin, capped by max_steps.
int64_t checkpoint_slots(const mpath_grid* g, const mpath_cast_desc* d, const std::vector<ObsDev>& obs)
{
    if (d->checkpoint_every <= 0) return 0;
    double chi = 0.0;
    for (const ObsDev& o : obs) chi = std::max(chi, g->eta0 - o.eta_s);
    const double ds_min = g->box / g->n0 / std::ldexp(1.0, d->adaptive ? g->max_level : 0) / d->steps_per_cell;
    const double est = std::floor(1.02 * chi / ds_min) + 16.0;
    const int64_t steps = (int64_t)std::min((double)d->max_steps, est);
    return (steps + d->checkpoint_every - 1) / d->checkpoint_every;
}

CastArgs make_cast_args(const mpath_grid* g, const mpath_cast_desc* d, const CastLayout& lay, char* ws,
                        int64_t n_rays)
{
    CastArgs a;
    std::memset(&a, 0, sizeof a);
    a.grid = make_griddev(g);
    a.cosmo.table = g->table;
    a.cosmo.atable = g->atable;
    a.surface = d->stop_surface;
    a.cosmo.eta_lo = g->table_eta_lo;
    a.cosmo.deta = g->table_deta;
    a.cosmo.inv_deta = g->table_deta > 0 ? 1.0 / g->table_deta : 0.0;
    a.cosmo.n = kTableN;
    a.cosmo.is_static = g->bg.is_static ? 1 : 0;
    a.cosmo_eta0 = g->eta0;
    a.obs = (const ObsDev*)(ws + lay.off_obs);
    a.n_obs = d->n_obs;
    a.nside = d->nside;
    a.steps_per_cell = d->steps_per_cell;
    a.adaptive = d->adaptive ? 1 : 0;
    for (int l = 0; l <= kMaxLevels; ++l)
        a.ds_level[l] = (g->box / g->n0) / (double)(1 << (a.adaptive ? l : 0)) / (double)d->steps_per_cell;
    a.max_steps = std::min<int64_t>(d->max_steps, INT32_MAX);   // steps are counted in 32 bits
    a.n_rays = n_rays;
    a.queue = (unsigned long long*)(ws + lay.off_queue);
    a.ends = (RayEnd*)(ws + lay.off_ends);
    a.dirs = (double*)(ws + lay.off_dirs);
    a.batch = d->batch > 0 ? d->batch : 32;
    if (d->checkpoint_every > 0) {
        a.ckpt = (GeoState*)(ws + lay.off_ckpt);
        a.ckpt_every = d->checkpoint_every;
        a.ckpt_slots = (int32_t)lay.ckpt_slots;
        a.max_steps = std::min<int64_t>(a.max_steps, lay.ckpt_slots * (int64_t)d->checkpoint_every);
    }
    return a;
}

int cast_plan(const mpath_grid* g, const mpath_cast_desc* d, int64_t* n_rays, std::vector<ObsDev>& obs,
              CastLayout* lay)
{
    int rc = check_cast_desc(g, d, n_rays);
    if (rc) return rc;
    rc = make_obs_table(g, d, obs);
    if (rc) return rc;
    const int64_t slots = checkpoint_slots(g, d, obs);
    if (slots > (int64_t)1 << 30) return fail(MPATH_ERR_INVALID_ARG, "too many checkpoints: lower max_steps");
    *lay = cast_layout(d->n_obs, *n_rays, slots, d->n_surfaces);
    return MPATH_OK;
}

// (eta_s, a_s) of the intermediate stop surfaces, [n_obs][n_surfaces],
// nearest first and each nearer than the observer's own stop.
int make_surface_table(const mpath_grid* g, const mpath_cast_desc* d, const std::vector<ObsDev>& obs,
                       std::vector<double2>& surf)
{
    const int n = d->n_surfaces;
    surf.assign((size_t)d->n_obs * n, make_double2(0.0, 0.0));
    for (int j = 0; j < d->n_obs; ++j) {
        double prev = g->eta0;
        for (int k = 0; k < n; ++k) {
            const double v = d->surface_stops[(size_t)j * n + k];
            double eta_s, a_s;
            if (d->stop_kind == MPATH_STOP_REDSHIFT) {
                if (!(v > 0.0)) return fail(MPATH_ERR_INVALID_ARG, "surface redshifts must be > 0");
                a_s = 1.0 / (1.0 + v);
                eta_s = g->bg.eta_of_a(a_s);
            } else {
                if (!(v > 0.0)) return fail(MPATH_ERR_INVALID_ARG, "surface distances must be > 0");
                eta_s = g->eta0 - v;
                a_s = g->bg.a_of_eta(eta_s);
            }
            if (!(eta_s < prev) || !(eta_s > obs[j].eta_s))
                return fail(MPATH_ERR_INVALID_ARG,
                            "surfaces must increase in distance and lie nearer than the observer's stop");
            surf[(size_t)j * n + k] = make_double2(eta_s, a_s);
            prev = eta_s;
        }
    }
    return MPATH_OK;
}

// Adjoint workspace: one segment of step states per ray and the cell
// cotangents in library order.
struct AdjointLayout {
    size_t off_tape, off_grad, total;
};

AdjointLayout adjoint_layout(const mpath_grid* g, const mpath_cast_desc* d, int64_t n_rays)
{
    AdjointLayout L;
    L.off_tape = 0;
    L.off_grad = align_up((size_t)d->checkpoint_every * (size_t)n_rays * sizeof(GeoState), 256);
    L.total = align_up(L.off_grad + (size_t)grad_accumulator_floats(g->n_cells) * 4, 256);
    return L;
}

}  // namespace

extern "C" {

int mpath_cast_count_rays(const mpath_cast_desc* d, int64_t* n_rays)
{
    if (!d || !n_rays) return fail(MPATH_ERR_INVALID_ARG, "NULL argument");
    if (d->n_obs < 1 || d->nside < 1) return fail(MPATH_ERR_INVALID_ARG, "bad n_obs or nside");
    const int64_t npix = 12ll * d->nside * d->nside;
    int64_t t = 0;
    for (int j = 0; j < d->n_obs; ++j) t += d->pix_count ? d->pix_count[j] : npix;
    *n_rays = t;
    return MPATH_OK;
}

int mpath_cast_workspace_bytes(const mpath_grid* g, const mpath_cast_desc* d, size_t* bytes)
{
    if (!bytes) return fail(MPATH_ERR_INVALID_ARG, "bytes is NULL");
    int64_t n_rays;
    std::vector<ObsDev> obs;
    CastLayout lay;
    const int rc = cast_plan(g, d, &n_rays, obs, &lay);
    if (rc) return rc;
    *bytes = lay.total;
    return MPATH_OK;
}

}  // extern "C"

namespace {

// Outputs of the forward-mode derivative (mpath_cast_jacobian).
struct TangentOut {
    TanEnd* ends;
    float* jac;
    float* dz_dtheta;
};

// mpath_cast, or with inf set the cast that also integrates the
// infinitesimal-beam distortion matrix into inf_A (static schedule), or with
// tg set the cast that carries the two tangents (static schedule).
int cast_impl(const mpath_grid* g, const mpath_cast_desc* d, mpath_observables* out, void* dev_ws,
              size_t ws_bytes, void* stream, bool inf, float* inf_A, const double2* ray_stop = nullptr,
              const TangentOut* tg = nullptr)
{
    int64_t n_rays;
    std::vector<ObsDev> obs;
    CastLayout lay;
    int rc = cast_plan(g, d, &n_rays, obs, &lay);
    if (rc) return rc;
    if (!out) return fail(MPATH_ERR_INVALID_ARG, "out is NULL");
    if (!dev_ws) return fail(MPATH_ERR_INVALID_ARG, "dev_ws is NULL");
    if (ws_bytes < lay.total) return fail(MPATH_ERR_WORKSPACE_TOO_SMALL, "cast workspace too small");

    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)dev_ws;
    hipError_t e = hipMemcpyAsync(ws + lay.off_obs, obs.data(), obs.size() * sizeof(ObsDev),
                                  hipMemcpyHostToDevice, s);
    if (!e) e = hipStreamSynchronize(s);   // the host table is released on return
    if (e) return hip_fail(e, "observer table upload");

    CastArgs a = make_cast_args(g, d, lay, ws, n_rays);
    a.ray_stop = ray_stop;
    a.out.beta = out->beta;
    a.out.alpha = out->alpha;
    a.out.z5 = out->z5;
    a.out.z0 = out->z0;
    a.out.phi_src = out->phi_src;
    a.out.n_steps = out->n_steps;
    a.out.status = out->status;
    a.out.hash = out->hash;
    a.out.chi = out->chi;
    a.out.z1 = out->z1;
    a.out.z4 = out->z4;
    a.out.isw = out->isw;
    if (g->tdual && (inf || d->order != 1 || d->checkpoint_every > 0 || d->n_surfaces > 0))
        return fail(MPATH_ERR_UNSUPPORTED,
                    "a time-dependent potential is cast with order 1, one stop surface and no checkpoints");
    if (d->stop_surface != MPATH_SURFACE_ETA && (inf || ray_stop))
        return fail(MPATH_ERR_UNSUPPORTED, "the infinitesimal beam and the finder stop on iso-eta surfaces");
    if (d->dphidl != MPATH_DPHIDL_CHAIN && (inf || ray_stop))
        return fail(MPATH_ERR_UNSUPPORTED, "the infinitesimal beam and the finder use the chain-rule dPhi/dlambda");

    if (d->dirs) {
        e = n_rays ? hipMemcpyAsync(a.dirs, d->dirs, (size_t)n_rays * 24, hipMemcpyDeviceToDevice, s) : hipSuccess;
        if (e) return hip_fail(e, "ray directions copy");
    } else {
        e = launch_ray_dirs(a, s);
        if (e) return hip_fail(e, "ray directions launch");
    }
    if (d->n_surfaces > 0) {
        if (inf || ray_stop) return fail(MPATH_ERR_UNSUPPORTED, "several stop surfaces in a plain cast only");
        std::vector<double2> surf;
        rc = make_surface_table(g, d, obs, surf);
        if (rc) return rc;
        e = hipMemcpyAsync(ws + lay.off_surf, surf.data(), surf.size() * sizeof(double2), hipMemcpyHostToDevice, s);
        if (!e) e = hipStreamSynchronize(s);
        if (!e) e = launch_cast_surfaces(a, (const double2*)(ws + lay.off_surf), d->n_surfaces, s);
        // the observables of each surface block
        for (int k = 0; !e && k <= d->n_surfaces; ++k) {
            CastArgs ak = a;
            const int64_t o = (int64_t)k * n_rays;
            ak.ends = a.ends + o;
            if (ak.out.beta) ak.out.beta += 2 * o;
            if (ak.out.alpha) ak.out.alpha += 2 * o;
            if (ak.out.chi) ak.out.chi += o;
            e = launch_observables(ak, s);
        }
        if (e) return hip_fail(e, "cast launch");
        return MPATH_OK;
    }
    if (tg) {
        e = launch_cast_tangent(a, tg->ends, s);
        if (!e) e = launch_observables(a, s);
        if (!e) e = launch_tangent_observables(a, tg->ends, tg->jac, tg->dz_dtheta, s);
        return e ? hip_fail(e, "tangent cast launch") : MPATH_OK;
    }
    if (inf) {
        e = launch_cast_infbeam(a, inf_A, s);
    } else if (d->stop_surface != MPATH_SURFACE_ETA) {
        e = launch_cast_stop(a, s);
    } else if (d->dphidl != MPATH_DPHIDL_CHAIN) {
        e = launch_cast_diff(a, s);
    } else if (d->order != 1) {
        e = launch_cast_order(a, d->order, s);
    } else if (d->checkpoint_every > 0) {
        e = launch_cast_checkpointed(a, s);
    } else {
        int sched = d->schedule;
        if (sched == MPATH_SCHED_AUTO) sched = d->n_obs > 1 ? MPATH_SCHED_PERSISTENT : MPATH_SCHED_STATIC;
        const int block = d->block_size ? d->block_size : 256;
        if (sched == MPATH_SCHED_STATIC) {
            e = launch_cast_static(a, block, s);
        } else {
            int wpc = d->waves_per_cu;
            if (wpc <= 0)
                wpc = cast_occupancy_blocks_per_cu(block, g->max_level > 0, g->tdual != nullptr) * (block / 64);
            if (wpc <= 0) wpc = 8;
            const int cus = g->num_cus > 0 ? g->num_cus : 256;
            const int blocks = std::max(1, cus * wpc / (block / 64));
            e = launch_cast_persistent(a, block, blocks, s);
        }
    }
    if (!e) e = launch_observables(a, s);
    if (e) return hip_fail(e, "cast launch");
    return MPATH_OK;
}

}  // namespace

// Workspace of mpath_cast_noalloc: one static buffer per GPU, which the
// loader places in each device's memory with the code object.  Host code
// never uses its name as a device address: the address comes from
// hipGetSymbolAddress, once per device, at the first call there.
static __device__ __align__(256) unsigned char scratch[MPATH_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

int scratch_for_current_device(void** ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MPATH_ERR_UNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e || !p) return hip_fail(e ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return MPATH_OK;
}

}  // namespace

extern "C" {

int mpath_cast(const mpath_grid* g, const mpath_cast_desc* d, mpath_observables* out, void* dev_ws,
               size_t ws_bytes, void* stream)
{
    return cast_impl(g, d, out, dev_ws, ws_bytes, stream, false, nullptr);
}

int mpath_cast_noalloc(const mpath_grid* g, const mpath_cast_desc* d, mpath_observables* out, void* stream)
{
    int64_t n_rays;
    std::vector<ObsDev> obs;
    CastLayout lay;
    int rc = cast_plan(g, d, &n_rays, obs, &lay);
    if (rc) return rc;
    if (d->checkpoint_every != 0)
        return fail(MPATH_ERR_UNSUPPORTED, "mpath_cast_noalloc stores no checkpoints (checkpoint_every 0)");
    if (lay.total > (size_t)MPATH_NOALLOC_SCRATCH_BYTES)
        return fail(MPATH_ERR_WORKSPACE_TOO_SMALL,
                    "the cast needs " + std::to_string(lay.total) + " bytes of workspace, above the " +
                        std::to_string((size_t)MPATH_NOALLOC_SCRATCH_BYTES) + " of the static buffer");
    void* ws = nullptr;
    rc = scratch_for_current_device(&ws);
    if (rc) return rc;
    return cast_impl(g, d, out, ws, (size_t)MPATH_NOALLOC_SCRATCH_BYTES, stream, false, nullptr);
}

int mpath_born_beam(const mpath_grid* g, const mpath_cast_desc* d, float* A, int32_t* status, void* dev_ws,
                    size_t ws_bytes, void* stream)
{
    int64_t n_rays;
    std::vector<ObsDev> obs;
    CastLayout lay;
    int rc = cast_plan(g, d, &n_rays, obs, &lay);
    if (rc) return rc;
    if (d->checkpoint_every != 0) return fail(MPATH_ERR_INVALID_ARG, "the Born beam takes checkpoint_every 0");
    if (g->tdual) return fail(MPATH_ERR_UNSUPPORTED, "the Born beam of a time-dependent potential is not implemented");
    if (d->stop_surface != MPATH_SURFACE_ETA || d->dphidl != MPATH_DPHIDL_CHAIN)
        return fail(MPATH_ERR_UNSUPPORTED, "the Born beam stops on iso-eta surfaces (chain-rule dPhi/dlambda)");
    if (d->n_surfaces) return fail(MPATH_ERR_UNSUPPORTED, "the Born beam takes one stop surface");
    if (d->order != 1) return fail(MPATH_ERR_UNSUPPORTED, "the Born beam is implemented for order = 1 (CIC)");
    if (n_rays > 0 && !A) return fail(MPATH_ERR_INVALID_ARG, "A is NULL");
    if (!dev_ws) return fail(MPATH_ERR_INVALID_ARG, "dev_ws is NULL");
    if (ws_bytes < lay.total) return fail(MPATH_ERR_WORKSPACE_TOO_SMALL, "cast workspace too small");
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)dev_ws;
    hipError_t e = hipMemcpyAsync(ws + lay.off_obs, obs.data(), obs.size() * sizeof(ObsDev), hipMemcpyHostToDevice, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return hip_fail(e, "observer table upload");
    CastArgs a = make_cast_args(g, d, lay, ws, n_rays);
    if (d->dirs)
        e = n_rays ? hipMemcpyAsync(a.dirs, d->dirs, (size_t)n_rays * 24, hipMemcpyDeviceToDevice, s) : hipSuccess;
    else
        e = launch_ray_dirs(a, s);
    if (!e) e = launch_born_beam(a, A, status, s);
    return e ? hip_fail(e, "Born beam launch") : MPATH_OK;
}

int mpath_cast_jacobian_workspace_bytes(const mpath_grid* g, const mpath_cast_desc* d, size_t* bytes)
{
    if (!bytes) return fail(MPATH_ERR_INVALID_ARG, "bytes is NULL");
    int64_t n_rays;
    std::vector<ObsDev> obs;
    CastLayout lay;
    const int rc = cast_plan(g, d, &n_rays, obs, &lay);
    if (rc) return rc;
    *bytes = align_up(lay.total, 256) + (size_t)n_rays * sizeof(TanEnd);
    return MPATH_OK;
}

int mpath_cast_jacobian(const mpath_grid* g, const mpath_cast_desc* d, mpath_observables* out, float* jac,
                        float* dz_dtheta, void* dev_ws, size_t ws_bytes, void* stream)
{
    int64_t n_rays;
    std::vector<ObsDev> obs;
    CastLayout lay;
    int rc = cast_plan(g, d, &n_rays, obs, &lay);
    if (rc) return rc;
    if (d->order != 1 || d->stop_surface != MPATH_SURFACE_ETA || d->dphidl != MPATH_DPHIDL_CHAIN ||
        d->n_surfaces != 0 || g->tdual)
        return fail(MPATH_ERR_UNSUPPORTED, "the forward-mode Jacobian takes CIC casts to an iso-eta surface with the "
                                           "chain-rule dPhi/dlambda, one stop surface and a static potential");
    if (d->checkpoint_every != 0) return fail(MPATH_ERR_INVALID_ARG, "the forward-mode Jacobian stores no checkpoints");
    if (!dev_ws) return fail(MPATH_ERR_INVALID_ARG, "dev_ws is NULL");
    const size_t off = align_up(lay.total, 256);
    if (ws_bytes < off + (size_t)n_rays * sizeof(TanEnd))
        return fail(MPATH_ERR_WORKSPACE_TOO_SMALL, "jacobian workspace too small");
    TangentOut tg;
    tg.ends = (TanEnd*)((char*)dev_ws + off);
    tg.jac = jac;
    tg.dz_dtheta = dz_dtheta;
    return cast_impl(g, d, out, dev_ws, ws_bytes, stream, false, nullptr, nullptr, &tg);
}

int mpath_infinitesimal_beam(const mpath_grid* g, const mpath_cast_desc* d, mpath_observables* out, float* A,
                             void* dev_ws, size_t ws_bytes, void* stream)
{
    int64_t n_rays;
    int rc = check_cast_desc(g, d, &n_rays);
    if (rc) return rc;
    if (n_rays > 0 && !A) return fail(MPATH_ERR_INVALID_ARG, "A is NULL");
    if (d->checkpoint_every != 0)
        return fail(MPATH_ERR_INVALID_ARG, "the infinitesimal-beam cast stores no checkpoints (checkpoint_every 0)");
    if (d->order != 1) return fail(MPATH_ERR_UNSUPPORTED, "the infinitesimal beam is implemented for order = 1 (CIC)");
    return cast_impl(g, d, out, dev_ws, ws_bytes, stream, true, A);
}

int mpath_adjoint_workspace_bytes(const mpath_grid* g, const mpath_cast_desc* d, size_t* bytes)
{
    if (!bytes) return fail(MPATH_ERR_INVALID_ARG, "bytes is NULL");
    int64_t n_rays;
    std::vector<ObsDev> obs;
    CastLayout lay;
    const int rc = cast_plan(g, d, &n_rays, obs, &lay);
    if (rc) return rc;
    if (d->checkpoint_every <= 0) return fail(MPATH_ERR_INVALID_ARG, "the adjoint needs checkpoint_every > 0");
    if (g->tdual) return fail(MPATH_ERR_UNSUPPORTED, "the adjoint of a time-dependent potential is not implemented");
    *bytes = adjoint_layout(g, d, n_rays).total;
    return MPATH_OK;
}

}  // extern "C"

namespace {

int adjoint_impl(const mpath_grid* g, const mpath_cast_desc* d, const mpath_observables* fwd,
                 const void* cast_ws, size_t cast_ws_bytes, const mpath_adjoint_desc* ad, void* dev_ws,
                 size_t ws_bytes, void* stream, const double2* ray_stop)
{
    int64_t n_rays;
    std::vector<ObsDev> obs;
    CastLayout lay;
    int rc = cast_plan(g, d, &n_rays, obs, &lay);
    if (rc) return rc;
    if (d->checkpoint_every <= 0) return fail(MPATH_ERR_INVALID_ARG, "the adjoint needs checkpoint_every > 0");
    if (g->tdual) return fail(MPATH_ERR_UNSUPPORTED, "the adjoint of a time-dependent potential is not implemented");
    if (!fwd || !fwd->n_steps || !fwd->status)
        return fail(MPATH_ERR_INVALID_ARG, "the forward n_steps and status arrays are required");
    if (!ad) return fail(MPATH_ERR_INVALID_ARG, "adjoint desc is NULL");
    if (!cast_ws || !dev_ws) return fail(MPATH_ERR_INVALID_ARG, "a workspace is NULL");
    if (cast_ws_bytes < lay.total) return fail(MPATH_ERR_WORKSPACE_TOO_SMALL, "cast workspace too small");
    const AdjointLayout al = adjoint_layout(g, d, n_rays);
    if (ws_bytes < al.total) return fail(MPATH_ERR_WORKSPACE_TOO_SMALL, "adjoint workspace too small");
    if (ad->dL_dphi_total && !(g->max_level == 0 && g->periodic))
        return fail(MPATH_ERR_UNSUPPORTED, "dL_dphi_total needs a uniform periodic grid");
    if ((ad->dL_dvalues || ad->dL_dphi_total) && !g->perm)
        return fail(MPATH_ERR_UNSUPPORTED, "cell cotangents need the grid's auxiliary tables (mpath_grid_build_with_aux)");
    const bool jac = ad->jac || ad->dz_dtheta || ad->ray_status;
    const bool loss = ad->dL_dvalues || ad->dL_dphi_total;
    if (!jac && !loss) return MPATH_OK;

    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)dev_ws;
    AdjointArgs A;
    std::memset(&A, 0, sizeof A);
    A.c = make_cast_args(g, d, lay, (char*)cast_ws, n_rays);
    A.c.ray_stop = ray_stop;
    A.tape = (GeoState*)(ws + al.off_tape);
    A.n_steps = fwd->n_steps;
    A.status = fwd->status;
    A.dL_dalpha = ad->dL_dalpha;
    A.dL_dz = ad->dL_dz;
    A.jac = ad->jac;
    A.dz_dtheta = ad->dz_dtheta;
    A.ray_status = ad->ray_status;
    float* grad = (float*)(ws + al.off_grad);
    A.grad = loss ? grad : nullptr;
    A.n_cells = g->n_cells;
    hipError_t e = hipSuccess;
    if (loss) e = launch_fill_zero(grad, grad_accumulator_floats(g->n_cells), s);
    if (!e) e = launch_adjoint(A, jac && loss ? 4 : (jac ? 3 : 1), s);
    if (!e && ad->dL_dvalues)
        e = launch_scatter_grad(grad, g->perm, (float4*)ad->dL_dvalues, g->n_cells, s);
    if (!e && ad->dL_dphi_total)
        e = launch_central_transpose(grad, g->perm, ad->dL_dphi_total, g->n0, g->box / g->n0, g->n_cells, s);
    if (e) return hip_fail(e, "adjoint launch");
    return MPATH_OK;
}

}  // namespace

extern "C" {

int mpath_adjoint(const mpath_grid* g, const mpath_cast_desc* d, const mpath_observables* fwd,
                  const void* cast_ws, size_t cast_ws_bytes, const mpath_adjoint_desc* ad, void* dev_ws,
                  size_t ws_bytes, void* stream)
{
    return adjoint_impl(g, d, fwd, cast_ws, cast_ws_bytes, ad, dev_ws, ws_bytes, stream, nullptr);
}

}  // extern "C"

// ---- autotuner ----

namespace {

// The sample the tuner casts: the first ceil(count / sample_div) pixels of
// every observer, so that the mix of observers and path lengths is kept.
struct TuneSample {
    std::vector<int64_t> first, count;
    mpath_cast_desc desc;
};

TuneSample tune_sample(const mpath_cast_desc* d, int32_t sample_div)
{
    TuneSample t;
    const int64_t npix = 12ll * d->nside * d->nside;
    t.first.resize(d->n_obs);
    t.count.resize(d->n_obs);
    for (int j = 0; j < d->n_obs; ++j) {
        const int64_t c = d->pix_count ? d->pix_count[j] : npix;
        t.first[j] = d->pix_first ? d->pix_first[j] : 0;
        t.count[j] = c > 0 ? std::max<int64_t>(1, (c + sample_div - 1) / sample_div) : 0;
    }
    t.desc = *d;
    t.desc.pix_first = t.first.data();
    t.desc.pix_count = t.count.data();
    t.desc.checkpoint_every = 0;
    return t;
}

}  // namespace

extern "C" {

int mpath_autotune_workspace_bytes(const mpath_grid* g, const mpath_cast_desc* d, int32_t sample_div,
                                   size_t* bytes)
{
    if (!bytes || sample_div < 1) return fail(MPATH_ERR_INVALID_ARG, "bytes is NULL or sample_div < 1");
    int64_t n_rays;
    const int rc = check_cast_desc(g, d, &n_rays);
    if (rc) return rc;
    const TuneSample t = tune_sample(d, sample_div);
    return mpath_cast_workspace_bytes(g, &t.desc, bytes);
}

int mpath_autotune(const mpath_grid* g, const mpath_cast_desc* d, int32_t sample_div, void* dev_ws,
                   size_t ws_bytes, void* stream, mpath_cast_desc* tuned, float* best_ms)
{
    if (!tuned) return fail(MPATH_ERR_INVALID_ARG, "tuned is NULL");
    size_t need = 0;
    int rc = mpath_autotune_workspace_bytes(g, d, sample_div, &need);
    if (rc) return rc;
    if (!dev_ws || ws_bytes < need) return fail(MPATH_ERR_WORKSPACE_TOO_SMALL, "autotune workspace too small");
    const TuneSample t = tune_sample(d, sample_div);
    hipStream_t s = (hipStream_t)stream;
    // candidates: the static schedule, and the persistent one at the
    // resident occupancy, half and twice that, with refills every 8..128 steps
    const int occ = std::max(1, cast_occupancy_blocks_per_cu(256, g->max_level > 0, g->tdual != nullptr) * 4);
    struct Cand { int32_t schedule, wpc, batch; };
    std::vector<Cand> cands = {{MPATH_SCHED_STATIC, 0, 0}};
    for (int w : {occ, std::max(1, occ / 2), 2 * occ})
        for (int b : {8, 16, 32, 64, 128}) cands.push_back({MPATH_SCHED_PERSISTENT, w, b});
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(MPATH_ERR_DEVICE, "autotune: event creation failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(MPATH_ERR_DEVICE, "autotune: event creation failed");
    }
    mpath_observables none;
    std::memset(&none, 0, sizeof none);
    float best = 1e30f;
    Cand bestc = cands[0];
    for (size_t i = 0; i < cands.size() && rc == MPATH_OK; ++i) {
        mpath_cast_desc c = t.desc;
        c.schedule = cands[i].schedule;
        c.waves_per_cu = cands[i].wpc;
        c.batch = cands[i].batch;
        float ms = 1e30f;
        // the first candidate runs once more untimed (warm caches and code)
        for (int rep = (i == 0 ? -1 : 0); rep < 2 && rc == MPATH_OK; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(MPATH_ERR_DEVICE, "autotune: event record"); break; }
            rc = mpath_cast(g, &c, &none, dev_ws, ws_bytes, stream);
            if (rc) break;
            float m = 0.0f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&m, e0, e1) != hipSuccess) {
                rc = fail(MPATH_ERR_DEVICE, "autotune: event timing");
                break;
            }
            if (rep >= 0) ms = std::min(ms, m);
        }
        if (rc == MPATH_OK && ms < best) {
            best = ms;
            bestc = cands[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *tuned = *d;
    tuned->schedule = bestc.schedule;
    tuned->waves_per_cu = bestc.wpc;
    tuned->batch = bestc.batch;
    if (best_ms) *best_ms = best;
    return MPATH_OK;
}


int mpath_gather_probe(const void* table, size_t table_bytes, int32_t record_bytes, int32_t in_flight,
                       int64_t n_waves, int32_t iters, uint32_t seed, float* out, void* stream)
{
    if (!table || !out) return fail(MPATH_ERR_INVALID_ARG, "table and out must be device pointers");
    if (reinterpret_cast<uintptr_t>(table) % 16) return fail(MPATH_ERR_INVALID_ARG, "table must be 16-byte aligned");
    if (record_bytes != 16 && record_bytes != 64 && record_bytes != 128)
        return fail(MPATH_ERR_INVALID_ARG, "record_bytes must be 16, 64 or 128");
    if (table_bytes < (size_t)record_bytes) return fail(MPATH_ERR_INVALID_ARG, "table smaller than one record");
    if (in_flight != 1 && in_flight != 2 && in_flight != 4)
        return fail(MPATH_ERR_INVALID_ARG, "in_flight must be 1, 2 or 4");
    if (n_waves < 1 || n_waves > (1 << 24)) return fail(MPATH_ERR_INVALID_ARG, "n_waves must be in [1, 2^24]");
    if (iters < 1) return fail(MPATH_ERR_INVALID_ARG, "iters must be >= 1");
    const hipError_t e = launch_gather_probe(table, table_bytes, record_bytes, in_flight, n_waves, iters, seed, out,
                                             static_cast<hipStream_t>(stream));
    return e ? hip_fail(e, "gather probe launch") : MPATH_OK;
}


int mpath_lensing_maps(const float* A, int64_t n, float* out, void* stream)
{
    if (n < 0) return fail(MPATH_ERR_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!A || !out)) return fail(MPATH_ERR_INVALID_ARG, "A and out must be device pointers");
    const hipError_t e = launch_lensing_maps(A, n, out, static_cast<hipStream_t>(stream));
    return e ? hip_fail(e, "lensing maps launch") : MPATH_OK;
}

}  // extern "C"

namespace {

// The five-rays-per-beam cast behind mpath_finite_beam: workspace layout and
// the inner cast descriptor (caller's directions, 5 c_j rays per observer).
struct BeamPlan {
    int64_t n_rays = 0;
    std::vector<BeamObs> obs;
    std::vector<int64_t> count5;
    mpath_cast_desc desc5;
    size_t off_obs = 0, off_dirs5 = 0, off_status5 = 0, off_cast = 0, cast_bytes = 0, total = 0;
    CastLayout lay5;
};

int beam_plan(const mpath_grid* g, const mpath_cast_desc* d, BeamPlan& P)
{
    int rc = check_cast_desc(g, d, &P.n_rays);
    if (rc) return rc;
    if (d->n_surfaces) return fail(MPATH_ERR_UNSUPPORTED, "the finite beam takes one stop surface");
    const int64_t npix = 12ll * d->nside * d->nside;
    P.obs.resize(d->n_obs);
    P.count5.resize(d->n_obs);
    int64_t first = 0;
    for (int j = 0; j < d->n_obs; ++j) {
        P.obs[j].ray_first = first;
        P.obs[j].pix_first = (d->pix_first && !d->dirs) ? d->pix_first[j] : 0;
        P.obs[j].count = d->pix_count ? d->pix_count[j] : npix;
        P.count5[j] = 5 * P.obs[j].count;
        first += P.obs[j].count;
    }
    P.desc5 = *d;
    P.desc5.pix_first = nullptr;
    P.desc5.pix_count = P.count5.data();
    P.desc5.checkpoint_every = 0;
    P.desc5.dirs = reinterpret_cast<const double*>(16);   // placeholder until the workspace is known
    int64_t n5;
    std::vector<ObsDev> obs5;
    rc = cast_plan(g, &P.desc5, &n5, obs5, &P.lay5);
    if (rc) return rc;
    P.off_obs = 0;
    P.off_dirs5 = align_up((size_t)d->n_obs * sizeof(BeamObs), 256);
    P.off_status5 = align_up(P.off_dirs5 + (size_t)n5 * 24, 256);
    P.off_cast = align_up(P.off_status5 + (size_t)n5 * 4, 256);
    P.cast_bytes = P.lay5.total;
    P.total = P.off_cast + P.cast_bytes;
    return MPATH_OK;
}

}  // namespace

extern "C" {

int mpath_finite_beam_workspace_bytes(const mpath_grid* g, const mpath_cast_desc* d, size_t* bytes)
{
    if (!bytes) return fail(MPATH_ERR_INVALID_ARG, "bytes is NULL");
    BeamPlan P;
    const int rc = beam_plan(g, d, P);
    if (rc) return rc;
    *bytes = P.total;
    return MPATH_OK;
}

int mpath_finite_beam(const mpath_grid* g, const mpath_cast_desc* d, double eps, float* A, int32_t* status,
                      void* dev_ws, size_t ws_bytes, void* stream)
{
    if (!(eps > 0.0 && eps <= 0.1)) return fail(MPATH_ERR_INVALID_ARG, "eps must be in (0, 0.1] rad");
    BeamPlan P;
    int rc = beam_plan(g, d, P);
    if (rc) return rc;
    if (P.n_rays > 0 && !A) return fail(MPATH_ERR_INVALID_ARG, "A is NULL");
    if (!dev_ws) return fail(MPATH_ERR_INVALID_ARG, "dev_ws is NULL");
    if (ws_bytes < P.total) return fail(MPATH_ERR_WORKSPACE_TOO_SMALL, "finite-beam workspace too small");
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)dev_ws;
    BeamObs* obs_d = reinterpret_cast<BeamObs*>(ws + P.off_obs);
    double* dirs5 = reinterpret_cast<double*>(ws + P.off_dirs5);
    int32_t* status5 = reinterpret_cast<int32_t*>(ws + P.off_status5);
    hipError_t e = hipMemcpyAsync(obs_d, P.obs.data(), P.obs.size() * sizeof(BeamObs), hipMemcpyHostToDevice, s);
    if (!e) e = hipStreamSynchronize(s);   // the host table is released on return
    if (e) return hip_fail(e, "beam table upload");
    const double te = std::tan(eps);
    e = launch_beam_dirs(obs_d, d->n_obs, d->nside, d->dirs, te, P.n_rays, dirs5, s);
    if (e) return hip_fail(e, "beam directions launch");
    P.desc5.dirs = dirs5;
    mpath_observables out5;
    std::memset(&out5, 0, sizeof out5);
    out5.status = status5;
    rc = mpath_cast(g, &P.desc5, &out5, ws + P.off_cast, P.cast_bytes, stream);
    if (rc) return rc;
    const RayEnd* ends = reinterpret_cast<const RayEnd*>(ws + P.off_cast + P.lay5.off_ends);
    e = launch_finite_beam(obs_d, d->n_obs, ends, dirs5, status5, g->eta0, te, P.n_rays, A, status, s);
    return e ? hip_fail(e, "finite-beam launch") : MPATH_OK;
}


}  // extern "C"

namespace {

// Host side of the geodesic finder: per-source stop surfaces and targets,
// the cast descriptor of the iterations, and the workspace layout.
struct FinderPlan {
    int64_t n = 0;
    std::vector<double2> stop;          // (eta_s, a_s)
    std::vector<double> target;         // beta, [n][3]
    double chi_max = 0.0;
    int64_t count = 0;
    mpath_cast_desc cd;
    size_t off_stop = 0, off_target = 0, off_iter = 0, off_status = 0, off_sep = 0, off_jac = 0, off_nsteps = 0,
           off_active = 0, off_cast = 0, off_adj = 0, cast_bytes = 0, adj_bytes = 0, total = 0;
    CastLayout lay;
    // grid search: at most m_max sources, g x g candidates each
    int64_t m_max = 0, gcount = 0;
    int g = 0;
    mpath_cast_desc gcd;
    size_t off_gidx = 0, off_gw = 0, off_gdirs = 0, off_gstop = 0, off_gstatus = 0, off_gcast = 0, gcast_bytes = 0;
};

int finder_plan(const mpath_grid* g, const mpath_finder_desc* f, FinderPlan& P, bool tables)
{
    if (!g) return fail(MPATH_ERR_INVALID_ARG, "grid is NULL");
    if (!f) return fail(MPATH_ERR_INVALID_ARG, "finder desc is NULL");
    if (!f->obs_pos) return fail(MPATH_ERR_INVALID_ARG, "obs_pos is NULL");
    if (f->n_src < 0 || (f->n_src > 0 && !f->src_pos)) return fail(MPATH_ERR_INVALID_ARG, "bad n_src or src_pos");
    if (f->order != 1) return fail(MPATH_ERR_UNSUPPORTED, "only order = 1 (CIC) is implemented");
    if (g->tdual)
        return fail(MPATH_ERR_UNSUPPORTED, "the finder's exact Jacobian (the adjoint) needs a static potential");
    if (!(f->tol > 0.0)) return fail(MPATH_ERR_INVALID_ARG, "tol must be > 0");
    if (f->max_iter < 1) return fail(MPATH_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (f->identity_iters < 0) return fail(MPATH_ERR_INVALID_ARG, "identity_iters must be >= 0");
    if (f->checkpoint_every < 1) return fail(MPATH_ERR_INVALID_ARG, "checkpoint_every must be >= 1");
    if (f->grid_rounds < 0) return fail(MPATH_ERR_INVALID_ARG, "grid_rounds must be >= 0");
    if (f->grid_rounds > 0 && (f->grid_n < 3 || f->grid_n > 15 || f->grid_n % 2 == 0))
        return fail(MPATH_ERR_INVALID_ARG, "grid_n must be odd in [3, 15]");
    if (f->grid_max < 0) return fail(MPATH_ERR_INVALID_ARG, "grid_max must be >= 0");
    P.n = f->n_src;
    const double amin = 1.0 / (1.0 + kZMaxTable);
    const double eta_min = g->bg.is_static ? -INFINITY : g->bg.eta_of_a(amin);
    if (tables) {
        P.stop.resize(P.n);
        P.target.resize(3 * P.n);
    }
    P.chi_max = 0.0;
    for (int64_t i = 0; i < P.n; ++i) {
        double r[3];
        for (int k = 0; k < 3; ++k) r[k] = f->src_pos[3 * i + k] - f->obs_pos[k];
        const double chi = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        if (!(chi > 0.0) || !std::isfinite(chi)) return fail(MPATH_ERR_INVALID_ARG, "a source sits at the observer");
        const double eta_s = g->eta0 - chi;
        if (eta_s < eta_min) return fail(MPATH_ERR_UNSUPPORTED, "a source lies beyond the background table (z > 20)");
        P.chi_max = std::max(P.chi_max, chi);
        if (tables) {
            P.stop[i] = make_double2(eta_s, g->bg.a_of_eta(eta_s));
            for (int k = 0; k < 3; ++k) P.target[3 * i + k] = r[k] / chi;
        }
    }
    P.count = P.n;
    std::memset(&P.cd, 0, sizeof P.cd);
    P.cd.n_obs = 1;
    P.cd.obs_pos = f->obs_pos;
    P.cd.stop_value = &P.chi_max;     // bounds every source's surface (checkpoint sizing)
    P.cd.stop_kind = MPATH_STOP_CHI;
    P.cd.nside = 1;
    P.cd.pix_count = &P.count;
    P.cd.order = 1;
    P.cd.steps_per_cell = f->steps_per_cell;
    P.cd.adaptive = f->adaptive;
    P.cd.max_steps = f->max_steps;
    P.cd.schedule = MPATH_SCHED_STATIC;
    P.cd.checkpoint_every = f->checkpoint_every;
    P.cd.dirs = reinterpret_cast<const double*>(16);   // the working theta once the workspace is known
    int64_t nr;
    std::vector<ObsDev> obs;
    int rc = cast_plan(g, &P.cd, &nr, obs, &P.lay);
    if (rc) return rc;
    const size_t n = (size_t)P.n;
    P.off_stop = 0;
    P.off_target = align_up(P.off_stop + n * 16, 256);
    P.off_iter = align_up(P.off_target + n * 24, 256);
    P.off_status = align_up(P.off_iter + n * 4, 256);
    P.off_sep = align_up(P.off_status + n * 4, 256);
    P.off_jac = align_up(P.off_sep + n * 8, 256);
    P.off_nsteps = align_up(P.off_jac + n * 16, 256);
    P.off_active = align_up(P.off_nsteps + n * 4, 256);
    P.off_cast = align_up(P.off_active + 256, 256);
    P.cast_bytes = P.lay.total;
    P.off_adj = align_up(P.off_cast + P.cast_bytes, 256);
    P.adj_bytes = adjoint_layout(g, &P.cd, P.n).total;
    P.total = P.off_adj + P.adj_bytes;
    if (f->grid_rounds > 0 && P.n > 0) {
        P.g = f->grid_n;
        P.m_max = f->grid_max > 0 ? std::min<int64_t>(f->grid_max, P.n) : P.n;
        const size_t mg = (size_t)P.m_max * P.g * P.g;
        P.gcount = (int64_t)mg;
        P.gcd = P.cd;
        P.gcd.pix_count = &P.gcount;
        P.gcd.checkpoint_every = 0;
        CastLayout gl;
        rc = cast_plan(g, &P.gcd, &nr, obs, &gl);
        if (rc) return rc;
        P.off_gidx = align_up(P.total, 256);
        P.off_gw = align_up(P.off_gidx + (size_t)P.m_max * 8, 256);
        P.off_gdirs = align_up(P.off_gw + (size_t)P.m_max * 8, 256);
        P.off_gstop = align_up(P.off_gdirs + mg * 24, 256);
        P.off_gstatus = align_up(P.off_gstop + mg * 16, 256);
        P.off_gcast = align_up(P.off_gstatus + mg * 4, 256);
        P.gcast_bytes = gl.total;
        P.total = P.off_gcast + P.gcast_bytes;
    }
    return MPATH_OK;
}

}  // namespace

extern "C" {

int mpath_find_geodesics_workspace_bytes(const mpath_grid* g, const mpath_finder_desc* f, size_t* bytes)
{
    if (!bytes) return fail(MPATH_ERR_INVALID_ARG, "bytes is NULL");
    FinderPlan P;
    const int rc = finder_plan(g, f, P, false);
    if (rc) return rc;
    *bytes = P.total;
    return MPATH_OK;
}

int mpath_find_geodesics(const mpath_grid* g, const mpath_finder_desc* f, mpath_finder_out* out, void* dev_ws,
                         size_t ws_bytes, void* stream)
{
    FinderPlan P;
    int rc = finder_plan(g, f, P, true);
    if (rc) return rc;
    if (!out || (P.n > 0 && !out->theta)) return fail(MPATH_ERR_INVALID_ARG, "out or out->theta is NULL");
    if (!dev_ws) return fail(MPATH_ERR_INVALID_ARG, "dev_ws is NULL");
    if (ws_bytes < P.total) return fail(MPATH_ERR_WORKSPACE_TOO_SMALL, "finder workspace too small");
    if (P.n == 0) return MPATH_OK;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)dev_ws;
    const double2* stop = reinterpret_cast<const double2*>(ws + P.off_stop);
    const double* target = reinterpret_cast<const double*>(ws + P.off_target);
    int32_t* n_iter = reinterpret_cast<int32_t*>(ws + P.off_iter);
    int32_t* status = reinterpret_cast<int32_t*>(ws + P.off_status);
    double* sep = reinterpret_cast<double*>(ws + P.off_sep);
    float* jac = reinterpret_cast<float*>(ws + P.off_jac);
    int32_t* nsteps = reinterpret_cast<int32_t*>(ws + P.off_nsteps);
    unsigned int* active = reinterpret_cast<unsigned int*>(ws + P.off_active);
    char* cws = ws + P.off_cast;
    char* aws = ws + P.off_adj;
    double* theta = out->theta;
    const size_t n = (size_t)P.n;
    hipError_t e = hipMemcpyAsync(ws + P.off_stop, P.stop.data(), n * 16, hipMemcpyHostToDevice, s);
    if (!e) e = hipMemcpyAsync(ws + P.off_target, P.target.data(), n * 24, hipMemcpyHostToDevice, s);
    if (!e) e = hipMemcpyAsync(theta, ws + P.off_target, n * 24, hipMemcpyDeviceToDevice, s);   // theta_0 = beta
    if (!e) e = hipStreamSynchronize(s);   // host tables are released on return
    if (!e) e = launch_fill_i32(n_iter, P.n, -1, s);
    if (e) return hip_fail_drain(e, s, "finder set-up");
    P.cd.dirs = theta;
    const RayEnd* ends = reinterpret_cast<const RayEnd*>(cws + P.lay.off_ends);
    const int K = f->checkpoint_every;
    for (int it = 0; it < f->max_iter; ++it) {
        const bool exact = it >= f->identity_iters;
        P.cd.checkpoint_every = exact ? K : 0;
        mpath_observables fo;
        std::memset(&fo, 0, sizeof fo);
        fo.status = status;
        fo.n_steps = nsteps;
        rc = cast_impl(g, &P.cd, &fo, cws, P.cast_bytes, stream, false, nullptr, stop);
        if (rc) return rc;
        if (exact) {
            mpath_adjoint_desc ad;
            std::memset(&ad, 0, sizeof ad);
            ad.jac = jac;
            rc = adjoint_impl(g, &P.cd, &fo, cws, P.cast_bytes, &ad, aws, P.adj_bytes, stream, stop);
            if (rc) return rc;
        }
        e = launch_finder_update(P.n, ends, target, status, exact ? jac : nullptr, g->eta0, f->tol, it, theta,
                                 n_iter, sep, active, s);
        unsigned int left = 0;
        if (!e) e = hipMemcpyAsync(&left, active, sizeof left, hipMemcpyDeviceToHost, s);
        if (!e) e = hipStreamSynchronize(s);
        if (e) return hip_fail(e, "finder iteration");
        if (left == 0) break;
    }
    if (f->grid_rounds > 0) {
        // the last-resort root finder for the sources still iterating
        std::vector<int32_t> it_h(n);
        e = hipMemcpyAsync(it_h.data(), n_iter, n * 4, hipMemcpyDeviceToHost, s);
        if (!e) e = hipStreamSynchronize(s);
        if (e) return hip_fail(e, "grid search set-up");
        std::vector<int64_t> idx;
        for (int64_t i = 0; i < P.n && (int64_t)idx.size() < P.m_max; ++i)
            if (it_h[i] == -1) idx.push_back(i);
        const int64_t m = (int64_t)idx.size();
        if (m > 0) {
            int64_t* gidx = reinterpret_cast<int64_t*>(ws + P.off_gidx);
            double* gw = reinterpret_cast<double*>(ws + P.off_gw);
            double* gdirs = reinterpret_cast<double*>(ws + P.off_gdirs);
            double2* gstop = reinterpret_cast<double2*>(ws + P.off_gstop);
            int32_t* gstatus = reinterpret_cast<int32_t*>(ws + P.off_gstatus);
            char* gws = ws + P.off_gcast;
            e = hipMemcpyAsync(gidx, idx.data(), (size_t)m * 8, hipMemcpyHostToDevice, s);
            if (!e) e = hipStreamSynchronize(s);
            if (!e) e = launch_grid_init(m, gidx, sep, gw, s);
            if (e) return hip_fail(e, "grid search set-up");
            mpath_cast_desc gcd = P.gcd;
            int64_t count = m * P.g * P.g;
            gcd.pix_count = &count;
            gcd.dirs = gdirs;
            int64_t nr;
            std::vector<ObsDev> gobs;
            CastLayout gl;
            rc = cast_plan(g, &gcd, &nr, gobs, &gl);
            if (rc) return rc;
            const RayEnd* gends = reinterpret_cast<const RayEnd*>(gws + gl.off_ends);
            for (int r = 0; r < f->grid_rounds; ++r) {
                e = launch_grid_dirs(m, P.g, gidx, theta, gw, stop, gdirs, gstop, s);
                if (e) return hip_fail(e, "grid search directions");
                mpath_observables go;
                std::memset(&go, 0, sizeof go);
                go.status = gstatus;
                rc = cast_impl(g, &gcd, &go, gws, P.gcast_bytes, stream, false, nullptr, gstop);
                if (rc) return rc;
                e = launch_grid_pick(m, P.g, gidx, gends, gdirs, gstatus, target, g->eta0, f->tol, f->max_iter + r,
                                     theta, sep, n_iter, gw, active, s);
                unsigned int left = 0;
                if (!e) e = hipMemcpyAsync(&left, active, sizeof left, hipMemcpyDeviceToHost, s);
                if (!e) e = hipStreamSynchronize(s);
                if (e) return hip_fail(e, "grid search round");
                if (left == 0) break;
            }
        }
    }
    // final cast along theta, checkpointed for the distortion matrix there
    P.cd.checkpoint_every = K;
    mpath_observables fo;
    std::memset(&fo, 0, sizeof fo);
    fo.status = status;
    fo.n_steps = nsteps;
    fo.z5 = out->z5;
    fo.z0 = out->z0;
    fo.z1 = out->z1;
    fo.phi_src = out->phi_src;
    rc = cast_impl(g, &P.cd, &fo, cws, P.cast_bytes, stream, false, nullptr, stop);
    if (rc) return rc;
    if (out->A || out->dz_dtheta) {
        mpath_adjoint_desc ad;
        std::memset(&ad, 0, sizeof ad);
        ad.jac = out->A;
        ad.dz_dtheta = out->dz_dtheta;
        rc = adjoint_impl(g, &P.cd, &fo, cws, P.cast_bytes, &ad, aws, P.adj_bytes, stream, stop);
        if (rc) return rc;
    }
    e = launch_finder_sep(P.n, ends, target, theta, status, g->eta0, out->sep ? out->sep : sep, s);
    if (!e && out->n_iter) e = hipMemcpyAsync(out->n_iter, n_iter, n * 4, hipMemcpyDeviceToDevice, s);
    if (!e && out->status) e = hipMemcpyAsync(out->status, status, n * 4, hipMemcpyDeviceToDevice, s);
    return e ? hip_fail(e, "finder output") : MPATH_OK;
}

}  // extern "C"
