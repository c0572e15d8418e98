// Host-side paths of the library's C ABI, for a build whose host code runs
// under AddressSanitizer and UndefinedBehaviorSanitizer (test
// infrastructure; the CPU tests build and run it without a GPU): argument
// and tree validation, workspace sizes, ray counts, and the host part of the
// grid build (ordering, packing, central differences for grad = NULL) up to
// the first upload, which fails for want of a device.  Exits 0 when every
// call returns as expected; the sanitizers abort on a memory or UB error.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <vector>

#include "mpath.h"

#define CHECK(c)                                                                                   \
    do {                                                                                           \
        if (!(c)) {                                                                                \
            std::fprintf(stderr, "abi driver: check failed: %s (line %d): %s\n", #c, __LINE__,    \
                         mpath_last_error());                                                      \
            return 1;                                                                              \
        }                                                                                          \
    } while (0)

struct Tree {
    int n0, max_level;
    std::vector<uint8_t> level;
    std::vector<int32_t> ijk;
    std::vector<double> phi, grad;

    void add(int l, int i, int j, int k)
    {
        level.push_back((uint8_t)l);
        ijk.insert(ijk.end(), {i, j, k});
        phi.push_back(1e-5 * ((i * 7 + j * 3 + k) % 11 - 5) / (1 + l));
        grad.insert(grad.end(), {1e-7 * i, -2e-7 * j, 3e-7 * k});
    }
};

// n0^3 coarse cells, the cells (1..2, 1, 1) refined, and one child of each refined again
static Tree make_tree(int n0)
{
    Tree t;
    t.n0 = n0;
    t.max_level = 2;
    for (int k = 0; k < n0; ++k)
        for (int j = 0; j < n0; ++j)
            for (int i = 0; i < n0; ++i) t.add(0, i, j, k);
    for (int p = 1; p <= 2; ++p)
        for (int o = 0; o < 8; ++o) t.add(1, 2 * p + (o & 1), 2 + ((o >> 1) & 1), 2 + (o >> 2));
    for (int p = 1; p <= 2; ++p)
        for (int o = 0; o < 8; ++o) t.add(2, 4 * p + (o & 1), 4 + ((o >> 1) & 1), 4 + (o >> 2));
    return t;
}

static mpath_grid_desc desc_of(const Tree& t, int periodic, bool with_grad)
{
    mpath_grid_desc d;
    std::memset(&d, 0, sizeof d);
    d.box = 100.0;
    d.n0 = t.n0;
    d.max_level = t.max_level;
    d.periodic = periodic;
    d.value_dtype = MPATH_F64;
    d.n_cells = (int64_t)t.level.size();
    d.level = t.level.data();
    d.ijk = t.ijk.data();
    d.phi = t.phi.data();
    d.grad = with_grad ? t.grad.data() : nullptr;
    return d;
}

int main()
{
    size_t bytes = 0;
    const Tree t = make_tree(4);
    mpath_grid_desc d = desc_of(t, 1, true);
    CHECK(mpath_grid_workspace_bytes(&d, &bytes) == MPATH_OK && bytes > 0);
    CHECK(mpath_grid_aux_bytes(&d, &bytes) == MPATH_OK && bytes >= 40 * t.level.size());
    // invalid descriptors and trees, all refused before any device work
    void* fake = reinterpret_cast<void*>(0x100000);
    mpath_cosmo cz = {0.3, 0.7, 0.7};
    mpath_grid* g = nullptr;
    {
        mpath_grid_desc b = d;
        b.n0 = 3;
        CHECK(mpath_grid_workspace_bytes(&b, &bytes) == MPATH_ERR_INVALID_ARG);
        b = d;
        b.value_dtype = 7;
        CHECK(mpath_grid_build(&b, &cz, fake, 1 << 30, nullptr, &g) == MPATH_ERR_INVALID_ARG);
        b = d;
        b.phi = nullptr;
        CHECK(mpath_grid_build(&b, &cz, fake, 1 << 30, nullptr, &g) == MPATH_ERR_INVALID_ARG);
        b = d;
        b.n_cells -= 1;                    // a refined cell with 7 children
        CHECK(mpath_grid_build(&b, &cz, fake, 1 << 30, nullptr, &g) == MPATH_ERR_NOT_FULL_TREE);
        b = d;
        b.max_level = 1;                   // cells above max_level
        CHECK(mpath_grid_build(&b, &cz, fake, 1 << 30, nullptr, &g) == MPATH_ERR_INVALID_ARG);
        Tree u = t;
        u.ijk[3 * 5] = 99;                 // a coarse cell out of range
        b = desc_of(u, 1, true);
        CHECK(mpath_grid_build(&b, &cz, fake, 1 << 30, nullptr, &g) == MPATH_ERR_INVALID_ARG);
        u = t;
        u.ijk[3 * 5] = 4 - 1;              // a repeated coarse cell
        u.ijk[3 * 5 + 1] = 0;
        u.ijk[3 * 5 + 2] = 0;
        b = desc_of(u, 1, true);
        CHECK(mpath_grid_build(&b, &cz, fake, 1 << 30, nullptr, &g) == MPATH_ERR_NOT_FULL_TREE);
        u = t;
        const size_t c2 = 64 + 16;         // first level-2 cell: move its family under a missing parent
        for (int o = 0; o < 8; ++o) u.ijk[3 * (c2 + o) + 1] += 4;   // parent (2, 4, 2) at level 1: absent
        b = desc_of(u, 1, true);
        CHECK(mpath_grid_build(&b, &cz, fake, 1 << 30, nullptr, &g) == MPATH_ERR_NOT_FULL_TREE);
        CHECK(mpath_grid_build(&d, &cz, fake, 16, nullptr, &g) == MPATH_ERR_WORKSPACE_TOO_SMALL);
        mpath_cosmo open = {0.3, 0.5, 0.7};
        CHECK(mpath_grid_build_with_aux(&d, &cz, fake, 1 << 30, fake, 8, nullptr, &g) ==
              MPATH_ERR_WORKSPACE_TOO_SMALL);
        CHECK(mpath_grid_build(&d, &open, fake, 1 << 30, nullptr, &g) == MPATH_ERR_UNSUPPORTED);
        CHECK(g == nullptr);
    }
    // the whole host part of a build (grad = NULL: central differences per
    // level, periodic and not) up to the first upload; only without a GPU,
    // where that upload fails
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    if (ndev == 0) {
        for (int periodic = 0; periodic <= 1; ++periodic) {
            mpath_grid_desc b = desc_of(t, periodic, false);
            CHECK(mpath_grid_workspace_bytes(&b, &bytes) == MPATH_OK);
            CHECK(mpath_grid_build_with_aux(&b, &cz, fake, bytes, fake, 1 << 30, nullptr, &g) == MPATH_ERR_DEVICE);
            CHECK(g == nullptr);
        }
    }
    // ray counts and cast descriptors without a grid
    mpath_cast_desc cd;
    std::memset(&cd, 0, sizeof cd);
    const double obs[6] = {1, 2, 3, 4, 5, 6}, zs[2] = {0.5, 1.0};
    const int64_t first[2] = {0, 10}, count[2] = {5, 7};
    cd.n_obs = 2;
    cd.obs_pos = obs;
    cd.stop_value = zs;
    cd.nside = 4;
    cd.pix_first = first;
    cd.pix_count = count;
    cd.order = 1;
    cd.steps_per_cell = 4;
    cd.max_steps = 1000;
    int64_t nr = 0;
    CHECK(mpath_cast_count_rays(&cd, &nr) == MPATH_OK && nr == 12);
    CHECK(mpath_cast_workspace_bytes(nullptr, &cd, &bytes) == MPATH_ERR_INVALID_ARG);
    CHECK(mpath_cast_noalloc(nullptr, &cd, nullptr, nullptr) == MPATH_ERR_INVALID_ARG);
    CHECK(mpath_cast_jacobian_workspace_bytes(nullptr, &cd, &bytes) == MPATH_ERR_INVALID_ARG);
    CHECK(std::strcmp(mpath_status_string(MPATH_ERR_NOT_FULL_TREE), "not a full octree") == 0);
    CHECK(mpath_version() != nullptr);
    std::printf("abi driver ok\n");
    return 0;
}
