// Host-side driver for the sanitizer test: links the library's host sources
// (plan building, batch and autotuner argument handling) built with
// AddressSanitizer and UndefinedBehaviorSanitizer, and exercises every path
// that needs no GPU: host-only plans over many geometries, grids, tilings and
// flags (their tables are walked and checked), and the argument checks of
// every entry point.  The device launchers are stubs that abort: no path
// exercised here may reach them.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hodmas_internal.h"

namespace hodmas {
int launch_frame(const FrameArgs&, int, int, bool, bool, bool, int64_t, void*) { std::abort(); }
int launch_orders(const FrameArgs&, const OrderImages&, int, int, bool, int64_t, void*) { std::abort(); }
const void* batch_kernel(int, bool) { std::abort(); }
int launch_batch(int, const BatchHeader*, const BatchFrame*, const BatchUnit*, int, bool, int64_t, void*)
{
    std::abort();
}
}  // namespace hodmas

namespace {

int failures = 0;

void expect(bool ok, const char* what, int line)
{
    if (!ok) {
        std::fprintf(stderr, "FAILED line %d: %s\n", line, what);
        ++failures;
    }
}
#define EXPECT(c) expect((c), #c, __LINE__)

struct Case {
    int n;
    double pitch, t0;
    int nx, nz;
    double x0, dx, z0, dz;
    int S, dtype, max_order;
    hodmas_tiling tiling;
    uint32_t flags;
    bool irregular;
    bool ok;   // expected to plan
};

// Check the tables of a host-only plan: every tile covers its pixels, every
// entry's LDS offset lies in its slot's window row, stage entries are in
// element order, and the plan's LDS size holds the staged chunk.
void check_tables(hodmas_plan_t p, const Case& c)
{
    hodmas_plan_info inf;
    EXPECT(hodmas_plan_get_info(p, &inf) == HODMAS_OK);
    const hodmas_tile_desc* tiles = nullptr;
    const hodmas_chan_entry* ent = nullptr;
    const hodmas_stage_entry* st = nullptr;
    int32_t nt = 0;
    int64_t ne = 0;
    EXPECT(hodmas_plan_tables(p, &tiles, &ent, &st, &nt, &ne) == HODMAS_OK);
    EXPECT(nt == inf.n_tiles && ne == inf.active_pairs);
    std::vector<int> covered(size_t(c.nx) * c.nz, 0);
    const int chunk = inf.tiling.chunk;
    const int rows = (c.flags & HODMAS_FLAG_MIRROR) ? 2 : 1;
    EXPECT(int64_t(chunk) * inf.max_window * 4 * rows <= inf.lds_bytes);
    for (int t = 0; t < nt; ++t) {
        const hodmas_tile_desc& td = tiles[t];
        EXPECT(td.nx >= 1 && td.nz >= 1 && td.ix0 + td.nx <= c.nx && td.iz0 + td.nz <= c.nz);
        for (int z = td.iz0; z < td.iz0 + td.nz; ++z)
            for (int x = td.ix0; x < td.ix0 + td.nx; ++x)
                ++covered[size_t(z) * c.nx + x];
        EXPECT(td.n_active >= 0 && td.n_active <= c.n);
        EXPECT(td.window >= 2 && td.window <= inf.max_window);
        EXPECT(td.first_entry >= 0 && td.first_entry + td.n_active <= ne);
        for (int s = 0; s < td.n_active; ++s) {
            const hodmas_stage_entry& se = st[td.first_entry + s];
            EXPECT(se.channel >= 0 && se.channel < c.n);
            if (s > 0)
                EXPECT(se.channel > st[td.first_entry + s - 1].channel);
            const hodmas_chan_entry& e = ent[td.first_entry + s];
            EXPECT(e.channel >= 0 && e.channel < c.n);
            EXPECT(std::isfinite(e.a) && std::isfinite(e.d0sq) && e.d0 > 0.f && e.frac0 >= 0.f && e.frac0 <= 1.f);
            // the entry's offset, in floats, lies in the window part of some slot's
            // row of the chunk (rows of window + 2 floats)
            const int off = e.off / 4, stride = td.window + 2;
            EXPECT(e.off % 4 == 0 && off >= 0 && off < chunk * stride && off % stride < td.window);
        }
    }
    for (int v : covered)
        EXPECT(v == 1);
}

void run(const Case& c)
{
    std::vector<double> ex(c.n);
    for (int i = 0; i < c.n; ++i)
        ex[i] = (i - (c.n - 1) / 2.0) * c.pitch + (c.irregular ? 0.37 * c.pitch * std::sin(3.0 * i) : 0.0);
    hodmas_geometry g{c.n, c.pitch, 1540.0, 40e6, c.t0, c.irregular ? ex.data() : nullptr};
    hodmas_grid gr{c.nx, c.nz, c.x0, c.dx, c.z0, c.dz};
    hodmas_rf_desc rd{c.dtype, c.S, c.S, 1.0f / 8191.0f, 1.0f};
    hodmas_plan_t p = nullptr;
    const hodmas_status st =
        hodmas_plan(&g, &gr, &rd, c.max_order, c.flags | HODMAS_FLAG_HOST_ONLY, &c.tiling, &p);
    EXPECT((st == HODMAS_OK) == c.ok);
    if (st != HODMAS_OK) {
        EXPECT(p == nullptr);
        return;
    }
    check_tables(p, c);
    // a host-only plan refuses every device call before touching the device
    float* img = reinterpret_cast<float*>(0x1000);
    EXPECT(hodmas_beamform(p, img, 1, img, nullptr) == HODMAS_EINVAL);
    float* imgs[HODMAS_MAX_ORDER] = {img, img, img, img, img, img};
    EXPECT(hodmas_beamform_orders(p, img, 1, imgs, nullptr) == HODMAS_EINVAL);
    EXPECT(hodmas_destroy(p) == HODMAS_OK);
}

}  // namespace

int main()
{
    const hodmas_tiling deflt{0, 0, 0, 0};
    const double lam = 1540.0 / 40e6;
    std::vector<Case> cases = {
        // configs 1-3 and their default tilings
        {64, 0.3e-3, 0.0, 128, 128, -9.6e-3 + 0.075e-3, 0.15e-3, 0.078e-3, 0.156e-3, 1024, HODMAS_F32, 4, deflt, 0, false, true},
        {128, 0.3e-3, 0.0, 512, 512, -19.2e-3 + 0.0375e-3, 0.075e-3, 0.039e-3, 0.078e-3, 2048, HODMAS_F32, 6, deflt, 0, false, true},
        {256, 0.3e-3, 0.0, 1024, 1024, -38.4e-3 + 0.0375e-3, 0.075e-3, 0.02e-3, 0.039e-3, 2048, HODMAS_I16, 6, deflt, 0, false, true},
        // ragged grids, explicit tilings and small chunks, checks at the record ends
        {24, 0.3e-3, 0.0, 41, 37, -10e-3, 0.5e-3, 0.3e-3, 0.55e-3, 400, HODMAS_F32, 6, {16, 16, 1, 8}, 0, false, true},
        {16, 0.3e-3, 2e-6, 30, 50, -2.4e-3, 0.16e-3, 0.08e-3, 0.16e-3, 400, HODMAS_F16, 6, {16, 8, 2, 5}, 0, false, true},
        {13, 0.46e-3, 0.0, 19, 23, -2e-3, 0.21e-3, 0.5e-3, 0.33e-3, 400, HODMAS_F32, 3, {8, 8, 4, 3}, 0, true, true},
        {32, 0.3e-3, 0.0, 24, 24, -4.8e-3, 0.4e-3, 0.25e-3, 0.5e-3, 400, HODMAS_F32, 6, {32, 16, 1, 64}, HODMAS_FLAG_FORCE_CHECK, false, true},
        // flags: plain sums, coherence factor, mirror pairs (symmetric grids)
        {24, 0.3e-3, 0.0, 64, 45, -(63 / 2.0) * 0.16e-3, 0.16e-3, 0.2e-3, 0.3e-3, 330, HODMAS_F32, 6, {16, 16, 1, 8}, HODMAS_FLAG_MIRROR | HODMAS_FLAG_CF, false, true},
        {13, 0.3e-3, 0.0, 64, 53, -(63 / 2.0) * 0.17e-3, 0.17e-3, 0.2e-3, 0.21e-3, 300, HODMAS_F16, 6, {8, 8, 4, 3}, HODMAS_FLAG_MIRROR, false, true},
        {16, 0.3e-3, 0.0, 48, 40, -(47 / 2.0) * 0.15e-3, 0.15e-3, 0.2e-3, 0.25e-3, 512, HODMAS_F32, 6, deflt, HODMAS_FLAG_MIRROR | HODMAS_FLAG_ACC_PLAIN, false, true},
        // degenerate sizes
        {1, 0.3e-3, 0.0, 1, 1, 0.0, 0.1e-3, 3e-3, 0.1e-3, 256, HODMAS_F32, 6, deflt, 0, false, true},
        {16, 0.3e-3, 0.0, 1, 37, -0.3e-3, 0.2e-3, 3e-3, 0.15e-3, 400, HODMAS_F32, 6, deflt, 0, false, true},
        {16, 0.3e-3, 0.0, 53, 1, -0.3e-3, 0.2e-3, 3e-3, 0.15e-3, 400, HODMAS_F32, 6, {8, 8, 4, 5}, 0, false, true},
        {16, 0.3e-3, 0.0, 8, 8, -1e-3, 0.3e-3, 40e-3, 0.3e-3, 128, HODMAS_F32, 3, deflt, 0, false, true},   // nothing in the record
        {4096, 0.01e-3, 0.0, 40, 24, -1.5e-3, 0.075e-3, 5e-3, 0.075e-3, 2048, HODMAS_F32, 6, deflt, 0, false, true},
        {8, 0.3e-3, 0.0, 16384, 4, -8e-3, 1e-6, 2e-3, 0.075e-3, 512, HODMAS_F32, 6, deflt, 0, false, true},
        {8, 0.3e-3, 0.0, 24, 16, -1e-3, 0.075e-3, 10.0, 0.075e-3, 1 << 20, HODMAS_F32, 6, deflt, 0, false, true},
        // refused
        {0, 0.3e-3, 0.0, 8, 8, -1e-3, 0.3e-3, 1e-3, 0.3e-3, 128, HODMAS_F32, 3, deflt, 0, false, false},
        {16, 0.3e-3, 0.0, 8, 8, -1e-3, 0.3e-3, 1e-3, 0.3e-3, 128, HODMAS_F32, 7, deflt, 0, false, false},
        {16, 0.3e-3, 0.0, 8, 8, -1e-3, 0.3e-3, 0.0, 0.3e-3, 128, HODMAS_F32, 3, deflt, 0, false, false},
        {16, 0.3e-3, 0.0, 8, 8, -1e-3, 0.3e-3, 1e-3, 0.3e-3, 128, HODMAS_F32, 3, {16, 8, 1, 0}, 0, false, false},
        {16, 0.3e-3, 0.0, 4, 4, 0.0, 1e-4, 1e4, 1e-4, 256, HODMAS_F32, 3, deflt, 0, false, false},     // delays past 2^22
        {16, 0.3e-3, 0.0, 64, 40, -(63 / 2.0) * 0.15e-3 + 0.1 * lam, 0.15e-3, 1e-3, 0.2e-3, 512, HODMAS_F32, 3, deflt, HODMAS_FLAG_MIRROR, false, false},
        {16, 0.3e-3, 0.0, 60, 40, -(59 / 2.0) * 0.15e-3, 0.15e-3, 1e-3, 0.2e-3, 512, HODMAS_F32, 3, {16, 16, 1, 0}, HODMAS_FLAG_MIRROR, false, false},
        {16, 0.3e-3, 0.0, 64, 40, -(63 / 2.0) * 0.15e-3, 0.15e-3, 1e-3, 0.2e-3, 512, HODMAS_F32, 3, deflt, HODMAS_FLAG_MIRROR, true, false},
    };
    for (const Case& c : cases)
        run(c);

    // argument checks that return before any device call
    hodmas_plan_t out = nullptr;
    EXPECT(hodmas_plan(nullptr, nullptr, nullptr, 1, 0, nullptr, &out) == HODMAS_EINVAL);
    EXPECT(hodmas_plan(nullptr, nullptr, nullptr, 1, 0, nullptr, nullptr) == HODMAS_EINVAL);
    EXPECT(hodmas_destroy(nullptr) == HODMAS_OK);
    EXPECT(hodmas_beamform(nullptr, nullptr, 1, nullptr, nullptr) == HODMAS_EINVAL);
    EXPECT(hodmas_plan_get_info(nullptr, nullptr) == HODMAS_EINVAL);
    for (int s = 0; s <= HODMAS_EBUSY + 1; ++s)
        EXPECT(hodmas_status_string(static_cast<hodmas_status>(s)) != nullptr);
    EXPECT(hodmas_version() != nullptr);
    hodmas_batch_t b = nullptr;
    EXPECT(hodmas_batch_create(0, 10, 0, 0, &b) == HODMAS_EINVAL);
    EXPECT(hodmas_batch_create(4, 0, 0, 0, &b) == HODMAS_EINVAL);
    EXPECT(hodmas_batch_create(4, 10, -1, 0, &b) == HODMAS_EINVAL);
    EXPECT(hodmas_batch_create(4, 10, 0, 0x80, &b) == HODMAS_EINVAL);
    EXPECT(hodmas_batch_create(4, 10, 0, 0, nullptr) == HODMAS_EINVAL);
    EXPECT(hodmas_batch_set(nullptr, nullptr, nullptr, nullptr, nullptr, 1, nullptr) == HODMAS_EINVAL);
    EXPECT(hodmas_batch_launch(nullptr, nullptr) == HODMAS_EINVAL);
    EXPECT(hodmas_batch_capture(nullptr) == HODMAS_EINVAL);
    EXPECT(hodmas_batch_replay(nullptr, nullptr) == HODMAS_EINVAL);
    EXPECT(hodmas_batch_destroy(nullptr) == HODMAS_OK);
    hodmas_tiling t{};
    hodmas_geometry g{16, 0.3e-3, 1540.0, 40e6, 0.0, nullptr};
    hodmas_grid gr{8, 8, -1e-3, 0.3e-3, 1e-3, 0.3e-3};
    hodmas_rf_desc rd{HODMAS_F32, 128, 128, 1.0f, 1.0f};
    EXPECT(hodmas_autotune(nullptr, &gr, &rd, 1, 0, nullptr, &t) == HODMAS_EINVAL);
    EXPECT(hodmas_autotune(&g, &gr, &rd, 0, 0, nullptr, &t) == HODMAS_EINVAL);
    EXPECT(hodmas_autotune(&g, &gr, &rd, 1, HODMAS_FLAG_HOST_ONLY, nullptr, &t) == HODMAS_EINVAL);

    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host sanitizer driver: %zu plan cases ok\n", cases.size());
    return 0;
}
