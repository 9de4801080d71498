// Autotuner: times candidate tilings (tile shape, element split, LDS chunk) of
// a plan on the current device and keeps the fastest, cached in a JSON-lines
// file keyed by architecture, geometry, grid, RF layout, order and flags.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hodmas_internal.h"

namespace {

// Batch-mode timing: copies of the frame per persistent launch -- enough units
// (quarter-size tiles as the unit estimate) to fill the device, within an
// image budget.
constexpr int64_t kTuneBatchCopies = 256;
constexpr int64_t kTuneBatchUnits = 8192;
constexpr size_t kTuneImageBytes = size_t(256) << 20;

std::string tune_key(const char* arch, const hodmas_geometry* g, const hodmas_grid* gr,
                     const hodmas_rf_desc* rf, int32_t order, uint32_t flags)
{
    // element positions enter through a checksum of their bits
    unsigned long long h = 1469598103934665603ull;
    if (g->element_x_m) {
        for (int i = 0; i < g->n_elements; ++i) {
            unsigned long long b;
            std::memcpy(&b, &g->element_x_m[i], sizeof(b));
            h = (h ^ b) * 1099511628211ull;
        }
    }
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "%s|v2|n%d|p%.9g|c%.9g|fs%.9g|t0%.9g|x%016llx|g%dx%d|x0%.9g|dx%.9g|z0%.9g|dz%.9g|"
                  "dt%d|S%d|st%lld|k%d|f%u",
                  arch, g->n_elements, g->pitch_m, g->sound_speed_m_s, g->fs_hz, g->t0_s, h, gr->nx,
                  gr->nz, gr->x0_m, gr->dx_m, gr->z0_m, gr->dz_m, rf->dtype, rf->n_samples,
                  (long long)rf->channel_stride, order,
                  (unsigned)(flags & (HODMAS_FLAG_ACC_PLAIN | HODMAS_FLAG_TUNE_BATCH | HODMAS_FLAG_CF |
                                      HODMAS_FLAG_MIRROR)));
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, hodmas_tiling* out)
{
    if (!path)
        return false;
    FILE* f = std::fopen(path, "r");
    if (!f)
        return false;
    char line[1024];
    bool found = false;
    const std::string want = "{\"key\": \"" + key + "\", \"tiling\": [";
    while (std::fgets(line, sizeof(line), f)) {
        if (std::strncmp(line, want.c_str(), want.size()) != 0)
            continue;
        hodmas_tiling t;
        if (std::sscanf(line + want.size(), "%d, %d, %d, %d", &t.tile_x, &t.tile_z, &t.split, &t.chunk) == 4) {
            *out = t;  // the last entry for a key wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, const hodmas_tiling& t, double us)
{
    if (!path)
        return;
    FILE* f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f, "{\"key\": \"%s\", \"tiling\": [%d, %d, %d, %d], \"us\": %.3f}\n", key.c_str(), t.tile_x,
                 t.tile_z, t.split, t.chunk, us);
    std::fclose(f);
}

}  // namespace

extern "C" hodmas_status hodmas_autotune(const hodmas_geometry* geometry, const hodmas_grid* grid,
                                         const hodmas_rf_desc* rf, int32_t order, uint32_t flags,
                                         const char* cache_path, hodmas_tiling* out)
{
    if (!geometry || !grid || !rf || !out || order < 1 || order > HODMAS_MAX_ORDER)
        return HODMAS_EINVAL;
    if (flags & HODMAS_FLAG_HOST_ONLY)
        return HODMAS_EINVAL;
    int dev = -1;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return HODMAS_EDEVICE;
    const std::string key = tune_key(prop.gcnArchName, geometry, grid, rf, order, flags);
    if (cache_lookup(cache_path, key, out))
        return HODMAS_OK;

    static const hodmas_tiling kCandidates[] = {
        {16, 16, 1, 64}, {16, 16, 1, 128}, {32, 8, 1, 64},  {8, 32, 1, 64},  {16, 8, 2, 64},
        {8, 8, 4, 64},   {16, 16, 2, 64},  {32, 8, 2, 64},  {32, 16, 1, 64}, {16, 8, 4, 64},
        {16, 16, 1, 32}, {32, 8, 1, 32},   {16, 4, 4, 64},
    };
    // (coherence-weighted batch kinds exist for compensated sums only)
    const bool batch = (flags & HODMAS_FLAG_TUNE_BATCH) &&
                       !((flags & HODMAS_FLAG_CF) && (flags & HODMAS_FLAG_ACC_PLAIN));
    const size_t esz = rf->dtype == HODMAS_F32 ? 4 : 2;
    const size_t rf_bytes = esz * (size_t)rf->channel_stride * (size_t)geometry->n_elements;
    const size_t img_bytes = 4 * (size_t)grid->nx * (size_t)grid->nz;
    // A batch member is timed the way a batch runs it: enough copies of the
    // frame in one persistent launch to fill the device (a single small frame
    // would favour tilings that split elements for parallelism, which a
    // batch does not need), each copy with its own image.
    const int64_t tiles_x = (grid->nx + 7) / 8, tiles_z = (grid->nz + 7) / 8;
    const int copies = batch ? (int)std::max<int64_t>(
                                   1, std::min<int64_t>({kTuneBatchCopies, kTuneBatchUnits / std::max<int64_t>(
                                                                               1, tiles_x * tiles_z / 4),
                                                         (int64_t)(kTuneImageBytes / std::max<size_t>(img_bytes, 1))}))
                             : 1;
    void* d_rf = nullptr;
    float* d_img = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
        if (d_rf) (void)hipFree(d_rf);
        if (d_img) (void)hipFree(d_img);
    };
    // timing does not depend on sample values: a zero record suffices
    if (hipMalloc(&d_rf, rf_bytes) != hipSuccess || hipMalloc((void**)&d_img, img_bytes * copies) != hipSuccess ||
        hipMemset(d_rf, 0, rf_bytes) != hipSuccess || hipStreamCreate(&st) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return HODMAS_ENOMEM;
    }
    double best_us = 1e300;
    hodmas_tiling best{};
    for (const hodmas_tiling& cand : kCandidates) {
        if ((flags & HODMAS_FLAG_TUNE_BATCH) && cand.tile_x * cand.tile_z * cand.split != hodmas::kBlock)
            continue;   // members of a batch run 256-thread tiles
        hodmas_plan_t p = nullptr;
        if (hodmas_plan(geometry, grid, rf, order, flags & ~(HODMAS_FLAG_HOST_ONLY | HODMAS_FLAG_TUNE_BATCH),
                        &cand, &p) != HODMAS_OK)
            continue;
        bool ok = true;
        hodmas_batch_t bt = nullptr;
        if (batch) {
            hodmas_plan_info pi;
            ok = hodmas_plan_get_info(p, &pi) == HODMAS_OK &&
                 hodmas_batch_create(copies, (int64_t)pi.n_tiles * copies, pi.lds_bytes,
                                     flags & HODMAS_FLAG_ACC_PLAIN, &bt) == HODMAS_OK;
            if (ok) {
                std::vector<hodmas_plan_t> plans(copies, p);
                std::vector<const void*> rfs(copies, d_rf);
                std::vector<int32_t> orders(copies, order);
                std::vector<float*> imgs(copies);
                for (int c = 0; c < copies; ++c)
                    imgs[c] = d_img + (size_t)c * grid->nx * grid->nz;
                ok = hodmas_batch_set(bt, plans.data(), rfs.data(), orders.data(), imgs.data(), copies, st) ==
                     HODMAS_OK;
            }
        }
        auto run = [&]() {
            return batch ? hodmas_batch_launch(bt, st) == HODMAS_OK
                         : hodmas_beamform(p, d_rf, order, d_img, st) == HODMAS_OK;
        };
        for (int w = 0; w < 2 && ok; ++w)
            ok = run();
        std::vector<float> times;
        for (int r = 0; r < 5 && ok; ++r) {
            ok = hipEventRecord(e0, st) == hipSuccess && run() && hipEventRecord(e1, st) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.f;
            if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
                times.push_back(ms / copies);
        }
        if (bt)
            (void)hodmas_batch_destroy(bt);
        if (ok && hipStreamSynchronize(st) != hipSuccess)
            ok = false;
        hodmas_plan_info inf;
        if (ok && !times.empty() && hodmas_plan_get_info(p, &inf) == HODMAS_OK) {
            std::sort(times.begin(), times.end());
            const double us = 1e3 * times[times.size() / 2];
            if (us < best_us) {
                best_us = us;
                best = inf.tiling;   // the chunk may have been reduced to fit LDS
            }
        }
        (void)hodmas_destroy(p);
    }
    cleanup();
    if (best_us >= 1e300)
        return HODMAS_EUNSUPPORTED;
    *out = best;
    cache_store(cache_path, key, best, best_us);
    return HODMAS_OK;
}
