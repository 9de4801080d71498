// Host side of the HO-DMAS library: argument validation, the float64 plan
// (per-tile delay anchors and LDS sample windows) and the C ABI entry points.
//
// The paper computes every (pixel, element) delay on the CPU before the kernel
// call and keeps it in GPU memory (Sec. V).  Here the plan keeps only one
// float64-derived anchor per (tile, element); the kernel rebuilds each pixel's
// delay from it in registers.  Per pixel this is t = T0 + frac0 + (d - d0) with
// d - d0 = (d^2 - d0^2) / (d + d0), which keeps the delay's rounding error
// proportional to the small in-tile offset instead of to the full flight time.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "hodmas_internal.h"

using hodmas::FrameArgs;

using hodmas::kPlanMagic;

namespace {

// Compute units of the MI355X, for the plan's estimate of workgroup rounds
// (hodmas_plan may run with no device: HODMAS_FLAG_HOST_ONLY).
constexpr int64_t kComputeUnits = 256;

// Rounds of workgroups a one-frame launch of `units` tiles needs over the
// CUs when each takes `lds` bytes of LDS and `block` threads (a CU holds at
// most 32 waves).
int64_t launch_rounds(int64_t units, int64_t lds, int64_t block)
{
    const int64_t by_waves = std::max<int64_t>(1, 32 / std::max<int64_t>(1, block / 64));
    const int64_t by_lds = std::max<int64_t>(1, hodmas::kMaxLdsBytes / std::max<int64_t>(lds, 1));
    const int64_t per_cu = std::min(by_waves, by_lds);
    return (units + per_cu * kComputeUnits - 1) / (per_cu * kComputeUnits);
}

constexpr uint32_t kMagic = kPlanMagic;
constexpr double kMaxDistanceSamples = 4194304.0;  // 2^22: delays stay exact-integer in float32

}  // namespace


namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

hodmas_status validate(const hodmas_geometry* g, const hodmas_grid* gr, const hodmas_rf_desc* rf,
                       int32_t max_order, const hodmas_tiling* t)
{
    if (!g || !gr || !rf)
        return HODMAS_EINVAL;
    if (g->n_elements < 1 || g->n_elements > HODMAS_MAX_ELEMENTS)
        return HODMAS_EINVAL;
    if (!finite_pos(g->sound_speed_m_s) || !finite_pos(g->fs_hz) || !std::isfinite(g->t0_s))
        return HODMAS_EINVAL;
    if (g->element_x_m) {
        for (int i = 0; i < g->n_elements; ++i)
            if (!std::isfinite(g->element_x_m[i]))
                return HODMAS_EINVAL;
    } else if (!finite_pos(g->pitch_m)) {
        return HODMAS_EINVAL;
    }
    if (gr->nx < 1 || gr->nz < 1 || gr->nx > HODMAS_MAX_GRID_SIDE || gr->nz > HODMAS_MAX_GRID_SIDE)
        return HODMAS_EINVAL;
    if (!std::isfinite(gr->x0_m) || !finite_pos(gr->dx_m) || !finite_pos(gr->z0_m) ||
        !finite_pos(gr->dz_m))
        return HODMAS_EINVAL;
    if (rf->dtype != HODMAS_F32 && rf->dtype != HODMAS_F16 && rf->dtype != HODMAS_I16)
        return HODMAS_EINVAL;
    if (rf->n_samples < 1 || rf->n_samples > HODMAS_MAX_SAMPLES || rf->channel_stride < rf->n_samples)
        return HODMAS_EINVAL;
    if (rf->channel_stride > (int64_t(1) << 40))
        return HODMAS_EINVAL;
    if (rf->dtype == HODMAS_I16 && !finite_pos(rf->dequant_scale))
        return HODMAS_EINVAL;
    if (!std::isfinite(rf->frame_max) || rf->frame_max < 0.f)
        return HODMAS_EINVAL;
    if (max_order < 1 || max_order > HODMAS_MAX_ORDER)
        return HODMAS_EINVAL;
    if (t) {
        bool any = t->tile_x || t->tile_z || t->split || t->chunk;
        if (any) {
            if (t->tile_x < 1 || t->tile_z < 1 || t->chunk < 0)
                return HODMAS_EINVAL;
            if (t->split != 1 && t->split != 2 && t->split != 4)
                return HODMAS_EINVAL;
            const int64_t block = int64_t(t->tile_x) * t->tile_z * t->split;
            if (block != hodmas::kBlock && block != hodmas::kMaxBlock)
                return HODMAS_EINVAL;
        }
    }
    return HODMAS_OK;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// LDS of one staged chunk: `chunk` rows (twice that with pairing) of the
// window and two more floats (after the first row's window: a pair of zeros,
// the target of delays outside the record).
int64_t row_stride(int64_t window) { return window + 2; }
int64_t staged_bytes(int64_t chunk, int64_t window, int rows) { return chunk * row_stride(window) * 4 * rows; }

// Mirror pairing needs whole tile columns, an even number of them.
bool mirror_columns(int32_t nx, int32_t tile_x) { return nx % tile_x == 0 && (nx / tile_x) % 2 == 0; }

// Library default: 16x16 pixel tiles; split the channels of a pixel over 2 or 4
// waves when the grid has too few tiles (pairs of tiles, when mirrored) to give
// every CU a few workgroups.  Mirrored grids that 16 does not divide into an
// even number of columns get 8-pixel-wide tiles.
hodmas_tiling default_tiling(const hodmas_grid& gr, bool mirror)
{
    const int64_t want = 2 * 256;  // two workgroups per CU
    const int per_wg = mirror ? 2 : 1;
    const int tx = (mirror && !mirror_columns(gr.nx, 16)) ? 8 : 16;
    const hodmas_tiling cand[2] = {{tx, 256 / tx, 1, 0}, {tx, 128 / tx, 2, 0}};
    for (const hodmas_tiling& t : cand)
        if (ceil_div(gr.nx, t.tile_x) * ceil_div(gr.nz, t.tile_z) / per_wg >= want)
            return t;
    return {tx, 64 / tx, 4, 0};
}

// The array and the grid are mirror images of themselves about x = 0, to
// `tol` metres.
bool symmetric(const hodmas_plan_s* p, double tol)
{
    const int n = p->geom.n_elements;
    for (int i = 0; i < n; ++i)
        if (!(std::fabs(p->elem_x[i] + p->elem_x[n - 1 - i]) <= tol))
            return false;
    return std::fabs(2.0 * p->grid.x0_m + (p->grid.nx - 1) * p->grid.dx_m) <= 2.0 * tol;
}

void free_device(hodmas_plan_s* p)
{
    if (p->d_tiles) (void)hipFree(p->d_tiles);
    if (p->d_entries) (void)hipFree(p->d_entries);
    if (p->d_stage) (void)hipFree(p->d_stage);
    p->d_tiles = nullptr;
    p->d_entries = nullptr;
    p->d_stage = nullptr;
}

// Build the per-tile tables in float64.  For every tile and element:
//   anchor delay ta = |anchor - element| - t0 (samples), T0 = floor(ta);
//   the delay range [tmin, tmax] over the tile's pixel rectangle (closed form:
//   nearest and farthest points of the rectangle), which bounds the LDS window;
//   elements whose whole range misses [0, S-1] are left out (they contribute 0).
hodmas_status build_tables(hodmas_plan_s* p)
{
    const hodmas_grid& gr = p->grid;
    const int n = p->geom.n_elements;
    const int S = p->rf.n_samples;
    const int tx = p->tiling.tile_x, tz = p->tiling.tile_z;
    const int ntx = (int)ceil_div(gr.nx, tx), ntz = (int)ceil_div(gr.nz, tz);
    const double lam = p->geom.sound_speed_m_s / p->geom.fs_hz;  // metres per sample
    p->x0s = gr.x0_m / lam;
    p->dxs = gr.dx_m / lam;
    p->z0s = gr.z0_m / lam;
    p->dzs = gr.dz_m / lam;
    p->t0s = p->geom.t0_s * p->geom.fs_hz;
    std::vector<double> xe(n);
    for (int i = 0; i < n; ++i)
        xe[i] = p->elem_x[i] / lam;

    // every delay must stay far inside float32's exact-integer range
    double xmin = *std::min_element(xe.begin(), xe.end()), xmax = *std::max_element(xe.begin(), xe.end());
    double gx_lo = p->x0s, gx_hi = p->x0s + (gr.nx - 1) * p->dxs;
    double gz_hi = p->z0s + (gr.nz - 1) * p->dzs;
    double far = std::sqrt(std::pow(std::max(std::fabs(gx_hi - xmin), std::fabs(gx_lo - xmax)), 2) +
                           gz_hi * gz_hi) + std::fabs(p->t0s);
    if (!(far < kMaxDistanceSamples))
        return HODMAS_EINVAL;

    try {
        p->tiles.assign((size_t)ntx * ntz, hodmas_tile_desc{});
        p->entries.clear();
        p->stage.clear();
        p->entries.reserve((size_t)ntx * ntz * n);
        p->stage.reserve((size_t)ntx * ntz * n);
    } catch (const std::bad_alloc&) {
        return HODMAS_ENOMEM;
    }
    // FP32 / FP16 rows are copied straight into LDS through one buffer
    // resource over the frame, whose range is a 32-bit byte count
    const int64_t esz = p->rf.dtype == HODMAS_F32 ? 4 : 2;
    const bool copies = p->rf.dtype == HODMAS_I16 ||
                        int64_t(n) * p->rf.channel_stride * esz < (int64_t(1) << 31);
    const int chunk = p->tiling.chunk;
    const int split = p->tiling.split;
    int32_t max_window = 2;
    std::vector<int32_t> T0(n), wlo(n), whi(n);
    std::vector<float> fr(n), aa(n), d0sq(n), d0(n);
    std::vector<char> act(n), chk(n);
    for (int bz = 0; bz < ntz; ++bz) {
        for (int bx = 0; bx < ntx; ++bx) {
            hodmas_tile_desc& td = p->tiles[(size_t)bz * ntx + bx];
            td.ix0 = bx * tx;
            td.iz0 = bz * tz;
            td.nx = std::min(tx, gr.nx - td.ix0);
            td.nz = std::min(tz, gr.nz - td.iz0);
            const int ia = td.ix0 + (td.nx - 1) / 2, ja = td.iz0 + (td.nz - 1) / 2;
            td.xa = p->x0s + ia * p->dxs;
            td.za = p->z0s + ja * p->dzs;
            const double xlo = p->x0s + td.ix0 * p->dxs, xhi = p->x0s + (td.ix0 + td.nx - 1) * p->dxs;
            const double zlo = p->z0s + td.iz0 * p->dzs, zhi = p->z0s + (td.iz0 + td.nz - 1) * p->dzs;
            int32_t window = 2;
            int32_t n_active = 0;
            bool check = (p->flags & HODMAS_FLAG_FORCE_CHECK) != 0;
            for (int i = 0; i < n; ++i) {
                const double a = td.xa - xe[i];
                const double sq = a * a + td.za * td.za;
                const double d = std::sqrt(sq);
                const double ta = d - p->t0s;
                const double fl = std::floor(ta);
                const double dxn = xe[i] < xlo ? xlo - xe[i] : (xe[i] > xhi ? xe[i] - xhi : 0.0);
                const double dxf = std::max(std::fabs(xlo - xe[i]), std::fabs(xhi - xe[i]));
                const double tmin = std::sqrt(dxn * dxn + zlo * zlo) - p->t0s;
                const double tmax = std::sqrt(dxf * dxf + zhi * zhi) - p->t0s;
                act[i] = !(tmax < 0.0 || tmin > double(S - 1));
                if (!act[i])
                    continue;
                ++n_active;
                chk[i] = (tmin < 0.5 || tmax > double(S - 1) - 0.5);
                check = check || chk[i];
                T0[i] = (int32_t)fl;
                fr[i] = (float)(ta - fl);
                aa[i] = (float)a;
                d0sq[i] = (float)sq;
                d0[i] = (float)d;
                wlo[i] = (int32_t)std::floor(tmin) - 1;
                whi[i] = (int32_t)std::floor(tmax) + 2;
                window = std::max(window, whi[i] - wlo[i] + 1);
            }
            // every staged row -- `window` samples from the element's first --
            // must lie inside the record for the untested path, which copies
            // FP32 and FP16 rows without bounds and tests no delay; so must
            // the whole record inside one 32-bit buffer range
            for (int i = 0; i < n && !check; ++i)
                check = act[i] && (wlo[i] < 0 || int64_t(wlo[i]) + window > S);
            check = check || !copies;
            td.n_active = n_active;
            td.window = window;
            td.check = check ? 1 : 0;
            td.first_entry = (int32_t)p->entries.size();
            max_window = std::max(max_window, window);
            // slots in element order; the LDS row of slot s starts at float (s % chunk) * (window + 2)
            std::vector<int> slot_elem;
            for (int i = 0; i < n; ++i)
                if (act[i])
                    slot_elem.push_back(i);
            for (int sl = 0; sl < n_active; ++sl) {
                const int i = slot_elem[sl];
                p->stage.push_back(hodmas_stage_entry{i, wlo[i]});
            }
            // per-element constants: within each chunk, the slots of split group g
            // (g, g+split, ...) are stored together, so a wave reads them in order
            for (int c0 = 0; c0 < n_active; c0 += chunk) {
                const int nch = std::min(chunk, n_active - c0);
                for (int g = 0; g < split; ++g) {
                    for (int sl = c0 + g; sl < c0 + nch; sl += split) {
                        const int i = slot_elem[sl];
                        hodmas_chan_entry e;
                        e.a = aa[i];
                        e.d0sq = d0sq[i];
                        e.d0 = d0[i];
                        e.frac0 = fr[i];
                        e.lo = (float)(-(double)T0[i]);
                        e.hi = (float)((double)(S - 1) - (double)T0[i]);
                        e.off = (int32_t)(4 * (T0[i] - wlo[i] + (sl % chunk) * row_stride(window)));
                        e.channel = i;
                        p->entries.push_back(e);
                    }
                }
            }
        }
    }
    p->max_window = max_window;
    return HODMAS_OK;
}

// Delays shared along translated pixels (unpaired, unweighted plans, in the
// tiles that stay inside the record): the element pitch is exactly four pixel
// columns of the grid, every tile is 16 columns wide and has one element group,
// and each tile's contributing elements are consecutive, in index order.
// The moved pixel's delay (four columns left of the tile's own pixels) is
// formed from the tile's anchor like the others; it stays as accurate only
// where the pixels lie deeper than a tile is wide, so tile rows above that
// depth compute every delay (shared_first_row).
int32_t shared_first_row(const hodmas_plan_s* p)
{
    const int tz = p->tiling.tile_z;
    int32_t r = 0;
    while (r < p->grid.nz && p->z0s + r * p->dzs < 16.0 * p->dxs)
        r += tz;
    return r;
}

int32_t shared_delay_step(const hodmas_plan_s* p)
{
    const int n = p->geom.n_elements;
    const double step = 4.0 * p->grid.dx_m;
    if ((p->flags & (HODMAS_FLAG_NO_SHARE | HODMAS_FLAG_MIRROR | HODMAS_FLAG_CF)) || p->tiling.tile_x != 16 ||
        p->tiling.split != 1 ||
        p->grid.nx % 16 != 0 || !(step > 0.0) || n < 2)
        return 0;
    for (int i = 0; i + 1 < n; ++i)
        if (!(std::fabs(p->elem_x[i + 1] - p->elem_x[i] - step) <= 1e-12 * step))
            return 0;
    for (const hodmas_tile_desc& td : p->tiles)
        for (int sl = 1; sl < td.n_active; ++sl)
            if (p->stage[(size_t)td.first_entry + sl].channel != p->stage[(size_t)td.first_entry + sl - 1].channel + 1)
                return 0;
    return 4;
}

hodmas_status upload(hodmas_plan_s* p)
{
    if (hipGetDevice(&p->device) != hipSuccess)
        return HODMAS_EDEVICE;
    size_t tb = p->tiles.size() * sizeof(hodmas_tile_desc);
    size_t eb = std::max<size_t>(p->entries.size(), 1) * sizeof(hodmas_chan_entry);
    size_t sb = std::max<size_t>(p->stage.size(), 1) * sizeof(hodmas_stage_entry);
    if (hipMalloc((void**)&p->d_tiles, tb) != hipSuccess ||
        hipMalloc((void**)&p->d_entries, eb) != hipSuccess ||
        hipMalloc((void**)&p->d_stage, sb) != hipSuccess) {
        free_device(p);
        (void)hipGetLastError();
        return HODMAS_ENOMEM;
    }
    if (hipMemcpy(p->d_tiles, p->tiles.data(), tb, hipMemcpyHostToDevice) != hipSuccess ||
        (!p->entries.empty() &&
         hipMemcpy(p->d_entries, p->entries.data(), p->entries.size() * sizeof(hodmas_chan_entry),
                   hipMemcpyHostToDevice) != hipSuccess) ||
        (!p->stage.empty() &&
         hipMemcpy(p->d_stage, p->stage.data(), p->stage.size() * sizeof(hodmas_stage_entry),
                   hipMemcpyHostToDevice) != hipSuccess)) {
        free_device(p);
        (void)hipGetLastError();
        return HODMAS_EDEVICE;
    }
    p->table_bytes = (int64_t)(tb + eb + sb);
    return HODMAS_OK;
}

}  // namespace

extern "C" {

hodmas_status hodmas_plan(const hodmas_geometry* geometry, const hodmas_grid* grid,
                          const hodmas_rf_desc* rf, int32_t max_order, uint32_t flags,
                          const hodmas_tiling* tiling, hodmas_plan_t* out)
{
    if (!out)
        return HODMAS_EINVAL;
    *out = nullptr;
    hodmas_status st = validate(geometry, grid, rf, max_order, tiling);
    if (st != HODMAS_OK)
        return st;
    hodmas_plan_s* p = new (std::nothrow) hodmas_plan_s;
    if (!p)
        return HODMAS_ENOMEM;
    p->geom = *geometry;
    p->geom.element_x_m = nullptr;
    p->grid = *grid;
    p->rf = *rf;
    p->max_order = max_order;
    p->flags = flags;
    try {
        p->elem_x.resize(geometry->n_elements);
    } catch (const std::bad_alloc&) {
        delete p;
        return HODMAS_ENOMEM;
    }
    for (int i = 0; i < geometry->n_elements; ++i)
        p->elem_x[i] = geometry->element_x_m
                           ? geometry->element_x_m[i]
                           : (i - (geometry->n_elements - 1) / 2.0) * geometry->pitch_m;
    bool given = tiling && (tiling->tile_x || tiling->tile_z || tiling->split || tiling->chunk);
    const bool mirror = (flags & HODMAS_FLAG_MIRROR) != 0;
    p->tiling = given ? *tiling : default_tiling(*grid, mirror);
    if (mirror) {
        const double lam = geometry->sound_speed_m_s / geometry->fs_hz;
        if (!mirror_columns(grid->nx, p->tiling.tile_x) || !symmetric(p, 1e-6 * lam)) {
            delete p;
            return HODMAS_EINVAL;
        }
    }
    const int rows = mirror ? 2 : 1;   // LDS rows per staged slot (own, mirrored)
    // chunk 0: every element at once for now; the windows (which do not depend
    // on the chunk) then decide how many fit the LDS budget
    const bool auto_chunk = p->tiling.chunk == 0;
    if (auto_chunk)
        p->tiling.chunk = std::max(1, geometry->n_elements);
    st = build_tables(p);
    if (st != HODMAS_OK) {
        delete p;
        return st;
    }
    // LDS: `chunk` windows of `max_window` floats and a pair of zeros (the
    // target of delays outside the record), per row set; shrink the chunk
    // until it fits.
    const int64_t block = int64_t(p->tiling.tile_x) * p->tiling.tile_z * p->tiling.split;
    // split-group combination: (sum, compensation) of up to MAX_ORDER power
    // sums plus the two coherence-factor sums per pixel, for each of `rows`
    // pixels per lane, plus one padding float (an odd stride across lanes)
    const int64_t reduce_bytes = int64_t(block / p->tiling.split) * (p->tiling.split - 1) *
                                 ((HODMAS_MAX_ORDER + 2) * 2 * rows + 1) * 4;
    // 40 KB keeps four workgroups on a CU (160 KB); an explicit chunk may use 64 KB
    int64_t cap = auto_chunk ? 40 * 1024 : 64 * 1024;
    if (staged_bytes(1, p->max_window, rows) > hodmas::kMaxLdsBytes) {
        delete p;
        return HODMAS_EUNSUPPORTED;
    }
    // A grid with more workgroups than one round over the CUs at that size
    // (1024^2: 4096 tiles, or 2048 mirror pairs) takes chunks of at most 20 KB
    // instead when that needs fewer rounds: eight workgroups per CU, the most
    // a CU holds, outweigh the extra staging rounds (measured 2-16 % faster
    // per frame at 1024^2).
    if (auto_chunk) {
        const int64_t units = int64_t(p->tiles.size()) / rows;   // a mirror pair is one workgroup
        const int64_t row_bytes = int64_t(row_stride(p->max_window)) * 4;
        auto lds_at = [&](int64_t c) {
            const int64_t cc = ceil_div(p->tiling.chunk, ceil_div(p->tiling.chunk, c));   // equal chunks
            return std::max(staged_bytes((int)cc, p->max_window, rows), reduce_bytes);
        };
        const int64_t at40 = lds_at(std::max<int64_t>(1, cap / row_bytes));
        const int64_t at20 = lds_at(std::max<int64_t>(1, 20 * 1024 / row_bytes));
        if (launch_rounds(units, at20, block) < launch_rounds(units, at40, block))
            cap = 20 * 1024;
    }
    if (staged_bytes(p->tiling.chunk, p->max_window, rows) > cap) {
        const int c = (int)std::max<int64_t>(1, cap / (row_stride(p->max_window) * 4 * rows));
        // as many chunks as the cap needs, of equal size: no short last chunk
        // pays a full staging round, and the smaller LDS footprint can keep
        // more workgroups on a CU
        const int n_chunks = (int)ceil_div(p->tiling.chunk, c);
        p->tiling.chunk = (int)ceil_div(p->tiling.chunk, n_chunks);
        st = build_tables(p);  // entry offsets depend on the chunk
        if (st != HODMAS_OK) {
            delete p;
            return st;
        }
    }
    p->lds_bytes = std::max<int64_t>(staged_bytes(p->tiling.chunk, p->max_window, rows), reduce_bytes);
    // int16: dequantised codes are normalised by frame_max and the result
    // scaled back; FP32 and FP16 samples are used as stored (e_k is of degree
    // one in the samples), so the kernel may copy their rows into LDS untouched
    const double fm = rf->frame_max > 0.f && rf->dtype == HODMAS_I16 ? (double)rf->frame_max : 1.0;
    const double dq = rf->dtype == HODMAS_I16 ? (double)rf->dequant_scale : 1.0;
    p->in_scale = (float)(dq / fm);
    p->out_scale = (float)fm;
    p->shift = shared_delay_step(p);
    p->shift_iz0 = shared_first_row(p);
    p->lds_unshared = p->lds_bytes;
    if (p->shift) {
        // each row of 16 lanes passes delays through 32 (4 floor(delay), fraction)
        // entries, the rows 48 entries apart (no LDS bank shared by two rows)
        const int32_t off = (int32_t)((staged_bytes(p->tiling.chunk, p->max_window, rows) + 7) / 8 * 8);
        const int64_t with = std::max<int64_t>(p->lds_bytes, off + block / 16 * 48 * 8);
        // The buffers take LDS; where that leaves fewer workgroups per CU and a
        // one-frame launch then needs more rounds of workgroups over the CUs
        // (a 1024^2 grid: 16 tiles per CU, 3 rounds at 6 per CU, 4 at 5), the
        // lost round costs more than the shared delays save: keep every delay.
        const int64_t n_tiles = (int64_t)p->tiles.size();
        if (launch_rounds(n_tiles, with, block) <= launch_rounds(n_tiles, p->lds_bytes, block)) {
            p->shift_off = off;
            p->lds_bytes = with;
        } else {
            p->shift = 0;
        }
    }
    if (!(flags & HODMAS_FLAG_HOST_ONLY)) {
        st = upload(p);
        if (st != HODMAS_OK) {
            delete p;
            return st;
        }
    }
    *out = p;
    return HODMAS_OK;
}

}  // extern "C"

FrameArgs hodmas::frame_args(const hodmas_plan_s* plan, const void* rf_dev, float* image_dev)
{
    FrameArgs a;
    a.tiles = plan->d_tiles;
    a.entries = plan->d_entries;
    a.stage = plan->d_stage;
    a.rf = rf_dev;
    a.image = image_dev;
    a.stride = plan->rf.channel_stride;
    a.n_samples = plan->rf.n_samples;
    a.nx = plan->grid.nx;
    a.nz = plan->grid.nz;
    a.tile_x = plan->tiling.tile_x;
    a.split = plan->tiling.split;
    a.chunk = plan->tiling.chunk;
    a.n_tiles = (int32_t)plan->tiles.size();
    a.n_elements = plan->geom.n_elements;
    a.block = plan->tiling.tile_x * plan->tiling.tile_z * plan->tiling.split;
    a.x0s = plan->x0s;
    a.dxs = plan->dxs;
    a.z0s = plan->z0s;
    a.dzs = plan->dzs;
    a.in_scale = plan->in_scale;
    a.out_scale = plan->out_scale;
    a.shift = plan->shift;
    a.shift_iz0 = plan->shift_iz0;
    a.shift_off = plan->shift_off;
    return a;
}

extern "C" {

hodmas_status hodmas_beamform(hodmas_plan_t plan, const void* rf_dev, int32_t order,
                              float* image_dev, void* stream)
{
    if (!plan || plan->magic != kMagic || !rf_dev || !image_dev)
        return HODMAS_EINVAL;
    if (plan->flags & HODMAS_FLAG_HOST_ONLY)
        return HODMAS_EINVAL;
    if (order < 1 || order > plan->max_order || order > HODMAS_MAX_ORDER)
        return HODMAS_EUNSUPPORTED;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess)
        return HODMAS_EDEVICE;
    if (cur != plan->device && hipSetDevice(plan->device) != hipSuccess)
        return HODMAS_EDEVICE;
    const FrameArgs a = hodmas::frame_args(plan, rf_dev, image_dev);
    const bool comp = !(plan->flags & HODMAS_FLAG_ACC_PLAIN);
    const bool cf = (plan->flags & HODMAS_FLAG_CF) != 0;
    const bool mirror = (plan->flags & HODMAS_FLAG_MIRROR) != 0;
    int rc = hodmas::launch_frame(a, order, plan->rf.dtype, comp, cf, mirror, hodmas::launch_lds(plan, order),
                                  stream);
    if (cur != plan->device)
        (void)hipSetDevice(cur);
    return rc == 0 ? HODMAS_OK : HODMAS_EDEVICE;
}

hodmas_status hodmas_beamform_orders(hodmas_plan_t plan, const void* rf_dev, int32_t max_order,
                                     float* const* images_dev, void* stream)
{
    if (!plan || plan->magic != kMagic || !rf_dev || !images_dev)
        return HODMAS_EINVAL;
    if (plan->flags & HODMAS_FLAG_HOST_ONLY)
        return HODMAS_EINVAL;
    if (max_order < 1 || max_order > plan->max_order || max_order > HODMAS_MAX_ORDER ||
        (plan->flags & HODMAS_FLAG_CF))
        return HODMAS_EUNSUPPORTED;
    hodmas::OrderImages out{};
    for (int k = 0; k < max_order; ++k) {
        if (!images_dev[k])
            return HODMAS_EINVAL;
        out.img[k] = images_dev[k];
    }
    // LDS: the staged windows, or the cross-group combination of the power sums
    const int64_t nt = hodmas::kOrderSums;
    const int64_t block = int64_t(plan->tiling.tile_x) * plan->tiling.tile_z * plan->tiling.split;
    const int64_t reduce = block / plan->tiling.split * (plan->tiling.split - 1) * (2 * nt + 1) * 4;
    const int64_t lds = std::max<int64_t>(staged_bytes(plan->tiling.chunk, plan->max_window, 1), reduce);
    if (lds > 64 * 1024)
        return HODMAS_EUNSUPPORTED;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess)
        return HODMAS_EDEVICE;
    if (cur != plan->device && hipSetDevice(plan->device) != hipSuccess)
        return HODMAS_EDEVICE;
    const FrameArgs a = hodmas::frame_args(plan, rf_dev, nullptr);
    const bool comp = !(plan->flags & HODMAS_FLAG_ACC_PLAIN);
    int rc = hodmas::launch_orders(a, out, max_order, plan->rf.dtype, comp, lds, stream);
    if (cur != plan->device)
        (void)hipSetDevice(cur);
    return rc == 0 ? HODMAS_OK : HODMAS_EDEVICE;
}

hodmas_status hodmas_sync(void* stream)
{
    const hipError_t a = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    const hipError_t b = hipGetLastError();   // also clears a sticky launch error
    return a == hipSuccess && b == hipSuccess ? HODMAS_OK : HODMAS_EDEVICE;
}

hodmas_status hodmas_destroy(hodmas_plan_t plan)
{
    if (!plan)
        return HODMAS_OK;
    if (plan->magic != kMagic)
        return HODMAS_EINVAL;
    int cur = -1;
    bool switched = false;
    if (plan->d_tiles && hipGetDevice(&cur) == hipSuccess && cur != plan->device)
        switched = hipSetDevice(plan->device) == hipSuccess;
    free_device(plan);
    if (switched)
        (void)hipSetDevice(cur);
    plan->magic = 0;
    delete plan;
    return HODMAS_OK;
}

const char* hodmas_status_string(hodmas_status s)
{
    switch (s) {
    case HODMAS_OK: return "ok";
    case HODMAS_EINVAL: return "invalid argument";
    case HODMAS_ENOMEM: return "out of memory";
    case HODMAS_EDEVICE: return "HIP device error";
    case HODMAS_EUNSUPPORTED: return "unsupported request";
    case HODMAS_EBUSY: return "busy";
    }
    return "unknown status";
}

hodmas_status hodmas_plan_get_info(hodmas_plan_t plan, hodmas_plan_info* info)
{
    if (!plan || plan->magic != kMagic || !info)
        return HODMAS_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->n_elements = plan->geom.n_elements;
    info->n_samples = plan->rf.n_samples;
    info->nx = plan->grid.nx;
    info->nz = plan->grid.nz;
    info->max_order = plan->max_order;
    info->dtype = plan->rf.dtype;
    info->tiling = plan->tiling;
    info->n_tiles = (int32_t)plan->tiles.size();
    info->max_window = plan->max_window;
    info->active_pairs = (int64_t)plan->entries.size();
    info->lds_bytes = plan->lds_bytes;
    info->table_bytes = plan->table_bytes;
    info->flags = plan->flags;
    if (plan->shift)
        info->flags |= HODMAS_INFO_SHARED_DELAYS;
    return HODMAS_OK;
}

hodmas_status hodmas_plan_tables(hodmas_plan_t plan, const hodmas_tile_desc** tiles,
                                 const hodmas_chan_entry** entries,
                                 const hodmas_stage_entry** stage, int32_t* n_tiles,
                                 int64_t* n_entries)
{
    if (!plan || plan->magic != kMagic || !tiles || !entries || !stage || !n_tiles || !n_entries)
        return HODMAS_EINVAL;
    *tiles = plan->tiles.data();
    *entries = plan->entries.data();
    *stage = plan->stage.data();
    *n_tiles = (int32_t)plan->tiles.size();
    *n_entries = (int64_t)plan->entries.size();
    return HODMAS_OK;
}

const char* hodmas_version(void) { return "hodmas 0.1 (gfx950)"; }

}  // extern "C"
