// Batched form: a work list of (frame, tile) units over many frames, grouped by
// kind (order x storage type x mirror pairing x coherence weighting) and walked by one persistent
// kernel per kind; a HIP graph holds the kernels so one graph launch runs the
// batch.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "hodmas_internal.h"

using hodmas::BatchFrame;
using hodmas::BatchHeader;
using hodmas::BatchUnit;

namespace {

constexpr uint32_t kBatchMagic = 0x48424154u;  // "HBAT"
constexpr size_t kAlign = 256;
// Estimated VALU slots per pixel-element by order (delay, gather, root, sums):
// only used to order the work list, heaviest units first.
constexpr int64_t kSlots[7] = {0, 19, 25, 32, 32, 36, 38};
constexpr int64_t kCfSlots = 4;   // coherence weighting: two more compensated sums

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct hodmas_batch_s {
    uint32_t magic = kBatchMagic;
    int device = -1;
    int32_t max_frames = 0;
    int64_t max_units = 0;
    int64_t lds_bytes = 0;
    uint32_t flags = 0;
    int cus = 0;                          // compute units of the device
    int grid[hodmas::kBatchKinds] = {};   // persistent workgroups per kind at lds_bytes
    // the current work list's kinds: LDS of their largest member plan and the
    // persistent grid that LDS allows
    int64_t kind_lds[hodmas::kBatchKinds] = {};
    int kind_grid[hodmas::kBatchKinds] = {};
    // the last occupancy answer per kind (a serving loop sets a list per launch)
    int64_t occ_lds[hodmas::kBatchKinds] = {};
    int occ_per_cu[hodmas::kBatchKinds] = {};
    size_t off_frames = 0, off_units = 0, bytes = 0;
    char* d_buf = nullptr;
    char* h_buf = nullptr;           // pinned staging of the work list
    hipEvent_t copied = nullptr;     // last host->device copy of h_buf
    bool copy_pending = false;
    bool has_list = false;
    int32_t begin[hodmas::kBatchKinds] = {}, end[hodmas::kBatchKinds] = {};   // host copy of the ranges
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node[hodmas::kBatchKinds] = {};   // one kernel node per kind
    int node_grid[hodmas::kBatchKinds] = {};         // its current grid in `exec`
    int64_t node_lds[hodmas::kBatchKinds] = {};      // and its dynamic LDS
    bool node_on[hodmas::kBatchKinds] = {};          // enabled in `exec`
    hipEvent_t replayed = nullptr;   // the last replay's completion
    bool replay_pending = false;
    hipEvent_t launched = nullptr;   // the last direct launch's completion (destroy waits for it)
    hodmas_batch_info info{};
};

namespace {

void release(hodmas_batch_s* b)
{
    if (b->launched) {
        (void)hipEventSynchronize(b->launched);
        (void)hipEventDestroy(b->launched);
        b->launched = nullptr;
    }
    if (b->replayed) {
        (void)hipEventSynchronize(b->replayed);
        (void)hipEventDestroy(b->replayed);
    }
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->copied) {
        (void)hipEventSynchronize(b->copied);
        (void)hipEventDestroy(b->copied);
    }
    if (b->d_buf) (void)hipFree(b->d_buf);
    if (b->h_buf) (void)hipHostFree(b->h_buf);
    b->exec = nullptr;
    b->graph = nullptr;
    b->replayed = nullptr;
    b->copied = nullptr;
    b->d_buf = nullptr;
    b->h_buf = nullptr;
}

bool valid_batch(const hodmas_batch_s* b) { return b && b->magic == kBatchMagic; }

// Persistent workgroups a kind's kernel launches with: as many as its LDS lets
// the device hold, cut to its unit count.
int launch_grid(const hodmas_batch_s* b, int kind)
{
    return (int)std::min<int64_t>(b->kind_grid[kind], b->end[kind] - b->begin[kind]);
}

}  // namespace

extern "C" {

hodmas_status hodmas_batch_create(int32_t max_frames, int64_t max_units, int64_t max_lds_bytes,
                                  uint32_t flags, hodmas_batch_t* out)
{
    if (!out)
        return HODMAS_EINVAL;
    *out = nullptr;
    if (max_frames < 1 || max_units < 1 || max_units > (int64_t(1) << 31) || max_lds_bytes < 0 ||
        max_lds_bytes > hodmas::kMaxLdsBytes || (flags & ~HODMAS_FLAG_ACC_PLAIN))
        return HODMAS_EINVAL;
    hodmas_batch_s* b = new (std::nothrow) hodmas_batch_s;
    if (!b)
        return HODMAS_ENOMEM;
    b->max_frames = max_frames;
    b->max_units = max_units;
    b->lds_bytes = max_lds_bytes > 0 ? max_lds_bytes : 64 * 1024;
    b->flags = flags;
    const bool comp = !(flags & HODMAS_FLAG_ACC_PLAIN);
    hipDeviceProp_t prop;
    if (hipGetDevice(&b->device) != hipSuccess || hipGetDeviceProperties(&prop, b->device) != hipSuccess) {
        delete b;
        return HODMAS_EDEVICE;
    }
    int max_grid = 0;
    for (int kind = 0; kind < hodmas::kBatchKinds; ++kind) {
        const void* fn = hodmas::batch_kernel(kind, comp);
        if (!fn)
            continue;   // no such kind under this accumulation mode
        if (b->lds_bytes > 64 * 1024 &&
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_bytes) != hipSuccess) {
            (void)hipGetLastError();
            delete b;
            return HODMAS_EUNSUPPORTED;
        }
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, hodmas::kBlock, (size_t)b->lds_bytes) !=
                hipSuccess || per_cu < 1) {
            (void)hipGetLastError();
            delete b;
            return HODMAS_EUNSUPPORTED;
        }
        b->grid[kind] = per_cu * prop.multiProcessorCount;
        max_grid = std::max(max_grid, per_cu * prop.multiProcessorCount);
    }
    b->cus = prop.multiProcessorCount;
    b->off_frames = align_up(sizeof(BatchHeader));
    b->off_units = b->off_frames + align_up(sizeof(BatchFrame) * (size_t)max_frames);
    b->bytes = b->off_units + align_up(sizeof(BatchUnit) * (size_t)max_units);
    if (hipMalloc((void**)&b->d_buf, b->bytes) != hipSuccess ||
        hipHostMalloc((void**)&b->h_buf, b->bytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->copied, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->launched, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        release(b);
        delete b;
        return HODMAS_ENOMEM;
    }
    std::memset(b->h_buf, 0, b->bytes);
    if (hipMemcpy(b->d_buf, b->h_buf, b->bytes, hipMemcpyHostToDevice) != hipSuccess) {
        release(b);
        delete b;
        return HODMAS_EDEVICE;
    }
    b->info.grid = max_grid;
    b->info.lds_bytes = b->lds_bytes;
    *out = b;
    return HODMAS_OK;
}

hodmas_status hodmas_batch_set(hodmas_batch_t b, const hodmas_plan_t* plans, const void* const* rf,
                               const int32_t* orders, float* const* images, int32_t n_frames,
                               void* stream)
{
    if (!valid_batch(b) || !plans || !rf || !orders || !images || n_frames < 1 ||
        n_frames > b->max_frames)
        return HODMAS_EINVAL;
    struct Unit {
        int64_t cost;
        int32_t kind, frame, tile;
    };
    std::vector<Unit> units;
    int64_t pixch = 0;
    int64_t kl[hodmas::kBatchKinds] = {};   // LDS each kind's largest plan needs
    try {
        for (int32_t f = 0; f < n_frames; ++f) {
            const hodmas_plan_s* p = plans[f];
            if (!p || p->magic != hodmas::kPlanMagic || !rf[f] || !images[f])
                return HODMAS_EINVAL;
            if ((p->flags & HODMAS_FLAG_HOST_ONLY) || p->device != b->device)
                return HODMAS_EINVAL;
            if ((p->flags & HODMAS_FLAG_ACC_PLAIN) != (b->flags & HODMAS_FLAG_ACC_PLAIN))
                return HODMAS_EINVAL;
            const int cf = (p->flags & HODMAS_FLAG_CF) ? 1 : 0;
            if (cf && (b->flags & HODMAS_FLAG_ACC_PLAIN))
                return HODMAS_EUNSUPPORTED;   // coherence-weighted kinds accumulate compensated
            if (orders[f] < 1 || orders[f] > p->max_order)
                return HODMAS_EUNSUPPORTED;
            if (p->lds_bytes > b->lds_bytes)
                return HODMAS_EINVAL;
            if (p->tiling.tile_x * p->tiling.tile_z * p->tiling.split != hodmas::kBlock)
                return HODMAS_EINVAL;   // the persistent kernels run 256-thread tiles
            // a mirror plan's units are the pairs: each left-half tile with its mirror
            const int pairing = (p->flags & HODMAS_FLAG_MIRROR) ? 2 : 1;
            const int n_units = (int)p->tiles.size() / pairing;
            const int half = p->grid.nx / p->tiling.tile_x / 2;   // tile columns left of the centre
            if ((int64_t)units.size() + n_units > b->max_units)
                return HODMAS_EINVAL;
            pixch += int64_t(p->grid.nx) * p->grid.nz * p->geom.n_elements;
            const int kind = hodmas::batch_kind(orders[f], p->rf.dtype, pairing, cf);
            kl[kind] = std::max(kl[kind], hodmas::launch_lds(p, orders[f]));
            for (int i = 0; i < n_units; ++i) {
                const int t = pairing == 1 ? i : i / half * 2 * half + i % half;
                const hodmas_tile_desc& td = p->tiles[t];
                const int64_t pix = int64_t(td.nx) * td.nz;
                int64_t cost = pix;  // zero-fill only
                if (td.n_active >= orders[f])
                    cost = td.n_active * (pix * (kSlots[orders[f]] + kCfSlots * cf) + int64_t(td.window) * 2);
                units.push_back(Unit{cost, kind, f, (int32_t)t});
            }
        }
    } catch (const std::bad_alloc&) {
        return HODMAS_ENOMEM;
    }
    // Each kind runs with the LDS its own plans need, and as many persistent
    // workgroups as that LDS lets a CU hold: one large-LDS plan no longer
    // holds every other kind to its occupancy.
    int kg[hodmas::kBatchKinds] = {};
    const bool comp = !(b->flags & HODMAS_FLAG_ACC_PLAIN);
    for (int kind = 0; kind < hodmas::kBatchKinds; ++kind) {
        if (kl[kind] == 0)
            continue;
        if (b->occ_lds[kind] != kl[kind]) {
            const void* fn = hodmas::batch_kernel(kind, comp);
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, hodmas::kBlock, (size_t)kl[kind]) !=
                    hipSuccess || per_cu < 1) {
                (void)hipGetLastError();
                return HODMAS_EDEVICE;
            }
            b->occ_lds[kind] = kl[kind];
            b->occ_per_cu[kind] = per_cu;
        }
        kg[kind] = b->occ_per_cu[kind] * b->cus;
    }
    // grouped by kind (one persistent kernel each), in frame and tile order
    std::stable_sort(units.begin(), units.end(), [](const Unit& x, const Unit& y) { return x.kind < y.kind; });
    int32_t kb[hodmas::kBatchKinds] = {}, ke[hodmas::kBatchKinds] = {};
    for (size_t u = 0; u < units.size(); ++u) {
        const int k = units[u].kind;
        if (u == 0 || units[u - 1].kind != k)
            kb[k] = (int32_t)u;
        ke[k] = (int32_t)u + 1;
    }
    // Each kind's units, in frame and tile order (tile rows are depth bands),
    // are cut into one contiguous run per XCD that has workgroups, of about
    // equal estimated cost: an XCD then stages the RF of one frame, or of a
    // band of depths, and reads that frame's tables, instead of every XCD
    // fetching every frame.  Within a run the heaviest units go first.
    int32_t cuts[hodmas::kBatchKinds][hodmas::kXcds + 1] = {};
    try {
        std::vector<int64_t> pre;
        for (int k = 0; k < hodmas::kBatchKinds; ++k) {
            const int n = ke[k] - kb[k];
            if (n <= 0)
                continue;
            const int used = std::min<int>(hodmas::kXcds, (int)std::min<int64_t>(kg[k], n));
            Unit* run = units.data() + kb[k];
            pre.assign((size_t)n + 1, 0);
            for (int u = 0; u < n; ++u)
                pre[u + 1] = pre[u] + run[u].cost;
            int32_t* cut = cuts[k];
            for (int x = 1; x < used; ++x) {
                const int64_t target = pre[n] * x / used;
                int i = (int)(std::lower_bound(pre.begin(), pre.end(), target) - pre.begin());
                i = std::max(i, cut[x - 1] + 1);     // every XCD in use gets a unit
                i = std::min(i, n - (used - x));
                cut[x] = i;
            }
            for (int x = used; x <= hodmas::kXcds; ++x)
                cut[x] = n;
            for (int x = 0; x < used; ++x)
                std::stable_sort(run + cut[x], run + cut[x + 1],
                                 [](const Unit& a, const Unit& c) { return a.cost > c.cost; });
        }
    } catch (const std::bad_alloc&) {
        return HODMAS_ENOMEM;
    }
    // the pinned staging buffer may still feed the previous asynchronous copy
    if (b->copy_pending && hipEventSynchronize(b->copied) != hipSuccess)
        return HODMAS_EDEVICE;
    b->copy_pending = false;
    BatchHeader* hdr = reinterpret_cast<BatchHeader*>(b->h_buf);
    BatchFrame* frames = reinterpret_cast<BatchFrame*>(b->h_buf + b->off_frames);
    BatchUnit* list = reinterpret_cast<BatchUnit*>(b->h_buf + b->off_units);
    std::memset(hdr, 0, sizeof(BatchHeader));
    hdr->n_units = (int32_t)units.size();
    hdr->n_frames = n_frames;
    std::memcpy(hdr->begin, kb, sizeof(kb));
    std::memcpy(hdr->end, ke, sizeof(ke));
    std::memcpy(hdr->xcd, cuts, sizeof(cuts));
    std::memcpy(b->begin, hdr->begin, sizeof(b->begin));
    std::memcpy(b->end, hdr->end, sizeof(b->end));
    std::memcpy(b->kind_lds, kl, sizeof(kl));
    std::memcpy(b->kind_grid, kg, sizeof(kg));
    for (int32_t f = 0; f < n_frames; ++f) {
        std::memset(&frames[f], 0, sizeof(BatchFrame));
        frames[f].args = hodmas::frame_args(plans[f], rf[f], images[f]);
        frames[f].order = orders[f];
        frames[f].dtype = plans[f]->rf.dtype;
    }
    for (size_t u = 0; u < units.size(); ++u)
        list[u] = BatchUnit{units[u].frame, units[u].tile};
    const size_t used = b->off_units + sizeof(BatchUnit) * units.size();
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(b->d_buf, b->h_buf, used, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(b->copied, st) != hipSuccess) {
        (void)hipGetLastError();
        return HODMAS_EDEVICE;
    }
    b->copy_pending = true;
    b->has_list = true;
    b->info.n_frames = n_frames;
    b->info.n_units = (int64_t)units.size();
    b->info.pixel_channels = pixch;
    b->info.grid = *std::max_element(kg, kg + hodmas::kBatchKinds);
    b->info.lds_bytes = *std::max_element(kl, kl + hodmas::kBatchKinds);
    return HODMAS_OK;
}

hodmas_status hodmas_batch_launch(hodmas_batch_t b, void* stream)
{
    if (!valid_batch(b) || !b->has_list)
        return HODMAS_EINVAL;
    const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(b->d_buf);
    const BatchFrame* frames = reinterpret_cast<const BatchFrame*>(b->d_buf + b->off_frames);
    const BatchUnit* units = reinterpret_cast<const BatchUnit*>(b->d_buf + b->off_units);
    const bool comp = !(b->flags & HODMAS_FLAG_ACC_PLAIN);
    for (int kind = 0; kind < hodmas::kBatchKinds; ++kind) {
        if (b->end[kind] <= b->begin[kind])
            continue;
        if (hodmas::launch_batch(kind, hdr, frames, units, launch_grid(b, kind), comp, b->kind_lds[kind], stream) !=
            0) {
            (void)hipGetLastError();
            return HODMAS_EDEVICE;
        }
    }
    if (hipEventRecord(b->launched, static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return HODMAS_EDEVICE;
    }
    return HODMAS_OK;
}

}  // extern "C"

// The graph holds one node per kind of the work list it was captured for and
// no edges between them: kinds write disjoint images, so one kind's last
// units overlap the next kind's start instead of the GPU draining between
// kinds.  Each node reads its unit range from the device header, so a later
// hodmas_batch_set with the same kinds (or fewer) needs no re-capture; a set
// that brings a kind the graph lacks has the graph rebuilt at the next
// replay, with a node for every kind seen so far.  Nodes are not made for
// absent kinds: every node of a graph launch costs time even when switched
// off.  Before each replay the nodes are fitted to the current work list in
// the instantiated graph itself: a kind that is absent is switched off, and a
// present kind runs with the LDS its own plans need and the persistent grid
// that LDS allows, cut to its unit count.
namespace {

hipKernelNodeParams node_params(const hodmas_batch_s* b, int kind, int grid, int64_t lds, void** args)
{
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void*>(hodmas::batch_kernel(kind, !(b->flags & HODMAS_FLAG_ACC_PLAIN)));
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(hodmas::kBlock);
    kp.sharedMemBytes = (unsigned)lds;
    kp.kernelParams = args;
    kp.extra = nullptr;
    return kp;
}

// (Re)build the graph with a node for every kind in `want`.
bool build_graph(hodmas_batch_s* b, const bool* want)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(b->d_buf);
    const BatchFrame* frames = reinterpret_cast<const BatchFrame*>(b->d_buf + b->off_frames);
    const BatchUnit* units = reinterpret_cast<const BatchUnit*>(b->d_buf + b->off_units);
    void* args[] = {(void*)&hdr, (void*)&frames, (void*)&units};
    bool ok = hipGraphCreate(&b->graph, 0) == hipSuccess;
    for (int kind = 0; kind < hodmas::kBatchKinds && ok; ++kind) {
        b->node[kind] = nullptr;
        b->node_on[kind] = false;
        if (!want[kind] || !hodmas::batch_kernel(kind, !(b->flags & HODMAS_FLAG_ACC_PLAIN)))
            continue;   // not wanted, or no such kind under this accumulation mode
        const hipKernelNodeParams kp = node_params(b, kind, b->grid[kind], b->lds_bytes, args);
        hipGraphNode_t node = nullptr;
        ok = hipGraphAddKernelNode(&node, b->graph, nullptr, 0, &kp) == hipSuccess;
        b->node[kind] = node;
        b->node_grid[kind] = b->grid[kind];
        b->node_lds[kind] = b->lds_bytes;
        b->node_on[kind] = true;
    }
    if (ok)
        ok = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
    if (ok && !b->replayed)
        ok = hipEventCreateWithFlags(&b->replayed, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
        b->exec = nullptr;
        for (int kind = 0; kind < hodmas::kBatchKinds; ++kind)
            b->node[kind] = nullptr;
    }
    return ok;
}

}  // namespace

extern "C" {

hodmas_status hodmas_batch_capture(hodmas_batch_t b)
{
    if (!valid_batch(b))
        return HODMAS_EINVAL;
    if (b->exec)
        return HODMAS_OK;
    // the kinds of the current work list, or every kind before any list is set
    bool want[hodmas::kBatchKinds];
    for (int kind = 0; kind < hodmas::kBatchKinds; ++kind)
        want[kind] = !b->has_list || b->end[kind] > b->begin[kind];
    return build_graph(b, want) ? HODMAS_OK : HODMAS_EDEVICE;
}

hodmas_status hodmas_batch_replay(hodmas_batch_t b, void* stream)
{
    if (!valid_batch(b) || !b->exec || !b->has_list)
        return HODMAS_EINVAL;
    const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(b->d_buf);
    const BatchFrame* frames = reinterpret_cast<const BatchFrame*>(b->d_buf + b->off_frames);
    const BatchUnit* units = reinterpret_cast<const BatchUnit*>(b->d_buf + b->off_units);
    void* args[] = {(void*)&hdr, (void*)&frames, (void*)&units};
    // a launch of `exec` still in flight must not see its nodes change
    bool change = false, missing = false;
    for (int kind = 0; kind < hodmas::kBatchKinds; ++kind) {
        const int n = b->end[kind] - b->begin[kind];
        missing = missing || (n > 0 && !b->node[kind]);
        change = change || (n > 0) != b->node_on[kind] ||
                 (n > 0 && (launch_grid(b, kind) != b->node_grid[kind] ||
                            b->kind_lds[kind] != b->node_lds[kind]));
    }
    if ((change || missing) && b->replay_pending) {
        if (hipEventSynchronize(b->replayed) != hipSuccess) {
            (void)hipGetLastError();
            return HODMAS_EDEVICE;
        }
        b->replay_pending = false;
    }
    if (missing) {
        // a kind the graph has no node for: rebuild with every kind seen so far
        bool want[hodmas::kBatchKinds];
        for (int kind = 0; kind < hodmas::kBatchKinds; ++kind)
            want[kind] = b->node[kind] != nullptr || b->end[kind] > b->begin[kind];
        if (!build_graph(b, want))
            return HODMAS_EDEVICE;
        change = true;
    }
    for (int kind = 0; kind < hodmas::kBatchKinds && change; ++kind) {
        if (!b->node[kind])
            continue;
        const int n = b->end[kind] - b->begin[kind];
        const bool on = n > 0;
        if (on) {
            const int grid = launch_grid(b, kind);
            if (grid != b->node_grid[kind] || b->kind_lds[kind] != b->node_lds[kind]) {
                const hipKernelNodeParams kp = node_params(b, kind, grid, b->kind_lds[kind], args);
                if (hipGraphExecKernelNodeSetParams(b->exec, b->node[kind], &kp) != hipSuccess) {
                    (void)hipGetLastError();
                    return HODMAS_EDEVICE;
                }
                b->node_grid[kind] = grid;
                b->node_lds[kind] = b->kind_lds[kind];
            }
        }
        if (on != b->node_on[kind]) {
            if (hipGraphNodeSetEnabled(b->exec, b->node[kind], on ? 1 : 0) != hipSuccess) {
                (void)hipGetLastError();
                return HODMAS_EDEVICE;
            }
            b->node_on[kind] = on;
        }
    }
    if (hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)) != hipSuccess ||
        hipEventRecord(b->replayed, static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return HODMAS_EDEVICE;
    }
    b->replay_pending = true;
    return HODMAS_OK;
}

hodmas_status hodmas_batch_get_info(hodmas_batch_t b, hodmas_batch_info* info)
{
    if (!valid_batch(b) || !info)
        return HODMAS_EINVAL;
    *info = b->info;
    return HODMAS_OK;
}

hodmas_status hodmas_batch_destroy(hodmas_batch_t b)
{
    if (!b)
        return HODMAS_OK;
    if (b->magic != kBatchMagic)
        return HODMAS_EINVAL;
    release(b);
    b->magic = 0;
    delete b;
    return HODMAS_OK;
}

}  // extern "C"
