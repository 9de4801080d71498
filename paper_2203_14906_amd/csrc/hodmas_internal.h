// Internal interface between the host plan code and the gfx950 kernels.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/hodmas.h"

namespace hodmas {

constexpr int kBlock = 256;                 // threads per workgroup of the batched kernels
constexpr int kMaxBlock = 512;              // per-frame kernel: 256 or 512 threads
constexpr int64_t kMaxLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950
// distinct power sums behind orders 1..6 in the all-orders kernel
constexpr int kOrderSums = 15;

// Everything one launch over one frame needs, passed by value as kernel
// arguments.  Positions are in samples of one-way flight (metres * fs / c).
struct FrameArgs {
    const hodmas_tile_desc* tiles;
    const hodmas_chan_entry* entries;
    const hodmas_stage_entry* stage;
    const void* rf;
    float* image;
    int64_t stride;          // elements between channel records
    int32_t n_samples;
    int32_t nx, nz;
    int32_t tile_x, split, chunk;
    int32_t n_tiles;
    int32_t n_elements;      // array elements (the coherence factor's N)
    int32_t block;           // threads per workgroup: tile_x * tile_z * split
    int32_t shift;           // 4: element pitch = 4 pixel columns, delays shared along translated pixels; else 0
    int32_t shift_iz0;       // ... in the tiles whose first row is at least this one
    int32_t shift_off;       // LDS byte offset of the rows' delay buffers (after the staged rows)
    double x0s, dxs, z0s, dzs;  // grid in samples
    float in_scale;          // stored value -> kernel value (int16: dequant / frame_max, else 1)
    float out_scale;         // kernel result -> image units (int16: frame_max, else 1)
};

// Output images of the all-orders kernel: img[k-1] receives order k.
struct OrderImages {
    float* img[HODMAS_MAX_ORDER];
};

// Work list of the persistent batched kernels (device memory).  Units are
// grouped by kind = (coherence weighting, order, storage type, pixels per
// delay: 1, or 2 for mirror pairs); kind k owns units [begin[k], end[k]).
constexpr int kBatchKinds = 2 * HODMAS_MAX_ORDER * 3 * 2;
constexpr int batch_kind(int order, int dtype, int pairing, int cf)
{
    return ((cf * HODMAS_MAX_ORDER + order - 1) * 3 + dtype) * 2 + pairing - 1;
}
constexpr int kind_order(int kind) { return kind / 6 % HODMAS_MAX_ORDER + 1; }
constexpr int kind_dtype(int kind) { return kind / 2 % 3; }
constexpr int kind_pairing(int kind) { return kind % 2 + 1; }
constexpr int kind_cf(int kind) { return kind / (6 * HODMAS_MAX_ORDER); }
static_assert(batch_kind(kind_order(kBatchKinds - 1), kind_dtype(kBatchKinds - 1), kind_pairing(kBatchKinds - 1),
                         kind_cf(kBatchKinds - 1)) == kBatchKinds - 1 &&
                  batch_kind(kind_order(40), kind_dtype(40), kind_pairing(40), kind_cf(40)) == 40,
              "kind decoding");

constexpr int kXcds = 8;                    // workgroup b runs on XCD b mod 8

// xcd[k][x] .. xcd[k][x+1]: the units of kind k (relative to begin[k]) that
// the workgroups on XCD x walk -- a run of neighbouring tiles of one or a few
// frames, so the RF and tables they read stay in that XCD's L2.
struct BatchHeader {
    int32_t n_units;
    int32_t n_frames;
    int32_t begin[kBatchKinds];
    int32_t end[kBatchKinds];
    int32_t xcd[kBatchKinds][kXcds + 1];
};

struct BatchFrame {
    FrameArgs args;
    int32_t order;
    int32_t dtype;
    int32_t pad[2];
};

// tile: the tile to form, or for a mirror-pair kind the pair's left tile
struct BatchUnit {
    int32_t frame;
    int32_t tile;
};

// Launch one frame on `stream`.  Returns hipSuccess or the launch error code.
// mirror: pair each tile of the grid's left half with its mirror image (grid
// n_tiles / 2); the plan has checked that the geometry allows it.
int launch_frame(const FrameArgs& a, int order, int dtype, bool compensated, bool coherence,
                 bool mirror, int64_t lds_bytes, void* stream);

constexpr uint32_t kPlanMagic = 0x484f444du;  // "HODM"

}  // namespace hodmas

// A plan: validated inputs, float64-derived host tables and their device copies.
struct hodmas_plan_s {
    uint32_t magic = hodmas::kPlanMagic;
    hodmas_geometry geom{};
    hodmas_grid grid{};
    hodmas_rf_desc rf{};
    int32_t max_order = 0;
    uint32_t flags = 0;
    hodmas_tiling tiling{};
    std::vector<double> elem_x;           // metres
    double x0s = 0, dxs = 0, z0s = 0, dzs = 0, t0s = 0;
    std::vector<hodmas_tile_desc> tiles;
    std::vector<hodmas_chan_entry> entries;
    std::vector<hodmas_stage_entry> stage;
    int32_t max_window = 0;
    int64_t lds_bytes = 0;
    float in_scale = 1.f, out_scale = 1.f;
    int32_t shift = 0, shift_iz0 = 0, shift_off = 0;   // FrameArgs::shift, ::shift_iz0, ::shift_off
    int64_t lds_unshared = 0;             // lds_bytes without the delay buffers
    int device = -1;
    hodmas_tile_desc* d_tiles = nullptr;
    hodmas_chan_entry* d_entries = nullptr;
    hodmas_stage_entry* d_stage = nullptr;
    int64_t table_bytes = 0;
};

namespace hodmas {

// Dynamic LDS of a launch of `plan` at `order`: the kernels share delays
// along translated pixels from order 2 on (at order 1 the buffer's round
// trip costs more than the delays it saves), so order 1 runs without the
// buffers.
inline int64_t launch_lds(const hodmas_plan_s* plan, int order)
{
    return plan->shift && order >= 2 ? plan->lds_bytes : plan->lds_unshared;
}

// Kernel arguments of one frame under `plan`.
FrameArgs frame_args(const hodmas_plan_s* plan, const void* rf_dev, float* image_dev);

// Orders 1..kmax of one frame in one pass.
int launch_orders(const FrameArgs& a, const OrderImages& out, int kmax, int dtype, bool compensated,
                  int64_t lds_bytes, void* stream);

// The persistent batched kernel of one kind (for graph nodes) and a launch of
// it.  Coherence-weighted kinds exist for compensated accumulation only
// (batch_kernel returns null for the others).
const void* batch_kernel(int kind, bool compensated);
int launch_batch(int kind, const BatchHeader* hdr, const BatchFrame* frames, const BatchUnit* units, int grid,
                 bool compensated, int64_t lds_bytes, void* stream);

}  // namespace hodmas
