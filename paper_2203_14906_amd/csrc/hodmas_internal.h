// Internal interface between the host plan code and the gfx950 kernels.
#pragma once

#include <cstdint>
#include "../../include/hodmas.h"

namespace hodmas {

constexpr int kBlock = 256;                 // threads per workgroup (4 wave64)
constexpr int64_t kMaxLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950

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
    double x0s, dxs, z0s, dzs;  // grid in samples
    float in_scale;          // stored value -> kernel value (dequant / frame_max)
    float out_scale;         // frame_max: kernel result -> image units
};

// Launch one frame on `stream`.  Returns hipSuccess or the launch error code.
int launch_frame(const FrameArgs& a, int order, int dtype, bool compensated, int64_t lds_bytes,
                 void* stream);

}  // namespace hodmas
