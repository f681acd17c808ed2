// julia_device.h -- layouts shared by the kernels and the host runtime of
// libjulia.so (internal; the public interface is include/julia.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jr {

enum { kFP64 = 0, kFP32 = 1, kFF = 2 };
enum { kModeJulia = 0, kModeMandelbrot = 1 };

// One frame of the device frame table (112 bytes).  Built on the host from a
// jr_frame: the mapping scalars hx, hy, cx, cy are computed there in binary64
// with the same expressions as in the header's pixel-centre formula.
struct alignas(16) DevFrame {
    double cr, ci;           // C (Julia mode)
    double cx, cy, hx, hy;   // pixel-centre mapping
    int64_t out_offset;      // element offset of pixel (0, 0) in the arena
    int64_t tile_begin;      // global index of this frame's first tile
    int32_t width, height;
    int32_t max_iter;
    int32_t dtype;           // kFP64 / kFP32 / kFF
    int32_t mode;            // kModeJulia / kModeMandelbrot
    int32_t defer;           // 1: escape absorbing over the whole frame
    int32_t row_begin, row_end;
    int32_t tiles_x;         // tiles per tile row of this frame
    int32_t tile_w, tile_h;
    int32_t claim;           // tiles taken per atomic claim while in this frame
};
static_assert(sizeof(DevFrame) == 112, "DevFrame layout");

struct PlainArgs {
    int32_t* out;
    double cr, ci, cx, cy, hx, hy;
    int32_t W, H, max_iter, mode;
};

hipError_t launch_persistent(int unroll, int dtmask, int blocks, const DevFrame* frames,
                             int nframes, int64_t total_tiles, int32_t* out_base,
                             unsigned long long* ctr, int refill, hipStream_t stream);
hipError_t launch_plain(int dtype, const PlainArgs& args, hipStream_t stream);
hipError_t launch_zero_counters(unsigned long long* ctr, hipStream_t stream);

}  // namespace jr
