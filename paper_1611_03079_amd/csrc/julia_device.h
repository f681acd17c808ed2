// julia_device.h -- layouts shared by the kernels and the host runtime of
// libjulia.so (internal; the public interface is include/julia.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jr {

enum { kFP64 = 0, kFP32 = 1, kFF = 2 };
enum { kModeJulia = 0, kModeMandelbrot = 1 };

enum { kMapPoly = 0, kMapRational = 1 };

// One frame of the device frame table (144 bytes).  Built on the host from a
// jr_frame: the mapping scalars hx, hy, cx, cy are computed there in binary64
// with the same expressions as in the header's pixel-centre formula.
struct alignas(16) DevFrame {
    double cr, ci;           // C (Julia mode)
    double cx, cy, hx, hy;   // pixel-centre mapping
    int64_t out_offset;      // element offset of pixel (0, 0) in the arena
    int64_t tile_begin;      // global index of this frame's first tile
    double lr, li;           // lambda of the rational map (kMapRational)
    int32_t width, height;
    int32_t max_iter;
    int32_t dtype;           // kFP64 / kFP32 / kFF
    int32_t mode;            // kModeJulia / kModeMandelbrot
    int32_t defer;           // 1: escape absorbing over the whole frame
    int32_t row_begin, row_end;
    int32_t tiles_x;         // tiles per tile row of this frame
    int32_t tile_w, tile_h;
    int32_t degree;          // map Z^degree + C (2: the quadratic map)
    int32_t map;             // kMapPoly, or kMapRational: Z^degree + C + lambda / Z^degree
    int32_t index;           // the frame's position in the caller's list (progress counters)
    int32_t reserved[2];
};
static_assert(sizeof(DevFrame) == 144, "DevFrame layout");

// Work queues of the persistent kernel.  Same-address device-scope atomics
// serialise (about 12 ns each on MI355X), so the tile counter is split into
// kQueues counters on separate 4 KiB lines: granule u (a run of `granule`
// consecutive tiles) belongs to queue u % kQueues.
constexpr int kQueues = 64;
constexpr int kQueueStride = 512;  // u64 elements between two counters (4 KiB)
constexpr size_t kCounterBytes = (size_t)kQueues * kQueueStride * sizeof(unsigned long long);

struct PersistentArgs {
    DevFrame frame0;         // the frame itself when frames == nullptr (one-frame launches)
    const DevFrame* frames;  // device frame table, or nullptr: use frame0
    int32_t* out_base;
    unsigned long long* ctr;
    int64_t total_tiles;
    int64_t granules;
    int32_t nframes;
    int32_t granule;     // tiles per granule
    int32_t refill;
    int32_t persistent;  // 1: work queues; 0: one wave per tile
    int32_t hybrid;      // 1: fresh packets + survivor queue (run_hybrid)
    int32_t bail;        // hybrid: iterations of a fresh packet before its survivors park;
                         // rows: length of the first counted block of every row
    int32_t rows;        // 1: two-phase row-packet kernel (jr_rows)
    int32_t handoff;     // rows: a row group leaves its first block once at most
                         // this many of its pixels are still inside
    int32_t palette_len; // > 0: a pixel stores palette[min(count, palette_len - 1)]
    const uint32_t* palette;
    // Progress (rows and plain kernels; both null otherwise): done[f] gains
    // the pixel count of each tile of frame f once all of them are stored;
    // a nonzero *stop makes waves claim no further tiles.
    int32_t* done;
    const int32_t* stop;
};

// Largest colour table of the fused colour store; it is staged in LDS.
constexpr int kPaletteMax = 8192;
// Row-packet kernel: a wave's survivor list holds this many rows' worth of
// pixels (64 each): 8 for FP32-only launches (512 entries, 5 KiB of LDS per
// wave, so 32 one-wave workgroups fit a CU), 4 when FP64, float-float or
// general-map frames are in (4.5 KiB).  The list is drained whenever it could
// not take the next group's survivors, so tiles may be taller than the list.
constexpr int kRowsFP32 = 8;
constexpr int kRowsWide = 4;
// Rows per group in the rows kernel's first phase for FP32 (FP64 takes 2).
constexpr int kGroupFP32 = 4;
// Largest palette (entries) that one-wave workgroups of the rows kernel stage
// each for themselves; larger palettes keep four-wave workgroups.
constexpr int kOneWavePalette = 256;
// Kernel variants that store colours carry this bit beside the dtype bits
// (compile-time, so the counting kernels hold no colour code).
constexpr int kColorBit = 8;
// Kernel variants that also hold the general maps Z^d + C (d = 3..8).
constexpr int kGeneralBit = 16;
// Kernel variants (rows and plain kernels only) that also hold the rational
// maps Z^d + C + lambda / Z^d; they carry kGeneralBit too.
constexpr int kRationalBit = 32;
// Kernel variants (rows and plain kernels, every map and dtype) that keep
// progress: the stop flag and the per-frame done counters.  Launches without
// progress run variants that hold no progress code at all.
constexpr int kProgressBit = 64;

struct PlainArgs {
    int32_t* out;
    double cr, ci, cx, cy, hx, hy;
    int32_t W, H, max_iter, mode;
};

// Allocation-free batch launches (julia_render_batch_noalloc) keep the queue
// counters and the frame table in one fixed device array of the library, the
// counters first (kCounterBytes), then room for kNoAllocMaxFrames frames.
constexpr int kNoAllocMaxFrames = 1024;
constexpr int kPutFrames = 24;  // frame records per jr_put_frames launch (kernel arguments <= 4 KiB)
constexpr size_t kNoAllocScratchBytes = kCounterBytes + (size_t)kNoAllocMaxFrames * sizeof(DevFrame);
// Device address of that array on the current device (looked up once per
// device; `dev` is the current device's index, 0 <= dev < 64).
hipError_t noalloc_scratch(int dev, void** ptr);
// Writes rows[0, n) to the device table dst in stream order through kernel
// arguments (no copy call, no staging memory): ceil(n / kPutFrames) launches.
hipError_t put_frames(const DevFrame* rows, int n, DevFrame* dst, hipStream_t stream);

// Frame table of a prescribed cardioid path, written on the device: frame k
// is `tmpl` with C_k (see julia.h), out_offset0 + k * frame_px and first tile
// k * tiles_per_frame.
struct CardioidArgs {
    DevFrame tmpl;
    DevFrame* dst;
    double step_re, step_im, a0, da;
    int64_t out_offset0, frame_px, tiles_per_frame;
    int32_t frames;
};
hipError_t launch_cardioid_table(const CardioidArgs& g, hipStream_t stream);
// Zeroes n int32 words with a kernel (not a memset, so that it can sit in a
// captured hipGraph).
hipError_t launch_zero_words(int32_t* p, int64_t n, hipStream_t stream);

// Runs the tiled kernel; in persistent mode a small kernel zeroes the queue
// counters first (both may be captured into a hipGraph).
hipError_t launch_tiled(int unroll, int defer, int dtmask, int blocks, const PersistentArgs& args,
                        hipStream_t stream);
// Workgroups a launch_tiled call with this many `blocks` actually launches.
int launch_workgroups(int dtmask, const PersistentArgs& args, int blocks);
hipError_t launch_plain(int dtype, const PlainArgs& args, hipStream_t stream);

// One thread per pixel over the frame table (tiles of 16 x 16, one workgroup each).
hipError_t launch_plain_batch(int dtmask, const PersistentArgs& args, hipStream_t stream);

}  // namespace jr
