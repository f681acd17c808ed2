// julia_host.cpp -- host runtime and C ABI of libjulia.so (see include/julia.h).
//
// Frame setup (pixel-centre mapping scalars in binary64), argument validation,
// per-(device, stream) workspaces with a pinned staging ring for the frame
// table and the work-queue counters of the persistent kernel, prepared plans
// and their hipGraph capture.  Compiled with -ffp-contract=off so that
// the mapping scalars are the same rounded expressions on every build.

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "julia.h"
#include "julia_device.h"

using jr::DevFrame;

namespace {

// The last failure's message on this thread (a fixed buffer: recording an
// error allocates nothing).
thread_local char g_last_msg[512];

static_assert(jr::kPaletteMax == JR_PALETTE_MAX, "one palette limit");

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_msg, sizeof g_last_msg, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    int code = (e == hipErrorOutOfMemory) ? JR_ENOMEM
               : (e == hipErrorNoDevice || e == hipErrorInvalidDevice) ? JR_ENODEV
                                                                      : JR_ELAUNCH;
    return fail(code, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Escape is absorbing when |C| <= 1.9: |Z| > 2 gives |Z^2 + C| >= |Z|^2 - |C|
// > 4 - 1.9 > 2, with a margin far above rounding in every formulation.
constexpr double kAbsorbingC = 1.9;
constexpr int32_t kMaxFrames = 1 << 22;
constexpr int32_t kMaxDegree = 8;

// ------------------------------------------------------------- validation
bool finite(double v) { return std::isfinite(v); }

int check_window(const jr_window& w, const char* who) {
    if (!finite(w.re_min) || !finite(w.re_max) || !finite(w.im_min) || !finite(w.im_max))
        return fail(JR_EINVAL, "%s: window bounds must be finite", who);
    if (!(w.re_min < w.re_max) || !(w.im_min < w.im_max))
        return fail(JR_EINVAL, "%s: window needs re_min < re_max and im_min < im_max", who);
    if (!finite(w.re_max - w.re_min) || !finite(w.im_max - w.im_min))
        return fail(JR_EINVAL, "%s: window extent overflows binary64", who);
    return JR_OK;
}

int check_image(int32_t W, int32_t H, int32_t max_iter, int32_t dtype, int32_t mode,
                const jr_complex& c, const jr_window& w, const char* who) {
    if (W < 1 || H < 1)
        return fail(JR_EINVAL, "%s: width and height must be >= 1 (got %d x %d)", who, W, H);
    if ((int64_t)W * (int64_t)H > (int64_t)INT32_MAX)
        return fail(JR_EINVAL, "%s: width*height must be < 2^31", who);
    if (max_iter < 0 || max_iter > JR_MAX_ITER)
        return fail(JR_EINVAL, "%s: max_iter %d outside 0..%d", who, max_iter, JR_MAX_ITER);
    if (dtype != JR_FP64 && dtype != JR_FP32 && dtype != JR_FF)
        return fail(JR_EINVAL, "%s: unknown dtype %d", who, dtype);
    if (mode != JR_JULIA && mode != JR_MANDELBROT)
        return fail(JR_EINVAL, "%s: unknown mode %d", who, mode);
    if (mode == JR_JULIA && (!finite(c.re) || !finite(c.im)))
        return fail(JR_EINVAL, "%s: C must be finite", who);
    return check_window(w, who);
}

int check_out(const void* p, const char* who) {
    if (p == nullptr) return fail(JR_EINVAL, "%s: output pointer is null", who);
    if (((uintptr_t)p & 3u) != 0) return fail(JR_EINVAL, "%s: output pointer not 4-byte aligned", who);
    return JR_OK;
}

int check_schedule(const jr_schedule& s) {
    if (s.tile_w < 1 || s.tile_w > 64 || s.tile_h < 1 || s.tile_h > 64)
        return fail(JR_EINVAL, "schedule: tile %d x %d out of range", s.tile_w, s.tile_h);
    if (s.defer != 0 && s.defer != 1)
        return fail(JR_EINVAL, "schedule: defer must be 0 or 1 (got %d)", s.defer);
    if (!s.defer && s.unroll != 1 && s.unroll != 2 && s.unroll != 4 && s.unroll != 8)
        return fail(JR_EINVAL, "schedule: unroll must be 1, 2, 4 or 8 (got %d)", s.unroll);
    if (s.defer && s.unroll != 4 && s.unroll != 8 && s.unroll != 16)
        return fail(JR_EINVAL, "schedule: with defer, unroll must be 4, 8 or 16 (got %d)", s.unroll);
    if (s.persistent != 0 && s.persistent != 1)
        return fail(JR_EINVAL, "schedule: persistent must be 0 or 1 (got %d)", s.persistent);
    if (s.refill < 1 || s.refill > 64)
        return fail(JR_EINVAL, "schedule: refill must be in 1..64 (got %d)", s.refill);
    if (s.waves_per_cu < 4 || s.waves_per_cu > 32 || (s.waves_per_cu % 4) != 0)
        return fail(JR_EINVAL, "schedule: waves_per_cu must be 4..32, a multiple of 4");
    if (s.order != JR_ORDER_TABLE && s.order != JR_ORDER_COST)
        return fail(JR_EINVAL, "schedule: unknown order %d", s.order);
    if (s.kernel != JR_KERNEL_TILED && s.kernel != JR_KERNEL_PLAIN &&
        s.kernel != JR_KERNEL_HYBRID && s.kernel != JR_KERNEL_ROWS)
        return fail(JR_EINVAL, "schedule: unknown kernel %d", s.kernel);
    if (s.kernel == JR_KERNEL_HYBRID && (s.bail < 1 || s.bail > 4096))
        return fail(JR_EINVAL, "schedule: bail must be in 1..4096 (got %d)", s.bail);
    if (s.kernel == JR_KERNEL_ROWS) {
        if (s.unroll != 4 && s.unroll != 8)
            return fail(JR_EINVAL, "schedule: the rows kernel takes unroll 4 or 8");
        if (s.bail < 1 || s.bail > 64)
            return fail(JR_EINVAL, "schedule: rows kernel bail must be in 1..64 (got %d)", s.bail);
        if (s.handoff < 0 || s.handoff > 256)
            return fail(JR_EINVAL, "schedule: rows kernel handoff must be in 0..256 (got %d)",
                        s.handoff);
    }
    return JR_OK;
}

int check_frames(const jr_frame* frames, int32_t n, int64_t capacity) {
    if (frames == nullptr) return fail(JR_EINVAL, "batch: frames is null");
    if (n < 1 || n > kMaxFrames) return fail(JR_EINVAL, "batch: n must be in 1..%d", kMaxFrames);
    if (capacity < 0) return fail(JR_EINVAL, "batch: out_capacity must be >= 0");
    for (int32_t k = 0; k < n; ++k) {
        const jr_frame& f = frames[k];
        char who[48];
        snprintf(who, sizeof who, "frame %d", k);
        int rc = check_image(f.width, f.height, f.max_iter, f.dtype, f.mode, f.c, f.w, who);
        if (rc) return rc;
        const int32_t rend = f.row_end == 0 ? f.height : f.row_end;
        if (f.row_begin < 0 || rend > f.height || f.row_begin >= rend)
            return fail(JR_EINVAL, "%s: rows [%d, %d) outside [0, %d)", who, f.row_begin, rend, f.height);
        if (f.degree != 0 && (f.degree < 2 || f.degree > kMaxDegree))
            return fail(JR_EINVAL, "%s: degree %d not 0 or 2..%d", who, f.degree, kMaxDegree);
        if (f.map != JR_MAP_POLY && f.map != JR_MAP_RATIONAL)
            return fail(JR_EINVAL, "%s: unknown map %d", who, f.map);
        if (f.map == JR_MAP_RATIONAL) {
            if (f.mode != JR_JULIA)
                return fail(JR_EINVAL, "%s: rational maps render Julia images only", who);
            if (f.dtype == JR_FF)
                return fail(JR_EINVAL, "%s: rational maps run in FP64 or FP32", who);
            if (!finite(f.lambda.re) || !finite(f.lambda.im))
                return fail(JR_EINVAL, "%s: lambda must be finite", who);
        }
        if (f.out_offset < 0) return fail(JR_EINVAL, "%s: out_offset must be >= 0", who);
        const int64_t px = (int64_t)f.width * f.height;
        if (f.out_offset > capacity - px)
            return fail(JR_EINVAL, "%s: out_offset + width*height exceeds out_capacity", who);
    }
    return JR_OK;
}

// ------------------------------------------------------------- schedules
std::mutex g_sched_mu;
// Defaults per dtype; the autotuner can replace them (jr_set_default_schedule).
// Starting points from the autotuner's runs on MI355X.  FP32 takes the
// two-phase rows kernel, which won every FP32 workload measured; one wave per
// tile keeps one-image calls free of the work queues (and so capturable).
jr_schedule g_default[3] = {
    // tile_w, tile_h, unroll, defer, refill, persistent, waves_per_cu, order, kernel, bail,
    // handoff
    {16, 16, 8, 0, 16, 0, 16, JR_ORDER_COST, JR_KERNEL_TILED, 8, 0},  // FP64
    {64, 8, 8, 0, 32, 0, 16, JR_ORDER_COST, JR_KERNEL_ROWS, 6, 0},    // FP32
    {16, 16, 8, 1, 64, 0, 16, JR_ORDER_COST, JR_KERNEL_TILED, 8, 0},  // FF
};

jr_schedule default_schedule(int dtype) {
    std::lock_guard<std::mutex> g(g_sched_mu);
    return g_default[dtype];
}

// Schedules of one-image calls by size (jr_set_image_schedule).
struct ImageSchedule {
    int32_t dtype;
    int32_t max_iter_limit;
    int64_t pixels_limit;
    jr_schedule s;
};
constexpr size_t kMaxImageSchedules = 64;
std::vector<ImageSchedule> g_image;

// The entry of this dtype with the smallest cap limit covering max_iter and,
// among those, the smallest pixel limit covering px; when no pixel limit
// covers px, the largest one below it; otherwise the dtype's default.
jr_schedule image_schedule(int dtype, int32_t max_iter, int64_t px) {
    std::lock_guard<std::mutex> g(g_sched_mu);
    const ImageSchedule* best = nullptr;
    for (const ImageSchedule& e : g_image) {
        if (e.dtype != dtype || max_iter > e.max_iter_limit) continue;
        if (!best) {
            best = &e;
            continue;
        }
        if (e.max_iter_limit != best->max_iter_limit) {
            if (e.max_iter_limit < best->max_iter_limit) best = &e;
            continue;
        }
        const bool e_covers = px <= e.pixels_limit, b_covers = px <= best->pixels_limit;
        if (e_covers != b_covers) {
            if (e_covers) best = &e;
        } else if (e_covers ? e.pixels_limit < best->pixels_limit
                            : e.pixels_limit > best->pixels_limit) {
            best = &e;
        }
    }
    return best ? best->s : g_default[dtype];
}

// ------------------------------------------------------------- frame table
double dtype_cost(int dtype) {
    // Relative cost of one pixel-iteration (vector-ALU instructions).
    return dtype == JR_FF ? 20.0 : dtype == JR_FP64 ? 1.75 : 1.0;
}

double frame_cost(const jr_frame& f) {
    const int32_t rend = f.row_end == 0 ? f.height : f.row_end;
    const double px = (double)f.width * (double)(rend - f.row_begin);
    // a general map's iteration costs about degree - 1 complex products; the
    // rational term adds |W|^2, lambda conj(W) and two divisions
    double deg = f.degree > 2 ? (double)(f.degree - 1) : 1.0;
    if (f.map == JR_MAP_RATIONAL) deg += 3.0;
    return px * (4.0 + std::min<double>(f.max_iter, 256.0)) * dtype_cost(f.dtype) * deg;
}

bool absorbing(const jr_frame& f) {
    if (f.map == JR_MAP_RATIONAL) {
        // |Z| > 2 gives |W| = |Z|^d > 2^d and |W + C + lambda / W| >=
        // |W| - |C| - |lambda| / |W| > 2^d - |C| - |lambda| / 2^d, which
        // stays above 2 (margin 0.1) under this condition
        const double p = std::ldexp(1.0, f.degree == 0 ? 2 : f.degree);
        return std::hypot(f.c.re, f.c.im) + std::hypot(f.lambda.re, f.lambda.im) / p <=
               p - 2.1;
    }
    if (f.mode == JR_JULIA) return std::hypot(f.c.re, f.c.im) <= kAbsorbingC;
    // Mandelbrot: C ranges over the window; its largest modulus is at a corner.
    const double xs[2] = {f.w.re_min, f.w.re_max}, ys[2] = {f.w.im_min, f.w.im_max};
    double m = 0.0;
    for (double x : xs)
        for (double y : ys) m = std::max(m, std::hypot(x, y));
    return m <= kAbsorbingC;
}

// Totals of a frame table, for the launch shape and the kernel variant.
struct TableStats {
    int64_t total_tiles = 0;
    double total_cost = 0.0;     // estimated, arbitrary units
    double max_tile_cost = 0.0;  // estimated cost of the most expensive tile
    int dtmask = 0;
};

struct Table : TableStats {
    std::vector<DevFrame> rows;
};

// Tiles per granule (one atomic claim): aim at ~16 granules per wave for the
// most expensive tiles, so that claims stay rare on cheap work and a single
// claim never holds a large share of a wave's work on expensive frames.
int32_t granule_size(const TableStats& t, int blocks) {
    const double waves = 4.0 * blocks;
    const double target = t.total_cost / (waves * 16.0);
    const double g = std::floor(target / std::max(t.max_tile_cost, 1.0));
    return (int32_t)std::max(1.0, std::min(32.0, g));
}

jr::PersistentArgs make_args(const TableStats& t, const DevFrame* d_table, int32_t* out,
                             unsigned long long* ctr, int32_t n, int blocks, const jr_schedule& s) {
    jr::PersistentArgs a;
    std::memset(&a, 0, sizeof a);
    a.frames = d_table;
    a.out_base = out;
    a.ctr = ctr;
    a.total_tiles = t.total_tiles;
    a.nframes = n;
    a.granule = granule_size(t, blocks);
    a.granules = (t.total_tiles + a.granule - 1) / a.granule;
    a.refill = s.refill;
    a.persistent = s.persistent;
    a.hybrid = s.kernel == JR_KERNEL_HYBRID ? 1 : 0;
    a.rows = s.kernel == JR_KERNEL_ROWS ? 1 : 0;
    a.bail = s.bail;
    a.handoff = s.kernel == JR_KERNEL_ROWS ? s.handoff : 0;
    return a;
}

// The device record of frame f whose first tile is global tile `tile_begin`;
// returns its tile count.
int64_t fill_frame(const jr_frame& f, const jr_schedule& s, int64_t tile_begin, DevFrame& d) {
    std::memset(&d, 0, sizeof d);
    const double W = (double)f.width, H = (double)f.height;
    d.hx = (f.w.re_max - f.w.re_min) / (2.0 * W);
    d.hy = (f.w.im_max - f.w.im_min) / (2.0 * H);
    d.cx = 0.5 * (f.w.re_min + f.w.re_max);
    d.cy = 0.5 * (f.w.im_min + f.w.im_max);
    d.cr = f.mode == JR_JULIA ? f.c.re : 0.0;
    d.ci = f.mode == JR_JULIA ? f.c.im : 0.0;
    d.out_offset = f.out_offset;
    d.width = f.width;
    d.height = f.height;
    d.max_iter = f.max_iter;
    d.dtype = f.dtype;
    d.mode = f.mode;
    d.defer = absorbing(f) ? 1 : 0;
    d.degree = f.degree == 0 ? 2 : f.degree;
    d.map = f.map;
    d.lr = f.map == JR_MAP_RATIONAL ? f.lambda.re : 0.0;
    d.li = f.map == JR_MAP_RATIONAL ? f.lambda.im : 0.0;
    d.row_begin = f.row_begin;
    d.row_end = f.row_end == 0 ? f.height : f.row_end;
    const int32_t tw = s.kernel == JR_KERNEL_PLAIN ? 16 : s.tile_w;
    const int32_t th = s.kernel == JR_KERNEL_PLAIN ? 16 : s.tile_h;
    d.tile_w = std::min(tw, f.width);
    d.tile_h = std::min(th, d.row_end - d.row_begin);
    d.tiles_x = (f.width + d.tile_w - 1) / d.tile_w;
    const int64_t tiles_y = (d.row_end - d.row_begin + d.tile_h - 1) / d.tile_h;
    d.tile_begin = tile_begin;
    return (int64_t)d.tiles_x * tiles_y;
}

// The order frames go into the table: as given, or (JR_ORDER_COST) most
// expensive first, equal costs in the order given.  std::sort with the index
// as tie-break needs no scratch memory, unlike a stable sort.
void order_frames(const jr_frame* frames, int32_t n, const jr_schedule& s, int32_t* idx) {
    std::iota(idx, idx + n, 0);
    if (s.order == JR_ORDER_COST)
        std::sort(idx, idx + n, [&](int32_t a, int32_t b) {
            const double ca = frame_cost(frames[a]), cb = frame_cost(frames[b]);
            return ca > cb || (ca == cb && a < b);
        });
}

// Adds a frame's tiles to the table totals.
void account(TableStats& t, const jr_frame& f, const DevFrame& d, int64_t tiles) {
    t.total_tiles += tiles;
    t.total_cost += frame_cost(f);
    t.max_tile_cost = std::max(t.max_tile_cost, frame_cost(f) / (double)tiles);
    t.dtmask |= 1 << f.dtype;
    if (d.degree > 2) t.dtmask |= jr::kGeneralBit;
    if (d.map == jr::kMapRational) t.dtmask |= jr::kGeneralBit | jr::kRationalBit;
}

// Launches holding rational frames run the rows kernel (or the plain kernel):
// a schedule that asks for the tiled or hybrid stream is carried over to the
// rows kernel with the same tiles, scheduling mode and refill threshold.
void route_rational(const TableStats& t, jr_schedule& s) {
    if (!(t.dtmask & jr::kRationalBit)) return;
    if (s.kernel != JR_KERNEL_TILED && s.kernel != JR_KERNEL_HYBRID) return;
    s.kernel = JR_KERNEL_ROWS;
    s.unroll = s.unroll >= 8 ? 8 : 4;
    s.defer = 0;
    s.bail = 8;
    s.handoff = 0;
}

// Fills rows[0, n) in launch order and returns the table's totals; idx is
// room for n frame indices.  Allocates nothing.
void build_rows(const jr_frame* frames, int32_t n, const jr_schedule& s, DevFrame* rows,
                int32_t* idx, TableStats& t) {
    order_frames(frames, n, s, idx);
    t = TableStats();
    for (int32_t k = 0; k < n; ++k) {
        const jr_frame& f = frames[idx[k]];
        const int64_t tiles = fill_frame(f, s, t.total_tiles, rows[k]);
        rows[k].index = idx[k];
        account(t, f, rows[k], tiles);
    }
}

void build_table(const jr_frame* frames, int32_t n, const jr_schedule& s, Table& t) {
    std::vector<int32_t> idx(n);
    t.rows.resize(n);
    build_rows(frames, n, s, t.rows.data(), idx.data(), t);
}

// The schedule of a batch call: the caller's, checked, or the default of the
// dtype with the most estimated work.
int batch_schedule(const jr_frame* frames, int32_t n, const jr_schedule* sched, jr_schedule& s) {
    if (sched) {
        s = *sched;
        return check_schedule(s);
    }
    double w[3] = {0, 0, 0};
    for (int32_t k = 0; k < n; ++k) w[frames[k].dtype] += frame_cost(frames[k]);
    s = default_schedule((int)(std::max_element(w, w + 3) - w));
    return JR_OK;
}

// ------------------------------------------------------------- devices
struct DeviceInfo {
    bool probed = false;
    int rc = JR_OK;
    int num_cus = 0;
    int64_t hbm = 0;
};
std::mutex g_dev_mu;
constexpr int kMaxDevices = 64;
DeviceInfo g_dev[kMaxDevices];

int current_device(int* dev, DeviceInfo* info) {
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (*dev < 0 || *dev >= kMaxDevices)
        return fail(JR_ENODEV, "device %d beyond the library's %d", *dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_dev_mu);
    DeviceInfo& d = g_dev[*dev];
    if (!d.probed) {
        d.probed = true;
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, *dev);
        if (e != hipSuccess) {
            d.rc = hip_fail(e, "hipGetDeviceProperties");
        } else if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            d.rc = fail(JR_ENODEV, "device %d is %s; libjulia.so is built for gfx950 only",
                        *dev, prop.gcnArchName);
        } else {
            d.num_cus = prop.multiProcessorCount;
            d.hbm = (int64_t)prop.totalGlobalMem;
        }
    }
    if (d.rc != JR_OK) return fail(d.rc, "device %d unusable", *dev);
    *info = d;
    return JR_OK;
}

// ------------------------------------------------------------- workspaces
constexpr int kStages = 4;

struct Workspace {
    std::mutex mu;
    DevFrame* d_table = nullptr;
    size_t table_cap = 0;
    unsigned long long* d_ctr = nullptr;
    DevFrame* h_stage[kStages] = {};
    size_t stage_cap[kStages] = {};
    hipEvent_t ev[kStages] = {};
    bool ev_used[kStages] = {};
    int slot = 0;
};

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

int get_workspace(int dev, hipStream_t stream, Workspace** out) {
    std::lock_guard<std::mutex> g(g_ws_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *out = it->second;
        return JR_OK;
    }
    // The queue counters need no initial value: every persistent launch is
    // preceded by the kernel that zeroes them.
    Workspace* ws = new Workspace();
    hipError_t e = hipMalloc((void**)&ws->d_ctr, jr::kCounterBytes);
    for (int k = 0; k < kStages && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&ws->ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        if (ws->d_ctr) (void)hipFree(ws->d_ctr);
        for (int k = 0; k < kStages; ++k)
            if (ws->ev[k]) (void)hipEventDestroy(ws->ev[k]);
        delete ws;
        return hip_fail(e, "workspace setup");
    }
    g_ws[key] = ws;
    *out = ws;
    return JR_OK;
}

// The workspace's device frame table holds at least `bytes` (caller holds ws->mu).
int ensure_table(Workspace* ws, size_t bytes, hipStream_t stream) {
    if (ws->table_cap >= bytes) return JR_OK;
    // The old table may still be read by work queued on this stream.
    HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (ws->d_table) HIP_TRY(hipFree(ws->d_table), "hipFree");
    ws->d_table = nullptr;
    ws->table_cap = 0;
    size_t cap_bytes = std::max<size_t>(bytes, 64 * sizeof(DevFrame));
    HIP_TRY(hipMalloc((void**)&ws->d_table, cap_bytes), "hipMalloc frame table");
    ws->table_cap = cap_bytes;
    return JR_OK;
}

int grid_blocks(const DeviceInfo& info, const jr_schedule& s, int64_t total_tiles) {
    if (s.kernel == JR_KERNEL_PLAIN) return (int)std::min<int64_t>(total_tiles, INT32_MAX);
    if (!s.persistent) return (int)std::min<int64_t>((total_tiles + 3) / 4, INT32_MAX);
    int64_t blocks = (int64_t)info.num_cus * (s.waves_per_cu / 4);
    // No more waves than tiles: extra waves would only claim and leave.
    const int64_t need = (total_tiles + 3) / 4;
    blocks = std::max<int64_t>(1, std::min(blocks, need));
    return (int)blocks;
}

int check_palette(const uint32_t* palette, int32_t len, bool required, const char* who) {
    if (!required && palette == nullptr && len == 0) return JR_OK;
    if (palette == nullptr) return fail(JR_EINVAL, "%s: palette is null", who);
    if (reinterpret_cast<uintptr_t>(palette) % 4 != 0)
        return fail(JR_EINVAL, "%s: palette is not 4-byte aligned", who);
    if (len < 1 || len > JR_PALETTE_MAX)
        return fail(JR_EINVAL, "%s: palette_len %d outside 1..%d", who, len, JR_PALETTE_MAX);
    return JR_OK;
}

int enqueue_batch(const jr_frame* frames, int32_t n, int32_t* out_base, int64_t capacity,
                  const jr_schedule* sched, hipStream_t stream, const uint32_t* palette = nullptr,
                  int32_t palette_len = 0) {
    int rc = check_frames(frames, n, capacity);
    if (rc) return rc;
    if ((rc = check_out(out_base, "batch"))) return rc;
    jr_schedule s;
    if ((rc = batch_schedule(frames, n, sched, s))) return rc;
    int dev;
    DeviceInfo info;
    if ((rc = current_device(&dev, &info))) return rc;
    Table t;
    build_table(frames, n, s, t);
    route_rational(t, s);
    const int blocks = grid_blocks(info, s, t.total_tiles);
    const bool queues = s.persistent && s.kernel != JR_KERNEL_PLAIN;
    if (n == 1 && !queues) {
        // One frame travels inside the kernel arguments and no workspace is
        // touched: a single launch, which a hipGraph capture may record.
        jr::PersistentArgs args = make_args(t, nullptr, out_base, nullptr, n, blocks, s);
        args.frame0 = t.rows[0];
        args.palette = palette;
        args.palette_len = palette_len;
        hipError_t e = s.kernel == JR_KERNEL_PLAIN
                           ? jr::launch_plain_batch(t.dtmask, args, stream)
                           : jr::launch_tiled(s.unroll, s.defer, t.dtmask, blocks, args, stream);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        return JR_OK;
    }
    Workspace* ws;
    if ((rc = get_workspace(dev, stream, &ws))) return rc;
    std::lock_guard<std::mutex> g(ws->mu);
    if (n == 1) {
        jr::PersistentArgs args = make_args(t, nullptr, out_base, ws->d_ctr, n, blocks, s);
        args.frame0 = t.rows[0];
        args.palette = palette;
        args.palette_len = palette_len;
        hipError_t e = jr::launch_tiled(s.unroll, s.defer, t.dtmask, blocks, args, stream);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        return JR_OK;
    }
    // Several frames go through the pinned staging ring, whose copy a graph
    // would replay from memory the ring reuses: refuse capture (plans capture).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(stream, &cap), "hipStreamIsCapturing");
    if (cap != hipStreamCaptureStatusNone)
        return fail(JR_EINVAL, "batch of %d frames on a capturing stream; use jr_plan_capture", n);
    const size_t bytes = (size_t)n * sizeof(DevFrame);
    if ((rc = ensure_table(ws, bytes, stream))) return rc;
    const int k = ws->slot;
    ws->slot = (ws->slot + 1) % kStages;
    if (ws->ev_used[k]) HIP_TRY(hipEventSynchronize(ws->ev[k]), "hipEventSynchronize");
    if (ws->stage_cap[k] < bytes) {
        if (ws->h_stage[k]) HIP_TRY(hipHostFree(ws->h_stage[k]), "hipHostFree");
        ws->h_stage[k] = nullptr;
        ws->stage_cap[k] = 0;
        size_t cap_bytes = std::max<size_t>(bytes, 64 * sizeof(DevFrame));
        HIP_TRY(hipHostMalloc((void**)&ws->h_stage[k], cap_bytes, hipHostMallocDefault),
                "hipHostMalloc staging");
        ws->stage_cap[k] = cap_bytes;
    }
    std::memcpy(ws->h_stage[k], t.rows.data(), bytes);
    HIP_TRY(hipMemcpyAsync(ws->d_table, ws->h_stage[k], bytes, hipMemcpyHostToDevice, stream),
            "hipMemcpyAsync frame table");
    HIP_TRY(hipEventRecord(ws->ev[k], stream), "hipEventRecord");
    ws->ev_used[k] = true;
    jr::PersistentArgs args = make_args(t, ws->d_table, out_base, ws->d_ctr, n, blocks, s);
    args.palette = palette;
    args.palette_len = palette_len;
    hipError_t e = s.kernel == JR_KERNEL_PLAIN
                       ? jr::launch_plain_batch(t.dtmask, args, stream)
                       : jr::launch_tiled(s.unroll, s.defer, t.dtmask, blocks, args, stream);
    if (e != hipSuccess) return hip_fail(e, "persistent kernel launch");
    return JR_OK;
}

// Allocation-free batches: the table is built in these fixed host arrays
// (under g_na_mu) and written to the device array of jr::noalloc_scratch by
// kernel arguments, which the runtime copies when a launch is enqueued.
static_assert(jr::kNoAllocMaxFrames == JR_NOALLOC_MAX_FRAMES, "one frame limit");
static_assert(jr::kNoAllocScratchBytes == JR_NOALLOC_SCRATCH_BYTES, "one scratch size");
std::mutex g_na_mu;
DevFrame g_na_rows[jr::kNoAllocMaxFrames];
int32_t g_na_idx[jr::kNoAllocMaxFrames];

int enqueue_batch_noalloc(const jr_frame* frames, int32_t n, int32_t* out_base, int64_t capacity,
                          const jr_schedule* sched, hipStream_t stream) {
    const char* who = "julia_render_batch_noalloc";
    if (frames != nullptr && n > JR_NOALLOC_MAX_FRAMES)
        return fail(JR_EINVAL, "%s: %d frames exceed the allocation-free limit of %d (split the "
                    "batch, or use julia_render_batch)", who, n, JR_NOALLOC_MAX_FRAMES);
    int rc = check_frames(frames, n, capacity);
    if (rc) return rc;
    if ((rc = check_out(out_base, who))) return rc;
    jr_schedule s;
    if ((rc = batch_schedule(frames, n, sched, s))) return rc;
    int dev;
    DeviceInfo info;
    if ((rc = current_device(&dev, &info))) return rc;
    void* base = nullptr;
    HIP_TRY(jr::noalloc_scratch(dev, &base), "hipGetSymbolAddress of the scratch array");
    unsigned long long* ctr = static_cast<unsigned long long*>(base);
    DevFrame* table = reinterpret_cast<DevFrame*>(static_cast<char*>(base) + jr::kCounterBytes);
    std::lock_guard<std::mutex> g(g_na_mu);
    TableStats t;
    build_rows(frames, n, s, g_na_rows, g_na_idx, t);
    route_rational(t, s);
    const int blocks = grid_blocks(info, s, t.total_tiles);
    jr::PersistentArgs args = make_args(t, n == 1 ? nullptr : table, out_base, ctr, n, blocks, s);
    if (n == 1) {
        args.frame0 = g_na_rows[0];
    } else {
        HIP_TRY(jr::put_frames(g_na_rows, n, table, stream), "frame table launch");
    }
    hipError_t e = s.kernel == JR_KERNEL_PLAIN
                       ? jr::launch_plain_batch(t.dtmask, args, stream)
                       : jr::launch_tiled(s.unroll, s.defer, t.dtmask, blocks, args, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return JR_OK;
}

jr_frame single_frame(jr_complex c, jr_window w, int32_t W, int32_t H, int32_t max_iter,
                      int32_t dtype, int32_t mode) {
    jr_frame f;
    std::memset(&f, 0, sizeof f);
    f.c = c;
    f.w = w;
    f.width = W;
    f.height = H;
    f.max_iter = max_iter;
    f.dtype = dtype;
    f.mode = mode;
    return f;
}

int render_plain(jr_complex c, jr_window w, int32_t W, int32_t H, int32_t max_iter,
                 int32_t dtype, int32_t mode, int32_t* out, void* stream, const char* who);

int render_one(jr_complex c, jr_window w, int32_t W, int32_t H, int32_t max_iter, int32_t dtype,
               int32_t mode, int32_t* out, void* stream, const char* who) {
    int rc = check_image(W, H, max_iter, dtype, mode, c, w, who);
    if (rc) return rc;
    if ((rc = check_out(out, who))) return rc;
    jr_schedule s = image_schedule(dtype, max_iter, (int64_t)W * H);
    // one image on the one-thread-per-pixel kernel: its 2-D grid form
    if (s.kernel == JR_KERNEL_PLAIN) return render_plain(c, w, W, H, max_iter, dtype, mode, out,
                                                         stream, who);
    jr_frame f = single_frame(c, w, W, H, max_iter, dtype, mode);
    return enqueue_batch(&f, 1, out, (int64_t)W * H, &s, (hipStream_t)stream);
}

int render_one_colored(jr_complex c, jr_window w, int32_t W, int32_t H, int32_t max_iter,
                       int32_t dtype, const uint32_t* palette, int32_t palette_len,
                       uint32_t* out, void* stream) {
    const char* who = "julia_render_colored";
    int rc = check_image(W, H, max_iter, dtype, JR_JULIA, c, w, who);
    if (rc) return rc;
    if ((rc = check_out(out, who))) return rc;
    if ((rc = check_palette(palette, palette_len, true, who))) return rc;
    jr_frame f = single_frame(c, w, W, H, max_iter, dtype, JR_JULIA);
    jr_schedule s = image_schedule(dtype, max_iter, (int64_t)W * H);
    return enqueue_batch(&f, 1, reinterpret_cast<int32_t*>(out), (int64_t)W * H, &s,
                         (hipStream_t)stream, palette, palette_len);
}

int render_plain(jr_complex c, jr_window w, int32_t W, int32_t H, int32_t max_iter,
                 int32_t dtype, int32_t mode, int32_t* out, void* stream, const char* who) {
    int rc = check_image(W, H, max_iter, dtype, mode, c, w, who);
    if (rc) return rc;
    if ((rc = check_out(out, who))) return rc;
    int dev;
    DeviceInfo info;
    if ((rc = current_device(&dev, &info))) return rc;
    jr::PlainArgs a;
    a.out = out;
    a.hx = (w.re_max - w.re_min) / (2.0 * (double)W);
    a.hy = (w.im_max - w.im_min) / (2.0 * (double)H);
    a.cx = 0.5 * (w.re_min + w.re_max);
    a.cy = 0.5 * (w.im_min + w.im_max);
    a.cr = mode == JR_JULIA ? c.re : 0.0;
    a.ci = mode == JR_JULIA ? c.im : 0.0;
    a.W = W;
    a.H = H;
    a.max_iter = max_iter;
    a.mode = mode;
    hipError_t e = jr::launch_plain(dtype, a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "plain kernel launch");
    return JR_OK;
}

// ------------------------------------------------------------- cardioid paths
int check_cardioid(const jr_cardioid_path* p, int64_t capacity, const char* who) {
    if (p == nullptr) return fail(JR_EINVAL, "%s: path is null", who);
    if (p->frames < 1 || p->frames > kMaxFrames)
        return fail(JR_EINVAL, "%s: frames must be in 1..%d", who, kMaxFrames);
    int rc = check_image(p->width, p->height, p->max_iter, p->dtype, JR_JULIA,
                         jr_complex{0.0, 0.0}, p->w, who);
    if (rc) return rc;
    if (!finite(p->step.re) || !finite(p->step.im) || !finite(p->a0) || !finite(p->da))
        return fail(JR_EINVAL, "%s: step, a0 and da must be finite", who);
    const double m = std::hypot(p->step.re, p->step.im);
    if (!(m > 0.0) || std::fabs(std::log(m)) * (double)p->frames > 1e-6)
        return fail(JR_EINVAL, "%s: frames * |log|step|| must be <= 1e-6", who);
    const double a_last = p->a0 - p->da * (double)(p->frames - 1);
    if (!(p->a0 >= JR_CARDIOID_MIN_A) || !(a_last >= JR_CARDIOID_MIN_A))
        return fail(JR_EINVAL, "%s: a must stay >= %g along the path (a0 %g, last %g)", who,
                    JR_CARDIOID_MIN_A, p->a0, a_last);
    const int64_t px = (int64_t)p->width * p->height;
    if (p->out_offset < 0 || p->out_offset > capacity ||
        (int64_t)p->frames > (capacity - p->out_offset) / px)
        return fail(JR_EINVAL, "%s: out_offset + frames*width*height exceeds out_capacity", who);
    return JR_OK;
}

jr_schedule path_schedule(const jr_cardioid_path& p, const jr_schedule* sched, int* rc) {
    *rc = JR_OK;
    if (sched) {
        *rc = check_schedule(*sched);
        return *sched;
    }
    return default_schedule(p.dtype);
}

// The generator's arguments (the record every frame shares; C, offset and
// first tile are set per frame on the device) and the launch totals.
jr::CardioidArgs cardioid_args(const jr_cardioid_path& p, const jr_schedule& s, DevFrame* dst,
                               TableStats& t) {
    jr::CardioidArgs g;
    std::memset(&g, 0, sizeof g);
    jr_frame f = single_frame(jr_complex{0.0, 0.0}, p.w, p.width, p.height, p.max_iter,
                              p.dtype, JR_JULIA);
    f.out_offset = p.out_offset;
    const int64_t tiles = fill_frame(f, s, 0, g.tmpl);
    g.tmpl.defer = 1;  // every |C_k| < 1.9 (check_cardioid): escape is absorbing
    g.dst = dst;
    g.step_re = p.step.re;
    g.step_im = p.step.im;
    g.a0 = p.a0;
    g.da = p.da;
    g.out_offset0 = p.out_offset;
    g.frame_px = (int64_t)p.width * p.height;
    g.tiles_per_frame = tiles;
    g.frames = p.frames;
    t = TableStats();
    t.total_tiles = tiles * p.frames;
    t.total_cost = frame_cost(f) * (double)p.frames;
    t.max_tile_cost = frame_cost(f) / (double)tiles;
    t.dtmask = 1 << p.dtype;
    return g;
}

int render_cardioid(const jr_cardioid_path* path, int32_t* out, int64_t capacity,
                    const jr_schedule* sched, hipStream_t stream) {
    const char* who = "julia_render_cardioid_path";
    int rc = check_cardioid(path, capacity, who);
    if (rc) return rc;
    if ((rc = check_out(out, who))) return rc;
    jr_schedule s = path_schedule(*path, sched, &rc);
    if (rc) return rc;
    int dev;
    DeviceInfo info;
    if ((rc = current_device(&dev, &info))) return rc;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(stream, &cap), "hipStreamIsCapturing");
    if (cap != hipStreamCaptureStatusNone)
        return fail(JR_EINVAL, "%s on a capturing stream; use jr_plan_create_cardioid", who);
    Workspace* ws;
    if ((rc = get_workspace(dev, stream, &ws))) return rc;
    std::lock_guard<std::mutex> g(ws->mu);
    if ((rc = ensure_table(ws, (size_t)path->frames * sizeof(DevFrame), stream))) return rc;
    TableStats t;
    jr::CardioidArgs gen = cardioid_args(*path, s, ws->d_table, t);
    const int blocks = grid_blocks(info, s, t.total_tiles);
    HIP_TRY(jr::launch_cardioid_table(gen, stream), "cardioid table launch");
    jr::PersistentArgs args = make_args(t, ws->d_table, out, ws->d_ctr, path->frames, blocks, s);
    hipError_t e = s.kernel == JR_KERNEL_PLAIN
                       ? jr::launch_plain_batch(t.dtmask, args, stream)
                       : jr::launch_tiled(s.unroll, s.defer, t.dtmask, blocks, args, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return JR_OK;
}

}  // namespace

// ======================================================================== C ABI
struct jr_plan {
    int dev = 0;
    DevFrame* d_table = nullptr;
    unsigned long long* d_ctr = nullptr;
    int64_t total_tiles = 0;
    int32_t nframes = 0;
    int dtmask = 0;
    int unroll = 1, defer = 0, blocks = 1, kernel = JR_KERNEL_TILED;
    jr::PersistentArgs args;
    bool generated = false;       // the table is written on the device per launch
    jr::CardioidArgs gen;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* jr_strerror(int code) {
    switch (code) {
        case JR_OK: return "success";
        case JR_EINVAL: return "invalid argument";
        case JR_ENOMEM: return "out of memory";
        case JR_ENODEV: return "no usable gfx950 device";
        case JR_ELAUNCH: return "HIP launch or copy failed";
        case JR_EINTERNAL: return "internal error";
        default: return "unknown error code";
    }
}

const char* jr_last_error_message(void) { return g_last_msg; }

int jr_check_schedule(const jr_schedule* s) {
    if (!s) return fail(JR_EINVAL, "schedule is null");
    return check_schedule(*s);
}

int jr_check_frames(const jr_frame* frames, int32_t n, int64_t out_capacity) {
    return check_frames(frames, n, out_capacity);
}

int jr_get_default_schedule(int32_t dtype, int32_t max_iter, jr_schedule* out) {
    if (!out) return fail(JR_EINVAL, "out is null");
    if (max_iter < 0 || max_iter > JR_MAX_ITER)
        return fail(JR_EINVAL, "max_iter %d outside 0..%d", max_iter, JR_MAX_ITER);
    if (dtype < 0 || dtype > 2) return fail(JR_EINVAL, "unknown dtype %d", dtype);
    *out = default_schedule(dtype);
    return JR_OK;
}

int jr_set_image_schedule(int32_t dtype, int32_t max_iter_limit, int64_t pixels_limit,
                          const jr_schedule* s) {
    if (!s) return fail(JR_EINVAL, "schedule is null");
    if (dtype < 0 || dtype > 2) return fail(JR_EINVAL, "unknown dtype %d", dtype);
    if (max_iter_limit < 0 || pixels_limit < 1)
        return fail(JR_EINVAL, "limits must be max_iter_limit >= 0, pixels_limit >= 1");
    int rc = check_schedule(*s);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(g_sched_mu);
    for (ImageSchedule& e : g_image) {
        if (e.dtype == dtype && e.max_iter_limit == max_iter_limit &&
            e.pixels_limit == pixels_limit) {
            e.s = *s;
            return JR_OK;
        }
    }
    if (g_image.size() >= kMaxImageSchedules)
        return fail(JR_EINVAL, "at most %d image schedules", (int)kMaxImageSchedules);
    g_image.push_back(ImageSchedule{dtype, max_iter_limit, pixels_limit, *s});
    return JR_OK;
}

int jr_get_image_schedule(int32_t dtype, int32_t max_iter, int64_t pixels, jr_schedule* out) {
    if (!out) return fail(JR_EINVAL, "out is null");
    if (dtype < 0 || dtype > 2) return fail(JR_EINVAL, "unknown dtype %d", dtype);
    *out = image_schedule(dtype, max_iter, pixels);
    return JR_OK;
}

void jr_clear_image_schedules(void) {
    std::lock_guard<std::mutex> g(g_sched_mu);
    g_image.clear();
}

int jr_set_default_schedule(int32_t dtype, const jr_schedule* s) {
    if (!s) return fail(JR_EINVAL, "schedule is null");
    if (dtype < 0 || dtype > 2) return fail(JR_EINVAL, "unknown dtype %d", dtype);
    int rc = check_schedule(*s);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(g_sched_mu);
    g_default[dtype] = *s;
    return JR_OK;
}

int julia_render(jr_complex c, jr_window w, int32_t width, int32_t height, int32_t max_iter,
                 int32_t dtype, int32_t* out, void* stream) {
    return render_one(c, w, width, height, max_iter, dtype, JR_JULIA, out, stream, "julia_render");
}

int julia_render_plain(jr_complex c, jr_window w, int32_t width, int32_t height,
                       int32_t max_iter, int32_t dtype, int32_t* out, void* stream) {
    return render_plain(c, w, width, height, max_iter, dtype, JR_JULIA, out, stream,
                        "julia_render_plain");
}

int mandelbrot_render(jr_window w, int32_t width, int32_t height, int32_t max_iter,
                      int32_t dtype, int32_t* out, void* stream) {
    return render_one(jr_complex{0.0, 0.0}, w, width, height, max_iter, dtype, JR_MANDELBROT,
                      out, stream, "mandelbrot_render");
}

int mandelbrot_render_plain(jr_window w, int32_t width, int32_t height, int32_t max_iter,
                            int32_t dtype, int32_t* out, void* stream) {
    return render_plain(jr_complex{0.0, 0.0}, w, width, height, max_iter, dtype, JR_MANDELBROT,
                        out, stream, "mandelbrot_render_plain");
}

int julia_render_batch(const jr_frame* frames, int32_t n, int32_t* out_base,
                       int64_t out_capacity, const jr_schedule* sched, void* stream) {
    return enqueue_batch(frames, n, out_base, out_capacity, sched, (hipStream_t)stream);
}

int julia_render_cardioid_path(const jr_cardioid_path* path, int32_t* out_base,
                               int64_t out_capacity, const jr_schedule* sched, void* stream) {
    return render_cardioid(path, out_base, out_capacity, sched, (hipStream_t)stream);
}

int jr_plan_create_cardioid(const jr_cardioid_path* path, int32_t* out_base,
                            int64_t out_capacity, const jr_schedule* sched, jr_plan** plan) {
    const char* who = "jr_plan_create_cardioid";
    if (!plan) return fail(JR_EINVAL, "plan is null");
    *plan = nullptr;
    int rc = check_cardioid(path, out_capacity, who);
    if (rc) return rc;
    if ((rc = check_out(out_base, who))) return rc;
    jr_schedule s = path_schedule(*path, sched, &rc);
    if (rc) return rc;
    int dev;
    DeviceInfo info;
    if ((rc = current_device(&dev, &info))) return rc;
    jr_plan* p = new jr_plan();
    p->dev = dev;
    const size_t bytes = (size_t)path->frames * sizeof(DevFrame);
    hipError_t e = hipMalloc((void**)&p->d_table, bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_ctr, jr::kCounterBytes);
    if (e == hipSuccess) e = hipMemset(p->d_ctr, 0, jr::kCounterBytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        jr_plan_destroy(p);
        return hip_fail(e, "plan setup");
    }
    TableStats t;
    p->gen = cardioid_args(*path, s, p->d_table, t);
    p->generated = true;
    p->nframes = path->frames;
    p->total_tiles = t.total_tiles;
    p->dtmask = t.dtmask;
    p->unroll = s.unroll;
    p->defer = s.defer;
    p->kernel = s.kernel;
    p->blocks = grid_blocks(info, s, t.total_tiles);
    p->args = make_args(t, p->d_table, out_base, p->d_ctr, path->frames, p->blocks, s);
    *plan = p;
    return JR_OK;
}

int julia_render_batch_noalloc(const jr_frame* frames, int32_t n, int32_t* out_base,
                               int64_t out_capacity, const jr_schedule* sched, void* stream) {
    return enqueue_batch_noalloc(frames, n, out_base, out_capacity, sched, (hipStream_t)stream);
}

int julia_render_batch_colored(const jr_frame* frames, int32_t n, const uint32_t* palette,
                               int32_t palette_len, uint32_t* out_base, int64_t out_capacity,
                               const jr_schedule* sched, void* stream) {
    int rc = check_palette(palette, palette_len, true, "julia_render_batch_colored");
    if (rc) return rc;
    return enqueue_batch(frames, n, reinterpret_cast<int32_t*>(out_base), out_capacity, sched,
                         (hipStream_t)stream, palette, palette_len);
}

int julia_render_colored(jr_complex c, jr_window w, int32_t width, int32_t height,
                         int32_t max_iter, int32_t dtype, const uint32_t* palette,
                         int32_t palette_len, uint32_t* out, void* stream) {
    return render_one_colored(c, w, width, height, max_iter, dtype, palette, palette_len, out,
                              stream);
}

int jr_plan_create(const jr_frame* frames, int32_t n, int32_t* out_base, int64_t out_capacity,
                   const jr_schedule* sched, jr_plan** plan) {
    if (!plan) return fail(JR_EINVAL, "plan is null");
    *plan = nullptr;
    int rc = check_frames(frames, n, out_capacity);
    if (rc) return rc;
    if ((rc = check_out(out_base, "plan"))) return rc;
    jr_schedule s;
    if ((rc = batch_schedule(frames, n, sched, s))) return rc;
    int dev;
    DeviceInfo info;
    if ((rc = current_device(&dev, &info))) return rc;
    Table t;
    build_table(frames, n, s, t);
    route_rational(t, s);
    jr_plan* p = new jr_plan();
    p->dev = dev;
    p->nframes = n;
    p->total_tiles = t.total_tiles;
    p->dtmask = t.dtmask;
    p->unroll = s.unroll;
    p->defer = s.defer;
    p->kernel = s.kernel;
    p->blocks = grid_blocks(info, s, t.total_tiles);
    const size_t bytes = (size_t)n * sizeof(DevFrame);
    hipError_t e = hipMalloc((void**)&p->d_table, bytes);
    if (e == hipSuccess) e = hipMemcpy(p->d_table, t.rows.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_ctr, jr::kCounterBytes);
    if (e == hipSuccess) e = hipMemset(p->d_ctr, 0, jr::kCounterBytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        jr_plan_destroy(p);
        return hip_fail(e, "plan setup");
    }
    p->args = make_args(t, p->d_table, out_base, p->d_ctr, n, p->blocks, s);
    *plan = p;
    return JR_OK;
}

static hipError_t plan_enqueue(const jr_plan* p, hipStream_t stream) {
    if (p->generated) {
        hipError_t e = jr::launch_cardioid_table(p->gen, stream);
        if (e != hipSuccess) return e;
    }
    if (p->args.done) {
        hipError_t e = jr::launch_zero_words(p->args.done, p->nframes, stream);
        if (e != hipSuccess) return e;
    }
    return p->kernel == JR_KERNEL_PLAIN
               ? jr::launch_plain_batch(p->dtmask, p->args, stream)
               : jr::launch_tiled(p->unroll, p->defer, p->dtmask, p->blocks, p->args, stream);
}

int jr_plan_launch(jr_plan* p, void* stream) {
    if (!p) return fail(JR_EINVAL, "plan is null");
    hipError_t e = plan_enqueue(p, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "plan launch");
    return JR_OK;
}

int jr_plan_capture(jr_plan* p, void* stream) {
    if (!p) return fail(JR_EINVAL, "plan is null");
    if (p->exec) return JR_OK;
    hipStream_t s = (hipStream_t)stream;
    hipStream_t own = nullptr;
    if (s == nullptr) {
        HIP_TRY(hipStreamCreateWithFlags(&own, hipStreamNonBlocking), "hipStreamCreate");
        s = own;
    }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = plan_enqueue(p, s);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (e == hipSuccess && le != hipSuccess) e = le;
        if (e == hipSuccess) {
            p->graph = g;
            e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    if (own) (void)hipStreamDestroy(own);
    if (e != hipSuccess) return hip_fail(e, "plan capture");
    return JR_OK;
}

int jr_plan_replay(jr_plan* p, void* stream) {
    if (!p) return fail(JR_EINVAL, "plan is null");
    if (!p->exec) return fail(JR_EINVAL, "plan has no captured graph; call jr_plan_capture");
    HIP_TRY(hipGraphLaunch(p->exec, (hipStream_t)stream), "hipGraphLaunch");
    return JR_OK;
}

int jr_plan_set_palette(jr_plan* p, const uint32_t* palette, int32_t palette_len) {
    if (!p) return fail(JR_EINVAL, "plan is null");
    int rc = check_palette(palette, palette_len, false, "jr_plan_set_palette");
    if (rc) return rc;
    if (p->exec) {
        // The captured launch carries the old table in its arguments.
        HIP_TRY(hipGraphExecDestroy(p->exec), "hipGraphExecDestroy");
        p->exec = nullptr;
    }
    if (p->graph) {
        HIP_TRY(hipGraphDestroy(p->graph), "hipGraphDestroy");
        p->graph = nullptr;
    }
    p->args.palette = palette;
    p->args.palette_len = palette_len;
    return JR_OK;
}

int jr_plan_set_progress(jr_plan* p, int32_t* done, const int32_t* stop) {
    if (!p) return fail(JR_EINVAL, "plan is null");
    if ((done || stop) && p->kernel != JR_KERNEL_ROWS && p->kernel != JR_KERNEL_PLAIN)
        return fail(JR_EINVAL, "progress counters need the rows or plain kernel (plan has %s)",
                    p->kernel == JR_KERNEL_HYBRID ? "hybrid" : "tiled");
    if (stop && !done) return fail(JR_EINVAL, "a stop flag needs done counters");
    if (done) {
        int rc = check_out(done, "jr_plan_set_progress (done)");
        if (!rc && stop) rc = check_out(stop, "jr_plan_set_progress (stop)");
        if (rc) return rc;
    }
    if (p->exec) {
        // The captured launch carries the old pointers in its arguments.
        HIP_TRY(hipGraphExecDestroy(p->exec), "hipGraphExecDestroy");
        p->exec = nullptr;
    }
    if (p->graph) {
        HIP_TRY(hipGraphDestroy(p->graph), "hipGraphDestroy");
        p->graph = nullptr;
    }
    p->args.done = done;
    p->args.stop = stop;
    return JR_OK;
}

int jr_plan_info(const jr_plan* p, int64_t* tiles, int32_t* workgroups) {
    if (!p) return fail(JR_EINVAL, "plan is null");
    if (tiles) *tiles = p->total_tiles;
    if (workgroups)
        *workgroups = p->kernel == JR_KERNEL_PLAIN
                          ? p->blocks
                          : jr::launch_workgroups(p->dtmask, p->args, p->blocks);
    return JR_OK;
}

void jr_plan_destroy(jr_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_table) (void)hipFree(p->d_table);
    if (p->d_ctr) (void)hipFree(p->d_ctr);
    delete p;
}

int jr_device_info(int32_t* num_cus, int64_t* hbm_bytes) {
    int dev;
    DeviceInfo info;
    int rc = current_device(&dev, &info);
    if (rc) return rc;
    if (num_cus) *num_cus = info.num_cus;
    if (hbm_bytes) *hbm_bytes = info.hbm;
    return JR_OK;
}

void jr_shutdown(void) {
    std::lock_guard<std::mutex> g(g_ws_mu);
    for (auto& kv : g_ws) {
        Workspace* ws = kv.second;
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(kv.first.first);
        for (int k = 0; k < kStages; ++k) {
            if (ws->ev_used[k]) (void)hipEventSynchronize(ws->ev[k]);
            if (ws->ev[k]) (void)hipEventDestroy(ws->ev[k]);
            if (ws->h_stage[k]) (void)hipHostFree(ws->h_stage[k]);
        }
        if (ws->d_table) (void)hipFree(ws->d_table);
        if (ws->d_ctr) (void)hipFree(ws->d_ctr);
        if (prev >= 0) (void)hipSetDevice(prev);
        delete ws;
    }
    g_ws.clear();
}

}  // extern "C"
