/*
 * julia.h -- C ABI of the MI355X (gfx950) escape-time renderer, libjulia.so.
 *
 * The operation (Mayfield et al., "Fractal Art Generation using GPUs",
 * Section 2): every pixel of a width x height image is scaled onto a window of
 * the complex plane to give Z_0 ("region-covering"), the map
 * Z_{n+1} = Z_n^2 + C is iterated, and the pixel receives the number of
 * iterations taken before |Z_n|^2 > 4, capped at max_iter (the paper caps at
 * 100).  Section 3 adds the Mandelbrot variant: the pixel gives C and Z_0 = 0.
 *
 * Conventions shared by every entry point
 *   - Counts are int32, row-major, row 0 = the top of the window (im_max),
 *     column 0 = re_min.  Count n in [0, max_iter] is the index of the first
 *     iterate with |Z_n|^2 > 4 (strict); max_iter when none below max_iter is.
 *   - Pixel (i, j) has its centre at
 *       x = cx + (2i + 1 - W) hx,  y = cy - (2j + 1 - H) hy,
 *       hx = (re_max - re_min) / 2W, hy = (im_max - im_min) / 2H,
 *       cx = (re_min + re_max) / 2,  cy = (im_min + im_max) / 2,
 *     computed in binary64 with every product rounded before the sum.
 *   - dtype selects the arithmetic of the iteration:
 *       JR_FP64  binary64, each operation rounded: x' = (x*x - y*y) + cr,
 *                y' = ((2x)*y) + ci, test fl(x*x + y*y) > 4.  Exact counts.
 *       JR_FP32  binary32 with fused multiply-add: with t = fma(x, x, cr),
 *                test fma(y, y, t) > fl(4 + cr), x' = fma(-y, y, t),
 *                y' = fma(x+x, y, ci); Z_0 and C are the binary64 values
 *                rounded to binary32.
 *       JR_FF    float-float (a value is hi + lo of two binary32 numbers),
 *                for narrow (deep-zoom) windows.  Z^2 + C: the double-word
 *                square (TwoProd of hi plus a fused 2*hi*lo), the double-word
 *                product for (2x)*y and the "sloppy" double-word sum (TwoSum
 *                of the high words, the low words added to its error, one
 *                Fast2Sum); escape when not (hi < 4 or (hi = 4 and lo <= 0))
 *                for the sum of the two squares.  The general maps use the
 *                accurate double-word sum and product throughout.
 *     The three give the same count on most pixels; FP32 and FF differ from
 *     FP64 on a small fraction of pixels near the set's boundary.
 *   - Memory: `out` / `out_base` are DEVICE pointers owned by the caller
 *     (for example torch int32 tensors), 4-byte aligned, not aliased by a call
 *     still in flight.  The library never frees caller memory.  Host arrays
 *     passed in (frames, schedules) are copied before the call returns.
 *   - Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *     stream-ordered and asynchronous; the return code reports argument and
 *     launch errors only.  A device fault shows at the caller's next
 *     synchronisation, as in HIP.
 *   - Errors: every function returns an int, JR_OK (0) on success or a
 *     negative JR_E* code; jr_strerror() names it and jr_last_error_message()
 *     gives the detail of the last failure on the calling thread.  Arguments
 *     are validated before any HIP call, so an invalid call touches no device.
 *   - Thread safety: calls may come from several host threads.  Work on one
 *     stream is ordered; calls on different streams use separate workspaces.
 */
#ifndef JULIA_H
#define JULIA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    JR_OK = 0,
    JR_EINVAL = -1,    /* an argument is out of range, non-finite or null  */
    JR_ENOMEM = -2,    /* device or pinned-host allocation failed          */
    JR_ENODEV = -3,    /* no usable gfx950 device                          */
    JR_ELAUNCH = -4,   /* a HIP launch, copy or graph call failed          */
    JR_EINTERNAL = -5  /* broken invariant inside the library              */
};

/*
 * Largest iteration cap of any call (2^30).  The kernels keep iteration
 * counters in 32-bit integers and test a block's end as n + K >= max_iter;
 * a lane whose pixel is done keeps advancing its counter until the wave's
 * last orbit ends, by up to max_iter more.  With max_iter <= 2^30 no counter
 * passes 2^31 - 1.  Larger caps are rejected with JR_EINVAL.
 */
#define JR_MAX_ITER (1 << 30)

typedef enum { JR_FP64 = 0, JR_FP32 = 1, JR_FF = 2 } jr_dtype;
typedef enum { JR_JULIA = 0, JR_MANDELBROT = 1 } jr_mode;
typedef enum { JR_ORDER_TABLE = 0, JR_ORDER_COST = 1 } jr_order;

typedef struct { double re, im; } jr_complex;
/* Window of the complex plane: re_min < re_max, im_min < im_max, finite. */
typedef struct { double re_min, re_max, im_min, im_max; } jr_window;

/*
 * One image of a batch.  The image occupies width*height consecutive int32
 * elements of the output arena starting at element out_offset; only rows
 * [row_begin, row_end) are computed by this call (row_end = 0 means height),
 * so a large frame can be split over several calls.  `c` is ignored in
 * Mandelbrot mode.  Limits: width, height >= 1, width*height < 2^31,
 * 0 <= max_iter <= JR_MAX_ITER, out_offset >= 0, out_offset + width*height <=
 * out_capacity.
 *
 * degree selects the map (the paper's further functions, Section 4):
 * 0 or 2 is Z^2 + C; 3..8 is the general map Z^degree + C, with Z^degree
 * formed by degree - 1 complex products W <- W Z from W = Z, each product
 * (a + ib)(x + iy) taken as (a x - b y) + i (a y + b x) and every operation
 * rounded, then C added.  Its FP64 and FP32 forms use no fused operations
 * and test fl(fl(x x) + fl(y y)) > 4; float-float uses its double-word
 * operations throughout.  Count, escape radius and pixel mapping are those
 * of Z^2 + C.
 *
 * map selects the family (the further functions and parameters of Section 4
 * and the closing discussion):
 *   JR_MAP_POLY      Z^degree + C (above);
 *   JR_MAP_RATIONAL  the two-parameter rational map
 *                        Z_{n+1} = W + C + lambda / W,  W = Z_n^degree
 *                    (degree 0 means 2), Julia mode only, dtype JR_FP64 or
 *                    JR_FP32.  W is formed as for the general maps; with
 *                    q = wr*wr + wi*wi, the update is
 *                        x' = (wr + cr) + (lr*wr + li*wi) / q,
 *                        y' = (wi + ci) + (li*wr - lr*wi) / q,
 *                    every product, sum and quotient rounded (IEEE division,
 *                    no fused operations); a pixel escapes unless
 *                    fl(fl(x*x) + fl(y*y)) <= 4, so the iterate after a hit on
 *                    the pole Z = 0 (0/0, not a number) counts as escaped.
 *                    Launches holding such frames run the rows kernel (a
 *                    schedule asking for the tiled or hybrid kernels is
 *                    carried over to it) or, when asked, the plain kernel.
 */
typedef enum { JR_MAP_POLY = 0, JR_MAP_RATIONAL = 1 } jr_map;
typedef struct {
    jr_complex c;
    jr_window w;
    int32_t width, height;
    int32_t max_iter;
    int32_t dtype;      /* jr_dtype */
    int32_t mode;       /* jr_mode  */
    int32_t row_begin;  /* first row computed (0 = top)        */
    int32_t row_end;    /* one past the last row; 0 = height   */
    int32_t degree;     /* 0 or 2: Z^2 + C; 3..8: Z^degree + C */
    int64_t out_offset; /* element offset of pixel (0, 0)      */
    int32_t map;        /* jr_map                               */
    int32_t reserved;   /* 0                                    */
    jr_complex lambda;  /* JR_MAP_RATIONAL: lambda; finite      */
} jr_frame;

/*
 * Schedule of a batch launch.  None of these fields changes a count: they
 * decide which lane computes which pixel and when, never the arithmetic.
 *   tile_w, tile_h  pixels per work tile: 1 <= tile_w <= 64, 1 <= tile_h <= 64.
 *   unroll          iterations per branch-free block: 1, 2, 4 or 8, or with
 *                   defer = 1: 4, 8 or 16.
 *   defer           0: every iterate is tested inside the block and the
 *                   leading non-escaped iterates are counted; 1: only the
 *                   block's last iterate is tested and lanes found escaped are
 *                   replayed from the block start.  Both give the counts of a
 *                   test on every iteration; frames where escape is not known
 *                   to be absorbing (|C| > 1.9 somewhere) run with unroll 1.
 *   refill          idle lanes in a wave that trigger a refill round, 1..64:
 *                   finished lanes store their count and take the next pixels,
 *                   from the next tile when the current one is used up.
 *   persistent      1: waves_per_cu resident waves per compute unit take tiles
 *                   from 64 atomic work queues, stealing from other queues when
 *                   theirs is empty; 0: one wave per tile, placed by the
 *                   hardware dispatcher.
 *   waves_per_cu    persistent mode: resident waves per compute unit
 *                   (4..32, a multiple of 4).
 *   order           JR_ORDER_TABLE: frames in the order given;
 *                   JR_ORDER_COST: most expensive frames first (estimated
 *                   from size, cap and dtype).
 *   kernel          JR_KERNEL_TILED: the tiled kernel above;
 *                   JR_KERNEL_PLAIN: one thread per pixel over the whole batch
 *                   (16 x 16 tiles, one workgroup each, a test on every
 *                   iteration); the other fields are then ignored;
 *                   JR_KERNEL_HYBRID: the tiled kernel where each wave runs 64
 *                   fresh pixels at a time with a test on every iteration and
 *                   only the pixels still running after `bail` iterations
 *                   continue in refilled blocks (they wait in shared memory).
 *                   JR_KERNEL_ROWS: each wave takes a tile row by row (lane
 *                   = column); every pixel of a row first runs up to `bail`
 *                   counted iterations (rounded up to a multiple of 4), with
 *                   no exchange between lanes.  Pixels that finish store at
 *                   once; the others wait in a per-wave list in shared
 *                   memory, which the wave drains with refilled blocks of
 *                   `unroll` (4 or 8) whenever it could not take the next
 *                   rows' survivors, and at the end of the tile: counted
 *                   blocks with defer 0; with defer 1, in launches of FP32
 *                   frames only or FP64 frames only, blocks that test their
 *                   last iterate, the lanes found escaped being replayed
 *                   with the counted test at the next refill round (other
 *                   launches take counted blocks).
 *   bail            JR_KERNEL_HYBRID: 1..4096; JR_KERNEL_ROWS: 1..64 (other
 *                   kernels ignore it).
 *   handoff         JR_KERNEL_ROWS, 0..256: rows run in groups for FP32 and
 *                   FP64 (quadratic maps): four rows at a time in batches of
 *                   FP32 frames only, two otherwise.  A group stops its first
 *                   iterations, after a multiple of 4 of them, once at most
 *                   `handoff` of its pixels are still inside the disc; those
 *                   join the list with their count so far.  With 0 a group
 *                   stops once all its pixels have escaped.  Single rows
 *                   always stop then.  Other kernels ignore it.
 */
typedef enum {
    JR_KERNEL_TILED = 0,
    JR_KERNEL_PLAIN = 1,
    JR_KERNEL_HYBRID = 2,
    JR_KERNEL_ROWS = 3
} jr_kernel;
typedef struct {
    int32_t tile_w, tile_h;
    int32_t unroll;
    int32_t defer;
    int32_t refill;
    int32_t persistent;
    int32_t waves_per_cu;
    int32_t order;
    int32_t kernel;
    int32_t bail;
    int32_t handoff;
} jr_schedule;

/*
 * Render one Julia image (Section 2) with the tuned kernels.
 * out: device, width*height int32, row-major.  The schedule is the one
 * jr_get_image_schedule gives for (dtype, max_iter, width*height): the
 * per-image entry installed by jr_set_image_schedule that covers the cap and
 * size (the Python binding installs the autotuner's winners), else the
 * dtype's default (jr_get_default_schedule).
 */
int julia_render(jr_complex c, jr_window w, int32_t width, int32_t height,
                 int32_t max_iter, int32_t dtype, int32_t *out, void *stream);

/*
 * Same image and the same counts with the plain kernel: one thread per pixel
 * on a 2-D grid of 16x16 workgroups, escape test on every iteration.  The
 * comparator the tuned kernels are measured against.
 */
int julia_render_plain(jr_complex c, jr_window w, int32_t width, int32_t height,
                       int32_t max_iter, int32_t dtype, int32_t *out, void *stream);

/* Mandelbrot image (Section 3: C = pixel, Z_0 = 0), tuned and plain kernels. */
int mandelbrot_render(jr_window w, int32_t width, int32_t height, int32_t max_iter,
                      int32_t dtype, int32_t *out, void *stream);
int mandelbrot_render_plain(jr_window w, int32_t width, int32_t height,
                            int32_t max_iter, int32_t dtype, int32_t *out,
                            void *stream);

/*
 * Render n frames (any mix of sizes, caps, dtypes and modes) in ONE launch of
 * the tiled kernel (persistent work-stealing waves by default).  frames: host array of n >= 1
 * descriptors, copied before return.  out_base: device arena of out_capacity
 * int32 elements holding every frame at its out_offset.  sched: NULL for the
 * default schedule of the batch's dominant dtype.  Frames must not overlap in
 * the arena where their computed rows overlap.  A one-frame call passes the
 * frame inside the kernel arguments; without the persistent work queues it is
 * a single kernel launch that a hipGraph capture may record.  A call with
 * several frames uploads a table and returns JR_EINVAL on a capturing stream
 * (use jr_plan_capture).
 */
int julia_render_batch(const jr_frame *frames, int32_t n, int32_t *out_base,
                       int64_t out_capacity, const jr_schedule *sched, void *stream);

/*
 * Allocation-free form of julia_render_batch, for callers that cannot allocate
 * memory: code under hipGraph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, frames, schedules, kernels and counts as
 * julia_render_batch, but the call allocates nothing, on the device or the
 * host: the frame table and the work-queue counters live in one fixed device
 * array of the library (JR_NOALLOC_SCRATCH_BYTES, one copy per GPU, held until
 * the process ends), and the table reaches it through kernel arguments, in
 * stream order, so `frames` may be reused once the call returns.  The queue
 * counters are zeroed by a kernel before each launch that uses them.
 *   n            1 .. JR_NOALLOC_MAX_FRAMES; more frames are rejected with
 *                JR_EINVAL before anything reaches the device.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (on different streams, or from
 * several threads without ordering) race and may render wrong images.  Order
 * them, on one stream or with events.  Other errors are julia_render_batch's.
 */
#define JR_NOALLOC_MAX_FRAMES 1024
#define JR_NOALLOC_SCRATCH_BYTES (64 * 4096 + JR_NOALLOC_MAX_FRAMES * 144)
int julia_render_batch_noalloc(const jr_frame *frames, int32_t n, int32_t *out_base,
                               int64_t out_capacity, const jr_schedule *sched, void *stream);

/*
 * Prescribed parameter path (Section 3) with its constants generated on the
 * device: frames 0 .. frames-1 of one size, window, cap and dtype, whose
 * constants lie on the cardioid
 *     f(t) = ((2 cos t - cos 2t) / a, (2 sin t - sin 2t) / a) = (2u - u^2) / a,
 * u = e^{it}, stepping by `step` = e^{i dt} per frame while the cardioid grows
 * (a decreasing: a_k = a0 - da k; a = 4 is the main cardioid's border).  A
 * kernel writes the frame table, frame k's constant being
 *     u_k = step^k  by square-and-multiply over the bits of k, highest first
 *                   (p = 1; per bit: p = p*p, then p = p*step if it is set),
 *     C_k = (2 u_k - u_k*u_k) / (a0 - da k),
 * with every complex product (a + ib)(c + id) = (a*c - b*d) + i (a*d + b*c)
 * and every real operation rounded to binary64; then the batch is rendered as
 * julia_render_batch renders it.  Frame k occupies width*height elements at
 * out_offset + k*width*height.
 *   step     finite; frames * |log|step|| <= 1e-6 (so |u_k| stays within
 *            1e-6 of 1).
 *   a0, da   finite; a0 and a0 - da (frames - 1) at least JR_CARDIOID_MIN_A,
 *            so that |C_k| <= 3.000003 / 1.6 < 1.9 and escape is absorbing.
 *   frames   1 .. 2^22; dtype any; Julia mode, Z^2 + C.
 * Errors as julia_render_batch; JR_EINVAL for a path outside these limits.
 */
#define JR_CARDIOID_MIN_A 1.6
typedef struct {
    jr_complex step;
    double a0, da;
    jr_window w;
    int32_t frames;
    int32_t width, height, max_iter, dtype;
    int32_t reserved;
    int64_t out_offset;
} jr_cardioid_path;
int julia_render_cardioid_path(const jr_cardioid_path *path, int32_t *out_base,
                               int64_t out_capacity, const jr_schedule *sched, void *stream);

/*
 * Fused count -> colour store (Section 2: every pixel is given a colour level
 * by its iteration count).  The frames, schedules and kernels are those of
 * julia_render_batch; only the stored value changes: each pixel stores the
 * 32-bit table entry
 *     palette[min(count, palette_len - 1)]
 * in place of its count (for example an RGBA8 colour packed into 32 bits), so
 * no count image is written and read back to colour it.
 *   palette      device, palette_len uint32 entries, 4-byte aligned.  It is
 *                read when the kernel runs, so it must stay valid and
 *                unchanged until the stream has passed the launch.  Each
 *                workgroup copies it into shared memory: a long table lowers
 *                the number of resident workgroups.
 *   palette_len  1 .. JR_PALETTE_MAX.
 *   out_base     device arena as in julia_render_batch, one uint32 per pixel.
 * Errors: JR_EINVAL for a null or misaligned palette, a length out of range,
 * or what julia_render_batch rejects.  Capture rules are julia_render_batch's.
 */
#define JR_PALETTE_MAX 8192
int julia_render_batch_colored(const jr_frame *frames, int32_t n, const uint32_t *palette,
                               int32_t palette_len, uint32_t *out_base,
                               int64_t out_capacity, const jr_schedule *sched,
                               void *stream);

/*
 * One Julia image (Section 2) with the fused colour store: the image of
 * julia_render, each pixel stored as palette[min(count, palette_len - 1)].
 * out: device, width*height uint32, row-major.  Palette rules as above.
 */
int julia_render_colored(jr_complex c, jr_window w, int32_t width, int32_t height,
                         int32_t max_iter, int32_t dtype, const uint32_t *palette,
                         int32_t palette_len, uint32_t *out, void *stream);

/*
 * Prepared batch: validates and uploads the frame table once (synchronously),
 * so that repeated launches or a captured hipGraph replay cost one kernel
 * launch.  A plan's launches must not overlap each other (they share the
 * plan's tile counter); run them on one stream or order them.
 */
typedef struct jr_plan jr_plan;
int jr_plan_create(const jr_frame *frames, int32_t n, int32_t *out_base,
                   int64_t out_capacity, const jr_schedule *sched, jr_plan **plan);
/* A plan over a prescribed cardioid path (julia_render_cardioid_path): each
 * launch (and a captured graph) first generates the frame table on the
 * device, then renders it. */
int jr_plan_create_cardioid(const jr_cardioid_path *path, int32_t *out_base,
                            int64_t out_capacity, const jr_schedule *sched, jr_plan **plan);
int jr_plan_launch(jr_plan *plan, void *stream);
/* Capture one launch into a hipGraph on `stream` (once), then replay it. */
int jr_plan_capture(jr_plan *plan, void *stream);
int jr_plan_replay(jr_plan *plan, void *stream);
/*
 * Make the plan's launches store colours from this table (see
 * julia_render_batch_colored); palette NULL with palette_len 0 returns to
 * counts.  A graph captured earlier is discarded: capture again before the
 * next replay (replay returns JR_EINVAL until then).  The table must stay
 * valid while launches that use it are in flight.
 */
int jr_plan_set_palette(jr_plan *plan, const uint32_t *palette, int32_t palette_len);
/*
 * Progress of a plan's launches: per-frame done counters and a stop flag, the
 * bookkeeping of the long batches of Section 3 (parameter paths and zooms of
 * many frames), so that a launch stopped early leaves a record of which
 * frames are complete and a caller re-renders only the others.
 *   done   device memory, one int32 per frame of the plan, done[k] for frame k
 *          of the list given to jr_plan_create (frame k of the path for a
 *          cardioid plan), caller-owned, valid while launches that use it are
 *          in flight.  Each launch first
 *          zeroes it (a kernel, in stream order, so a captured graph does too),
 *          then adds each tile's pixel count to its frame's counter once all
 *          of the tile's pixels are stored.  Frame f is complete when
 *          done[f] == width * (row_end - row_begin) of its descriptor.
 *   stop   NULL, or an int32 flag the kernel reads (device memory, or pinned
 *          host memory from hipHostMalloc) before each tile it claims: while
 *          it is nonzero, waves claim no further tiles and exit.  Tiles already
 *          claimed are finished and counted, so a stopped launch leaves whole
 *          tiles and exact counters; the pixels of incomplete frames are
 *          partly written.  Requires done.
 * done NULL (with stop NULL) turns progress off.  Only plans whose schedule
 * runs the rows or plain kernel count progress; others return JR_EINVAL.  A
 * graph captured earlier is discarded (capture again).  A counting launch
 * runs a kernel variant that holds every map and dtype plus the progress
 * code, and adds one atomic per tile; launches without progress run variants
 * that hold none of it.
 */
int jr_plan_set_progress(jr_plan *plan, int32_t *done, const int32_t *stop);
/* Number of tiles of the plan and the workgroups it launches (for
 * accounting): one per tile where the rows kernel runs one wave per tile. */
int jr_plan_info(const jr_plan *plan, int64_t *tiles, int32_t *workgroups);
void jr_plan_destroy(jr_plan *plan);

/* Library default schedule of a dtype, used by batch calls with sched NULL
 * and by one-image calls that no per-image entry covers.  There is one
 * default per dtype, the same for every cap: max_iter is checked (0 ..
 * JR_MAX_ITER, JR_EINVAL otherwise) and does not change the result. */
int jr_get_default_schedule(int32_t dtype, int32_t max_iter, jr_schedule *out);
int jr_set_default_schedule(int32_t dtype, const jr_schedule *sched);

/*
 * Schedules of one-image calls (julia_render, mandelbrot_render,
 * julia_render_colored), chosen by the image's cap and size: a call takes the
 * entry of its dtype with the smallest max_iter_limit >= max_iter and, among
 * those, the smallest pixels_limit >= width*height, or when no entry's
 * pixels_limit covers the image, the one with the largest pixels_limit; with
 * no entry for its dtype and cap it takes the dtype's default.  An entry whose
 * kernel is JR_KERNEL_PLAIN runs the 2-D kernel of julia_render_plain (the
 * colored call runs the batched plain kernel).  An entry with the same
 * (dtype, max_iter_limit, pixels_limit) is replaced; at most 64 entries
 * (JR_EINVAL beyond).  The Python binding installs the autotuner's per-image
 * winners here.
 */
int jr_set_image_schedule(int32_t dtype, int32_t max_iter_limit, int64_t pixels_limit,
                          const jr_schedule *sched);
/* The schedule a one-image call of this dtype, cap and pixel count takes. */
int jr_get_image_schedule(int32_t dtype, int32_t max_iter, int64_t pixels, jr_schedule *out);
void jr_clear_image_schedules(void);

/* Validate a schedule or a frame table without touching the device. */
int jr_check_schedule(const jr_schedule *sched);
int jr_check_frames(const jr_frame *frames, int32_t n, int64_t out_capacity);

const char *jr_strerror(int code);
const char *jr_last_error_message(void);

/* Compute units and HBM bytes of the current device (for admission control). */
int jr_device_info(int32_t *num_cus, int64_t *hbm_bytes);

/* Free the library's per-stream workspaces (frame tables, counters, staging).
 * No call may be in flight. */
void jr_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* JULIA_H */
