// julia_kernels.hip -- device code of libjulia.so (gfx950 / CDNA4, wave64).
//
// Escape-time iteration Z_{n+1} = Z_n^2 + C over a pixel grid scaled onto a
// window of the complex plane, count = first n with |Z_n|^2 > 4, capped at
// max_iter (Mayfield et al., Section 2); Mandelbrot variant with C = pixel and
// Z_0 = 0 (Section 3).
//
// The work is plain vector-ALU arithmetic (about 8 flops per pixel-iteration,
// nothing is read from memory, 4 bytes are written per pixel), so there is no
// matrix-core path.  Two kernel families:
//
//   jr_plain<A>       one thread per pixel on a 2-D grid, escape test on every
//                     iteration.  The straightforward design (the paper's own
//                     GPU version assigns one thread to each point) and the
//                     comparator for the tuned kernel.
//
//   jr_persistent<K,M> persistent waves over a table of frames.  Each wave
//                     claims granules of tiles from atomic counters (64
//                     queues; an idle wave steals from any queue that still
//                     has work, across frames of different cost), and
//                     inside a tile its 64 lanes take pixels one after the
//                     other: a lane that finishes stores its count and takes
//                     the tile's next pixel (lane refill), so divergent escape
//                     counts do not leave lanes idle until the slowest pixel of
//                     a fixed 64-pixel block ends.  With K > 1 the escape test
//                     runs once every K iterations; a lane found escaped is
//                     replayed from its saved state with a test on every
//                     iteration, which gives the same count bit for bit
//                     because escape is absorbing when |C| <= 1.9.
//
// This translation unit is compiled with -ffp-contract=off: every a*b + c
// below is a rounded product and a rounded sum unless fmaf() is written out.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "julia_device.h"

namespace jr {

// ---------------------------------------------------------------------------
// Arithmetic formulations.  Each provides a state Z, a constant C, construction
// from binary64 values, inside() = (|Z|^2 <= 4, false for NaN), step() and
// check_step() (tests the current Z, then advances it, sharing the squares).
// ---------------------------------------------------------------------------
struct ArF64 {
    struct Z { double x, y; };
    struct C { double r, i; };
    __device__ static Z make(double x, double y) { return Z{x, y}; }
    __device__ static C cmake(double r, double i) { return C{r, i}; }
    __device__ static bool inside(const Z& z) {
        double x2 = z.x * z.x;
        double y2 = z.y * z.y;
        return x2 + y2 <= 4.0;
    }
    __device__ static void advance(Z& z, const C& c, double x2, double y2) {
        double re = x2 - y2;
        double xn = re + c.r;
        double tx = z.x + z.x;           // 2x, exact
        double im = tx * z.y;
        double yn = im + c.i;
        z.x = xn;
        z.y = yn;
    }
    __device__ static void step(Z& z, const C& c) {
        double x2 = z.x * z.x;
        double y2 = z.y * z.y;
        advance(z, c, x2, y2);
    }
    __device__ static bool check_step(Z& z, const C& c) {
        double x2 = z.x * z.x;
        double y2 = z.y * z.y;
        bool ok = (x2 + y2 <= 4.0);
        advance(z, c, x2, y2);
        return ok;
    }
};

struct ArF32 {
    struct Z { float x, y; };
    struct C { float r, i; };
    __device__ static Z make(double x, double y) { return Z{(float)x, (float)y}; }
    __device__ static C cmake(double r, double i) { return C{(float)r, (float)i}; }
    __device__ static bool inside(const Z& z) {
        float yy = z.y * z.y;
        return __builtin_fmaf(z.x, z.x, yy) <= 4.0f;
    }
    __device__ static void step(Z& z, const C& c) {
        float t = __builtin_fmaf(z.x, z.x, c.r);
        float xn = __builtin_fmaf(-z.y, z.y, t);
        float tx = z.x + z.x;
        float yn = __builtin_fmaf(tx, z.y, c.i);
        z.x = xn;
        z.y = yn;
    }
    __device__ static bool check_step(Z& z, const C& c) {
        bool ok = inside(z);
        step(z, c);
        return ok;
    }
};

// Float-float: value = hi + lo.  TwoSum (Knuth), Fast2Sum (Dekker), FMA-based
// TwoProd, and the double-word sum and product of Joldes, Muller and Popescu
// (ACM TOMS 2017): accurate double-word + double-word (error < 3u^2) and
// FMA double-word x double-word (error < 4u^2), u = 2^-24.
struct ArFF {
    struct D { float hi, lo; };
    struct Z { D x, y; };
    struct C { D r, i; };

    __device__ static void two_sum(float a, float b, float& s, float& e) {
        s = a + b;
        float bv = s - a;
        float av = s - bv;
        e = (a - av) + (b - bv);
    }
    __device__ static void quick_two_sum(float a, float b, float& s, float& e) {
        s = a + b;
        float bv = s - a;
        e = b - bv;
    }
    __device__ static D add(D a, D b) {
        float s, se, t, te, v, ve;
        two_sum(a.hi, b.hi, s, se);
        two_sum(a.lo, b.lo, t, te);
        float c = se + t;
        quick_two_sum(s, c, v, ve);
        float w = te + ve;
        D r;
        quick_two_sum(v, w, r.hi, r.lo);
        return r;
    }
    __device__ static D mul(D a, D b) {
        float p = a.hi * b.hi;
        float pe = __builtin_fmaf(a.hi, b.hi, -p);
        float ll = a.lo * b.lo;
        float m1 = __builtin_fmaf(a.hi, b.lo, ll);
        float m2 = __builtin_fmaf(a.lo, b.hi, m1);
        float q = pe + m2;
        D r;
        quick_two_sum(p, q, r.hi, r.lo);
        return r;
    }
    __device__ static D split(double v) {
        D r;
        r.hi = (float)v;
        r.lo = (float)(v - (double)r.hi);
        return r;
    }
    __device__ static Z make(double x, double y) { return Z{split(x), split(y)}; }
    __device__ static C cmake(double r, double i) { return C{split(r), split(i)}; }
    __device__ static bool le4(D m) { return (m.hi < 4.0f) || (m.hi == 4.0f && m.lo <= 0.0f); }
    __device__ static bool inside(const Z& z) {
        return le4(add(mul(z.x, z.x), mul(z.y, z.y)));
    }
    __device__ static void advance(Z& z, const C& c, D x2, D y2) {
        D ny2 = D{-y2.hi, -y2.lo};
        D re = add(x2, ny2);
        D xn = add(re, c.r);
        D tx = D{z.x.hi + z.x.hi, z.x.lo + z.x.lo};  // 2x, exact
        D im = mul(tx, z.y);
        D yn = add(im, c.i);
        z.x = xn;
        z.y = yn;
    }
    __device__ static void step(Z& z, const C& c) {
        D x2 = mul(z.x, z.x);
        D y2 = mul(z.y, z.y);
        advance(z, c, x2, y2);
    }
    __device__ static bool check_step(Z& z, const C& c) {
        D x2 = mul(z.x, z.x);
        D y2 = mul(z.y, z.y);
        bool ok = le4(add(x2, y2));
        advance(z, c, x2, y2);
        return ok;
    }
};

// Pixel centre in binary64: cx + (2i + 1 - W) hx, cy - (2j + 1 - H) hy.  The
// odd integer is formed exactly in binary64 (|values| < 2^33).
__device__ __forceinline__ double pixel_re(double cx, double hx, int i, int W) {
    double o = ((double)i + (double)i) + (double)(1 - W);
    double p = o * hx;
    return cx + p;
}
__device__ __forceinline__ double pixel_im(double cy, double hy, int j, int H) {
    double o = ((double)j + (double)j) + (double)(1 - H);
    double p = o * hy;
    return cy - p;
}

// ---------------------------------------------------------------------------
// Plain kernel: one thread per pixel, 16x16 workgroups, test every iteration.
// ---------------------------------------------------------------------------
template <class A>
__global__ __launch_bounds__(256) void jr_plain(PlainArgs p) {
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    if (i >= p.W) return;
    for (int j = blockIdx.y * 16 + (threadIdx.x >> 4); j < p.H; j += gridDim.y * 16) {
        double px = pixel_re(p.cx, p.hx, i, p.W);
        double py = pixel_im(p.cy, p.hy, j, p.H);
        typename A::Z z;
        typename A::C c;
        if (p.mode == kModeMandelbrot) {
            z = A::make(0.0, 0.0);
            c = A::cmake(px, py);
        } else {
            z = A::make(px, py);
            c = A::cmake(p.cr, p.ci);
        }
        int n = 0;
        while (n < p.max_iter) {
            if (!A::check_step(z, c)) break;
            n++;
        }
        p.out[(int64_t)j * p.W + i] = n;
    }
}

// ---------------------------------------------------------------------------
// Persistent kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

struct TileCtx {
    int32_t* out;          // frame pixel (0, 0)
    double cx, cy, hx, hy, cr, ci;
    int W, H, max_iter, mode;
    int col0, row0, tw, th;
};

// One tile of tw x th pixels, row-major inside the tile, processed by one
// wave with lane refill.  Lane state: z (current iterate), zs (iterate at the
// start of the running block), n (iterations done), and one of
//   active   iterating a pixel,
//   pending  escaped inside the last block, count found by replay,
//   done     final count in cnt, store outstanding,
//   idle     nothing.
// Refill rounds run when at least `refill` lanes are not active or none is.
template <class A, int K>
__device__ void run_tile(const TileCtx& T, int refill) {
    const int npix = T.tw * T.th;
    const float rtw = 1.0f / (float)T.tw;
    int next = 0;  // wave-uniform: first pixel of the tile not yet handed out
    bool active = false, pending = false, done = false;
    int n = 0, cnt = 0, off = 0;
    typename A::Z z = A::make(0.0, 0.0);
    typename A::Z zs = z;
    typename A::C c = A::cmake(0.0, 0.0);

    for (;;) {
        const uint64_t busy = __ballot(active);
        const int nidle = 64 - __popcll(busy);
        if (nidle >= refill || busy == 0) {
            if (K > 1 && __ballot(pending) != 0) {
                if (pending) {
                    // Replay the block from its saved start with a test on
                    // every iteration.  The block-end test said |Z|^2 > 4 at
                    // n + K, and escape is absorbing, so the first escaped
                    // iterate lies in [n, n + K]; the cap may come first.
                    z = zs;
                    const int lim = min(K, T.max_iter - n);
                    int j = 0;
                    while (j < lim && A::check_step(z, c)) j++;
                    cnt = n + j;
                    done = true;
                    pending = false;
                }
            }
            if (done) {
                T.out[off] = cnt;
                done = false;
            }
            if (next < npix) {
                const int k = next + lanes_below(~busy);
                if (!active && k < npix) {
                    int row = (int)((float)k * rtw);
                    int col = k - row * T.tw;
                    if (col < 0) { row -= 1; col += T.tw; }
                    else if (col >= T.tw) { row += 1; col -= T.tw; }
                    const int gi = T.col0 + col;
                    const int gj = T.row0 + row;
                    const double px = pixel_re(T.cx, T.hx, gi, T.W);
                    const double py = pixel_im(T.cy, T.hy, gj, T.H);
                    if (T.mode == kModeMandelbrot) {
                        z = A::make(0.0, 0.0);
                        c = A::cmake(px, py);
                    } else {
                        z = A::make(px, py);
                        c = A::cmake(T.cr, T.ci);
                    }
                    n = 0;
                    off = gj * T.W + gi;
                    active = true;
                }
                next += nidle;
            }
            if (__ballot(active) == 0) break;
        }
        if (active) {
            if (K == 1) {
                const bool ok = A::check_step(z, c);
                if (!ok || n >= T.max_iter) {
                    cnt = n;
                    done = true;
                    active = false;
                } else {
                    n++;
                }
            } else {
                zs = z;
#pragma unroll
                for (int u = 0; u < K; ++u) A::step(z, c);
                if (!A::inside(z)) {
                    pending = true;
                    active = false;
                } else {
                    n += K;
                    if (n >= T.max_iter) {  // no escape up to n >= cap: absorbing
                        cnt = T.max_iter;
                        done = true;
                        active = false;
                    }
                }
            }
        }
    }
}

template <class A, int K>
__device__ __forceinline__ void run_frame_tile(const TileCtx& T, int defer, int refill) {
    if (K > 1 && defer)
        run_tile<A, K>(T, refill);
    else
        run_tile<A, 1>(T, refill);
}

__device__ __forceinline__ unsigned long long* queue_ctr(unsigned long long* ctr, int q) {
    return ctr + (size_t)q * kQueueStride;
}

// Granules in queue q: granules q, q + kQueues, q + 2 kQueues, ...
__device__ __forceinline__ int64_t queue_len(int64_t granules, int q) {
    return granules > q ? (granules - q + kQueues - 1) / kQueues : 0;
}

// Largest frame index f with frames[f].tile_begin <= t.  Tiles of one granule
// are consecutive and a queue's granules increase, so a short forward scan
// from the previous frame usually ends it; otherwise binary search.
__device__ __forceinline__ int find_frame(const DevFrame* __restrict__ frames, int nframes,
                                          int64_t t, int f) {
    if (frames[f].tile_begin <= t) {
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
            if (f + 1 < nframes && frames[f + 1].tile_begin <= t)
                f++;
            else
                return f;
        }
    }
    int lo = 0, hi = nframes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (frames[mid].tile_begin <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int K, int DTMASK>
__device__ __forceinline__ void run_global_tile(const PersistentArgs& a, int f, int64_t t) {
    const DevFrame& F = a.frames[f];
    const int64_t local = t - F.tile_begin;
    const int ty = (int)(local / F.tiles_x);
    const int tx = (int)(local - (int64_t)ty * F.tiles_x);
    TileCtx T;
    T.out = a.out_base + F.out_offset;
    T.cx = F.cx; T.cy = F.cy; T.hx = F.hx; T.hy = F.hy; T.cr = F.cr; T.ci = F.ci;
    T.W = F.width; T.H = F.height; T.max_iter = F.max_iter; T.mode = F.mode;
    T.col0 = tx * F.tile_w;
    T.row0 = F.row_begin + ty * F.tile_h;
    T.tw = min(F.tile_w, F.width - T.col0);
    T.th = min(F.tile_h, F.row_end - T.row0);
    const int dt = F.dtype;
    if ((DTMASK & (1 << kFP32)) && dt == kFP32)
        run_frame_tile<ArF32, K>(T, F.defer, a.refill);
    else if ((DTMASK & (1 << kFP64)) && dt == kFP64)
        run_frame_tile<ArF64, K>(T, F.defer, a.refill);
    else if ((DTMASK & (1 << kFF)) && dt == kFF)
        run_frame_tile<ArFF, K>(T, F.defer, a.refill);
}

// Persistent workgroups of 256 threads: 4 independent waves.  Wave w starts on
// queue w % kQueues and always holds one claim in flight (the atomic for the
// next granule is issued before the current one is computed).  When its queue
// is empty, the wave reads all kQueues counters at once (one per lane) and
// moves to the next queue that still has granules; it leaves when none has.
template <int K, int DTMASK>
__global__ __launch_bounds__(256) void jr_persistent(PersistentArgs a) {
    const int lane = lane_id();
    const int wave = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    int q = wave % kQueues;
    int64_t qlen = queue_len(a.granules, q);
    unsigned long long raw = 0;
    if (lane == 0) raw = atomicAdd(queue_ctr(a.ctr, q), 1ull);
    int f = 0;
    for (;;) {
        const int64_t j = uniform64((int64_t)raw);
        if (j >= qlen) {
            bool has = false;
            if (lane < kQueues) {
                const unsigned long long c = __hip_atomic_load(
                    queue_ctr(a.ctr, lane), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                has = (int64_t)c < queue_len(a.granules, lane);
            }
            const uint64_t m = __ballot(has);
            if (m == 0) break;
            const int s = (q + 1) & (kQueues - 1);
            const uint64_t rot = s ? ((m >> s) | (m << (64 - s))) : m;
            q = (s + __builtin_ctzll(rot)) & (kQueues - 1);
            qlen = queue_len(a.granules, q);
            if (lane == 0) raw = atomicAdd(queue_ctr(a.ctr, q), 1ull);
            continue;
        }
        if (lane == 0) raw = atomicAdd(queue_ctr(a.ctr, q), 1ull);  // next claim, in flight
        const int64_t t0 = (j * kQueues + q) * (int64_t)a.granule;
        const int64_t t1 = min(t0 + (int64_t)a.granule, a.total_tiles);
        for (int64_t t = t0; t < t1; ++t) {
            f = find_frame(a.frames, a.nframes, t, f);
            run_global_tile<K, DTMASK>(a, f, t);
        }
    }
}

// Zeroes the kQueues counters before a persistent launch (a kernel, not a
// memset, so that it can sit inside a captured hipGraph).
__global__ void jr_reset_queues(unsigned long long* ctr) {
    if (threadIdx.x < kQueues) ctr[(size_t)threadIdx.x * kQueueStride] = 0ull;
}

}  // namespace jr

// ---------------------------------------------------------------------------
// Launch helpers used by the host runtime (julia_host.hip).
// ---------------------------------------------------------------------------
namespace jr {

using PersistentFn = void (*)(PersistentArgs);

template <int K>
static PersistentFn pick_mask(int dtmask) {
    switch (dtmask) {
        case 1 << kFP64: return jr_persistent<K, 1 << kFP64>;
        case 1 << kFP32: return jr_persistent<K, 1 << kFP32>;
        case 1 << kFF: return jr_persistent<K, 1 << kFF>;
        default: return jr_persistent<K, 7>;
    }
}

hipError_t launch_persistent(int unroll, int dtmask, int blocks, const PersistentArgs& args,
                             hipStream_t stream) {
    PersistentFn fn;
    switch (unroll) {
        case 1: fn = pick_mask<1>(dtmask); break;
        case 4: fn = pick_mask<4>(dtmask); break;
        case 8: fn = pick_mask<8>(dtmask); break;
        case 16: fn = pick_mask<16>(dtmask); break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(jr_reset_queues, dim3(1), dim3(kQueues), 0, stream, args.ctr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), 0, stream, args);
    return hipGetLastError();
}

hipError_t launch_plain(int dtype, const PlainArgs& args, hipStream_t stream) {
    const unsigned gx = (unsigned)((args.W + 15) / 16);
    const int64_t rows16 = ((int64_t)args.H + 15) / 16;
    const unsigned gy = (unsigned)(rows16 < 65535 ? rows16 : 65535);
    dim3 grid(gx, gy);
    switch (dtype) {
        case kFP64: hipLaunchKernelGGL(jr_plain<ArF64>, grid, dim3(256), 0, stream, args); break;
        case kFP32: hipLaunchKernelGGL(jr_plain<ArF32>, grid, dim3(256), 0, stream, args); break;
        case kFF: hipLaunchKernelGGL(jr_plain<ArFF>, grid, dim3(256), 0, stream, args); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace jr
