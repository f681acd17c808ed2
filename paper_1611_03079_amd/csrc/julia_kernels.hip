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
//   jr_tiled<K,D,M>   waves over a table of frames.  In persistent mode each
//                     wave claims granules of tiles from atomic counters (64
//                     queues; an idle wave steals from any queue that still
//                     has work, across frames of different cost); otherwise
//                     one wave per tile.  The 64 lanes of a wave take pixels
//                     one after the other: a lane that finishes stores its
//                     count and takes the next pixel (lane refill), from the
//                     next tile when the current one runs out, so divergent
//                     escape counts do not leave lanes idle until the slowest
//                     pixel of a fixed block ends.  Iterations run in blocks
//                     of K without branches; the escape test is counted on
//                     every iterate, or (D = 1) run once per block with a
//                     replay of the lanes found escaped.  Both give the counts
//                     of a test on every iteration bit for bit, because escape
//                     is absorbing when |C| <= 1.9 (other frames use K = 1).
//
// This translation unit is compiled with -ffp-contract=off: every a*b + c
// below is a rounded product and a rounded sum unless fmaf() is written out.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "julia_device.h"

namespace jr {

// ---------------------------------------------------------------------------
// Arithmetic formulations.  Each provides a state Z, a constant C, construction
// from binary64 values, inside() = (|Z|^2 <= 4, false for NaN), step() and
// check_step() (tests the current Z, then advances it, sharing the squares).
// ---------------------------------------------------------------------------
struct ArF64 {
    static constexpr bool kRational = false;
    struct Z { double x, y; };
    struct C { double r, i; };
    using V = double;  // one coordinate
    __device__ static V coord(double v) { return v; }
    __device__ static V shfl(V v, int src) { return __shfl(v, src); }
    __device__ static Z make(V x, V y) { return Z{x, y}; }
    __device__ static C cmake(V r, V i) { return C{r, i}; }
    __device__ static bool inside(const Z& z, const C&, int) {
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
    __device__ static void step(Z& z, const C& c, int) {
        double x2 = z.x * z.x;
        double y2 = z.y * z.y;
        advance(z, c, x2, y2);
    }
    __device__ static bool check_step(Z& z, const C& c, int) {
        double x2 = z.x * z.x;
        double y2 = z.y * z.y;
        bool ok = (x2 + y2 <= 4.0);
        advance(z, c, x2, y2);
        return ok;
    }
};

// FP32: with t = fma(x, x, cr) = x^2 + Re C, the escape test is
// fma(y, y, t) > lim, lim = fl(4 + cr) (both sides carry Re C), and the update
// x' = fma(-y, y, t), y' = fma(x + x, y, ci): the test shares t with the
// update, 7 vector instructions per tested iteration with the count.
struct ArF32 {
    static constexpr bool kRational = false;
    struct Z { float x, y; };
    struct C { float r, i, lim; };
    using V = float;
    __device__ static V coord(double v) { return (float)v; }  // one rounding
    __device__ static V shfl(V v, int src) { return __shfl(v, src); }
    __device__ static Z make(V x, V y) { return Z{x, y}; }
    __device__ static C cmake(V r, V i) { return C{r, i, 4.0f + r}; }
    __device__ static bool inside(const Z& z, const C& c, int) {
        float t = __builtin_fmaf(z.x, z.x, c.r);
        return __builtin_fmaf(z.y, z.y, t) <= c.lim;
    }
    __device__ static void advance(Z& z, const C& c, float t) {
        float xn = __builtin_fmaf(-z.y, z.y, t);
        float tx = z.x + z.x;
        float yn = __builtin_fmaf(tx, z.y, c.i);
        z.x = xn;
        z.y = yn;
    }
    __device__ static void step(Z& z, const C& c, int) {
        advance(z, c, __builtin_fmaf(z.x, z.x, c.r));
    }
    __device__ static bool check_step(Z& z, const C& c, int) {
        float t = __builtin_fmaf(z.x, z.x, c.r);
        bool ok = __builtin_fmaf(z.y, z.y, t) <= c.lim;
        advance(z, c, t);
        return ok;
    }
};

// Float-float: value = hi + lo.  TwoSum (Knuth), Fast2Sum (Dekker), FMA-based
// TwoProd, and the double-word sum and product of Joldes, Muller and Popescu
// (ACM TOMS 2017): accurate double-word + double-word (error < 3u^2) and
// FMA double-word x double-word (error < 4u^2), u = 2^-24.  The quadratic
// map's iteration uses two cheaper forms: the square (TwoProd of the high
// word plus one fused 2*hi*lo term, the lo*lo term dropped: error < 4u^2)
// and the "sloppy" sum (TwoSum of the high words, the low words added to its
// error, one Fast2Sum: error < 3u^2 of the result for operands of one sign,
// < 3u^2 of |a| + |b| otherwise).  The escape test sums the two squares,
// which are of one sign, so it keeps the relative bound.
struct ArFF {
    static constexpr bool kRational = false;
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
    __device__ static D add_cheap(D a, D b) {
        float s, se;
        two_sum(a.hi, b.hi, s, se);
        float lows = a.lo + b.lo;
        float err = se + lows;
        D r;
        quick_two_sum(s, err, r.hi, r.lo);
        return r;
    }
    __device__ static D sqr(D a) {
        float p = a.hi * a.hi;
        float pe = __builtin_fmaf(a.hi, a.hi, -p);
        float q = __builtin_fmaf(a.hi + a.hi, a.lo, pe);
        D r;
        quick_two_sum(p, q, r.hi, r.lo);
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
    using V = D;
    __device__ static V coord(double v) { return split(v); }
    __device__ static V shfl(V v, int src) { return D{__shfl(v.hi, src), __shfl(v.lo, src)}; }
    __device__ static Z make(V x, V y) { return Z{x, y}; }
    __device__ static C cmake(V r, V i) { return C{r, i}; }
    __device__ static bool le4(D m) { return (m.hi < 4.0f) || (m.hi == 4.0f && m.lo <= 0.0f); }
    __device__ static bool inside(const Z& z, const C&, int) {
        return le4(add_cheap(sqr(z.x), sqr(z.y)));
    }
    __device__ static void advance(Z& z, const C& c, D x2, D y2) {
        D ny2 = D{-y2.hi, -y2.lo};
        D re = add_cheap(x2, ny2);
        D xn = add_cheap(re, c.r);
        D tx = D{z.x.hi + z.x.hi, z.x.lo + z.x.lo};  // 2x, exact
        D im = mul(tx, z.y);
        D yn = add_cheap(im, c.i);
        z.x = xn;
        z.y = yn;
    }
    __device__ static void step(Z& z, const C& c, int) {
        D x2 = sqr(z.x);
        D y2 = sqr(z.y);
        advance(z, c, x2, y2);
    }
    __device__ static bool check_step(Z& z, const C& c, int) {
        D x2 = sqr(z.x);
        D y2 = sqr(z.y);
        bool ok = le4(add_cheap(x2, y2));
        advance(z, c, x2, y2);
        return ok;
    }
};

// General maps Z^d + C (d = 2..8; the paper's further functions).  Z^d comes
// from d - 1 complex products W <- W Z starting at W = Z, each
// (a + ib)(x + iy) taken as (a x - b y) + i (a y + b x) with every operation
// rounded, then C is added.  FP64 and FP32 round each operation in their own
// precision (no fused operations; escape test fl(fl(x x) + fl(y y)) > 4);
// float-float uses the accurate double-word product and sum throughout (its
// escape test too).  The degree is
// the same for every lane of a wave (it is part of the stream variant), so the
// product loop does not diverge.
struct ArF64G : ArF64 {
    __device__ static void power_add(Z& z, const C& c, int d) {
        double wr = z.x, wi = z.y;
#pragma unroll 1
        for (int k = 1; k < d; ++k) {
            double p_rr = wr * z.x;
            double p_ii = wi * z.y;
            double p_ri = wr * z.y;
            double p_ir = wi * z.x;
            double nr = p_rr - p_ii;
            double ni = p_ri + p_ir;
            wr = nr;
            wi = ni;
        }
        z.x = wr + c.r;
        z.y = wi + c.i;
    }
    __device__ static void step(Z& z, const C& c, int d) { power_add(z, c, d); }
    __device__ static bool check_step(Z& z, const C& c, int d) {
        bool ok = inside(z, c, d);
        power_add(z, c, d);
        return ok;
    }
};

struct ArF32G : ArF32 {
    __device__ static bool inside(const Z& z, const C&, int) {
        float x2 = z.x * z.x;
        float y2 = z.y * z.y;
        return x2 + y2 <= 4.0f;
    }
    __device__ static void power_add(Z& z, const C& c, int d) {
        float wr = z.x, wi = z.y;
#pragma unroll 1
        for (int k = 1; k < d; ++k) {
            float p_rr = wr * z.x;
            float p_ii = wi * z.y;
            float p_ri = wr * z.y;
            float p_ir = wi * z.x;
            float nr = p_rr - p_ii;
            float ni = p_ri + p_ir;
            wr = nr;
            wi = ni;
        }
        z.x = wr + c.r;
        z.y = wi + c.i;
    }
    __device__ static void step(Z& z, const C& c, int d) { power_add(z, c, d); }
    __device__ static bool check_step(Z& z, const C& c, int d) {
        bool ok = inside(z, c, d);
        power_add(z, c, d);
        return ok;
    }
};

struct ArFFG : ArFF {
    __device__ static bool inside(const Z& z, const C&, int) {
        return le4(add(mul(z.x, z.x), mul(z.y, z.y)));
    }
    __device__ static void power_add(Z& z, const C& c, int d) {
        D wr = z.x, wi = z.y;
#pragma unroll 1
        for (int k = 1; k < d; ++k) {
            D p_rr = mul(wr, z.x);
            D p_ii = mul(wi, z.y);
            D p_ri = mul(wr, z.y);
            D p_ir = mul(wi, z.x);
            D nr = add(p_rr, D{-p_ii.hi, -p_ii.lo});
            D ni = add(p_ri, p_ir);
            wr = nr;
            wi = ni;
        }
        z.x = add(wr, c.r);
        z.y = add(wi, c.i);
    }
    __device__ static void step(Z& z, const C& c, int d) { power_add(z, c, d); }
    __device__ static bool check_step(Z& z, const C& c, int d) {
        bool ok = inside(z, c, d);
        power_add(z, c, d);
        return ok;
    }
};

// Rational maps with two parameters: Z' = W + C + lambda / W, W = Z^d (d =
// 2..8, formed as for the general maps), lambda / W = (lambda conj W) / |W|^2
// with every product, sum and quotient rounded (IEEE division, no fused
// operations).  A pixel escapes unless |Z|^2 <= 4: the iterate after a hit on
// the pole Z = 0 is 0/0, not a number, and counts as escaped.  Julia images in
// FP64 and FP32; the constant carries lambda beside C.
template <class T>
struct RationalOps {
    __device__ static void map(T& x, T& y, T cr, T ci, T lr, T li, int d) {
        T wr = x, wi = y;
#pragma unroll 1
        for (int k = 1; k < d; ++k) {
            T p_rr = wr * x;
            T p_ii = wi * y;
            T p_ri = wr * y;
            T p_ir = wi * x;
            T nr = p_rr - p_ii;
            T ni = p_ri + p_ir;
            wr = nr;
            wi = ni;
        }
        T q_r = wr * wr;
        T q_i = wi * wi;
        T q = q_r + q_i;
        T a = lr * wr;
        T b = li * wi;
        T e = li * wr;
        T f = lr * wi;
        T num_r = a + b;
        T num_i = e - f;
        T tr = num_r / q;
        T ti = num_i / q;
        T sr = wr + cr;
        T si = wi + ci;
        x = sr + tr;
        y = si + ti;
    }
};

struct ArF64R : ArF64 {
    static constexpr bool kRational = true;
    struct C { double r, i, lr, li; };
    __device__ static C cmake(V r, V i) { return C{r, i, 0.0, 0.0}; }
    __device__ static C cmake_rational(V r, V i, V lr, V li) { return C{r, i, lr, li}; }
    __device__ static bool inside(const Z& z, const C&, int) {
        double x2 = z.x * z.x;
        double y2 = z.y * z.y;
        return x2 + y2 <= 4.0;
    }
    __device__ static void step(Z& z, const C& c, int d) {
        RationalOps<double>::map(z.x, z.y, c.r, c.i, c.lr, c.li, d);
    }
    __device__ static bool check_step(Z& z, const C& c, int d) {
        bool ok = inside(z, c, d);
        step(z, c, d);
        return ok;
    }
};

struct ArF32R : ArF32 {
    static constexpr bool kRational = true;
    struct C { float r, i, lr, li; };
    __device__ static C cmake(V r, V i) { return C{r, i, 0.0f, 0.0f}; }
    __device__ static C cmake_rational(V r, V i, V lr, V li) { return C{r, i, lr, li}; }
    __device__ static bool inside(const Z& z, const C&, int) {
        float x2 = z.x * z.x;
        float y2 = z.y * z.y;
        return x2 + y2 <= 4.0f;
    }
    __device__ static void step(Z& z, const C& c, int d) {
        RationalOps<float>::map(z.x, z.y, c.r, c.i, c.lr, c.li, d);
    }
    __device__ static bool check_step(Z& z, const C& c, int d) {
        bool ok = inside(z, c, d);
        step(z, c, d);
        return ok;
    }
};

// p ? a : b for an iterate, one 32-bit word at a time.  Written on the whole
// struct, the select of a 16-byte iterate (FP64, float-float) became a select
// between two stack slots and a load from per-lane stack memory.
template <class T>
__device__ __forceinline__ T select_words(bool p, const T& a, const T& b) {
    constexpr int W = (int)(sizeof(T) / 4);
    static_assert(sizeof(T) % 4 == 0, "whole words");
    uint32_t wa[W], wb[W];
    __builtin_memcpy(wa, &a, sizeof(T));
    __builtin_memcpy(wb, &b, sizeof(T));
#pragma unroll
    for (int j = 0; j < W; ++j) wa[j] = p ? wa[j] : wb[j];
    T r;
    __builtin_memcpy(&r, wa, sizeof(T));
    return r;
}

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
// Fused colour store: the workgroup copies the colour table into LDS once, and
// a pixel then stores palette[min(count, palette_len - 1)] in place of its
// count.  Only the kernel variants built with COLOR = 1 (launched when a table
// is given) hold this code; every thread of their workgroups reaches the
// barrier.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t* palette_lds() {
    extern __shared__ uint32_t jr_dynamic_lds[];
    return jr_dynamic_lds;
}

template <int COLOR>
__device__ __forceinline__ void stage_palette(const PersistentArgs& a) {
    if (!COLOR) return;
    uint32_t* pal = palette_lds();
    for (int k = threadIdx.x; k < a.palette_len; k += blockDim.x) pal[k] = a.palette[k];
    __syncthreads();
}

// The 32 bits a pixel stores: its count, or (COLOR) its colour.
template <int COLOR, class Args>
__device__ __forceinline__ int32_t shade(const Args& a, int cnt) {
    if (!COLOR) return cnt;
    return (int32_t)palette_lds()[min(cnt, a.palette_len - 1)];
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
            z = A::make(A::coord(0.0), A::coord(0.0));
            c = A::cmake(A::coord(px), A::coord(py));
        } else {
            z = A::make(A::coord(px), A::coord(py));
            c = A::cmake(A::coord(p.cr), A::coord(p.ci));
        }
        constexpr int deg = 2;
        int n = 0;
        while (n < p.max_iter) {
            if (!A::check_step(z, c, deg)) break;
            n++;
        }
        p.out[(int64_t)j * p.W + i] = n;
    }
}

// ---------------------------------------------------------------------------
// Tiled kernel: waves stream pixels from tiles with lane refill.
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

__device__ __forceinline__ unsigned long long* queue_ctr(unsigned long long* ctr, int q) {
    return ctr + (size_t)q * kQueueStride;
}

// Granules in queue q: granules q, q + kQueues, q + 2 kQueues, ...
__device__ __forceinline__ int64_t queue_len(int64_t granules, int q) {
    return granules > q ? (granules - q + kQueues - 1) / kQueues : 0;
}

// Hands out global tile indices to one wave.  Persistent mode: granules of
// tiles from kQueues atomic counters; the wave starts on queue w % kQueues,
// always holds the claim of its next granule in flight, and when its queue is
// empty reads all counters at once (one per lane) and moves to the next queue
// that still has granules.  Dispatch mode: the wave's own tile, once.
struct Claimer {
    unsigned long long raw;  // lane 0: result of the claim in flight
    int64_t cur, end;        // remaining tiles of the current granule
    int64_t qlen;
    int q;
    int wave;
    bool started;
};

__device__ __forceinline__ void claimer_init(Claimer& cl, const PersistentArgs& a) {
    // threadIdx.x / 64 is the same for the whole wave; readfirstlane tells the
    // compiler so, which keeps the claimer and the tile state in SGPRs.
    cl.wave = (int)__builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / 64) +
                                                  (threadIdx.x >> 6));
    cl.cur = cl.end = 0;
    cl.started = false;
    cl.raw = 0;
    cl.q = cl.wave % kQueues;
    cl.qlen = queue_len(a.granules, cl.q);
    if (a.persistent && lane_id() == 0) cl.raw = atomicAdd(queue_ctr(a.ctr, cl.q), 1ull);
}

__device__ __forceinline__ int64_t next_tile(Claimer& cl, const PersistentArgs& a) {
    if (!a.persistent) {
        if (cl.started) return -1;
        cl.started = true;
        return cl.wave < a.total_tiles ? (int64_t)cl.wave : -1;
    }
    if (cl.cur < cl.end) return cl.cur++;
    for (;;) {
        const int64_t j = uniform64((int64_t)cl.raw);
        if (j < cl.qlen) {
            if (lane_id() == 0) cl.raw = atomicAdd(queue_ctr(a.ctr, cl.q), 1ull);
            const int64_t t0 = (j * kQueues + cl.q) * (int64_t)a.granule;
            cl.cur = t0 + 1;
            cl.end = min(t0 + (int64_t)a.granule, a.total_tiles);
            return t0;
        }
        bool has = false;
        if (lane_id() < kQueues) {
            const unsigned long long c = __hip_atomic_load(
                queue_ctr(a.ctr, lane_id()), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            has = (int64_t)c < queue_len(a.granules, lane_id());
        }
        const uint64_t m = __ballot(has);
        if (m == 0) return -1;
        const int s = (cl.q + 1) & (kQueues - 1);
        const uint64_t rot = s ? ((m >> s) | (m << (64 - s))) : m;
        cl.q = (s + __builtin_ctzll(rot)) & (kQueues - 1);
        cl.qlen = queue_len(a.granules, cl.q);
        if (lane_id() == 0) cl.raw = atomicAdd(queue_ctr(a.ctr, cl.q), 1ull);
    }
}

// The frame table is read-only during a launch.  Reading it through the
// constant address space lets the compiler use scalar loads (the table index
// is wave-uniform), which it cannot prove safe through a generic pointer that
// might alias the output.
typedef const __attribute__((address_space(4))) DevFrame CFrame;
typedef const __attribute__((address_space(4))) char CByte;

// Progress of a launch (rows and plain kernels).  A wave reads the stop flag
// before it claims a tile; the host may write the flag while the kernel runs
// (pinned host memory or device memory), so the load is a system-scope
// atomic, and the wave acts on lane 0's value.
__device__ __forceinline__ bool stop_requested(const int32_t* stop) {
    if (stop == nullptr) return false;
    const int v = __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return __builtin_amdgcn_readfirstlane(v) != 0;
}

// Adds `pixels` to a frame's counter once the wave's stores are done (the
// release fence orders them first: a reader that sees the count sees the
// pixels); one active lane adds.
__device__ __forceinline__ void add_done(int32_t* slot, int pixels) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint64_t active = __ballot(true);
    if (lane_id() == __builtin_ctzll(active))
        __hip_atomic_fetch_add(slot, pixels, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A frame's constant in the arithmetic A (C, and lambda for the rational maps).
template <class A>
__device__ __forceinline__ typename A::C frame_c(CFrame& F) {
    if constexpr (A::kRational)
        return A::cmake_rational(A::coord(F.cr), A::coord(F.ci), A::coord(F.lr),
                                 A::coord(F.li));
    else
        return A::cmake(A::coord(F.cr), A::coord(F.ci));
}

// The frame table of a launch: the device table, or for a one-frame launch
// the copy inside the kernel arguments (the single by-value PersistentArgs
// argument sits at offset 0 of the kernel-argument segment), which saves the
// host a table upload per image.
__device__ __forceinline__ CFrame* cframes(const PersistentArgs& a) {
    if (a.frames) return (CFrame*)a.frames;
    CByte* k = (CByte*)__builtin_amdgcn_kernarg_segment_ptr();
    return (CFrame*)(k + offsetof(PersistentArgs, frame0));
}

// Largest frame index f with frames[f].tile_begin <= t.  A short forward scan
// from the previous frame usually ends it; otherwise binary search.
__device__ __forceinline__ int find_frame(CFrame* frames, int nframes, int64_t t, int f) {
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

// The tile that lanes currently refill from (wave-uniform).  Kept small: it
// lives in scalar registers for the whole stream.
struct Src {
    int64_t t;          // global tile index, -1: none left
    int f;              // its frame
    int variant;        // stream variant the tile needs (variant_of)
    int32_t* out;       // count of the tile's pixel (0, 0)
    int W, max_iter, mode;
    int tw, npix, next;
    uint32_t magic;     // k / tw == (k * magic) >> 18 for k < 4096, tw <= 64
};

// Which stream variant a frame needs: its dtype, and whether the blocked test
// may be used (escape absorbing, |C| <= 1.9) or every iteration is tested.
__device__ __forceinline__ int variant_of(int dtype, int absorbing, int degree) {
    return ((degree - 2) * 3 + dtype) * 2 + (absorbing ? 1 : 0);
}

// The map's degree of a stream variant.
__device__ __forceinline__ int degree_of(int variant) { return variant / 6 + 2; }

// Makes tile t the refill source.  Lane L receives the binary64 coordinate of
// the tile's column L (xd) and row L (yd), and every lane the frame's C.
__device__ __forceinline__ void load_src(Src& s, const PersistentArgs& a, int64_t t,
                                         double& xd, double& yd, double& cr, double& ci) {
    s.t = t;
    if (t < 0) return;
    CFrame* frames = cframes(a);
    s.f = find_frame(frames, a.nframes, t, s.f);
    CFrame& F = frames[s.f];
    const uint32_t local = (uint32_t)(t - F.tile_begin);  // < 2^31 tiles per frame
    const int ty = (int)(local / (uint32_t)F.tiles_x);
    const int tx = (int)(local - (uint32_t)ty * (uint32_t)F.tiles_x);
    const int col0 = tx * F.tile_w;
    const int row0 = F.row_begin + ty * F.tile_h;
    const int th = min(F.tile_h, F.row_end - row0);
    s.variant = variant_of(F.dtype, F.defer, F.degree);
    s.W = F.width;
    s.max_iter = F.max_iter;
    s.mode = F.mode;
    s.tw = min(F.tile_w, F.width - col0);
    s.npix = s.tw * th;
    s.next = 0;
    s.magic = ((1u << 18) + (uint32_t)s.tw - 1u) / (uint32_t)s.tw;
    s.out = a.out_base + F.out_offset + ((int64_t)row0 * F.width + col0);
    const int lane = lane_id();
    xd = pixel_re(F.cx, F.hx, col0 + min(lane, s.tw - 1), F.width);
    yd = pixel_im(F.cy, F.hy, row0 + min(lane, th - 1), F.height);
    cr = F.cr;
    ci = F.ci;
}

// Streams pixels through one wave while the tiles handed out need this
// variant (A, absorbing or not).  Lane state: z (iterate), zs (iterate at the
// start of a deferred block), n (iterations done), mi (cap of the pixel's
// frame), outp (where its count goes), and three flags:
//   it  the lane iterates an unfinished pixel,
//   pe  (DEFER) it escaped inside the last block; the count needs a replay,
//   fi  its final count is in cnt and not yet stored.
// Blocks of K iterations run on every lane without branches (a lane that is
// not iterating computes values nobody reads), and the bookkeeping after a
// block is selects, so a block costs vector instructions and few scalar ones.
//   DEFER = 0: every iterate is tested and the leading non-escaped iterates
//     are counted (lead += |Z|^2 <= 4).  Escape being absorbing, the first
//     escaped iterate is n + lead.  With K = 1 this is the exact test on every
//     iteration and needs no absorbing property.
//   DEFER = 1: the K steps run untested and only the last iterate is tested;
//     lanes found escaped replay the block from zs with the counted test.
// A refill round runs when at least `refill` lanes are not iterating (or no
// lane is): replays are resolved, finished lanes store, and free lanes take
// the next pixels of the tile, and of the following tiles when it runs out.
// Returns when the next tile needs another variant (left in s, its coordinate
// tables in xd, yd and its constant in crd, cid) or none is left.
template <class A, int K, int DEFER, int COLOR>
__device__ void run_stream(Src& s, Claimer& cl, const PersistentArgs& a, double& xd, double& yd,
                           double& crd, double& cid) {
    using V = typename A::V;
    const int my_variant = s.variant;
    const int deg = degree_of(my_variant);
    const V zero = A::coord(0.0);
    V xcol = A::coord(xd), yrow = A::coord(yd);
    V cre = A::coord(crd), cim = A::coord(cid);
    bool src_ok = true;
    bool it = false, pe = false, fi = false;
    int n = 0, cnt = 0, mi = 0;
    int32_t* outp = s.out;
    typename A::Z z = A::make(zero, zero);
    typename A::Z zs = z;
    typename A::C c = A::cmake(zero, zero);
    uint64_t running = 0;  // wave-uniform: ballot(it)

    // refill <= 64, so a wave with no running lane always takes this branch
    const int busy_max = 64 - a.refill;
    for (;;) {
        if (__popcll(running) <= busy_max) {
            if (DEFER && __ballot(pe) != 0) {
                // replay the last block from its start, on every lane
                typename A::Z zr = zs;
                int lead = 0;
#pragma unroll
                for (int u = 0; u < K; ++u) lead += A::check_step(zr, c, deg) ? 1 : 0;
                if (pe) {
                    cnt = min(n + lead, mi);
                    fi = true;
                    pe = false;
                }
            }
            if (fi) {
                *outp = shade<COLOR>(a, cnt);
                fi = false;
            }
            uint64_t idle = ~running;
            while (idle != 0 && src_ok) {
                const int k = s.next + lanes_below(idle);
                const int kk = min(k, s.npix - 1);
                const int row = (int)(((uint32_t)kk * s.magic) >> 18);
                const int col = kk - row * s.tw;
                const V x0 = A::shfl(xcol, col);
                const V y0 = A::shfl(yrow, row);
                if (!it && k < s.npix) {
                    if (s.mode == kModeMandelbrot) {
                        z = A::make(zero, zero);
                        c = A::cmake(x0, y0);
                    } else {
                        z = A::make(x0, y0);
                        c = A::cmake(cre, cim);
                    }
                    n = 0;
                    mi = s.max_iter;
                    outp = s.out + (row * s.W + col);
                    it = true;
                }
                s.next += __popcll(idle);
                if (s.next >= s.npix) {
                    load_src(s, a, next_tile(cl, a), xd, yd, crd, cid);
                    if (s.t < 0 || s.variant != my_variant) {
                        src_ok = false;
                    } else {
                        xcol = A::coord(xd);
                        yrow = A::coord(yd);
                        cre = A::coord(crd);
                        cim = A::coord(cid);
                    }
                }
                idle = ~__ballot(it);
            }
            running = __ballot(it);
            if (running == 0) return;
        }
        if (DEFER) {
            zs = select_words(pe, zs, z);  // a lane waiting for its replay keeps its block start
#pragma unroll
            for (int u = 0; u < K; ++u) A::step(z, c, deg);
            const bool esc = !A::inside(z, c, deg);
            const bool capped = n + K >= mi;  // no escape up to n + K >= cap: absorbing
            cnt = (it && !esc && capped) ? mi : cnt;
            fi = fi || (it && !esc && capped);
            pe = pe || (it && esc);
            it = it && !esc && !capped;
            n += K;
            n -= (pe && !it) ? K : 0;  // a lane to replay keeps n at the block start
        } else {
            int lead = 0;
#pragma unroll
            for (int u = 0; u < K; ++u) lead += A::check_step(z, c, deg) ? 1 : 0;
            const bool stop = (lead < K) || (n + K >= mi);
            const int final_cnt = min(n + lead, mi);
            cnt = (it && stop) ? final_cnt : cnt;
            fi = fi || (it && stop);
            it = it && !stop;
            n += K;
        }
        running = __ballot(it);
    }
}

// ---------------------------------------------------------------------------
// Hybrid stream: fresh pixels run like the plain kernel, survivors refill.
// ---------------------------------------------------------------------------
// A wave takes 64 fresh pixels at a time (a packet) and iterates them with
// the exact per-iteration test; the packet ends as soon as every lane has
// escaped or hit its cap, or after `bail` iterations.  Pixels still running
// then (the survivors, typically a small minority) are parked in a per-wave
// queue in LDS.  When a packet's survivors no longer fit, the wave drains the
// queue with the refill stream (blocks of K, lanes refilled from the queue);
// once the queue is empty and few lanes are still running, those are parked
// and fresh packets resume.  Fresh pixels so pay no block overshoot, and the
// long orbits still keep every lane busy.
constexpr int kQ = 64;            // queue slots per wave
constexpr int kQWordsMax = 12;    // 32-bit words of one parked lane, at most

template <class A>
struct Parked {
    typename A::Z z;
    typename A::C c;
    int n, mi;
    int32_t* outp;
};

template <class A>
__device__ __forceinline__ void park(uint32_t* q, int slot, const Parked<A>& p) {
    constexpr int W = (int)(sizeof(Parked<A>) / 4);
    static_assert(W <= kQWordsMax, "parked lane too large");
    uint32_t w[W];
    __builtin_memcpy(w, &p, sizeof(Parked<A>));
#pragma unroll
    for (int j = 0; j < W; ++j) q[j * kQ + slot] = w[j];
}

template <class A>
__device__ __forceinline__ Parked<A> unpark(const uint32_t* q, int slot) {
    constexpr int W = (int)(sizeof(Parked<A>) / 4);
    uint32_t w[W];
#pragma unroll
    for (int j = 0; j < W; ++j) w[j] = q[j * kQ + slot];
    Parked<A> p;
    __builtin_memcpy(&p, w, sizeof(Parked<A>));
    return p;
}

template <class A, int K, int DEFER, int COLOR>
__device__ void run_hybrid(Src& s, Claimer& cl, const PersistentArgs& a, double& xd, double& yd,
                           double& crd, double& cid, uint32_t* q) {
    using V = typename A::V;
    const int my_variant = s.variant;
    const int deg = degree_of(my_variant);
    const V zero = A::coord(0.0);
    V xcol = A::coord(xd), yrow = A::coord(yd);
    V cre = A::coord(crd), cim = A::coord(cid);
    bool src_ok = true;
    bool it = false, pe = false, fi = false;
    int n = 0, cnt = 0, mi = 0;
    int32_t* outp = s.out;
    typename A::Z z = A::make(zero, zero);
    typename A::Z zs = z;
    typename A::C c = A::cmake(zero, zero);
    int qn = 0;  // wave-uniform: lanes parked in q
    const int busy_max = 64 - a.refill;

    for (;;) {
        // ------------------------------------------------ fresh packet
        if (src_ok) {
            uint64_t idle = ~__ballot(it);  // all lanes: nothing runs here
            while (idle != 0 && src_ok) {
                const int k = s.next + lanes_below(idle);
                const int kk = min(k, s.npix - 1);
                const int row = (int)(((uint32_t)kk * s.magic) >> 18);
                const int col = kk - row * s.tw;
                const V x0 = A::shfl(xcol, col);
                const V y0 = A::shfl(yrow, row);
                if (!it && k < s.npix) {
                    if (s.mode == kModeMandelbrot) {
                        z = A::make(zero, zero);
                        c = A::cmake(x0, y0);
                    } else {
                        z = A::make(x0, y0);
                        c = A::cmake(cre, cim);
                    }
                    n = 0;
                    mi = s.max_iter;
                    outp = s.out + (row * s.W + col);
                    it = true;
                }
                s.next += __popcll(idle);
                if (s.next >= s.npix) {
                    load_src(s, a, next_tile(cl, a), xd, yd, crd, cid);
                    if (s.t < 0 || s.variant != my_variant) {
                        src_ok = false;
                    } else {
                        xcol = A::coord(xd);
                        yrow = A::coord(yd);
                        cre = A::coord(crd);
                        cim = A::coord(cid);
                    }
                }
                idle = ~__ballot(it);
            }
            // the exact test on every iteration, until every lane is done
            for (int u = 0; u < a.bail; ++u) {
                const bool ok = A::check_step(z, c, deg);
                const bool stop = it && (!ok || n >= mi);
                cnt = stop ? n : cnt;
                fi = fi || stop;
                it = it && !stop;
                n += it ? 1 : 0;
                if (__ballot(it) == 0) break;
            }
            if (fi) {
                *outp = shade<COLOR>(a, cnt);
                fi = false;
            }
            const uint64_t surv = __ballot(it);
            const int ns = __popcll(surv);
            if (qn + ns <= kQ && (src_ok || ns == 0)) {
                if (it) {
                    Parked<A> p{z, c, n, mi, outp};
                    park<A>(q, qn + lanes_below(surv), p);
                    it = false;
                }
                qn += ns;
                if (src_ok) continue;
            }
            // survivors do not fit (or the source is done): drain below
        }
        // ------------------------------------------------ drain the queue
        uint64_t running = __ballot(it);
        for (;;) {
            if (__popcll(running) <= busy_max) {
                if (DEFER && __ballot(pe) != 0) {
                    typename A::Z zr = zs;
                    int lead = 0;
#pragma unroll
                    for (int u = 0; u < K; ++u) lead += A::check_step(zr, c, deg) ? 1 : 0;
                    if (pe) {
                        cnt = min(n + lead, mi);
                        fi = true;
                        pe = false;
                    }
                }
                if (fi) {
                    *outp = shade<COLOR>(a, cnt);
                    fi = false;
                }
                const uint64_t idle = ~__ballot(it);
                const int take = min(qn, __popcll(idle));
                if (take > 0) {
                    const int r = lanes_below(idle);
                    if (!it && r < take) {
                        const Parked<A> p = unpark<A>(q, qn - 1 - r);
                        z = p.z;
                        c = p.c;
                        n = p.n;
                        mi = p.mi;
                        outp = p.outp;
                        it = true;
                    }
                    qn -= take;
                }
                running = __ballot(it);
                if (qn == 0) {
                    if (src_ok && __popcll(running) <= busy_max) {
                        // park the few lanes still running and go back to fresh packets
                        if (it) {
                            Parked<A> p{z, c, n, mi, outp};
                            park<A>(q, lanes_below(running), p);
                            it = false;
                        }
                        qn = __popcll(running);
                        break;
                    }
                    if (!src_ok && running == 0) return;
                }
            }
            if (DEFER) {
                zs = select_words(pe, zs, z);
#pragma unroll
                for (int u = 0; u < K; ++u) A::step(z, c, deg);
                const bool esc = !A::inside(z, c, deg);
                const bool capped = n + K >= mi;
                cnt = (it && !esc && capped) ? mi : cnt;
                fi = fi || (it && !esc && capped);
                pe = pe || (it && esc);
                it = it && !esc && !capped;
                n += K;
                n -= (pe && !it) ? K : 0;
            } else {
                int lead = 0;
#pragma unroll
                for (int u = 0; u < K; ++u) lead += A::check_step(z, c, deg) ? 1 : 0;
                const bool stop = (lead < K) || (n + K >= mi);
                const int final_cnt = min(n + lead, mi);
                cnt = (it && stop) ? final_cnt : cnt;
                fi = fi || (it && stop);
                it = it && !stop;
                n += K;
            }
            running = __ballot(it);
        }
    }
}

// Persistent (or one-wave-per-tile) kernel over a table of frames: 256-thread
// workgroups of 4 independent waves.  Each wave takes tiles from its Claimer
// and hands them to the stream of the variant they need.
template <int K, int DEFER, int DTMASK, int HYB>
__global__ __launch_bounds__(256) void jr_tiled(PersistentArgs a) {
    constexpr int COLOR = (DTMASK & kColorBit) ? 1 : 0;
    constexpr bool GENERAL = (DTMASK & kGeneralBit) != 0;
    // per-wave survivor queues of the hybrid stream (unused otherwise)
    __shared__ uint32_t qmem[HYB ? 4 * kQWordsMax * kQ : 1];
    uint32_t* q = qmem + (HYB ? (threadIdx.x >> 6) * kQWordsMax * kQ : 0);
    stage_palette<COLOR>(a);
    Claimer cl;
    claimer_init(cl, a);
    Src s;
    s.f = 0;
    double xd, yd, cr, ci;
    load_src(s, a, next_tile(cl, a), xd, yd, cr, ci);
#define JR_STREAM(A_, K_, D_)                                         \
    do {                                                              \
        if (HYB)                                                      \
            run_hybrid<A_, K_, D_, COLOR>(s, cl, a, xd, yd, cr, ci, q); \
        else                                                          \
            run_stream<A_, K_, D_, COLOR>(s, cl, a, xd, yd, cr, ci); \
    } while (0)
    while (s.t >= 0) {
        const int v = s.variant % 6;  // dtype * 2 + absorbing
        const bool general = s.variant >= 6;
        if (GENERAL && general) {
            if (v == kFP32 * 2 + 1)
                JR_STREAM(ArF32G, K, DEFER);
            else if (v == kFP32 * 2)
                JR_STREAM(ArF32G, 1, 0);
            else if (v == kFP64 * 2 + 1)
                JR_STREAM(ArF64G, K, DEFER);
            else if (v == kFP64 * 2)
                JR_STREAM(ArF64G, 1, 0);
            else if (v == kFF * 2 + 1)
                JR_STREAM(ArFFG, K, DEFER);
            else
                JR_STREAM(ArFFG, 1, 0);
        } else if ((DTMASK & (1 << kFP32)) && v == kFP32 * 2 + 1)
            JR_STREAM(ArF32, K, DEFER);
        else if ((DTMASK & (1 << kFP32)) && v == kFP32 * 2)
            JR_STREAM(ArF32, 1, 0);
        else if ((DTMASK & (1 << kFP64)) && v == kFP64 * 2 + 1)
            JR_STREAM(ArF64, K, DEFER);
        else if ((DTMASK & (1 << kFP64)) && v == kFP64 * 2)
            JR_STREAM(ArF64, 1, 0);
        else if ((DTMASK & (1 << kFF)) && v == kFF * 2 + 1)
            JR_STREAM(ArFF, K, DEFER);
        else if ((DTMASK & (1 << kFF)) && v == kFF * 2)
            JR_STREAM(ArFF, 1, 0);
        else
            load_src(s, a, next_tile(cl, a), xd, yd, cr, ci);  // not reached
    }
#undef JR_STREAM
}

// One thread per pixel over a table of frames: workgroup b covers tile b
// (16 x 16 pixels) of the frame that holds it, and every thread runs the
// per-iteration test like jr_plain.  The batched form of the comparator,
// and a candidate of the autotuner for images whose counts are low and even.
template <class A, int COLOR>
__device__ __forceinline__ void plain_pixel(const PersistentArgs& a, CFrame& F, int i, int j,
                                            int32_t* out) {
    const int deg = F.degree;
    const double px = pixel_re(F.cx, F.hx, i, F.width);
    const double py = pixel_im(F.cy, F.hy, j, F.height);
    typename A::Z z;
    typename A::C c;
    if (F.mode == kModeMandelbrot) {
        z = A::make(A::coord(0.0), A::coord(0.0));
        c = A::cmake(A::coord(px), A::coord(py));
    } else {
        z = A::make(A::coord(px), A::coord(py));
        c = frame_c<A>(F);
    }
    int n = 0;
    while (n < F.max_iter) {
        if (!A::check_step(z, c, deg)) break;
        n++;
    }
    out[(int64_t)j * F.width + i] = shade<COLOR>(a, n);
}

template <int DTMASK>
__global__ __launch_bounds__(256) void jr_plain_batch(PersistentArgs a) {
    constexpr int COLOR = (DTMASK & kColorBit) ? 1 : 0;
    stage_palette<COLOR>(a);
    CFrame* frames = cframes(a);
    const int64_t t = blockIdx.x;
    int f = 0;
    if (a.nframes > 1) {
        // frames of equal size are common: start from the proportional guess
        int guess = (int)((double)t * (double)a.nframes / (double)a.total_tiles);
        guess = min(max(guess, 0), a.nframes - 1);
        f = find_frame(frames, a.nframes, t, frames[guess].tile_begin <= t ? guess : 0);
    }
    CFrame& F = frames[f];
    constexpr bool kProgress = (DTMASK & kProgressBit) != 0;
    if (kProgress && stop_requested(a.stop)) return;
    const uint32_t local = (uint32_t)(t - F.tile_begin);
    const int ty = (int)(local / (uint32_t)F.tiles_x);
    const int tx = (int)(local - (uint32_t)ty * (uint32_t)F.tiles_x);
    const int i = tx * F.tile_w + (int)(threadIdx.x & 15);
    const int j = F.row_begin + ty * F.tile_h + (int)(threadIdx.x >> 4);
    if (i >= F.width || j >= F.row_end) return;
    int32_t* out = a.out_base + F.out_offset;
    if ((DTMASK & kRationalBit) && F.map == kMapRational) {
        if (F.dtype == kFP32)
            plain_pixel<ArF32R, COLOR>(a, F, i, j, out);
        else
            plain_pixel<ArF64R, COLOR>(a, F, i, j, out);
    } else if ((DTMASK & kGeneralBit) && F.degree > 2) {
        if (F.dtype == kFP32)
            plain_pixel<ArF32G, COLOR>(a, F, i, j, out);
        else if (F.dtype == kFP64)
            plain_pixel<ArF64G, COLOR>(a, F, i, j, out);
        else
            plain_pixel<ArFFG, COLOR>(a, F, i, j, out);
    } else if ((DTMASK & (1 << kFP32)) && F.dtype == kFP32)
        plain_pixel<ArF32, COLOR>(a, F, i, j, out);
    else if ((DTMASK & (1 << kFP64)) && F.dtype == kFP64)
        plain_pixel<ArF64, COLOR>(a, F, i, j, out);
    else if ((DTMASK & (1 << kFF)) && F.dtype == kFF)
        plain_pixel<ArFF, COLOR>(a, F, i, j, out);
    // each wave counts its own stored pixels (its lanes inside the frame)
    if (kProgress && a.done) add_done(a.done + F.index, __popcll(__ballot(true)));
}

// ---------------------------------------------------------------------------
// Row-packet kernel (two phases per tile).
// ---------------------------------------------------------------------------
// Most pixels of a light image escape within a few iterations, and in the
// refill stream each of them still costs a block of K iterations and a share of
// a refill round.  Here a wave takes its tile (at most 64 x 64, lane L =
// column L) a group of rows at a time:
//   phase 1  every lane runs its pixel of each row of the group for up to P
//            counted iterations, in branch-free trips of four; the row's
//            coordinate is one value for the whole wave and the column's is
//            the lane's own, so nothing is exchanged between lanes.  Pixels
//            that escape (or reach the cap) store their count at once, one
//            coalesced store per row;
//   survivors append their iterate, their position and the number of
//            iterations run to the wave's list in LDS (stored one array per
//            word, so lanes hit distinct banks);
//   phase 2  whenever the list could not take the next group's survivors,
//            and at the end of the tile, the wave drains it with the refill
//            stream in counted blocks of K: idle lanes read the next entries
//            straight from the list, and C is the frame's constant.  A drain
//            usually holds several wave-loads of survivors, so the lanes left
//            idle while its last orbits finish cost little.
// Counts: a group that ran `done` iterations counts, per pixel, the leading
// non-escaped iterates of Z_0..Z_{done-1}; with escape absorbing (|C| <= 1.9)
// that is min(count, done), so a pixel with fewer than `done` is final and the
// others continue from Z_done with n = done.  A group stops before P once all
// its pixels have escaped (the iterates it skips would count nothing), or
// once at most the schedule's handoff of them are still inside.  Frames where
// escape may not be absorbing run P = 1 and K = 1, the exact test on every
// iteration.
template <int DTMASK>
struct RowsShape {
    static constexpr int kMask = DTMASK & 7;
    static constexpr int rows = kMask == (1 << kFP32) ? kRowsFP32 : kRowsWide;
    // 32-bit words of the widest iterate among the dtypes of the kernel
    static constexpr int zwords = (kMask & ((1 << kFP64) | (1 << kFF))) ? 4 : 2;
    // one wave's list in 32-bit words: the iterates, then 16-bit positions
    static constexpr int wave_words = zwords * 64 * rows + 32 * rows;
};

template <class A>
__device__ __forceinline__ typename A::V bcast(typename A::V v, int lane) {
    constexpr int W = (int)(sizeof(typename A::V) / 4);
    uint32_t w[W];
    __builtin_memcpy(w, &v, sizeof(v));
#pragma unroll
    for (int j = 0; j < W; ++j) w[j] = __builtin_amdgcn_readlane(w[j], lane);
    typename A::V r;
    __builtin_memcpy(&r, w, sizeof(r));
    return r;
}

// base[off] = v for a wave-uniform base and a per-lane offset 0 <= off < 2^30:
// an unsigned 32-bit byte offset lets the store take the base from scalar
// registers (no 64-bit address arithmetic per lane).
__device__ __forceinline__ void store_at(int32_t* base, int off, int32_t v) {
    *(int32_t*)((char*)base + (uint32_t)off * 4u) = v;
}

template <class A>
__device__ __forceinline__ void list_put(uint32_t* list, int cap, int e, const typename A::Z& z) {
    constexpr int W = (int)(sizeof(typename A::Z) / 4);
    uint32_t w[W];
    __builtin_memcpy(w, &z, sizeof(z));
#pragma unroll
    for (int j = 0; j < W; ++j) list[j * cap + e] = w[j];
}

template <class A>
__device__ __forceinline__ typename A::Z list_get(const uint32_t* list, int cap, int e) {
    constexpr int W = (int)(sizeof(typename A::Z) / 4);
    uint32_t w[W];
#pragma unroll
    for (int j = 0; j < W; ++j) w[j] = list[j * cap + e];
    typename A::Z z;
    __builtin_memcpy(&z, w, sizeof(z));
    return z;
}

// One tile: phase 1 over its rows, then phase 2 over the survivors.  `list`
// holds `cap` entries; word W of entry e's iterate is list[W * cap + e], and
// its position (row << 6 | column) is the 16-bit element e of the array that
// follows the iterate words.
// The kernel's arguments read in place, in the kernel-argument segment (the
// single by-value PersistentArgs argument sits at offset 0).  A function that
// is not inlined and takes the by-value argument by reference gets a copy of
// it in per-lane stack memory; through this reference it reads the arguments
// with scalar loads instead.  The general and rational maps' tiles, which
// are not inlined, take this; the quadratic maps' tiles are inlined and take
// the by-value argument, which keeps the hot loop's registers as they were
// (the kernel-argument reference there cost 16 more vector registers and
// about 10% of the parameter path's time).
typedef const __attribute__((address_space(4))) PersistentArgs CArgs;
__device__ __forceinline__ CArgs& kernel_args() {
    return *(CArgs*)__builtin_amdgcn_kernarg_segment_ptr();
}

template <class A, int K, int MANDEL, int COLOR, int LROWS, int DD, class Args>
__device__ void rows_tile(const Args& a, CFrame& F, int64_t t, int P, uint32_t* list,
                          int32_t* done_at) {
    constexpr int cap = 64 * LROWS;  // list entries
    // deferred drain blocks need escape to be absorbing (K > 1 means it is)
    constexpr bool kDeferDrain = DD != 0 && K > 1;
    using V = typename A::V;
    constexpr int ZW = (int)(sizeof(typename A::Z) / 4);
    const uint32_t local = (uint32_t)(t - F.tile_begin);
    const int ty = (int)(local / (uint32_t)F.tiles_x);
    const int tx = (int)(local - (uint32_t)ty * (uint32_t)F.tiles_x);
    const int col0 = tx * F.tile_w;
    const int row0 = F.row_begin + ty * F.tile_h;
    const int tw = min(F.tile_w, F.width - col0);
    const int th = min(F.tile_h, F.row_end - row0);  // at most 64 (one row per lane of yl)
    const int W = __builtin_amdgcn_readfirstlane(F.width);
    const int mi = __builtin_amdgcn_readfirstlane(F.max_iter);
    const int deg = __builtin_amdgcn_readfirstlane(F.degree);
    const int lane = lane_id();
    const V zero = A::coord(0.0);
    const V xl = A::coord(pixel_re(F.cx, F.hx, col0 + min(lane, tw - 1), W));
    const V yl = A::coord(pixel_im(F.cy, F.hy, row0 + min(lane, th - 1), F.height));
    const typename A::C cj = frame_c<A>(F);
    int32_t* tout = a.out_base + F.out_offset + ((int64_t)row0 * W + col0);
    const bool col_ok = lane < tw;
    const uint64_t cols = tw >= 64 ? ~0ull : ((1ull << tw) - 1ull);  // lanes inside the tile
    uint16_t* pos = (uint16_t*)(list + ZW * cap);

    // phase 1
    int qn = 0;
    auto start_row = [&](int r, typename A::Z& z, typename A::C& c) {
        const V y = bcast<A>(yl, r);
        if (MANDEL) {
            z = A::make(zero, zero);
            c = A::cmake(xl, y);
        } else {
            z = A::make(xl, y);
            c = cj;
        }
    };
    // A pixel survives when it is inside for all `done` iterates its group
    // ran (lead = done) and the cap lies beyond them; one compare against the
    // lane's bound gives the survivors' mask directly.  Finished pixels store,
    // survivors append.  An entry's position word holds the row and column
    // in the tile and, in its top four bits, done / 4 - 1 (done is a multiple
    // of 4 from 4 to 64 where K > 1; where K = 1 it is P = 1 and the bits are
    // unused).
    auto finish_row = [&](int r, int lead, const typename A::Z& z, int done) {
        const int p_lane = (col_ok && done < mi) ? done : 0x7fffffff;
        const bool sv = lead >= p_lane;
        const bool fin = col_ok && !sv;
        const uint64_t m = __ballot(sv);
        if (fin) store_at(tout + (int64_t)r * W, lane, shade<COLOR>(a, min(lead, mi)));
        if (sv) {
            const int e = qn + lanes_below(m);
            list_put<A>(list, cap, e, z);
            const int k = K == 1 ? 0 : (done >> 2) - 1;
            pos[e] = (uint16_t)((k << 12) | (r << 6) | lane);
        }
        qn += __popcll(m);
    };
    // Phase 2: the refill stream over the list's entries, in blocks of K;
    // idle lanes read the next entries straight from the list, and C is the
    // frame's constant.  It runs whenever the list could not take the next
    // group's survivors, and at the end of the tile, so a drain usually holds
    // several wave-loads of survivors and its tail stays short.  Counted
    // blocks test every iterate; deferred blocks (kDeferDrain) run K untested
    // steps and test the last iterate only.  A lane found escaped then keeps
    // its block start and its count before the block, and the next refill
    // round replays that block for it with the counted test, once for all
    // such lanes.  The survivors are long orbits, most of them running to the
    // cap, so most blocks need no replay.
    auto drain = [&]() {
        if (qn == 0) return;
        // Other lanes read the entries written above, and the next rows
        // overwrite them afterwards: keep the compiler from moving LDS
        // accesses across either point (one wave runs them in order).
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        bool it = false, fi = false, pe = false;
        int n = 0, cnt = 0, off = 0;
        typename A::Z z = A::make(zero, zero);
        typename A::Z zs = z;
        typename A::C c = cj;
        int next = 0;
        uint64_t running = 0;
        const int busy_max = 64 - a.refill;
        for (;;) {
            if (__popcll(running) <= busy_max) {
                if (kDeferDrain && __ballot(pe) != 0) {
                    // replay, counted, the block in which these lanes escaped
                    typename A::Z zr = zs;
                    int lead = 0;
#pragma unroll
                    for (int u = 0; u < K; ++u) lead += A::check_step(zr, c, deg) ? 1 : 0;
                    if (pe) {
                        cnt = min(n + lead, mi);
                        fi = true;
                        pe = false;
                    }
                }
                if (fi) {
                    // r * W + col fits an int (a frame holds < 2^31 pixels),
                    // but four times it may not fit 32 bits: index, so that
                    // the address is formed in 64 bits.
                    tout[off] = shade<COLOR>(a, cnt);
                    fi = false;
                }
                if (next < qn) {
                    const uint64_t idle = ~running;
                    const int e = next + lanes_below(idle);
                    const int ee = min(e, qn - 1);
                    const typename A::Z zl = list_get<A>(list, cap, ee);
                    const uint32_t id = pos[ee];
                    const int r = (int)((id >> 6) & 63u);
                    const int col = (int)(id & 63u);
                    const int done = K == 1 ? P : (int)((id >> 12) + 1u) * 4;
                    V cx = zero, cy = zero;
                    if (MANDEL) {
                        cx = A::shfl(xl, col);
                        cy = A::shfl(yl, r);
                    }
                    if (!it && e < qn) {
                        z = zl;
                        if (MANDEL) c = A::cmake(cx, cy);
                        off = r * W + col;
                        n = done;
                        it = true;
                    }
                    next += __popcll(idle);
                }
                running = __ballot(it);
                if (running == 0) break;
            }
            if (kDeferDrain) {
                zs = select_words(pe, zs, z);  // a lane awaiting its replay keeps its block start
#pragma unroll
                for (int u = 0; u < K; ++u) A::step(z, c, deg);
                const bool esc = !A::inside(z, c, deg);
                const bool capped = n + K >= mi;  // no escape in the block: count the cap
                cnt = (it && !esc && capped) ? mi : cnt;
                fi = fi || (it && !esc && capped);
                pe = pe || (it && esc);
                n = (it && !esc) ? n + K : n;
                it = it && !esc && !capped;
            } else {
                // Escape is absorbing (or K = 1): a running lane escapes in
                // this block exactly when its last test fails, and its count
                // is then n plus the tests it passed; a block in which no
                // running lane escapes spends no instruction on counts.
                bool in[K];
#pragma unroll
                for (int u = 0; u < K; ++u) in[u] = A::check_step(z, c, deg);
                const bool esc = it && !in[K - 1];
                const bool capped = n + K >= mi;
                if (__ballot(esc) != 0) {
                    int lead = 0;
#pragma unroll
                    for (int u = 0; u < K - 1; ++u) lead += in[u] ? 1 : 0;
                    cnt = esc ? min(n + lead, mi) : cnt;
                }
                cnt = (it && !esc && capped) ? mi : cnt;  // inside through the cap
                fi = fi || esc || (it && capped);
                it = it && !esc && !capped;
                n += K;
            }
            running = __ballot(it);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        qn = 0;
    };
    int r = 0;
    // Row groups for the quadratic FP32 and FP64 maps; float-float and the
    // general maps hold too much state per orbit (registers would cost
    // resident waves).  FP32 takes four rows at a time where its list holds
    // eight rows' survivors (FP32-only kernels), two otherwise, as FP64
    // does: a drain should find several groups' survivors waiting.
    constexpr bool kGroups = std::is_same<A, ArF32>::value || std::is_same<A, ArF64>::value;
    constexpr int G = (std::is_same<A, ArF32>::value && LROWS >= 2 * kGroupFP32) ? kGroupFP32 : 2;
    static_assert(2 * G <= LROWS, "the list holds at least two groups' survivors");
    if (K != 1 && kGroups) {
        // G rows at a time, four iterations per trip (P is a multiple of 4
        // here): G independent orbits per lane keep the pipeline full.  The
        // group leaves its first block early once at most `handoff` of its
        // pixels inside the tile are still inside the disc: with 0, once all
        // have escaped (absorbing: later iterates would count nothing);
        // otherwise the few still running go to the list with the count so
        // far instead of holding the wave.  Lanes past the tile's width
        // repeat its last column and are not counted.
        const int handoff = __builtin_amdgcn_readfirstlane(a.handoff);
        for (; r + G <= th; r += G) {
            if (qn + 64 * G > cap) drain();  // room for the group's survivors
            typename A::Z z[G];
            typename A::C c[G];
            int l[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                start_row(r + g, z[g], c[g]);
                l[g] = 0;
            }
            // one trip: four counted iterations of every row, then the number
            // of the group's pixels still inside
            auto trip = [&]() {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
#pragma unroll
                    for (int g = 0; g < G; ++g) l[g] += A::check_step(z[g], c[g], deg) ? 1 : 0;
                }
                int still = 0;
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const bool in = A::check_step(z[g], c[g], deg);
                    l[g] += in ? 1 : 0;
                    still += __popcll(__ballot(in) & cols);
                }
                return still;
            };
            // The first trip always runs (P >= 4) and is written out apart
            // from the loop, so it reads the rows' starting values where they
            // are instead of from copies made for the loop.  In FP64 it ends
            // early, after its second or third test, once every pixel of the
            // group has escaped (light regions escape within a test or two;
            // no pixel survives, so `done` need not be a multiple of 4).  The
            // same early end made FP32 groups slower and is left out there.
            constexpr bool kEarly = std::is_same<A, ArF64>::value;
            auto first_trip = [&]() {
                if constexpr (kEarly) {
#pragma unroll
                    for (int g = 0; g < G; ++g) l[g] += A::check_step(z[g], c[g], deg) ? 1 : 0;
#pragma unroll
                    for (int k = 2; k <= 3; ++k) {
                        uint64_t alive = 0;
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            const bool in = A::check_step(z[g], c[g], deg);
                            l[g] += in ? 1 : 0;
                            alive |= __ballot(in);
                        }
                        if ((alive & cols) == 0) return -k;  // all escaped after k tests
                    }
                    int still = 0;
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const bool in = A::check_step(z[g], c[g], deg);
                        l[g] += in ? 1 : 0;
                        still += __popcll(__ballot(in) & cols);
                    }
                    return still;
                } else {
                    return trip();
                }
            };
            int done = 4;
            const int s1 = first_trip();
            if (s1 < 0) {
                done = -s1;  // every pixel escaped: no survivors
            } else if (s1 > handoff) {
#pragma unroll 1
                while (done < P) {
                    done += 4;
                    if (trip() <= handoff) break;
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) finish_row(r + g, l[g], z[g], done);
        }
    }
    for (; r < th; ++r) {  // single rows: an odd tile height's last, P = 1, wide types
        if (qn + 64 > cap) drain();  // room for one row's survivors
        typename A::Z z;
        typename A::C c;
        start_row(r, z, c);
        int lead = 0, done = P;
        if (K == 1) {
            lead = A::check_step(z, c, deg) ? 1 : 0;  // P = 1: the exact test
        } else {
#pragma unroll 1
            for (int u = 0; u < P; u += 4) {
                lead += A::check_step(z, c, deg) ? 1 : 0;
                lead += A::check_step(z, c, deg) ? 1 : 0;
                lead += A::check_step(z, c, deg) ? 1 : 0;
                const bool in = A::check_step(z, c, deg);
                lead += in ? 1 : 0;
                // all escaped: no survivors, whatever `done` says
                if (__ballot(in) == 0) break;
            }
        }
        finish_row(r, lead, z, done);
    }
    drain();
    if (done_at) add_done(done_at, tw * th);  // the frame's progress counter
}

// Waves of 64 lanes, one tile at a time (from the dispatcher or the work
// queues), each tile in two phases (rows_tile).  P, the first block's length,
// is the schedule's bail field rounded up to a multiple of 4; K is the second
// phase's block length.  WPB is the number of waves per workgroup: 4 for the
// work queues and for large palettes (which the workgroup stages once), 1 for
// dispatched tiles, so that a wave's LDS is released as soon as its own tile
// is done instead of when the slowest of four tiles is.
template <int K, int DTMASK, int WPB, int DD>
__global__ __launch_bounds__(64 * WPB) void jr_rows(PersistentArgs a) {
    constexpr int COLOR = (DTMASK & kColorBit) ? 1 : 0;
    static_assert(WPB == 4 || WPB == 1, "one or four waves per workgroup");
    using S = RowsShape<DTMASK>;
    __shared__ uint32_t lmem[WPB * S::wave_words];
    uint32_t* list =
        WPB == 1 ? lmem
                 : lmem + (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * S::wave_words;
    stage_palette<COLOR>(a);
    Claimer cl;
    claimer_init(cl, a);
    CFrame* frames = cframes(a);
    CArgs& ka = kernel_args();
    int f = 0;
    constexpr bool kProgress = (DTMASK & kProgressBit) != 0;
    for (;;) {
        if (kProgress && stop_requested(a.stop)) break;
        const int64_t t = next_tile(cl, a);
        if (t < 0) break;
        f = find_frame(frames, a.nframes, t, f);
        CFrame& F = frames[f];
        const bool abs = F.defer != 0;
        // The first block's length: the schedule's, rounded up to a multiple
        // of 4 (four iterations per trip), or 1 where escape may not be
        // absorbing.
        // Wave-uniform; readfirstlane says so to the compiler, which otherwise
        // may keep the trip count in a vector register.
        const int P = __builtin_amdgcn_readfirstlane(abs ? (a.bail + 3) & ~3 : 1);
        const bool mandel = F.mode == kModeMandelbrot;
        int32_t* const done_at = kProgress && a.done ? a.done + F.index : nullptr;
#define JR_ROWS(A_, ARGS_)                                                               \
    do {                                                                                 \
        if (abs && !mandel) rows_tile<A_, K, 0, COLOR, S::rows, DD>(ARGS_, F, t, P, list, done_at); \
        else if (abs) rows_tile<A_, K, 1, COLOR, S::rows, DD>(ARGS_, F, t, P, list, done_at);       \
        else if (!mandel) rows_tile<A_, 1, 0, COLOR, S::rows, 0>(ARGS_, F, t, P, list, done_at);    \
        else rows_tile<A_, 1, 1, COLOR, S::rows, 0>(ARGS_, F, t, P, list, done_at);                 \
    } while (0)
        // quadratic maps: kernels that also hold the general maps call tiles
        // that are not inlined, which take the arguments in place
#define JR_ROWS_Q(A_)                          \
    do {                                       \
        if constexpr ((DTMASK & kGeneralBit) != 0) \
            JR_ROWS(A_, ka);                   \
        else                                   \
            JR_ROWS(A_, a);                    \
    } while (0)
        // rational maps: Julia images in FP64 or FP32 (the host checks)
#define JR_ROWS_R(A_)                                                              \
    do {                                                                           \
        if (abs) rows_tile<A_, K, 0, COLOR, S::rows, DD>(ka, F, t, P, list, done_at);      \
        else rows_tile<A_, 1, 0, COLOR, S::rows, 0>(ka, F, t, P, list, done_at);           \
    } while (0)
        if ((DTMASK & kRationalBit) && F.map == kMapRational) {
            if (F.dtype == kFP32)
                JR_ROWS_R(ArF32R);
            else
                JR_ROWS_R(ArF64R);
        } else if ((DTMASK & kGeneralBit) && F.degree > 2) {
            if (F.dtype == kFP32)
                JR_ROWS(ArF32G, ka);
            else if (F.dtype == kFP64)
                JR_ROWS(ArF64G, ka);
            else
                JR_ROWS(ArFFG, ka);
        } else if ((DTMASK & (1 << kFP32)) && F.dtype == kFP32)
            JR_ROWS_Q(ArF32);
        else if ((DTMASK & (1 << kFP64)) && F.dtype == kFP64)
            JR_ROWS_Q(ArF64);
        else if ((DTMASK & (1 << kFF)) && F.dtype == kFF)
            JR_ROWS_Q(ArFF);
#undef JR_ROWS
#undef JR_ROWS_R
#undef JR_ROWS_Q
    }
}

// Zeroes n words (progress counters) before a launch that counts.
__global__ __launch_bounds__(256) void jr_zero_words(int32_t* p, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) p[k] = 0;
}

// Zeroes the kQueues counters before a persistent launch (a kernel, not a
// memset, so that it can sit inside a captured hipGraph).
__global__ void jr_reset_queues(unsigned long long* ctr) {
    if (threadIdx.x < kQueues) ctr[(size_t)threadIdx.x * kQueueStride] = 0ull;
}

// Frame table of a prescribed cardioid path (Section 3), one thread per
// frame: u_k = step^k by square-and-multiply over the bits of k from the
// highest, C_k = (2 u_k - u_k^2) / (a0 - da k), each complex product taken as
// (a c - b d) + i (a d + b c) and every operation rounded (this translation
// unit does not contract a*b + c).
__device__ __forceinline__ void cmul_rounded(double a, double b, double c, double d, double& re,
                                             double& im) {
    const double ac = a * c;
    const double bd = b * d;
    const double ad = a * d;
    const double bc = b * c;
    re = ac - bd;
    im = ad + bc;
}

__global__ __launch_bounds__(256) void jr_cardioid_table(CardioidArgs g) {
    const int k = (int)(blockIdx.x * 256u + threadIdx.x);
    if (k >= g.frames) return;
    double pr = 1.0, pi = 0.0;
    for (int bit = 30; bit >= 0; --bit) {
        double r, i;
        cmul_rounded(pr, pi, pr, pi, r, i);
        pr = r;
        pi = i;
        if ((k >> bit) & 1) {
            cmul_rounded(pr, pi, g.step_re, g.step_im, r, i);
            pr = r;
            pi = i;
        }
    }
    double wr, wi;
    cmul_rounded(pr, pi, pr, pi, wr, wi);
    const double dk = g.da * (double)k;
    const double a = g.a0 - dk;
    const double nr = 2.0 * pr - wr;
    const double ni = 2.0 * pi - wi;
    DevFrame f = g.tmpl;
    f.cr = nr / a;
    f.ci = ni / a;
    f.out_offset = g.out_offset0 + (int64_t)k * g.frame_px;
    f.tile_begin = (int64_t)k * g.tiles_per_frame;
    f.index = (int32_t)k;
    g.dst[k] = f;
}

// Up to kPutFrames frame records travel inside the kernel arguments of
// jr_put_frames, which writes them to a device frame table: the table of an
// allocation-free launch needs neither a copy call nor staging memory, and the
// caller's host array may be reused as soon as the launch call returns.
struct FrameChunk {
    DevFrame f[kPutFrames];
    DevFrame* dst;
    int32_t count;
};
static_assert(sizeof(FrameChunk) <= 4096, "kernel arguments are at most 4 KiB");

__global__ __launch_bounds__(256) void jr_put_frames(FrameChunk c) {
    // Read the records straight from the kernel-argument segment (the single
    // by-value argument sits at offset 0): indexing the by-value array with
    // the thread index would copy it to per-lane stack memory first.
    constexpr int kWords = (int)(sizeof(DevFrame) / 8);
    typedef const __attribute__((address_space(4))) uint64_t CWord;
    CWord* src = (CWord*)__builtin_amdgcn_kernarg_segment_ptr();
    uint64_t* dst = reinterpret_cast<uint64_t*>(c.dst);
    for (int k = (int)threadIdx.x; k < c.count * kWords; k += (int)blockDim.x) dst[k] = src[k];
}
static_assert(sizeof(DevFrame) % 8 == 0 && offsetof(FrameChunk, f) == 0,
              "frame records are whole 8-byte words at the start of the arguments");

// The fixed device array of allocation-free launches (see julia_device.h).
// Every process holds one copy per GPU until it ends.  In host code the name
// stands for a host-side shadow, not a device address: host code uses the
// address noalloc_scratch() looks up for the current device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

}  // namespace jr

// ---------------------------------------------------------------------------
// Launch helpers used by the host runtime (julia_host.cpp).
// ---------------------------------------------------------------------------
namespace jr {

using TiledFn = void (*)(PersistentArgs);

template <int K, int DEFER, int HYB>
static TiledFn pick_mask(int dtmask) {
    if (dtmask & kRationalBit) return nullptr;  // the host runs these on the rows kernel
    if (dtmask & kGeneralBit)  // general maps: every dtype, refill stream
        return (dtmask & kColorBit) ? jr_tiled<K, DEFER, 7 | kGeneralBit | kColorBit, 0>
                                    : jr_tiled<K, DEFER, 7 | kGeneralBit, 0>;
    if (dtmask & kColorBit) {
        // one-dtype colour kernels for the common cases (the all-dtype
        // variant holds the float-float registers and runs fewer waves)
        if (!HYB && dtmask == ((1 << kFP32) | kColorBit))
            return jr_tiled<K, DEFER, (1 << kFP32) | kColorBit, HYB>;
        if (!HYB && dtmask == ((1 << kFP64) | kColorBit))
            return jr_tiled<K, DEFER, (1 << kFP64) | kColorBit, HYB>;
        return jr_tiled<K, DEFER, 7 | kColorBit, HYB>;
    }
    switch (dtmask) {
        case 1 << kFP64: return jr_tiled<K, DEFER, 1 << kFP64, HYB>;
        case 1 << kFP32: return jr_tiled<K, DEFER, 1 << kFP32, HYB>;
        case 1 << kFF: return jr_tiled<K, DEFER, 1 << kFF, HYB>;
        default: return jr_tiled<K, DEFER, 7, HYB>;
    }
}

template <int HYB>
static TiledFn pick_block(int unroll, int defer, int dtmask) {
    if (defer) {
        switch (unroll) {
            case 4: return pick_mask<4, 1, HYB>(dtmask);
            case 8: return pick_mask<8, 1, HYB>(dtmask);
            case 16: return pick_mask<16, 1, HYB>(dtmask);
            default: return nullptr;
        }
    }
    switch (unroll) {
        case 1: return pick_mask<1, 0, HYB>(dtmask);
        case 2: return pick_mask<2, 0, HYB>(dtmask);
        case 4: return pick_mask<4, 0, HYB>(dtmask);
        case 8: return pick_mask<8, 0, HYB>(dtmask);
        default: return nullptr;
    }
}

template <int K>
static TiledFn pick_rows_mask(int dtmask, bool one_wave, int defer) {
    // deferred drain blocks: launches of FP32 or FP64 frames only, counts
    if (defer && dtmask == (1 << kFP32))
        return one_wave ? jr_rows<K, 1 << kFP32, 1, 1> : jr_rows<K, 1 << kFP32, 4, 1>;
    if (defer && dtmask == (1 << kFP64))
        return one_wave ? jr_rows<K, 1 << kFP64, 1, 1> : jr_rows<K, 1 << kFP64, 4, 1>;
    constexpr int kGR = 7 | kGeneralBit | kRationalBit;
    if (dtmask & kProgressBit) {  // any frames, counted
        constexpr int kGRP = kGR | kProgressBit;
        if (dtmask & kColorBit) return jr_rows<K, kGRP | kColorBit, 4, 0>;
        return one_wave ? jr_rows<K, kGRP, 1, 0> : jr_rows<K, kGRP, 4, 0>;
    }
    if (dtmask & kRationalBit) {
        if (dtmask & kColorBit) return jr_rows<K, kGR | kColorBit, 4, 0>;
        return one_wave ? jr_rows<K, kGR, 1, 0> : jr_rows<K, kGR, 4, 0>;
    }
    if (one_wave && dtmask == ((1 << kFP32) | kColorBit))
        return jr_rows<K, (1 << kFP32) | kColorBit, 1, 0>;
    if (one_wave && !(dtmask & kColorBit)) {
        if (dtmask & kGeneralBit) return jr_rows<K, 7 | kGeneralBit, 1, 0>;
        switch (dtmask) {
            case 1 << kFP32: return jr_rows<K, 1 << kFP32, 1, 0>;
            case 1 << kFP64: return jr_rows<K, 1 << kFP64, 1, 0>;
            case 1 << kFF: return jr_rows<K, 1 << kFF, 1, 0>;
            default: return jr_rows<K, 7, 1, 0>;
        }
    }
    if (dtmask & kGeneralBit)
        return (dtmask & kColorBit) ? jr_rows<K, 7 | kGeneralBit | kColorBit, 4, 0>
                                    : jr_rows<K, 7 | kGeneralBit, 4, 0>;
    switch (dtmask) {
        case 1 << kFP32: return jr_rows<K, 1 << kFP32, 4, 0>;
        case 1 << kFP64: return jr_rows<K, 1 << kFP64, 4, 0>;
        case 1 << kFF: return jr_rows<K, 1 << kFF, 4, 0>;
        case (1 << kFP32) | kColorBit: return jr_rows<K, (1 << kFP32) | kColorBit, 4, 0>;
        default: return (dtmask & kColorBit) ? jr_rows<K, 7 | kColorBit, 4, 0> : jr_rows<K, 7, 4, 0>;
    }
}

static TiledFn pick_rows(int unroll, int dtmask, bool one_wave, int defer) {
    switch (unroll) {
        case 4: return pick_rows_mask<4>(dtmask, one_wave, defer);
        case 8: return pick_rows_mask<8>(dtmask, one_wave, defer);
        default: return nullptr;
    }
}

static TiledFn pick(int unroll, int defer, int dtmask, int hybrid) {
    return hybrid ? pick_block<1>(unroll, defer, dtmask) : pick_block<0>(unroll, defer, dtmask);
}

static TiledFn pick_plain(int dtmask) {
    if (dtmask & kProgressBit)
        return (dtmask & kColorBit)
                   ? jr_plain_batch<7 | kGeneralBit | kRationalBit | kProgressBit | kColorBit>
                   : jr_plain_batch<7 | kGeneralBit | kRationalBit | kProgressBit>;
    if (dtmask & kRationalBit)
        return (dtmask & kColorBit) ? jr_plain_batch<7 | kGeneralBit | kRationalBit | kColorBit>
                                    : jr_plain_batch<7 | kGeneralBit | kRationalBit>;
    if (dtmask & kGeneralBit)
        return (dtmask & kColorBit) ? jr_plain_batch<7 | kGeneralBit | kColorBit>
                                    : jr_plain_batch<7 | kGeneralBit>;
    if (dtmask == ((1 << kFP32) | kColorBit)) return jr_plain_batch<(1 << kFP32) | kColorBit>;
    if (dtmask == ((1 << kFP64) | kColorBit)) return jr_plain_batch<(1 << kFP64) | kColorBit>;
    if (dtmask & kColorBit) return jr_plain_batch<7 | kColorBit>;
    switch (dtmask) {
        case 1 << kFP64: return jr_plain_batch<1 << kFP64>;
        case 1 << kFP32: return jr_plain_batch<1 << kFP32>;
        case 1 << kFF: return jr_plain_batch<1 << kFF>;
        default: return jr_plain_batch<7>;
    }
}

static unsigned palette_bytes(const PersistentArgs& a) {
    return a.palette_len > 0 ? (unsigned)a.palette_len * 4u : 0u;
}

hipError_t launch_plain_batch(int dtmask, const PersistentArgs& args, hipStream_t stream) {
    if (args.palette_len > kPaletteMax) return hipErrorInvalidValue;
    if (args.total_tiles > 0x7fffffffLL) return hipErrorInvalidValue;
    if (args.palette_len > 0) dtmask |= kColorBit;
    if (args.done) dtmask |= kProgressBit;
    hipLaunchKernelGGL(pick_plain(dtmask), dim3((unsigned)args.total_tiles), dim3(256),
                       palette_bytes(args), stream, args);
    return hipGetLastError();
}

// Dispatched rows tiles (one tile per wave) run in one-wave workgroups, one
// per tile, unless they store colours from a palette larger than
// kOneWavePalette or of a batch that is not FP32 only (such workgroups of
// four waves stage the palette once).
static bool one_wave_launch(int dtmask, const PersistentArgs& args) {
    if (args.palette_len > 0) dtmask |= kColorBit;
    // (the counting kernels' colour variant has four-wave workgroups)
    const bool small_palette = dtmask == ((1 << kFP32) | kColorBit) &&
                               args.palette_len <= kOneWavePalette && !args.done;
    return args.rows && !args.persistent && (!(dtmask & kColorBit) || small_palette) &&
           args.total_tiles <= 0x7fffffffLL;
}

int launch_workgroups(int dtmask, const PersistentArgs& args, int blocks) {
    return one_wave_launch(dtmask, args) ? (int)args.total_tiles : blocks;
}

hipError_t launch_tiled(int unroll, int defer, int dtmask, int blocks, const PersistentArgs& args,
                        hipStream_t stream) {
    const bool one_wave = one_wave_launch(dtmask, args);
    blocks = launch_workgroups(dtmask, args, blocks);
    if (args.palette_len > 0) dtmask |= kColorBit;
    const unsigned threads = one_wave ? 64u : 256u;
    if (args.done) {
        if (!args.rows) return hipErrorInvalidValue;  // progress: rows and plain kernels
        dtmask |= kProgressBit;
    }
    TiledFn fn = args.rows ? pick_rows(unroll, dtmask, one_wave, defer)
                           : pick(unroll, defer, dtmask, args.hybrid);
    if (!fn || args.palette_len > kPaletteMax) return hipErrorInvalidValue;
    if (args.persistent) {
        hipLaunchKernelGGL(jr_reset_queues, dim3(1), dim3(kQueues), 0, stream, args.ctr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), palette_bytes(args), stream, args);
    return hipGetLastError();
}

hipError_t noalloc_scratch(int dev, void** ptr) {
    constexpr int kDevices = 64;
    static std::mutex mu;
    static void* addr[kDevices] = {};
    if (dev < 0 || dev >= kDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        // Each GPU holds its own copy of the array at its own address; the
        // caller has made `dev` the current device.
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_cardioid_table(const CardioidArgs& g, hipStream_t stream) {
    if (g.frames < 1) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((g.frames + 255) / 256);
    hipLaunchKernelGGL(jr_cardioid_table, dim3(blocks), dim3(256), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_zero_words(int32_t* p, int64_t n, hipStream_t stream) {
    if (n < 1 || p == nullptr) return hipErrorInvalidValue;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(jr_zero_words, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t put_frames(const DevFrame* rows, int n, DevFrame* dst, hipStream_t stream) {
    for (int k0 = 0; k0 < n; k0 += kPutFrames) {
        FrameChunk c;
        c.count = n - k0 < kPutFrames ? n - k0 : kPutFrames;
        c.dst = dst + k0;
        for (int k = 0; k < c.count; ++k) c.f[k] = rows[k0 + k];
        hipLaunchKernelGGL(jr_put_frames, dim3(1), dim3(256), 0, stream, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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
