/*
 * dsr_kernels.hip -- generic-mode region kernel of the data-sharing runtime.
 *
 * One workgroup per team.  The last wave is the master wave (section 4,
 * Figure 2: the master is isolated from the workers); it interprets the
 * region's program of PUSH / PUBLISH / POP operations, i.e. the sequential
 * code block that declares the shared locals.  Worker waves sit in the
 * await loop of Figure 3 and run whichever outlined body the master
 * publishes, reading the shared locals through the published frame
 * (section 5.1: sharing by reference), then reduce into the frame's shared
 * variable and join.  After its program the master publishes TERMINATE;
 * the last team to finish combines the teams' partial reductions.
 *
 * Exact fp64 reduction: every loop value y must be a multiple of 2^-75 with
 * |y| < 2^32.  Each lane splits y exactly into three parts on the grids
 * 2^-5, 2^-40 and 2^-75 (y + C - C rounding with a constant C whose last
 * bit has the grid's weight) and adds each part into its own fp64 bin.  A
 * bin's values have at most 37 significant bits above its grid, so up to
 * 2^16 of them sum exactly in fp64.  At the end of the loop each lane turns
 * its bins into one signed 192-bit integer of 2^-75 units; waves, teams and
 * the region add those integers, and the region total is rounded to double
 * once.  The result is the correctly rounded sum whatever the team, wave or
 * launch layout.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsr.h"
#include "dsr_device.h"
#include "dsr_internal.h"

using namespace dsr;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

/* Element pairs per lane and batch in the run-time fma chain (256- and
 * 512-thread instances), and in the fixed chains of up to four scalars. */
#ifndef DSR_FIXED_U_LIGHT
#define DSR_FIXED_U_LIGHT 8
#endif
#ifndef DSR_RT_PAIRS
#define DSR_RT_PAIRS 8
#endif

extern __shared__ __align__(16) uint8_t dsr_lds[];

/* Address-space qualifiers: loop buffers are global memory; without the
 * qualifier the compiler emits flat instructions for them, which also wait
 * on the LDS counter and cannot use scalar-base addressing. */
#define GLB __attribute__((address_space(1)))
#define LDSQ __attribute__((address_space(3)))

/* ---- exact accumulation ------------------------------------------------ */
struct i192 { uint64_t w0, w1, w2; };

__device__ __forceinline__ i192 add192(i192 a, i192 b)
{
    i192 r;
    r.w0 = a.w0 + b.w0;
    const uint64_t c0 = r.w0 < a.w0;
    const uint64_t t = a.w1 + b.w1;
    const uint64_t c1a = t < a.w1;
    r.w1 = t + c0;
    const uint64_t c1b = r.w1 < t;
    r.w2 = a.w2 + b.w2 + c1a + c1b;
    return r;
}

__device__ __forceinline__ i192 from_i64(int64_t v)
{
    return i192{(uint64_t)v, (uint64_t)(v >> 63), (uint64_t)(v >> 63)};
}

/* v * 2^sh for a signed 64-bit v and 0 <= sh < 128. */
__device__ __forceinline__ i192 shl192(int64_t v, int sh)
{
    const uint64_t ext = (uint64_t)(v >> 63);
    uint64_t w0 = (uint64_t)v, w1 = ext, w2 = ext;
    if (sh >= 64) { w2 = w1; w1 = w0; w0 = 0; sh -= 64; }
    if (sh) {
        w2 = (w2 << sh) | (w1 >> (64 - sh));
        w1 = (w1 << sh) | (w0 >> (64 - sh));
        w0 <<= sh;
    }
    return i192{w0, w1, w2};
}

struct lane_acc {
    double b1, b2, b3;   /* bins on the 2^-5, 2^-40 and 2^-75 grids        */
    int64_t i;           /* integer bodies: wrap-around int64 sum          */
    uint32_t bad;        /* a value fell outside the exact-sum window      */
    i192 big;            /* bins flushed so far, in 2^-75 units            */
};

__device__ __forceinline__ lane_acc acc_zero()
{
    lane_acc a;
    a.b1 = a.b2 = a.b3 = 0.0;
    a.i = 0;
    a.bad = 0;
    a.big = i192{0, 0, 0};
    return a;
}

__device__ __forceinline__ void acc_add_i64(lane_acc &a, int64_t v)
{
    a.i = (int64_t)((uint64_t)a.i + (uint64_t)v);
}

/* Split y exactly into y = t1 + t2 + r2 with t1 on the 2^-5 grid, t2 on
 * the 2^-40 grid and |r2| <= 2^-41, and add the parts to the bins.  r2 must
 * itself be on the 2^-75 grid (checked by rounding it there). */
__device__ __forceinline__ void acc_add_f64(lane_acc &a, double y)
{
    const double C1 = 0x1.8p47, C2 = 0x1.8p12, C3 = 0x1.8p-23;
    const double t1 = (y + C1) - C1;
    const double r1 = y - t1;
    const double t2 = (r1 + C2) - C2;
    const double r2 = r1 - t2;
    const double t3 = (r2 + C3) - C3;
    a.bad |= (uint32_t)((t3 != r2) | !(__builtin_fabs(y) < 0x1p32));
    a.b1 += t1;
    a.b2 += t2;
    a.b3 += r2;
}

/* Bins of the same grid add exactly while each holds fewer than 2^16
 * values. */
__device__ __forceinline__ void acc_merge(lane_acc &a, const lane_acc &b)
{
    a.b1 += b.b1;
    a.b2 += b.b2;
    a.b3 += b.b3;
    a.bad |= b.bad;
}

/* A lane's bins as one integer of 2^-75 units (bin values are integers of
 * their grid below 2^53 in magnitude, so the conversions are exact). */
__device__ __forceinline__ i192 bins_fixed(const lane_acc &a)
{
    const int64_t k1 = (int64_t)(a.b1 * 0x1p5);
    const int64_t k2 = (int64_t)(a.b2 * 0x1p40);
    const int64_t k3 = (int64_t)(a.b3 * 0x1p75);
    i192 s = add192(shl192(k1, 70), shl192(k2, 35));
    return add192(s, from_i64(k3));
}

/* Move the bins into the 192-bit accumulator (keeps them exact however
 * many values a lane adds). */
__device__ __forceinline__ void acc_flush(lane_acc &a)
{
    a.big = add192(a.big, bins_fixed(a));
    a.b1 = a.b2 = a.b3 = 0.0;
}

__device__ __forceinline__ i192 widen(const lane_acc &a)
{
    return add192(add192(a.big, bins_fixed(a)), from_i64(a.i));
}

/* One DPP step of the wave sum: every 32-bit part of v moved from the lane
 * the control selects (zero where that lane is outside the row, and in the
 * rows the mask leaves out), then added with carries. */
template <int CTRL, int ROWS>
__device__ __forceinline__ i192 dpp_add192(i192 v)
{
    const uint32_t p[6] = {(uint32_t)v.w0, (uint32_t)(v.w0 >> 32), (uint32_t)v.w1,
                           (uint32_t)(v.w1 >> 32), (uint32_t)v.w2, (uint32_t)(v.w2 >> 32)};
    uint32_t q[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) q[k] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)p[k], CTRL, ROWS, 0xf, true);
    return add192(v, i192{q[0] | ((uint64_t)q[1] << 32), q[2] | ((uint64_t)q[3] << 32), q[4] | ((uint64_t)q[5] << 32)});
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

/* Sum over the 64 lanes of a wave, returned to every lane: a running sum
 * inside each row of 16 lanes (row shifts by 1, 2, 4 and 8), then the row
 * totals carried across rows (lane 15 into row 1 and 3, lane 31 into rows 2
 * and 3), so lane 63 holds the total; all in VALU moves, no LDS round
 * trips.  Every lane of the wave takes part. */
__device__ __forceinline__ i192 wave_sum192(i192 v)
{
    v = dpp_add192<0x111, 0xf>(v);   /* row_shr:1 */
    v = dpp_add192<0x112, 0xf>(v);   /* row_shr:2 */
    v = dpp_add192<0x114, 0xf>(v);   /* row_shr:4 */
    v = dpp_add192<0x118, 0xf>(v);   /* row_shr:8 */
    v = dpp_add192<0x142, 0xa>(v);   /* row_bcast:15 into rows 1 and 3 */
    v = dpp_add192<0x143, 0xc>(v);   /* row_bcast:31 into rows 2 and 3 */
    return i192{readlane64(v.w0, 63), readlane64(v.w1, 63), readlane64(v.w2, 63)};
}

__device__ __forceinline__ uint64_t bits64(uint64_t w0, uint64_t w1, uint64_t w2, int p)
{
    const int q = p >> 6, r = p & 63;
    const uint64_t a = q == 0 ? w0 : (q == 1 ? w1 : w2);
    const uint64_t b = q == 0 ? w1 : (q == 1 ? w2 : 0ull);
    return r ? ((a >> r) | (b << (64 - r))) : a;
}

__device__ __forceinline__ bool any_below(uint64_t w0, uint64_t w1, uint64_t w2, int p)
{
    if (p <= 0) return false;
    const int q = p >> 6, r = p & 63;
    if (q > 0 && w0) return true;
    if (q > 1 && w1) return true;
    if (r == 0) return false;
    const uint64_t w = q == 0 ? w0 : (q == 1 ? w1 : w2);
    return (w & ((1ull << r) - 1ull)) != 0;
}

/* Nearest-even double of the signed 192-bit value times 2^-75. */
__device__ double fixed_to_double(i192 v)
{
    const bool neg = (int64_t)v.w2 < 0;
    uint64_t w0 = v.w0, w1 = v.w1, w2 = v.w2;
    if (neg) {
        w0 = ~w0; w1 = ~w1; w2 = ~w2;
        w0 += 1;
        uint64_t c = (w0 == 0);
        w1 += c;
        c = c && (w1 == 0);
        w2 += c;
    }
    int top;
    if (w2) top = 128 + 63 - __clzll((long long)w2);
    else if (w1) top = 64 + 63 - __clzll((long long)w1);
    else if (w0) top = 63 - __clzll((long long)w0);
    else return 0.0;
    uint64_t mant;
    bool round = false, sticky = false;
    if (top <= 52) {
        mant = w0 << (52 - top);
    } else {
        const int p = top - 52;
        mant = bits64(w0, w1, w2, p) & ((1ull << 53) - 1ull);
        round = bits64(w0, w1, w2, p - 1) & 1ull;
        sticky = any_below(w0, w1, w2, p - 1);
    }
    if (round && (sticky || (mant & 1ull))) {
        mant += 1;
        if (mant >> 53) { mant >>= 1; top += 1; }
    }
    const uint64_t E = (uint64_t)(top - 75 + 1023);
    const uint64_t bits = ((uint64_t)neg << 63) | (E << 52) | (mant & ((1ull << 52) - 1ull));
    return __longlong_as_double((long long)bits);
}

/* ---- loop bodies --------------------------------------------------------- */
/* A span is a range [lo, hi) of loop iterations shared cyclically by P
 * lanes, of which this lane is number p. */
struct span_t {
    uint64_t lo, hi;
    uint32_t p, P;
};

/* Drive a body over this lane's static share `sp` and then, under the
 * dynamic-tail schedule, over the blocks its wave claims from the loop's
 * device counter (the next claim is issued before the current block runs,
 * so its latency overlaps the work).  Claimed blocks are shared by the 64
 * lanes of the claiming wave. */
/* Balanced split of a team's static range among its waves: the range is
 * cut into blocks of DSR_TEAM_BLOCK iterations that the waves claim from a
 * counter in the team's LDS control block.  A wave then streams contiguous
 * 8 KiB stretches of x (one batch of eight pairs per lane), and a wave on a
 * SIMD it shares with fewer others takes more blocks: with three worker
 * waves per team and two teams per CU some SIMDs hold two worker waves and
 * some one.  Measured on the fma chains against the fixed per-lane share:
 * 2.2-2.7 us faster per 2^24-element region for up to 16 scalars, 0.5-1.2 us
 * for 32 and 64; 2048-, 4096- and 8192-iteration blocks were slower. */
/* teams up to this many arrive at one counter (no group level) */
#ifndef DSR_FLAT_TEAMS
#define DSR_FLAT_TEAMS 512
#endif
#ifndef DSR_ARRIVE_FENCE
#define DSR_ARRIVE_FENCE 1
#endif
#ifndef DSR_TEAM_BLOCK
#define DSR_TEAM_BLOCK 1024u
#endif
/* chains of at least this many scalars take the balanced split (all) */
#ifndef DSR_BALANCE_MIN
#define DSR_BALANCE_MIN 1
#endif
/* fixed chains stream their balanced blocks pipelined across blocks */
#ifndef DSR_STREAM_BLOCKS
#define DSR_STREAM_BLOCKS 1
#endif

template <class F>
__device__ __forceinline__ void team_blocks(span_t sp, uint32_t lane, lane_acc &A, F &&f)
{
    LDSQ uint32_t *ctr = (LDSQ uint32_t *)(dsr_lds + offsetof(cb_header, blocks));
    const uint64_t lo = sp.lo;
    const uint32_t nblk = sp.hi > lo ? (uint32_t)((sp.hi - lo + DSR_TEAM_BLOCK - 1) / DSR_TEAM_BLOCK) : 0u;
    uint32_t c = 0;
    if (lane == 0) c = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    c = uniform((uint32_t)__shfl((int)c, 0, 64));
    uint32_t since = 0;
    while (c < nblk) {
        uint32_t cn = 0;
        if (lane == 0) cn = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint64_t b = lo + (uint64_t)c * DSR_TEAM_BLOCK;
        f(span_t{b, min(sp.hi, b + DSR_TEAM_BLOCK), lane, 64u});
        /* a block adds 32 values per lane: flush well before 2^16 */
        if (++since == 256) { acc_flush(A); since = 0; }
        c = uniform((uint32_t)__shfl((int)cn, 0, 64));
    }
}

template <class F>
__device__ __forceinline__ void for_spans(const dsr_dloop &L, span_t sp, uint32_t lane,
                                          uint32_t *claim, lane_acc &A, F &&f, bool balanced = false)
{
    if (balanced && L.schedule == DSR_SCHED_STATIC) {
        team_blocks(sp, lane, A, f);
        return;
    }
    f(sp);
    if (L.schedule != DSR_SCHED_DYNAMIC_TAIL) return;
    uint32_t c = 0;
    if (lane == 0) c = atomicAdd(claim, 1u);
    c = (uint32_t)__shfl((int)c, 0, 64);
    uint32_t since = 0;
    for (;;) {
        const uint64_t lo = L.dyn_start + (uint64_t)c * L.block;
        if (lo >= L.n) break;
        uint32_t cn = 0;
        if (lane == 0) cn = atomicAdd(claim, 1u);
        f(span_t{lo, min(L.n, lo + (uint64_t)L.block), lane, 64u});
        /* a block adds at most 1024 values per lane: flush well before 2^16 */
        if (++since == 16) { acc_flush(A); since = 0; }
        c = (uint32_t)__shfl((int)cn, 0, 64);
    }
}

__device__ __forceinline__ void affine_span(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                            GLB int32_t *out, span_t sp, lane_acc &A)
{
    int64_t s = 0;
    for (uint64_t i = sp.lo + sp.p; i < sp.hi; i += sp.P) {
        const uint32_t ui = (uint32_t)i;
        const int32_t o = (int32_t)(a * ui + b - (c ^ ui) + d);
        out[i] = o;
        s += o;
    }
    acc_add_i64(A, s);
}

/* fma chain with the scalar counts known at compile time. */
template <int NI, int NF>
__device__ __forceinline__ double chain(const double (&s)[NI + NF], double xd)
{
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < NI + NF; ++k) acc = __builtin_fma(s[k], xd, acc);
    return acc;
}

/* Lane-to-element mapping of the streaming loop: a lane takes element
 * pairs (8 B of x, 16 B of y), so every load instruction of a wave covers
 * 512 contiguous bytes of x and every store 1 KB of y; consecutive batches
 * of U pairs per lane are software-pipelined (the next batch's loads are in
 * flight while the current batch computes). */
template <int NI, int NF>
__device__ __forceinline__ void fma_span(const double (&s)[NI + NF], const GLB float *__restrict__ x,
                                         GLB double *__restrict__ y, span_t sp, lane_acc &A)
{
    /* head element when the range starts on an odd index */
    const uint64_t plo = min(sp.hi, (sp.lo + 1) & ~1ull);
    const uint64_t phi = max(plo, sp.hi & ~1ull);
    if (sp.lo < plo && sp.p == 0) {
        const double v = chain<NI, NF>(s, (double)x[sp.lo]);
        y[sp.lo] = v;
        acc_add_f64(A, v);
    }
    lane_acc Ac[2] = {acc_zero(), acc_zero()};
    const GLB f32x2 *__restrict__ x2 = (const GLB f32x2 *)x;
    GLB f64x2 *__restrict__ y2 = (GLB f64x2 *)y;
    const uint64_t nv1 = phi >> 1;
    constexpr int U = (NI + NF >= 64) ? 4 : (NI + NF <= 4 ? DSR_FIXED_U_LIGHT : 8);
    /* the 64-scalar chain computes a batch for as long as the memory takes
     * to return one, so it keeps two batches in flight ahead of the one it
     * computes: 1.3 us faster per 2^24-element region on the lean instance */
    constexpr bool DEEP = NI + NF >= 64;
    const uint64_t step = (uint64_t)U * sp.P;
    uint64_t v = (plo >> 1) + sp.p;
    if (DEEP && v + (uint64_t)(U - 1) * sp.P < nv1) {
        /* two batches in flight ahead of the one being computed */
        f32x2 b0[U], b1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) b0[u] = __builtin_nontemporal_load(&x2[v + (uint64_t)u * sp.P]);
        bool m1 = v + step + (uint64_t)(U - 1) * sp.P < nv1;
        if (m1) {
#pragma unroll
            for (int u = 0; u < U; ++u) b1[u] = __builtin_nontemporal_load(&x2[v + step + (uint64_t)u * sp.P]);
        }
        for (;;) {
            const uint64_t v2 = v + 2 * step;
            const bool m2 = m1 && v2 + (uint64_t)(U - 1) * sp.P < nv1;
            f32x2 b2[U];
            if (m2) {
#pragma unroll
                for (int u = 0; u < U; ++u) b2[u] = __builtin_nontemporal_load(&x2[v2 + (uint64_t)u * sp.P]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                f64x2 r;
                r.x = chain<NI, NF>(s, (double)b0[u].x);
                r.y = chain<NI, NF>(s, (double)b0[u].y);
                __builtin_nontemporal_store(r, &y2[v + (uint64_t)u * sp.P]);
                acc_add_f64(Ac[0], r.x);
                acc_add_f64(Ac[1], r.y);
            }
            v += step;
            if (!m1) break;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                b0[u] = b1[u];
                b1[u] = b2[u];
            }
            m1 = m2;
        }
    } else if (v + (uint64_t)(U - 1) * sp.P < nv1) {
        f32x2 cur[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = __builtin_nontemporal_load(&x2[v + (uint64_t)u * sp.P]);
        for (;;) {
            const uint64_t vn = v + step;
            const bool more = vn + (uint64_t)(U - 1) * sp.P < nv1;
            f32x2 nxt[U];
            if (more) {
#pragma unroll
                for (int u = 0; u < U; ++u) nxt[u] = __builtin_nontemporal_load(&x2[vn + (uint64_t)u * sp.P]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                f64x2 r;
                r.x = chain<NI, NF>(s, (double)cur[u].x);
                r.y = chain<NI, NF>(s, (double)cur[u].y);
                __builtin_nontemporal_store(r, &y2[v + (uint64_t)u * sp.P]);
                acc_add_f64(Ac[0], r.x);
                acc_add_f64(Ac[1], r.y);
            }
            v = vn;
            if (!more) break;
#pragma unroll
            for (int u = 0; u < U; ++u) cur[u] = nxt[u];
        }
    }
    for (; v < nv1; v += sp.P) {
        const f32x2 xv = __builtin_nontemporal_load(&x2[v]);
        f64x2 r;
        r.x = chain<NI, NF>(s, (double)xv.x);
        r.y = chain<NI, NF>(s, (double)xv.y);
        __builtin_nontemporal_store(r, &y2[v]);
        acc_add_f64(Ac[0], r.x);
        acc_add_f64(Ac[1], r.y);
    }
    if (phi < sp.hi && sp.p == 0) {
        const double r = chain<NI, NF>(s, (double)x[phi]);
        y[phi] = r;
        acc_add_f64(A, r);
    }
    acc_merge(A, Ac[0]);
    acc_merge(A, Ac[1]);
}

/* Shared scalars are wave-uniform: read them once as uniform values, so
 * they live in scalar registers and no frame load is still in flight when
 * the streaming loop starts (an outstanding frame load would make every
 * iteration wait for all memory operations). */
__device__ __forceinline__ uint32_t uniform_u32(const uint8_t *p)
{
    return uniform(*(const uint32_t *)p);
}

__device__ __forceinline__ double uniform_f64(const uint8_t *p)
{
    const uint64_t lo = uniform_u32(p), hi = uniform_u32(p + 4);
    return __longlong_as_double((long long)(lo | (hi << 32)));
}

/* The balanced split for a fixed chain, pipelined across blocks: a block is
 * one batch (U pairs per lane, 128·U elements); a wave claims its next
 * block and issues that block's loads before it computes the current one,
 * so two batches stay in flight however the blocks fall.  A partial last
 * block of the range goes through fma_span.  Measured 0.2-0.8 us faster
 * per 2^24-element region than one fma_span per claimed block for up to 32
 * scalars, 0.8 us slower for 64 (whose batches are half as long), which
 * keeps the per-block spans. */
template <int NI, int NF>
__device__ __forceinline__ void fma_blocks(const double (&s)[NI + NF], const GLB float *__restrict__ x,
                                           GLB double *__restrict__ y, span_t sp, uint32_t lane, lane_acc &A)
{
    constexpr int U = (NI + NF >= 64) ? 4 : (NI + NF <= 4 ? DSR_FIXED_U_LIGHT : 8);
    constexpr uint32_t BLK = 128u * U;
    LDSQ uint32_t *ctr = (LDSQ uint32_t *)(dsr_lds + offsetof(cb_header, blocks));
    const uint64_t lo = sp.lo;
    const uint32_t nfull = sp.hi > lo ? (uint32_t)((sp.hi - lo) / BLK) : 0u;
    const bool tail = sp.hi > lo + (uint64_t)nfull * BLK;
    const GLB f32x2 *__restrict__ x2 = (const GLB f32x2 *)x;
    GLB f64x2 *__restrict__ y2 = (GLB f64x2 *)y;
    lane_acc Ac[2] = {acc_zero(), acc_zero()};
    uint32_t c = 0;
    if (lane == 0) c = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    c = uniform((uint32_t)__shfl((int)c, 0, 64));
    f32x2 cur[U];
    if (c < nfull) {
        const uint64_t v = (lo >> 1) + (uint64_t)c * (BLK / 2) + lane;
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = __builtin_nontemporal_load(&x2[v + 64u * u]);
    }
    uint32_t since = 0;
    while (c < nfull) {
        uint32_t cn = 0;
        if (lane == 0) cn = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        cn = uniform((uint32_t)__shfl((int)cn, 0, 64));
        f32x2 nxt[U];
        if (cn < nfull) {
            const uint64_t vn = (lo >> 1) + (uint64_t)cn * (BLK / 2) + lane;
#pragma unroll
            for (int u = 0; u < U; ++u) nxt[u] = __builtin_nontemporal_load(&x2[vn + 64u * u]);
        }
        const uint64_t v = (lo >> 1) + (uint64_t)c * (BLK / 2) + lane;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            f64x2 r;
            r.x = chain<NI, NF>(s, (double)cur[u].x);
            r.y = chain<NI, NF>(s, (double)cur[u].y);
            __builtin_nontemporal_store(r, &y2[v + 64u * u]);
            acc_add_f64(Ac[0], r.x);
            acc_add_f64(Ac[1], r.y);
        }
        /* a block adds U values to each of the two bins: flush well before 2^16 */
        if (++since == 2048) {
            acc_merge(A, Ac[0]);
            acc_merge(A, Ac[1]);
            Ac[0] = acc_zero();
            Ac[1] = acc_zero();
            acc_flush(A);
            since = 0;
        }
        c = cn;
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }
    acc_merge(A, Ac[0]);
    acc_merge(A, Ac[1]);
    /* the claim that went past the full blocks takes the partial block */
    if (c == nfull && tail) fma_span<NI, NF>(s, x, y, span_t{lo + (uint64_t)nfull * BLK, sp.hi, lane, 64u}, A);
}

/* BLOCKS: the static schedule streams the balanced block split (general
 * instances); without it every participating wave takes its fixed per-lane
 * share of the team's range.  On the lean instances the fixed share
 * measured 0.3-1.0 us faster per 2^24-element region for 8 to 32 scalars
 * and the same below (both builds timed interleaved on one GPU). */
template <int NI, int NF, bool BLOCKS = true>
__device__ __forceinline__ void fma_fixed_spans(const double (&s)[NI + NF], const dsr_dloop &L, span_t sp,
                                                lane_acc &A, uint32_t *claim, uint32_t lane)
{
    const GLB float *x = (const GLB float *)L.in;
    GLB double *y = (GLB double *)L.out;
    if (!BLOCKS && L.schedule == DSR_SCHED_STATIC) {
        fma_span<NI, NF>(s, x, y, sp, A);
        return;
    }
    /* (a team range starting on an odd element keeps the per-span path) */
    if (DSR_STREAM_BLOCKS && NI + NF < 64 && L.schedule == DSR_SCHED_STATIC && !(uniform((uint32_t)sp.lo) & 1u)) {
        fma_blocks<NI, NF>(s, x, y, sp, lane, A);
        return;
    }
    for_spans(L, sp, lane, claim, A, [&](span_t q) { fma_span<NI, NF>(s, x, y, q, A); }, NI + NF >= DSR_BALANCE_MIN);
}

template <int NI, int NF, bool BLOCKS = true>
__device__ __forceinline__ void body_fma_fixed(const team_t &T, frame_t f, const dsr_dloop &L, span_t sp,
                                               lane_acc &A, uint32_t *claim, uint32_t lane)
{
    /* frame layout: [24 B exact sum][NF fp64][NI int32] */
    double s[NI + NF];
#pragma unroll
    for (int k = 0; k < NI; ++k)
        s[k] = (double)(int32_t)uniform_u32((const uint8_t *)slot<int32_t>(T, f, 24 + 8 * NF + 4 * k));
#pragma unroll
    for (int k = 0; k < NF; ++k) s[NI + k] = uniform_f64((const uint8_t *)slot<double>(T, f, 24 + 8 * k));
    fma_fixed_spans<NI, NF, BLOCKS>(s, L, sp, A, claim, lane);
}

/* The same chain with its scalars held one per lane (lane k: scalar k). */
template <int NI, int NF>
__device__ __forceinline__ void lanes_fma_fixed(double sv, const dsr_dloop &L, span_t sp, lane_acc &A,
                                                uint32_t *claim, uint32_t lane);

/* fma chain with a run-time scalar count (at most 64) and an optional
 * shared int32 array (the chain then starts from the array element).  The
 * scalars come from one of two sources:
 *   lds_scalars   the frame is in LDS: each chain step reads its scalar with
 *                 a wave-uniform LDS load (a broadcast) shared by every
 *                 element of the batch; int32 scalars are read in pairs.
 *   lane_scalars  the frame is in HBM: lane k holds scalar k as a double
 *                 (loaded once per body) and each step takes it with two
 *                 readlanes.
 * The array index i mod alen is carried from element to element (one
 * conditional subtraction per step) instead of divided.  The element
 * layout, batching and software pipelining are those of fma_span. */
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double readlane_f64(double v, uint32_t k)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, k);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), k);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int NI, int NF>
__device__ __forceinline__ void lanes_fma_fixed(double sv, const dsr_dloop &L, span_t sp, lane_acc &A,
                                                uint32_t *claim, uint32_t lane)
{
    double s[NI + NF];
#pragma unroll
    for (int k = 0; k < NI + NF; ++k) s[k] = readlane_f64(sv, k);
    fma_fixed_spans<NI, NF>(s, L, sp, A, claim, lane);
}

__device__ __forceinline__ uint32_t mod_step(uint32_t j, uint32_t d, uint32_t m)
{
    j += d;
    return j >= m ? j - m : j;
}

template <int E>
__device__ __forceinline__ void fma_all(double s, double (&acc)[E], const double (&xd)[E])
{
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = __builtin_fma(s, xd[e], acc[e]);
}

struct lds_scalars {
    const LDSQ int32_t *si;   /* ni int32 scalars (8-byte aligned) */
    const LDSQ double *sf;    /* nf fp64 scalars                   */
    uint32_t ni, nf;

    template <int E>
    __device__ __forceinline__ void chain(double (&acc)[E], const double (&xd)[E]) const
    {
        uint32_t k = 0;
#pragma unroll 2
        for (; k + 2 <= ni; k += 2) {
            const i32x2 q = *(const LDSQ i32x2 *)(si + k);
            fma_all<E>((double)q.x, acc, xd);
            fma_all<E>((double)q.y, acc, xd);
        }
        if (k < ni) fma_all<E>((double)si[k], acc, xd);
#pragma unroll 4
        for (uint32_t f = 0; f < nf; ++f) fma_all<E>(sf[f], acc, xd);
    }
};

struct lane_scalars {
    double sv;                /* lane k: scalar k */
    uint32_t n;

    template <int E>
    __device__ __forceinline__ void chain(double (&acc)[E], const double (&xd)[E]) const
    {
        for (uint32_t k = 0; k < n; ++k) fma_all<E>(readlane_f64(sv, k), acc, xd);
    }
};

/* The scalars read through the published reference list on every batch:
 * each chain step reads reference 1 + k (a space and an offset), then the
 * variable it names, as outlined code must when stores in its loop may
 * alias the shared variables (section 5.1's sharing by reference).  The
 * list is on chip or in a list frame on the HBM stack, the variables on
 * either stack; all of it is read through generic pointers, as the outlined
 * function receives them. */
struct list_scalars {
    const uint32_t *lst;
    const uint8_t *stack_lds, *stack_hbm;
    uint32_t ni, nf;

    template <int E>
    __device__ __forceinline__ void chain(double (&acc)[E], const double (&xd)[E]) const
    {
        for (uint32_t k = 0; k < ni + nf; ++k) {
            const uint32_t sp = uniform(lst[2 * (1 + k)]), off = uniform(lst[2 * (1 + k) + 1]);
            const uint8_t *p = (sp == SPACE_LDS ? stack_lds : stack_hbm) + off;
            const double v = k < ni ? (double)*(const int32_t *)p : *(const double *)p;
            fma_all<E>(v, acc, xd);
        }
    }
};

template <bool ARR, class AP, class SC>
__device__ __forceinline__ double rt_one(const SC &sc, AP arr, uint32_t alen, double xd, uint64_t i)
{
    double acc[1] = {0.0};
    const double x1[1] = {xd};
    if constexpr (ARR) acc[0] = (double)arr[(uint32_t)(i % alen)];
    sc.template chain<1>(acc, x1);
    return acc[0];
}

template <int U, bool ARR, class AP, class SC>
__device__ __forceinline__ void fma_rt_span(const SC &sc, AP arr, uint32_t alen,
                                            const GLB float *__restrict__ x, GLB double *__restrict__ y,
                                            span_t sp, lane_acc &A)
{
    const uint64_t plo = min(sp.hi, (sp.lo + 1) & ~1ull);
    const uint64_t phi = max(plo, sp.hi & ~1ull);
    if (sp.lo < plo && sp.p == 0) {
        const double v = rt_one<ARR>(sc, arr, alen, (double)x[sp.lo], sp.lo);
        y[sp.lo] = v;
        acc_add_f64(A, v);
    }
    lane_acc Ac[2] = {acc_zero(), acc_zero()};
    const GLB f32x2 *__restrict__ x2 = (const GLB f32x2 *)x;
    GLB f64x2 *__restrict__ y2 = (GLB f64x2 *)y;
    const uint64_t nv1 = phi >> 1;
    const uint64_t step = (uint64_t)U * sp.P;
    uint64_t v = (plo >> 1) + sp.p;
    /* array index of element 2v and its advance per pair stride */
    uint32_t j = 0, dj = 0;
    if constexpr (ARR) {
        j = (uint32_t)((2 * v) % alen);
        dj = (uint32_t)((2ull * sp.P) % alen);
    }
    if (v + (uint64_t)(U - 1) * sp.P < nv1) {
        f32x2 cur[U];
        int32_t ca[2 * U];
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = __builtin_nontemporal_load(&x2[v + (uint64_t)u * sp.P]);
        if constexpr (ARR) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                ca[2 * u] = arr[j];
                ca[2 * u + 1] = arr[j + 1 == alen ? 0 : j + 1];
                j = mod_step(j, dj, alen);
            }
        }
        for (;;) {
            const uint64_t vn = v + step;
            const bool more = vn + (uint64_t)(U - 1) * sp.P < nv1;
            f32x2 nxt[U];
            int32_t na[2 * U];
            if (more) {
#pragma unroll
                for (int u = 0; u < U; ++u) nxt[u] = __builtin_nontemporal_load(&x2[vn + (uint64_t)u * sp.P]);
                if constexpr (ARR) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        na[2 * u] = arr[j];
                        na[2 * u + 1] = arr[j + 1 == alen ? 0 : j + 1];
                        j = mod_step(j, dj, alen);
                    }
                }
            }
            double xd[2 * U], acc[2 * U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                xd[2 * u] = (double)cur[u].x;
                xd[2 * u + 1] = (double)cur[u].y;
                acc[2 * u] = ARR ? (double)ca[2 * u] : 0.0;
                acc[2 * u + 1] = ARR ? (double)ca[2 * u + 1] : 0.0;
            }
            sc.template chain<2 * U>(acc, xd);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                f64x2 r;
                r.x = acc[2 * u];
                r.y = acc[2 * u + 1];
                __builtin_nontemporal_store(r, &y2[v + (uint64_t)u * sp.P]);
                acc_add_f64(Ac[0], r.x);
                acc_add_f64(Ac[1], r.y);
            }
            v = vn;
            if (!more) break;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cur[u] = nxt[u];
                if constexpr (ARR) {
                    ca[2 * u] = na[2 * u];
                    ca[2 * u + 1] = na[2 * u + 1];
                }
            }
        }
    }
    for (; v < nv1; v += sp.P) {
        const f32x2 xv = __builtin_nontemporal_load(&x2[v]);
        f64x2 r;
        r.x = rt_one<ARR>(sc, arr, alen, (double)xv.x, 2 * v);
        r.y = rt_one<ARR>(sc, arr, alen, (double)xv.y, 2 * v + 1);
        __builtin_nontemporal_store(r, &y2[v]);
        acc_add_f64(Ac[0], r.x);
        acc_add_f64(Ac[1], r.y);
    }
    if (phi < sp.hi && sp.p == 0) {
        const double r = rt_one<ARR>(sc, arr, alen, (double)x[phi], phi);
        y[phi] = r;
        acc_add_f64(A, r);
    }
    acc_merge(A, Ac[0]);
    acc_merge(A, Ac[1]);
}

template <int U, class AP, class SC>
__device__ __forceinline__ void rt_spans(const SC &sc, AP arr, const dsr_dloop &L, uint32_t alen, span_t sp,
                                         lane_acc &A, uint32_t *claim, uint32_t lane)
{
    const GLB float *x = (const GLB float *)L.in;
    GLB double *y = (GLB double *)L.out;
    const bool balanced = uniform(L.ni + L.nf) >= DSR_BALANCE_MIN;
    if (alen)
        for_spans(L, sp, lane, claim, A, [&](span_t q) { fma_rt_span<U, true>(sc, arr, alen, x, y, q, A); },
                  balanced);
    else
        for_spans(L, sp, lane, claim, A, [&](span_t q) { fma_rt_span<U, false>(sc, arr, alen, x, y, q, A); },
                  balanced);
}

/* Body entry for the run-time chain, frame in LDS (offset `off` in the
 * dynamic LDS) or in HBM (`fb`); the array follows the scalars at the next
 * 16-byte boundary.  U element pairs per lane and batch. */
template <int U>
__device__ __forceinline__ void body_fma_rt(const team_t &T, frame_t f, const dsr_dloop &L, span_t sp,
                                            lane_acc &A, uint32_t *claim, uint32_t lane)
{
    const uint32_t ni = uniform(L.ni), nf = uniform(L.nf), alen = uniform(L.alen);
    const uint32_t aoff = (24 + 8 * nf + 4 * ni + 15) & ~15u;
    if (f.space == SPACE_LDS) {
        const LDSQ uint8_t *fb = (const LDSQ uint8_t *)(dsr_lds + cb_bytes(T.nw) + f.off);
        const lds_scalars sc{(const LDSQ int32_t *)(fb + 24 + 8 * nf), (const LDSQ double *)(fb + 24), ni, nf};
        rt_spans<U>(sc, (const LDSQ int32_t *)(fb + aoff), L, alen, sp, A, claim, lane);
    } else {
        const GLB uint8_t *fb = (const GLB uint8_t *)frame_hbm(T, f);
        double sv = 0.0;
        if (lane < ni) sv = (double)*(const GLB int32_t *)(fb + 24 + 8 * nf + 4 * lane);
        else if (lane < ni + nf) sv = *(const GLB double *)(fb + 24 + 8 * (lane - ni));
        const lane_scalars sc{sv, ni + nf};
        rt_spans<U>(sc, (const GLB int32_t *)(fb + aoff), L, alen, sp, A, claim, lane);
    }
}

/* Shared-array gather; arrays at `arr` (LDS or global pointer), `len`
 * elements each. */
__device__ __forceinline__ i32x4 load4(const LDSQ int32_t *p) { return *(const LDSQ i32x4 *)p; }
__device__ __forceinline__ i32x4 load4(const GLB int32_t *p) { return *(const GLB i32x4 *)p; }

template <int NA, class AP>
__device__ __forceinline__ i32x4 gather4(AP arr, uint32_t len, uint32_t na, uint32_t idx)
{
    i32x4 s = {0, 0, 0, 0};
    if (NA > 0) {
#pragma unroll
        for (int j = 0; j < NA; ++j) s += load4(arr + (uint64_t)j * len + idx);
    } else {
        for (uint32_t j = 0; j < na; ++j) s += load4(arr + (uint64_t)j * len + idx);
    }
    return s;
}

/* Vectors [v0, v1) of 4 elements, visited v0 + k*stride; len % 4 == 0.
 * BATCH4: four vectors at a time (false where registers are scarce). */
template <int NA, class AP, bool BATCH4 = true>
__device__ __forceinline__ void gather_vectors(AP arr, const dsr_dloop &L, uint64_t v0, uint64_t v1,
                                               uint64_t stride)
{
    const uint32_t len = L.len;
    GLB i32x4 *__restrict__ out4 = (GLB i32x4 *)L.out;
    uint32_t idx = (uint32_t)((v0 * 4) % len);
    const uint32_t step = (uint32_t)((stride * 4) % len);
    uint64_t v = v0;
    /* four vectors at a time, their array reads (LDS or global) all in flight */
    for (; BATCH4 && v + 3 * stride < v1; v += 4 * stride) {
        const uint32_t i1 = mod_step(idx, step, len), i2 = mod_step(i1, step, len), i3 = mod_step(i2, step, len);
        i32x4 s[4] = {gather4<NA>(arr, len, L.arrays, idx), gather4<NA>(arr, len, L.arrays, i1),
                      gather4<NA>(arr, len, L.arrays, i2), gather4<NA>(arr, len, L.arrays, i3)};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t w = v + u * stride;
            const uint32_t base = (uint32_t)(w * 4);
            s[u] += i32x4{(int32_t)base, (int32_t)(base + 1), (int32_t)(base + 2), (int32_t)(base + 3)};
            __builtin_nontemporal_store(s[u], &out4[w]);
        }
        idx = mod_step(i3, step, len);
    }
    for (; v < v1; v += stride) {
        i32x4 s = gather4<NA>(arr, len, L.arrays, idx);
        const uint32_t base = (uint32_t)(v * 4);
        s += i32x4{(int32_t)base, (int32_t)(base + 1), (int32_t)(base + 2), (int32_t)(base + 3)};
        __builtin_nontemporal_store(s, &out4[v]);
        idx = mod_step(idx, step, len);
    }
}

template <class AP>
__device__ __forceinline__ void gather_scalar(AP arr, const dsr_dloop &L, uint64_t i0, uint64_t i1,
                                              uint64_t stride)
{
    GLB int32_t *out = (GLB int32_t *)L.out;
    for (uint64_t i = i0; i < i1; i += stride) {
        uint32_t s = (uint32_t)i;
        const uint32_t k = (uint32_t)(i % L.len);
        for (uint32_t j = 0; j < L.arrays; ++j) s += (uint32_t)arr[(uint64_t)j * L.len + k];
        out[i] = (int32_t)s;
    }
}

template <int NA, class AP>
__device__ __forceinline__ void gather_span(AP arr, const dsr_dloop &L, span_t sp)
{
    if ((L.len & 3u) || (sp.lo & 3u)) {
        gather_scalar(arr, L, sp.lo + sp.p, sp.hi, sp.P);
        return;
    }
    const uint64_t nv = (sp.hi - sp.lo) >> 2;
    gather_vectors<NA>(arr, L, (sp.lo >> 2) + sp.p, (sp.lo >> 2) + nv, sp.P);
    gather_scalar(arr, L, sp.lo + 4 * nv + sp.p, sp.hi, sp.P);
}

/* ---- nested levels ----------------------------------------------------------
 * Part k of [lo, hi) cut into `parts` contiguous pieces whose lengths are
 * multiples of `gran` elements (4 keeps every piece on 16-byte vectors). */
__device__ __forceinline__ void split_range(uint64_t lo, uint64_t hi, uint32_t parts, uint32_t k, uint32_t gran,
                                            uint64_t &a, uint64_t &b)
{
    const uint64_t n = hi > lo ? hi - lo : 0;
    uint64_t per = (n + parts - 1) / parts;
    per = (per + gran - 1) / gran * gran;
    a = min(hi, lo + (uint64_t)k * per);
    b = min(hi, a + per);
}

/* The innermost members' loop: elements [a, b) over G lanes (q = this
 * lane's index), on 16-byte vectors when `vec` (a is then a multiple of 4). */
template <int NA, bool BATCH4, class AP>
__device__ __forceinline__ void gather_leaf(AP arr, const dsr_dloop &L, uint64_t a, uint64_t b, uint32_t q,
                                            uint32_t G, bool vec)
{
    if (vec) {
        const uint64_t v1 = b >> 2;
        gather_vectors<NA, AP, BATCH4>(arr, L, (a >> 2) + q, v1, G);
        gather_scalar(arr, L, (v1 << 2) + q, b, G);
    } else {
        gather_scalar(arr, L, a + q, b, G);
    }
}

/* The gather through a reference to the team's frame (space, offset). */
template <int NA, bool BATCH4>
__device__ __forceinline__ void gather_leaf_at(const team_t &T, uint32_t space, uint32_t off, const dsr_dloop &L,
                                               uint64_t a, uint64_t b, uint32_t q, uint32_t G, bool vec)
{
    if (space == SPACE_LDS)
        gather_leaf<NA, BATCH4>((const LDSQ int32_t *)(dsr_lds + cb_bytes(T.nw) + off), L, a, b, q, G, vec);
    else
        gather_leaf<NA, BATCH4>((const GLB int32_t *)(T.stack_hbm + off), L, a, b, q, G, vec);
}

/* A nested fork or join inside one wave: the leader lanes' frame and
 * descriptor writes (LDS, or the global part of a member stack) become
 * visible to the wave's other lanes.  Workgroup scope covers both memories
 * (the wave's own CU). */
__device__ __forceinline__ void nest_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ uint32_t pack_place(frame_t f) { return (f.space << 24) | f.off; }

/* Nested levels below the team's fork (section 3.1.2; section 7's sharing
 * at worker level).  Level 1: this wave is member `member` of `members`
 * and takes its piece of the team's range.  It pushes the frame {lo, hi,
 * team frame's space, offset} on its own member stack, publishes it in its
 * descriptor and forks its inner team, the four 16-lane groups.  Level 2:
 * each group reads the descriptor, then the frame, and takes its piece.  At
 * depth 2 its lanes gather through the team frame the frame names.  At
 * depth 3 each group's leader lane pushes a frame {lo, hi, the wave frame's
 * space, offset} on the group's own member stack and forks the group's
 * inner team, four 4-lane groups, which reach the team frame by following
 * the two references.  Frames are popped in LIFO order after each inner
 * team joins.  A member stack's frame goes to its on-chip part, or to its
 * global part when the on-chip part is full or `nest_global` is set; each
 * global part holds several nested frames, so no nested push fails. */
template <int NA, bool BATCH4>
__device__ __forceinline__ void body_gather_nested(team_t &T, frame_t outer, const dsr_dloop &L, span_t sp,
                                                   uint32_t member, uint32_t members, uint32_t &inner_pushes,
                                                   GLB uint32_t *tr)
{
    static_assert(DSR_NEST_WAVE_HBM >= DSR_NEST_FRAME && DSR_NEST_GROUP_HBM >= DSR_NEST_FRAME,
                  "a global part holds at least one nested frame");
    const uint32_t depth = uniform(L.depth);
    const bool vec = !((L.len & 3u) || (sp.lo & 3u));
    const uint32_t gran = vec ? 4u : 1u;
    const uint32_t lane = T.lane;
    uint32_t *desc = nest_desc(T, member);
    /* level 1: this wave's piece and its frame */
    uint64_t mlo, mhi;
    split_range(sp.lo, sp.hi, members, member, gran, mlo, mhi);
    mstack_t ws = mstack(member * DSR_NEST_WAVE_LDS, DSR_NEST_WAVE_LDS, member * DSR_NEST_WAVE_HBM,
                         DSR_NEST_WAVE_HBM);
    const frame_t f2 = mpush(ws, DSR_NEST_FRAME, T.nest_global != 0);
    uint32_t *p2 = nest_addr(T, f2.space, f2.off);
    if (lane == 0) {
        p2[0] = (uint32_t)mlo;
        p2[1] = (uint32_t)mhi;
        p2[2] = outer.space;
        p2[3] = outer.off;
        desc[0] = f2.space;
        desc[1] = f2.off;
        if (tr) tr[128 + 8 * member] = pack_place(f2);
    }
    inner_pushes += 1;
    nest_sync();
    /* level 2: lane group g reads the published frame */
    const uint32_t g = lane >> 4, l = lane & 15u;
    const uint32_t d2s = desc[0], d2o = desc[1];
    const uint32_t *q2 = nest_addr(T, d2s, d2o);
    const uint32_t vlo = q2[0], vhi = q2[1], osp = q2[2], ooff = q2[3];
    uint64_t glo, ghi;
    split_range(vlo, vhi, DSR_NEST_GROUPS, g, gran, glo, ghi);
    if (depth == 2) {
        gather_leaf_at<NA, BATCH4>(T, osp, ooff, L, glo, ghi, l, 16u, vec);
    } else {
        const uint32_t k = member * DSR_NEST_GROUPS + g;
        mstack_t gs = mstack(members * DSR_NEST_WAVE_LDS + k * DSR_NEST_GROUP_LDS, DSR_NEST_GROUP_LDS,
                             members * DSR_NEST_WAVE_HBM + k * DSR_NEST_GROUP_HBM, DSR_NEST_GROUP_HBM);
        const frame_t f3 = mpush(gs, DSR_NEST_FRAME, T.nest_global != 0);
        uint32_t *p3 = nest_addr(T, f3.space, f3.off);
        if (l == 0) {
            p3[0] = (uint32_t)glo;
            p3[1] = (uint32_t)ghi;
            p3[2] = d2s;
            p3[3] = d2o;
            desc[2 + 2 * g] = f3.space;
            desc[3 + 2 * g] = f3.off;
            if (tr) tr[129 + 8 * member + g] = pack_place(f3);
        }
        inner_pushes += DSR_NEST_GROUPS;
        nest_sync();
        /* level 3: 4-lane group s of group g */
        const uint32_t s = l >> 2, q = l & 3u;
        const uint32_t *q3 = nest_addr(T, desc[2 + 2 * g], desc[3 + 2 * g]);
        const uint32_t slo = q3[0], shi = q3[1];
        const uint32_t *pp = nest_addr(T, q3[2], q3[3]);      /* the wave's frame */
        uint64_t a, b;
        split_range(slo, shi, DSR_NEST_GROUPS, s, gran, a, b);
        gather_leaf_at<NA, BATCH4>(T, pp[2], pp[3], L, a, b, q, 4u, vec);
        nest_sync();                                            /* inner join */
        if (!mpop(gs, f3) && tr) tr[133 + 8 * member] = 1;
    }
    nest_sync();                                                /* inner join */
    if (!mpop(ws, f2) && tr && lane == 0) tr[133 + 8 * member] = 1;
    if (tr && lane == 0) tr[134 + 8 * member] = inner_pushes;
}

/* Cross-team traffic (partials, arrival counters, results) uses
 * device-scope relaxed atomics: on gfx950 these are performed at the
 * device's coherence point, past the per-XCD L2 (which is not coherent
 * across XCDs), so a team's partial needs no L2 write-back (what a
 * device-scope release costs every team).  The hardware assumption this
 * rests on: a team waits for its partial's stores to complete (s_waitcnt)
 * before issuing its arrival atomic, and a store to the coherence point
 * that has completed is seen by any later device-scope read.  The last
 * arriver of a group and of the region takes a device-scope acquire
 * before reading the partials, once per group. */
__device__ __forceinline__ void store_dev(uint64_t *p, uint64_t v)
{
    __hip_atomic_store((GLB uint64_t *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t load_dev(const uint64_t *p)
{
    return __hip_atomic_load((const GLB uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void drain_memory() { __builtin_amdgcn_s_waitcnt(0); }


/* ---- region execution ---------------------------------------------------- */
__device__ __forceinline__ const uint8_t *frame_ptr(const team_t &T, frame_t f)
{
    return f.space == SPACE_LDS ? frame_lds(T, f) : frame_hbm(T, f);
}

/* VARIANT selects which fixed-length fma chains are compiled into the
 * kernel: the worker code is specialised to the bodies a region can
 * publish, so a region of short chains does not pay the register budget
 * of the longest one.  0: chains up to 8+8 scalars (workgroups of up to
 * 512 threads); 1: adds 16+16; 2: adds 32+32; -1 (workgroups above 512
 * threads, 128 registers per lane): run-time chains only.  Other lengths
 * (at most 64 scalars) use the run-time chain, one pair per batch at -1. */
/* Lean instances (VARIANT >= DSR_LEAN_BASE) run single-region launches
 * whose every publish is one fixed fma chain, DSR_LEAN_NI/NF of the
 * variant: the kernel then holds only that body and only the single-region
 * form, so its code and registers are those of the sweep's own path. */
template <int VARIANT>
struct lean_chain {
    static constexpr int k = VARIANT - DSR_LEAN_BASE;
    static constexpr int ni = DSR_LEAN_NI(k), nf = DSR_LEAN_NF(k);
};

template <int VARIANT>
__device__ __forceinline__ void run_body(team_t &T, uint32_t body, frame_t f, const dsr_dloop &L, span_t sp,
                                         lane_acc &A, uint32_t *claim, uint32_t member,
                                         uint32_t members, uint32_t &inner_pushes, GLB uint32_t *tr)
{
    const uint32_t lane = T.lane;
    if constexpr (VARIANT >= DSR_LEAN_BASE) {
        /* the host dispatches only regions made of this chain here */
        /* every scalar stays in registers: reading them once per batch
         * instead (the general instances' run-time chain) measured slower
         * here for every chain length */
        if (body == DSR_BODY_FMA_CHAIN)
            body_fma_fixed<lean_chain<VARIANT>::ni, lean_chain<VARIANT>::nf, false>(T, f, L, sp, A, claim, lane);
        return;
    }
    switch (body) {
    case DSR_BODY_AFFINE_XOR: {
        /* frame layout: [8 B int64 sum][a][b][c][d] */
        const uint32_t a = uniform_u32((const uint8_t *)slot<int32_t>(T, f, 8));
        const uint32_t b = uniform_u32((const uint8_t *)slot<int32_t>(T, f, 12));
        const uint32_t c = uniform_u32((const uint8_t *)slot<int32_t>(T, f, 16));
        const uint32_t d = uniform_u32((const uint8_t *)slot<int32_t>(T, f, 20));
        GLB int32_t *out = (GLB int32_t *)L.out;
        for_spans(L, sp, lane, claim, A, [&](span_t q) { affine_span(a, b, c, d, out, q, A); });
        break;
    }
    case DSR_BODY_FMA_CHAIN: {
        const uint32_t ni = L.ni, nf = L.nf;
        if (VARIANT >= 0 && L.alen == 0) {
            if (ni == 1 && nf == 0) { body_fma_fixed<1, 0>(T, f, L, sp, A, claim, lane); break; }
            if (ni == 1 && nf == 1) { body_fma_fixed<1, 1>(T, f, L, sp, A, claim, lane); break; }
            if (ni == 2 && nf == 2) { body_fma_fixed<2, 2>(T, f, L, sp, A, claim, lane); break; }
            if (ni == 4 && nf == 4) { body_fma_fixed<4, 4>(T, f, L, sp, A, claim, lane); break; }
            if (ni == 8 && nf == 8) { body_fma_fixed<8, 8>(T, f, L, sp, A, claim, lane); break; }
            if constexpr (VARIANT >= 1)
                if (ni == 16 && nf == 16) { body_fma_fixed<16, 16>(T, f, L, sp, A, claim, lane); break; }
            if constexpr (VARIANT >= 2)
                if (ni == 32 && nf == 32) { body_fma_fixed<32, 32>(T, f, L, sp, A, claim, lane); break; }
        }
        /* run-time chain (the host admits at most 64 scalars); workgroups
         * above 512 threads have 128 registers per lane */
        body_fma_rt<VARIANT < 0 ? 1 : DSR_RT_PAIRS>(T, f, L, sp, A, claim, lane);
        break;
    }
    case DSR_BODY_FMA_CHAIN_REFS: {
        /* the wrapper of section 5.1 over a list of references: lane j
         * reads reference 1 + j (scalar j), then the scalar through it; the
         * array's reference is read by every lane */
        const uint32_t ni = uniform(L.ni), nf = uniform(L.nf), alen = uniform(L.alen);
        const uint32_t *lst = f.space == SPACE_LIST ? ref_list(T) : (const uint32_t *)frame_hbm(T, f);
        double sv = 0.0;
        if (lane < ni + nf) {
            const uint32_t sp_ = lst[2 * (1 + lane)], off = lst[2 * (1 + lane) + 1];
            const uint8_t *p = sp_ == SPACE_LDS ? T.stack_lds + off : T.stack_hbm + off;
            sv = lane < ni ? (double)*(const int32_t *)p : *(const double *)p;
        }
        /* with the counts of a compiled fixed chain, run that chain */
        if (VARIANT >= 0 && alen == 0 && !uniform(L.deref)) {
            if (ni == 1 && nf == 0) { lanes_fma_fixed<1, 0>(sv, L, sp, A, claim, lane); break; }
            if (ni == 1 && nf == 1) { lanes_fma_fixed<1, 1>(sv, L, sp, A, claim, lane); break; }
            if (ni == 2 && nf == 2) { lanes_fma_fixed<2, 2>(sv, L, sp, A, claim, lane); break; }
            if (ni == 4 && nf == 4) { lanes_fma_fixed<4, 4>(sv, L, sp, A, claim, lane); break; }
            if (ni == 8 && nf == 8) { lanes_fma_fixed<8, 8>(sv, L, sp, A, claim, lane); break; }
        }
        constexpr int U = VARIANT < 0 ? 1 : DSR_RT_PAIRS;
        if (uniform(L.deref) && alen == 0) {
            const list_scalars ls{lst, T.stack_lds, T.stack_hbm, ni, nf};
            rt_spans<U>(ls, (const GLB int32_t *)nullptr, L, 0, sp, A, claim, lane);
            break;
        }
        const lane_scalars sc{sv, ni + nf};
        if (alen) {
            const uint32_t asp = uniform(lst[2 * (1 + ni + nf)]), aoff = uniform(lst[2 * (1 + ni + nf) + 1]);
            if (asp == SPACE_LDS)
                rt_spans<U>(sc, (const LDSQ int32_t *)(dsr_lds + cb_bytes(T.nw) + aoff), L, alen, sp, A, claim, lane);
            else
                rt_spans<U>(sc, (const GLB int32_t *)(T.stack_hbm + aoff), L, alen, sp, A, claim, lane);
        } else {
            rt_spans<U>(sc, (const GLB int32_t *)nullptr, L, 0, sp, A, claim, lane);
        }
        break;
    }
    case DSR_BODY_GATHER: {
        if (f.space == SPACE_LDS) {
            const LDSQ int32_t *arr = (const LDSQ int32_t *)(dsr_lds + cb_bytes(T.nw) + f.off);
            switch (L.arrays) {
#define GATHER_CASE(NA) for_spans(L, sp, lane, claim, A, [&](span_t q) { gather_span<NA>(arr, L, q); }); break;
            case 1: GATHER_CASE(1)
            case 2: GATHER_CASE(2)
            case 3: GATHER_CASE(3)
            case 4: GATHER_CASE(4)
            default: GATHER_CASE(0)
            }
        } else {
            const GLB int32_t *arr = (const GLB int32_t *)frame_hbm(T, f);
            switch (L.arrays) {
            case 1: GATHER_CASE(1)
            case 2: GATHER_CASE(2)
            case 3: GATHER_CASE(3)
            case 4: GATHER_CASE(4)
            default: GATHER_CASE(0)
#undef GATHER_CASE
            }
        }
        break;
    }
    case DSR_BODY_GATHER_NESTED: {
        switch (L.arrays) {
        case 1: body_gather_nested<1, (VARIANT >= 0)>(T, f, L, sp, member, members, inner_pushes, tr); break;
        case 2: body_gather_nested<2, (VARIANT >= 0)>(T, f, L, sp, member, members, inner_pushes, tr); break;
        case 3: body_gather_nested<3, (VARIANT >= 0)>(T, f, L, sp, member, members, inner_pushes, tr); break;
        case 4: body_gather_nested<4, (VARIANT >= 0)>(T, f, L, sp, member, members, inner_pushes, tr); break;
        default: body_gather_nested<0, (VARIANT >= 0)>(T, f, L, sp, member, members, inner_pushes, tr); break;
        }
        break;
    }
    default:
        break;
    }
}

__device__ __forceinline__ span_t team_span(const dsr_dloop &L, uint32_t team, uint32_t p, uint32_t P)
{
    span_t s;
    s.lo = min(L.dyn_start, (uint64_t)team * L.chunk);
    s.hi = min(L.dyn_start, s.lo + L.chunk);
    s.p = p;
    s.P = P;
    return s;
}

/* Run one participating wave's share of a published body and join. */
template <int VARIANT>
__device__ __forceinline__ void participate(team_t &T, const dsr_dregion &R, const dsr_dconfig &C,
                                            uint32_t team, uint32_t body, frame_t f, uint32_t loop,
                                            const dsr_dloop &L, uint32_t &inner_pushes)
{
    const uint32_t nwork = C.master_joins ? T.nw : T.nw - 1;
    lane_acc A = acc_zero();
    GLB uint32_t *tr = (C.trace && R.trace) ? (GLB uint32_t *)(R.trace + (uint64_t)team * DSR_TRACE_WORDS) : nullptr;
    if (tr && T.lane == 0) tr[96 + 2 * T.wave] = (uint32_t)wall_clock64();
    run_body<VARIANT>(T, body, f, L, team_span(L, team, T.wave * 64 + T.lane, nwork * 64), A,
                      &R.result->claim[loop], T.wave, nwork, inner_pushes, tr);
    if (tr && T.lane == 0) tr[97 + 2 * T.wave] = (uint32_t)wall_clock64();
    /* served form: the request completes while the kernel keeps running,
     * so this wave's output stores must have reached L2 before the join
     * (the master then writes the L2 back before the team arrives) */
    if (VARIANT < DSR_LEAN_BASE && C.serve) drain_memory();
    const i192 w = wave_sum192(widen(A));
    const uint32_t bad = __any(A.bad != 0);
    end_parallel(T, w.w0, w.w1, w.w2, bad);
}

/* Bytes o .. o+3 of src as a little-endian word, zero from `lim` on. */
__device__ __forceinline__ uint32_t ragged_word(const uint8_t *src, uint32_t o, uint32_t lim)
{
    uint32_t w = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q)
        if (o + q < lim) w |= (uint32_t)src[o + q] << (8 * q);
    return w;
}

/* Copy a frame's initial bytes (or zeros) with the whole master wave.  The
 * 16-byte vectors that lie wholly inside the initial bytes go in rounds of
 * eight per lane, all loads of a round in flight together (a 32 KiB frame
 * is four round trips, not thirty-two); the rest is zeros or a ragged
 * edge. */
__device__ __forceinline__ void init_frame(team_t &T, frame_t f, const uint8_t *src, uint32_t init_bytes,
                                           uint32_t nbytes)
{
    uint8_t *dst = (uint8_t *)frame_ptr(T, f);
    const uint32_t nvec = nbytes >> 4;
    const bool src_aligned = (((uintptr_t)src) & 15u) == 0;
    const uint32_t full = src_aligned ? min(init_bytes, nbytes) >> 4 : 0;
    const uint4 *s4 = (const uint4 *)src;
    uint4 *d4 = (uint4 *)dst;
    for (uint32_t k0 = T.lane; k0 < full; k0 += 512) {
        const uint32_t k1 = k0 + 64, k2 = k0 + 128, k3 = k0 + 192, k4 = k0 + 256, k5 = k0 + 320,
                       k6 = k0 + 384, k7 = k0 + 448;
        /* indices past the end reload the last vector (always in bounds);
         * their stores are skipped */
        const uint32_t last = full - 1;
        const uint4 v0 = s4[k0];
        const uint4 v1 = s4[min(k1, last)], v2 = s4[min(k2, last)], v3 = s4[min(k3, last)];
        const uint4 v4 = s4[min(k4, last)], v5 = s4[min(k5, last)], v6 = s4[min(k6, last)];
        const uint4 v7 = s4[min(k7, last)];
        d4[k0] = v0;
        if (k1 < full) d4[k1] = v1;
        if (k2 < full) d4[k2] = v2;
        if (k3 < full) d4[k3] = v3;
        if (k4 < full) d4[k4] = v4;
        if (k5 < full) d4[k5] = v5;
        if (k6 < full) d4[k6] = v6;
        if (k7 < full) d4[k7] = v7;
    }
    for (uint32_t k = full + T.lane; k < nvec; k += 64) {
        const uint32_t o = k * 16;
        d4[k] = make_uint4(ragged_word(src, o, init_bytes), ragged_word(src, o + 4, init_bytes),
                           ragged_word(src, o + 8, init_bytes), ragged_word(src, o + 12, init_bytes));
    }
    for (uint32_t o = nvec * 16 + T.lane; o < nbytes; o += 64) dst[o] = o < init_bytes ? src[o] : 0;
}

/* The region's program, one op per lane of the master wave: all ops are
 * loaded in one round trip when the program starts, and each step takes
 * its op with readlanes, so no op load waits behind the parallel region. */
struct op_lanes {
    uint32_t w[10];
};

__device__ __forceinline__ op_lanes load_ops(const dsr_op *ops, uint32_t n, uint32_t lane)
{
    op_lanes o;
#pragma unroll
    for (int i = 0; i < 10; ++i) o.w[i] = 0;
    if (lane < n) {
        const uint4 *p = (const uint4 *)(ops + lane);
        const uint4 a = p[0], b = p[1], c = p[2];
        o.w[0] = a.x; o.w[1] = a.y; o.w[2] = a.z; o.w[3] = a.w;
        o.w[4] = b.x; o.w[5] = b.y; o.w[6] = b.z; o.w[7] = b.w;
        o.w[8] = c.x; o.w[9] = c.y;
    }
    return o;
}

__device__ __forceinline__ dsr_op op_at(const op_lanes &o, uint32_t k)
{
    dsr_op op;
    op.kind = __builtin_amdgcn_readlane(o.w[0], k);
    op.frame = __builtin_amdgcn_readlane(o.w[1], k);
    op.nbytes = __builtin_amdgcn_readlane(o.w[2], k);
    op.init_bytes = __builtin_amdgcn_readlane(o.w[3], k);
    op.init_stride = __builtin_amdgcn_readlane(o.w[4], k);
    op.body = __builtin_amdgcn_readlane(o.w[5], k);
    op.loop = __builtin_amdgcn_readlane(o.w[6], k);
    op.red = __builtin_amdgcn_readlane(o.w[7], k);
    op.init_off = (uint64_t)__builtin_amdgcn_readlane(o.w[8], k) |
                  ((uint64_t)__builtin_amdgcn_readlane(o.w[9], k) << 32);
    op.pad = 0;
    return op;
}

/* The region descriptor fields the arrival and the combine use, held in
 * registers: read once before the arrival atomics, so no fence between
 * them makes the last team reload the descriptor from memory. */
struct region_sums {
    uint64_t *partials;
    dsr_dresult *result;
    uint32_t teams, n_red, red_kind_mask;
};

__device__ __forceinline__ region_sums sums_of(const dsr_dregion &R)
{
    region_sums S;
    S.partials = R.partials;
    S.result = R.result;
    S.teams = uniform(R.teams);
    S.n_red = uniform(R.n_red);
    S.red_kind_mask = uniform(R.red_kind_mask);
    return S;
}

/* Master wave: this team's partial of one reduction (lane 0 stores). */
__device__ __forceinline__ void store_partial(uint64_t *pp, i192 sv, uint32_t lane)
{
    if (lane == 0) {
        store_dev(pp, sv.w0);
        store_dev(pp + 1, sv.w1);
        store_dev(pp + 2, sv.w2);
    }
}

/* Master wave: add the join's total into the shared sum at c (an int64
 * for the integer body, else a 192-bit integer in 2^-75 units) and return
 * the new value as 192 bits. */
template <class P>
__device__ __forceinline__ i192 update_sum(P c, i192 tot, bool integer_sum, uint32_t lane)
{
    i192 sv;
    if (integer_sum) {
        const int64_t nv = (int64_t)(c[0] + tot.w0);
        sv = i192{(uint64_t)nv, (uint64_t)(nv >> 63), (uint64_t)(nv >> 63)};
        wave_sync();
        if (lane == 0) c[0] = (uint64_t)nv;
    } else {
        sv = add192(tot, i192{c[0], c[1], c[2]});
        wave_sync();
        if (lane == 0) {
            c[0] = sv.w0;
            c[1] = sv.w1;
            c[2] = sv.w2;
        }
    }
    return sv;
}

/* Master wave: the sequential code block of one region for one team
 * (Figure 2): pushes, publishes and pops.  Returns the team's error. */
template <int VARIANT>
__device__ __forceinline__ int32_t run_program(team_t &T, const dsr_dregion &R, const dsr_dconfig &C,
                                               const dsr_dlaunch &LP, bool single, uint32_t region,
                                               uint32_t team, uint32_t &barriers, uint32_t &inner_pushes)
{
    cb_header *h = header(T);
    /* trace words go through a global-space pointer: a generic store is
     * counted with the LDS accesses too, and the next LDS wait would wait
     * for the stamp to reach memory */
    GLB uint32_t *tr = (C.trace && R.trace) ? (GLB uint32_t *)(R.trace + (uint64_t)team * DSR_TRACE_WORDS) : nullptr;
    if (tr && T.lane == 0) tr[86] = (uint32_t)wall_clock64();
    wave_sync();
    int32_t err = 0;
    uint32_t npush = 0;
    bool stamped = false;
    const uint32_t nwork = C.master_joins ? T.nw : T.nw - 1;
    const uint32_t n_ops = min(uniform(R.n_ops), (uint32_t)DSR_MAX_OPS);
    /* read once, before any join: after a barrier the compiler would load
     * them from memory again, behind this wave's outstanding stores */
    const region_sums RS = sums_of(R);
    /* a short program of a single-region launch, its first loop and its
     * first frame's image come with the kernel arguments; the image is read
     * into registers (16 bytes a lane) before anything else */
    const bool inl = VARIANT >= DSR_LEAN_BASE && single && LP.inl_ops == n_ops && n_ops > 0;
    i32x4 img = {0, 0, 0, 0};
    if (inl && LP.inl_img && 16u * T.lane < LP.inl_img) img = *(const i32x4 *)(LP.inl_image + 16u * T.lane);
    /* the 1024-thread instance has no registers to spare: it reads each op
     * when it gets to it */
    const op_lanes prog = load_ops(R.ops, (VARIANT < 0 || inl) ? 0 : n_ops, T.lane);
    for (uint32_t k = 0; k < n_ops; ++k) {
        const dsr_op op = inl ? LP.inl_op[k] : (VARIANT < 0 ? R.ops[k] : op_at(prog, k));
        if (op.kind == DSR_OP_PUSH) {
            const frame_t f = push(T, op.nbytes);
            if (f.space == SPACE_NONE) { err = DSR_E_NOMEM; break; }
            if (tr && T.lane == 0 && npush < 16) {
                tr[1 + 3 * npush] = f.space;
                tr[2 + 3 * npush] = f.off;
                tr[3 + 3 * npush] = f.size;
            }
            npush++;
            if (k == 0 && inl && LP.inl_img && f.size <= 16u * 64u) {
                /* the image (zero-padded to a multiple of 16 bytes) from
                 * registers, zeros after it */
                if (16u * T.lane < f.size) {
                    if (f.space == SPACE_LDS)
                        *(LDSQ i32x4 *)(dsr_lds + cb_bytes(T.nw) + f.off + 16u * T.lane) = img;
                    else
                        *(GLB i32x4 *)(T.stack_hbm + f.off + 16u * T.lane) = img;
                }
                wave_sync();
            } else {
                init_frame(T, f, R.init + op.init_off + (uint64_t)team * op.init_stride, op.init_bytes,
                           op.nbytes);
            }
        } else if (op.kind == DSR_OP_PUBLISH) {
            frame_t f, lf{SPACE_NONE, 0, 0};
            if (VARIANT < DSR_LEAN_BASE && op.body == DSR_BODY_FMA_CHAIN_REFS) {
                /* section 5.2: resolve each (frame, offset) reference to a
                 * stack address and write the list on chip, or to a list
                 * frame on the HBM stack when it is longer than the on-chip
                 * list (or global lists are asked for) */
                const uint32_t n = op.nbytes;
                const uint32_t *tab = (const uint32_t *)(R.init + op.init_off);
                const bool glist = n > DSR_REF_LIST || C.global_lists;
                uint32_t *dst = ref_list(T);
                if (glist) {
                    lf = push(T, 8 * n, true);
                    if (lf.space == SPACE_NONE) { err = DSR_E_NOMEM; break; }
                    dst = (uint32_t *)frame_hbm(T, lf);
                    f = frame_t{SPACE_HBM, lf.off, n};
                } else {
                    f = frame_t{SPACE_LIST, 0, n};
                }
                for (uint32_t k = T.lane; k < n; k += 64) {
                    const uint32_t *fte = frame_table(T) + 4 * tab[2 * k];
                    dst[2 * k] = fte[0];
                    dst[2 * k + 1] = fte[1] + tab[2 * k + 1];
                }
                if (tr && T.lane == 0) {
                    tr[89] = glist ? SPACE_HBM : SPACE_LIST;
                    tr[90] = f.off;
                    tr[91] = n;
                }
            } else {
                const uint32_t *ft = frame_table(T) + 4 * op.frame;
                f.space = uniform(ft[0]);
                f.off = uniform(ft[1]);
                f.size = uniform(ft[2]);
            }
            if (T.lane == 0) {
                h->region = region;
                h->team = team;
            }
            publish(T, f, op.body, op.loop);
            barriers++;
            if (tr && T.lane == 0 && !stamped) {
                const uint64_t t0 = wall_clock64();
                tr[82] = (uint32_t)t0;
                tr[83] = (uint32_t)(t0 >> 32);
            }
            stamped = true;
            /* the 1024-thread instance has no registers for a participating
             * master; the host never asks it to (teams above 512 threads) */
            if (VARIANT >= 0 && C.master_joins) {
                participate<VARIANT>(T, R, C, team, op.body, f, op.loop,
                                     (inl && LP.inl_loop && op.loop == 0) ? LP.inl_loop0 : R.loops[op.loop],
                                     inner_pushes);
            } else {
                end_parallel(T, 0, 0, 0, 0);
            }
            barriers++;
            if (tr && T.lane == 0) {
                const uint64_t t1 = wall_clock64();
                tr[84] = (uint32_t)t1;
                tr[85] = (uint32_t)(t1 >> 32);
            }
            /* join done: combine the participating waves' partials */
            i192 tot{0, 0, 0};
            for (uint32_t w = 0; w < T.nw; ++w) {
                if (w == T.nw - 1 && !C.master_joins) continue;
                const uint64_t *r = red_slot(T, w);
                tot = add192(tot, i192{r[0], r[1], r[2]});
            }
            const uint32_t bad = uniform(h->bad);
            if (bad) { err = DSR_E_RANGE; }
            wave_sync();
            if (T.lane == 0) h->bad = 0;
            if (op.red != 0xffffffffu) {
                /* the shared sum: the frame's first bytes, or where reference
                 * 0 of the list points; read and written through a pointer
                 * of its own memory space (a generic access would also wait
                 * for this wave's outstanding loop stores) */
                uint32_t s_space = f.space, s_off = f.off;
                if (VARIANT < DSR_LEAN_BASE && op.body == DSR_BODY_FMA_CHAIN_REFS) {
                    const uint32_t *lst = f.space == SPACE_LIST ? ref_list(T) : (const uint32_t *)frame_hbm(T, f);
                    s_space = uniform(lst[0]);
                    s_off = uniform(lst[1]);
                }
                const bool integer_sum = op.body == DSR_BODY_AFFINE_XOR;
                /* the team's partial is stored inside each branch: where the
                 * two would merge the compiler waits for every outstanding
                 * memory operation of the wave, its loop stores included */
                uint64_t *pp = RS.partials + ((uint64_t)op.red * RS.teams + team) * DSR_PART_WORDS;
                if (s_space == SPACE_LDS)
                    store_partial(pp, update_sum((LDSQ uint64_t *)(dsr_lds + cb_bytes(T.nw) + s_off), tot,
                                                 integer_sum, T.lane), T.lane);
                else
                    store_partial(pp, update_sum((GLB uint64_t *)(T.stack_hbm + s_off), tot, integer_sum, T.lane),
                                  T.lane);
            }
            wave_sync();
            /* a global reference list dies with its parallel region */
            if (lf.space == SPACE_HBM && !pop(T, lf)) err = DSR_E_ORDER;
            if (err) break;
        } else if (op.kind == DSR_OP_POP) {
            const uint32_t nf = uniform(h->nframes);
            if (nf == 0) { err = DSR_E_UNDERFLOW; break; }
            const uint32_t *ft = frame_table(T) + 4 * (nf - 1);
            frame_t f;
            f.space = uniform(ft[0]);
            f.off = uniform(ft[1]);
            f.size = uniform(ft[2]);
            if (!pop(T, f)) { err = DSR_E_ORDER; break; }
        }
    }
    (void)nwork;
    if (tr && T.lane == 0) {
        tr[0] = npush;
        tr[81] = (uint32_t)err;
    }
    if (err && T.lane == 0) atomicCAS(&R.result->error, 0, err);
    return err;
}

/* Sum `cnt` 192-bit partials (three words each, `stride` partials apart)
 * with the whole wave: each lane issues up to eight independent loads per
 * round, so up to 512 partials cost one memory round trip. */
__device__ __forceinline__ i192 sum_partials(const uint64_t *base, uint32_t cnt, uint32_t stride, uint32_t lane)
{
    i192 s{0, 0, 0};
    for (uint32_t j0 = 0; j0 < cnt; j0 += 512) {
        uint64_t w[8][3];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t j = j0 + 64u * u + lane;
            const uint64_t *pp = base + (uint64_t)DSR_PART_WORDS * j * stride;
            const bool in = j < cnt;
            w[u][0] = in ? load_dev(pp) : 0;
            w[u][1] = in ? load_dev(pp + 1) : 0;
            w[u][2] = in ? load_dev(pp + 2) : 0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s = add192(s, i192{w[u][0], w[u][1], w[u][2]});
    }
    return wave_sum192(s);
}

/* Last team: the region's reductions from the (group) partials, exact in
 * 192-bit integers, rounded once for fp64. */
__device__ __forceinline__ void combine_teams(const region_sums &R, uint32_t cnt, uint32_t stride, uint32_t lane,
                                              dsr_drec *rec)
{
    for (uint32_t r = 0; r < R.n_red; ++r) {
        const i192 s = sum_partials(R.partials + (uint64_t)r * R.teams * DSR_PART_WORDS, cnt, stride, lane);
        if (lane == 0) {
            GLB dsr_dresult *res = (GLB dsr_dresult *)R.result;
            const double f = ((R.red_kind_mask >> r) & 1u) ? fixed_to_double(s) : (double)(int64_t)s.w0;
            res->fixed[r][0] = s.w0;
            res->fixed[r][1] = s.w1;
            res->fixed[r][2] = s.w2;
            res->i64[r] = (int64_t)s.w0;
            res->f64[r] = f;
            /* served form: the completion record gets the same values
             * directly, not read back from the result block */
            if (rec && r < DSR_MAX_RED) {
                rec->fixed[r][0] = s.w0;
                rec->fixed[r][1] = s.w1;
                rec->fixed[r][2] = s.w2;
                rec->i64[r] = (int64_t)s.w0;
                rec->f64[r] = f;
            }
        }
    }
}

/* Served form: finish a region's host-coherent completion record (its
 * sums are already there) and release the ticket; the system-scope release
 * also writes this XCD's L2 back, outputs included. */
__device__ __forceinline__ void publish_record(const dsr_dregion &R, dsr_drec *rec, int32_t err, uint32_t lane)
{
    if (lane != 0) return;
    rec->status = err;
    rec->n_red = R.n_red;
    rec->ticks = wall_clock64();
    __hip_atomic_store(&rec->seq, R.tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

/* A team's arrival after its program.  Arrivals go through a two-level
 * tree (groups of teams, then groups) so that no counter sees more than a
 * few dozen simultaneous atomics.  With up to 512 teams the last team
 * reads every partial in one round; with more, the last team of each group
 * first adds up its group's partials and leaves the sum in the group's
 * first partial slot, and the last team overall adds the group sums. */
__device__ __forceinline__ void finish_team(const dsr_dregion &RD, uint32_t team, uint32_t lane,
                                            uint64_t *done_ts, dsr_drec *rec = nullptr, GLB uint32_t *tr = nullptr)
{
    const region_sums R = sums_of(RD);
    const uint32_t gsize = R.teams <= DSR_FLAT_TEAMS ? R.teams : (R.teams + DSR_ARRIVE_GROUPS - 1) / DSR_ARRIVE_GROUPS;
    const uint32_t ngroups = (R.teams + gsize - 1) / gsize;
    const uint32_t g = team / gsize;
    const uint32_t in_group = min(gsize, R.teams - g * gsize);
    const bool group_sums = R.teams > 512;
    drain_memory();                      /* this team's partials are stored */
    if (tr && lane == 0) tr[92] = (uint32_t)wall_clock64();
    GLB dsr_dresult *res = (GLB dsr_dresult *)R.result;
    uint32_t prev = 0;
    /* a region of one team has nothing to arrive at: this wave wrote every
     * partial and the error word itself */
    if (R.teams > 1) {
        if (lane == 0)
            prev = __hip_atomic_fetch_add(&res->group[g * 16], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        prev = uniform((uint32_t)__shfl((int)prev, 0, 64));
        if (tr && lane == 0) tr[93] = (uint32_t)wall_clock64();
        if (prev != in_group - 1) return;
        /* the last arriver of a group reads the others' partials: acquire */
        if (DSR_ARRIVE_FENCE) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (lane == 0) __hip_atomic_store(&res->group[g * 16], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (tr && lane == 0) {
        tr[93] = (uint32_t)wall_clock64();
    }
    if (ngroups > 1) {
        if (group_sums) {
            for (uint32_t r = 0; r < R.n_red; ++r) {
                uint64_t *gp = R.partials + ((uint64_t)r * R.teams + (uint64_t)g * gsize) * DSR_PART_WORDS;
                const i192 s = sum_partials(gp, in_group, 1, lane);
                if (lane == 0) {
                    store_dev(gp, s.w0);
                    store_dev(gp + 1, s.w1);
                    store_dev(gp + 2, s.w2);
                }
            }
            drain_memory();              /* the group sums are stored */
        }
        if (lane == 0)
            prev = __hip_atomic_fetch_add(&res->arrived, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        prev = uniform((uint32_t)__shfl((int)prev, 0, 64));
        if (prev != ngroups - 1) return;
        if (DSR_ARRIVE_FENCE) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (lane == 0) __hip_atomic_store(&res->arrived, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tr && lane == 0) tr[94] = (uint32_t)wall_clock64();
    /* the error word, the partials and the counters are read and reset in
     * one round trip: nothing below waits on anything but the loads */
    int32_t err = 0;
    if (lane == 0) err = __hip_atomic_exchange(&res->error, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lane < DSR_MAX_LOOPS) __hip_atomic_store(&res->claim[lane], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ngroups > 1 && group_sums) combine_teams(R, ngroups, gsize, lane, rec);
    else combine_teams(R, R.teams, 1, lane, rec);
    if (lane == 0) {
        res->final_error = err;
        __hip_atomic_fetch_add(&res->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done_ts) *done_ts = wall_clock64();
        if (tr) tr[95] = (uint32_t)wall_clock64();
    }
    if (rec) publish_record(RD, rec, err, lane);
}

/* Served form: close the server (one workgroup does it; see wait_item).
 * The device announces the close in host memory, then reads the host's
 * published count once more: the host publishes, then reads the closing
 * flag, so at least one side sees the other's write (both orders are
 * sequentially consistent at system scope, and a read from the device to
 * host memory does not pass the device's earlier write to it).  Every item
 * below the count read here is served; none above it is.  The count is
 * returned to the host, which takes back a request it published too late. */
__device__ __forceinline__ void close_server(const dsr_dlaunch &LP, uint32_t reason, uint32_t it, uint32_t pub,
                                             uint64_t idle)
{
    uint32_t *ctr = LP.counter;
    uint32_t open = 0;
    if (!__hip_atomic_compare_exchange_strong(ctr + DSR_SRV_STATE, &open, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT))
        return;
    /* why, for the host's status: the reason (1 stop, 2 idle), the closing
     * workgroup, the item it waited for, the published count it saw and
     * the idle ticks it measured */
    uint32_t *why = LP.closing + 1;
    __hip_atomic_store(why, reason, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(why + 1, (uint32_t)blockIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(why + 2, it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(why + 3, pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(why + 4, (uint32_t)idle, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(why + 5, (uint32_t)(idle >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(LP.closing, 1u, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_SYSTEM);
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
    const uint32_t h = __hip_atomic_load(LP.published, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_fetch_max(ctr + DSR_SRV_PUB, h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(ctr + DSR_SRV_FINAL, h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(LP.final_items, h + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(ctr + DSR_SRV_STATE, 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

/* Served form: wait until item `it` is published (true: run it) or the
 * server has closed below it (false: leave).
 *
 * The host's published count lives in host memory, so polling it crosses
 * the host link; only the DSR_HOST_POLLERS workgroups holding the next
 * unpublished items poll the host, and they mirror what they see into
 * device memory, where every other waiting workgroup polls.  Polls are
 * relaxed (an acquire per poll would invalidate the L2 each time) and back
 * off with sleeps; once the item is seen, one agent-scope acquire makes
 * the request's device-memory inputs visible.
 *
 * Closing is one decision for the whole server, never a workgroup's own:
 * it happens when the host asks to stop, or when a waiting workgroup has
 * seen the device copy of the published count stay unchanged for
 * idle_limit ticks of its own clock.  The server then serves every item published before
 * the close and no other, so a workgroup leaves only while holding an
 * item nobody will publish to it, and no claimed item is lost.  Nothing
 * here waits for another workgroup, so the server does not rely on its
 * whole grid being resident at once. */
#define DSR_HOST_POLLERS 16u

__device__ __forceinline__ bool wait_item(const dsr_dlaunch &LP, uint32_t it, uint32_t lane, uint64_t &item)
{
    uint32_t ok = 0;
    const uint64_t *ring = (const uint64_t *)LP.items;
    if (lane == 0) {
        uint32_t *ctr = LP.counter;
        uint32_t nap = 0;
        /* idleness is timed on this wave's own clock from the last change
         * of the published count it saw: clocks of different workgroups
         * (other XCDs) are never compared */
        uint32_t seen = __hip_atomic_load(ctr + DSR_SRV_PUB, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint64_t seen_at = (uint64_t)wall_clock64();
        for (;;) {
            const uint32_t pub = __hip_atomic_load(ctr + DSR_SRV_PUB, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (it < pub) { ok = 1; break; }
            if (pub != seen) {
                seen = pub;
                seen_at = (uint64_t)wall_clock64();
            }
            const uint32_t st = __hip_atomic_load(ctr + DSR_SRV_STATE, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            if (st == 2) {
                /* closed: items below the final count were made visible
                 * through the published copy above; this one is beyond it */
                if (it >= __hip_atomic_load(ctr + DSR_SRV_FINAL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                continue;
            }
            if (st == 0) {
                if (it - pub < DSR_HOST_POLLERS) {
                    /* the workgroups holding the next items read the host's
                     * count themselves (a later team of a request need not
                     * wait for the device copy); the item is read in the same
                     * round, and its sequence field tells whether it is
                     * already this one */
                    const uint32_t h = __hip_atomic_load(LP.published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    item = __hip_atomic_load(ring + (it & LP.ring_mask), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    /* taken only while the server is still open: once a
                     * close has begun, items count as published up to the
                     * close's final count alone, which the closed branch
                     * above hands out */
                    if ((int32_t)(h - it) > 0 &&
                        __hip_atomic_load(ctr + DSR_SRV_STATE, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                        __hip_atomic_fetch_max(ctr + DSR_SRV_PUB, h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 1;
                        break;
                    }
                    if (it == pub && __hip_atomic_load(LP.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
                        close_server(LP, 1u, it, pub, 0);
                        continue;
                    }
                    nap = 0;
                }
                const uint64_t idle = (uint64_t)wall_clock64() - seen_at;
                if (idle > LP.idle_limit) {
                    close_server(LP, 2u, it, pub, idle);
                    continue;
                }
            }
            /* s_sleep takes an immediate (64 * n clocks); workgroups whose
             * item is far from the next one published sleep longest */
            if (it - pub >= 64) {
                __builtin_amdgcn_s_sleep(127);
                __builtin_amdgcn_s_sleep(127);
                __builtin_amdgcn_s_sleep(127);
                __builtin_amdgcn_s_sleep(127);
            } else {
                switch (nap) {
                case 0: __builtin_amdgcn_s_sleep(1); break;
                case 1: __builtin_amdgcn_s_sleep(2); break;
                case 2: __builtin_amdgcn_s_sleep(4); break;
                case 3: __builtin_amdgcn_s_sleep(8); break;
                case 4: __builtin_amdgcn_s_sleep(16); break;
                default: __builtin_amdgcn_s_sleep(32); break;
                }
                if (nap < 5) ++nap;
            }
        }
    }
    ok = __shfl((int)ok, 0, 64);
    if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (ok && lane == 0) {
        /* published before the count that was seen: a word still holding an
         * older sequence is read again (bounded, so a broken ring cannot
         * hold the workgroup) */
        for (uint32_t k = 0; (uint32_t)(item >> 32) != it && k < (1u << 22); ++k)
            item = __hip_atomic_load(ring + (it & LP.ring_mask), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    return ok != 0;
}

/* Served form: the request slot's descriptor, program and loop
 * descriptors live in host memory that the host rewrites between
 * requests; the master copies them into LDS with system-scope loads (never
 * through the scalar cache, which is not kept coherent with the host) and
 * points the copy's ops/loops at the LDS copies. */
__device__ __forceinline__ dsr_dregion *serve_area(const team_t &T)
{
    return (dsr_dregion *)(T.stack_lds + T.lds_cap);
}

/* Served form, large images: team 0 of the request copies the init blob
 * from the host slot into the slot's device buffer, and the other teams
 * wait for it there instead of each reading the whole blob across the
 * host link (64 teams of a 32 KiB image would move 2 MiB over it).  The
 * flag holds the ticket whose images the buffer holds; tickets are unique,
 * so it is never cleared.  A team that does not see its ticket within the
 * spin bound reads the host slot, which is always correct. */
__device__ __forceinline__ bool relay_images(const dsr_dregion *Rl, uint32_t team, uint32_t lane,
                                             uint32_t *count)
{
    GLB uint8_t *dst = (GLB uint8_t *)Rl->relay;
    GLB uint64_t *flag = (GLB uint64_t *)Rl->relay_flag;
    const uint64_t tag = Rl->tag;
    if (team == 0) {
        /* the slot is padded past the blob to a multiple of 256 bytes */
        const uint32_t nv = (Rl->init_size + 15u) >> 4;
        const i32x4 *src = (const i32x4 *)Rl->init;
        GLB i32x4 *d4 = (GLB i32x4 *)dst;
        for (uint32_t k0 = lane; k0 < nv; k0 += 512) {
            i32x4 v[8];
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) {
                const uint32_t k = k0 + 64u * u;
                v[u] = src[min(k, nv - 1)];
            }
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u)
                if (k0 + 64u * u < nv) d4[k0 + 64u * u] = v[u];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) {
            __hip_atomic_store(flag, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (count) __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return true;
    }
    uint32_t seen = 0;
    if (lane == 0) {
        for (uint32_t spin = 0; spin < (1u << 20); ++spin) {
            if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == tag) {
                seen = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (!seen && count) __hip_atomic_fetch_add(count + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    return __shfl((int)seen, 0, 64) != 0;
}

__device__ __forceinline__ const dsr_dregion &stage_request(team_t &T, const uint8_t *slot, uint32_t team,
                                                           uint32_t *relays)
{
    /* the slot's head has the layout of this LDS area: one round of loads
     * brings the descriptor, the ops and the loop descriptors together */
    dsr_dregion *Rl = serve_area(T);
    uint8_t *ops_l = (uint8_t *)Rl + DSR_SERVE_OPS_AT;
    uint8_t *loops_l = (uint8_t *)Rl + DSR_SERVE_LOOPS_AT;
    {
        /* every load issued before any store: one host round trip for the
         * head and the first DSR_SERVE_IMG_LDS bytes of the frame images */
        constexpr uint32_t NW = DSR_SERVE_AREA_BYTES / 8, PER = (NW + 63) / 64;
        const uint64_t *src = (const uint64_t *)slot;
        uint64_t *dst = (uint64_t *)Rl;
        uint64_t v[PER];
#pragma unroll
        for (uint32_t r = 0; r < PER; ++r) {
            const uint32_t k = T.lane + 64u * r;
            v[r] = k < NW ? __hip_atomic_load(src + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0ull;
        }
#pragma unroll
        for (uint32_t r = 0; r < PER; ++r) {
            const uint32_t k = T.lane + 64u * r;
            if (k < NW) dst[k] = v[r];
        }
    }
    wave_sync();
    const uint32_t n_ops = min(uniform(Rl->n_ops), (uint32_t)DSR_SERVE_MAX_OPS);
    const bool img_here = uniform(Rl->init_size) <= DSR_SERVE_IMG_LDS;
    /* (the host asks for a relay only for blobs larger than the LDS copy) */
    const bool relayed = !img_here && Rl->relay != nullptr && relay_images(Rl, team, T.lane, relays);
    /* the relayed bytes are read with plain loads below: acquire */
    if (relayed) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    wave_sync();
    if (T.lane == 0) {
        Rl->ops = (const dsr_op *)ops_l;
        Rl->loops = (const dsr_dloop *)loops_l;
        Rl->n_ops = n_ops;
        if (img_here) Rl->init = (const uint8_t *)Rl + DSR_SERVE_SLOT_HEAD;
        if (relayed) Rl->init = Rl->relay;
    }
    wave_sync();
    return *Rl;
}

/* One kernel for both launch forms.  The master wave runs region programs
 * (one per workgroup for a single region; claimed items for a batch) and
 * then terminates the workers; worker waves sit in the await loop and take
 * the region and team of each published body from the control block. */
template <int MAXWG, int VARIANT>
__global__ __launch_bounds__(MAXWG) void dsr_region_kernel(dsr_dlaunch LP, dsr_dconfig C)
{
    team_t T = team_init(dsr_lds, C.nw, C.lds_cap, C.threshold,
                         C.hbm_base + (uint64_t)blockIdx.x * C.hbm_slot_bytes, (uint32_t)C.hbm_slot_bytes);
    T.nest_hbm = C.nest_base + (uint64_t)blockIdx.x * DSR_NEST_SLOT;
    T.nest_global = C.nest_global;
    constexpr bool lean = VARIANT >= DSR_LEAN_BASE;
    const bool single = lean || LP.items == nullptr;
    uint32_t barriers = 0, inner_pushes = 0;
    if (!lean && LP.published && T.wave == C.nw - 1 && T.lane == 0) {
        const uint64_t now = wall_clock64();
        if (blockIdx.x == 0 && LP.done_ts)
            __hip_atomic_store(LP.done_ts, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(LP.wg_started + blockIdx.x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (LP.start_ts && blockIdx.x == 0 && T.wave == C.nw - 1 && T.lane == 0) *LP.start_ts = wall_clock64();
    if (T.wave == C.nw - 1) {
        for (uint32_t round = 0;; ++round) {
            uint32_t region, team;
            if (single) {
                if (round) break;
                region = 0;
                team = blockIdx.x;
            } else {
                uint32_t it = 0;
                if (T.lane == 0) it = atomicAdd(&LP.counter[DSR_SRV_CLAIM], 1u);
                it = uniform((uint32_t)__shfl((int)it, 0, 64));
                if (LP.published) {
                    /* served form: wait until the host has published item
                     * `it`; leave once the server has closed below it */
                    uint64_t item = 0;
                    if (!wait_item(LP, it, T.lane, item)) break;
                    const uint64_t w = (uint64_t)__shfl((long long)item, 0, 64);
                    region = uniform((uint32_t)(w >> 16) & 0xffffu);
                    team = uniform((uint32_t)w & 0xffffu);
                } else {
                    if (it >= LP.n_items) break;
                    if (it == 0 && LP.done_ts && T.lane == 0) LP.done_ts[LP.n_regions] = wall_clock64();
                    region = uniform(LP.items[2 * it]);
                    team = uniform(LP.items[2 * it + 1]);
                }
                team_reset(T);
            }
            const dsr_dregion &R = (!lean && C.serve)
                                       ? stage_request(T, (const uint8_t *)LP.regions + (uint64_t)region * LP.region_stride, team,
                                                   LP.relays)
                                                        : ((lean && LP.has_single) ? LP.single : LP.regions[region]);
            run_program<VARIANT>(T, R, C, LP, single, region, team, barriers, inner_pushes);
            GLB uint32_t *tr = (single && C.trace && R.trace) ? (GLB uint32_t *)(R.trace + (uint64_t)team * DSR_TRACE_WORDS) : nullptr;
            if (tr && T.lane == 0) tr[87] = (uint32_t)wall_clock64();
            /* outputs out of L2 before the arrival; a request of one team
             * has its completion record's system-scope release do it */
            if (!lean && C.serve && R.teams > 1) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            /* the 1024-thread instance reads fewer partials per round */
            finish_team(R, team, T.lane, (LP.done_ts && !LP.published) ? LP.done_ts + region : nullptr,
                        (!lean && LP.recs) ? LP.recs + region : nullptr, tr);
            if (tr && T.lane == 0) tr[88] = (uint32_t)wall_clock64();
        }
        if (!lean && LP.wg_exited && T.lane == 0)
            __hip_atomic_store(LP.wg_exited + blockIdx.x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        /* terminate the workers (Figure 3's terminate branch) */
        frame_t none{SPACE_NONE, 0, 0};
        publish(T, none, DSR_BODY_TERMINATE, 0);
        barriers++;
        if (!single && !LP.published && T.lane == 0) {
            if (__hip_atomic_fetch_add(&LP.counter[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                gridDim.x - 1) {
                __hip_atomic_store(&LP.counter[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&LP.counter[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    } else {
        for (;;) {
            uint32_t body, loop;
            frame_t f;
            const bool go = await(T, &body, &f, &loop);
            barriers++;
            if (!go) break;
            const uint32_t region = uniform(header(T)->region), team = uniform(header(T)->team);
            const dsr_dregion &R = (!lean && C.serve) ? *serve_area(T)
                                                      : ((lean && LP.has_single) ? LP.single : LP.regions[region]);
            participate<VARIANT>(T, R, C, team, body, f, loop,
                                 (lean && LP.inl_loop && loop == 0) ? LP.inl_loop0 : R.loops[loop], inner_pushes);
            barriers++;
        }
    }
    if (single && C.trace && LP.regions[0].trace && T.lane == 0) {
        GLB uint32_t *tr = (GLB uint32_t *)(LP.regions[0].trace + (uint64_t)blockIdx.x * DSR_TRACE_WORDS);
        tr[49 + T.wave] = barriers;
        tr[65 + T.wave] = inner_pushes;
    }
}

/* ---- this object's instance --------------------------------------------
 * The build compiles this file once per kernel instance, in parallel, with
 * DSR_INST_MAXWG, DSR_INST_VARIANT and DSR_INST_TAG defined; each object
 * exports its instance's launcher, occupancy and register queries under
 * names carrying the tag, and dsr_dispatch.cpp picks among them. */
#if !defined(DSR_INST_MAXWG) || !defined(DSR_INST_VARIANT) || !defined(DSR_INST_TAG)
#error "compile with -DDSR_INST_MAXWG=<threads> -DDSR_INST_VARIANT=<v> -DDSR_INST_TAG=<tag>"
#endif
#define DSR_INST_CAT2(a, b) a##b
#define DSR_INST_CAT(a, b) DSR_INST_CAT2(a, b)
#define DSR_INST_KERNEL dsr_region_kernel<DSR_INST_MAXWG, DSR_INST_VARIANT>

extern "C" int DSR_INST_CAT(dsr_inst_launch_, DSR_INST_TAG)(const dsr_dlaunch *lp, const dsr_dconfig *cfg,
                                                            uint32_t grid, uint32_t wg_size, uint32_t lds_bytes,
                                                            void *stream)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)DSR_INST_KERNEL, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL(DSR_INST_KERNEL, dim3(grid), dim3(wg_size), lds_bytes, (hipStream_t)stream, *lp, *cfg);
    return (int)hipGetLastError();
}

extern "C" int DSR_INST_CAT(dsr_inst_occupancy_, DSR_INST_TAG)(uint32_t wg_size, uint32_t lds_bytes)
{
    (void)hipFuncSetAttribute((const void *)DSR_INST_KERNEL, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)DSR_INST_KERNEL, (int)wg_size, lds_bytes) !=
        hipSuccess)
        return 0;
    return n;
}

extern "C" int DSR_INST_CAT(dsr_inst_regs_, DSR_INST_TAG)(void)
{
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, (const void *)DSR_INST_KERNEL) != hipSuccess) return 0;
    return a.numRegs;
}
