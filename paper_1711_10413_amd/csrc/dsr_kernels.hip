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
 * Exact fp64 reduction: every loop value y is converted exactly to a signed
 * integer number of 2^-75 units (it must lie on that grid with |y| < 2^32)
 * and summed in 128-bit (lane) and 192-bit (wave, team, region) integer
 * arithmetic; the region total is rounded to double once, so the result is
 * the correctly rounded sum whatever the team, wave or launch layout.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsr.h"
#include "dsr_device.h"
#include "dsr_internal.h"

using namespace dsr;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

extern __shared__ __align__(16) uint8_t dsr_lds[];

/* ---- 128/192-bit integer helpers --------------------------------------- */
struct lane_acc {
    uint64_t lo, hi;   /* signed 128-bit, two's complement */
    uint32_t bad;      /* a value fell outside the exact-sum window */
};

__device__ __forceinline__ void acc_add_i64(lane_acc &a, int64_t v)
{
    uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 63);
    uint64_t n = a.lo + lo;
    a.hi += hi + (n < a.lo);
    a.lo = n;
}

/* Add y exactly, in units of 2^-75.  y = m * 2^(e-1075) with m the 53-bit
 * significand, so y / 2^-75 = m * 2^(e-1000). */
__device__ __forceinline__ void acc_add_f64(lane_acc &a, double y)
{
    const uint64_t b = (uint64_t)__double_as_longlong(y);
    const uint32_t e = (uint32_t)(b >> 52) & 0x7ffu;
    const uint64_t frac = b & 0x000FFFFFFFFFFFFFull;
    const uint64_t m = frac | (1ull << 52);
    const int32_t s = (int32_t)e - 1000;
    const uint32_t ns = (uint32_t)(-s);
    const bool zero = (b << 1) == 0;
    const bool ok = zero || (e <= 1054u &&
                             (s >= 0 || (ns <= 52u && (m & ((1ull << ns) - 1ull)) == 0)));
    a.bad |= (uint32_t)!ok;
    uint64_t lo, hi;
    if (s >= 0) {
        const uint32_t sc = s > 54 ? 54u : (uint32_t)s;
        lo = m << sc;
        hi = sc ? (m >> (64u - sc)) : 0ull;
    } else {
        lo = m >> (ns & 63u);
        hi = 0;
    }
    if (zero || !ok) { lo = 0; hi = 0; }
    if (b >> 63) {
        const uint64_t nlo = ~lo + 1ull;
        hi = ~hi + (lo == 0 ? 1ull : 0ull);
        lo = nlo;
    }
    const uint64_t n = a.lo + lo;
    a.hi += hi + (n < a.lo);
    a.lo = n;
}

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

__device__ __forceinline__ i192 widen(const lane_acc &a)
{
    return i192{a.lo, a.hi, (uint64_t)((int64_t)a.hi >> 63)};
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m)
{
    return (uint64_t)__shfl_xor((unsigned long long)v, m, 64);
}

/* Sum over the 64 lanes of a wave (every lane gets the total). */
__device__ __forceinline__ i192 wave_sum192(i192 v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        i192 o{shfl_xor64(v.w0, m), shfl_xor64(v.w1, m), shfl_xor64(v.w2, m)};
        v = add192(v, o);
    }
    return v;
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
/* Lanes taking part in a body are numbered p in [0, P): worker waves first,
 * then the master wave if it joins.  Team range [lo, hi). */
struct span_t {
    uint64_t lo, hi;
    uint32_t p, P;
};

__device__ __forceinline__ void body_affine_xor(const uint8_t *fb, const dsr_dloop &L,
                                                span_t sp, lane_acc &A)
{
    const int32_t *fr = (const int32_t *)(fb + 8);
    const uint32_t a = (uint32_t)fr[0], b = (uint32_t)fr[1];
    const uint32_t c = (uint32_t)fr[2], d = (uint32_t)fr[3];
    int32_t *out = (int32_t *)L.out;
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

template <int NI, int NF>
__device__ __forceinline__ void body_fma_fixed(const uint8_t *fb, const dsr_dloop &L, span_t sp, lane_acc &A)
{
    double s[NI + NF];
    const int32_t *si = (const int32_t *)(fb + 24 + 8 * NF);
    const double *sf = (const double *)(fb + 24);
#pragma unroll
    for (int k = 0; k < NI; ++k) s[k] = (double)si[k];
#pragma unroll
    for (int k = 0; k < NF; ++k) s[NI + k] = sf[k];

    const float *__restrict__ x = (const float *)L.in;
    double *__restrict__ y = (double *)L.out;
    const uint64_t vlo = min(sp.hi, (sp.lo + 3) & ~3ull);
    const uint64_t vhi = max(vlo, sp.hi & ~3ull);
    for (uint64_t i = sp.lo + sp.p; i < vlo; i += sp.P) {
        const double v = chain<NI, NF>(s, (double)x[i]);
        y[i] = v;
        acc_add_f64(A, v);
    }
    const f32x4 *__restrict__ x4 = (const f32x4 *)x;
    f64x2 *__restrict__ y2 = (f64x2 *)y;
    const uint64_t nv1 = vhi >> 2;
    uint64_t v = (vlo >> 2) + sp.p;
    constexpr int U = (NI + NF >= 32) ? 2 : 4;
    for (; v + (uint64_t)(U - 1) * sp.P < nv1; v += (uint64_t)U * sp.P) {
        f32x4 xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = __builtin_nontemporal_load(&x4[v + (uint64_t)u * sp.P]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t w = v + (uint64_t)u * sp.P;
            f64x2 lo2, hi2;
            lo2.x = chain<NI, NF>(s, (double)xv[u].x);
            lo2.y = chain<NI, NF>(s, (double)xv[u].y);
            hi2.x = chain<NI, NF>(s, (double)xv[u].z);
            hi2.y = chain<NI, NF>(s, (double)xv[u].w);
            __builtin_nontemporal_store(lo2, &y2[2 * w]);
            __builtin_nontemporal_store(hi2, &y2[2 * w + 1]);
            acc_add_f64(A, lo2.x);
            acc_add_f64(A, lo2.y);
            acc_add_f64(A, hi2.x);
            acc_add_f64(A, hi2.y);
        }
    }
    for (; v < nv1; v += sp.P) {
        const f32x4 xv = __builtin_nontemporal_load(&x4[v]);
        f64x2 lo2, hi2;
        lo2.x = chain<NI, NF>(s, (double)xv.x);
        lo2.y = chain<NI, NF>(s, (double)xv.y);
        hi2.x = chain<NI, NF>(s, (double)xv.z);
        hi2.y = chain<NI, NF>(s, (double)xv.w);
        __builtin_nontemporal_store(lo2, &y2[2 * v]);
        __builtin_nontemporal_store(hi2, &y2[2 * v + 1]);
        acc_add_f64(A, lo2.x);
        acc_add_f64(A, lo2.y);
        acc_add_f64(A, hi2.x);
        acc_add_f64(A, hi2.y);
    }
    for (uint64_t i = vhi + sp.p; i < sp.hi; i += sp.P) {
        const double r = chain<NI, NF>(s, (double)x[i]);
        y[i] = r;
        acc_add_f64(A, r);
    }
}

/* fma chain with run-time scalar counts and an optional shared array:
 * the scalars are read from the frame (LDS broadcast or scalar-cache
 * loads) on every use. */
__device__ __forceinline__ void body_fma_generic(const uint8_t *fb, const dsr_dloop &L, span_t sp, lane_acc &A)
{
    const uint32_t ni = L.ni, nf = L.nf, alen = L.alen;
    const double *sf = (const double *)(fb + 24);
    const int32_t *si = (const int32_t *)(fb + 24 + 8 * nf);
    const int32_t *arr = (const int32_t *)(fb + ((24 + 8 * nf + 4 * ni + 15) & ~15u));
    const float *__restrict__ x = (const float *)L.in;
    double *__restrict__ y = (double *)L.out;
    for (uint64_t i = sp.lo + sp.p; i < sp.hi; i += sp.P) {
        const double xd = (double)x[i];
        double acc = alen ? (double)arr[i % alen] : 0.0;
        for (uint32_t k = 0; k < ni; ++k) acc = __builtin_fma((double)si[k], xd, acc);
        for (uint32_t k = 0; k < nf; ++k) acc = __builtin_fma(sf[k], xd, acc);
        y[i] = acc;
        acc_add_f64(A, acc);
    }
}

/* Shared-array gather; arrays at `arr` (LDS or HBM), `len` elements each. */
template <int NA>
__device__ __forceinline__ i32x4 gather4(const int32_t *arr, uint32_t len, uint32_t na, uint32_t idx)
{
    i32x4 s = {0, 0, 0, 0};
    if (NA > 0) {
#pragma unroll
        for (int j = 0; j < NA; ++j) s += *(const i32x4 *)(arr + (uint64_t)j * len + idx);
    } else {
        for (uint32_t j = 0; j < na; ++j) s += *(const i32x4 *)(arr + (uint64_t)j * len + idx);
    }
    return s;
}

/* Vectors [v0, v1) of 4 elements, visited v0 + k*stride; len % 4 == 0. */
template <int NA>
__device__ __forceinline__ void gather_vectors(const int32_t *arr, const dsr_dloop &L,
                                               uint64_t v0, uint64_t v1, uint64_t stride)
{
    const uint32_t len = L.len;
    i32x4 *__restrict__ out4 = (i32x4 *)L.out;
    uint32_t idx = (uint32_t)((v0 * 4) % len);
    const uint32_t step = (uint32_t)((stride * 4) % len);
    for (uint64_t v = v0; v < v1; v += stride) {
        i32x4 s = gather4<NA>(arr, len, L.arrays, idx);
        const uint32_t base = (uint32_t)(v * 4);
        s += i32x4{(int32_t)base, (int32_t)(base + 1), (int32_t)(base + 2), (int32_t)(base + 3)};
        __builtin_nontemporal_store(s, &out4[v]);
        idx += step;
        if (idx >= len) idx -= len;
    }
}

__device__ __forceinline__ void gather_scalar(const int32_t *arr, const dsr_dloop &L,
                                              uint64_t i0, uint64_t i1, uint64_t stride)
{
    int32_t *out = (int32_t *)L.out;
    for (uint64_t i = i0; i < i1; i += stride) {
        uint32_t s = (uint32_t)i;
        const uint32_t k = (uint32_t)(i % L.len);
        for (uint32_t j = 0; j < L.arrays; ++j) s += (uint32_t)arr[(uint64_t)j * L.len + k];
        out[i] = (int32_t)s;
    }
}

template <int NA>
__device__ __forceinline__ void body_gather_flat(const int32_t *arr, const dsr_dloop &L, span_t sp)
{
    if ((L.len & 3u) || (sp.lo & 3u)) {
        gather_scalar(arr, L, sp.lo + sp.p, sp.hi, sp.P);
        return;
    }
    const uint64_t nv = (sp.hi - sp.lo) >> 2;
    gather_vectors<NA>(arr, L, (sp.lo >> 2) + sp.p, (sp.lo >> 2) + nv, sp.P);
    gather_scalar(arr, L, sp.lo + 4 * nv + sp.p, sp.hi, sp.P);
}

/* Nested level: the outer member (this wave) pushes an inner frame on its
 * own sub-stack and hands it to its four 16-lane groups. */
template <int NA>
__device__ __forceinline__ void body_gather_nested(team_t &T, const int32_t *arr, frame_t outer,
                                   const dsr_dloop &L, span_t sp, uint32_t member,
                                   uint32_t members, uint32_t &inner_pushes)
{
    const bool vec = !((L.len & 3u) || (sp.lo & 3u));
    const uint64_t units = vec ? ((sp.hi - sp.lo) >> 2) : (sp.hi - sp.lo);
    const uint64_t per = (units + members - 1) / members;
    const uint64_t ulo = min(units, (uint64_t)member * per), uhi = min(units, ulo + per);
    /* push the inner frame {lo, hi, stride, outer frame offset} */
    uint32_t *inner = (uint32_t *)sub_stack(T, T.wave);
    if (T.lane == 0) {
        inner[0] = (uint32_t)ulo;
        inner[1] = (uint32_t)uhi;
        inner[2] = 64u;
        inner[3] = outer.off;
    }
    inner_pushes += 1;
    wave_sync();
    /* inner members: group g = lane / 16 reads the inner frame */
    const uint32_t ilo = uniform(inner[0]), ihi = uniform(inner[1]), istride = uniform(inner[2]);
    const uint32_t g = T.lane >> 4, l = T.lane & 15u;
    if (vec) {
        const uint64_t base = sp.lo >> 2;
        gather_vectors<NA>(arr, L, base + ilo + g * 16 + l, base + ihi, istride);
        if (member == members - 1) {
            const uint64_t tail = sp.lo + 4 * units;
            gather_scalar(arr, L, tail + T.lane, sp.hi, 64);
        }
    } else {
        gather_scalar(arr, L, sp.lo + ilo + g * 16 + l, sp.lo + ihi, istride);
    }
    /* pop: the inner frame dies with the outer member's body */
    wave_sync();
}

/* ---- region execution ---------------------------------------------------- */
__device__ __forceinline__ const uint8_t *frame_ptr(const team_t &T, frame_t f)
{
    return f.space == SPACE_LDS ? frame_lds(T, f) : frame_hbm(T, f);
}

/* VARIANT selects which fixed-length fma chains are compiled into the
 * kernel: the worker code is specialised to the bodies a region can
 * publish, so a region of short chains does not pay the register budget
 * of the longest one.  0: chains up to 8+8 scalars; 1: adds 16+16;
 * 2: adds 32+32; -1 (workgroups above 256 threads, 128 registers per
 * lane): run-time loop only.  Other lengths use the run-time loop. */
template <int VARIANT>
__device__ __forceinline__ void run_body(team_t &T, uint32_t body, frame_t f, const dsr_dloop &L, span_t sp,
                         lane_acc &A, uint32_t member, uint32_t members, uint32_t &inner_pushes)
{
    switch (body) {
    case DSR_BODY_AFFINE_XOR:
        body_affine_xor(frame_ptr(T, f), L, sp, A);
        break;
    case DSR_BODY_FMA_CHAIN: {
        const uint8_t *fb = frame_ptr(T, f);
        const uint32_t ni = L.ni, nf = L.nf;
        if (VARIANT >= 0 && L.alen == 0) {
            if (ni == 1 && nf == 0) { body_fma_fixed<1, 0>(fb, L, sp, A); break; }
            if (ni == 1 && nf == 1) { body_fma_fixed<1, 1>(fb, L, sp, A); break; }
            if (ni == 2 && nf == 2) { body_fma_fixed<2, 2>(fb, L, sp, A); break; }
            if (ni == 4 && nf == 4) { body_fma_fixed<4, 4>(fb, L, sp, A); break; }
            if (ni == 8 && nf == 8) { body_fma_fixed<8, 8>(fb, L, sp, A); break; }
            if constexpr (VARIANT >= 1)
                if (ni == 16 && nf == 16) { body_fma_fixed<16, 16>(fb, L, sp, A); break; }
            if constexpr (VARIANT >= 2)
                if (ni == 32 && nf == 32) { body_fma_fixed<32, 32>(fb, L, sp, A); break; }
        }
        body_fma_generic(fb, L, sp, A);
        break;
    }
    case DSR_BODY_GATHER: {
        if (f.space == SPACE_LDS) {
            const int32_t *arr = (const int32_t *)(dsr_lds + cb_bytes(T.nw) + f.off);
            switch (L.arrays) {
            case 1: body_gather_flat<1>(arr, L, sp); break;
            case 2: body_gather_flat<2>(arr, L, sp); break;
            case 3: body_gather_flat<3>(arr, L, sp); break;
            case 4: body_gather_flat<4>(arr, L, sp); break;
            default: body_gather_flat<0>(arr, L, sp); break;
            }
        } else {
            const int32_t *arr = (const int32_t *)frame_hbm(T, f);
            switch (L.arrays) {
            case 1: body_gather_flat<1>(arr, L, sp); break;
            case 2: body_gather_flat<2>(arr, L, sp); break;
            case 3: body_gather_flat<3>(arr, L, sp); break;
            case 4: body_gather_flat<4>(arr, L, sp); break;
            default: body_gather_flat<0>(arr, L, sp); break;
            }
        }
        break;
    }
    case DSR_BODY_GATHER_NESTED: {
        if (f.space == SPACE_LDS) {
            const int32_t *arr = (const int32_t *)(dsr_lds + cb_bytes(T.nw) + f.off);
            switch (L.arrays) {
            case 1: body_gather_nested<1>(T, arr, f, L, sp, member, members, inner_pushes); break;
            case 2: body_gather_nested<2>(T, arr, f, L, sp, member, members, inner_pushes); break;
            case 3: body_gather_nested<3>(T, arr, f, L, sp, member, members, inner_pushes); break;
            case 4: body_gather_nested<4>(T, arr, f, L, sp, member, members, inner_pushes); break;
            default: body_gather_nested<0>(T, arr, f, L, sp, member, members, inner_pushes); break;
            }
        } else {
            const int32_t *arr = (const int32_t *)frame_hbm(T, f);
            switch (L.arrays) {
            case 1: body_gather_nested<1>(T, arr, f, L, sp, member, members, inner_pushes); break;
            case 2: body_gather_nested<2>(T, arr, f, L, sp, member, members, inner_pushes); break;
            case 3: body_gather_nested<3>(T, arr, f, L, sp, member, members, inner_pushes); break;
            case 4: body_gather_nested<4>(T, arr, f, L, sp, member, members, inner_pushes); break;
            default: body_gather_nested<0>(T, arr, f, L, sp, member, members, inner_pushes); break;
            }
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
    s.lo = min(L.n, (uint64_t)team * L.chunk);
    s.hi = min(L.n, s.lo + L.chunk);
    s.p = p;
    s.P = P;
    return s;
}

/* Run one participating wave's share of a published body and join. */
template <int VARIANT>
__device__ __forceinline__ void participate(team_t &T, const dsr_dregion &R, const dsr_dconfig &C, uint32_t team,
                            uint32_t body, frame_t f, uint32_t loop, uint32_t &inner_pushes)
{
    const uint32_t nwork = C.master_joins ? T.nw : T.nw - 1;
    const dsr_dloop &L = R.loops[loop];
    lane_acc A{0, 0, 0};
    run_body<VARIANT>(T, body, f, L, team_span(L, team, T.wave * 64 + T.lane, nwork * 64), A, T.wave,
                      nwork, inner_pushes);
    const i192 w = wave_sum192(widen(A));
    const uint32_t bad = __any(A.bad != 0);
    end_parallel(T, w.w0, w.w1, w.w2, bad);
}

/* Copy a frame's initial bytes (or zeros) with the whole master wave. */
__device__ __forceinline__ void init_frame(team_t &T, frame_t f, const uint8_t *src, uint32_t init_bytes,
                           uint32_t nbytes)
{
    uint8_t *dst = (uint8_t *)frame_ptr(T, f);
    const uint32_t nvec = nbytes >> 4;
    const bool src_aligned = (((uintptr_t)src) & 15u) == 0;
    for (uint32_t k = T.lane; k < nvec; k += 64) {
        const uint32_t o = k * 16;
        uint4 v;
        if (o + 16 <= init_bytes && src_aligned) {
            v = *(const uint4 *)(src + o);
        } else {
            uint8_t tmp[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) tmp[q] = (o + q < init_bytes) ? src[o + q] : 0;
            v = *(const uint4 *)tmp;
        }
        *(uint4 *)(dst + o) = v;
    }
    for (uint32_t o = nvec * 16 + T.lane; o < nbytes; o += 64) dst[o] = o < init_bytes ? src[o] : 0;
}

/* Master wave: the sequential code block (Figure 2). */
template <int VARIANT>
__device__ __forceinline__ void master_program(team_t &T, const dsr_dregion &R, const dsr_dconfig &C, uint32_t team,
                               uint32_t &barriers, uint32_t &inner_pushes)
{
    cb_header *h = header(T);
    uint32_t *tr = C.trace ? R.trace + (uint64_t)team * DSR_TRACE_WORDS : nullptr;
    wave_sync();
    int32_t err = 0;
    uint32_t npush = 0;
    const uint32_t nwork = C.master_joins ? T.nw : T.nw - 1;
    for (uint32_t k = 0; k < R.n_ops; ++k) {
        const dsr_op op = R.ops[k];
        if (op.kind == DSR_OP_PUSH) {
            const frame_t f = push(T, op.nbytes);
            if (f.space == SPACE_NONE) { err = DSR_E_NOMEM; break; }
            if (tr && T.lane == 0 && npush < 16) {
                tr[1 + 3 * npush] = f.space;
                tr[2 + 3 * npush] = f.off;
                tr[3 + 3 * npush] = f.size;
            }
            npush++;
            init_frame(T, f, R.init + op.init_off + (uint64_t)team * op.init_stride, op.init_bytes,
                       op.nbytes);
        } else if (op.kind == DSR_OP_PUBLISH) {
            const uint32_t *ft = frame_table(T) + 4 * op.frame;
            frame_t f;
            f.space = uniform(ft[0]);
            f.off = uniform(ft[1]);
            f.size = uniform(ft[2]);
            publish(T, f, op.body, op.loop);
            barriers++;
            if (C.master_joins) {
                participate<VARIANT>(T, R, C, team, op.body, f, op.loop, inner_pushes);
            } else {
                end_parallel(T, 0, 0, 0, 0);
            }
            barriers++;
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
                uint8_t *fb = (uint8_t *)frame_ptr(T, f);
                i192 slot;
                if (op.body == DSR_BODY_AFFINE_XOR) {
                    const int64_t cur = *(const int64_t *)fb;
                    const int64_t nv = (int64_t)((uint64_t)cur + tot.w0);
                    slot = i192{(uint64_t)nv, (uint64_t)(nv >> 63), (uint64_t)(nv >> 63)};
                    wave_sync();
                    if (T.lane == 0) *(int64_t *)fb = nv;
                } else {
                    const uint64_t *c = (const uint64_t *)fb;
                    slot = add192(tot, i192{c[0], c[1], c[2]});
                    wave_sync();
                    if (T.lane == 0) {
                        uint64_t *cw = (uint64_t *)fb;
                        cw[0] = slot.w0; cw[1] = slot.w1; cw[2] = slot.w2;
                    }
                }
                if (T.lane == 0) {
                    uint64_t *pp = R.partials + ((uint64_t)op.red * R.teams + team) * 3;
                    pp[0] = slot.w0; pp[1] = slot.w1; pp[2] = slot.w2;
                }
            }
            wave_sync();
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
    /* terminate the workers (Figure 3's terminate branch) */
    frame_t none{SPACE_NONE, 0, 0};
    publish(T, none, DSR_BODY_TERMINATE, 0);
    barriers++;
    if (tr && T.lane == 0) {
        tr[0] = npush;
        tr[81] = (uint32_t)err;
    }
    if (err && T.lane == 0) atomicCAS(&R.result->error, 0, err);
}

/* Last team: combine every team's partials, in 192-bit integers. */
__device__ __forceinline__ void combine_teams(const dsr_dregion &R, uint32_t lane)
{
    for (uint32_t r = 0; r < R.n_red; ++r) {
        i192 s{0, 0, 0};
        for (uint32_t t = lane; t < R.teams; t += 64) {
            const uint64_t *pp = R.partials + ((uint64_t)r * R.teams + t) * 3;
            s = add192(s, i192{__builtin_nontemporal_load(pp), __builtin_nontemporal_load(pp + 1),
                               __builtin_nontemporal_load(pp + 2)});
        }
        s = wave_sum192(s);
        if (lane == 0) {
            R.result->fixed[r][0] = s.w0;
            R.result->fixed[r][1] = s.w1;
            R.result->fixed[r][2] = s.w2;
            R.result->i64[r] = (int64_t)s.w0;
            R.result->f64[r] = ((R.red_kind_mask >> r) & 1u) ? fixed_to_double(s) : (double)(int64_t)s.w0;
        }
    }
}

__device__ __forceinline__ void finish_team(const dsr_dregion &R, uint32_t lane)
{
    __threadfence();
    uint32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&R.result->arrived, 1u);
    prev = (uint32_t)__shfl((int)prev, 0, 64);
    if (prev == R.teams - 1) {
        __threadfence();
        combine_teams(R, lane);
        if (lane == 0) {
            R.result->final_error = atomicExch(&R.result->error, 0);
            R.result->done += 1;
            __threadfence();
            atomicExch(&R.result->arrived, 0u);
        }
    }
}

template <int MAXWG, int VARIANT>
__global__ __launch_bounds__(MAXWG) void dsr_region_kernel(dsr_dregion R, dsr_dconfig C)
{
    const uint32_t team = blockIdx.x;
    team_t T = team_init(dsr_lds, C.nw, C.lds_cap, C.threshold,
                         C.hbm_base + (uint64_t)team * C.hbm_slot_bytes, (uint32_t)C.hbm_slot_bytes);
    uint32_t barriers = 0, inner_pushes = 0;
    if (T.wave == C.nw - 1) {
        master_program<VARIANT>(T, R, C, team, barriers, inner_pushes);
        finish_team(R, T.lane);
    } else {
        for (;;) {
            uint32_t body, loop;
            frame_t f;
            const bool go = await(T, &body, &f, &loop);
            barriers++;
            if (!go) break;
            participate<VARIANT>(T, R, C, team, body, f, loop, inner_pushes);
            barriers++;
        }
    }
    if (C.trace && T.lane == 0) {
        uint32_t *tr = R.trace + (uint64_t)team * DSR_TRACE_WORDS;
        tr[49 + T.wave] = barriers;
        tr[65 + T.wave] = inner_pushes;
    }
}

template <int MAXWG, int VARIANT>
static hipError_t launch_variant(const dsr_dregion *reg, const dsr_dconfig *cfg, uint32_t wg_size,
                                 uint32_t lds_bytes, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)dsr_region_kernel<MAXWG, VARIANT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL((dsr_region_kernel<MAXWG, VARIANT>), dim3(reg->teams), dim3(wg_size), lds_bytes,
                       s, *reg, *cfg);
    return hipGetLastError();
}

extern "C" int dsr_launch_region_kernel(const dsr_dregion *reg, const dsr_dconfig *cfg,
                                        uint32_t wg_size, uint32_t lds_bytes, uint32_t variant,
                                        void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (wg_size > 256) return (int)launch_variant<1024, -1>(reg, cfg, wg_size, lds_bytes, s);
    switch (variant) {
    case 0: return (int)launch_variant<256, 0>(reg, cfg, wg_size, lds_bytes, s);
    case 1: return (int)launch_variant<256, 1>(reg, cfg, wg_size, lds_bytes, s);
    default: return (int)launch_variant<256, 2>(reg, cfg, wg_size, lds_bytes, s);
    }
}
