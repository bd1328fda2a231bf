/*
 * dsr_ceiling.hip -- the streaming ceiling the region kernel's loop is
 * measured against: y[i] = (double)x[i] * s over n elements, the same 4 B
 * read and 8 B write per element as the fma-chain loop, with no runtime
 * around it (no frames, barriers or reduction).  Each workgroup streams one
 * contiguous chunk; a lane takes element pairs (8 B of x, 16 B of y) with
 * the lanes of all waves interleaved, so every load instruction of a wave
 * covers 512 contiguous bytes, and batches of eight pairs per lane are
 * software-pipelined one batch ahead.  Not part of the paper's method: a
 * measuring stick for it.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsr.h"

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
#define GLB __attribute__((address_space(1)))

namespace {

constexpr int kBatch = 8;

__global__ __launch_bounds__(1024) void stream_convert(const float *x, double *y, uint64_t n, double s)
{
    const GLB f32x2 *__restrict__ x2 = (const GLB f32x2 *)x;
    GLB f64x2 *__restrict__ y2 = (GLB f64x2 *)y;
    const uint64_t npairs = n >> 1;
    const uint64_t chunk = (npairs + gridDim.x - 1) / gridDim.x;
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    const uint64_t hi = lo + chunk < npairs ? lo + chunk : npairs;
    const uint64_t P = blockDim.x;
    uint64_t v = lo + threadIdx.x;
    if (v + (kBatch - 1) * P < hi) {
        f32x2 cur[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) cur[u] = __builtin_nontemporal_load(&x2[v + u * P]);
        for (;;) {
            const uint64_t vn = v + kBatch * P;
            const bool more = vn + (kBatch - 1) * P < hi;
            f32x2 nxt[kBatch];
            if (more) {
#pragma unroll
                for (int u = 0; u < kBatch; ++u) nxt[u] = __builtin_nontemporal_load(&x2[vn + u * P]);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                f64x2 r;
                r.x = s * (double)cur[u].x;
                r.y = s * (double)cur[u].y;
                __builtin_nontemporal_store(r, &y2[v + u * P]);
            }
            v = vn;
            if (!more) break;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) cur[u] = nxt[u];
        }
    }
    for (; v < hi; v += P) {
        const f32x2 xv = __builtin_nontemporal_load(&x2[v]);
        f64x2 r;
        r.x = s * (double)xv.x;
        r.y = s * (double)xv.y;
        __builtin_nontemporal_store(r, &y2[v]);
    }
    /* an odd last element */
    if ((n & 1u) && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) y[n - 1] = s * (double)x[n - 1];
}

}  // namespace

extern "C" int dsr_stream_ceiling(const float *x, double *y, uint64_t n, uint32_t grid, uint32_t wg_size,
                                  void *stream)
{
    if ((n && (!x || !y)) || grid == 0 || wg_size == 0 || wg_size > 1024 || (wg_size & 63u)) return DSR_E_INVAL;
    if (!n) return DSR_OK;
    hipLaunchKernelGGL(stream_convert, dim3(grid), dim3(wg_size), 0, (hipStream_t)stream, x, y, n, 1.0);
    return hipGetLastError() == hipSuccess ? DSR_OK : DSR_E_HIP;
}
