/*
 * dsr_static.hip -- the library's fixed device workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).
 *
 * `scratch` is a file-scope device array of DSR_STATIC_SCRATCH_BYTES that
 * every GPU the library runs on holds until the process ends.  In host code
 * its name is only a host-side stand-in, so nothing here passes it to a
 * kernel or a copy: the device address is looked up once per device, with
 * that device current, through hipGetSymbolAddress, and every use goes
 * through the address kept for that device.  Calls that overlap on one GPU
 * share the array and race; the entry point that uses it says so.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsr.h"
#include "dsr_internal.h"

static __device__ __align__(256) uint8_t scratch[DSR_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
uint8_t *g_ptr[kMaxDevices];
bool g_have[kMaxDevices];

__global__ void fill_words(uint32_t *p, uint32_t words, uint32_t value)
{
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < words; k += gridDim.x * blockDim.x)
        p[k] = value;
}

/* The region kernel's result block (in the workspace) as the caller's
 * public record. */
__global__ void copy_result(const dsr_dresult *src, uint32_t n_red, dsr_result_rec *dst)
{
    const uint32_t t = threadIdx.x;
    if (t == 0) {
        dst->status = src->final_error;
        dst->n_red = (int32_t)n_red;
    }
    if (t < DSR_MAX_RED) {
        dst->f64[t] = t < n_red ? src->f64[t] : 0.0;
        dst->i64[t] = t < n_red ? src->i64[t] : 0;
        for (int w = 0; w < 3; ++w) dst->fixed[t][w] = t < n_red ? src->fixed[t][w] : 0;
    }
}

}  // namespace

/* The workspace's device address on `device` (looked up with the device
 * current, the first time, then kept). */
extern "C" int dsr_static_workspace(int device, uint8_t **out)
{
    if (!out || device < 0 || device >= kMaxDevices) return DSR_E_INVAL;
    *out = nullptr;
    if (!g_have[device]) {
        int prev = 0;
        if (hipGetDevice(&prev) != hipSuccess) return DSR_E_HIP;
        if (hipSetDevice(device) != hipSuccess) return DSR_E_HIP;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        (void)hipSetDevice(prev);
        if (e != hipSuccess || !p) return DSR_E_HIP;
        g_ptr[device] = (uint8_t *)p;
        g_have[device] = true;
    }
    *out = g_ptr[device];
    return DSR_OK;
}

/* Fill `words` 32-bit words at device address p with `value` on `stream`
 * (a kernel, not a memset node). */
extern "C" int dsr_static_fill(void *p, uint32_t words, uint32_t value, void *stream)
{
    if (!words) return DSR_OK;
    const uint32_t blocks = (words + 255u) / 256u < 64u ? (words + 255u) / 256u : 64u;
    hipLaunchKernelGGL(fill_words, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (uint32_t *)p, words, value);
    return hipGetLastError() == hipSuccess ? DSR_OK : DSR_E_HIP;
}

extern "C" int dsr_static_copy_result(const void *result_block, uint32_t n_red, void *dst, void *stream)
{
    hipLaunchKernelGGL(copy_result, dim3(1), dim3(64), 0, (hipStream_t)stream, (const dsr_dresult *)result_block,
                       n_red, (dsr_result_rec *)dst);
    return hipGetLastError() == hipSuccess ? DSR_OK : DSR_E_HIP;
}
