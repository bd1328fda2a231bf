/*
 * dsr_api.cpp -- host side of libdsr.so: the C ABI declared in dsr.h.
 *
 * The host records the master's program (push / publish / pop), checks it
 * on the CPU (LIFO pops, live frames at region end, frame sizes against
 * the bodies' layouts, loop coverage), uploads it once and launches the
 * generic-mode region kernel.  Frame placement (LDS or HBM slab) is left
 * to the device, as in the paper's runtime, where the stack lives on the
 * GPU (section 5.3.1) and the fallback is taken at run time (section 5.2).
 */
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "dsr.h"
#include "dsr_device.h"
#include "dsr_internal.h"

namespace {

constexpr uint32_t kDefaultLdsPerWg = 160 * 1024;  /* gfx950 */

}  // namespace

struct dsr_ctx {
    int device;                 /* -1: host-only context (validation only) */
    dsr_config cfg;
    uint32_t nw;
    uint32_t lds_bytes;         /* dynamic LDS per team                     */
    uint32_t threshold;
    uint8_t *hbm;
};

struct dsr_region {
    dsr_ctx *ctx;
    int32_t teams;
    std::vector<dsr_op> ops;
    std::vector<dsr_dloop> loops;
    std::vector<uint8_t> init;
    std::vector<int32_t> live;          /* live frame handles, bottom..top  */
    std::vector<uint32_t> nbytes;       /* declared bytes per handle        */
    std::vector<uint8_t> dead;          /* handle popped                    */
    uint32_t n_red;
    uint32_t red_kind_mask;
    uint32_t variant;                   /* widest fixed fma chain published */
    bool frozen;                        /* uploaded; program can't change   */
    /* device side */
    dsr_op *d_ops;
    dsr_dloop *d_loops;
    uint8_t *d_init;
    uint64_t *d_partials;
    dsr_dresult *d_result;
    uint32_t *d_trace;
    hipEvent_t ev0, ev1;
    bool timed;                         /* ev0 was recorded by the last launch */
    bool launched;
    dsr_dresult h_result;
    bool have_result;
};

extern "C" const char *dsr_strerror(int code)
{
    switch (code) {
    case DSR_OK: return "ok";
    case DSR_E_INVAL: return "invalid argument";
    case DSR_E_NOMEM: return "out of memory: frame fits neither the LDS stack nor the HBM slab";
    case DSR_E_LDS: return "configuration exceeds the LDS available to a workgroup";
    case DSR_E_UNDERFLOW: return "pop on an empty stack";
    case DSR_E_ORDER: return "pop of a frame that is not the top of the stack";
    case DSR_E_LIVE: return "a frame is still live at the end of the region";
    case DSR_E_STATE: return "operation not allowed in this state";
    case DSR_E_BUSY: return "busy";
    case DSR_E_HIP: return "HIP runtime error";
    case DSR_E_RANGE: return "loop value outside the exact-sum window";
    default: return "unknown error";
    }
}

extern "C" int dsr_init(dsr_ctx **out, const dsr_config *cfg, int device)
{
    if (!out || !cfg) return DSR_E_INVAL;
    *out = nullptr;
    const dsr_config c = *cfg;
    if (c.wg_size < 64 || c.wg_size > 1024 || (c.wg_size & 63u)) return DSR_E_INVAL;
    if (c.max_teams == 0) return DSR_E_INVAL;
    if (c.hbm_slab_bytes > 0xFFFFFFF0ull || (c.hbm_slab_bytes & 15u)) return DSR_E_INVAL;
    if (c.lds_slab_bytes & 15u) return DSR_E_INVAL;
    if (c.flags & ~(DSR_F_TRACE | DSR_F_TIMING)) return DSR_E_INVAL;
    const uint32_t nw = c.wg_size / 64;
    const uint64_t lds = (uint64_t)dsr::cb_bytes(nw) + c.lds_slab_bytes;
    uint32_t lds_max = kDefaultLdsPerWg;
    if (device >= 0) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device >= n) return DSR_E_HIP;
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
            v > 0)
            lds_max = (uint32_t)v;
    }
    if (lds > lds_max) return DSR_E_LDS;
    dsr_ctx *ctx = new (std::nothrow) dsr_ctx();
    if (!ctx) return DSR_E_NOMEM;
    ctx->device = device;
    ctx->cfg = c;
    if (nw == 1) ctx->cfg.master_joins = 1;   /* no worker wave otherwise */
    ctx->nw = nw;
    ctx->lds_bytes = (uint32_t)lds;
    ctx->threshold = c.overflow_threshold ? c.overflow_threshold : 0xFFFFFFFFu;
    ctx->hbm = nullptr;
    if (device >= 0) {
        if (hipSetDevice(device) != hipSuccess) { delete ctx; return DSR_E_HIP; }
        const uint64_t bytes = c.hbm_slab_bytes * (uint64_t)c.max_teams;
        if (bytes) {
            if (hipMalloc((void **)&ctx->hbm, bytes) != hipSuccess) { delete ctx; return DSR_E_NOMEM; }
        }
    }
    *out = ctx;
    return DSR_OK;
}

extern "C" int dsr_destroy(dsr_ctx *ctx)
{
    if (!ctx) return DSR_E_INVAL;
    if (ctx->hbm) {
        hipDeviceSynchronize();
        hipFree(ctx->hbm);
    }
    delete ctx;
    return DSR_OK;
}

extern "C" int dsr_region_begin(dsr_ctx *ctx, int32_t teams, dsr_region **out)
{
    if (!ctx || !out) return DSR_E_INVAL;
    *out = nullptr;
    if (teams < 1 || (uint32_t)teams > ctx->cfg.max_teams) return DSR_E_INVAL;
    dsr_region *r = new (std::nothrow) dsr_region();
    if (!r) return DSR_E_NOMEM;
    r->ctx = ctx;
    r->teams = teams;
    r->n_red = 0;
    r->red_kind_mask = 0;
    r->variant = 0;
    r->frozen = false;
    r->d_ops = nullptr;
    r->d_loops = nullptr;
    r->d_init = nullptr;
    r->d_partials = nullptr;
    r->d_result = nullptr;
    r->d_trace = nullptr;
    r->ev0 = r->ev1 = nullptr;
    r->timed = false;
    r->launched = false;
    r->have_result = false;
    *out = r;
    return DSR_OK;
}

extern "C" int dsr_push(dsr_region *r, uint32_t nbytes, const void *init, uint32_t init_bytes,
                        uint32_t init_stride, int32_t *frame_out)
{
    if (!r || !frame_out) return DSR_E_INVAL;
    if (r->frozen) return DSR_E_STATE;
    if (init_bytes > nbytes || (init_bytes && !init)) return DSR_E_INVAL;
    if (nbytes > 0x7FFFFFF0u) return DSR_E_INVAL;
    if (init_stride && (init_stride < init_bytes || (init_stride & 15u))) return DSR_E_INVAL;
    if (r->live.size() >= DSR_MAX_FRAMES || r->ops.size() >= DSR_MAX_OPS) return DSR_E_INVAL;
    dsr_op op{};
    op.kind = DSR_OP_PUSH;
    op.frame = (uint32_t)r->nbytes.size();
    op.nbytes = nbytes;
    op.init_bytes = init_bytes;
    op.init_stride = init_stride;
    op.red = 0xffffffffu;
    size_t off = (r->init.size() + 15) & ~(size_t)15;
    const size_t copy = init_stride ? (size_t)init_stride * r->teams : init_bytes;
    try {
        r->init.resize(off + copy, 0);
        if (copy) std::memcpy(r->init.data() + off, init, copy);
        op.init_off = off;
        r->ops.push_back(op);
        r->live.push_back((int32_t)op.frame);
        r->nbytes.push_back(nbytes);
        r->dead.push_back(0);
    } catch (...) {
        return DSR_E_NOMEM;
    }
    *frame_out = (int32_t)op.frame;
    return DSR_OK;
}

static int frame_depth(const dsr_region *r, int32_t frame)
{
    for (size_t d = 0; d < r->live.size(); ++d)
        if (r->live[d] == frame) return (int)d;
    return -1;
}

extern "C" int dsr_publish(dsr_region *r, int32_t frame, int32_t body, const dsr_loop *loop)
{
    if (!r || !loop) return DSR_E_INVAL;
    if (r->frozen) return DSR_E_STATE;
    const int depth = frame_depth(r, frame);
    if (depth < 0) return DSR_E_STATE;
    if (r->loops.size() >= DSR_MAX_LOOPS || r->ops.size() >= DSR_MAX_OPS) return DSR_E_INVAL;
    const dsr_loop L = *loop;
    const uint32_t nb = r->nbytes[frame];
    if (L.n > 0x7FFFFFFFull) return DSR_E_INVAL;
    uint64_t chunk = L.chunk;
    uint64_t dyn_start = L.n;
    uint32_t block = 0;
    if (L.schedule == DSR_SCHED_STATIC) {
        if (chunk == 0) {
            chunk = (L.n + r->teams - 1) / r->teams;
            chunk = (chunk + 63) & ~63ull;
            if (chunk == 0) chunk = 64;
        }
        if (chunk * (uint64_t)r->teams < L.n) return DSR_E_INVAL;
    } else if (L.schedule == DSR_SCHED_DYNAMIC_TAIL) {
        if (chunk != 0) return DSR_E_INVAL;
        const uint32_t pct = L.tail_pct ? L.tail_pct : 25;
        block = L.block ? L.block : 1024;
        if (pct > 99 || (block & 127u) || block > 65536) return DSR_E_INVAL;
        /* a block can run on any team: every team's frame must be the same */
        for (const dsr_op &o : r->ops)
            if (o.kind == DSR_OP_PUSH && o.frame == (uint32_t)frame && o.init_stride) return DSR_E_INVAL;
        chunk = (L.n * (100 - pct) / 100) / r->teams;
        chunk &= ~63ull;
        dyn_start = chunk * (uint64_t)r->teams;
        if (chunk == 0) chunk = 64;   /* all of the loop is the dynamic tail */
    } else {
        return DSR_E_INVAL;
    }
    if (L.n && !L.out) return DSR_E_INVAL;
    bool reduces = false;
    switch (body) {
    case DSR_BODY_AFFINE_XOR:
        if (nb < 24) return DSR_E_INVAL;
        reduces = true;
        break;
    case DSR_BODY_FMA_CHAIN: {
        if (L.ni + L.nf > 64) return DSR_E_INVAL;
        if (L.n && !L.in) return DSR_E_INVAL;
        uint64_t need = 24 + 8ull * L.nf + 4ull * L.ni;
        if (L.alen) need = ((need + 15) & ~15ull) + 4ull * L.alen;
        if (nb < need) return DSR_E_INVAL;
        /* a lane's fp64 bins stay exact for up to 2^16 values; the static
         * share is bounded here, dynamic blocks flush the bins as they go */
        {
            const uint64_t lanes = 64ull * (r->ctx->cfg.master_joins ? r->ctx->nw : r->ctx->nw - 1);
            if ((chunk + lanes - 1) / lanes > (1ull << 15)) return DSR_E_INVAL;
        }
        if (L.alen == 0 && L.ni == 16 && L.nf == 16 && r->variant < 1) r->variant = 1;
        if (L.alen == 0 && L.ni == 32 && L.nf == 32) r->variant = 2;
        reduces = true;
        break;
    }
    case DSR_BODY_GATHER:
    case DSR_BODY_GATHER_NESTED:
        if (body == DSR_BODY_GATHER_NESTED && L.schedule != DSR_SCHED_STATIC) return DSR_E_INVAL;
        if (L.arrays < 1 || L.arrays > 16 || L.len < 1) return DSR_E_INVAL;
        if ((uint64_t)nb < 4ull * L.arrays * L.len) return DSR_E_INVAL;
        break;
    default:
        return DSR_E_INVAL;
    }
    if (reduces && r->n_red >= DSR_MAX_RED) return DSR_E_INVAL;
    dsr_dloop dl{};
    dl.n = L.n;
    dl.chunk = chunk;
    dl.in = L.in;
    dl.out = L.out;
    dl.ni = L.ni;
    dl.nf = L.nf;
    dl.alen = L.alen;
    dl.arrays = L.arrays;
    dl.len = L.len;
    dl.schedule = L.schedule;
    dl.block = block;
    dl.dyn_start = dyn_start;
    dsr_op op{};
    op.kind = DSR_OP_PUBLISH;
    op.frame = (uint32_t)depth;
    op.body = (uint32_t)body;
    op.loop = (uint32_t)r->loops.size();
    op.red = 0xffffffffu;
    if (reduces) {
        op.red = r->n_red;
        if (body == DSR_BODY_FMA_CHAIN) r->red_kind_mask |= 1u << r->n_red;
        r->n_red++;
    }
    try {
        r->loops.push_back(dl);
        r->ops.push_back(op);
    } catch (...) {
        return DSR_E_NOMEM;
    }
    return DSR_OK;
}

extern "C" int dsr_pop(dsr_region *r, int32_t frame)
{
    if (!r) return DSR_E_INVAL;
    if (r->frozen) return DSR_E_STATE;
    if (r->live.empty()) return DSR_E_UNDERFLOW;
    if (r->live.back() != frame) return frame_depth(r, frame) >= 0 ? DSR_E_ORDER : DSR_E_STATE;
    if (r->ops.size() >= DSR_MAX_OPS) return DSR_E_INVAL;
    dsr_op op{};
    op.kind = DSR_OP_POP;
    op.frame = (uint32_t)frame;
    op.red = 0xffffffffu;
    r->ops.push_back(op);
    r->live.pop_back();
    r->dead[frame] = 1;
    return DSR_OK;
}

static int hip_ok(hipError_t e) { return e == hipSuccess ? DSR_OK : DSR_E_HIP; }

static int upload(dsr_region *r)
{
    const dsr_ctx *c = r->ctx;
    int rc;
    if ((rc = hip_ok(hipSetDevice(c->device)))) return rc;
    const size_t ops_b = r->ops.size() * sizeof(dsr_op);
    const size_t loops_b = (r->loops.empty() ? 1 : r->loops.size()) * sizeof(dsr_dloop);
    const size_t init_b = r->init.empty() ? 16 : r->init.size();
    const size_t part_b = (size_t)(r->n_red ? r->n_red : 1) * r->teams * 3 * sizeof(uint64_t);
    if (hipMalloc((void **)&r->d_ops, ops_b ? ops_b : sizeof(dsr_op)) != hipSuccess ||
        hipMalloc((void **)&r->d_loops, loops_b) != hipSuccess ||
        hipMalloc((void **)&r->d_init, init_b) != hipSuccess ||
        hipMalloc((void **)&r->d_partials, part_b) != hipSuccess ||
        hipMalloc((void **)&r->d_result, sizeof(dsr_dresult)) != hipSuccess)
        return DSR_E_NOMEM;
    if (c->cfg.flags & DSR_F_TRACE) {
        const size_t tb = (size_t)r->teams * DSR_TRACE_WORDS * sizeof(uint32_t);
        if (hipMalloc((void **)&r->d_trace, tb) != hipSuccess) return DSR_E_NOMEM;
        if ((rc = hip_ok(hipMemset(r->d_trace, 0, tb)))) return rc;
    }
    if (ops_b && (rc = hip_ok(hipMemcpy(r->d_ops, r->ops.data(), ops_b, hipMemcpyHostToDevice))))
        return rc;
    if (!r->loops.empty() &&
        (rc = hip_ok(hipMemcpy(r->d_loops, r->loops.data(), r->loops.size() * sizeof(dsr_dloop),
                               hipMemcpyHostToDevice))))
        return rc;
    if (!r->init.empty() &&
        (rc = hip_ok(hipMemcpy(r->d_init, r->init.data(), r->init.size(), hipMemcpyHostToDevice))))
        return rc;
    if ((rc = hip_ok(hipMemset(r->d_result, 0, sizeof(dsr_dresult))))) return rc;
    if ((rc = hip_ok(hipMemset(r->d_partials, 0, part_b)))) return rc;
    if ((rc = hip_ok(hipEventCreate(&r->ev0)))) return rc;
    if ((rc = hip_ok(hipEventCreate(&r->ev1)))) return rc;
    return DSR_OK;
}

extern "C" int dsr_launch(dsr_region *r, void *stream)
{
    if (!r) return DSR_E_INVAL;
    if (!r->live.empty()) return DSR_E_LIVE;
    dsr_ctx *c = r->ctx;
    if (c->device < 0) return DSR_E_STATE;     /* host-only context */
    if ((uint64_t)r->teams > c->cfg.max_teams) return DSR_E_INVAL;
    if (!r->frozen) {
        const int rc = upload(r);
        if (rc) return rc;
        r->frozen = true;
    }
    hipStream_t s = (hipStream_t)stream;
    dsr_dregion R{};
    R.ops = r->d_ops;
    R.loops = r->d_loops;
    R.init = r->d_init;
    R.partials = r->d_partials;
    R.result = r->d_result;
    R.trace = r->d_trace;
    R.n_ops = (uint32_t)r->ops.size();
    R.teams = (uint32_t)r->teams;
    R.n_red = r->n_red;
    R.red_kind_mask = r->red_kind_mask;
    dsr_dconfig C{};
    C.hbm_base = c->hbm;
    C.hbm_slot_bytes = c->cfg.hbm_slab_bytes;
    C.nw = c->nw;
    C.lds_cap = c->cfg.lds_slab_bytes;
    C.threshold = c->threshold;
    C.master_joins = c->cfg.master_joins ? 1u : 0u;
    C.trace = (c->cfg.flags & DSR_F_TRACE) ? 1u : 0u;
    const bool timing = (c->cfg.flags & DSR_F_TIMING) != 0;
    if (timing && hipEventRecord(r->ev0, s) != hipSuccess) return DSR_E_HIP;
    if (dsr_launch_region_kernel(&R, &C, c->cfg.wg_size, c->lds_bytes, r->variant, stream) != 0)
        return DSR_E_HIP;
    if (hipEventRecord(r->ev1, s) != hipSuccess) return DSR_E_HIP;
    r->timed = timing;
    r->launched = true;
    r->have_result = false;
    return DSR_OK;
}

extern "C" int dsr_region_sync(dsr_region *r)
{
    if (!r) return DSR_E_INVAL;
    if (!r->launched) return DSR_E_STATE;
    if (hipEventSynchronize(r->ev1) != hipSuccess) return DSR_E_HIP;
    if (hipMemcpy(&r->h_result, r->d_result, sizeof(dsr_dresult), hipMemcpyDeviceToHost) != hipSuccess)
        return DSR_E_HIP;
    r->have_result = true;
    return r->h_result.final_error;
}

extern "C" int dsr_region_reduction(dsr_region *r, int32_t index, int64_t *i64, double *f64,
                                    uint64_t *fixed3)
{
    if (!r) return DSR_E_INVAL;
    if (!r->have_result) return DSR_E_STATE;
    if (index < 0 || (uint32_t)index >= r->n_red) return DSR_E_INVAL;
    if (i64) *i64 = r->h_result.i64[index];
    if (f64) *f64 = r->h_result.f64[index];
    if (fixed3) for (int k = 0; k < 3; ++k) fixed3[k] = r->h_result.fixed[index][k];
    return DSR_OK;
}

extern "C" int dsr_region_trace(dsr_region *r, int32_t team, uint32_t *buf, uint32_t n)
{
    if (!r || !buf || n < DSR_TRACE_WORDS) return DSR_E_INVAL;
    if (!r->d_trace) return DSR_E_STATE;
    if (team < 0 || team >= r->teams) return DSR_E_INVAL;
    if (!r->launched) return DSR_E_STATE;
    if (hipEventSynchronize(r->ev1) != hipSuccess) return DSR_E_HIP;
    if (hipMemcpy(buf, r->d_trace + (size_t)team * DSR_TRACE_WORDS, DSR_TRACE_WORDS * sizeof(uint32_t),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return DSR_E_HIP;
    return DSR_OK;
}

extern "C" int dsr_region_elapsed(dsr_region *r, float *ms)
{
    if (!r || !ms) return DSR_E_INVAL;
    if (!r->launched || !r->timed) return DSR_E_STATE;
    if (hipEventSynchronize(r->ev1) != hipSuccess) return DSR_E_HIP;
    return hipEventElapsedTime(ms, r->ev0, r->ev1) == hipSuccess ? DSR_OK : DSR_E_HIP;
}

extern "C" int dsr_region_free(dsr_region *r)
{
    if (!r) return DSR_E_INVAL;
    if (r->launched) hipEventSynchronize(r->ev1);
    if (r->d_ops) hipFree(r->d_ops);
    if (r->d_loops) hipFree(r->d_loops);
    if (r->d_init) hipFree(r->d_init);
    if (r->d_partials) hipFree(r->d_partials);
    if (r->d_result) hipFree(r->d_result);
    if (r->d_trace) hipFree(r->d_trace);
    if (r->ev0) hipEventDestroy(r->ev0);
    if (r->ev1) hipEventDestroy(r->ev1);
    delete r;
    return DSR_OK;
}
