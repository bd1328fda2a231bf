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
#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "dsr.h"
#include "dsr_device.h"
#include "dsr_internal.h"

namespace {

constexpr uint32_t kDefaultLdsPerWg = 160 * 1024;  /* gfx950 */

}  // namespace

struct dsr_region;
namespace {
bool stack_peaks(const dsr_region *r, uint32_t lds_cap, uint32_t threshold, uint64_t hbm_cap,
                 uint64_t *lds_peak, uint64_t *hbm_peak);
}  // namespace

struct dsr_ctx {
    int device;                 /* -1: host-only context (validation only) */
    dsr_config cfg;
    uint32_t nw;
    uint32_t lds_bytes;         /* dynamic LDS per team                     */
    uint32_t threshold;
    uint8_t *hbm;
    uint8_t *nest;              /* nested members' global stacks, DSR_NEST_SLOT per team */
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
    int32_t lean;                       /* lean instance chain every publish uses
                                           (-1 none yet, -2 mixed or other bodies) */
    bool frozen;                        /* uploaded; program can't change   */
    /* device side */
    dsr_op *d_ops;
    dsr_dloop *d_loops;
    uint8_t *d_init;
    uint64_t *d_partials;
    dsr_dresult *d_result;
    uint32_t *d_trace;
    dsr_dregion *d_self;                /* this region's descriptor on the device */
    hipEvent_t ev0, ev1;
    bool timed;                         /* ev0, ev1 were recorded around the last launch */
    hipStream_t stream;                 /* stream of the last launch */
    bool launched;
    dsr_dresult h_result;
    dsr_dresult *h_pin;                 /* pinned landing buffer of the result copy,
                                           allocated at the first sync */
    bool have_result;
    uint32_t serve_refs;                /* served requests reading this frozen
                                           region's device images, not yet polled */
    dsr_dregion static_desc;            /* descriptor copied into the workspace by
                                           dsr_launch_static */
    dsr_dregion desc;                   /* host copy of the device descriptor */
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
    if (c.flags & ~(DSR_F_TRACE | DSR_F_TIMING | DSR_F_GLOBAL_LISTS | DSR_F_NESTED_GLOBAL)) return DSR_E_INVAL;
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
    if (nw > 8) ctx->cfg.master_joins = 0;    /* 1024-thread teams: workers only */
    ctx->nw = nw;
    ctx->lds_bytes = (uint32_t)lds;
    ctx->threshold = c.overflow_threshold ? c.overflow_threshold : 0xFFFFFFFFu;
    ctx->hbm = nullptr;
    ctx->nest = nullptr;
    if (device >= 0) {
        if (hipSetDevice(device) != hipSuccess) { delete ctx; return DSR_E_HIP; }
        const uint64_t bytes = c.hbm_slab_bytes * (uint64_t)c.max_teams;
        if (bytes) {
            if (hipMalloc((void **)&ctx->hbm, bytes) != hipSuccess) { delete ctx; return DSR_E_NOMEM; }
        }
        if (hipMalloc((void **)&ctx->nest, (uint64_t)DSR_NEST_SLOT * c.max_teams) != hipSuccess) {
            if (ctx->hbm) hipFree(ctx->hbm);
            delete ctx;
            return DSR_E_NOMEM;
        }
    }
    *out = ctx;
    return DSR_OK;
}

extern "C" int dsr_destroy(dsr_ctx *ctx)
{
    if (!ctx) return DSR_E_INVAL;
    if (ctx->hbm || ctx->nest) hipDeviceSynchronize();
    if (ctx->hbm) hipFree(ctx->hbm);
    if (ctx->nest) hipFree(ctx->nest);
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
    r->lean = -1;
    r->frozen = false;
    r->d_ops = nullptr;
    r->d_loops = nullptr;
    r->d_init = nullptr;
    r->d_partials = nullptr;
    r->d_result = nullptr;
    r->d_trace = nullptr;
    r->d_self = nullptr;
    r->h_pin = nullptr;
    r->serve_refs = 0;
    r->ev0 = r->ev1 = nullptr;
    r->stream = nullptr;
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

/* The loop part of a publish: schedule, coverage of [0, n) by the teams,
 * the device descriptor.  `frames` are the handles the body reads (a
 * dynamic tail runs blocks on any team, so none may have per-team bytes). */
static int prepare_loop(const dsr_region *r, const dsr_loop &L, const int32_t *frames, int nframes,
                        dsr_dloop *out)
{
    if (L.n > 0x7FFFFFFFull) return DSR_E_INVAL;
    uint64_t chunk = L.chunk;
    uint64_t dyn_start = L.n;
    uint32_t block = 0;
    if (L.schedule == DSR_SCHED_STATIC) {
        if (chunk == 0) {
            /* team ranges start on 64-element boundaries, and on 1024-element
             * ones (4 KiB of fp32 input) when a team gets at least 16384
             * iterations: the batched 256-thread form ran 4% faster */
            chunk = (L.n + r->teams - 1) / r->teams;
            const uint64_t g = chunk >= 16384 ? 1024 : 64;
            chunk = (chunk + g - 1) & ~(g - 1);
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
            for (int k = 0; k < nframes; ++k)
                if (o.kind == DSR_OP_PUSH && o.frame == (uint32_t)frames[k] && o.init_stride) return DSR_E_INVAL;
        chunk = (L.n * (100 - pct) / 100) / r->teams;
        chunk &= ~63ull;
        dyn_start = chunk * (uint64_t)r->teams;
        if (chunk == 0) chunk = 64;   /* all of the loop is the dynamic tail */
    } else {
        return DSR_E_INVAL;
    }
    if (L.n && !L.out) return DSR_E_INVAL;
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
    dl.depth = L.depth;
    dl.dyn_start = dyn_start;
    dl.deref = L.deref ? 1u : 0u;
    *out = dl;
    return DSR_OK;
}

/* A lane's fp64 bins stay exact for up to 2^16 values: the static share of
 * a lane is bounded here, dynamic blocks flush the bins as they go. */
static bool lane_share_ok(const dsr_region *r, uint64_t chunk)
{
    const uint64_t lanes = 64ull * (r->ctx->cfg.master_joins ? r->ctx->nw : r->ctx->nw - 1);
    return (chunk + lanes - 1) / lanes <= (1ull << 15);
}

/* The lean chain a publish of `body` over loop L would run on, or -2. */
static int32_t lean_chain_of(int32_t body, const dsr_loop &L)
{
    if (body != DSR_BODY_FMA_CHAIN || L.alen != 0 || L.schedule != DSR_SCHED_STATIC) return -2;
    for (int32_t k = 0; k < DSR_LEAN_CHAINS; ++k)
        if ((int)L.ni == DSR_LEAN_NI(k) && (int)L.nf == DSR_LEAN_NF(k)) return k;
    return -2;
}

static void note_lean(dsr_region *r, int32_t k)
{
    if (r->lean == -1) r->lean = k;
    else if (r->lean != k) r->lean = -2;
}

/* Kernel variant for a single-region launch of r with workgroups of wg. */
static uint32_t single_variant(const dsr_region *r, uint32_t wg)
{
    return (r->lean >= 0 && wg <= 256) ? (uint32_t)(DSR_LEAN_BASE + r->lean) : r->variant;
}

extern "C" int dsr_publish(dsr_region *r, int32_t frame, int32_t body, const dsr_loop *loop)
{
    if (!r || !loop) return DSR_E_INVAL;
    if (r->frozen) return DSR_E_STATE;
    const int depth = frame_depth(r, frame);
    if (depth < 0) return DSR_E_STATE;
    if (r->loops.size() >= DSR_MAX_LOOPS || r->ops.size() >= DSR_MAX_OPS) return DSR_E_INVAL;
    const dsr_loop L = *loop;
    if (L.deref) return DSR_E_INVAL;               /* a list publish only */
    const uint32_t nb = r->nbytes[frame];
    dsr_dloop dl{};
    int rc = prepare_loop(r, L, &frame, 1, &dl);
    if (rc) return rc;
    const uint64_t chunk = dl.chunk;
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
        if (!lane_share_ok(r, chunk)) return DSR_E_INVAL;
        if (L.alen == 0 && L.ni == 16 && L.nf == 16 && r->variant < 1) r->variant = 1;
        if (L.alen == 0 && L.ni == 32 && L.nf == 32) r->variant = 2;
        reduces = true;
        break;
    }
    case DSR_BODY_GATHER:
    case DSR_BODY_GATHER_NESTED:
        if (body == DSR_BODY_GATHER_NESTED) {
            if (L.schedule != DSR_SCHED_STATIC) return DSR_E_INVAL;
            if (L.depth != 0 && L.depth != 2 && L.depth != 3) return DSR_E_INVAL;
            dl.depth = L.depth ? L.depth : 2;
        }
        if (L.arrays < 1 || L.arrays > 16 || L.len < 1) return DSR_E_INVAL;
        if ((uint64_t)nb < 4ull * L.arrays * L.len) return DSR_E_INVAL;
        break;
    default:
        return DSR_E_INVAL;
    }
    if (reduces && r->n_red >= DSR_MAX_RED) return DSR_E_INVAL;
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
    note_lean(r, lean_chain_of(body, L));
    return DSR_OK;
}

extern "C" int dsr_publish_list(dsr_region *r, const dsr_ref *refs, int32_t n, int32_t body,
                                const dsr_loop *loop)
{
    if (!r || !loop || (n > 0 && !refs)) return DSR_E_INVAL;
    if (r->frozen) return DSR_E_STATE;
    if (body != DSR_BODY_FMA_CHAIN_REFS) return DSR_E_INVAL;
    if (r->loops.size() >= DSR_MAX_LOOPS || r->ops.size() >= DSR_MAX_OPS) return DSR_E_INVAL;
    const dsr_loop L = *loop;
    if (L.ni + L.nf > 64) return DSR_E_INVAL;
    if (L.deref && L.alen) return DSR_E_INVAL;      /* per-batch reads: scalars only */
    if (n != (int32_t)(1 + L.ni + L.nf + (L.alen ? 1 : 0))) return DSR_E_INVAL;
    if (L.n && !L.in) return DSR_E_INVAL;
    std::vector<uint32_t> table(2 * (size_t)n);
    std::vector<int32_t> handles(n);
    for (int32_t k = 0; k < n; ++k) {
        const int depth = frame_depth(r, refs[k].frame);
        if (depth < 0) return DSR_E_STATE;
        /* slot, int32 scalars, fp64 scalars, array */
        const uint64_t size = k == 0 ? 24 : (k <= (int32_t)L.ni ? 4 : (k <= (int32_t)(L.ni + L.nf) ? 8 : 4ull * L.alen));
        const uint32_t align = (k == 0 || (k > (int32_t)L.ni && k <= (int32_t)(L.ni + L.nf))) ? 8 : 4;
        if (refs[k].offset % align || (uint64_t)refs[k].offset + size > r->nbytes[refs[k].frame]) return DSR_E_INVAL;
        table[2 * k] = (uint32_t)depth;
        table[2 * k + 1] = refs[k].offset;
        handles[k] = refs[k].frame;
    }
    dsr_dloop dl{};
    int rc = prepare_loop(r, L, handles.data(), n, &dl);
    if (rc) return rc;
    if (!lane_share_ok(r, dl.chunk)) return DSR_E_INVAL;
    if (r->n_red >= DSR_MAX_RED) return DSR_E_INVAL;
    dsr_op op{};
    op.kind = DSR_OP_PUBLISH;
    op.frame = 0xffffffffu;
    op.body = (uint32_t)body;
    op.loop = (uint32_t)r->loops.size();
    op.nbytes = (uint32_t)n;
    op.red = r->n_red;
    try {
        const size_t off = (r->init.size() + 15) & ~(size_t)15;
        r->init.resize(off + table.size() * 4, 0);
        std::memcpy(r->init.data() + off, table.data(), table.size() * 4);
        op.init_off = off;
        r->loops.push_back(dl);
        r->ops.push_back(op);
    } catch (...) {
        return DSR_E_NOMEM;
    }
    note_lean(r, -2);
    r->red_kind_mask |= 1u << r->n_red;
    r->n_red++;
    return DSR_OK;
}

extern "C" uint32_t dsr_control_bytes(uint32_t wg_size)
{
    if (wg_size < 64 || wg_size > 1024 || (wg_size & 63u)) return 0;
    return dsr::cb_bytes(wg_size / 64);
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
    const size_t part_b = (size_t)(r->n_red ? r->n_red : 1) * r->teams * DSR_PART_WORDS * sizeof(uint64_t);
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
    R.n_loops = (uint32_t)r->loops.size();
    R.init_size = (uint32_t)r->init.size();
    if (hipMalloc((void **)&r->d_self, sizeof(dsr_dregion)) != hipSuccess) return DSR_E_NOMEM;
    if ((rc = hip_ok(hipMemcpy(r->d_self, &R, sizeof(R), hipMemcpyHostToDevice)))) return rc;
    r->desc = R;
    return DSR_OK;
}

/* A single-region launch carries the region's descriptor R (device
 * pointers) by value and, when its program is short, the program, its
 * first loop and the image of the frame op 0 pushes. */
static void fill_single(dsr_dlaunch &LP, const dsr_region *r, const dsr_dregion &R)
{
    LP.has_single = 1;
    LP.single = R;
    LP.inl_ops = LP.inl_loop = LP.inl_img = 0;
    if (r->ops.empty() || r->ops.size() > DSR_INLINE_OPS) return;
    LP.inl_ops = (uint32_t)r->ops.size();
    std::memcpy(LP.inl_op, r->ops.data(), r->ops.size() * sizeof(dsr_op));
    if (!r->loops.empty()) {
        LP.inl_loop = 1;
        LP.inl_loop0 = r->loops[0];
    }
    const dsr_op &op = r->ops[0];
    if (op.kind == DSR_OP_PUSH && op.init_stride == 0 && op.init_bytes > 0 && op.init_bytes <= DSR_INLINE_IMG &&
        op.init_off + op.init_bytes <= r->init.size()) {
        const uint32_t padded = (op.init_bytes + 15u) & ~15u;
        std::memset(LP.inl_image, 0, padded);
        std::memcpy(LP.inl_image, r->init.data() + op.init_off, op.init_bytes);
        LP.inl_img = padded;
    }
}

static dsr_dconfig make_dconfig(const dsr_ctx *c, uint32_t wg, uint32_t lds_slab, uint32_t threshold,
                                uint32_t joins, uint32_t trace)
{
    dsr_dconfig C{};
    C.serve = 0;
    C.hbm_base = c->hbm;
    C.hbm_slot_bytes = c->cfg.hbm_slab_bytes;
    C.nw = wg / 64;
    C.lds_cap = lds_slab;
    C.threshold = threshold ? threshold : 0xFFFFFFFFu;
    C.master_joins = ((joins && C.nw <= 8) || C.nw == 1) ? 1u : 0u;
    C.trace = trace;
    C.global_lists = (c->cfg.flags & DSR_F_GLOBAL_LISTS) ? 1u : 0u;
    C.nest_global = (c->cfg.flags & DSR_F_NESTED_GLOBAL) ? 1u : 0u;
    C.nest_base = c->nest;
    return C;
}

extern "C" int dsr_region_freeze(dsr_region *r)
{
    if (!r) return DSR_E_INVAL;
    if (!r->live.empty()) return DSR_E_LIVE;
    if (r->ctx->device < 0) return DSR_E_STATE;
    if ((uint64_t)r->teams > r->ctx->cfg.max_teams) return DSR_E_INVAL;
    if (!r->frozen) {
        const int rc = upload(r);
        if (rc) return rc;
        r->frozen = true;
    }
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
    dsr_dlaunch LP{};
    LP.regions = r->d_self;
    LP.items = nullptr;
    LP.n_regions = 1;
    fill_single(LP, r, r->desc);
    const dsr_dconfig C = make_dconfig(c, c->cfg.wg_size, c->cfg.lds_slab_bytes, c->cfg.overflow_threshold,
                                       c->cfg.master_joins, (c->cfg.flags & DSR_F_TRACE) ? 1u : 0u);
    /* events only when timing is asked for: a marker between back-to-back
     * launches costs about as much as a small region's fixed overhead */
    const bool timing = (c->cfg.flags & DSR_F_TIMING) != 0;
    if (timing && hipEventRecord(r->ev0, s) != hipSuccess) return DSR_E_HIP;
    if (dsr_launch_region_kernel(&LP, &C, (uint32_t)r->teams, c->cfg.wg_size, c->lds_bytes,
                                 single_variant(r, c->cfg.wg_size), stream) != 0)
        return DSR_E_HIP;
    if (timing && hipEventRecord(r->ev1, s) != hipSuccess) return DSR_E_HIP;
    r->stream = s;
    r->timed = timing;
    r->launched = true;
    r->have_result = false;
    return DSR_OK;
}

/* Wait for a region's last launch: its end event when it was timed, else
 * everything queued on its stream so far. */
static int wait_launch(dsr_region *r)
{
    const hipError_t e = r->timed ? hipEventSynchronize(r->ev1) : hipStreamSynchronize(r->stream);
    return e == hipSuccess ? DSR_OK : DSR_E_HIP;
}

extern "C" int dsr_region_sync(dsr_region *r)
{
    if (!r) return DSR_E_INVAL;
    if (!r->launched) return DSR_E_STATE;
    /* only the leading host fields of the result block, into pinned memory
     * on the launch's stream: a synchronous copy of the whole block from
     * pageable memory cost 13 us of a small region's launch-and-sync time */
    if (!r->h_pin && hipHostMalloc((void **)&r->h_pin, sizeof(dsr_dresult), hipHostMallocDefault) != hipSuccess)
        r->h_pin = nullptr;
    if (r->h_pin) {
        if (hipMemcpyAsync(r->h_pin, r->d_result, DSR_RESULT_HOST_BYTES, hipMemcpyDeviceToHost, r->stream) !=
                hipSuccess ||
            hipStreamSynchronize(r->stream) != hipSuccess)
            return DSR_E_HIP;
        std::memcpy(&r->h_result, r->h_pin, DSR_RESULT_HOST_BYTES);
    } else {
        if (wait_launch(r)) return DSR_E_HIP;
        if (hipMemcpy(&r->h_result, r->d_result, DSR_RESULT_HOST_BYTES, hipMemcpyDeviceToHost) != hipSuccess)
            return DSR_E_HIP;
    }
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
    if (wait_launch(r)) return DSR_E_HIP;
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
    if (r->serve_refs) return DSR_E_STATE;
    if (r->launched) (void)wait_launch(r);
    if (r->d_ops) hipFree(r->d_ops);
    if (r->d_loops) hipFree(r->d_loops);
    if (r->d_init) hipFree(r->d_init);
    if (r->d_partials) hipFree(r->d_partials);
    if (r->d_result) hipFree(r->d_result);
    if (r->d_trace) hipFree(r->d_trace);
    if (r->d_self) hipFree(r->d_self);
    if (r->h_pin) hipHostFree(r->h_pin);
    if (r->ev0) hipEventDestroy(r->ev0);
    if (r->ev1) hipEventDestroy(r->ev1);
    delete r;
    return DSR_OK;
}

/* ---- launch without allocation ------------------------------------------------ */
namespace {

struct static_layout {
    size_t desc, ops, loops, init, partials, result, hbm, nest, total;
    bool nested;
};

size_t up256(size_t v) { return (v + 255u) & ~(size_t)255u; }

/* Where each device buffer of region r goes in the fixed workspace. */
static_layout static_plan(const dsr_region *r)
{
    static_layout L{};
    L.nested = false;
    for (const dsr_op &op : r->ops)
        if (op.kind == DSR_OP_PUBLISH && op.body == DSR_BODY_GATHER_NESTED) L.nested = true;
    size_t o = 0;
    L.desc = o;
    o = up256(o + sizeof(dsr_dregion));
    L.ops = o;
    o = up256(o + std::max<size_t>(1, r->ops.size()) * sizeof(dsr_op));
    L.loops = o;
    o = up256(o + std::max<size_t>(1, r->loops.size()) * sizeof(dsr_dloop));
    L.init = o;
    o = up256(o + std::max<size_t>(16, r->init.size()));
    L.partials = o;
    o = up256(o + (size_t)(r->n_red ? r->n_red : 1) * r->teams * DSR_PART_WORDS * sizeof(uint64_t));
    L.result = o;
    o = up256(o + sizeof(dsr_dresult));
    L.hbm = o;
    o = up256(o + (size_t)r->teams * r->ctx->cfg.hbm_slab_bytes);
    L.nest = o;
    if (L.nested) o = up256(o + (size_t)r->teams * DSR_NEST_SLOT);
    L.total = o;
    return L;
}

}  // namespace

extern "C" uint64_t dsr_static_bytes(const dsr_region *r)
{
    return r ? (uint64_t)static_plan(r).total : 0;
}

extern "C" int dsr_launch_static(dsr_region *r, dsr_result_rec *result, void *stream)
{
    static_assert(DSR_MAX_RED == 8, "dsr_result_rec holds eight reductions");
    if (!r || !result) return DSR_E_INVAL;
    if (!r->live.empty()) return DSR_E_LIVE;
    dsr_ctx *c = r->ctx;
    if ((uint64_t)r->teams > c->cfg.max_teams) return DSR_E_INVAL;
    const static_layout L = static_plan(r);
    if (L.total > DSR_STATIC_SCRATCH_BYTES) return DSR_E_NOMEM;
    int dev = c->device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return DSR_E_HIP;
    if (hipSetDevice(dev) != hipSuccess) return DSR_E_HIP;
    uint8_t *ws = nullptr;
    int rc = dsr_static_workspace(dev, &ws);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    dsr_dregion &R = r->static_desc;
    R = dsr_dregion{};
    R.ops = (const dsr_op *)(ws + L.ops);
    R.loops = (const dsr_dloop *)(ws + L.loops);
    R.init = ws + L.init;
    R.partials = (uint64_t *)(ws + L.partials);
    R.result = (dsr_dresult *)(ws + L.result);
    R.trace = nullptr;
    R.n_ops = (uint32_t)r->ops.size();
    R.teams = (uint32_t)r->teams;
    R.n_red = r->n_red;
    R.red_kind_mask = r->red_kind_mask;
    R.n_loops = (uint32_t)r->loops.size();
    R.init_size = (uint32_t)r->init.size();
    R.relay = nullptr;
    R.relay_flag = nullptr;
    if (hipMemcpyAsync(ws + L.desc, &R, sizeof(R), hipMemcpyHostToDevice, s) != hipSuccess) return DSR_E_HIP;
    if (!r->ops.empty() &&
        hipMemcpyAsync(ws + L.ops, r->ops.data(), r->ops.size() * sizeof(dsr_op), hipMemcpyHostToDevice, s) !=
            hipSuccess)
        return DSR_E_HIP;
    if (!r->loops.empty() &&
        hipMemcpyAsync(ws + L.loops, r->loops.data(), r->loops.size() * sizeof(dsr_dloop), hipMemcpyHostToDevice,
                       s) != hipSuccess)
        return DSR_E_HIP;
    if (!r->init.empty() &&
        hipMemcpyAsync(ws + L.init, r->init.data(), r->init.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return DSR_E_HIP;
    /* counters, error word and arrival tree start at zero; partials and
     * stacks are written before they are read */
    if ((rc = dsr_static_fill(ws + L.result, sizeof(dsr_dresult) / 4, 0u, stream))) return rc;
    dsr_dlaunch LP{};
    LP.regions = (const dsr_dregion *)(ws + L.desc);
    LP.items = nullptr;
    LP.n_regions = 1;
    fill_single(LP, r, R);
    dsr_dconfig C = make_dconfig(c, c->cfg.wg_size, c->cfg.lds_slab_bytes, c->cfg.overflow_threshold,
                                 c->cfg.master_joins, 0u);
    C.hbm_base = ws + L.hbm;
    C.nest_base = L.nested ? ws + L.nest : nullptr;
    if (dsr_launch_region_kernel(&LP, &C, (uint32_t)r->teams, c->cfg.wg_size, c->lds_bytes,
                                 single_variant(r, c->cfg.wg_size), stream) != 0)
        return DSR_E_HIP;
    return dsr_static_copy_result(ws + L.result, r->n_red, result, stream);
}

/* ---- batched form ---------------------------------------------------------- */
struct dsr_batch {
    dsr_ctx *ctx;
    int32_t n;
    uint8_t *d_arena;
    dsr_dregion *d_regions;
    dsr_dresult *d_results;
    uint32_t *d_items;
    uint32_t n_items;
    uint32_t *d_counter;
    uint64_t *d_done;
    std::vector<int32_t> teams;
    std::vector<uint32_t> n_red;
    std::vector<std::vector<dsr_dloop>> loops;   /* host copies, for tune checks */
    std::vector<uint32_t> stack_peak;            /* per region: its stack's peak bytes */
    std::vector<dsr_dresult> h_results;
    uint8_t *h_pin;                     /* pinned: n leading host parts of the results */
    bool have_results;
    uint32_t variant;
    dsr_tune tune;
    uint32_t grid;
    uint32_t lds_bytes;
    uint32_t lds_max;
    uint32_t cus;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t own_stream;
    hipEvent_t ev0, ev1;
    int last;                                    /* 1 persistent, 2 one per region */
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

extern "C" int dsr_batch_create(dsr_ctx *ctx, dsr_region *const *regions, int32_t n, dsr_batch **out)
{
    if (!ctx || !regions || !out || n < 1) return DSR_E_INVAL;
    *out = nullptr;
    if (ctx->device < 0) return DSR_E_STATE;
    for (int32_t i = 0; i < n; ++i) {
        if (!regions[i] || regions[i]->ctx != ctx) return DSR_E_INVAL;
        if (!regions[i]->live.empty()) return DSR_E_LIVE;
    }
    /* arena layout */
    size_t off_ops = 0, sz = 0;
    std::vector<size_t> o_ops(n), o_loops(n), o_init(n), o_part(n);
    for (int32_t i = 0; i < n; ++i) { o_ops[i] = sz; sz += regions[i]->ops.size() * sizeof(dsr_op); }
    sz = align256(sz);
    for (int32_t i = 0; i < n; ++i) { o_loops[i] = sz; sz += regions[i]->loops.size() * sizeof(dsr_dloop); }
    sz = align256(sz);
    for (int32_t i = 0; i < n; ++i) { o_init[i] = sz; sz += (regions[i]->init.size() + 15) & ~(size_t)15; }
    sz = align256(sz);
    for (int32_t i = 0; i < n; ++i) {
        o_part[i] = sz;
        sz += (size_t)(regions[i]->n_red ? regions[i]->n_red : 1) * regions[i]->teams * DSR_PART_WORDS * sizeof(uint64_t);
    }
    sz = align256(sz);
    const size_t o_res = sz;
    sz = align256(sz + (size_t)n * sizeof(dsr_dresult));
    const size_t o_reg = sz;
    sz = align256(sz + (size_t)n * sizeof(dsr_dregion));
    /* items: (region, team), largest per-team work first */
    struct item { uint64_t work; uint32_t r, t; };
    std::vector<item> items;
    for (int32_t i = 0; i < n; ++i) {
        const dsr_region *r = regions[i];
        for (int32_t t = 0; t < r->teams; ++t) {
            uint64_t w = 0;
            for (const dsr_dloop &L : r->loops) {
                const uint64_t lo = std::min(L.dyn_start, (uint64_t)t * L.chunk);
                const uint64_t hi = std::min(L.dyn_start, lo + L.chunk);
                w += hi - lo;
            }
            items.push_back(item{w, (uint32_t)i, (uint32_t)t});
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const item &a, const item &b) { return a.work > b.work; });
    const size_t o_items = sz;
    sz = align256(sz + items.size() * 2 * sizeof(uint32_t));
    const size_t o_counter = sz;
    sz = align256(sz + 2 * sizeof(uint32_t));
    const size_t o_done = sz;
    sz = align256(sz + ((size_t)n + 1) * sizeof(uint64_t));
    (void)off_ops;

    dsr_batch *b = new (std::nothrow) dsr_batch();
    if (!b) return DSR_E_NOMEM;
    b->ctx = ctx;
    b->n = n;
    b->graph = nullptr;
    b->exec = nullptr;
    b->own_stream = nullptr;
    b->ev0 = b->ev1 = nullptr;
    b->last = 0;
    b->have_results = false;
    b->h_pin = nullptr;
    b->variant = 0;
    std::vector<uint8_t> stage;
    try {
        stage.assign(sz, 0);
        b->teams.resize(n);
        b->n_red.resize(n);
        b->loops.resize(n);
        b->stack_peak.resize(n);
        b->h_results.resize(n);
    } catch (...) {
        delete b;
        return DSR_E_NOMEM;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) { delete b; return DSR_E_HIP; }
    if (hipMalloc((void **)&b->d_arena, sz) != hipSuccess) { delete b; return DSR_E_NOMEM; }
    uint8_t *A = b->d_arena;
    for (int32_t i = 0; i < n; ++i) {
        const dsr_region *r = regions[i];
        if (!r->ops.empty()) std::memcpy(stage.data() + o_ops[i], r->ops.data(), r->ops.size() * sizeof(dsr_op));
        if (!r->loops.empty())
            std::memcpy(stage.data() + o_loops[i], r->loops.data(), r->loops.size() * sizeof(dsr_dloop));
        if (!r->init.empty()) std::memcpy(stage.data() + o_init[i], r->init.data(), r->init.size());
        dsr_dregion R{};
        R.ops = (const dsr_op *)(A + o_ops[i]);
        R.loops = (const dsr_dloop *)(A + o_loops[i]);
        R.init = A + o_init[i];
        R.partials = (uint64_t *)(A + o_part[i]);
        R.result = (dsr_dresult *)(A + o_res) + i;
        R.trace = nullptr;
        R.n_ops = (uint32_t)r->ops.size();
        R.teams = (uint32_t)r->teams;
        R.n_red = r->n_red;
        R.red_kind_mask = r->red_kind_mask;
        R.n_loops = (uint32_t)r->loops.size();
        R.init_size = (uint32_t)r->init.size();
        std::memcpy(stage.data() + o_reg + (size_t)i * sizeof(dsr_dregion), &R, sizeof(R));
        b->teams[i] = r->teams;
        b->n_red[i] = r->n_red;
        b->loops[i] = r->loops;
        b->variant = std::max(b->variant, r->variant);
        uint64_t lp = 0, hp = 0;
        (void)stack_peaks(r, 0xFFFFFFFFu, 0xFFFFFFFFu, ~0ull, &lp, &hp);
        b->stack_peak[i] = (uint32_t)std::min<uint64_t>(lp + hp, 0xFFFFFFFFull);
    }
    uint32_t *it = (uint32_t *)(stage.data() + o_items);
    for (size_t k = 0; k < items.size(); ++k) { it[2 * k] = items[k].r; it[2 * k + 1] = items[k].t; }
    if (hipMemcpy(b->d_arena, stage.data(), sz, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(b->d_arena);
        delete b;
        return DSR_E_HIP;
    }
    b->d_regions = (dsr_dregion *)(A + o_reg);
    b->d_results = (dsr_dresult *)(A + o_res);
    b->d_items = (uint32_t *)(A + o_items);
    b->n_items = (uint32_t)items.size();
    b->d_counter = (uint32_t *)(A + o_counter);
    b->d_done = (uint64_t *)(A + o_done);
    int v = 0;
    b->lds_max = kDefaultLdsPerWg;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) == hipSuccess && v > 0)
        b->lds_max = (uint32_t)v;
    b->cus = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, ctx->device) == hipSuccess && v > 0)
        b->cus = (uint32_t)v;
    if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
        dsr_batch_free(b);
        return DSR_E_HIP;
    }
    dsr_tune t{ctx->cfg.wg_size, ctx->cfg.lds_slab_bytes, ctx->cfg.overflow_threshold, ctx->cfg.master_joins, 0, 0};
    const int rc = dsr_batch_tune(b, &t);
    if (rc) {
        dsr_batch_free(b);
        return rc;
    }
    *out = b;
    return DSR_OK;
}

static void drop_graph(dsr_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

extern "C" int dsr_batch_tune(dsr_batch *b, const dsr_tune *tune)
{
    if (!b || !tune) return DSR_E_INVAL;
    dsr_tune t = *tune;
    if (t.wg_size < 64 || t.wg_size > 1024 || (t.wg_size & 63u)) return DSR_E_INVAL;
    if (t.lds_slab_bytes & 15u) return DSR_E_INVAL;
    const uint32_t nw = t.wg_size / 64;
    const uint64_t lds = (uint64_t)dsr::cb_bytes(nw) + t.lds_slab_bytes;
    if (lds > b->lds_max) return DSR_E_LDS;
    if (nw == 1) t.master_joins = 1;
    if (nw > 8) t.master_joins = 0;
    /* the static share of a lane must stay within the exact bins' range */
    const uint64_t lanes = 64ull * (t.master_joins ? nw : nw - 1);
    for (int32_t i = 0; i < b->n; ++i)
        for (const dsr_dloop &L : b->loops[i])
            if ((L.chunk + lanes - 1) / lanes > (1ull << 15)) return DSR_E_INVAL;
    const uint32_t variant = t.wg_size > 256 ? 0 : b->variant;
    uint32_t grid = t.grid;
    if (grid == 0) {
        const int occ = dsr_region_kernel_occupancy(t.wg_size, (uint32_t)lds, variant);
        if (occ <= 0) return DSR_E_LDS;
        grid = (uint32_t)occ * (b->cus ? b->cus : 1);
        grid = std::min(grid, b->ctx->cfg.max_teams);
    }
    grid = std::min(grid, b->n_items);
    if (grid > b->ctx->cfg.max_teams) return DSR_E_NOMEM;
    drop_graph(b);
    t.grid = grid;
    b->tune = t;
    b->grid = grid;
    b->lds_bytes = (uint32_t)lds;
    return DSR_OK;
}

extern "C" int dsr_batch_get_tune(dsr_batch *b, dsr_tune *out)
{
    if (!b || !out) return DSR_E_INVAL;
    *out = b->tune;
    return DSR_OK;
}

static int batch_kernel(dsr_batch *b, hipStream_t s)
{
    dsr_dlaunch LP{};
    LP.regions = b->d_regions;
    LP.items = b->d_items;
    LP.n_items = b->n_items;
    LP.n_regions = (uint32_t)b->n;
    LP.counter = b->d_counter;
    LP.done_ts = b->d_done;
    const dsr_dconfig C = make_dconfig(b->ctx, b->tune.wg_size, b->tune.lds_slab_bytes,
                                       b->tune.overflow_threshold, b->tune.master_joins, 0);
    return dsr_launch_region_kernel(&LP, &C, b->grid, b->tune.wg_size, b->lds_bytes, b->variant, s) ? DSR_E_HIP
                                                                                                     : DSR_OK;
}

extern "C" int dsr_batch_launch(dsr_batch *b, void *stream)
{
    if (!b) return DSR_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    if (b->tune.use_graph) {
        if (!s) {
            if (!b->own_stream && hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking) != hipSuccess)
                return DSR_E_HIP;
            s = b->own_stream;
        }
        if (!b->exec) {
            if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) return DSR_E_HIP;
            const int rc = batch_kernel(b, s);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &g);
            if (rc || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return DSR_E_HIP;
            }
            b->graph = g;
            if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
                drop_graph(b);
                return DSR_E_HIP;
            }
        }
        if (hipEventRecord(b->ev0, s) != hipSuccess) return DSR_E_HIP;
        if (hipGraphLaunch(b->exec, s) != hipSuccess) return DSR_E_HIP;
        if (hipEventRecord(b->ev1, s) != hipSuccess) return DSR_E_HIP;
    } else {
        if (hipEventRecord(b->ev0, s) != hipSuccess) return DSR_E_HIP;
        const int rc = batch_kernel(b, s);
        if (rc) return rc;
        if (hipEventRecord(b->ev1, s) != hipSuccess) return DSR_E_HIP;
    }
    b->last = 1;
    b->have_results = false;
    return DSR_OK;
}

extern "C" int dsr_batch_launch_each(dsr_batch *b, void *stream)
{
    if (!b) return DSR_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const dsr_dconfig C = make_dconfig(b->ctx, b->tune.wg_size, b->tune.lds_slab_bytes,
                                       b->tune.overflow_threshold, b->tune.master_joins, 0);
    const uint32_t variant = b->tune.wg_size > 256 ? 0 : b->variant;
    if (hipEventRecord(b->ev0, s) != hipSuccess) return DSR_E_HIP;
    for (int32_t i = 0; i < b->n; ++i) {
        dsr_dlaunch LP{};
        LP.regions = b->d_regions + i;
        LP.items = nullptr;
        LP.n_regions = 1;
        LP.done_ts = b->d_done + i;                  /* region i's completion */
        LP.start_ts = i == 0 ? b->d_done + b->n : nullptr;
        if (dsr_launch_region_kernel(&LP, &C, (uint32_t)b->teams[i], b->tune.wg_size, b->lds_bytes, variant, s))
            return DSR_E_HIP;
    }
    if (hipEventRecord(b->ev1, s) != hipSuccess) return DSR_E_HIP;
    b->last = 2;
    b->have_results = false;
    return DSR_OK;
}

/* Copy the leading host part of every region's result block (one strided
 * copy into pinned memory; the device-side counters stay behind): copying
 * the whole blocks of a 10,000-region batch moved 24 MB per sync. */
static int copy_batch_results(dsr_batch *b)
{
    const size_t hb = DSR_RESULT_HOST_BYTES;
    if (!b->h_pin && hipHostMalloc((void **)&b->h_pin, hb * (size_t)b->n, hipHostMallocDefault) != hipSuccess)
        b->h_pin = nullptr;
    if (b->h_pin) {
        if (hipMemcpy2D(b->h_pin, hb, b->d_results, sizeof(dsr_dresult), hb, (size_t)b->n,
                        hipMemcpyDeviceToHost) != hipSuccess)
            return DSR_E_HIP;
        for (int32_t i = 0; i < b->n; ++i) std::memcpy(&b->h_results[i], b->h_pin + hb * (size_t)i, hb);
    } else if (hipMemcpy2D(b->h_results.data(), sizeof(dsr_dresult), b->d_results, sizeof(dsr_dresult), hb,
                           (size_t)b->n, hipMemcpyDeviceToHost) != hipSuccess) {
        return DSR_E_HIP;
    }
    return DSR_OK;
}

extern "C" int dsr_batch_sync(dsr_batch *b)
{
    if (!b) return DSR_E_INVAL;
    if (!b->last) return DSR_E_STATE;
    if (hipEventSynchronize(b->ev1) != hipSuccess) return DSR_E_HIP;
    if (copy_batch_results(b) != DSR_OK) return DSR_E_HIP;
    b->have_results = true;
    for (int32_t i = 0; i < b->n; ++i)
        if (b->h_results[i].final_error) return b->h_results[i].final_error;
    return DSR_OK;
}

extern "C" int dsr_batch_result(dsr_batch *b, int32_t r, int32_t index, int64_t *i64, double *f64,
                                uint64_t *fixed3, int32_t *status)
{
    if (!b) return DSR_E_INVAL;
    if (!b->have_results) return DSR_E_STATE;
    if (r < 0 || r >= b->n || index < 0 || (uint32_t)index >= b->n_red[r]) return DSR_E_INVAL;
    const dsr_dresult &R = b->h_results[r];
    if (i64) *i64 = R.i64[index];
    if (f64) *f64 = R.f64[index];
    if (fixed3) for (int k = 0; k < 3; ++k) fixed3[k] = R.fixed[index][k];
    if (status) *status = R.final_error;
    return DSR_OK;
}

extern "C" int dsr_batch_times(dsr_batch *b, double *us, int32_t n)
{
    if (!b || !us || n < b->n) return DSR_E_INVAL;
    if (b->last != 1 && b->last != 2) return DSR_E_STATE;
    if (hipEventSynchronize(b->ev1) != hipSuccess) return DSR_E_HIP;
    std::vector<uint64_t> t((size_t)b->n + 1);
    if (hipMemcpy(t.data(), b->d_done, t.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return DSR_E_HIP;
    for (int32_t i = 0; i < b->n; ++i) us[i] = ((double)t[i] - (double)t[b->n]) / 100.0;
    return DSR_OK;
}

extern "C" int dsr_batch_elapsed(dsr_batch *b, float *ms)
{
    if (!b || !ms) return DSR_E_INVAL;
    if (!b->last) return DSR_E_STATE;
    if (hipEventSynchronize(b->ev1) != hipSuccess) return DSR_E_HIP;
    return hipEventElapsedTime(ms, b->ev0, b->ev1) == hipSuccess ? DSR_OK : DSR_E_HIP;
}

extern "C" int dsr_batch_free(dsr_batch *b)
{
    if (!b) return DSR_E_INVAL;
    if (b->last && b->ev1) (void)hipEventSynchronize(b->ev1);
    drop_graph(b);
    if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->d_arena) (void)hipFree(b->d_arena);
    if (b->h_pin) (void)hipHostFree(b->h_pin);
    delete b;
    return DSR_OK;
}

/* The occupancy model's parameters for `device` (gfx950: 4 SIMDs, each
 * with 512 VGPRs (arch + acc) per lane, allocated in 8s). */
static int device_model(int device, dsr_hw_model *hw)
{
    hipDeviceProp_t p{};
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return DSR_E_HIP;
    if (p.multiProcessorCount <= 0 || p.maxThreadsPerMultiProcessor <= 0 || p.warpSize <= 0) return DSR_E_HIP;
    const uint32_t wave = (uint32_t)p.warpSize, thr = (uint32_t)p.maxThreadsPerMultiProcessor;
    *hw = dsr_hw_model{(uint32_t)p.multiProcessorCount, 4u * 512u * wave, 8u, thr / wave, thr,
                       (uint32_t)p.maxSharedMemoryPerMultiProcessor, 128u, 4u, wave};
    return DSR_OK;
}

extern "C" int dsr_autotune_plan(dsr_batch *b, dsr_tune *out, int32_t max, int32_t *n_out)
{
    if (!b || !n_out || max < 0 || (max > 0 && !out)) return DSR_E_INVAL;
    *n_out = 0;
    dsr_hw_model hw{};
    int rc = device_model(b->ctx->device, &hw);
    if (rc) return rc;
    /* stack sizes the batch's frames ask for: the peaks at the median, the
     * 90th, 99th percentile and the largest, rounded up to 1 KiB */
    std::vector<uint32_t> peaks = b->stack_peak;
    std::sort(peaks.begin(), peaks.end());
    std::vector<uint32_t> slabs;
    for (double q : {0.5, 0.9, 0.99, 1.0}) {
        const uint32_t v = peaks.empty() ? 0u : peaks[std::min(peaks.size() - 1, (size_t)(q * (peaks.size() - 1)))];
        slabs.push_back(std::max(1024u, (v + 1023u) & ~1023u));
    }
    struct cand { dsr_tune t; uint32_t waves; };
    std::vector<cand> keep;
    for (uint32_t wg : {64u, 128u, 256u, 512u, 1024u}) {
        const uint32_t nw = wg / 64;
        const uint32_t variant = wg > 256 ? 0 : b->variant;
        const int regs = dsr_region_kernel_regs(wg, variant);
        if (regs <= 0) continue;
        /* per occupancy the largest slab: it keeps more frames on chip at
         * no cost in resident teams */
        std::vector<std::pair<uint32_t, uint32_t>> best;   /* (teams per CU, slab) */
        for (uint32_t slab : slabs) {
            const uint32_t room = b->lds_max > dsr::cb_bytes(nw) ? b->lds_max - dsr::cb_bytes(nw) : 0u;
            const uint32_t sl = std::min(slab, room & ~15u);
            dsr_occupancy o{};
            if (dsr_occupancy_model(&hw, wg, (uint32_t)regs, dsr::cb_bytes(nw) + sl, &o) || o.teams_per_cu == 0)
                continue;
            bool placed = false;
            for (auto &e : best)
                if (e.first == o.teams_per_cu) { e.second = std::max(e.second, sl); placed = true; }
            if (!placed) best.push_back({o.teams_per_cu, sl});
        }
        for (const auto &e : best)
            for (uint32_t joins : {0u, 1u}) {
                if ((nw == 1 && !joins) || (nw > 8 && joins)) continue;
                const uint32_t working = joins ? nw : nw - 1;
                cand c;
                c.t = dsr_tune{wg, e.second, 0u, joins, 0u, 1u};
                c.waves = e.first * working;
                keep.push_back(c);
            }
    }
    /* most working waves resident per CU first */
    std::stable_sort(keep.begin(), keep.end(), [](const cand &a, const cand &c) { return a.waves > c.waves; });
    const int32_t n = std::min<int32_t>(max, (int32_t)keep.size());
    for (int32_t k = 0; k < n; ++k) out[k] = keep[k].t;
    *n_out = (int32_t)keep.size();
    return DSR_OK;
}

extern "C" int dsr_autotune(dsr_batch *b, const dsr_tune *cand, int32_t n_cand, int32_t reps, void *stream,
                            dsr_tune *best, float *ms)
{
    if (!b || !cand || n_cand < 1 || reps < 1) return DSR_E_INVAL;
    const dsr_tune keep = b->tune;
    int32_t best_i = -1;
    float best_ms = 0;
    hipStream_t s = (hipStream_t)stream;
    for (int32_t i = 0; i < n_cand; ++i) {
        if (ms) ms[i] = -1.0f;
        if (dsr_batch_tune(b, &cand[i]) != DSR_OK) continue;
        int rc = dsr_batch_launch(b, s);                /* warm-up (and graph capture) */
        if (rc == DSR_OK) rc = dsr_batch_sync(b);
        if (rc != DSR_OK) continue;
        float tot = 0;
        bool ok = true;
        for (int32_t k = 0; k < reps && ok; ++k) {
            float t = 0;
            ok = dsr_batch_launch(b, s) == DSR_OK && dsr_batch_elapsed(b, &t) == DSR_OK;
            tot += t;
        }
        if (!ok) continue;
        const float m = tot / reps;
        if (ms) ms[i] = m;
        if (best_i < 0 || m < best_ms) { best_i = i; best_ms = m; }
    }
    if (best_i < 0) {
        (void)dsr_batch_tune(b, &keep);
        return DSR_E_INVAL;
    }
    const int rc = dsr_batch_tune(b, &cand[best_i]);
    if (best) *best = b->tune;
    return rc;
}

/* ---- served form ------------------------------------------------------------ */
namespace {

struct serve_slot {
    dsr_dregion *desc;      /* host-coherent: the slot's head (descriptor, ops, loops) */
    dsr_op *ops;            /* host-coherent */
    dsr_dloop *loops;       /* host-coherent */
    uint8_t *init;          /* host-coherent */
    uint64_t *d_partials;   /* device */
    dsr_dresult *d_result;  /* device */
    uint8_t *d_img;         /* device: relayed frame images */
    dsr_region *tmpl;       /* frozen template whose device images the request reads */
    uint64_t *d_flag;       /* device: ticket whose images d_img holds */
    bool busy;
    uint64_t ticket;
    uint32_t first_item;    /* in its class's item ring */
    uint32_t cls;           /* LDS class running the request */
    uint64_t lds_cost, hbm_cost;
};

/* Peak LDS and HBM stack bytes one team of `r` needs under the device's
 * placement rule; false if some frame fits neither space. */
bool stack_peaks(const dsr_region *r, uint32_t lds_cap, uint32_t threshold, uint64_t hbm_cap,
                 uint64_t *lds_peak, uint64_t *hbm_peak)
{
    uint64_t spl = 0, sph = 0;
    *lds_peak = 0;
    *hbm_peak = 0;
    std::vector<std::pair<int, uint64_t>> live;
    for (const dsr_op &op : r->ops) {
        if (op.kind == DSR_OP_PUSH) {
            const uint64_t size = ((uint64_t)op.nbytes + 15) & ~15ull;
            if (size <= threshold && spl + size <= lds_cap) {
                spl += size;
                live.push_back({0, size});
            } else if (sph + size <= hbm_cap) {
                sph += size;
                live.push_back({1, size});
            } else {
                return false;
            }
            *lds_peak = std::max(*lds_peak, spl);
            *hbm_peak = std::max(*hbm_peak, sph);
        } else if (op.kind == DSR_OP_POP && !live.empty()) {
            if (live.back().first == 0) spl -= live.back().second; else sph -= live.back().second;
            live.pop_back();
        } else if (op.kind == DSR_OP_PUBLISH && op.body == DSR_BODY_FMA_CHAIN_REFS &&
                   (op.nbytes > DSR_LIST_ONCHIP || (r->ctx->cfg.flags & DSR_F_GLOBAL_LISTS))) {
            /* a global reference list lives on the HBM stack for the region */
            const uint64_t size = (8ull * op.nbytes + 15) & ~15ull;
            if (sph + size > hbm_cap) return false;
            *hbm_peak = std::max(*hbm_peak, sph + size);
        }
    }
    return true;
}

}  // namespace

/* One LDS class of the server: a resident grid whose teams have `slab`
 * bytes of on-chip stack, with its own item ring, published count, close
 * handshake and stream.  Slots, completion records and tickets are shared
 * by every class. */
struct serve_class {
    uint32_t slab, grid, lds_bytes, first_wg;
    uint8_t *h_ctl;                   /* host-coherent: published, closing, final
                                         count, start/exit flags, item ring     */
    uint32_t *published;
    uint32_t *closing;                /* device: the class is closing           */
    uint32_t *final_items;            /* device: 1 + items served (0 = open)    */
    uint32_t *relays;                 /* device: relayed requests, relay time-outs */
    uint32_t *wg_started;             /* per resident workgroup                 */
    uint32_t *wg_exited;
    uint32_t *items;
    uint32_t *d_counter;              /* device control words                   */
    uint32_t pub;
    uint64_t lds_budget, lds_used;
    hipStream_t stream;
};

struct dsr_server {
    dsr_ctx *ctx;
    dsr_serve_cfg cfg;
    uint8_t *h_block;                 /* host-coherent: stop, start ticks,
                                         completion records                    */
    uint32_t *stop;
    uint64_t *start_ticks;
    dsr_drec *recs;
    uint8_t *h_arena;                 /* host-coherent slot arenas            */
    uint8_t *d_arena;                 /* device: partials, results, counters  */
    std::vector<serve_slot> slots;
    std::vector<uint32_t> free_slots;
    std::vector<serve_class> cls;
    uint64_t next_ticket;
    uint64_t hbm_budget, hbm_used;
    uint32_t variant;
    dsr_tune tune;
    uint32_t in_flight;
};

namespace {

void serve_free(dsr_server *S)
{
    /* the kernels have ended: uncollected requests read no template now */
    for (serve_slot &sl : S->slots)
        if (sl.busy && sl.tmpl) sl.tmpl->serve_refs--;
    for (serve_class &k : S->cls) {
        if (k.stream) (void)hipStreamDestroy(k.stream);
        if (k.h_ctl) (void)hipHostFree(k.h_ctl);
    }
    if (S->d_arena) (void)hipFree(S->d_arena);
    if (S->h_arena) (void)hipHostFree(S->h_arena);
    if (S->h_block) (void)hipHostFree(S->h_block);
    delete S;
}

/* Bytes of a region's stack at the most with every frame on chip (each
 * frame rounded to the kernel's 16 bytes). */
uint64_t full_stack(const dsr_region *r)
{
    uint64_t lp = 0, hp = 0;
    (void)stack_peaks(r, 0xFFFFFFFFu, 0xFFFFFFFFu, ~0ull, &lp, &hp);
    return lp;
}

}  // namespace

extern "C" int dsr_serve_class_for(const uint32_t *slabs, int32_t n, const dsr_region *r)
{
    if (!slabs || n < 1 || n > DSR_SERVE_CLASSES || !r) return DSR_E_INVAL;
    const uint64_t need = full_stack(r);
    int32_t best = -1;
    for (int32_t k = 0; k < n; ++k)
        if (slabs[k] >= need && (best < 0 || slabs[k] < slabs[best])) best = k;
    if (best >= 0) return best;
    for (int32_t k = 0; k < n; ++k)
        if (best < 0 || slabs[k] > slabs[best]) best = k;
    return best;
}

extern "C" int dsr_serve_start(dsr_ctx *ctx, const dsr_serve_cfg *cfg, dsr_server **out)
{
    if (!ctx || !cfg || !out) return DSR_E_INVAL;
    *out = nullptr;
    if (ctx->device < 0) return DSR_E_STATE;
    dsr_serve_cfg c = *cfg;
    /* a ring item holds the slot and the team in 16 bits each */
    if (c.slots == 0 || c.slots > 65536 || c.max_teams == 0 || c.max_teams > 65535 || c.slot_bytes == 0)
        return DSR_E_INVAL;
    if (c.ring_items == 0) c.ring_items = 1u << 16;
    if (c.ring_items & (c.ring_items - 1)) return DSR_E_INVAL;
    if ((uint64_t)c.slots * c.max_teams > c.ring_items) return DSR_E_INVAL;
    if (c.idle_ms == 0) c.idle_ms = 10000;
    if (c.budget_pct == 0 || c.budget_pct > 100) c.budget_pct = 100;
    if (c.n_classes > DSR_SERVE_CLASSES) return DSR_E_INVAL;
    dsr_tune t = c.tune;
    if (t.wg_size < 64 || t.wg_size > 1024 || (t.wg_size & 63u) || (t.lds_slab_bytes & 15u)) return DSR_E_INVAL;
    const uint32_t nw = t.wg_size / 64;
    if (nw == 1) t.master_joins = 1;
    if (nw > 8) t.master_joins = 0;
    int v = 0;
    uint32_t lds_max = kDefaultLdsPerWg, cus = 1;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) == hipSuccess && v > 0)
        lds_max = (uint32_t)v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, ctx->device) == hipSuccess && v > 0)
        cus = (uint32_t)v;
    const uint32_t variant = 0;
    /* the classes: one of the tune's slab and grid, or those given */
    const uint32_t n_cls = c.n_classes ? c.n_classes : 1u;
    std::vector<serve_class> cls(n_cls);
    uint32_t grid_total = 0;
    for (uint32_t k = 0; k < n_cls; ++k) {
        serve_class &K = cls[k];
        K = serve_class{};
        K.slab = c.n_classes ? c.class_slab[k] : t.lds_slab_bytes;
        if (K.slab & 15u) return DSR_E_INVAL;
        const uint64_t lds = (uint64_t)dsr::cb_bytes(nw) + K.slab + DSR_SERVE_AREA_BYTES;
        if (lds > lds_max) return DSR_E_LDS;
        K.lds_bytes = (uint32_t)lds;
        uint32_t grid = c.n_classes ? c.class_grid[k] : t.grid;
        if (grid == 0) {
            /* as many as fit less one workgroup slot per CU (one CU per 32
             * when only one fits), shared evenly between the classes.  The
             * runtime runs its copies as kernels of its own: with every
             * slot held by the resident grid a copy issued meanwhile, on
             * any stream, waits until the server closes (measured: a
             * device-to-host copy blocked for the whole idle limit at full
             * occupancy and took 0.6 ms with one slot per CU free). */
            const int occ = dsr_region_kernel_occupancy(t.wg_size, K.lds_bytes, variant);
            if (occ <= 0) return DSR_E_LDS;
            const uint32_t slots_all = (uint32_t)occ * cus;
            const uint32_t spare = occ >= 2 ? cus : std::max(1u, cus / 32);
            grid = std::max(1u, (slots_all > spare ? slots_all - spare : 1u) / n_cls);
        }
        K.grid = grid;
        K.first_wg = grid_total;
        grid_total += grid;
    }
    if (grid_total > ctx->cfg.max_teams) return DSR_E_NOMEM;
    t.grid = cls[0].grid;

    dsr_server *S = new (std::nothrow) dsr_server();
    if (!S) return DSR_E_NOMEM;
    S->ctx = ctx;
    S->cfg = c;
    S->tune = t;
    S->variant = variant;
    S->next_ticket = 1;
    S->in_flight = 0;
    S->hbm_used = 0;
    S->hbm_budget = (uint64_t)grid_total * ctx->cfg.hbm_slab_bytes * c.budget_pct / 100;
    S->cls = cls;
    for (serve_class &K : S->cls) {
        K.lds_used = 0;
        K.lds_budget = (uint64_t)K.grid * K.slab * c.budget_pct / 100;
    }
    /* shared host-coherent block: stop, start ticks, completion records;
     * a slot's host block: its head (the layout of the device's LDS copy:
     * descriptor, ops, loops), then its frame images */
    const size_t o_recs = 512;
    const size_t blk = o_recs + align256((size_t)c.slots * sizeof(dsr_drec));
    /* (a team reads DSR_SERVE_IMG_LDS image bytes whatever the request's size) */
    const size_t slot_h = DSR_SERVE_SLOT_HEAD + align256(std::max<size_t>(c.slot_bytes, DSR_SERVE_IMG_LDS));
    const size_t part_b = align256((size_t)DSR_MAX_RED * c.max_teams * DSR_PART_WORDS * sizeof(uint64_t));
    const size_t img_d = align256(c.slot_bytes);
    const size_t slot_d = part_b + align256(sizeof(dsr_dresult)) + 256 + img_d;
    const size_t ctl_d = DSR_SRV_WORDS * sizeof(uint32_t);
    if (hipSetDevice(ctx->device) != hipSuccess) { delete S; return DSR_E_HIP; }
    if (hipHostMalloc((void **)&S->h_block, blk, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        serve_free(S);
        return DSR_E_NOMEM;
    }
    std::memset(S->h_block, 0, blk);
    if (hipHostMalloc((void **)&S->h_arena, slot_h * c.slots, hipHostMallocCoherent | hipHostMallocMapped) !=
        hipSuccess) {
        serve_free(S);
        return DSR_E_NOMEM;
    }
    /* device arena: slot partials and results, then each class's control
     * words, cleared before any class's kernel can run */
    const size_t d_bytes = slot_d * c.slots + ctl_d * n_cls;
    if (hipMalloc((void **)&S->d_arena, d_bytes) != hipSuccess || hipMemset(S->d_arena, 0, d_bytes) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        serve_free(S);
        return DSR_E_NOMEM;
    }
    S->stop = (uint32_t *)(S->h_block + 64);
    S->start_ticks = (uint64_t *)(S->h_block + 128);
    S->recs = (dsr_drec *)(S->h_block + o_recs);
    S->slots.resize(c.slots);
    for (uint32_t i = 0; i < c.slots; ++i) {
        uint8_t *h = S->h_arena + slot_h * i;
        serve_slot &sl = S->slots[i];
        sl.desc = (dsr_dregion *)h;
        sl.ops = (dsr_op *)(h + DSR_SERVE_OPS_AT);
        sl.loops = (dsr_dloop *)(h + DSR_SERVE_LOOPS_AT);
        sl.init = h + DSR_SERVE_SLOT_HEAD;
        sl.d_partials = (uint64_t *)(S->d_arena + slot_d * i);
        sl.d_result = (dsr_dresult *)(S->d_arena + slot_d * i + part_b);
        sl.d_flag = (uint64_t *)(S->d_arena + slot_d * i + part_b + align256(sizeof(dsr_dresult)));
        sl.d_img = S->d_arena + slot_d * i + part_b + align256(sizeof(dsr_dresult)) + 256;
        sl.busy = false;
        sl.tmpl = nullptr;
        sl.cls = 0;
        S->free_slots.push_back(c.slots - 1 - i);
    }
    for (uint32_t k = 0; k < n_cls; ++k) {
        serve_class &K = S->cls[k];
        /* per class, host-coherent: published, closing, final count,
         * workgroup start and exit flags, item ring */
        const size_t o_wg = 256, o_items = o_wg + 2 * align256((size_t)K.grid * 4);
        const size_t ctl = o_items + align256((size_t)c.ring_items * 8);
        if (hipHostMalloc((void **)&K.h_ctl, ctl, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
            serve_free(S);
            return DSR_E_NOMEM;
        }
        std::memset(K.h_ctl, 0, ctl);
        K.published = (uint32_t *)K.h_ctl;
        K.closing = (uint32_t *)(K.h_ctl + 64);
        K.final_items = (uint32_t *)(K.h_ctl + 128);
        K.relays = (uint32_t *)(K.h_ctl + 192);
        K.wg_started = (uint32_t *)(K.h_ctl + o_wg);
        K.wg_exited = (uint32_t *)(K.h_ctl + o_wg + align256((size_t)K.grid * 4));
        K.items = (uint32_t *)(K.h_ctl + o_items);
        K.d_counter = (uint32_t *)(S->d_arena + slot_d * c.slots + ctl_d * k);
        K.pub = 0;
        if (hipStreamCreateWithFlags(&K.stream, hipStreamNonBlocking) != hipSuccess) {
            serve_free(S);
            return DSR_E_HIP;
        }
    }
    for (uint32_t k = 0; k < n_cls; ++k) {
        serve_class &K = S->cls[k];
        dsr_dlaunch LP{};
        LP.regions = (const dsr_dregion *)S->h_arena;
        LP.region_stride = (uint32_t)slot_h;
        LP.items = K.items;
        LP.n_items = 0;
        LP.n_regions = c.slots;
        LP.counter = K.d_counter;
        LP.done_ts = k == 0 ? S->start_ticks : nullptr;
        LP.published = K.published;
        LP.stop = S->stop;
        LP.recs = S->recs;
        LP.ring_mask = c.ring_items - 1;
        LP.idle_limit = (uint64_t)c.idle_ms * 100000ull;
        LP.closing = K.closing;
        LP.final_items = K.final_items;
        LP.relays = K.relays;
        LP.wg_started = K.wg_started;
        LP.wg_exited = K.wg_exited;
        dsr_dconfig C = make_dconfig(ctx, t.wg_size, K.slab, t.overflow_threshold, t.master_joins, 0);
        C.serve = 1;
        /* each class's teams take their own HBM stack and nested slots */
        C.hbm_base = ctx->hbm + (uint64_t)K.first_wg * ctx->cfg.hbm_slab_bytes;
        C.nest_base = ctx->nest + (uint64_t)K.first_wg * DSR_NEST_SLOT;
        if (dsr_launch_region_kernel(&LP, &C, K.grid, t.wg_size, K.lds_bytes, variant, K.stream) != 0) {
            __atomic_store_n(S->stop, 1u, __ATOMIC_RELEASE);
            for (uint32_t j = 0; j < k; ++j) (void)hipStreamSynchronize(S->cls[j].stream);
            serve_free(S);
            return DSR_E_HIP;
        }
    }
    *out = S;
    return DSR_OK;
}

/* Return slot k and its admission budget. */
static void serve_release(dsr_server *S, uint32_t k)
{
    serve_slot &sl = S->slots[k];
    sl.busy = false;
    if (sl.tmpl) sl.tmpl->serve_refs--;
    sl.tmpl = nullptr;
    S->cls[sl.cls].lds_used -= sl.lds_cost;
    S->hbm_used -= sl.hbm_cost;
    S->in_flight--;
    S->free_slots.push_back(k);
}

extern "C" int dsr_serve_submit(dsr_server *S, dsr_region *r, void *const *outs, int32_t n_outs,
                                uint64_t *ticket)
{
    if (!S || !r || !ticket || n_outs < 0) return DSR_E_INVAL;
    if (r->ctx != S->ctx) return DSR_E_INVAL;
    if (!r->live.empty()) return DSR_E_LIVE;
    if (r->ops.size() > DSR_SERVE_MAX_OPS || r->loops.size() > DSR_SERVE_MAX_LOOPS) return DSR_E_INVAL;
    if ((uint32_t)r->teams > S->cfg.max_teams || r->init.size() > S->cfg.slot_bytes) return DSR_E_INVAL;
    if ((size_t)n_outs > r->loops.size() || (n_outs && !outs)) return DSR_E_INVAL;
    /* fixed-length chains beyond 8+8 run through the run-time loop here */
    const uint64_t lanes = 64ull * (S->tune.master_joins ? S->tune.wg_size / 64 : S->tune.wg_size / 64 - 1);
    for (const dsr_dloop &L : r->loops)
        if ((L.chunk + lanes - 1) / lanes > (1ull << 15)) return DSR_E_INVAL;
    /* the class sized to the request's stack; a class that has closed
     * (stop, or idle) is passed over for the next larger one still open */
    uint32_t slabs[DSR_SERVE_CLASSES];
    const int32_t n_cls = (int32_t)S->cls.size();
    for (int32_t k = 0; k < n_cls; ++k) slabs[k] = S->cls[k].slab;
    std::vector<int32_t> order;
    const int32_t first = dsr_serve_class_for(slabs, n_cls, r);
    order.push_back(first);
    for (int32_t k = 0; k < n_cls; ++k)
        if (k != first && slabs[k] >= slabs[first]) order.push_back(k);
    std::sort(order.begin() + 1, order.end(), [&](int32_t a, int32_t b) { return slabs[a] < slabs[b]; });
    for (int32_t k = 0; k < n_cls; ++k)
        if (std::find(order.begin(), order.end(), k) == order.end()) order.push_back(k);
    int32_t kc = -1;
    bool busy = false, placeable = false;
    uint64_t lcost = 0, hcost = 0;
    const uint32_t thr = S->tune.overflow_threshold ? S->tune.overflow_threshold : 0xFFFFFFFFu;
    for (int32_t k : order) {
        serve_class &K = S->cls[k];
        uint64_t lp = 0, hp = 0;
        /* a class whose stacks cannot hold one of the request's frames is
         * passed over; NOMEM only when no class can */
        if (!stack_peaks(r, K.slab, thr, S->ctx->cfg.hbm_slab_bytes, &lp, &hp)) continue;
        placeable = true;
        if (__atomic_load_n(K.closing, __ATOMIC_SEQ_CST) != 0) continue;
        const uint64_t lc = lp * r->teams, hc = hp * r->teams;
        /* ring space: items of the oldest unfinished request bound the writer */
        uint32_t floor_item = K.pub;
        for (const serve_slot &sl : S->slots)
            if (sl.busy && sl.cls == (uint32_t)k && (int32_t)(sl.first_item - floor_item) < 0)
                floor_item = sl.first_item;
        const bool fits = (!S->in_flight || (K.lds_used + lc <= K.lds_budget && S->hbm_used + hc <= S->hbm_budget)) &&
                          K.pub + (uint32_t)r->teams - floor_item <= S->cfg.ring_items;
        if (!fits) {
            busy = true;
            /* a larger class takes it only while the sized one is full */
            continue;
        }
        kc = k;
        lcost = lc;
        hcost = hc;
        break;
    }
    if (kc < 0) return !placeable ? DSR_E_NOMEM : (busy ? DSR_E_BUSY : DSR_E_STATE);
    if (S->free_slots.empty()) return DSR_E_BUSY;
    serve_class &K = S->cls[kc];

    const uint32_t k = S->free_slots.back();
    S->free_slots.pop_back();
    serve_slot &sl = S->slots[k];
    std::memcpy(sl.ops, r->ops.data(), r->ops.size() * sizeof(dsr_op));
    std::vector<dsr_dloop> L = r->loops;
    for (int32_t i = 0; i < n_outs; ++i)
        if (outs[i]) L[i].out = outs[i];
    if (!L.empty()) std::memcpy(sl.loops, L.data(), L.size() * sizeof(dsr_dloop));
    /* images up to 1 KiB travel in the slot (the team stages them with the
     * program); larger ones of a frozen region are read from its device
     * copy */
    const bool dev_img = r->init.size() > DSR_SERVE_IMG_LDS && r->frozen && r->d_init;
    if (!r->init.empty() && !dev_img) std::memcpy(sl.init, r->init.data(), r->init.size());
    const uint64_t tk = S->next_ticket++;
    dsr_dregion R{};
    R.ops = sl.ops;
    R.loops = sl.loops;
    R.init = dev_img ? r->d_init : sl.init;
    R.partials = sl.d_partials;
    R.result = sl.d_result;
    R.trace = nullptr;
    R.n_ops = (uint32_t)r->ops.size();
    R.teams = (uint32_t)r->teams;
    R.n_red = r->n_red;
    R.red_kind_mask = r->red_kind_mask;
    R.tag = tk;
    R.n_loops = (uint32_t)r->loops.size();
    R.init_size = (uint32_t)r->init.size();
    /* tickets start at 1, and the flags at 0 */
    if (!dev_img && r->teams > 1 && r->init.size() > DSR_SERVE_IMG_LDS &&
        (uint64_t)r->teams * r->init.size() >= DSR_SERVE_RELAY_MIN) {
        R.relay = sl.d_img;
        R.relay_flag = sl.d_flag;
    }
    *sl.desc = R;
    uint64_t *ring = (uint64_t *)K.items;
    for (int32_t t = 0; t < r->teams; ++t) {
        const uint32_t seq = K.pub + (uint32_t)t;
        ring[seq & (S->cfg.ring_items - 1)] = ((uint64_t)seq << 32) | ((uint64_t)k << 16) | (uint32_t)t;
    }
    sl.busy = true;
    sl.tmpl = dev_img ? r : nullptr;
    if (dev_img) r->serve_refs++;
    sl.ticket = tk;
    sl.first_item = K.pub;
    sl.cls = (uint32_t)kc;
    sl.lds_cost = lcost;
    sl.hbm_cost = hcost;
    K.lds_used += lcost;
    S->hbm_used += hcost;
    S->in_flight++;
    K.pub += (uint32_t)r->teams;
    /* everything above is visible before the new count; then look for a
     * close the device may have begun meanwhile (its side writes the
     * closing flag, then reads the count: one of the two reads sees the
     * other side's write) */
    __atomic_store_n(K.published, K.pub, __ATOMIC_SEQ_CST);
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
    if (__atomic_load_n(K.closing, __ATOMIC_SEQ_CST) != 0) {
        /* the closing workgroup reports the count it read right away */
        uint32_t fin = 0;
        const auto t0 = std::chrono::steady_clock::now();
        while ((fin = __atomic_load_n(K.final_items, __ATOMIC_ACQUIRE)) == 0) {
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(10)) return DSR_E_HIP;
        }
        if ((int32_t)(K.pub - (fin - 1u)) > 0) {
            /* published after the close: the device will not run it */
            serve_release(S, k);
            return DSR_E_STATE;
        }
    }
    *ticket = tk;
    return DSR_OK;
}

extern "C" int dsr_serve_poll(dsr_server *S, dsr_done *out, int32_t max)
{
    if (!S || (!out && max > 0)) return DSR_E_INVAL;
    int32_t n = 0;
    for (uint32_t k = 0; k < S->slots.size() && n < max; ++k) {
        serve_slot &sl = S->slots[k];
        if (!sl.busy) continue;
        const uint64_t seq = __atomic_load_n(&S->recs[k].seq, __ATOMIC_ACQUIRE);
        if (seq != sl.ticket) continue;
        const dsr_drec &rec = S->recs[k];
        dsr_done &d = out[n++];
        std::memset(&d, 0, sizeof(d));
        d.ticket = sl.ticket;
        d.status = rec.status;
        d.n_red = (int32_t)rec.n_red;
        for (uint32_t i = 0; i < rec.n_red && i < 8; ++i) {
            d.f64[i] = rec.f64[i];
            d.i64[i] = rec.i64[i];
            for (int w = 0; w < 3; ++w) d.fixed[i][w] = rec.fixed[i][w];
        }
        const uint64_t t0 = __atomic_load_n(S->start_ticks, __ATOMIC_ACQUIRE);
        d.device_us = ((double)rec.ticks - (double)t0) / 100.0;
        d.lds_class = (int32_t)sl.cls;
        serve_release(S, k);
    }
    return n;
}

extern "C" int dsr_serve_pending(dsr_server *S)
{
    if (!S) return DSR_E_INVAL;
    return (int)S->in_flight;
}

extern "C" int dsr_serve_status(dsr_server *S, dsr_serve_stat *out)
{
    if (!S || !out) return DSR_E_INVAL;
    dsr_serve_stat st{};
    st.closed = 1;
    for (const serve_class &K : S->cls) {
        st.grid += K.grid;
        for (uint32_t b = 0; b < K.grid; ++b) {
            st.started += __atomic_load_n(K.wg_started + b, __ATOMIC_ACQUIRE) != 0;
            st.exited += __atomic_load_n(K.wg_exited + b, __ATOMIC_ACQUIRE) != 0;
        }
        /* closed: every class has closed */
        if (__atomic_load_n(K.closing, __ATOMIC_ACQUIRE) == 0) {
            st.closed = 0;
        } else if (!st.close_reason) {
            const uint32_t *why = K.closing + 1;
            st.close_reason = __atomic_load_n(why, __ATOMIC_ACQUIRE);
            st.close_block = why[1];
            st.close_item = why[2];
            st.close_seen = why[3];
            st.close_idle_us = (double)((uint64_t)why[4] | ((uint64_t)why[5] << 32)) / 100.0;
        }
        const uint32_t fin = __atomic_load_n(K.final_items, __ATOMIC_ACQUIRE);
        st.final_items += fin ? fin - 1 : 0;
        st.published += K.pub;
        st.relays += __atomic_load_n(K.relays, __ATOMIC_ACQUIRE);
        st.relay_misses += __atomic_load_n(K.relays + 1, __ATOMIC_ACQUIRE);
    }
    st.in_flight = S->in_flight;
    st.classes = (uint32_t)S->cls.size();
    *out = st;
    return DSR_OK;
}

extern "C" int dsr_serve_stop(dsr_server *S)
{
    if (!S) return DSR_E_INVAL;
    __atomic_store_n(S->stop, 1u, __ATOMIC_RELEASE);
    hipError_t e = hipSuccess;
    for (serve_class &K : S->cls) {
        const hipError_t ek = hipStreamSynchronize(K.stream);
        if (ek != hipSuccess) e = ek;
    }
    serve_free(S);
    return e == hipSuccess ? DSR_OK : DSR_E_HIP;
}

/* ---- schedule replays ------------------------------------------------------- */
#include <chrono>

namespace {
double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

extern "C" int dsr_serve_replay(dsr_server *S, dsr_region *const *programs, const int32_t *prog,
                                const double *arrival_s, int32_t n, void *const *slot_outs,
                                int32_t n_loops_max, double timeout_s, double *latency_us, dsr_done *done)
{
    if (!S || !programs || !prog || !arrival_s || n < 0 || !latency_us || !done) return DSR_E_INVAL;
    if (slot_outs && n_loops_max < 1) return DSR_E_INVAL;
    std::vector<int32_t> by_ticket;       /* ticket - first ticket -> request */
    const uint64_t first_ticket = S->next_ticket;
    try {
        by_ticket.assign((size_t)n, -1);
    } catch (...) {
        return DSR_E_NOMEM;
    }
    std::vector<dsr_done> buf(256);
    const double t0 = now_s();
    int32_t next = 0, completed = 0;
    const double last = n ? arrival_s[n - 1] : 0.0;
    while (completed < n) {
        const double now = now_s() - t0;
        while (next < n && arrival_s[next] <= now) {
            dsr_region *r = programs[prog[next]];
            if (S->free_slots.empty()) break;
            const uint32_t slot = S->free_slots.back();
            std::vector<void *> outs;
            if (slot_outs)
                for (size_t i = 0; i < r->loops.size(); ++i)
                    outs.push_back(slot_outs[(size_t)slot * n_loops_max + i]);
            uint64_t tk = 0;
            const int rc = dsr_serve_submit(S, r, outs.empty() ? nullptr : outs.data(), (int32_t)outs.size(), &tk);
            if (rc == DSR_E_BUSY) break;
            if (rc) return rc;
            by_ticket[tk - first_ticket] = next;
            ++next;
        }
        const int got = dsr_serve_poll(S, buf.data(), (int32_t)buf.size());
        if (got < 0) return got;
        const double tdone = now_s() - t0;
        for (int g = 0; g < got; ++g) {
            const int32_t q = by_ticket[buf[g].ticket - first_ticket];
            latency_us[q] = (tdone - arrival_s[q]) * 1e6;
            done[q] = buf[g];
            ++completed;
        }
        if (tdone > last + timeout_s) return DSR_E_BUSY;
    }
    return DSR_OK;
}

extern "C" int dsr_batch_replay_serial(dsr_batch *b, const int32_t *prog, const double *arrival_s, int32_t n,
                                       double *latency_us)
{
    if (!b || !prog || !arrival_s || n < 0 || !latency_us) return DSR_E_INVAL;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return DSR_E_HIP;
    const dsr_dconfig C = make_dconfig(b->ctx, b->tune.wg_size, b->tune.lds_slab_bytes,
                                       b->tune.overflow_threshold, b->tune.master_joins, 0);
    const uint32_t variant = b->tune.wg_size > 256 ? 0 : b->variant;
    const double t0 = now_s();
    int rc = DSR_OK;
    for (int32_t q = 0; q < n && rc == DSR_OK; ++q) {
        const int32_t i = prog[q];
        if (i < 0 || i >= b->n) { rc = DSR_E_INVAL; break; }
        while (now_s() - t0 < arrival_s[q]) {
        }
        dsr_dlaunch LP{};
        LP.regions = b->d_regions + i;
        LP.items = nullptr;
        LP.n_regions = 1;
        if (dsr_launch_region_kernel(&LP, &C, (uint32_t)b->teams[i], b->tune.wg_size, b->lds_bytes, variant, s) ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = DSR_E_HIP;
        latency_us[q] = (now_s() - t0 - arrival_s[q]) * 1e6;
    }
    (void)hipStreamDestroy(s);
    b->last = 0;
    if (rc == DSR_OK) {
        if (copy_batch_results(b) != DSR_OK) return DSR_E_HIP;
        b->have_results = true;
    }
    return rc;
}

/* ---- footprint and occupancy model ------------------------------------------ */
extern "C" int dsr_occupancy_model(const dsr_hw_model *hw, uint32_t threads, uint32_t regs,
                                   uint32_t shared, dsr_occupancy *out)
{
    if (!hw || !out || threads == 0 || regs == 0) return DSR_E_INVAL;
    if (hw->regs_per_cu == 0 || hw->max_teams_per_cu == 0 || hw->max_threads_per_cu == 0) return DSR_E_INVAL;
    const uint32_t rg = hw->reg_granule ? hw->reg_granule : 1;
    const uint32_t sg = hw->shared_granule ? hw->shared_granule : 1;
    const uint64_t r = ((uint64_t)regs + rg - 1) / rg * rg;
    const uint64_t sh = ((uint64_t)shared + sg - 1) / sg * sg;
    dsr_occupancy o{};
    o.regs_per_thread = (uint32_t)r;
    o.shared_per_team = (uint32_t)sh;
    if (hw->simds_per_cu && hw->wave_size) {
        /* registers live in the SIMDs' files: a SIMD holds as many waves as
         * its file has room for, and a team needs ceil(threads / wave) of
         * the CU's waves */
        const uint64_t per_lane = hw->regs_per_cu / ((uint64_t)hw->simds_per_cu * hw->wave_size);
        const uint64_t waves = per_lane / r * hw->simds_per_cu;
        const uint64_t team_waves = (threads + hw->wave_size - 1) / hw->wave_size;
        o.teams_by_registers = (uint32_t)(waves / team_waves);
    } else {
        o.teams_by_registers = (uint32_t)(hw->regs_per_cu / (r * threads));
    }
    o.teams_by_shared = sh ? (uint32_t)std::min<uint64_t>(hw->shared_per_cu / sh, 0xFFFFFFFFu) : 0xFFFFFFFFu;
    o.teams_by_threads = hw->max_threads_per_cu / threads;
    uint32_t t = hw->max_teams_per_cu;
    uint32_t lim = DSR_LIMIT_TEAMS;
    if (o.teams_by_registers < t) { t = o.teams_by_registers; lim = DSR_LIMIT_REGISTERS; }
    if (o.teams_by_shared < t) { t = o.teams_by_shared; lim = DSR_LIMIT_SHARED; }
    if (o.teams_by_threads < t) { t = o.teams_by_threads; lim = DSR_LIMIT_THREADS; }
    o.teams_per_cu = t;
    o.limiter = lim;
    o.shared_per_cu = (uint64_t)t * sh;
    *out = o;
    return DSR_OK;
}

extern "C" int dsr_region_occupancy(dsr_ctx *ctx, uint32_t variant, dsr_occupancy *out)
{
    if (!ctx || !out) return DSR_E_INVAL;
    if (variant > 2 && (variant < DSR_LEAN_BASE || variant >= DSR_LEAN_BASE + DSR_LEAN_CHAINS ||
                        ctx->cfg.wg_size > 256))
        return DSR_E_INVAL;
    if (ctx->device < 0) return DSR_E_STATE;
    hipDeviceProp_t p{};
    if (hipGetDeviceProperties(&p, ctx->device) != hipSuccess) return DSR_E_HIP;
    const int regs = dsr_region_kernel_regs(ctx->cfg.wg_size, variant);
    if (regs <= 0 || p.multiProcessorCount <= 0 || p.maxThreadsPerMultiProcessor <= 0 || p.warpSize <= 0)
        return DSR_E_HIP;
    /* gfx950: 4 SIMDs, each with 512 VGPRs (arch + acc) per lane, allocated
     * in 8s; the workgroup cap is one per wave slot, so waves, registers
     * and LDS are what limit a team */
    const uint32_t wave = (uint32_t)p.warpSize, thr = (uint32_t)p.maxThreadsPerMultiProcessor;
    dsr_hw_model hw{(uint32_t)p.multiProcessorCount, 4u * 512u * wave, 8u, thr / wave, thr,
                    (uint32_t)p.maxSharedMemoryPerMultiProcessor, 128u, 4u, wave};
    const int rc = dsr_occupancy_model(&hw, ctx->cfg.wg_size, (uint32_t)regs, ctx->lds_bytes, out);
    if (rc) return rc;
    out->hip_teams_per_cu = (uint32_t)dsr_region_kernel_occupancy(ctx->cfg.wg_size, ctx->lds_bytes, variant);
    return DSR_OK;
}
