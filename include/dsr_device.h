/*
 * dsr_device.h -- device API of the data-sharing runtime (HIP, gfx950).
 *
 * The calls mirror the runtime entry points of the paper's generic-mode
 * scheme (section 4, Figures 2 and 3; section 5.1):
 *   team_init     ~ __kmpc_kernel_init: carve the team's LDS into a control
 *                   block and a stack, bind the team's HBM slab slot.
 *   push / pop    the master's frame allocation on the per-team stack
 *                   (section 5.3.1's shared depot; overflow to the HBM slab
 *                   as in section 5.2's global fallback and section 7's
 *                   runtime-managed global stack).
 *   publish       ~ __kmpc_kernel_prepare_parallel + the first barrier of
 *                   Figure 2: hand a frame reference and a body to workers.
 *   await         ~ the worker's barrier + __kmpc_kernel_parallel of
 *                   Figure 3: false means terminate.
 *   end_parallel  ~ __kmpc_kernel_end_parallel + the second barrier.
 *
 * Roles (a wave64 rendering of section 4's warp-based split): the team's
 * last wave is the master wave and its lane 0 the OpenMP master; every
 * lane of the master wave runs the sequential code in lock-step (so the
 * other 63 lanes can assist bulk copies), the other waves are workers.
 * Master-only calls (push, pop, publish) must be made by the whole master
 * wave with uniform arguments; only lane 0 writes the shared state.
 *
 * A frame is a value {space, offset, size}, never a raw pointer: bodies
 * reach a shared variable in it with slot<V>(team, frame, offset), or take
 * the frame's base with frame_lds / frame_hbm.
 *
 * LDS layout of a team (dynamic shared memory):
 *   [header 64 B][frame table 16 x 16 B][reference list 20 x 8 B]
 *   [per-wave reduction slots nw x 32 B][nested area: nw x DSR_NEST_LDS_WAVE]
 *   [stack: lds_cap bytes]
 * The nested area holds the on-chip part of every nested member's stack
 * (section 7's sharing at worker level): with P participating waves,
 * wave m's stack at m * DSR_NEST_WAVE_LDS, then the stacks of lane group g
 * of wave m at P * DSR_NEST_WAVE_LDS + (m * DSR_NEST_GROUPS + g) *
 * DSR_NEST_GROUP_LDS, and, after room for every wave's stacks, each wave's
 * descriptors (the published frame of the wave and of each of its lane
 * groups).  The global-memory part of the member stacks is a separate
 * per-team slot, laid out the same way with the _HBM sizes.
 * The reference list is the on-chip list of section 5.2: a published list
 * of up to DSR_REF_LIST references lives there, a longer one in a list
 * frame on the HBM stack.
 */
#ifndef DSR_DEVICE_H
#define DSR_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DSR_MAX_FRAMES 16
#define DSR_MAX_WAVES 16
#define DSR_NEST_GROUPS 4u       /* inner members per member, at each nested level */
#define DSR_NEST_FRAME 16u       /* a nested frame: {lo, hi, parent space, parent offset} */
#define DSR_NEST_WAVE_LDS 64u    /* on-chip part of a wave's member stack        */
#define DSR_NEST_GROUP_LDS 16u   /* on-chip part of a lane group's member stack  */
#define DSR_NEST_WAVE_HBM 256u   /* global-memory part of a wave's member stack  */
#define DSR_NEST_GROUP_HBM 64u   /* global-memory part of a lane group's stack   */
#define DSR_NEST_DESC 48u        /* per wave: its descriptor + one per lane group */
/* nested area of one wave (on chip) and of one team per wave (global) */
#define DSR_NEST_LDS_WAVE (DSR_NEST_WAVE_LDS + DSR_NEST_GROUPS * DSR_NEST_GROUP_LDS + DSR_NEST_DESC)
#define DSR_NEST_HBM_WAVE (DSR_NEST_WAVE_HBM + DSR_NEST_GROUPS * DSR_NEST_GROUP_HBM)
#define DSR_ALIGN 16u
#define DSR_REF_LIST 20u        /* references the on-chip list holds (8 B each) */

namespace dsr {

/* SPACE_LIST names the on-chip reference list (a published list only);
 * SPACE_NEST_LDS / SPACE_NEST_HBM the on-chip and global parts of the
 * nested members' stacks. */
enum : uint32_t { SPACE_LDS = 0, SPACE_HBM = 1, SPACE_NONE = 2, SPACE_LIST = 3, SPACE_NEST_LDS = 4,
                  SPACE_NEST_HBM = 5 };

struct frame_t {
    uint32_t space;
    uint32_t off;
    uint32_t size;     /* rounded to DSR_ALIGN */
};

/* Control-block header (first 64 bytes of the team's LDS). */
struct cb_header {
    uint32_t body;     /* published body id; 0 = terminate        */
    uint32_t space;    /* published frame                          */
    uint32_t off;
    uint32_t size;
    uint32_t loop;     /* published loop descriptor index          */
    uint32_t sp_lds;   /* LDS stack pointer (bytes in use)         */
    uint32_t sp_hbm;   /* HBM stack pointer                        */
    uint32_t nframes;  /* live frames                              */
    int32_t error;     /* team error (DSR_E_* or 0)                */
    uint32_t bad;      /* OR of the workers' range flags           */
    uint32_t region;   /* launch-specific context published with the */
    uint32_t team;     /* body: which region and which of its teams  */
    uint32_t blocks;   /* blocks of the team's range claimed so far by its
                          waves (balanced split; reset at each publish) */
    uint32_t pad[3];
};

/* Bytes of control block for a team of nw waves. */
__host__ __device__ constexpr uint32_t cb_bytes(uint32_t nw)
{
    return 64u + DSR_MAX_FRAMES * 16u + DSR_REF_LIST * 8u + nw * 32u + nw * DSR_NEST_LDS_WAVE;
}

struct team_t {
    uint8_t *lds;        /* team's dynamic LDS base (control block)        */
    uint8_t *stack_lds;  /* LDS stack base                                 */
    uint8_t *stack_hbm;  /* this team's HBM slab slot                      */
    uint32_t lds_cap;
    uint32_t threshold;  /* frames larger than this go to HBM              */
    uint32_t hbm_cap;
    uint32_t nw;         /* waves in the team                              */
    uint32_t wave;       /* this wave (uniform)                            */
    uint32_t lane;
    uint8_t *nest_hbm;   /* this team's slot of the nested members' global stacks */
    uint32_t nest_global; /* 1: nested frames skip the on-chip stacks      */
};

__device__ inline uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

/* Make lane 0's LDS writes visible to the rest of its wave. */
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline cb_header *header(const team_t &T) { return (cb_header *)T.lds; }
__device__ inline uint32_t *frame_table(const team_t &T) { return (uint32_t *)(T.lds + 64); }
__device__ inline uint32_t *ref_list(const team_t &T) { return (uint32_t *)(T.lds + 64 + DSR_MAX_FRAMES * 16); }
__device__ inline uint64_t *red_slot(const team_t &T, uint32_t w)
{
    return (uint64_t *)(T.lds + 64 + DSR_MAX_FRAMES * 16 + DSR_REF_LIST * 8 + w * 32);
}
/* Base of the team's nested area (on chip). */
__device__ inline uint8_t *nest_lds(const team_t &T)
{
    return T.lds + 64 + DSR_MAX_FRAMES * 16 + DSR_REF_LIST * 8 + T.nw * 32;
}
/* Wave w's descriptor words: [0..1] its published nested frame, then
 * [2 + 2g .. 3 + 2g] the frame published by its lane group g. */
__device__ inline uint32_t *nest_desc(const team_t &T, uint32_t w)
{
    return (uint32_t *)(nest_lds(T) + T.nw * (DSR_NEST_WAVE_LDS + DSR_NEST_GROUPS * DSR_NEST_GROUP_LDS) +
                        w * DSR_NEST_DESC);
}

/* ~__kmpc_kernel_init.  Called by every thread of the team; the master
 * lane resets the stack.  The first barrier of the team (publish/await)
 * orders this before any worker reads the control block. */
__device__ inline team_t team_init(uint8_t *lds, uint32_t nw, uint32_t lds_cap,
                                   uint32_t threshold, uint8_t *hbm_slot, uint32_t hbm_cap)
{
    team_t T;
    T.lds = lds;
    T.nw = nw;
    T.stack_lds = lds + cb_bytes(nw);
    T.stack_hbm = hbm_slot;
    T.lds_cap = lds_cap;
    T.threshold = threshold;
    T.hbm_cap = hbm_cap;
    T.wave = uniform(threadIdx.x >> 6);
    T.lane = threadIdx.x & 63u;
    T.nest_hbm = nullptr;
    T.nest_global = 0;
    if (T.wave == nw - 1 && T.lane == 0) {
        cb_header *h = header(T);
        h->body = 0;
        h->sp_lds = 0;
        h->sp_hbm = 0;
        h->nframes = 0;
        h->error = 0;
        h->bad = 0;
    }
    return T;
}

/* Master wave: empty the stack before a new region program (a persistent
 * team runs many regions one after another). */
__device__ inline void team_reset(team_t &T)
{
    wave_sync();
    if (T.lane == 0) {
        cb_header *h = header(T);
        h->sp_lds = 0;
        h->sp_hbm = 0;
        h->nframes = 0;
        h->error = 0;
        h->bad = 0;
    }
    wave_sync();
}

/* Master wave: place a frame of nbytes (rounded up to 16).  LDS when it
 * fits and is not above the overflow threshold, else the HBM slot, else
 * SPACE_NONE (out of memory; nothing is allocated).  global_only keeps the
 * frame off the LDS stack (a global reference list). */
__device__ inline frame_t push(team_t &T, uint32_t nbytes, bool global_only = false)
{
    cb_header *h = header(T);
    const uint32_t size = (nbytes + DSR_ALIGN - 1) & ~(DSR_ALIGN - 1);
    uint32_t spl = uniform(h->sp_lds), sph = uniform(h->sp_hbm), nf = uniform(h->nframes);
    frame_t f;
    f.size = size;
    if (!global_only && size <= T.threshold && size <= T.lds_cap - spl) {
        f.space = SPACE_LDS; f.off = spl; spl += size;
    } else if (size <= T.hbm_cap - sph) {
        f.space = SPACE_HBM; f.off = sph; sph += size;
    } else {
        f.space = SPACE_NONE; f.off = 0;
        return f;
    }
    wave_sync();
    if (T.lane == 0) {
        h->sp_lds = spl;
        h->sp_hbm = sph;
        uint32_t *ft = frame_table(T) + 4 * nf;
        ft[0] = f.space; ft[1] = f.off; ft[2] = f.size; ft[3] = 0;
        h->nframes = nf + 1;
    }
    wave_sync();
    return f;
}

/* Master wave: pop the top frame.  Returns false if f is not the top
 * (the host rejects such programs before launch; this is a guard). */
__device__ inline bool pop(team_t &T, frame_t f)
{
    cb_header *h = header(T);
    uint32_t nf = uniform(h->nframes);
    if (nf == 0) return false;
    const uint32_t *ft = frame_table(T) + 4 * (nf - 1);
    if (uniform(ft[0]) != f.space || uniform(ft[1]) != f.off) return false;
    uint32_t spl = uniform(h->sp_lds), sph = uniform(h->sp_hbm);
    wave_sync();
    if (T.lane == 0) {
        if (f.space == SPACE_LDS) h->sp_lds = spl - f.size; else h->sp_hbm = sph - f.size;
        h->nframes = nf - 1;
    }
    wave_sync();
    return true;
}

/* Master wave: hand frame f and body to the workers (barrier 1). */
__device__ inline void publish(team_t &T, frame_t f, uint32_t body, uint32_t loop)
{
    cb_header *h = header(T);
    if (T.lane == 0) {
        h->body = body;
        h->space = f.space;
        h->off = f.off;
        h->size = f.size;
        h->loop = loop;
        h->blocks = 0;
    }
    __syncthreads();
}

/* Worker waves: wait for work (barrier 1).  Returns false on terminate. */
__device__ inline bool await(team_t &T, uint32_t *body, frame_t *f, uint32_t *loop)
{
    __syncthreads();
    cb_header *h = header(T);
    *body = uniform(h->body);
    f->space = uniform(h->space);
    f->off = uniform(h->off);
    f->size = uniform(h->size);
    *loop = uniform(h->loop);
    return *body != 0;
}

/* Every participating wave: deposit its reduction partial (a 192-bit
 * integer, three 64-bit words, low first) and its range flag, then join
 * (barrier 2).  Waves that did not run the body pass zeros. */
__device__ inline void end_parallel(team_t &T, uint64_t w0, uint64_t w1, uint64_t w2, uint32_t bad)
{
    if (T.lane == 0) {
        uint64_t *r = red_slot(T, T.wave);
        r[0] = w0; r[1] = w1; r[2] = w2;
        if (bad) atomicOr(&header(T)->bad, 1u);
    }
    __syncthreads();
}

/* Frame address in LDS or in the team's HBM slot. */
__device__ inline uint8_t *frame_lds(const team_t &T, frame_t f) { return T.stack_lds + f.off; }
__device__ inline uint8_t *frame_hbm(const team_t &T, frame_t f) { return T.stack_hbm + f.off; }

/* ---- nested levels (section 3.1.2 nesting; section 7 sharing at worker
 * level): a member of a parallel level is the master of an inner team.  It
 * pushes a frame on its own member stack, publishes it to its inner members
 * and pops it when they have joined.  A member stack has an on-chip part in
 * the team's nested area and a global-memory part in the team's nested
 * slot (the runtime-managed global stack of section 7, taken when the
 * on-chip part is exhausted).  The member's lanes hold the stack pointers
 * in registers; only the member's leader lane writes the frames. */
struct mstack_t {
    uint32_t lds_base, lds_cap;    /* offsets in the nested area              */
    uint32_t hbm_base, hbm_cap;    /* offsets in the team's nested slot       */
    uint32_t sp_lds, sp_hbm;
};

__device__ inline mstack_t mstack(uint32_t lds_base, uint32_t lds_cap, uint32_t hbm_base, uint32_t hbm_cap)
{
    return mstack_t{lds_base, lds_cap, hbm_base, hbm_cap, 0u, 0u};
}

/* Place a nested frame: the on-chip part if it fits, else the global part,
 * else SPACE_NONE (nothing allocated). */
__device__ inline frame_t mpush(mstack_t &S, uint32_t nbytes, bool global_only)
{
    const uint32_t size = (nbytes + DSR_ALIGN - 1) & ~(DSR_ALIGN - 1);
    frame_t f;
    f.size = size;
    if (!global_only && size <= S.lds_cap - S.sp_lds) {
        f.space = SPACE_NEST_LDS; f.off = S.lds_base + S.sp_lds; S.sp_lds += size;
    } else if (size <= S.hbm_cap - S.sp_hbm) {
        f.space = SPACE_NEST_HBM; f.off = S.hbm_base + S.sp_hbm; S.sp_hbm += size;
    } else {
        f.space = SPACE_NONE; f.off = 0;
    }
    return f;
}

/* Pop the member stack's top frame; false if f is not the top. */
__device__ inline bool mpop(mstack_t &S, frame_t f)
{
    if (f.space == SPACE_NEST_LDS && f.off + f.size == S.lds_base + S.sp_lds) { S.sp_lds -= f.size; return true; }
    if (f.space == SPACE_NEST_HBM && f.off + f.size == S.hbm_base + S.sp_hbm) { S.sp_hbm -= f.size; return true; }
    return false;
}

/* Address of (space, offset) in the nested stacks. */
__device__ inline uint32_t *nest_addr(const team_t &T, uint32_t space, uint32_t off)
{
    return (uint32_t *)(space == SPACE_NEST_LDS ? nest_lds(T) + off : T.nest_hbm + off);
}

/* Typed address of the shared variable `off` bytes into frame f, in
 * whichever space the frame lives (section 5.1: workers reach the master's
 * locals through the reference they are handed, not by copy).  `off` must
 * be a multiple of alignof(V) and off + sizeof(V) <= f.size. */
template <class V>
__device__ inline V *slot(const team_t &T, frame_t f, uint32_t off)
{
    return (V *)((f.space == SPACE_LDS ? T.stack_lds : T.stack_hbm) + f.off + off);
}

} // namespace dsr

#endif /* DSR_DEVICE_H */
