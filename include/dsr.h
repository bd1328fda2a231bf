/*
 * dsr.h -- host C ABI of the device data-sharing runtime (libdsr.so).
 *
 * Implicit data sharing for generic-mode OpenMP-style target regions on
 * MI355X (gfx950), after Bercea et al., "Implementing implicit OpenMP data
 * sharing on GPUs" (LLVM-HPC'17).
 *
 * Model (section 4, Figures 2 and 3; section 5):
 *   A region runs on `teams` workgroups.  In each team one master wave
 *   (the last wave; lane 0 is the OpenMP master) executes the sequential
 *   code: it pushes frames holding its implicitly shared locals onto a
 *   per-team stack, publishes a frame and an outlined loop body to the
 *   worker waves, waits for them to join, and pops its frames in LIFO
 *   order.  Workers read the shared locals through the frame reference
 *   (section 5.1: sharing by reference) and reduce into a shared variable
 *   held in the frame.  Frames live in LDS when they fit (the shared-memory
 *   stack of section 5.3.1) and otherwise in a pre-allocated HBM slab (the
 *   global-memory fallback of section 5.2 and the runtime-managed global
 *   stack proposed in section 7).
 *
 *   The host builds a region as a program of PUSH / PUBLISH / POP
 *   operations that every team's master runs; `dsr_launch` validates it and
 *   runs it in one kernel launch.
 *
 * Conventions for every call:
 *   - Return value: DSR_OK (0) or a negative DSR_E_* code.  No call aborts,
 *     throws or traps; errors that the host can see (bad arguments, pop
 *     order, live frames, state) are reported before any GPU work.
 *   - Device pointers are plain `void*` obtained from hipMalloc (or a
 *     framework such as PyTorch); the caller owns them and must keep them
 *     alive until the launch's stream has completed.  `stream` is a
 *     hipStream_t passed as `void*` (NULL = the null stream).
 *   - A context belongs to one host thread at a time.
 */
#ifndef DSR_H
#define DSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define DSR_OK            0
#define DSR_E_INVAL      -1  /* bad argument or unsupported combination        */
#define DSR_E_NOMEM      -2  /* a frame fits neither the LDS stack nor the HBM slab
                                (reported by the device), or a host allocation failed */
#define DSR_E_LDS        -3  /* configuration exceeds the device's LDS per workgroup */
#define DSR_E_UNDERFLOW  -4  /* pop on an empty stack                          */
#define DSR_E_ORDER      -5  /* pop of a frame that is not the top (not LIFO)  */
#define DSR_E_LIVE       -6  /* a frame is still live when the region ends     */
#define DSR_E_STATE      -7  /* operation not allowed in the current state
                                (publish of a dead frame, push after launch ...) */
#define DSR_E_BUSY       -8  /* server over budget; retry later               */
#define DSR_E_HIP        -9  /* a HIP runtime call failed                       */
#define DSR_E_RANGE     -10  /* a loop value lies outside the exact-sum window
                                (see DSR_BODY_FMA_CHAIN)                         */

/* ---- loop bodies (the "outlined parallel regions" of Figure 3) ------------
 * Each body fixes the layout of the frame it is published with, in the way
 * the wrapper of Figure 4 fixes the order of the shared arguments.
 * Offsets are bytes from the frame base; all values little-endian.
 *
 * DSR_BODY_AFFINE_XOR   frame: [0,8) int64 shared sum; [8,24) int32 a, b, c, d.
 *     out (int32[n]): out[i] = a*i + b - (c XOR i) + d, 32-bit wrap-around.
 *     reduction: sum += out[i] (int64, wrap-around), one value per publish.
 *
 * DSR_BODY_FMA_CHAIN    frame: [0,24) exact shared sum (signed 192-bit integer
 *     in units of 2^-75, three 64-bit words, low first); nf fp64 scalars at
 *     24; ni int32 scalars right after them; if alen > 0 an int32 array of
 *     alen elements at the next 16-byte boundary.
 *     in (float[n]) x, out (double[n]) y:
 *       acc = alen ? (double)arr[i mod alen] : +0.0;
 *       for each int32 scalar s (in order), then each fp64 scalar s:
 *           acc = fma((double)s, (double)x[i], acc);      (IEEE fused)
 *       y[i] = acc.
 *     reduction: sum += y[i] exactly.  The result is the exact total
 *     rounded once to nearest-even double, independent of teams, waves and
 *     launch form.  Every y[i] must be a multiple of 2^-75 with |y| < 2^32;
 *     otherwise the region fails with DSR_E_RANGE.
 *
 * DSR_BODY_GATHER       frame: A int32 arrays of `len` elements back to back.
 *     out (int32[n]): out[i] = sum_j arr_j[i mod len] + i (32-bit wrap).
 *
 * DSR_BODY_GATHER_NESTED  as DSR_BODY_GATHER, run as two nested parallel
 *     levels: each worker wave is a member of the outer level; it pushes a
 *     16-byte inner frame {lo, hi, stride, outer frame} on its own LDS
 *     sub-stack and hands it to its four 16-lane groups (the inner level),
 *     then pops it (section 3.1.2 nesting; section 7 worker-level sharing).
 */
#define DSR_BODY_TERMINATE      0
#define DSR_BODY_AFFINE_XOR     1
#define DSR_BODY_FMA_CHAIN      2
#define DSR_BODY_GATHER         3
#define DSR_BODY_GATHER_NESTED  4

/* ---- configuration -------------------------------------------------------- */
#define DSR_F_TRACE        1u  /* record frame placements and barrier counts   */
#define DSR_F_TIMING       2u  /* record HIP events around every launch        */

typedef struct dsr_config {
    uint32_t wg_size;            /* threads per team: multiple of 64 in [64, 1024] */
    uint32_t lds_slab_bytes;     /* LDS stack capacity per team; 0 = every frame
                                    goes to the HBM slab (global stack only)     */
    uint32_t overflow_threshold; /* frames larger than this go to HBM; 0 = no limit */
    uint32_t master_joins;       /* 1: the master wave also runs loop iterations
                                    (forced when wg_size == 64)                  */
    uint64_t hbm_slab_bytes;     /* HBM stack capacity per team slot              */
    uint32_t max_teams;          /* team slots in the HBM slab (allocated once by
                                    dsr_init); a launch may not exceed it        */
    uint32_t flags;              /* DSR_F_* */
} dsr_config;

/* One published parallel loop.  Pointers are device pointers. */
typedef struct dsr_loop {
    uint64_t n;        /* iterations of the worksharing loop                   */
    uint64_t chunk;    /* iterations per team (0: ceil(n/teams) rounded up to 64);
                          team t runs [t*chunk, min(n, (t+1)*chunk))            */
    const void *in;    /* FMA_CHAIN: float x[n]                                */
    void *out;         /* int32 out[n] or double y[n]                           */
    uint32_t ni, nf;   /* FMA_CHAIN: int32 and fp64 scalar counts (ni+nf <= 64) */
    uint32_t alen;     /* FMA_CHAIN: array length (0 = none)                    */
    uint32_t arrays;   /* GATHER: number of arrays A (1..16)                     */
    uint32_t len;      /* GATHER: elements per array                            */
    uint32_t schedule; /* DSR_SCHED_STATIC or DSR_SCHED_DYNAMIC_TAIL            */
    uint32_t tail_pct; /* DYNAMIC_TAIL: percent of iterations claimed dynamically
                          (1..99; 0 = 25)                                        */
    uint32_t block;    /* DYNAMIC_TAIL: iterations per claim (multiple of 128,
                          at most 65536; 0 = 1024)                               */
} dsr_loop;

/* Loop schedules.
 * STATIC: team t runs [t*chunk, min(n, (t+1)*chunk)); its worker lanes take
 *   the iterations cyclically.
 * DYNAMIC_TAIL: the first (100 - tail_pct)% of the iterations are split
 *   statically as above (chunk is computed by the runtime and must be 0 on
 *   input); the rest is cut into blocks of `block` iterations that worker
 *   waves of any team claim one at a time from a device counter, so teams
 *   that run faster take more of the tail.  Allowed only when every team's
 *   copy of the published frame is initialised identically (no init_stride),
 *   since a block may run on any team.  Results are the same as STATIC's. */
#define DSR_SCHED_STATIC        0
#define DSR_SCHED_DYNAMIC_TAIL  1

typedef struct dsr_ctx dsr_ctx;
typedef struct dsr_region dsr_region;

/* Create a context on HIP device `device`: validates `cfg` against the
 * device (DSR_E_LDS if the LDS stack plus the team's control block exceeds
 * the LDS per workgroup) and allocates the HBM slab
 * (max_teams * hbm_slab_bytes) once (section 5.2's device malloc is replaced
 * by this pre-allocation).  *out owns that memory until dsr_destroy. */
int dsr_init(dsr_ctx **out, const dsr_config *cfg, int device);
int dsr_destroy(dsr_ctx *ctx);

/* Start building a region that runs on `teams` teams (1 .. cfg.max_teams). */
int dsr_region_begin(dsr_ctx *ctx, int32_t teams, dsr_region **out);

/* Master code block: push a frame of `nbytes` declared bytes (rounded up to
 * 16 on the stack).  The frame's first `init_bytes` bytes are copied from
 * the host buffer `init` (copied at this call; NULL if init_bytes == 0) and
 * the rest is zero.  If `init_stride` is nonzero, team t copies from
 * init + t*init_stride instead (the buffer then holds teams*init_stride
 * bytes): each team is a separate contention group with its own copy of
 * the master's locals.  *frame_out receives a small handle valid until the
 * matching pop.  Placement (LDS or HBM) is decided on the device. */
int dsr_push(dsr_region *r, uint32_t nbytes, const void *init, uint32_t init_bytes,
             uint32_t init_stride, int32_t *frame_out);

/* Publish live frame `frame` with loop body `body` (DSR_BODY_*) and loop
 * descriptor `loop` to the team's workers (the fork of Figure 2, barrier 1),
 * wait for them to join (barrier 2) and combine their reduction into the
 * frame's shared variable.  Bodies with a reduction produce one result per
 * publish, numbered in publish order across the region. */
int dsr_publish(dsr_region *r, int32_t frame, int32_t body, const dsr_loop *loop);

/* Pop frame `frame`; it must be the most recently pushed live frame.
 * DSR_E_UNDERFLOW on an empty stack, DSR_E_ORDER if not the top. */
int dsr_pop(dsr_region *r, int32_t frame);

/* Validate the program (DSR_E_LIVE if a frame is still live) and launch it
 * as one kernel of `teams` workgroups on `stream`.  Asynchronous: results
 * are available after dsr_region_sync.  A region may be launched again
 * (the same program over the same buffers) after its previous launch has
 * completed. */
int dsr_launch(dsr_region *r, void *stream);

/* Wait for the region's last launch and return its device status: DSR_OK,
 * DSR_E_NOMEM (a frame fit neither stack) or DSR_E_RANGE. */
int dsr_region_sync(dsr_region *r);

/* Result of reducing publish `index` of the last launch (after
 * dsr_region_sync): for AFFINE_XOR *i64 is the int64 sum; for FMA_CHAIN *f64
 * is the correctly rounded sum and fixed[0..2] the exact 192-bit total in
 * units of 2^-75 (any output pointer may be NULL). */
int dsr_region_reduction(dsr_region *r, int32_t index, int64_t *i64, double *f64,
                         uint64_t *fixed3);

/* Copy team `team`'s trace of the last launch (needs DSR_F_TRACE) into
 * `buf` (capacity `n` uint32 words; DSR_TRACE_WORDS words are written):
 *   [0]                   number of pushes recorded (k <= 16)
 *   [1 + 3p .. 3 + 3p]    push p: space (0 LDS, 1 HBM), offset, rounded size
 *   [49 .. 64]            barriers passed by wave 0 .. 15
 *   [65 .. 80]            inner frames pushed by wave 0 .. 15 (nested body)
 *   [81]                  team error code
 *   [82 .. 83]            wall clock (100 MHz, low word first) when the
 *                         workers were released for the first publish
 *   [84 .. 85]            wall clock when the last publish joined
 *   [86]                  low word of the wall clock at team start
 *   [96 + 2w, 97 + 2w]    low words of the wall clock when wave w started
 *                         and finished its share of the last body it ran   */
#define DSR_TRACE_WORDS 128
int dsr_region_trace(dsr_region *r, int32_t team, uint32_t *buf, uint32_t n);

/* Duration of the last launch's kernel in milliseconds, from HIP events
 * recorded around it on its stream (needs DSR_F_TIMING; DSR_E_STATE
 * otherwise). */
int dsr_region_elapsed(dsr_region *r, float *ms);

/* Release a region's host and device memory (syncs its last launch). */
int dsr_region_free(dsr_region *r);

/* Static string for a DSR_* code. */
const char *dsr_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* DSR_H */
