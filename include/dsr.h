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
 * DSR_BODY_GATHER_NESTED  as DSR_BODY_GATHER, run as `depth` (2 or 3)
 *     nested parallel levels (section 3.1.2 nesting; section 7 sharing at
 *     worker level).  Each participating wave is a member of the first
 *     level and takes a contiguous piece of the team's range; it pushes a
 *     16-byte frame {lo, hi, team frame's space, offset} on its own member
 *     stack and forks its inner team, four 16-lane groups, which take
 *     pieces of [lo, hi).  At depth 3 each group pushes a frame of the same
 *     shape, naming the wave's frame, on its own lane-group stack for four
 *     4-lane groups.  The innermost lanes reach the arrays by following the
 *     references.  Member stacks are on chip (64 B per wave, 16 B per lane
 *     group) with a global part (256 B, 64 B) taken when the on-chip part
 *     is full or DSR_F_NESTED_GLOBAL is set.
 *
 * DSR_BODY_FMA_CHAIN_REFS  the DSR_BODY_FMA_CHAIN loop, published with
 *     dsr_publish_list: no frame layout, a list of references instead
 *     (section 5.2): reference 0 the 24-byte exact sum slot, then ni int32
 *     scalars, nf fp64 scalars and, if alen > 0, the int32 array, each
 *     anywhere in any live frame.
 */
#define DSR_BODY_TERMINATE      0
#define DSR_BODY_AFFINE_XOR     1
#define DSR_BODY_FMA_CHAIN      2
#define DSR_BODY_GATHER         3
#define DSR_BODY_GATHER_NESTED  4
#define DSR_BODY_FMA_CHAIN_REFS 5

/* ---- configuration -------------------------------------------------------- */
#define DSR_F_TRACE        1u  /* record frame placements and barrier counts   */
#define DSR_F_TIMING       2u  /* record HIP events around every launch        */
#define DSR_F_GLOBAL_LISTS 4u  /* every published reference list goes to the
                                  HBM stack, however short (the global list of
                                  section 5.2, for comparison)                */
#define DSR_F_NESTED_GLOBAL 8u /* nested members' frames skip the on-chip part
                                  of their stacks (section 7's global stack,
                                  as when the on-chip part is exhausted)     */

typedef struct dsr_config {
    uint32_t wg_size;            /* threads per team: multiple of 64 in [64, 1024] */
    uint32_t lds_slab_bytes;     /* LDS stack capacity per team; 0 = every frame
                                    goes to the HBM slab (global stack only)     */
    uint32_t overflow_threshold; /* frames larger than this go to HBM; 0 = no limit */
    uint32_t master_joins;       /* 1: the master wave also runs loop iterations
                                    (forced when wg_size == 64; ignored above
                                    512 threads)                                 */
    uint64_t hbm_slab_bytes;     /* HBM stack capacity per team slot              */
    uint32_t max_teams;          /* team slots in the HBM slab (allocated once by
                                    dsr_init); a launch may not exceed it        */
    uint32_t flags;              /* DSR_F_* */
} dsr_config;

/* One published parallel loop.  Pointers are device pointers. */
typedef struct dsr_loop {
    uint64_t n;        /* iterations of the worksharing loop                   */
    uint64_t chunk;    /* iterations per team (0: ceil(n/teams) rounded up to 64,
                          or to 1024 when that is at least 16384);
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
    uint32_t depth;    /* GATHER_NESTED: parallel levels, 2 or 3 (0 = 2)        */
    uint32_t deref;    /* FMA_CHAIN_REFS: 1 = every batch of the loop reads each
                          shared scalar through its reference again, as outlined
                          code does when stores in the loop may alias the shared
                          variables (section 5.1); 0 = once per body call.
                          Scalars only (alen must be 0); 0 for other bodies    */
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

/* Start building a generic-mode target region that runs on `teams` teams
 * (1 .. cfg.max_teams).  Each team is its own contention group: one master
 * runs the sequential code while its workers wait to be handed parallel
 * work (section 4, Figure 2).  *out receives the region's program, empty;
 * the caller owns it until dsr_region_free.  DSR_E_INVAL for a bad team
 * count or NULL arguments. */
int dsr_region_begin(dsr_ctx *ctx, int32_t teams, dsr_region **out);

/* Master code block: push a frame of `nbytes` declared bytes (rounded up to
 * 16 on the stack).  This is the allocation of the master's implicitly
 * shared locals on the per-team shared-memory stack that replaces the
 * local depot (section 5.3.1), with the global-memory fallback of section
 * 5.2 taken on the device when the frame does not fit.  The frame's first `init_bytes` bytes are copied from
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

/* A reference to a shared variable: `offset` bytes into live frame `frame`. */
typedef struct dsr_ref {
    int32_t frame;
    uint32_t offset;
} dsr_ref;

#define DSR_LIST_ONCHIP 20     /* references the on-chip list holds (160 bytes) */

/* Publish `body` (DSR_BODY_FMA_CHAIN_REFS) through a list of `n` references
 * to the shared variables instead of a frame (section 5.1: the master hands
 * the workers a list of references; section 5.2: the runtime keeps a
 * 20-entry list in on-chip memory per team and falls back to a list in
 * global memory when more are needed).  Here a list of up to
 * DSR_LIST_ONCHIP references is written to the team's on-chip list; a
 * longer one (or any, with DSR_F_GLOBAL_LISTS) to a list frame of 8n bytes
 * pushed on the HBM stack at the fork and popped at the join, so a region
 * fails with DSR_E_NOMEM when the HBM stack cannot hold it.  Workers read
 * each reference, then the variable it names.  refs[k] must name a live
 * frame with the variable inside it and naturally aligned (slot and fp64:
 * 8 bytes; int32 and array: 4); n must be 1 + ni + nf + (alen > 0).
 * Errors as dsr_publish, DSR_E_STATE for a frame that is not live. */
int dsr_publish_list(dsr_region *r, const dsr_ref *refs, int32_t n, int32_t body, const dsr_loop *loop);

/* Bytes of LDS a team of `wg_size` threads uses besides its stack slab
 * (control block: descriptor, frame table, reference list, per-wave
 * reduction slots and nested-level sub-stacks); 0 for a bad size. */
uint32_t dsr_control_bytes(uint32_t wg_size);

/* Pop frame `frame`; it must be the most recently pushed live frame (the
 * shared stack of section 5.3.1 is released in LIFO order when the
 * master's locals go out of scope).  DSR_E_UNDERFLOW on an empty stack,
 * DSR_E_ORDER if not the top, DSR_E_STATE if `frame` is not live. */
int dsr_pop(dsr_region *r, int32_t frame);

/* Validate the program (DSR_E_LIVE if a frame is still live) and launch it
 * as one kernel of `teams` workgroups on `stream` (hipStream_t as void*):
 * the generic-mode kernel of section 4 (Figure 2: team init, the master's
 * sequential code with its forks and joins, the workers' loop of Figure 3,
 * terminate).
 * Asynchronous: results are available after dsr_region_sync.  A region may
 * be launched again (the same program over the same buffers) after its
 * previous launch, e.g. next on the same stream.  The stream must stay
 * valid until the region is synchronised or freed. */
int dsr_launch(dsr_region *r, void *stream);

/* Wait for the region's last launch and return its device status: DSR_OK,
 * DSR_E_NOMEM (a frame fit neither stack) or DSR_E_RANGE.  Without
 * DSR_F_TIMING no event marks the launch, so this waits for everything
 * queued on the launch stream so far. */
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
 *   [87], [88]            low words of the wall clock when the team's
 *                         program ended and when its arrival (and, for the
 *                         last team, the cross-team combine) was done
 *   [89 .. 91]            last reference list published: where (3 on chip,
 *                         1 HBM list frame), its offset, its entries (0: none)
 *   [92], [93]            low words of the wall clock when the team's
 *                         partials were stored and when its arrival atomic
 *                         returned
 *   [94], [95]            the team that combined the partials (the last to
 *                         arrive): when it began and when it finished
 *   [96 + 2w, 97 + 2w]    low words of the wall clock when wave w started
 *                         and finished its share of the last body it ran
 *   [128 + 8m .. 135 + 8m] nested member m (last nested body): its frame's
 *                         placement (space << 24 | offset; space 4 on chip,
 *                         5 global), its lane groups' frames (depth 3), a
 *                         pop-order error flag, nested pushes by the wave   */
#define DSR_TRACE_WORDS 256
int dsr_region_trace(dsr_region *r, int32_t team, uint32_t *buf, uint32_t n);

/* Duration of the last launch's kernel in milliseconds, from HIP events
 * recorded around it on its stream (needs DSR_F_TIMING; DSR_E_STATE
 * otherwise). */
int dsr_region_elapsed(dsr_region *r, float *ms);

/* Release a region's host and device memory (syncs its last launch).
 * DSR_E_STATE (nothing released) while a server holds requests of the
 * frozen region that read its device images and have not been collected
 * by dsr_serve_poll (or ended by dsr_serve_stop). */
int dsr_region_free(dsr_region *r);

/* Upload a finished region's program and frame images to the device
 * without launching it (what its first dsr_launch does; not in the paper):
 * the program can no longer change.  A served request of a frozen region
 * initialises frames larger than 1 KiB from this device copy instead of
 * from its request slot in host memory; dsr_region_free refuses the region
 * until those requests have been collected.  Synchronous (it allocates device memory): call
 * it before dsr_serve_start.  DSR_E_LIVE while a frame is live, DSR_E_INVAL
 * for more teams than max_teams, DSR_E_STATE for a host-only context,
 * DSR_E_NOMEM or DSR_E_HIP from the device.  Freezing twice is a no-op. */
int dsr_region_freeze(dsr_region *r);

/* ---- launch without allocation --------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * dsr_launch_static runs the same region kernel as dsr_launch, but every
 * device buffer the launch needs -- the region's descriptor, program, loop
 * descriptors and frame images, its teams' HBM stack slots (cfg.hbm_slab_bytes
 * each) and, when a nested body is published, their nested members' global
 * stacks, the cross-team partials and the result block -- lies in one fixed
 * device workspace of DSR_STATIC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends.  It calls no hipMalloc,
 * hipFree or other allocating routine: the program is copied in with
 * hipMemcpyAsync, the result block is cleared by a fill kernel, and the
 * result is written by a kernel to `result`, a device pointer to one
 * dsr_result_rec owned by the caller.  The region's context may be
 * host-only (device < 0: the current device is used) or a device context
 * (its own slab is not used).  Every call on one GPU uses the same
 * workspace and leaves its contents behind: calls whose launches overlap
 * on one GPU (other streams, or other threads) race and must be
 * serialised by the caller; one stream serialises them.
 * Errors: DSR_E_INVAL (null argument, or more teams than the context's
 * max_teams), DSR_E_LIVE (a frame still live), DSR_E_NOMEM (the launch
 * needs more than DSR_STATIC_SCRATCH_BYTES: teams x hbm_slab_bytes plus
 * the program and partials; see dsr_static_bytes), DSR_E_HIP.
 * Asynchronous; the record is complete when `stream` has reached it. */
#define DSR_STATIC_SCRATCH_BYTES (16u << 20)
typedef struct dsr_result_rec {
    int32_t status;           /* DSR_OK, DSR_E_NOMEM or DSR_E_RANGE              */
    int32_t n_red;            /* reductions recorded (publishes with a reduction) */
    double f64[8];            /* FMA_CHAIN: correctly rounded sums               */
    int64_t i64[8];           /* AFFINE_XOR: int64 sums                          */
    uint64_t fixed[8][3];     /* FMA_CHAIN: exact totals in units of 2^-75       */
} dsr_result_rec;
int dsr_launch_static(dsr_region *r, dsr_result_rec *result, void *stream);

/* Workspace bytes dsr_launch_static needs for region r (0 if r is NULL). */
uint64_t dsr_static_bytes(const dsr_region *r);

/* ---- batched form ---------------------------------------------------------
 * Not in the paper: the batched workload (10,000 region instances in one
 * persistent, graph-captured launch) built on the paper's runtime.
 * Many regions run in one persistent launch: workgroups stay resident and
 * their master waves claim (region, team) items from a device counter,
 * largest per-team work first, running each region's program as that team;
 * worker waves stay in the await loop across items (the paper's dynamic
 * work allocation, section 4, applied across regions).  The last team of a
 * region combines its reductions and stamps the region's completion time.
 * Results equal those of launching every region alone.  */
typedef struct dsr_batch dsr_batch;

typedef struct dsr_tune {
    uint32_t wg_size;            /* threads per workgroup (multiple of 64, 64..1024) */
    uint32_t lds_slab_bytes;     /* LDS stack per workgroup                        */
    uint32_t overflow_threshold; /* frames above this go to HBM (0 = no limit)     */
    uint32_t master_joins;       /* master wave runs iterations too                */
    uint32_t grid;               /* persistent workgroups (0 = as many as fit)     */
    uint32_t use_graph;          /* 1: capture the launch in a hipGraph once and
                                    replay it                                       */
} dsr_tune;

/* Pack `n` finished regions of context `ctx` (every frame popped) into a
 * batch: their programs, loop descriptors, initial frame bytes, partial
 * sums and results are copied into a few device arenas once.  The regions
 * may be freed afterwards.  The tune starts as the context's configuration. */
int dsr_batch_create(dsr_ctx *ctx, dsr_region *const *regions, int32_t n, dsr_batch **out);

/* Set the launch configuration (DSR_E_LDS / DSR_E_INVAL as for dsr_init;
 * DSR_E_NOMEM if `grid` exceeds the context's HBM slab slots). */
int dsr_batch_tune(dsr_batch *b, const dsr_tune *tune);

/* The tune in effect, with `grid` resolved to the workgroup count used. */
int dsr_batch_get_tune(dsr_batch *b, dsr_tune *out);

/* Run every region of the batch in one persistent launch on `stream`
 * (hipStream_t as void*; with use_graph the launch is a graph replay). */
int dsr_batch_launch(dsr_batch *b, void *stream);

/* Run the same regions with one kernel launch per region, in order, on
 * `stream` (the comparison form). */
int dsr_batch_launch_each(dsr_batch *b, void *stream);

/* Wait for the batch's last launch; returns the first region error or 0. */
int dsr_batch_sync(dsr_batch *b);

/* Reduction `index` of region `r` from the last launch (after sync), as
 * dsr_region_reduction; *status receives the region's error code. */
int dsr_batch_result(dsr_batch *b, int32_t r, int32_t index, int64_t *i64, double *f64,
                     uint64_t *fixed3, int32_t *status);

/* Completion times of the last launch in microseconds on the device's
 * 100 MHz clock: us[r] for region r, counted from the first item's claim
 * (persistent form) or from the start of the first region's kernel (one
 * launch per region). */
int dsr_batch_times(dsr_batch *b, double *us, int32_t n);

/* Duration of the last launch (either form) in milliseconds, from HIP
 * events around it. */
int dsr_batch_elapsed(dsr_batch *b, float *ms);

int dsr_batch_free(dsr_batch *b);

/* Autotuner (not in the paper): time `reps` persistent launches of the batch under each of
 * the `n_cand` candidate tunes (candidates that do not fit the device are
 * skipped), leave the fastest in effect, and return it in *best and every
 * candidate's mean milliseconds in ms[i] (negative if skipped). */
int dsr_autotune(dsr_batch *b, const dsr_tune *cand, int32_t n_cand, int32_t reps, void *stream,
                 dsr_tune *best, float *ms);

/* Candidates for dsr_autotune from the footprint and occupancy model (the
 * arithmetic of section 6.2 and Tables 4-7, applied to this kernel's
 * registers and the batch's stacks on this device; not in the paper): for
 * every workgroup size, LDS slabs sized to the batch's region stacks (the
 * median, 90th and 99th percentile and largest peak, rounded up to 1 KiB),
 * pruned to the largest slab per predicted number of resident teams per CU
 * (a larger slab keeps more frames on chip at no cost in residency), with
 * and without the master joining; ordered by predicted working waves per
 * CU.  Writes up to `max` tunes to `out` and the number of candidates to
 * *n_out.  DSR_E_INVAL for null arguments, DSR_E_HIP if the device cannot
 * be queried. */
int dsr_autotune_plan(dsr_batch *b, dsr_tune *out, int32_t max, int32_t *n_out);

/* ---- served form ----------------------------------------------------------
 * Not in the paper: the served workload (Poisson-arriving region requests
 * with admission by LDS and HBM budget) built on the paper's runtime.
 * A resident server kernel runs region requests as they arrive.  The host
 * submits a request (a finished region used as a program template) into a
 * free slot: its program, loop descriptors and frame images are copied into
 * the slot's host-coherent arena, its teams become items in a ring, and the
 * published count is advanced.  Persistent workgroups claim items as they
 * are published, so requests that arrive while others run overlap on the
 * device (continuous batching).  The last team of a request writes a
 * completion record that the host polls.
 *
 * Admission: a request is rejected with DSR_E_NOMEM if one of its teams'
 * frames fits neither the LDS stack of any class nor the HBM slot of a
 * server team (the same rule the device applies), and deferred with
 * DSR_E_BUSY while no slot
 * is free or while the LDS or HBM bytes of the admitted, unfinished
 * requests' team stacks would exceed the server's budget (the resident
 * teams' LDS slabs and HBM slots).  Budgets are returned on completion.
 *
 * The server closes when dsr_serve_stop is called, or by itself once no
 * request has been published for `idle_ms` (one decision for the whole
 * server, on the device clock).  Closing is all-or-none: every request
 * published before the close completes, and a submit that races the close
 * either runs or fails with DSR_E_STATE and takes its request back; after
 * the close every submit fails with DSR_E_STATE.  A device-wide
 * synchronisation (hipDeviceSynchronize) waits for the resident server
 * kernel, i.e. until it has closed and drained. */
typedef struct dsr_server dsr_server;

typedef struct dsr_serve_cfg {
    dsr_tune tune;            /* resident workgroups (grid 0 = as many as fit on
                                 the device less one per CU, or less one CU in
                                 32 when only one fits per CU)                    */
    uint32_t slots;           /* requests in flight at most                      */
    uint32_t slot_bytes;      /* frame-image bytes per slot                      */
    uint32_t max_teams;       /* teams per request at most (1 .. 65535)          */
    uint32_t ring_items;      /* item ring capacity (power of two)               */
    uint32_t idle_ms;         /* server exits after this long without new work  */
    uint32_t budget_pct;      /* admission budget, percent of the resident stacks
                                 (0 = 100)                                        */
    /* LDS classes (section 7's shared memory sized to what is needed, per
     * request): with n_classes > 0 the server runs one resident grid per
     * class, class k's teams having class_slab[k] bytes of on-chip stack
     * (a multiple of 16) and class_grid[k] workgroups (0: as for tune.grid
     * with that slab, divided by the number of classes); tune's
     * lds_slab_bytes and grid are then unused.  A request is admitted to
     * the smallest class whose slab holds its whole stack (dsr_serve_class_for),
     * or, while that class is full or closed, to the next larger one. */
    uint32_t n_classes;       /* 0: one class, tune.lds_slab_bytes            */
    uint32_t class_slab[4];
    uint32_t class_grid[4];
} dsr_serve_cfg;
#define DSR_SERVE_CLASSES 4

typedef struct dsr_done {
    uint64_t ticket;
    int32_t status;           /* DSR_OK, DSR_E_NOMEM or DSR_E_RANGE              */
    int32_t n_red;
    double f64[8];            /* reductions in publish order                     */
    int64_t i64[8];
    uint64_t fixed[8][3];
    double device_us;         /* device completion time, microseconds on the
                                 device clock since the server started           */
    int32_t lds_class;        /* the LDS class that ran the request              */
    int32_t pad;
} dsr_done;

/* Launch the server kernel on its own stream (not in the paper).  Regions submitted later must
 * belong to `ctx` and use one of the bodies compiled into the server (all
 * bodies; fixed-length fma chains up to 8+8 scalars, longer ones through the
 * run-time loop).  The server's kernel stays resident until it closes, and
 * other device work shares the CUs with it: the runtime's copies
 * (host<->device, staged or not) and fills run as kernels, so a grid that
 * holds every workgroup slot of the device (an explicit grid at the
 * occupancy limit) makes them wait until the server closes, and a caller
 * blocked on one then sees the server close after idle_ms with its later
 * submits failing with DSR_E_STATE.  The default grid leaves room for them.
 * A device-wide synchronisation, or an allocation or free that performs
 * one, also waits for the resident kernel: allocate the buffers requests use
 * before starting the server.  Fails with DSR_E_INVAL when slots is not in
 * 1 .. 65536, max_teams not in 1 .. 65535 (a ring item holds the slot and
 * the team in 16 bits each), slot_bytes is 0, ring_items is not a power of
 * two or below slots * max_teams, n_classes exceeds DSR_SERVE_CLASSES or
 * a class slab is not a multiple of 16. */
int dsr_serve_start(dsr_ctx *ctx, const dsr_serve_cfg *cfg, dsr_server **out);

/* Submit region `program` (its frames all popped) (not in the paper).
 * `outs` (may be NULL) replaces the output pointer of each of its loops,
 * so one template can serve many requests with separate output buffers.
 * *ticket identifies the request in dsr_serve_poll.  The server runs on a
 * stream of its own and may start the request at once: its input and
 * output buffers must be ready (any work producing or clearing them
 * finished) when this is called.  The program, its loop descriptors and
 * its frame images are copied into a request slot in host memory; frame
 * images over 1 KiB of a frozen template (dsr_region_freeze) are read from
 * the template's device copy instead, so such a template must outlive its
 * requests.  DSR_E_BUSY while no slot, ring space or stack budget is free
 * (poll and retry), DSR_E_NOMEM when no LDS class can place a frame,
 * DSR_E_INVAL for more than 16 ops, 4 loops, max_teams teams or
 * slot_bytes of images, DSR_E_LIVE for a live frame, DSR_E_STATE once the
 * server has closed. */
int dsr_serve_submit(dsr_server *s, dsr_region *program, void *const *outs, int32_t n_outs,
                     uint64_t *ticket);

/* Collect up to `max` completed requests (never blocks); returns how many
 * were written to `out`, or a negative error. */
int dsr_serve_poll(dsr_server *s, dsr_done *out, int32_t max);

/* Requests submitted and not yet collected by dsr_serve_poll. */
int dsr_serve_pending(dsr_server *s);

/* Replay an open-loop arrival schedule against the server from the calling
 * thread: request q (program programs[prog[q]]) arrives arrival_s[q] seconds
 * after the call (non-decreasing).  Requests are submitted in arrival
 * order as soon as they have arrived and are admitted (a deferred request
 * holds back the ones behind it); each writes its loops' outputs to
 * slot_outs[slot * n_loops_max + i] of the slot it was admitted into.  On
 * return latency_us[q] is its time from arrival to the host observing its
 * completion and done[q] its result.  Fails with DSR_E_BUSY if the
 * schedule has not finished `timeout_s` seconds after its last arrival. */
int dsr_serve_replay(dsr_server *s, dsr_region *const *programs, const int32_t *prog,
                     const double *arrival_s, int32_t n, void *const *slot_outs,
                     int32_t n_loops_max, double timeout_s, double *latency_us, dsr_done *done);

/* The comparison form: the same schedule served by one kernel launch per
 * request (batch region prog[q]) followed by a stream synchronisation, on
 * one stream; a request that arrives while another runs waits for it.
 * latency_us[q] is arrival to the end of its synchronisation; results are
 * read with dsr_batch_result after the call (they hold each region's last
 * run). */
int dsr_batch_replay_serial(dsr_batch *b, const int32_t *prog, const double *arrival_s, int32_t n,
                            double *latency_us);

/* Stop the server: the kernel runs every request published before the stop
 * and exits; then frees the server.  Completed requests not yet polled are
 * dropped. */
int dsr_serve_stop(dsr_server *s);

/* State of a server, for monitoring: its grid, how many of its workgroups
 * have started and left, whether it has closed (stop or idle) and how many
 * items it serves in all once closed, the items published so far and the
 * requests not yet collected.  A grid that never fully starts means the
 * device holds fewer of the server's workgroups at once than the occupancy
 * query promised; the server stays correct (no workgroup waits for
 * another) but serves with fewer teams. */
typedef struct dsr_serve_stat {
    uint32_t grid;
    uint32_t started;
    uint32_t exited;
    uint32_t closed;
    uint32_t final_items;
    uint32_t published;
    uint32_t in_flight;
    uint32_t classes;         /* LDS classes (resident grids)                    */
    /* the first class to close: why (0 open, 1 stop, 2 idle), its closing
     * workgroup, the item that workgroup waited for, the published count
     * it saw and the idle time it measured (microseconds) */
    uint32_t close_reason, close_block, close_item, close_seen;
    double close_idle_us;
    /* requests whose frame images team 0 relayed through device memory for
     * the other teams, and teams that stopped waiting for such a relay and
     * read the host slot instead (a nonzero count means a relay stalled) */
    uint32_t relays, relay_misses;
} dsr_serve_stat;
int dsr_serve_status(dsr_server *s, dsr_serve_stat *out);

/* The LDS class a request with program `r` is admitted to among `n`
 * classes of on-chip stack sizes `slabs` (1 <= n <= DSR_SERVE_CLASSES): the
 * smallest slab that holds the request's whole stack (the largest sum of
 * its live frames, each rounded up to 16 bytes), else the largest slab.
 * Host-only; returns the class index or DSR_E_INVAL. */
int dsr_serve_class_for(const uint32_t *slabs, int32_t n, const dsr_region *r);

/* ---- footprint and occupancy model ------------------------------------------
 * How many teams a compute unit holds at once, and what limits it, from
 * the resources one team needs (section 6.2: teams per SM from registers
 * per thread, threads per team, shared memory per team and the hardware's
 * block cap; section 8 notes such a model is easy to build).  Pure host
 * arithmetic: with K40/P100 parameters it reproduces the paper's
 * Tables 4-7, with gfx950's it predicts this runtime's occupancy. */
typedef struct dsr_hw_model {
    uint32_t compute_units;
    uint32_t regs_per_cu;          /* 32-bit registers per CU (SM)            */
    uint32_t reg_granule;          /* registers per thread are allocated in
                                      multiples of this                       */
    uint32_t max_teams_per_cu;     /* concurrent workgroups (blocks) per CU   */
    uint32_t max_threads_per_cu;
    uint32_t shared_per_cu;        /* shared memory (LDS) bytes per CU        */
    uint32_t shared_granule;       /* shared memory allocation granule        */
    uint32_t simds_per_cu;         /* 0: registers are one pool per CU (the
                                      paper's SM model); else each SIMD owns
                                      regs_per_cu / simds_per_cu registers
                                      and holds whole waves                   */
    uint32_t wave_size;            /* lanes per wave (used when simds_per_cu) */
} dsr_hw_model;

#define DSR_LIMIT_TEAMS      0     /* the hardware's workgroup cap            */
#define DSR_LIMIT_REGISTERS  1
#define DSR_LIMIT_SHARED     2
#define DSR_LIMIT_THREADS    3

typedef struct dsr_occupancy {
    uint32_t teams_per_cu;
    uint32_t teams_by_registers;
    uint32_t teams_by_shared;
    uint32_t teams_by_threads;
    uint32_t limiter;              /* DSR_LIMIT_*                             */
    uint32_t shared_per_team;      /* bytes, as allocated                     */
    uint64_t shared_per_cu;        /* teams_per_cu * shared_per_team          */
    uint32_t regs_per_thread;      /* as allocated                            */
    uint32_t hip_teams_per_cu;     /* dsr_region_occupancy: the HIP runtime's
                                      own answer for the kernel (0 otherwise) */
} dsr_occupancy;

int dsr_occupancy_model(const dsr_hw_model *hw, uint32_t threads_per_team,
                        uint32_t regs_per_thread, uint32_t shared_per_team,
                        dsr_occupancy *out);

/* The model for this runtime's region kernel on the context's device: the
 * kernel's registers per thread (compiled variant `variant` of the
 * context's workgroup size: 0..2 for the general instances, which hold
 * fixed fma chains up to 8+8, 16+16 and 32+32 scalars; 10 + k for the lean
 * instance of fixed chain k of (1,0) (1,1) (2,2) (4,4) (8,8) (16,16)
 * (32,32), which a single-region launch of workgroups up to 256 threads
 * runs when every publish of the region is that chain), the team's LDS
 * (control block plus stack slab) and the device's parameters. */
int dsr_region_occupancy(dsr_ctx *ctx, uint32_t variant, dsr_occupancy *out);

/* ---- measuring stick (not in the paper) -----------------------------------
 * The streaming ceiling of the fma-chain loop: y[i] = (double)x[i] for
 * i < n (x: n fp32, y: n fp64, device pointers), the loop's 4 B read and
 * 8 B write per element with no runtime around it: `grid` workgroups of
 * `wg_size` threads (a multiple of 64, at most 1024), each streaming one
 * contiguous chunk.  Asynchronous on `stream`.  DSR_E_INVAL for a bad shape
 * or a null buffer with n > 0. */
int dsr_stream_ceiling(const float *x, double *y, uint64_t n, uint32_t grid, uint32_t wg_size, void *stream);

/* Static string for a DSR_* code. */
const char *dsr_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* DSR_H */
