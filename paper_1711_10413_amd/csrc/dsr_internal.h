/*
 * Internal device-side descriptors shared by the host library and the
 * kernels of libdsr.so (not part of the public ABI).
 */
#ifndef DSR_INTERNAL_H
#define DSR_INTERNAL_H

#include <stddef.h>
#include <stdint.h>

#define DSR_MAX_RED 8
#define DSR_MAX_OPS 64
#define DSR_PART_WORDS 3   /* a 192-bit partial: three 64-bit words, low first */
#define DSR_MAX_LOOPS 16
#ifndef DSR_ARRIVE_GROUPS
#define DSR_ARRIVE_GROUPS 32
#endif

enum : uint32_t { DSR_OP_PUSH = 1, DSR_OP_PUBLISH = 2, DSR_OP_POP = 3 };

/* One step of the master's program. */
struct dsr_op {
    uint32_t kind;
    uint32_t frame;        /* frame handle (push index)                    */
    uint32_t nbytes;       /* PUSH: declared bytes                          */
    uint32_t init_bytes;   /* PUSH: bytes copied from the init blob         */
    uint32_t init_stride;  /* PUSH: per-team stride in the blob (0 = shared) */
    uint32_t body;         /* PUBLISH: body id                              */
    uint32_t loop;         /* PUBLISH: loop descriptor index                */
    uint32_t red;          /* PUBLISH: reduction index or 0xffffffff        */
    uint64_t init_off;     /* PUSH: offset of the init bytes in the blob    */
    uint64_t pad;
};

struct dsr_dloop {
    uint64_t n;
    uint64_t chunk;        /* static iterations per team                    */
    const void *in;
    void *out;
    uint32_t ni, nf, alen, arrays;
    uint32_t len, schedule, block, depth;   /* depth: nested levels (nested body) */
    uint64_t dyn_start;    /* first iteration of the dynamic tail (= n if none) */
    uint32_t deref;        /* list body: re-read the references every batch  */
    uint32_t pad;
};

/* Per-launch result block (device memory, written by the last team).  The
 * fields the host reads come first: it copies only DSR_RESULT_HOST_BYTES. */
struct dsr_dresult {
    int32_t error;         /* accumulating: first team error of this launch */
    uint32_t arrived;      /* teams that finished; reset by the last team   */
    int32_t final_error;   /* the launch's error, written by the last team  */
    uint32_t done;         /* launch counter, bumped by the last team       */
    uint64_t fixed[DSR_MAX_RED][3];
    double f64[DSR_MAX_RED];
    int64_t i64[DSR_MAX_RED];
    /* device-side counters from here on */
    uint32_t claim[DSR_MAX_LOOPS]; /* dynamic-tail block counters; reset by the last team */
    /* arrival tree: teams count into DSR_ARRIVE_GROUPS group counters (64 B
     * apart), the last team of each group into `arrived` */
    uint32_t group[DSR_ARRIVE_GROUPS * 16];
};
#define DSR_RESULT_HOST_BYTES offsetof(dsr_dresult, claim)

/* Everything one region needs on the device. */
struct dsr_dregion {
    const dsr_op *ops;
    const dsr_dloop *loops;
    const uint8_t *init;
    uint64_t *partials;    /* [n_red][teams][DSR_PART_WORDS] */
    dsr_dresult *result;
    uint32_t *trace;       /* [teams][DSR_TRACE_WORDS] or null */
    uint32_t n_ops;
    uint32_t teams;
    uint32_t n_red;
    uint32_t red_kind_mask; /* bit r set: reduction r is FMA_CHAIN (exact fp64) */
    uint64_t tag;           /* served form: request ticket written on completion */
    uint32_t n_loops;
    uint32_t init_size;     /* bytes of the init blob                          */
    /* served form: a device buffer the request's team 0 copies the init
     * blob into from the host slot (null: every team reads the slot), and
     * the word it then sets to `tag` */
    uint8_t *relay;
    uint64_t *relay_flag;
};

/* Program parts a single-region launch carries in its kernel arguments. */
#define DSR_INLINE_OPS 4
#define DSR_INLINE_IMG 512

/* Served form limits (a request's program is copied into LDS per item).  A
 * request slot in host memory has the layout of the LDS copy: its
 * descriptor (128 B reserved), DSR_SERVE_MAX_OPS ops at 128,
 * DSR_SERVE_MAX_LOOPS loop descriptors at 896 and the frame images from
 * DSR_SERVE_SLOT_HEAD on, so a team copies the head and the images' first
 * bytes in one round of loads.
 * A ring item is one 64-bit word: the item's position in the ring's
 * sequence (upper 32 bits), the slot (bits 16-31) and the team (bits 0-15),
 * so a reader can tell a stale word from the item it waits for. */
#define DSR_SERVE_MAX_OPS 16
#define DSR_SERVE_MAX_LOOPS 4
#define DSR_SERVE_OPS_AT 128
#define DSR_SERVE_LOOPS_AT (DSR_SERVE_OPS_AT + DSR_SERVE_MAX_OPS * 48)
#define DSR_SERVE_LDS_BYTES (DSR_SERVE_LOOPS_AT + DSR_SERVE_MAX_LOOPS * 80)
#define DSR_SERVE_SLOT_HEAD 1280
/* The first DSR_SERVE_IMG_LDS bytes of the frame images come in the same
 * round; a request whose whole init blob fits initialises its frames from
 * that LDS copy.  The LDS area a server team reserves after its stack: */
#define DSR_SERVE_IMG_LDS 1024
#define DSR_SERVE_AREA_BYTES (DSR_SERVE_SLOT_HEAD + DSR_SERVE_IMG_LDS)
/* A request whose teams would read at least this many image bytes from the
 * host slot in all has them relayed through device memory by its team 0. */
#define DSR_SERVE_RELAY_MIN (64u * 1024u)
static_assert(sizeof(dsr_op) == 48 && sizeof(dsr_dloop) == 80, "served LDS copy layout");
static_assert(sizeof(dsr_dregion) <= DSR_SERVE_OPS_AT, "served descriptor fits the slot head");
static_assert(DSR_SERVE_LDS_BYTES <= DSR_SERVE_SLOT_HEAD && DSR_SERVE_LDS_BYTES % 16 == 0, "served slot head");

/* Served form: completion record of one request slot, in host-coherent
 * memory.  The device fills it and then stores `seq` (the request ticket)
 * with system-scope release; the host polls `seq`. */
struct dsr_drec {
    uint64_t seq;
    int32_t status;
    uint32_t n_red;
    uint64_t ticks;         /* device wall clock at completion (100 MHz) */
    double f64[DSR_MAX_RED];
    int64_t i64[DSR_MAX_RED];
    uint64_t fixed[DSR_MAX_RED][3];
};

/* What one launch runs.  Single region: regions[0] on gridDim.x teams,
 * team = blockIdx.x.  Batch: persistent workgroups claim items (region,
 * team) from counter[0] until n_items are done; the last workgroup to
 * leave resets the counters. */
struct dsr_dlaunch {
    const dsr_dregion *regions;
    const uint32_t *items;  /* [n_items][2] = {region, team}, or null; served
                               form: the ring of 64-bit items */
    uint32_t n_items;
    uint32_t n_regions;
    uint32_t *counter;      /* [0] next item, [1] workgroups finished;
                               served form, see DSR_SRV_* below */
    uint64_t *done_ts;      /* per region: wall clock when its result was written;
                               [n_regions]: when item 0 was claimed */
    /* served form (published != null): items arrive over time in a ring */
    const uint32_t *published; /* host-coherent: items published so far   */
    const uint32_t *stop;      /* host-coherent: nonzero = close the server */
    dsr_drec *recs;            /* host-coherent completion records, per slot */
    uint32_t ring_mask;        /* ring capacity - 1 (power of two)          */
    uint32_t region_stride;    /* served form: bytes between request slots
                                  (regions[] is then the first slot)       */
    uint32_t *closing;         /* host-coherent: set by the device when it
                                  starts to close the server                */
    uint32_t *final_items;     /* host-coherent: 1 + the published count the
                                  device serves before it leaves (0 = open)  */
    uint32_t *wg_started;      /* host-coherent, per workgroup: 1 once it runs */
    uint32_t *wg_exited;       /* host-coherent, per workgroup: 1 once it left */
    uint32_t *relays;          /* host-coherent: [0] requests whose images team 0
                                  relayed, [1] teams that gave up waiting */
    uint64_t *start_ts;        /* if set, block 0 stamps its start time here */
    uint64_t idle_limit;       /* close after a waiting workgroup saw the
                                  published count unchanged for this many
                                  ticks of its own clock                    */
    /* Single-region launches (items == null) may carry the region's
     * descriptor by value and, for a program of at most DSR_INLINE_OPS ops,
     * its ops, its first loop descriptor and the initial image of the frame
     * its first op pushes (the same image for every team), so that a team
     * forks without reading any of them from memory first. */
    uint32_t has_single;       /* `single` holds regions[0]                 */
    uint32_t inl_ops;          /* ops held in inl_op (0: read them from memory) */
    uint32_t inl_loop;         /* inl_loop0 holds loop 0                    */
    uint32_t inl_img;          /* image bytes held in inl_image (a multiple
                                  of 16, zero-padded; 0: none)              */
    dsr_dregion single;
    dsr_dloop inl_loop0;
    dsr_op inl_op[DSR_INLINE_OPS];
    uint8_t inl_image[DSR_INLINE_IMG];
};

/* Served form: control words in device memory (LP.counter, 32-bit words).
 * The claim counter, the device copy of the host's published count, the
 * server state and the item count it serves before leaving. */
#define DSR_SRV_CLAIM 0
#define DSR_SRV_PUB 16
#define DSR_SRV_STATE 32      /* 0 open, 1 closing, 2 closed            */
#define DSR_SRV_FINAL 48      /* valid once the state is 2              */
#define DSR_SRV_WORDS 128

/* Launch-wide configuration. */
struct dsr_dconfig {
    uint8_t *hbm_base;     /* HBM slab: max_teams slots                     */
    uint64_t hbm_slot_bytes;
    uint32_t nw;           /* waves per team                                */
    uint32_t lds_cap;
    uint32_t threshold;
    uint32_t master_joins;
    uint32_t trace;
    uint32_t serve;        /* served form: per-item program copy after the stack */
    uint32_t global_lists; /* every reference list goes to the HBM stack      */
    uint32_t nest_global;  /* nested frames skip the on-chip member stacks     */
    uint8_t *nest_base;    /* nested members' global stacks: one slot of
                              DSR_NEST_SLOT bytes per workgroup               */
};

/* Global part of the nested member stacks per workgroup: room for the
 * largest team (16 waves) whatever the launch's workgroup size. */
#define DSR_NEST_SLOT (16u * DSR_NEST_HBM_WAVE)

/* Compiled instances of the region kernel: (tag, largest workgroup, variant).
 * The build compiles dsr_kernels.hip once per entry, in parallel, and
 * dsr_dispatch.cpp routes each launch to one of them. */
#define DSR_INSTANCES(X) \
    X(256_0, 256, 0)     \
    X(256_1, 256, 1)     \
    X(256_2, 256, 2)     \
    X(512_0, 512, 0)     \
    X(1024_m1, 1024, -1) \
    X(256_l0, 256, 10)   \
    X(256_l1, 256, 11)   \
    X(256_l2, 256, 12)   \
    X(256_l3, 256, 13)   \
    X(256_l4, 256, 14)   \
    X(256_l5, 256, 15)   \
    X(256_l6, 256, 16)

/* Lean instances: variant DSR_LEAN_BASE + k runs single-region launches of
 * workgroups up to 256 threads whose publishes are all the fixed fma chain
 * k, (DSR_LEAN_NI(k) int32, DSR_LEAN_NF(k) fp64 scalars), with no array. */
#define DSR_LEAN_BASE 10
#define DSR_LEAN_CHAINS 7
#define DSR_LEAN_NI(k) ((k) == 0 ? 1 : (k) == 1 ? 1 : (k) == 2 ? 2 : (k) == 3 ? 4 : (k) == 4 ? 8 : (k) == 5 ? 16 : 32)
#define DSR_LEAN_NF(k) ((k) == 0 ? 0 : DSR_LEAN_NI(k))

#ifdef __cplusplus
extern "C" {
#endif
/* The fixed device workspace (dsr_static.hip): its address on `device`,
 * a word fill kernel and the result-record copy kernel. */
int dsr_static_workspace(int device, uint8_t **out);
int dsr_static_fill(void *p, uint32_t words, uint32_t value, void *stream);
int dsr_static_copy_result(const void *result_block, uint32_t n_red, void *dst, void *stream);
/* Kernel launchers (dsr_dispatch.cpp). Return hipError_t as int. */
int dsr_launch_region_kernel(const dsr_dlaunch *lp, const dsr_dconfig *cfg, uint32_t grid,
                             uint32_t wg_size, uint32_t lds_bytes, uint32_t variant,
                             void *stream);
/* Workgroups of the region kernel that fit on one CU at once (0 on error). */
int dsr_region_kernel_occupancy(uint32_t wg_size, uint32_t lds_bytes, uint32_t variant);
/* Registers per thread of the region kernel variant (0 on error). */
int dsr_region_kernel_regs(uint32_t wg_size, uint32_t variant);
#ifdef __cplusplus
}
#endif

#endif
