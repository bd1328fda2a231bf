/*
 * Internal device-side descriptors shared by the host library and the
 * kernels of libdsr.so (not part of the public ABI).
 */
#ifndef DSR_INTERNAL_H
#define DSR_INTERNAL_H

#include <stdint.h>

#define DSR_MAX_RED 8
#define DSR_MAX_OPS 64
#define DSR_MAX_LOOPS 16

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
    uint32_t len, schedule, block, pad;
    uint64_t dyn_start;    /* first iteration of the dynamic tail (= n if none) */
};

/* Per-launch result block (device memory, written by the last team). */
struct dsr_dresult {
    int32_t error;         /* accumulating: first team error of this launch */
    uint32_t arrived;      /* teams that finished; reset by the last team   */
    int32_t final_error;   /* the launch's error, written by the last team  */
    uint32_t done;         /* launch counter, bumped by the last team       */
    uint32_t claim[DSR_MAX_LOOPS]; /* dynamic-tail block counters; reset by the last team */
    uint64_t fixed[DSR_MAX_RED][3];
    double f64[DSR_MAX_RED];
    int64_t i64[DSR_MAX_RED];
};

/* Everything one region needs on the device. */
struct dsr_dregion {
    const dsr_op *ops;
    const dsr_dloop *loops;
    const uint8_t *init;
    uint64_t *partials;    /* [n_red][teams][3] */
    dsr_dresult *result;
    uint32_t *trace;       /* [teams][DSR_TRACE_WORDS] or null */
    uint32_t n_ops;
    uint32_t teams;
    uint32_t n_red;
    uint32_t red_kind_mask; /* bit r set: reduction r is FMA_CHAIN (exact fp64) */
};

/* Launch-wide configuration. */
struct dsr_dconfig {
    uint8_t *hbm_base;     /* HBM slab: max_teams slots                     */
    uint64_t hbm_slot_bytes;
    uint32_t nw;           /* waves per team                                */
    uint32_t lds_cap;
    uint32_t threshold;
    uint32_t master_joins;
    uint32_t trace;
    uint32_t pad;
};

#ifdef __cplusplus
extern "C" {
#endif
/* Kernel launchers (dsr_kernels.hip). Return hipError_t as int. */
int dsr_launch_region_kernel(const dsr_dregion *reg, const dsr_dconfig *cfg,
                             uint32_t wg_size, uint32_t lds_bytes, uint32_t variant,
                             void *stream);
#ifdef __cplusplus
}
#endif

#endif
