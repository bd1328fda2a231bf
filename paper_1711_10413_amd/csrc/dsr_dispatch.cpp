/*
 * dsr_dispatch.cpp -- routes a launch to the compiled instance of the
 * region kernel that fits its workgroup size and the bodies its regions
 * publish.  Each instance lives in its own object (dsr_kernels.hip built
 * once per entry of DSR_INSTANCES).
 */
#include <stdint.h>

#include "dsr_internal.h"

#define DSR_DECLARE(tag, maxwg, variant)                                                                    \
    extern "C" int dsr_inst_launch_##tag(const dsr_dlaunch *, const dsr_dconfig *, uint32_t, uint32_t,     \
                                         uint32_t, void *);                                                 \
    extern "C" int dsr_inst_occupancy_##tag(uint32_t, uint32_t);                                           \
    extern "C" int dsr_inst_regs_##tag(void);
DSR_INSTANCES(DSR_DECLARE)
#undef DSR_DECLARE

namespace {

struct instance {
    uint32_t maxwg;
    int variant;
    int (*launch)(const dsr_dlaunch *, const dsr_dconfig *, uint32_t, uint32_t, uint32_t, void *);
    int (*occupancy)(uint32_t, uint32_t);
    int (*regs)(void);
};

#define DSR_ENTRY(tag, maxwg, variant) \
    {maxwg, variant, dsr_inst_launch_##tag, dsr_inst_occupancy_##tag, dsr_inst_regs_##tag},
const instance kInstances[] = {DSR_INSTANCES(DSR_ENTRY)};
#undef DSR_ENTRY

/* Workgroups above 512 threads run the 1024-thread instance (run-time
 * chains only), 257-512 the 512-thread one; up to 256 threads the variant
 * the regions need, or the lean instance a single region of one fixed
 * chain asks for. */
const instance *pick(uint32_t wg_size, uint32_t variant)
{
    if (variant >= DSR_LEAN_BASE) {
        if (wg_size > 256 || variant >= DSR_LEAN_BASE + DSR_LEAN_CHAINS) return nullptr;
        for (const instance &k : kInstances)
            if (k.maxwg == 256u && k.variant == (int)variant) return &k;
        return nullptr;
    }
    const uint32_t maxwg = wg_size > 512 ? 1024u : (wg_size > 256 ? 512u : 256u);
    const int want = maxwg == 1024 ? -1 : (maxwg == 512 ? 0 : (int)(variant > 2 ? 2 : variant));
    for (const instance &k : kInstances)
        if (k.maxwg == maxwg && k.variant == want) return &k;
    return nullptr;
}

}  // namespace

extern "C" int dsr_launch_region_kernel(const dsr_dlaunch *lp, const dsr_dconfig *cfg, uint32_t grid,
                                        uint32_t wg_size, uint32_t lds_bytes, uint32_t variant, void *stream)
{
    const instance *k = pick(wg_size, variant);
    return k ? k->launch(lp, cfg, grid, wg_size, lds_bytes, stream) : 1 /* hipErrorInvalidValue */;
}

extern "C" int dsr_region_kernel_occupancy(uint32_t wg_size, uint32_t lds_bytes, uint32_t variant)
{
    const instance *k = pick(wg_size, variant);
    return k ? k->occupancy(wg_size, lds_bytes) : 0;
}

extern "C" int dsr_region_kernel_regs(uint32_t wg_size, uint32_t variant)
{
    const instance *k = pick(wg_size, variant);
    return k ? k->regs() : 0;
}
