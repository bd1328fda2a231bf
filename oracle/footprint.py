"""The paper's static shared-memory and occupancy arithmetic -- TEST
INFRASTRUCTURE.

Section 6.2.1: a team's static shared memory is its shared stack plus the
pre-allocated list of 20 references (160 bytes) plus the thread-private
runtime state (49 bytes).  The shared stack holds 16 bytes of runtime
locals (two 8-byte slots: team number and thread number) plus one 8-byte
slot per shared scalar, or 24 bytes plus the arrays' bytes (96 int32 each)
for the array program.  More than 20 shared entities need a dynamically
allocated global list of 8 bytes per entity (section 5.2).

Sections 6.2.2-6.2.4: teams per SM are limited by registers (65536 per SM,
128 threads per team), by the hardware cap on concurrent blocks, and by
shared memory; shared memory per SM is teams times the team footprint.
"""

PREALLOC = 160       # 20 references x 8 bytes (section 5.2)
PRIVATE = 49         # thread-private runtime state (section 6.2.1)
LIST_ENTRIES = 20


def shared_stack_scalars(n):
    return 16 + 8 * n


def shared_stack_arrays(n, elems=96, elem_bytes=4):
    return 24 + n * elems * elem_bytes


def team_footprint(stack):
    return stack + PREALLOC + PRIVATE


def dynamic_global_list(n_shared):
    return 8 * n_shared if n_shared > LIST_ENTRIES else 0


def teams_by_registers(regs, threads=128, regs_per_sm=65536, cap=16):
    return min(cap, regs_per_sm // (regs * threads))


def teams_actual(potential, footprint, shared_per_sm):
    return min(potential, shared_per_sm // footprint)


def max_regs_for_teams(teams, threads=128, regs_per_sm=65536, reg_cap=255):
    return min(reg_cap, regs_per_sm // (teams * threads))
