"""Pins of the served form's LDS classes (section 7: shared memory sized to
what a request needs): the class a request goes to is the smallest whose
on-chip stack makes the contention-group simulator place every one of the
request's frames on chip, else the largest; and the library's host rule
gives the same class for the same programs."""
import itertools
import random

import pytest

from oracle import sim as S


def programs(rng, n):
    """Random push/pop programs (LIFO, every frame popped) of up to four
    frames of 1..600 bytes."""
    out = []
    for _ in range(n):
        prog, live, pushes = [], [], 0
        for _ in range(rng.randint(1, 8)):
            if live and rng.random() < 0.4:
                prog.append(S.Pop(live.pop()))
            elif pushes < 4:
                prog.append(S.Push(rng.randint(1, 600)))
                live.append(pushes)
                pushes += 1
        while live:
            prog.append(S.Pop(live.pop()))
        out.append(prog)
    return out


def all_on_chip(program, slab, align):
    """The simulator's own placement: every frame of the program on chip
    when the team's on-chip stack holds `slab` bytes."""
    cfg = S.Config(lds_bytes=slab, hbm_bytes=1 << 16, align=align)
    tr, _ = S.run_region(program, 1, cfg)
    return tr[0].error is None and all(sp == "lds" for sp, _, _ in tr[0].placements)


@pytest.mark.parametrize("align", [8, 16])
def test_class_is_smallest_slab_that_keeps_every_frame_on_chip(align):
    rng = random.Random(5)
    slabs = [256, 1024, 64, 4096]
    for prog in programs(rng, 300):
        k = S.lds_class(prog, slabs, align)
        ok = [c for c in range(len(slabs)) if all_on_chip(prog, slabs[c], align)]
        if ok:
            assert k in ok and slabs[k] == min(slabs[c] for c in ok)
        else:
            assert slabs[k] == max(slabs)


def test_stack_peak_brute_force():
    """The peak against every prefix of the program, frame by frame."""
    for sizes in itertools.product([1, 8, 9, 24], repeat=3):
        for shape in ("nested", "sequential", "mixed"):
            if shape == "nested":
                prog = [S.Push(s) for s in sizes] + [S.Pop(2), S.Pop(1), S.Pop(0)]
            elif shape == "sequential":
                prog = [S.Push(sizes[0]), S.Pop(0), S.Push(sizes[1]), S.Pop(1), S.Push(sizes[2]), S.Pop(2)]
            else:
                prog = [S.Push(sizes[0]), S.Push(sizes[1]), S.Pop(1), S.Push(sizes[2]), S.Pop(2), S.Pop(0)]
            r8 = [((s + 7) // 8) * 8 for s in sizes]
            want = {"nested": sum(r8), "sequential": max(r8), "mixed": r8[0] + max(r8[1], r8[2])}[shape]
            assert S.stack_peak(prog, 8) == want


def test_library_rule_matches_simulator():
    """dsr_serve_class_for on host-only regions built from the same programs
    gives the simulator's class (the kernel rounds frames to 16 bytes)."""
    from paper_1711_10413_amd import dsr as D
    ctx = D.dsr_init(device=-1, wg_size=256, lds_slab_bytes=4096, hbm_slab_bytes=1 << 16, max_teams=4)
    rng = random.Random(9)
    slab_sets = [[256, 1024, 64, 4096], [512], [16, 32], [2048, 128, 8192]]
    for prog in programs(rng, 200):
        r = D.dsr_region_begin(ctx, 1)
        handles = []
        for op in prog:
            if isinstance(op, S.Push):
                handles.append(D.dsr_push(r, op.nbytes, b""))
            else:
                D.dsr_pop(r, handles[op.frame])
        for slabs in slab_sets:
            assert D.dsr_serve_class_for(slabs, r) == S.lds_class(prog, slabs, 16), (prog, slabs)
        D.dsr_region_free(r)
    D.dsr_destroy(ctx)
