"""Pins the simulator's list-of-references publish (section 5.2) to the
plain fma-chain definition in oracle/ref.c, Python's math.fsum and the
stack invariants: where the list lives (on-chip for up to 20 references,
a global-memory list frame beyond), that the list frame lives exactly from
the fork to the join, and the errors of bad references."""
import math
import struct

import numpy as np
import pytest

import dsr_workloads as W
from oracle import ref as R
from oracle import sim as S


def chain_inputs(ni, nf, alen, n, seed=11):
    from dsr_workloads.gen import draws, uniform_int, uniform_f64
    s_i = uniform_int(draws(seed, 0, 0, ni), -(1 << 20), 1 << 20).astype(np.int32)
    s_f = uniform_f64(draws(seed, 1, 0, nf)) if nf else np.zeros(0)
    arr = uniform_int(draws(seed, 16, 0, alen), 0, (1 << 16) - 1).astype(np.int32) if alen else None
    x = W.uniform_f32_draws(seed, 2, 0, n)
    return s_i, s_f, arr, x


def refs_into_one_frame(ni, nf, alen):
    """References to the variables of one frame laid out as fma_chain's."""
    size, aoff = S.fma_chain_layout(ni, nf, alen)
    refs = [(0, 0)] + [(0, 24 + 8 * nf + 4 * k) for k in range(ni)] + [(0, 24 + 8 * k) for k in range(nf)]
    if alen:
        refs.append((0, aoff))
    return size, refs


@pytest.mark.parametrize("ni,nf,alen", [(1, 0, 0), (4, 4, 0), (8, 11, 0), (10, 9, 7), (16, 8, 0),
                                        (32, 16, 100)])
def test_list_publish_matches_plain_definition(ni, nf, alen):
    n = 203
    s_i, s_f, arr, x = chain_inputs(ni, nf, alen, n)
    size, refs = refs_into_one_frame(ni, nf, alen)
    y = np.zeros(n)
    prog = [S.Push(size, S.fma_chain_init(s_i, s_f, arr)),
            S.PublishList(refs, "fma_chain_refs", {"n": n, "x": x, "y": y, "ni": ni, "nf": nf, "alen": alen}),
            S.Pop(0)]
    tr, red = S.run_region(prog, 3, S.Config(workers=3, schedule="random", interleave="random", seed=2))
    yr = R.fma_chain(x, s_i, s_f, arr)
    assert np.array_equal(y, yr)
    assert red == [R.exact_sum(yr)] == [math.fsum(yr)]
    nrefs = len(refs)
    for t in tr:
        assert t.error is None
        space, off, entries = t.lists[0]
        assert entries == nrefs
        assert space == ("ctl" if nrefs <= 20 else "hbm")
        assert t.placements == [("lds", 0, S.round_up(size, 8))]    # the list frame is not a push


def test_list_spanning_frames_and_spaces():
    """Slot, scalars and array in three frames, one of them in global
    memory: the references reach each where it is."""
    ni, nf, alen, n = 3, 2, 50, 177
    s_i, s_f, arr, x = chain_inputs(ni, nf, alen, n, seed=12)
    scal = struct.pack("<%di" % ni, *s_i) + bytes(4) + struct.pack("<%dd" % nf, *s_f)
    y = np.zeros(n)
    refs = ([(2, 0)] + [(0, 4 * k) for k in range(ni)] + [(0, 16 + 8 * k) for k in range(nf)]
            + [(1, 0)])
    prog = [S.Push(len(scal), scal), S.Push(4 * alen, arr.tobytes()), S.Push(24),
            S.PublishList(refs, "fma_chain_refs", {"n": n, "x": x, "y": y, "ni": ni, "nf": nf, "alen": alen}),
            S.Pop(2), S.Pop(1), S.Pop(0)]
    cfg = S.Config(lds_bytes=128, workers=2, seed=3)         # the array goes to global memory
    tr, red = S.run_region(prog, 2, cfg)
    yr = R.fma_chain(x, s_i, s_f, arr)
    assert np.array_equal(y, yr) and red == [math.fsum(yr)]
    assert [p[0] for p in tr[0].placements] == ["lds", "hbm", "lds"]


def test_global_list_frame_lives_from_fork_to_join():
    ni, nf = 16, 8                                          # 25 references
    n = 64
    s_i, s_f, _, x = chain_inputs(ni, nf, 0, n, seed=13)
    size, refs = refs_into_one_frame(ni, nf, 0)
    y = np.zeros(n)
    loop = {"n": n, "x": x, "y": y, "ni": ni, "nf": nf}
    prog = [S.Push(size, S.fma_chain_init(s_i, s_f)), S.PublishList(refs, "fma_chain_refs", loop),
            S.PublishList(refs, "fma_chain_refs", loop), S.Pop(0)]
    tr, red = S.run_region(prog, 1, S.Config(workers=3))
    t = tr[0]
    # both lists sat at the bottom of the (otherwise empty) global stack
    assert t.lists == [("hbm", 0, 25), ("hbm", 0, 25)]
    yr = R.fma_chain(x, s_i, s_f)
    assert red == [math.fsum(yr), math.fsum(np.concatenate([yr, yr]))]


def test_global_list_out_of_memory():
    ni, nf = 16, 8
    size, refs = refs_into_one_frame(ni, nf, 0)
    s_i, s_f, _, x = chain_inputs(ni, nf, 0, 8, seed=14)
    prog = [S.Push(size, S.fma_chain_init(s_i, s_f)),
            S.PublishList(refs, "fma_chain_refs", {"n": 8, "x": x, "y": np.zeros(8), "ni": ni, "nf": nf}),
            S.Pop(0)]
    tr, red = S.run_region(prog, 1, S.Config(hbm_bytes=192))   # 25 * 8 = 200 bytes do not fit
    assert tr[0].error == "NOMEM" and red is None


def test_bad_references():
    s_i, s_f, _, x = chain_inputs(2, 1, 0, 8, seed=15)
    size, refs = refs_into_one_frame(2, 1, 0)
    loop = {"n": 8, "x": x, "y": np.zeros(8), "ni": 2, "nf": 1}
    init = S.fma_chain_init(s_i, s_f)
    cases = [
        ([S.Push(size, init), S.Pop(0), S.PublishList(refs, "fma_chain_refs", loop)], "STATE"),
        ([S.Push(size, init), S.PublishList([(0, 0), (0, size - 2), (0, 0), (0, 0)], "fma_chain_refs", loop),
          S.Pop(0)], "INVAL"),
        ([S.Push(size, init), S.PublishList(refs[:-1], "fma_chain_refs", loop), S.Pop(0)], "INVAL"),
        ([S.Push(size, init), S.PublishList([(0, 0), (0, 36), (0, 40), (0, 28)], "fma_chain_refs", loop),
          S.Pop(0)], "INVAL"),                                   # fp64 not 8-byte aligned
    # (section 5.3.1 keeps the shared stack's variables 8-byte aligned, so a
    # reference to an fp64 variable is to an 8-byte boundary)
        ([S.Push(size, init), S.PublishList(refs, "fma_chain", loop), S.Pop(0)], "INVAL"),
    ]
    for prog, code in cases:
        tr, _ = S.run_region(prog, 1)
        assert tr[0].error == code, (prog, tr[0].error)
