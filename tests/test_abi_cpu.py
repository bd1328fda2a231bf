"""The C-ABI library on a machine without a GPU: it loads, exports every
entry point its header declares, and rejects bad programs on the host with
the same error the contention-group simulator gives."""
import os
import re

import numpy as np
import pytest

from paper_1711_10413_amd import dsr as D
from oracle import sim as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h") or h == "dsr_device.h":
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"^\s*(?:int|uint32_t|uint64_t|const char \*)\s*(dsr_\w+)\s*\(", text, re.M))
    return names


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert names >= set(D.EXPORTS)
    lib = D.lib()
    for n in names:
        assert hasattr(lib, n), n


def host_ctx(**kw):
    return D.dsr_init(device=-1, **kw)


def test_bad_configs():
    for kw, code in [({"wg_size": 100}, D.DSR_E_INVAL), ({"wg_size": 2048}, D.DSR_E_INVAL),
                     ({"max_teams": 0}, D.DSR_E_INVAL), ({"lds_slab_bytes": 20}, D.DSR_E_INVAL),
                     ({"lds_slab_bytes": 160 * 1024}, D.DSR_E_LDS),
                     ({"hbm_slab_bytes": 17}, D.DSR_E_INVAL), ({"flags": 16}, D.DSR_E_INVAL),
                     ({"flags": 32}, D.DSR_E_INVAL)]:
        with pytest.raises(D.DsrError) as e:
            host_ctx(**kw)
        assert e.value.code == code, kw
    ctx = host_ctx(lds_slab_bytes=160 * 1024 - 2048)     # fits with a 4-wave control block
    D.dsr_destroy(ctx)


def run_host(prog_ops, teams=2):
    """Apply a list of ('push', n) / ('pop', h) / ('publish', h) to a region
    of a host-only context; returns the first error name or None, and then
    tries to launch (LIVE if a frame remains)."""
    ctx = host_ctx(lds_slab_bytes=64, hbm_slab_bytes=1024)
    r = D.dsr_region_begin(ctx, teams)
    try:
        for op, arg in prog_ops:
            if op == "push":
                D.dsr_push(r, arg)
            elif op == "pop":
                D.dsr_pop(r, arg)
            else:
                D.dsr_publish(r, arg, D.DSR_BODY_AFFINE_XOR, 8, out=0x1000)
        D.dsr_launch(r)
    except D.DsrError as e:
        return e.name
    finally:
        D.dsr_region_free(r)
        D.dsr_destroy(ctx)
    return None


def test_host_errors_match_simulator():
    out = np.zeros(8, np.int64)
    cases = [
        ([("push", 24), ("publish", 0)], [S.Push(24), S.Publish(0, "affine_xor", {"n": 8, "out": out})]),
        ([("push", 24), ("push", 8), ("pop", 0)], [S.Push(24), S.Push(8), S.Pop(0)]),
        ([("pop", 0)], [S.Pop(0)]),
        ([("push", 24), ("pop", 0), ("pop", 0)], [S.Push(24), S.Pop(0), S.Pop(0)]),
        ([("push", 24), ("pop", 0), ("publish", 0)],
         [S.Push(24), S.Pop(0), S.Publish(0, "affine_xor", {"n": 8, "out": out})]),
    ]
    for host_prog, sim_prog in cases:
        got = run_host(host_prog)
        tr, _ = S.run_region(sim_prog, 2, S.Config(lds_bytes=64, hbm_bytes=1024))
        want = tr[0].error
        # a pop of a never-pushed / dead handle is a state error on both sides
        assert got == want, (host_prog, got, want)
    # a host-only context validates but cannot launch
    assert run_host([("push", 24), ("pop", 0)]) == "STATE"


def test_publish_validation():
    ctx = host_ctx()
    r = D.dsr_region_begin(ctx, 4)
    f = D.dsr_push(r, 16)
    bad = [
        dict(body=D.DSR_BODY_AFFINE_XOR, n=8, out=0x1000),                  # frame < 24 B
        dict(body=D.DSR_BODY_FMA_CHAIN, n=8, inp=0x1000, out=0x2000, ni=1),  # frame < 28 B
        dict(body=D.DSR_BODY_GATHER, n=8, out=0x1000, arrays=1, length=8),   # frame < 32 B
        dict(body=D.DSR_BODY_GATHER, n=8, out=0x1000, arrays=0, length=4),
        dict(body=99, n=8, out=0x1000),
        dict(body=D.DSR_BODY_GATHER, n=64, out=0x1000, arrays=1, length=4, chunk=8),  # uncovered
        dict(body=D.DSR_BODY_GATHER, n=8, out=0, arrays=1, length=4),
    ]
    for kw in bad:
        body = kw.pop("body")
        with pytest.raises(D.DsrError) as e:
            D.dsr_publish(r, f, body, **kw)
        assert e.value.code == D.DSR_E_INVAL, kw
    D.dsr_publish(r, f, D.DSR_BODY_GATHER, 8, out=0x1000, arrays=1, length=4)
    D.dsr_pop(r, f)
    # a chain of more than 64 scalars is refused even when its frame is big enough
    g = D.dsr_push(r, 24 + 8 * 64 + 4)
    with pytest.raises(D.DsrError) as e:
        D.dsr_publish(r, g, D.DSR_BODY_FMA_CHAIN, 8, inp=0x1000, out=0x2000, ni=1, nf=64)
    assert e.value.code == D.DSR_E_INVAL
    D.dsr_publish(r, g, D.DSR_BODY_FMA_CHAIN, 8, inp=0x1000, out=0x2000, ni=0, nf=64)
    D.dsr_pop(r, g)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_region_limits():
    ctx = host_ctx(max_teams=8)
    with pytest.raises(D.DsrError):
        D.dsr_region_begin(ctx, 9)
    r = D.dsr_region_begin(ctx, 8)
    hs = [D.dsr_push(r, 16) for _ in range(16)]
    with pytest.raises(D.DsrError):
        D.dsr_push(r, 16)                       # deeper than 16 live frames
    for h in reversed(hs):
        D.dsr_pop(r, h)
    with pytest.raises(D.DsrError) as e:
        D.dsr_pop(r, 0)
    assert e.value.code == D.DSR_E_UNDERFLOW
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_dynamic_tail_validation():
    ctx = host_ctx()
    r = D.dsr_region_begin(ctx, 4)
    f = D.dsr_push(r, 64)
    g = D.dsr_push(r, 64, bytes(64 * 4), init_stride=64)      # per-team frame copies
    bad = [dict(frame=f, chunk=128), dict(frame=f, block=100), dict(frame=f, block=1 << 17),
           dict(frame=f, tail_pct=100), dict(frame=g), dict(frame=f, body=D.DSR_BODY_GATHER_NESTED)]
    for kw in bad:
        frame = kw.pop("frame")
        body = kw.pop("body", D.DSR_BODY_GATHER)
        with pytest.raises(D.DsrError) as e:
            D.dsr_publish(r, frame, body, 1000, out=0x1000, arrays=1, length=4, schedule=1, **kw)
        assert e.value.code == D.DSR_E_INVAL, kw
    D.dsr_publish(r, f, D.DSR_BODY_GATHER, 1000, out=0x1000, arrays=1, length=4, schedule=1)
    with pytest.raises(D.DsrError):
        D.dsr_publish(r, f, D.DSR_BODY_GATHER, 1000, out=0x1000, arrays=1, length=4, schedule=2)
    D.dsr_pop(r, g)
    D.dsr_pop(r, f)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_publish_list_validation():
    """Host checks of dsr_publish_list, with the simulator's code where it
    has the same case."""
    ctx = host_ctx()
    r = D.dsr_region_begin(ctx, 2)
    f = D.dsr_push(r, 24 + 8 * 2 + 4 * 3)          # slot, 2 fp64, 3 int32
    good = [(f, 0), (f, 40), (f, 44), (f, 48), (f, 24), (f, 32)]
    kw = dict(inp=0x1000, out=0x2000, ni=3, nf=2)
    bad = [
        (good[:-1], {}, D.DSR_E_INVAL),                              # one reference short
        ([(f, 0), (f, 40), (f, 44), (f, 48), (f, 26), (f, 32)], {}, D.DSR_E_INVAL),  # fp64 misaligned
        ([(f, 0), (f, 40), (f, 44), (f, 60), (f, 24), (f, 32)], {}, D.DSR_E_INVAL),  # outside the frame
        ([(f + 1, 0)] + good[1:], {}, D.DSR_E_STATE),                 # no such frame
        (good, {"body": D.DSR_BODY_FMA_CHAIN}, D.DSR_E_INVAL),        # body takes a frame
    ]
    for refs, extra, code in bad:
        body = extra.get("body", D.DSR_BODY_FMA_CHAIN_REFS)
        with pytest.raises(D.DsrError) as e:
            D.dsr_publish_list(r, refs, body, 8, **kw)
        assert e.value.code == code, (refs, extra)
    with pytest.raises(D.DsrError) as e:                              # fma_chain_refs needs a list
        D.dsr_publish(r, f, D.DSR_BODY_FMA_CHAIN_REFS, 8, **kw)
    assert e.value.code == D.DSR_E_INVAL
    D.dsr_publish_list(r, good, D.DSR_BODY_FMA_CHAIN_REFS, 8, **kw)
    D.dsr_pop(r, f)
    with pytest.raises(D.DsrError) as e:                              # frame popped
        D.dsr_publish_list(r, good, D.DSR_BODY_FMA_CHAIN_REFS, 8, **kw)
    assert e.value.code == D.DSR_E_STATE
    D.dsr_region_free(r)
    # the simulator reports the same codes for a popped frame and a reference
    # outside its frame
    x = np.zeros(8, np.float32)
    for refs, prog_tail, code in [(good, "popped", "STATE"),
                                  ([(0, 0), (0, 40), (0, 44), (0, 60), (0, 24), (0, 32)], "", "INVAL")]:
        refs = [(0, o) for _, o in refs]
        prog = [S.Push(52)]
        if prog_tail == "popped":
            prog.append(S.Pop(0))
        prog.append(S.PublishList(refs, "fma_chain_refs", {"n": 8, "x": x, "y": np.zeros(8), "ni": 3, "nf": 2}))
        if prog_tail != "popped":
            prog.append(S.Pop(0))
        tr, _ = S.run_region(prog, 1)
        assert tr[0].error == code
    assert D.dsr_control_bytes(256) == 64 + 16 * 16 + 20 * 8 + 4 * 32 + 4 * (64 + 4 * 16 + 48)
    D.dsr_destroy(ctx)


@pytest.mark.parametrize("ni,nf,alen,lds,flags", [(4, 4, 0, 4096, 0), (10, 9, 33, 4096, 0), (32, 32, 0, 4096, 0),
                                                  (32, 31, 100, 8192, 0), (8, 8, 0, 4096, 4), (16, 4, 50, 0, 0)])
def test_list_programs_pass_host_checks(ni, nf, alen, lds, flags):
    """The GPU list tests' programs, through a host-only context."""
    ctx = host_ctx(wg_size=256, lds_slab_bytes=lds, hbm_slab_bytes=8192, max_teams=64, flags=flags | 1)
    size, aoff = S.fma_chain_layout(ni, nf, alen)
    refs = [(0, 0)] + [(0, 24 + 8 * nf + 4 * k) for k in range(ni)] + [(0, 24 + 8 * k) for k in range(nf)]
    if alen:
        refs.append((0, aoff))
    r = D.dsr_region_begin(ctx, 5)
    f = D.dsr_push(r, size)
    D.dsr_publish_list(r, refs, D.DSR_BODY_FMA_CHAIN_REFS, 100003, inp=0x1000, out=0x2000, ni=ni, nf=nf, alen=alen)
    D.dsr_pop(r, f)
    D.dsr_region_free(r)
    # three frames: scalars (fp64 after 8-byte padding), array, slot
    r = D.dsr_region_begin(ctx, 4)
    f0 = D.dsr_push(r, 5 * 4 + 4 + 3 * 8)
    f1 = D.dsr_push(r, 4 * 3000)
    f2 = D.dsr_push(r, 24)
    refs = [(f2, 0)] + [(f0, 4 * k) for k in range(5)] + [(f0, 24 + 8 * k) for k in range(3)] + [(f1, 0)]
    D.dsr_publish_list(r, refs, D.DSR_BODY_FMA_CHAIN_REFS, 77777, inp=0x1000, out=0x2000, ni=5, nf=3, alen=3000)
    D.dsr_pop(r, f2)
    D.dsr_pop(r, f1)
    D.dsr_pop(r, f0)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_nested_depth_is_checked_on_the_host():
    ctx = host_ctx(lds_slab_bytes=4096, hbm_slab_bytes=4096)
    for depth, code in ((0, 0), (2, 0), (3, 0), (1, D.DSR_E_INVAL), (4, D.DSR_E_INVAL)):
        r = D.dsr_region_begin(ctx, 2)
        f = D.dsr_push(r, 64)
        try:
            D.dsr_publish(r, f, D.DSR_BODY_GATHER_NESTED, 100, out=1 << 20, arrays=1, length=16, depth=depth)
            got = 0
        except D.DsrError as e:
            got = e.code
        assert got == code, depth
        D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_static_launch_host_checks():
    """The launch without allocation rejects, before any device work, a
    region whose buffers exceed the fixed workspace, a live frame and a
    missing result pointer."""
    ctx = host_ctx(wg_size=256, lds_slab_bytes=4096, hbm_slab_bytes=65536, max_teams=1024)
    r = D.dsr_region_begin(ctx, 256)           # 256 x 64 KiB stack slots = 16 MiB + program
    f = D.dsr_push(r, 24, D.affine_xor_frame(1, 2, 3, 4))
    assert D.lib().dsr_launch_static(r, 16, None) == D.DSR_E_LIVE
    D.dsr_publish(r, f, D.DSR_BODY_AFFINE_XOR, 1024, out=16)
    D.dsr_pop(r, f)
    assert D.dsr_static_bytes(r) > D.DSR_STATIC_SCRATCH_BYTES
    assert D.lib().dsr_launch_static(r, 16, None) == D.DSR_E_NOMEM
    assert D.lib().dsr_launch_static(r, None, None) == D.DSR_E_INVAL
    r2 = D.dsr_region_begin(ctx, 128)
    f = D.dsr_push(r2, 24, D.affine_xor_frame(1, 2, 3, 4))
    D.dsr_publish(r2, f, D.DSR_BODY_AFFINE_XOR, 1024, out=16)
    D.dsr_pop(r2, f)
    assert 128 * 65536 < D.dsr_static_bytes(r2) <= D.DSR_STATIC_SCRATCH_BYTES
    D.dsr_region_free(r)
    D.dsr_region_free(r2)
    D.dsr_destroy(ctx)


def test_freeze_host_checks():
    """Freezing refuses a live frame and a host-only context before any
    device work."""
    ctx = host_ctx(wg_size=256, lds_slab_bytes=4096, hbm_slab_bytes=65536, max_teams=4)
    r = D.dsr_region_begin(ctx, 4)
    f = D.dsr_push(r, 24, D.affine_xor_frame(1, 2, 3, 4))
    assert D.lib().dsr_region_freeze(r) == D.DSR_E_LIVE
    D.dsr_publish(r, f, D.DSR_BODY_AFFINE_XOR, 1024, out=16)
    D.dsr_pop(r, f)
    assert D.lib().dsr_region_freeze(r) == D.DSR_E_STATE
    assert D.lib().dsr_region_freeze(None) == D.DSR_E_INVAL
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_deref_only_for_scalar_lists():
    """Per-batch reads through the list (deref) exist for the list publish of
    scalars only: a frame publish or a list with an array is refused."""
    ctx = host_ctx(wg_size=256, lds_slab_bytes=4096, hbm_slab_bytes=4096, max_teams=8)
    r = D.dsr_region_begin(ctx, 2)
    f = D.dsr_push(r, 48, b"")
    L = D.dsr_loop(100, 0, 16, 16, 2, 1, 0, 0, 0, 0, 0, 0, 0, 1)
    assert D.lib().dsr_publish(r, f, D.DSR_BODY_FMA_CHAIN, D.C.byref(L)) == D.DSR_E_INVAL
    refs = [(f, 0), (f, 32), (f, 36), (f, 24)]
    D.dsr_publish_list(r, refs, D.DSR_BODY_FMA_CHAIN_REFS, 100, inp=16, out=16, ni=2, nf=1, deref=1)
    g = D.dsr_push(r, 64, b"")
    with pytest.raises(D.DsrError) as e:
        D.dsr_publish_list(r, [(g, 0), (g, 32), (g, 36), (g, 24), (g, 48)], D.DSR_BODY_FMA_CHAIN_REFS, 100,
                           inp=16, out=16, ni=2, nf=1, alen=3, deref=1)
    assert e.value.code == D.DSR_E_INVAL
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)
