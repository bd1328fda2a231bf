"""GPU parity of the list-of-references publish (section 5.2) with the CPU
oracle: the fma chain through up to 66 references, on-chip lists (up to 20
references) and global lists on the HBM stack, variables spread over
frames in LDS and HBM, against oracle/ref.c and the simulator's list
placement."""
import math
import struct
import sys

import numpy as np
import pytest

import dsr_workloads as W
from oracle import ref as R
from oracle import sim as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1711_10413_amd import dsr as D  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def stream():
    return torch.cuda.current_stream().cuda_stream


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the HIP path")
    torch.cuda.init()
    yield


def chain_inputs(ni, nf, alen, n, seed=21):
    from dsr_workloads.gen import draws, uniform_int, uniform_f64
    s_i = uniform_int(draws(seed, 0, 0, ni), -(1 << 20), 1 << 20).astype(np.int32)
    s_f = uniform_f64(draws(seed, 1, 0, nf)) if nf else np.zeros(0)
    arr = uniform_int(draws(seed, 16, 0, alen), 0, (1 << 16) - 1).astype(np.int32) if alen else None
    return s_i, s_f, arr, W.uniform_f32_draws(seed, 2, 0, n)


def one_frame_refs(ni, nf, alen):
    size, aoff = S.fma_chain_layout(ni, nf, alen)
    refs = [(0, 0)] + [(0, 24 + 8 * nf + 4 * k) for k in range(ni)] + [(0, 24 + 8 * k) for k in range(nf)]
    if alen:
        refs.append((0, aoff))
    return size, refs


def check(r, x_np, s_i, s_f, y, arr=None):
    yr = R.fma_chain(x_np, s_i, s_f, arr)
    assert np.array_equal(y.cpu().numpy().view(np.uint64), yr.view(np.uint64))
    _, f64, fixed = D.dsr_region_reduction(r, 0)
    assert fixed == R.fixed75_sum(yr)
    assert f64 == R.exact_sum(yr) == math.fsum(yr)


@pytest.mark.parametrize("ni,nf,alen,lds,flags", [
    (4, 4, 0, 4096, 0),            # 9 references: on-chip list
    (10, 9, 0, 4096, 0),           # 20: the on-chip list's capacity
    (10, 9, 33, 4096, 0),          # 21 with the array: a global list
    (32, 32, 0, 4096, 0),          # 65 references (two rounds of lanes)
    (32, 31, 100, 8192, 0),        # 65 with an array
    (8, 8, 0, 4096, D.DSR_F_GLOBAL_LISTS),   # short list forced to global memory
    (16, 4, 50, 0, 0),             # every frame in HBM, global list
])
def test_list_publish(ni, nf, alen, lds, flags):
    n = 100003
    say("list", ni, nf, alen, lds, flags)
    s_i, s_f, arr, x_np = chain_inputs(ni, nf, alen, n)
    size, refs = one_frame_refs(ni, nf, alen)
    init = S.fma_chain_init(s_i, s_f, arr)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=lds, hbm_slab_bytes=8192, max_teams=64,
                     flags=flags | D.DSR_F_TRACE)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    r = D.dsr_region_begin(ctx, 5)
    f = D.dsr_push(r, size, init)
    D.dsr_publish_list(r, refs, D.DSR_BODY_FMA_CHAIN_REFS, n, inp=x.data_ptr(), out=y.data_ptr(),
                       ni=ni, nf=nf, alen=alen)
    D.dsr_pop(r, f)
    D.dsr_launch(r, stream())
    assert D.dsr_region_sync(r) == 0
    check(r, x_np, s_i, s_f, y, arr)
    # placement of the list against the simulator's
    cfg = S.Config(lds_bytes=lds, hbm_bytes=8192, align=16)   # the kernel's frame rounding
    ys = np.zeros(64)
    prog = [S.Push(size, init),
            S.PublishList(refs, "fma_chain_refs", {"n": 64, "x": x_np[:64], "y": ys, "ni": ni, "nf": nf,
                                                   "alen": alen}), S.Pop(0)]
    tr, _ = S.run_region(prog, 1, cfg)
    sspace, soff, sn = tr[0].lists[0]
    glist = bool(flags & D.DSR_F_GLOBAL_LISTS) or len(refs) > D.DSR_LIST_ONCHIP
    assert (sspace == "hbm") == (len(refs) > D.DSR_LIST_ONCHIP)
    space, off, entries = D.dsr_region_trace(r, 0)["list"]
    assert entries == len(refs) == sn
    assert space == ("hbm" if glist else "onchip")
    if glist and sspace == "hbm":
        assert off == soff
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_list_across_frames_and_spaces():
    """Slot, scalars and array in three frames, the array in HBM."""
    ni, nf, alen, n = 5, 3, 3000, 77777
    s_i, s_f, arr, x_np = chain_inputs(ni, nf, alen, n, seed=22)
    scal = struct.pack("<%di" % ni, *s_i) + bytes(4) + struct.pack("<%dd" % nf, *s_f)
    refs = ([(2, 0)] + [(0, 4 * k) for k in range(ni)] + [(0, 24 + 8 * k) for k in range(nf)]
            + [(1, 0)])
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=1024, hbm_slab_bytes=16384, max_teams=64,
                     flags=D.DSR_F_TRACE)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    r = D.dsr_region_begin(ctx, 4)
    f0 = D.dsr_push(r, len(scal), scal)
    f1 = D.dsr_push(r, 4 * alen, arr.tobytes())
    f2 = D.dsr_push(r, 24)
    D.dsr_publish_list(r, refs, D.DSR_BODY_FMA_CHAIN_REFS, n, inp=x.data_ptr(), out=y.data_ptr(),
                       ni=ni, nf=nf, alen=alen)
    D.dsr_pop(r, f2)
    D.dsr_pop(r, f1)
    D.dsr_pop(r, f0)
    D.dsr_launch(r, stream())
    assert D.dsr_region_sync(r) == 0
    check(r, x_np, s_i, s_f, y, arr)
    assert [p[0] for p in D.dsr_region_trace(r, 0)["placements"]] == ["lds", "hbm", "lds"]
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_global_list_nomem_and_relaunch():
    ni, nf = 16, 8                                   # 25 references: 200 bytes of list
    s_i, s_f, _, x_np = chain_inputs(ni, nf, 0, 5000, seed=23)
    size, refs = one_frame_refs(ni, nf, 0)
    init = S.fma_chain_init(s_i, s_f)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(x.numel(), dtype=torch.float64, device="cuda")
    # no room for the list in a 192-byte HBM slot
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=4096, hbm_slab_bytes=192, max_teams=8)
    r = D.dsr_region_begin(ctx, 2)
    f = D.dsr_push(r, size, init)
    D.dsr_publish_list(r, refs, D.DSR_BODY_FMA_CHAIN_REFS, x.numel(), inp=x.data_ptr(), out=y.data_ptr(),
                       ni=ni, nf=nf)
    D.dsr_pop(r, f)
    D.dsr_launch(r, stream())
    assert D.dsr_region_sync(r) == D.DSR_E_NOMEM
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)
    # two list publishes in one region, launched twice: the list frame is
    # popped at each join, so both sit at the bottom of the HBM stack
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=4096, hbm_slab_bytes=256, max_teams=8,
                     flags=D.DSR_F_TRACE)
    r = D.dsr_region_begin(ctx, 3)
    f = D.dsr_push(r, size, init)
    for _ in range(2):
        D.dsr_publish_list(r, refs, D.DSR_BODY_FMA_CHAIN_REFS, x.numel(), inp=x.data_ptr(),
                           out=y.data_ptr(), ni=ni, nf=nf)
    D.dsr_pop(r, f)
    yr = R.fma_chain(x_np, s_i, s_f)
    for _ in range(2):
        D.dsr_launch(r, stream())
        assert D.dsr_region_sync(r) == 0
        assert D.dsr_region_trace(r, 1)["list"] == ("hbm", 0, 25)
        assert D.dsr_region_reduction(r, 0)[1] == math.fsum(yr)
        assert D.dsr_region_reduction(r, 1)[1] == math.fsum(np.concatenate([yr, yr]))
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_list_regions_in_a_batch():
    """List-published and frame-published regions side by side in one
    persistent launch."""
    regs, want, ys = [], [], []
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=8192, hbm_slab_bytes=8192, max_teams=256)
    keep = []
    for q, (ni, nf, alen) in enumerate([(4, 4, 0), (16, 8, 20), (2, 1, 5), (32, 32, 0)]):
        n = 20000 + 3001 * q
        s_i, s_f, arr, x_np = chain_inputs(ni, nf, alen, n, seed=30 + q)
        size, refs = one_frame_refs(ni, nf, alen)
        x = torch.from_numpy(x_np).cuda()
        y = torch.zeros(n, dtype=torch.float64, device="cuda")
        keep += [x, y]
        r = D.dsr_region_begin(ctx, 3)
        f = D.dsr_push(r, size, S.fma_chain_init(s_i, s_f, arr))
        if q % 2:
            D.dsr_publish(r, f, D.DSR_BODY_FMA_CHAIN, n, inp=x.data_ptr(), out=y.data_ptr(),
                          ni=ni, nf=nf, alen=alen)
        else:
            D.dsr_publish_list(r, refs, D.DSR_BODY_FMA_CHAIN_REFS, n, inp=x.data_ptr(), out=y.data_ptr(),
                               ni=ni, nf=nf, alen=alen)
        D.dsr_pop(r, f)
        regs.append(r)
        yr = R.fma_chain(x_np, s_i, s_f, arr)
        want.append(yr)
        ys.append(y)
    torch.cuda.synchronize()
    b = D.dsr_batch_create(ctx, regs)
    for use_graph in (0, 1):
        for y in ys:
            y.zero_()
        torch.cuda.synchronize()
        D.dsr_batch_tune(b, wg_size=256, lds_slab_bytes=8192, use_graph=use_graph)
        D.dsr_batch_launch(b, stream())
        assert D.dsr_batch_sync(b) == 0
        for q, yr in enumerate(want):
            _, f64, fixed, st = D.dsr_batch_result(b, q)
            assert st == 0 and f64 == math.fsum(yr) and fixed == R.fixed75_sum(yr)
            assert np.array_equal(ys[q].cpu().numpy(), yr)
    D.dsr_batch_free(b)
    for r in regs:
        D.dsr_region_free(r)
    D.dsr_destroy(ctx)


@pytest.mark.parametrize("ni,nf,lds,flags", [
    (4, 4, 4096, 0),                       # on-chip list, frame in LDS
    (10, 9, 4096, D.DSR_F_GLOBAL_LISTS),   # global list, frame in LDS
    (32, 32, 4096, 0),                     # 65 references: a global list
    (3, 5, 0, 0),                          # frame in HBM, on-chip list
])
def test_list_read_every_batch(ni, nf, lds, flags):
    """deref=1: every batch reads each scalar through its reference again;
    the results are those of the hoisted reads and of the oracle."""
    n = (1 << 17) + 77
    say("list deref", ni, nf, lds, flags)
    s_i, s_f, _, x_np = chain_inputs(ni, nf, 0, n, seed=23)
    size, refs = one_frame_refs(ni, nf, 0)
    init = S.fma_chain_init(s_i, s_f, None)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=lds, hbm_slab_bytes=8192, max_teams=64, flags=flags)
    x = torch.from_numpy(x_np).cuda()
    for deref in (1, 0):
        y = torch.full((n,), -3.0, dtype=torch.float64, device="cuda")
        r = D.dsr_region_begin(ctx, 7)
        f = D.dsr_push(r, size, init)
        D.dsr_publish_list(r, refs, D.DSR_BODY_FMA_CHAIN_REFS, n, inp=x.data_ptr(), out=y.data_ptr(),
                           ni=ni, nf=nf, deref=deref)
        D.dsr_pop(r, f)
        D.dsr_launch(r, stream())
        assert D.dsr_region_sync(r) == 0
        check(r, x_np, s_i, s_f, y)
        D.dsr_region_free(r)
    D.dsr_destroy(ctx)
