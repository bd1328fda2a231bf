"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer and index results must be bit-exact; fp64 results too (every y is a
correctly rounded fma chain, and the reduction is the exactly rounded sum),
so all comparisons here are exact equality.  Stack behaviour (frame
placement, barrier counts) is compared with the contention-group
simulator's trace.
"""
import math
import sys

import numpy as np
import pytest

import dsr_workloads as W
from oracle import ref as R
from oracle import sim as S

# frame rounding of the kernel (an implementation choice: 128-bit LDS reads)
KERNEL_ALIGN = 16

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1711_10413_amd import dsr as D  # noqa: E402

LDS_MAX4 = 163840 - D.dsr_control_bytes(256)   # LDS stack that fills a 4-wave team's 160 KiB


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


def t_i32(n):
    return torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")


def run_region(ctx, teams, build):
    """build(region) pushes/publishes/pops; returns (status, region)."""
    r = D.dsr_region_begin(ctx, teams)
    build(r)
    D.dsr_launch(r, stream())
    return D.dsr_region_sync(r), r


# ---- Figure 1b pattern: four shared int32 scalars --------------------------
def affine_program(c, n, out):
    def build(r):
        f = D.dsr_push(r, 24, D.affine_xor_frame(c.a, c.b, c.c, c.d))
        D.dsr_publish(r, f, D.DSR_BODY_AFFINE_XOR, n, out=out.data_ptr())
        D.dsr_pop(r, f)
    return build


@pytest.mark.parametrize("wg,joins", [(256, 0), (256, 1), (64, 0), (1024, 0)])
def test_cfg1_plain_region(wg, joins):
    say("cfg1 wg", wg, "joins", joins)
    c = W.cfg1_inputs()
    ctx = D.dsr_init(wg_size=wg, lds_slab_bytes=4096, hbm_slab_bytes=4096, max_teams=4,
                     master_joins=joins, flags=D.DSR_F_TRACE)
    out = t_i32(1024)
    st, r = run_region(ctx, 4, affine_program(c, 1024, out))
    assert st == 0
    i64, _, _ = D.dsr_region_reduction(r, 0)
    ro, rs = R.affine_xor(c.a, c.b, c.c, c.d, 0, 1024)
    assert np.array_equal(out.cpu().numpy(), ro)
    assert i64 == rs == 523776 * c.a + 1024 * (c.b + c.d) - 1024 * (c.c & ~1023) - 523776
    # trace against the simulator: placement and Figure 2/3 barrier counts
    sim_out = np.zeros(1024, np.int64)
    prog = [S.Push(24, S.affine_xor_init(c.a, c.b, c.c, c.d)),
            S.Publish(0, "affine_xor", {"n": 1024, "out": sim_out}), S.Pop(0)]
    nw = wg // 64
    # the kernel rounds frames to 16 bytes (its LDS reads are 128-bit), not the
    # paper's 8: the simulator takes the kernel's rounding for this comparison
    traces, red = S.run_region(prog, 4, S.Config(lds_bytes=4096, hbm_bytes=4096,
                                                 workers=max(1, nw - 1), align=KERNEL_ALIGN))
    assert red == [rs]
    for t in range(4):
        tr = D.dsr_region_trace(r, t)
        assert tr["error"] == 0
        assert tr["placements"] == traces[t].placements
        assert tr["barriers"][:nw] == [traces[t].master_barriers] * nw
    # the same region launched again gives the same answer
    for _ in range(3):
        out.zero_()
        D.dsr_launch(r, stream())
        assert D.dsr_region_sync(r) == 0
        assert D.dsr_region_reduction(r, 0)[0] == rs
        assert np.array_equal(out.cpu().numpy(), ro)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_cfg1_each_team_reads_its_own_frame():
    say("cfg1 per-team frames")
    teams = 4
    cs = [W.cfg1_inputs(team=t) for t in range(teams)]
    img = b"".join(D.affine_xor_frame(c.a, c.b, c.c, c.d) + bytes(8) for c in cs)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=1024, max_teams=teams)
    out = t_i32(1024)

    def build(r):
        f = D.dsr_push(r, 24, img, init_stride=32, init_bytes=24)
        D.dsr_publish(r, f, D.DSR_BODY_AFFINE_XOR, 1024, out=out.data_ptr(), chunk=256)
        D.dsr_pop(r, f)
    st, r = run_region(ctx, teams, build)
    assert st == 0
    want, total = [], 0
    for t, c in enumerate(cs):
        o, s = R.affine_xor(c.a, c.b, c.c, c.d, 256 * t, 256 * (t + 1))
        want.append(o)
        total += s
    assert np.array_equal(out.cpu().numpy(), np.concatenate(want))
    assert D.dsr_region_reduction(r, 0)[0] == total
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


# ---- Figure 5 pattern: K shared scalars, fma chain, exact reduction ---------
def fma_region(ctx, teams, s_i32, s_f64, x, y, arr=None, chunk=0, schedule=0, tail_pct=0, block=0):
    img, size = D.fma_chain_frame(s_i32, s_f64, arr)

    def build(r):
        f = D.dsr_push(r, size, img)
        D.dsr_publish(r, f, D.DSR_BODY_FMA_CHAIN, x.numel(), inp=x.data_ptr(), out=y.data_ptr(),
                      ni=len(s_i32), nf=len(s_f64), alen=0 if arr is None else len(arr),
                      chunk=chunk, schedule=schedule, tail_pct=tail_pct, block=block)
        D.dsr_pop(r, f)
    return run_region(ctx, teams, build)


def check_fma(r, x_np, s_i32, s_f64, y, arr=None):
    yr = R.fma_chain(x_np, s_i32, s_f64, arr)
    yg = y.cpu().numpy()
    assert np.array_equal(yg.view(np.uint64), yr.view(np.uint64))
    _, f64, fixed = D.dsr_region_reduction(r, 0)
    assert fixed == R.fixed75_sum(yr)
    assert f64 == R.exact_sum(yr) == math.fsum(yr)


@pytest.mark.parametrize("K", W.CFG2_KS)
@pytest.mark.parametrize("wg,joins", [(256, 0), (256, 1)])
def test_cfg2_scalar_sweep_small(K, wg, joins):
    say("cfg2 small K", K, "wg", wg, "joins", joins)
    n = 3 * 4096 + 13                                   # several teams, a ragged tail
    cf, x_np = W.cfg2_inputs(K, n=n)
    ctx = D.dsr_init(wg_size=wg, lds_slab_bytes=4096, max_teams=64, master_joins=joins)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, 5, cf.s_i32, cf.s_f64, x, y)
    assert st == 0
    check_fma(r, x_np, cf.s_i32, cf.s_f64, y)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


@pytest.mark.parametrize("K", W.CFG2_KS)
@pytest.mark.parametrize("schedule", [D.DSR_SCHED_STATIC, D.DSR_SCHED_DYNAMIC_TAIL])
def test_cfg2_full_size(K, schedule):
    """512 teams x 256 threads over 2**24 elements: the benchmarked shape,
    launched twice (the dynamic-tail counters reset between launches)."""
    say("cfg2 full K", K, "schedule", schedule)
    cf, x_np = W.cfg2_inputs(K)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=4096, max_teams=512)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(x.numel(), dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, 512, cf.s_i32, cf.s_f64, x, y, schedule=schedule)
    assert st == 0
    check_fma(r, x_np, cf.s_i32, cf.s_f64, y)
    y.zero_()
    D.dsr_launch(r, stream())
    assert D.dsr_region_sync(r) == 0
    check_fma(r, x_np, cf.s_i32, cf.s_f64, y)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


@pytest.mark.parametrize("K", [1, 8, 64])
@pytest.mark.parametrize("tail_pct,block,joins", [(25, 1024, 0), (99, 128, 1), (50, 65536, 0),
                                                  (10, 384, 1)])
def test_cfg2_dynamic_tail_small(K, tail_pct, block, joins):
    say("cfg2 dynamic K", K, tail_pct, block, joins)
    n = 200003
    cf, x_np = W.cfg2_inputs(K, n=n)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=4096, max_teams=64, master_joins=joins)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, 9, cf.s_i32, cf.s_f64, x, y, schedule=1, tail_pct=tail_pct, block=block)
    assert st == 0
    check_fma(r, x_np, cf.s_i32, cf.s_f64, y)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_dynamic_tail_many_blocks_per_lane():
    """A single team claims every block of a long tail: each lane adds far
    more than 2**16 values, which the bins only hold exactly because the
    claimed blocks flush them."""
    say("dynamic tail long")
    n = 1 << 23
    cf, x_np = W.cfg2_inputs(8, n=n)
    ctx = D.dsr_init(wg_size=64, lds_slab_bytes=4096, max_teams=4)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, 1, cf.s_i32, cf.s_f64, x, y, schedule=1, tail_pct=99, block=65536)
    assert st == 0
    check_fma(r, x_np, cf.s_i32, cf.s_f64, y)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


@pytest.mark.parametrize("A,length,hbm_only", [(1, 16, 0), (4, 4096, 0), (2, 16384, 1), (3, 100, 0)])
def test_gather_dynamic_tail(A, length, hbm_only):
    say("gather dynamic", A, length, hbm_only)
    arrs = W.cfg3_arrays(A, length)
    n = (1 << 18) + 5
    frame = 4 * A * length
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=0 if hbm_only else LDS_MAX4,
                     hbm_slab_bytes=(frame + 15) // 16 * 16, max_teams=16)
    out = t_i32(n)

    def build(r):
        f = D.dsr_push(r, frame, D.gather_frame(arrs))
        D.dsr_publish(r, f, D.DSR_BODY_GATHER, n, out=out.data_ptr(), arrays=A, length=length,
                      schedule=1, tail_pct=40, block=512)
        D.dsr_pop(r, f)
    st, r = run_region(ctx, 16, build)
    assert st == 0
    assert np.array_equal(out.cpu().numpy(), R.gather(arrs, 0, n))
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_affine_dynamic_tail():
    say("affine dynamic")
    c = W.cfg1_inputs()
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=4096, max_teams=4)
    n = 100000
    out = t_i32(n)

    def build(r):
        f = D.dsr_push(r, 24, D.affine_xor_frame(c.a, c.b, c.c, c.d))
        D.dsr_publish(r, f, D.DSR_BODY_AFFINE_XOR, n, out=out.data_ptr(), schedule=1,
                      tail_pct=60, block=256)
        D.dsr_pop(r, f)
    st, r = run_region(ctx, 4, build)
    assert st == 0
    ro, rs = R.affine_xor(c.a, c.b, c.c, c.d, 0, n)
    assert np.array_equal(out.cpu().numpy(), ro) and D.dsr_region_reduction(r, 0)[0] == rs
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


@pytest.mark.parametrize("inst", [0, 1, 7, 42, 1234, 9999])
@pytest.mark.parametrize("lds", [LDS_MAX4, 0])
def test_generic_chain_with_array(inst, lds):
    """Batched-workload instances: run-time scalar counts plus a shared
    int32 array, frames in LDS or forced to the HBM slab."""
    Ls, Fs = W.cfg4_descriptors()
    L = int(min(Ls[inst], 70001))
    ins = W.cfg4_instance(inst, L, int(Fs[inst]))
    say("generic inst", inst, "L", L, "F", ins.F, "lds", lds)
    x_np = W.instance_x(inst, L)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=lds, hbm_slab_bytes=65536, max_teams=64)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(L, dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, 3, ins.s_i32, ins.s_f64, x, y, arr=ins.arr)
    assert st == 0
    check_fma(r, x_np, ins.s_i32, ins.s_f64, y, ins.arr)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def rt_inputs(ni, nf, alen, n, seed=5):
    from dsr_workloads.gen import draws, uniform_int, uniform_f64
    s_i = uniform_int(draws(seed, 0, 0, ni), -(1 << 20), 1 << 20).astype(np.int32)
    s_f = uniform_f64(draws(seed, 1, 0, nf)) if nf else np.zeros(0)
    arr = uniform_int(draws(seed, 16, 0, alen), 0, (1 << 16) - 1).astype(np.int32) if alen else None
    return s_i, s_f, arr, W.uniform_f32_draws(seed, 2, 0, n)


@pytest.mark.parametrize("ni,nf,alen,n,wg,teams,joins", [
    (3, 2, 0, 100003, 256, 5, 0),        # odd count, no array, ragged tail
    (2, 1, 1, 4099, 256, 3, 0),          # one-element array
    (5, 4, 7, 65537, 256, 4, 1),         # odd array length, master joins
    (32, 16, 1000, 70001, 256, 3, 0),    # the batched workload's common shape
    (33, 31, 5, 50001, 256, 2, 0),       # 64 scalars: the run-time chain's limit
    (4, 4, 384, 77777, 256, 3, 0),       # array length = pair stride of 3 waves
    (4, 4, 385, 77777, 256, 3, 0),       # one past it
    (16, 16, 96, 123457, 512, 3, 1),     # 512-thread workgroups
    (32, 32, 0, 99999, 1024, 2, 0),      # 1024-thread workgroups, one pair per batch
    (6, 3, 130, 3, 256, 2, 0),           # fewer elements than lanes
])
def test_runtime_chain_shapes(ni, nf, alen, n, wg, teams, joins):
    """Run-time scalar counts with and without a shared array: array index
    carried across batches, odd lengths, every workgroup size class."""
    say("rt chain", ni, nf, alen, n, wg, teams, joins)
    s_i, s_f, arr, x_np = rt_inputs(ni, nf, alen, n)
    ctx = D.dsr_init(wg_size=wg, lds_slab_bytes=8192, hbm_slab_bytes=8192, max_teams=64,
                     master_joins=joins)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, teams, s_i, s_f, x, y, arr=arr)
    assert st == 0
    check_fma(r, x_np, s_i, s_f, y, arr)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_runtime_chain_frame_in_hbm():
    """The run-time chain with its frame (scalars and array) in the HBM slab."""
    say("rt chain hbm frame")
    s_i, s_f, arr, x_np = rt_inputs(20, 10, 333, 90001, seed=6)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=0, hbm_slab_bytes=4096, max_teams=64,
                     flags=D.DSR_F_TRACE)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(x.numel(), dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, 4, s_i, s_f, x, y, arr=arr)
    assert st == 0
    assert D.dsr_region_trace(r, 0)["placements"][0][0] == "hbm"
    check_fma(r, x_np, s_i, s_f, y, arr)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


@pytest.mark.parametrize("teams", [1, 33, 511, 512, 513, 1000, 4000])
def test_cross_team_combine_team_counts(teams):
    """Exact reduction across team counts on both sides of the one-round
    combine limit (512) and with ragged arrival groups."""
    say("combine teams", teams)
    s_i, s_f, arr, x_np = rt_inputs(3, 2, 0, teams * 97 + 13, seed=7)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=1024, hbm_slab_bytes=256, max_teams=4096)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(x.numel(), dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, teams, s_i, s_f, x, y)
    assert st == 0
    check_fma(r, x_np, s_i, s_f, y)
    y.zero_()
    torch.cuda.synchronize()
    D.dsr_launch(r, stream())           # the arrival counters reset themselves
    assert D.dsr_region_sync(r) == 0
    check_fma(r, x_np, s_i, s_f, y)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


@pytest.mark.parametrize("K,chunk,teams", [(8, 10001, 4), (1, 1025, 7), (64, 4099, 3), (16, 2048, 5)])
def test_fixed_chain_user_chunks(K, chunk, teams):
    """Caller-chosen team chunks: odd team starts, chunks that are and are
    not whole numbers of streaming blocks."""
    say("user chunk", K, chunk, teams)
    n = chunk * teams - 17
    cf, x_np = W.cfg2_inputs(K, n=n)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=4096, max_teams=64)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, teams, cf.s_i32, cf.s_f64, x, y, chunk=chunk)
    assert st == 0
    check_fma(r, x_np, cf.s_i32, cf.s_f64, y)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_fma_wide_workgroup_and_empty():
    say("fma wg 1024, n 0")
    cf, x_np = W.cfg2_inputs(8, n=100003)
    ctx = D.dsr_init(wg_size=1024, lds_slab_bytes=4096, max_teams=64)
    x = torch.from_numpy(x_np).cuda()
    y = torch.zeros(x.numel(), dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, 7, cf.s_i32, cf.s_f64, x, y)
    assert st == 0
    check_fma(r, x_np, cf.s_i32, cf.s_f64, y)
    D.dsr_region_free(r)
    e = torch.zeros(1, dtype=torch.float32, device="cuda")
    st, r = fma_region(ctx, 2, cf.s_i32, cf.s_f64, e[:0], y)
    assert st == 0 and D.dsr_region_reduction(r, 0)[1:] == (0.0, 0)
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_range_error_off_grid():
    say("range error")
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=4096, max_teams=4)
    x = torch.full((1000,), 2.0 ** -30, dtype=torch.float32, device="cuda")
    y = torch.zeros(1000, dtype=torch.float64, device="cuda")
    st, r = fma_region(ctx, 2, [], [2.0 ** -50], x, y)
    assert st == D.DSR_E_RANGE
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_nomem_when_frame_fits_neither_stack():
    say("nomem")
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=64, hbm_slab_bytes=64, max_teams=4,
                     flags=D.DSR_F_TRACE)
    out = t_i32(1024)
    st, r = run_region(ctx, 4, lambda r: (D.dsr_pop(r, D.dsr_push(r, 1024))))
    assert st == D.DSR_E_NOMEM
    traces, _ = S.run_region([S.Push(1024), S.Pop(0)], 4,
                             S.Config(lds_bytes=64, hbm_bytes=64, align=KERNEL_ALIGN))
    for t in range(4):
        assert D.dsr_region_trace(r, t)["error"] == D.DSR_E_NOMEM
        assert traces[t].error == "NOMEM"
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


# ---- Figure 6 pattern: shared arrays, flat and nested, LDS vs HBM-only -----
@pytest.mark.parametrize("nested", [0, 1])
@pytest.mark.parametrize("hbm_only", [0, 1])
@pytest.mark.parametrize("A,length", [(1, 16), (2, 256), (4, 4096), (1, 16384), (2, 16384),
                                      (3, 16384), (4, 16384), (3, 100)])
def test_cfg3_gather(A, length, hbm_only, nested):
    say("cfg3 A", A, "len", length, "hbm_only", hbm_only, "nested", nested)
    arrs = W.cfg3_arrays(A, length)
    n = (1 << 18) + 7
    teams = 16
    frame = 4 * A * length
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=0 if hbm_only else LDS_MAX4,
                     hbm_slab_bytes=(frame + 15) // 16 * 16, max_teams=teams, flags=D.DSR_F_TRACE)
    out = t_i32(n)
    body = D.DSR_BODY_GATHER_NESTED if nested else D.DSR_BODY_GATHER

    def build(r):
        f = D.dsr_push(r, frame, D.gather_frame(arrs))
        D.dsr_publish(r, f, body, n, out=out.data_ptr(), arrays=A, length=length)
        D.dsr_pop(r, f)
    st, r = run_region(ctx, teams, build)
    assert st == 0
    assert np.array_equal(out.cpu().numpy(), R.gather(arrs, 0, n))
    want = "hbm" if (hbm_only or frame > LDS_MAX4) else "lds"
    for t in (0, teams - 1):
        tr = D.dsr_region_trace(r, t)
        assert tr["placements"] == [(want, 0, (frame + 15) // 16 * 16)]
        if nested:
            assert tr["inner_pushes"][:3] == [1, 1, 1]
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


@pytest.mark.parametrize("A,length,hbm_only", [(2, 4096, 0), (2, 4096, 1), (3, 16384, 0)])
def test_cfg3_full_size(A, length, hbm_only):
    """The nested gather at its full size and launch shape (2^26 outputs,
    2048 teams of 256 threads, the stack sized as the bench sizes it): a
    32 KiB frame on chip or on the HBM-only stack, and a 192 KiB frame that
    only the HBM slot holds; every output element against the oracle."""
    say("cfg3 full A", A, "len", length, "hbm_only", hbm_only)
    arrs = W.cfg3_arrays(A, length)
    n, teams = 1 << 26, 2048
    frame = 4 * A * length
    slab = 0 if (hbm_only or frame > LDS_MAX4) else (frame + 15) // 16 * 16
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=slab, hbm_slab_bytes=(frame + 15) // 16 * 16,
                     max_teams=teams, master_joins=1)
    out = torch.full((n,), -1, dtype=torch.int32, device="cuda")

    def build(r):
        f = D.dsr_push(r, frame, D.gather_frame(arrs))
        D.dsr_publish(r, f, D.DSR_BODY_GATHER_NESTED, n, out=out.data_ptr(), arrays=A, length=length)
        D.dsr_pop(r, f)
    st, r = run_region(ctx, teams, build)
    assert st == 0
    assert np.array_equal(out.cpu().numpy(), R.gather(arrs, 0, n))
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)
    del out
    torch.cuda.empty_cache()


def test_two_frames_spill_and_lifo():
    """Two frames: the first fills the LDS stack, the second spills; a
    gather over each; pops in LIFO order.  Placement matches the simulator."""
    say("two frames")
    a1, a2 = W.cfg3_arrays(1, 4096), W.cfg3_arrays(2, 256)
    n = 50000
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=16384 + 64, hbm_slab_bytes=1 << 16, max_teams=8,
                     flags=D.DSR_F_TRACE)
    o1, o2 = t_i32(n), t_i32(n)

    def build(r):
        f1 = D.dsr_push(r, 16384, D.gather_frame(a1))
        f2 = D.dsr_push(r, 2048, D.gather_frame(a2))
        D.dsr_publish(r, f1, D.DSR_BODY_GATHER, n, out=o1.data_ptr(), arrays=1, length=4096)
        D.dsr_publish(r, f2, D.DSR_BODY_GATHER_NESTED, n, out=o2.data_ptr(), arrays=2, length=256)
        D.dsr_pop(r, f2)
        D.dsr_pop(r, f1)
    st, r = run_region(ctx, 3, build)
    assert st == 0
    assert np.array_equal(o1.cpu().numpy(), R.gather(a1, 0, n))
    assert np.array_equal(o2.cpu().numpy(), R.gather(a2, 0, n))
    traces, _ = S.run_region([S.Push(16384), S.Push(2048), S.Pop(1), S.Pop(0)], 3,
                             S.Config(lds_bytes=16384 + 64, hbm_bytes=1 << 16, align=KERNEL_ALIGN))
    for t in range(3):
        tr = D.dsr_region_trace(r, t)
        assert tr["placements"] == traces[t].placements == [("lds", 0, 16384), ("hbm", 0, 2048)]
        assert tr["barriers"][:4] == [5, 5, 5, 5]      # two regions + terminate
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)
