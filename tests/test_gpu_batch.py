"""GPU parity of the batched form: many regions with uneven loop lengths
and frame sizes in one persistent launch (plain and hipGraph-replayed) and
one launch per region, against the CPU oracle; each region's result must be
the same alone and in the batch (bit-exact: the reduction is exact)."""
import sys

import numpy as np
import pytest

import dsr_workloads as W
from oracle import ref as R

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1711_10413_amd import dsr as D  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def stream():
    return torch.cuda.current_stream().cuda_stream


def build_instances(n_inst, seed, lcap, chunk):
    Ls, Fs = W.cfg4_descriptors(n_inst, seed=seed)
    Ls = np.minimum(Ls, lcap)
    offs = np.zeros(n_inst + 1, np.int64)
    offs[1:] = np.cumsum((Ls + 63) // 64 * 64)
    x = np.zeros(int(offs[-1]), np.float32)
    insts = []
    for r in range(n_inst):
        ins = W.cfg4_instance(r, int(Ls[r]), int(Fs[r]), seed=seed)
        x[offs[r]:offs[r] + Ls[r]] = W.instance_x(r, int(Ls[r]), seed=seed)
        insts.append(ins)
    return insts, offs, x


def make_batch(ctx, insts, offs, x_d, y_d, chunk):
    regions = []
    for r, ins in enumerate(insts):
        teams = max(1, -(-ins.L // chunk))
        regions.append(D.fma_chain_region(ctx, teams, ins.s_i32, ins.s_f64, ins.arr, ins.L,
                                          x_d.data_ptr() + 4 * int(offs[r]),
                                          y_d.data_ptr() + 8 * int(offs[r])))
    return regions


def check_all(b, insts, offs, x_np, y_d, label):
    yg = y_d.cpu().numpy()
    for r, ins in enumerate(insts):
        lo, hi = int(offs[r]), int(offs[r]) + ins.L
        yr = R.fma_chain(x_np[lo:hi], ins.s_i32, ins.s_f64, ins.arr)
        assert np.array_equal(yg[lo:hi].view(np.uint64), yr.view(np.uint64)), (label, r)
        _, f64, fixed, st = D.dsr_batch_result(b, r)
        assert st == 0 and fixed == R.fixed75_sum(yr) and f64 == R.exact_sum(yr), (label, r)


@pytest.mark.parametrize("wg,lds,thr", [(256, 65536, 0), (128, 16384, 4096), (512, 0, 0),
                                        (64, 32768, 0)])
def test_batch_forms_match_oracle(wg, lds, thr):
    say("batch", wg, lds, thr)
    insts, offs, x_np = build_instances(300, seed=3, lcap=1 << 17, chunk=16384)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=65536, hbm_slab_bytes=65536, max_teams=2048)
    x_d = torch.from_numpy(x_np).cuda()
    y_d = torch.zeros(x_np.size, dtype=torch.float64, device="cuda")
    regions = make_batch(ctx, insts, offs, x_d, y_d, 16384)
    b = D.dsr_batch_create(ctx, regions)
    for r in regions:
        D.dsr_region_free(r)
    D.dsr_batch_tune(b, wg_size=wg, lds_slab_bytes=lds, overflow_threshold=thr)
    for form in ("persistent", "graph", "each"):
        y_d.zero_()
        if form == "graph":
            D.dsr_batch_tune(b, wg_size=wg, lds_slab_bytes=lds, overflow_threshold=thr, use_graph=1)
        if form == "each":
            D.dsr_batch_launch_each(b, stream())
        else:
            for rep in range(3 if form == "graph" else 1):     # replays reuse the graph
                if rep:
                    y_d.zero_()
                D.dsr_batch_launch(b, stream())
                assert D.dsr_batch_sync(b) == 0
                if form == "graph" and rep < 2:
                    check_all(b, insts, offs, x_np, y_d, form + str(rep))
        assert D.dsr_batch_sync(b) == 0
        check_all(b, insts, offs, x_np, y_d, form)
        if form != "each":
            t = D.dsr_batch_times(b, len(insts))
            assert np.all(t >= 0) and np.all(np.isfinite(t))
    D.dsr_batch_free(b)
    D.dsr_destroy(ctx)


def test_batch_result_equals_region_alone():
    """Isolation: every region's result is the same launched alone (its own
    single-region launch) and inside the batch."""
    say("isolation")
    insts, offs, x_np = build_instances(40, seed=4, lcap=1 << 16, chunk=8192)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=65536, hbm_slab_bytes=65536, max_teams=1024)
    x_d = torch.from_numpy(x_np).cuda()
    y_b = torch.zeros(x_np.size, dtype=torch.float64, device="cuda")
    y_a = torch.zeros(x_np.size, dtype=torch.float64, device="cuda")
    b = D.dsr_batch_create(ctx, make_batch(ctx, insts, offs, x_d, y_b, 8192))
    D.dsr_batch_launch(b, stream())
    assert D.dsr_batch_sync(b) == 0
    alone = make_batch(ctx, insts, offs, x_d, y_a, 8192)
    for r, reg in enumerate(alone):
        D.dsr_launch(reg, stream())
        assert D.dsr_region_sync(reg) == 0
        _, fa, xa = D.dsr_region_reduction(reg, 0)
        _, fb, xb, st = D.dsr_batch_result(b, r)
        assert (fa, xa) == (fb, xb)
        D.dsr_region_free(reg)
    assert torch.equal(y_a, y_b)
    D.dsr_batch_free(b)
    D.dsr_destroy(ctx)


def test_autotune_picks_a_valid_candidate():
    say("autotune")
    insts, offs, x_np = build_instances(120, seed=3, lcap=1 << 16, chunk=16384)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=65536, hbm_slab_bytes=65536, max_teams=2048)
    x_d = torch.from_numpy(x_np).cuda()
    y_d = torch.zeros(x_np.size, dtype=torch.float64, device="cuda")
    b = D.dsr_batch_create(ctx, make_batch(ctx, insts, offs, x_d, y_d, 16384))
    cands = [dict(wg_size=256, lds_slab_bytes=65536), dict(wg_size=512, lds_slab_bytes=32768),
             dict(wg_size=128, lds_slab_bytes=200000),          # does not fit: skipped
             dict(wg_size=64, lds_slab_bytes=16384, use_graph=1)]
    best, ms = D.dsr_autotune(b, cands, reps=2, stream=stream())
    assert ms[2] < 0 and all(m > 0 for i, m in enumerate(ms) if i != 2)
    k = int(np.argmin([m if m > 0 else 1e30 for m in ms]))
    assert best["wg_size"] == cands[k]["wg_size"]
    y_d.zero_()
    D.dsr_batch_launch(b, stream())
    assert D.dsr_batch_sync(b) == 0
    check_all(b, insts, offs, x_np, y_d, "tuned")
    D.dsr_batch_free(b)
    D.dsr_destroy(ctx)


def test_cfg4_full_batch_sampled():
    """The batched workload at its full size: 10,000 regions with loop
    lengths log-uniform on [256, 2^20] and frames on [8, 32768] bytes (about
    1.3e9 elements) in one persistent launch.  Every region must report
    success; the 8 longest regions, the 8 with the largest frames and 32
    drawn at random are checked against the oracle element by element and
    by their exact sums."""
    say("cfg4 full batch")
    n_inst, seed, chunk = 10000, 3, 65536
    Ls, Fs = W.cfg4_descriptors(n_inst, seed=seed)
    offs = np.zeros(n_inst + 1, np.int64)
    offs[1:] = np.cumsum((Ls + 63) // 64 * 64)
    x_d = torch.empty(int(offs[-1]), dtype=torch.float32, device="cuda")
    r = 0
    while r < n_inst:                       # host pieces of ~256 MB
        r1 = r
        while r1 < n_inst and offs[r1] - offs[r] < (1 << 26):
            r1 += 1
        host = np.empty(int(offs[r1] - offs[r]), np.float32)
        for q in range(r, r1):
            a = int(offs[q] - offs[r])
            host[a:a + int(Ls[q])] = W.instance_x(q, int(Ls[q]), seed=seed)
        x_d[int(offs[r]):int(offs[r1])].copy_(torch.from_numpy(host))
        r = r1
    y_d = torch.zeros(int(offs[-1]), dtype=torch.float64, device="cuda")
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=65536, hbm_slab_bytes=65536, max_teams=4096)
    insts = [W.cfg4_instance(q, int(Ls[q]), int(Fs[q]), seed=seed) for q in range(n_inst)]
    regions = [D.fma_chain_region(ctx, max(1, -(-int(Ls[q]) // chunk)), ins.s_i32, ins.s_f64, ins.arr,
                                  int(Ls[q]), x_d.data_ptr() + 4 * int(offs[q]),
                                  y_d.data_ptr() + 8 * int(offs[q])) for q, ins in enumerate(insts)]
    b = D.dsr_batch_create(ctx, regions)
    for reg in regions:
        D.dsr_region_free(reg)
    D.dsr_batch_launch(b, stream())
    assert D.dsr_batch_sync(b) == 0
    statuses = [D.dsr_batch_result(b, q)[3] for q in range(n_inst)]
    assert all(st == 0 for st in statuses)
    rng = np.random.default_rng(11)
    pick = sorted(set(np.argsort(Ls)[-8:].tolist()) | set(np.argsort(Fs)[-8:].tolist())
                  | set(rng.choice(n_inst, 32, replace=False).tolist()))
    x_np = None
    for q in pick:
        ins = insts[q]
        lo, hi = int(offs[q]), int(offs[q]) + ins.L
        x_np = x_d[lo:hi].cpu().numpy()
        yr = R.fma_chain(x_np, ins.s_i32, ins.s_f64, ins.arr)
        assert np.array_equal(y_d[lo:hi].cpu().numpy().view(np.uint64), yr.view(np.uint64)), q
        _, f64, fixed, st = D.dsr_batch_result(b, int(q))
        assert st == 0 and fixed == R.fixed75_sum(yr) and f64 == R.exact_sum(yr), q
    D.dsr_batch_free(b)
    D.dsr_destroy(ctx)
    del x_d, y_d
    torch.cuda.empty_cache()
