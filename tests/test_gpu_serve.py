"""GPU parity of the served form: a resident server kernel that admits
region requests as they arrive (continuous batching), against the CPU
oracle; each result must be the same alone and in the mix."""
import sys
import time

import numpy as np
import pytest

import dsr_workloads as W
from oracle import ref as R

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1711_10413_amd import dsr as D  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def instances(n, seed=4, lcap=1 << 16):
    Ls, Fs = W.cfg4_descriptors(n, seed=seed)
    Ls = np.minimum(Ls, lcap)
    out = []
    for r in range(n):
        ins = W.cfg4_instance(r, int(Ls[r]), int(Fs[r]), seed=seed)
        x = W.instance_x(r, int(Ls[r]), seed=seed)
        yr = R.fma_chain(x, ins.s_i32, ins.s_f64, ins.arr)
        out.append((ins, x, yr, R.exact_sum(yr), R.fixed75_sum(yr)))
    return out


def programs(ctx, insts, chunk, xs, ys):
    regs = []
    for k, (ins, x, yr, rs, fx) in enumerate(insts):
        teams = max(1, -(-ins.L // chunk))
        regs.append(D.fma_chain_region(ctx, teams, ins.s_i32, ins.s_f64, ins.arr, ins.L,
                                       xs[k].data_ptr(), ys[k].data_ptr()))
    return regs


def submit_retry(srv, region, outs=None, sink=None, timeout=60.0):
    """Submit, polling completions into `sink` while the server is busy."""
    t0 = time.time()
    while True:
        try:
            return D.dsr_serve_submit(srv, region, outs)
        except D.DsrError as e:
            if e.code != D.DSR_E_BUSY:
                raise
            if sink is not None:
                sink += D.dsr_serve_poll(srv)
            assert time.time() - t0 < timeout, "admission never freed up"


# A request of these sizes runs in tens of microseconds on the device; a
# completion that takes longer than this means the server stalled.
REQUEST_BOUND_S = 0.1


def drain(srv, want, timeout=5.0):
    got = []
    t0 = time.time()
    while len(got) < want:
        got += D.dsr_serve_poll(srv)
        assert time.time() - t0 < timeout, "server did not finish"
    return got


def wait_started(srv, timeout=2.0):
    """Every workgroup of the server's grid runs: the device holds the
    whole grid at once, as the occupancy query promised."""
    t0 = time.time()
    while True:
        st = D.dsr_serve_status(srv)
        if st["started"] == st["grid"]:
            return st
        assert time.time() - t0 < timeout, ("grid not resident", st)
        time.sleep(0.001)


def run_one(srv, region, outs=None):
    """Submit one request and wait for it; returns (done, seconds)."""
    t0 = time.perf_counter()
    try:
        D.dsr_serve_submit(srv, region, outs)
    except D.DsrError as e:
        # a refused submit names the server's state (and why it closed)
        raise AssertionError((str(e), D.dsr_serve_status(srv)))
    got = []
    while not got:
        got = D.dsr_serve_poll(srv)
        assert time.perf_counter() - t0 < 5.0, "request did not complete"
    return got[0], time.perf_counter() - t0


@pytest.fixture(scope="module")
def setup():
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=32768, hbm_slab_bytes=65536, max_teams=2048)
    insts = instances(48)
    xs = [torch.from_numpy(x).cuda() for _, x, _, _, _ in insts]
    ys = [torch.zeros(ins.L, dtype=torch.float64, device="cuda") for ins, *_ in insts]
    regs = programs(ctx, insts, 8192, xs, ys)
    # half the templates frozen: their requests initialise frames over 1 KiB
    # from the device copy; the others' come from the host slot, directly
    # or relayed through device memory by team 0 when their teams would
    # read 64 KiB or more from it
    for r in regs[::2]:
        D.dsr_region_freeze(r)
    torch.cuda.current_stream().synchronize()
    yield ctx, insts, xs, ys, regs
    for r in regs:
        D.dsr_region_free(r)
    D.dsr_destroy(ctx)


def test_serve_output_visible_at_completion(setup):
    """Each request's output must be fully visible to the host as soon as
    its completion is polled, while the server keeps running."""
    ctx, insts, xs, ys, regs = setup
    say("serve visibility")
    # every output buffer exists before the server starts: an allocation
    # that synchronises the device waits for the resident kernel
    outs = [torch.zeros_like(ys[k]) for k in range(12)]
    torch.cuda.current_stream().synchronize()
    srv = D.dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=32768, slots=16, slot_bytes=40960,
                            max_teams=64, idle_ms=20000)
    try:
        wait_started(srv)
        for k in range(12):
            ins, x, yr, rs, fx = insts[k]
            out = outs[k]
            d, secs = run_one(srv, regs[k], [out.data_ptr()])
            assert d["status"] == 0 and d["f64"] == [rs]
            assert secs < REQUEST_BOUND_S, (k, secs)
            assert np.array_equal(out.cpu().numpy().view(np.uint64), yr.view(np.uint64)), k
    finally:
        D.dsr_serve_stop(srv)


def test_serve_leaves_room_for_copies(setup):
    """The default grid leaves workgroup slots free, so the runtime's copy
    and fill kernels, issued on other streams while the server is resident,
    run at once instead of waiting for the server to close."""
    ctx, insts, xs, ys, regs = setup
    say("serve room for copies")
    side = torch.cuda.Stream()
    host = torch.zeros(ys[0].shape, dtype=torch.float64, pin_memory=True)
    dev = torch.zeros(1 << 20, device="cuda")
    torch.cuda.synchronize()
    srv = D.dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=32768, slots=16, slot_bytes=40960,
                            max_teams=64, idle_ms=20000)
    try:
        wait_started(srv)
        d, _ = run_one(srv, regs[0], [ys[0].data_ptr()])
        assert d["status"] == 0
        waits = []
        for name, work in (("device-to-host copy", lambda: host.copy_(ys[0], non_blocking=True)),
                           ("fill", lambda: dev.fill_(2.0))):
            with torch.cuda.stream(side):
                work()
            t0 = time.perf_counter()
            while not side.query() and time.perf_counter() - t0 < 2.0:
                time.sleep(0.001)
            waits.append((name, side.query(), time.perf_counter() - t0))
        st = D.dsr_serve_status(srv)
        assert all(done for _, done, _ in waits) and not st["closed"], (waits, st)
        assert np.array_equal(host.numpy(), ys[0].cpu().numpy())
    finally:
        D.dsr_serve_stop(srv)
    torch.cuda.synchronize()


def test_serve_light_load_and_idle_close(setup):
    """One request every 50 ms for 1 s with a 200 ms idle limit: the
    server keeps serving (idle means no new request for the whole server,
    not one workgroup's wait), every request completes within the bound,
    and 200 ms after the last one the server closes as a whole: every
    workgroup leaves and a later submit is refused."""
    ctx, insts, xs, ys, regs = setup
    say("serve light load")
    srv = D.dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=32768, slots=16, slot_bytes=40960,
                            max_teams=64, idle_ms=200)
    try:
        wait_started(srv)
        t_next = time.perf_counter()
        for q in range(20):
            while time.perf_counter() < t_next:
                pass
            t_next += 0.05
            k = q % len(regs)
            d, secs = run_one(srv, regs[k])
            assert d["status"] == 0 and d["f64"] == [insts[k][3]], q
            assert secs < REQUEST_BOUND_S, (q, secs)
            st = D.dsr_serve_status(srv)
            assert st["closed"] == 0 and st["exited"] == 0, (q, st)
        time.sleep(0.6)
        st = D.dsr_serve_status(srv)
        assert st["closed"] == 1 and st["exited"] == st["grid"], st
        assert st["final_items"] == st["published"], st
        with pytest.raises(D.DsrError) as e:
            D.dsr_serve_submit(srv, regs[0])
        assert e.value.code == D.DSR_E_STATE
    finally:
        D.dsr_serve_stop(srv)


def test_serve_stop_runs_published_requests(setup):
    """Requests published before a stop all run to completion (the close
    drains them), and the stop returns promptly."""
    ctx, insts, xs, ys, regs = setup
    say("serve stop drains")
    outs = [torch.zeros_like(y) for y in ys[:16]]
    torch.cuda.current_stream().synchronize()
    srv = D.dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=32768, slots=16, slot_bytes=40960,
                            max_teams=64, idle_ms=20000)
    try:
        for k in range(16):
            D.dsr_serve_submit(srv, regs[k], [outs[k].data_ptr()])
    finally:
        t0 = time.perf_counter()
        D.dsr_serve_stop(srv)
        assert time.perf_counter() - t0 < 2.0
    for k in range(16):
        assert np.array_equal(outs[k].cpu().numpy().view(np.uint64), insts[k][2].view(np.uint64)), k


def test_serve_requests_match_oracle(setup):
    ctx, insts, xs, ys, regs = setup
    say("serve basic")
    # every instance twice, the second copy into a separate output buffer:
    # both copies run concurrently in the mix.  The buffers exist before the
    # server starts (an allocation that synchronises the device waits for
    # the resident kernel)
    extra = [torch.zeros_like(y) for y in ys]
    torch.cuda.current_stream().synchronize()
    srv = D.dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=32768, slots=64, slot_bytes=40960,
                            max_teams=64, idle_ms=20000)
    try:
        tickets = {}
        done = []
        for k, r in enumerate(regs):
            tickets[submit_retry(srv, r, sink=done)] = (k, ys[k])
            tickets[submit_retry(srv, r, [extra[k].data_ptr()], sink=done)] = (k, extra[k])
        done += drain(srv, len(tickets) - len(done))
        assert D.dsr_serve_pending(srv) == 0
        # outputs are complete when the request is: check them while the
        # server is still resident (no kernel end has flushed anything)
        for d in done:
            k, y = tickets[d["ticket"]]
            ins, x, yr, rs, fx = insts[k]
            assert d["status"] == 0 and d["f64"] == [rs] and d["fixed"] == [fx], k
        for k, (ins, x, yr, rs, fx) in enumerate(insts):
            assert np.array_equal(ys[k].cpu().numpy().view(np.uint64), yr.view(np.uint64)), k
            assert torch.equal(ys[k], extra[k])
        # two of the unfrozen templates (6 teams, 12-16 KiB images) have
        # their images relayed by team 0, and no team gave up waiting
        st = D.dsr_serve_status(srv)
        assert st["relays"] >= 2 and st["relay_misses"] == 0, st
    finally:
        D.dsr_serve_stop(srv)


def test_serve_admission(setup):
    ctx, insts, xs, ys, regs = setup
    say("serve admission")
    # a frozen template with a large image, made before the server starts
    # (allocation and free synchronise with a resident kernel)
    kt = next(i for i, (ins, *_) in enumerate(insts)
              if len(D.fma_chain_frame(ins.s_i32, ins.s_f64, ins.arr)[0]) > 1024)
    ins = insts[kt][0]
    t = D.fma_chain_region(ctx, 2, ins.s_i32, ins.s_f64, ins.arr, ins.L, xs[kt].data_ptr(), ys[kt].data_ptr())
    D.dsr_region_freeze(t)
    torch.cuda.current_stream().synchronize()
    # a ring item holds the team in 16 bits; the slot count is bounded too
    for kw in (dict(max_teams=65536, ring_items=1 << 17, slots=1), dict(slots=65537),
               dict(ring_items=3000)):
        with pytest.raises(D.DsrError) as e:
            D.dsr_serve_start(ctx, **kw)
        assert e.value.code == D.DSR_E_INVAL, kw
    srv = D.dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=32768, slots=4, slot_bytes=40960,
                            max_teams=64, idle_ms=20000)
    try:
        # a frame larger than both the LDS stack and the HBM slot: rejected
        big = D.dsr_region_begin(ctx, 1)
        f = D.dsr_push(big, 200000)
        D.dsr_pop(big, f)
        with pytest.raises(D.DsrError) as e:
            D.dsr_serve_submit(srv, big)
        assert e.value.code == D.DSR_E_NOMEM
        D.dsr_region_free(big)
        # more requests than slots: the fifth is deferred until one completes
        n_ok = 0
        for k in range(4):
            D.dsr_serve_submit(srv, regs[k])
            n_ok += 1
        with pytest.raises(D.DsrError) as e:
            D.dsr_serve_submit(srv, regs[4])
        assert e.value.code == D.DSR_E_BUSY
        done = drain(srv, n_ok)
        assert all(d["status"] == 0 for d in done)
        D.dsr_serve_submit(srv, regs[4])
        done = drain(srv, 1)
        assert done[0]["f64"] == [insts[4][3]]
        # a frozen template whose device images a request reads cannot be
        # freed until the request has been collected (the refusal frees
        # nothing, so it does not synchronise with the resident server)
        D.dsr_serve_submit(srv, t)
        assert D.lib().dsr_region_free(t) == D.DSR_E_STATE
        done = drain(srv, 1)
        assert done[0]["status"] == 0 and done[0]["f64"] == [insts[kt][3]]
    finally:
        D.dsr_serve_stop(srv)
    D.dsr_region_free(t)


def test_serve_replay_and_serial(setup):
    ctx, insts, xs, ys, regs = setup
    say("serve replay")
    arrivals = W.poisson_schedule(5000.0, 0.1, seed=4)
    prog = (np.arange(len(arrivals)) * 7919) % len(regs)
    slots = 32
    pool = [torch.zeros(1 << 16, dtype=torch.float64, device="cuda") for _ in range(slots)]
    torch.cuda.current_stream().synchronize()
    srv = D.dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=32768, slots=slots,
                            slot_bytes=40960, max_teams=64, idle_ms=20000)
    try:
        lat, done = D.dsr_serve_replay(srv, regs, prog, arrivals, [p.data_ptr() for p in pool], 1,
                                       timeout_s=30.0)
    finally:
        D.dsr_serve_stop(srv)
    assert np.all(lat > 0)
    for q, d in enumerate(done):
        ins, x, yr, rs, fx = insts[prog[q]]
        assert d["status"] == 0 and d["f64"] == [rs] and d["fixed"] == [fx], q
    # the comparison form: one launch + sync per request, same schedule
    b = D.dsr_batch_create(ctx, regs)
    lat2 = D.dsr_batch_replay_serial(b, prog, arrivals)
    assert np.all(lat2 > 0)
    for k, (ins, x, yr, rs, fx) in enumerate(insts):
        if k in set(prog.tolist()):
            assert D.dsr_batch_result(b, k)[1] == rs
    D.dsr_batch_free(b)


def test_serve_lds_classes(setup):
    """Two LDS classes (4 KiB and 40 KiB of on-chip stack per team): every
    request runs in the class sized to its frames unless that class is full,
    and its outputs and exact sum equal the oracle's in the mix."""
    ctx, insts, xs, ys, regs = setup
    say("serve lds classes")
    slabs = [4096, 40960]
    outs = {k: torch.zeros_like(ys[k]) for k in range(24)}
    torch.cuda.current_stream().synchronize()
    srv = D.dsr_serve_start(ctx, wg_size=256, slots=16, slot_bytes=40960, max_teams=64, idle_ms=20000,
                            classes=[(slabs[0], 0), (slabs[1], 0)])
    want_cls, got = {}, []
    try:
        st = wait_started(srv)
        assert st["classes"] == 2
        tickets = {}
        for k in range(24):
            tickets[submit_retry(srv, regs[k], [outs[k].data_ptr()], sink=got)] = k
            want_cls[k] = D.dsr_serve_class_for(slabs, regs[k])
        got += drain(srv, 24 - len(got))
    finally:
        D.dsr_serve_stop(srv)
    seen = set()
    for d in got:
        k = tickets[d["ticket"]]
        ins, x, yr, rs, fx = insts[k]
        assert d["status"] == 0 and d["f64"] == [rs] and d["fixed"] == [fx], k
        assert np.array_equal(outs[k].cpu().numpy().view(np.uint64), yr.view(np.uint64)), k
        # a request runs in its own class, or a larger one while that is full
        assert slabs[d["lds_class"]] >= slabs[want_cls[k]], (k, d["lds_class"], want_cls[k])
        seen.add(d["lds_class"])
    assert sorted(tickets.values()) == list(range(24))
    assert set(want_cls.values()) == {0, 1}      # the instances need both classes


def test_serve_image_size_boundaries(setup):
    """Init blobs just under, at and just over the 1 KiB staged with the
    program, on 1, 8 and 64 teams, from frozen and unfrozen templates:
    LDS-staged images, images read from the host slot, images relayed by
    team 0 (64 teams of a 1040-byte blob read 65 KiB in all) and images
    read from the template's device copy all match the oracle."""
    ctx = setup[0]
    say("serve image boundaries")
    s_i32 = np.array([3, -2, 5, 1], dtype=np.int32)
    s_f64 = np.array([0.5, -1.25, 2.0, 0.75])
    cases, keep = [], []
    for alen in (232, 236, 240):                   # 1008, 1024, 1040-byte blobs
        arr = ((np.arange(alen) * 7919) % 65536).astype(np.int32)
        assert len(D.fma_chain_frame(s_i32, s_f64, arr)[0]) == 1008 + 16 * ((alen - 232) // 4)
        for teams in (1, 8, 64):
            L = teams * 16384
            x = W.instance_x(teams * 1000 + alen, L, seed=7)
            yr = R.fma_chain(x, s_i32, s_f64, arr)
            for frozen in (False, True):
                xd = torch.from_numpy(x).cuda()
                yd = torch.zeros(L, dtype=torch.float64, device="cuda")
                r = D.fma_chain_region(ctx, teams, s_i32, s_f64, arr, L, xd.data_ptr(), yd.data_ptr())
                if frozen:
                    D.dsr_region_freeze(r)
                keep.append((xd, yd))
                cases.append((r, yd, yr, R.exact_sum(yr), R.fixed75_sum(yr), (alen, teams, frozen)))
    torch.cuda.current_stream().synchronize()
    srv = D.dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=32768, slots=32, slot_bytes=40960,
                            max_teams=64, idle_ms=20000)
    try:
        tickets, done = {}, []
        for c in cases:
            tickets[submit_retry(srv, c[0], sink=done)] = c
        done += drain(srv, len(cases) - len(done))
        for d in done:
            r, yd, yr, rs, fx, what = tickets[d["ticket"]]
            assert d["status"] == 0 and d["f64"] == [rs] and d["fixed"] == [fx], what
            assert np.array_equal(yd.cpu().numpy().view(np.uint64), yr.view(np.uint64)), what
        st = D.dsr_serve_status(srv)
        assert st["relays"] == 1 and st["relay_misses"] == 0, st
    finally:
        D.dsr_serve_stop(srv)
    for c in cases:
        D.dsr_region_free(c[0])
