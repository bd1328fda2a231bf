"""Benchmark of the data-sharing runtime on one MI355X.

Headline workload (one step): the scalar-sharing sweep.  For each K in
{1, 2, 4, 8, 16, 32, 64} one region of 512 teams x 256 threads (one master
wave, three worker waves; by default the master joins the loop once it has
published): the master shares K scalars (ceil(K/2) int32, floor(K/2) fp64)
through its LDS team stack, the participating waves run
y[i] = fma chain over x[i] for 2**24 fp32 elements and reduce exactly into
the shared slot.  `value` is region instances per second over the timed
steps.  Inputs are seeded synthetic data resident in HBM before timing;
four (x, y) buffer sets rotate so the 256 MB Infinity Cache cannot hold the
working set.

The same JSON line also reports the other workloads of the method:
  plain      4 teams x 256, four shared int32 scalars, 1024 iterations:
             region latency (launch + sync) and back-to-back rate
  arrays     1-4 shared int32 arrays x {16, 256, 4096, 16384} elements,
             two nested parallel levels, 2**26 outputs, 2048 teams:
             LDS team stack vs HBM-only (global) stack
  batched    10,000 regions with log-uniform loop lengths and frames in one
             persistent launch (autotuned, hipGraph replay) vs one launch
             per region (the faster of the tuned configuration and plain
             256-thread teams): instances/s and p50/p99 completion
  served     Poisson arrivals at 1k, 10k, 50k requests/s: p50/p99 latency
             and instances/s, resident server vs one launch + sync per
             request
  ceiling    a plain streaming kernel with the sweep's read/write mix at the
             sweep's launch shape and at a full grid
  lists      the sweep's chain published through reference lists (section 5.2)
and the CPU oracle (one core and all cores, medians of five runs).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_ELEM = 12          # 4 B of x read + 8 B of y written
N = 1 << 24
TEAMS = 512
WG = 256
SETS = 4


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


# ---- scalar sweep (headline) -------------------------------------------------
def build_sweep(D, ctx, xs, ys, ks, W, schedule=0):
    regions = {}
    for K in ks:
        cf, _ = W.cfg2_inputs(K, n=N, with_x=False)
        img, size = D.fma_chain_frame(cf.s_i32, cf.s_f64)
        for s in range(SETS):
            r = D.dsr_region_begin(ctx, TEAMS)
            f = D.dsr_push(r, size, img)
            D.dsr_publish(r, f, D.DSR_BODY_FMA_CHAIN, N, inp=xs[s].data_ptr(), out=ys[s].data_ptr(),
                          ni=len(cf.s_i32), nf=len(cf.s_f64), schedule=schedule)
            D.dsr_pop(r, f)
            regions[(K, s)] = r
    return regions


def time_sweep(torch, D, regions, ks, steps, warmup, stream):
    """Warmup, then the timed region: for each K its `steps` launches back
    to back (buffer sets rotating), with one HIP event on the launch stream
    after each K's group; a launch's duration is its group's time / steps."""
    cur = torch.cuda.current_stream()
    for w in range(warmup):
        for K in ks:
            D.dsr_launch(regions[(K, w % SETS)], stream)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True)]
    t0 = time.perf_counter()
    evs[0].record(cur)
    for K in ks:
        for st in range(steps):
            D.dsr_launch(regions[(K, st % SETS)], stream)
        e = torch.cuda.Event(enable_timing=True)
        e.record(cur)
        evs.append(e)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    per_k = {K: evs[i].elapsed_time(evs[i + 1]) / steps for i, K in enumerate(ks)}
    return secs, per_k


LEAN_CHAINS = [(1, 0), (1, 1), (2, 2), (4, 4), (8, 8), (16, 16), (32, 32)]
STREAM_KS = (1, 2, 4, 8, 16)       # the HBM-bound chains timed as the dominant kernel
DOMINANT = "dsr_region_kernel<256, 10..14>"


def kernel_variant(K):
    """Compiled instance of the region kernel a K-scalar sweep region runs:
    the lean instance 10 + k of fixed chain k ((1,0) (1,1) (2,2) (4,4)
    (8,8) (16,16) (32,32) int32/fp64 scalars), which holds only that chain."""
    return 10 + LEAN_CHAINS.index(((K + 1) // 2, K // 2))


def run_sweep(torch, np, D, W, args, stream):
    dev = torch.device("cuda:0")
    ks = list(W.CFG2_KS)
    _, x_np = W.cfg2_inputs(1, n=N)
    x0 = torch.from_numpy(x_np).to(dev)
    xs = [x0] + [x0.clone() for _ in range(SETS - 1)]
    ys = [torch.empty(N, dtype=torch.float64, device=dev) for _ in range(SETS)]
    sched = 1 if args.schedule == "dynamic" else 0
    ctx = D.dsr_init(wg_size=WG, lds_slab_bytes=4096, hbm_slab_bytes=4096, max_teams=TEAMS,
                     master_joins=args.master_joins)
    regions = build_sweep(D, ctx, xs, ys, ks, W, sched)
    secs, by_k = time_sweep(torch, D, regions, ks, args.steps, args.warmup, stream)
    n_regions = args.steps * len(ks)
    loop_us, phases = {}, {}
    if not args.no_phases:
        # after the timed region: one traced launch per K for the loop phase
        # and the teams' phase stamps (tracing adds a few stores per team)
        ctx_t = D.dsr_init(wg_size=WG, lds_slab_bytes=4096, hbm_slab_bytes=4096, max_teams=TEAMS,
                           master_joins=args.master_joins, flags=D.DSR_F_TRACE)
        traced = build_sweep(D, ctx_t, xs, ys, ks, W, sched)
        for K in ks:
            for s in range(2):
                D.dsr_launch(traced[(K, s)], stream)
            r = traced[(K, 1)]
            D.dsr_region_sync(r)
            tr = [D.dsr_region_trace(r, t) for t in range(TEAMS)]
            loop_us[K] = (max(t["t_end"] for t in tr) - min(t["t_start"] for t in tr)) / 100.0
            base = min(t["t_team"] for t in tr)

            def late(key, mask=0xFFFFFFFF):
                return max(((t[key] & mask) - base) & 0xFFFFFFFF for t in tr) / 100.0
            phases[K] = {"last_release": late("t_start"), "last_join": late("t_end"),
                         "last_program_end": late("t_program_end"), "last_arrival": late("t_arrived")}
        for r in traced.values():
            D.dsr_region_free(r)
        D.dsr_destroy(ctx_t)
    verified = None
    if not args.no_verify:
        from oracle import ref as R
        verified = True
        last = (args.steps - 1) % SETS
        for K in ks:
            r = regions[(K, last)]
            if D.dsr_region_sync(r) != 0:
                verified = False
                continue
            cf, _ = W.cfg2_inputs(K, n=N, with_x=False)
            yr = R.fma_chain(x_np, cf.s_i32, cf.s_f64)
            verified &= bool(D.dsr_region_reduction(r, 0)[1] == R.exact_sum(yr))
            if K == ks[-1]:
                verified &= bool(np.array_equal(ys[last].cpu().numpy(), yr))
    hbm_only = None
    if not args.no_hbm_only:
        ctx2 = D.dsr_init(wg_size=WG, lds_slab_bytes=0, hbm_slab_bytes=4096, max_teams=TEAMS,
                          master_joins=args.master_joins)
        regions2 = build_sweep(D, ctx2, xs, ys, ks, W, sched)
        secs2, per2 = time_sweep(torch, D, regions2, ks, args.steps, args.warmup, stream)
        hbm_only = {"regions_per_s": n_regions / secs2, "per_k_kernel_ms": per2}
        for r in regions2.values():
            D.dsr_region_free(r)
        D.dsr_destroy(ctx2)
    occupancy = {}
    for v in sorted({kernel_variant(K) for K in ks}):
        o = D.dsr_region_occupancy(ctx, v)
        occupancy["dsr_region_kernel<256, %d>" % v] = {k: o[k] for k in ("teams_per_cu", "limiter", "regs_per_thread",
                                                                        "shared_per_team", "teams_by_registers",
                                                                        "teams_by_shared", "hip_teams_per_cu")}
    for r in regions.values():
        D.dsr_region_free(r)
    D.dsr_destroy(ctx)
    del xs, ys, x0
    torch.cuda.empty_cache()
    algo = BYTES_PER_ELEM * N
    return {
        "value": n_regions / secs, "secs": secs, "algo_bytes": algo,
        "per_k_kernel_ms": by_k,
        "per_k_gbs": {K: algo / (ms * 1e-3) / 1e9 for K, ms in by_k.items()},
        "loop_phase_us": loop_us,
        "loop_phase_gbs": {K: algo / (us * 1e-6) / 1e9 for K, us in loop_us.items() if us > 0},
        "team_phases_us": phases, "occupancy": occupancy,
        "lds_bytes_per_team": D.dsr_control_bytes(WG) + 4096, "hbm_only_stack": hbm_only, "verified": verified,
    }


# ---- HBM traffic from counters --------------------------------------------------
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dsr_region_kernel_sweep_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1711_10413_amd", "csrc", "dsr_kernels.hip"),
                  os.path.join(ROOT, "paper_1711_10413_amd", "csrc", "dsr_internal.h"),
                  os.path.join(ROOT, "include", "dsr_device.h")]
CALIB_N = 1 << 24            # calibration copy: fp32[2^24] -> fp64[2^24]
CALIB_REPS = 4


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name):
    """HBM bytes per launch of kernel `name` from the committed counter
    summary, or None when there is none or the kernel source changed since
    the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            line = line.strip().lstrip("-").strip()
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash() or kv.get("kernel") != name:
        return None
    return float(kv["traffic_bytes_per_launch"])


def run_calib(torch):
    """A plain conversion copy of known size (4 B read + 8 B written per
    element, the sweep's own mix): its counter readings scale FETCH_SIZE and
    WRITE_SIZE to bytes."""
    x = torch.zeros(CALIB_N, dtype=torch.float32, device="cuda")
    y = torch.empty(CALIB_N, dtype=torch.float64, device="cuda")
    for _ in range(CALIB_REPS):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"elements": CALIB_N, "reps": CALIB_REPS, "read_bytes": 4 * CALIB_N, "write_bytes": 8 * CALIB_N}


def traffic_from_counters(fetch_csv, write_csv, fetch_cmd, write_cmd):
    """Turn two rocprofv3 counter-collection CSVs (FETCH_SIZE, WRITE_SIZE, KiB
    per dispatch) into the committed traffic summary: the region kernel's
    mean per-launch readings, scaled by what the same counters read for the
    calibration copy of known size."""
    import csv
    import statistics

    def per_kernel(path, counter):
        vals = {}
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
        return vals

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    cal = [k for k in fetch if "copy" in k.lower() and "rocclr" not in k.lower()
           and len(fetch[k]) == CALIB_REPS]
    if len(cal) != 1:
        raise SystemExit("calibration copy kernel not found uniquely: %s" % cal)
    cal = cal[0]
    f_scale = 4 * CALIB_N / (1024 * statistics.mean(fetch[cal]))
    w_scale = 8 * CALIB_N / (1024 * statistics.mean(write[cal]))
    name = DOMINANT
    keys = [k for k in fetch if any(k.startswith("void dsr_region_kernel<256, %d>" % kernel_variant(K))
                                    for K in STREAM_KS)]
    if len(keys) != len(STREAM_KS):
        raise SystemExit("region kernel instances not found: %s" % keys)
    fk = statistics.mean(v for k in keys for v in fetch[k]) * 1024 * f_scale
    wk = statistics.mean(v for k in keys for v in write[k]) * 1024 * w_scale
    lines = [
        "# HBM traffic of %s on the scalar sweep (K <= 16 regions)" % name, "",
        "Per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) from two rocprofv3 counter runs,",
        "each scaled by the same counter's reading for a plain fp32 -> fp64 copy of",
        "2^24 elements (64 MiB read, 128 MiB written) in the same process.", "",
        "fetch run: `%s`" % fetch_cmd, "", "write run: `%s`" % write_cmd, "",
        "| kernel | dispatches | FETCH_SIZE KiB (mean) | WRITE_SIZE KiB (mean) |",
        "|---|---|---|---|"]
    for k in sorted(fetch):
        if k in write:
            lines.append("| %s | %d | %.1f | %.1f |" % (k[:80], len(fetch[k]), statistics.mean(fetch[k]),
                                                      statistics.mean(write[k])))
    lines += ["",
              "- calibration_read_scale: %.4f" % f_scale,
              "- calibration_write_scale: %.4f" % w_scale,
              "- algorithmic_bytes_per_launch: %d" % (BYTES_PER_ELEM * N),
              "- kernel: %s" % name,
              "- fetch_bytes_per_launch: %.0f" % fk,
              "- write_bytes_per_launch: %.0f" % wk,
              "- traffic_bytes_per_launch: %.0f" % (fk + wk),
              "- kernel_source_sha256: %s" % kernel_source_hash(), ""]
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


# ---- publish by reference list (section 5.2) ---------------------------------------
def run_lists(torch, np, D, W, stream, reps=20):
    """The sweep's fma chain published five ways, per launch: one frame
    (this runtime's form), a list of references on chip (up to 20), the
    same list in global memory (DSR_F_GLOBAL_LISTS), and both lists read
    again on every batch of the loop (deref=1: each chain step reads the
    reference, then the scalar, as outlined code must when the loop's stores
    may alias the shared variables); at the sweep's size and at a small size
    where per-region costs dominate."""
    from oracle import ref as R
    dev = torch.device("cuda:0")
    out = {}
    for n, teams in ((N, TEAMS), (1 << 16, 64)):
        _, x_np = W.cfg2_inputs(1, n=n)
        x = torch.from_numpy(x_np).to(dev)
        y = torch.empty(n, dtype=torch.float64, device=dev)
        rows = {}
        for K in (8, 16, 38):
            cf, _ = W.cfg2_inputs(K, n=n, with_x=False)
            ni, nf = len(cf.s_i32), len(cf.s_f64)
            img, size = D.fma_chain_frame(cf.s_i32, cf.s_f64)
            refs = [(0, 0)] + [(0, 24 + 8 * nf + 4 * k) for k in range(ni)] + [(0, 24 + 8 * k) for k in range(nf)]
            want = R.exact_sum(R.fma_chain(x_np, cf.s_i32, cf.s_f64))
            row = {"references": len(refs)}
            for mode, flags in (("frame", 0), ("list", 0), ("global_list", D.DSR_F_GLOBAL_LISTS),
                                ("list_deref", 0), ("global_list_deref", D.DSR_F_GLOBAL_LISTS)):
                ctx = D.dsr_init(wg_size=WG, lds_slab_bytes=4096, hbm_slab_bytes=4096, max_teams=teams,
                                 flags=flags | D.DSR_F_TRACE)
                r = D.dsr_region_begin(ctx, teams)
                f = D.dsr_push(r, size, img)
                if mode == "frame":
                    D.dsr_publish(r, f, D.DSR_BODY_FMA_CHAIN, n, inp=x.data_ptr(), out=y.data_ptr(), ni=ni, nf=nf)
                else:
                    D.dsr_publish_list(r, refs, D.DSR_BODY_FMA_CHAIN_REFS, n, inp=x.data_ptr(),
                                       out=y.data_ptr(), ni=ni, nf=nf, deref=int(mode.endswith("deref")))
                D.dsr_pop(r, f)
                for _ in range(3):
                    D.dsr_launch(r, stream)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                cur = torch.cuda.current_stream()
                e0.record(cur)
                for _ in range(reps):
                    D.dsr_launch(r, stream)
                e1.record(cur)
                torch.cuda.synchronize()
                ok = D.dsr_region_sync(r) == 0 and D.dsr_region_reduction(r, 0)[1] == want
                lst = D.dsr_region_trace(r, 0).get("list")
                row[mode] = {"us_per_launch": e0.elapsed_time(e1) * 1e3 / reps, "verified": bool(ok),
                             "list_in": lst[0] if lst else None}
                D.dsr_region_free(r)
                D.dsr_destroy(ctx)
            rows["K%d" % K] = row
            say("lists", n, K, {m: round(row[m]["us_per_launch"], 2)
                                for m in ("frame", "list", "global_list", "list_deref", "global_list_deref")})
        out["n%d_teams%d" % (n, teams)] = rows
        del x, y
    torch.cuda.empty_cache()
    return out


# ---- streaming ceiling ------------------------------------------------------------
def run_ceiling(torch, D, stream, reps=40):
    """The loop's streaming ceiling (dsr_stream_ceiling: y = double(x) over
    2^24 elements, 12 B per element, no runtime around it) at the sweep's
    own shape (512 x 256) and at a grid that fills every CU (4096 x 256),
    with four buffer sets rotating as in the sweep."""
    xs = [torch.zeros(N, dtype=torch.float32, device="cuda") for _ in range(SETS)]
    ys = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in range(SETS)]
    out = {}
    for grid, wg in ((TEAMS, WG), (4096, WG)):
        for i in range(4):
            D.dsr_stream_ceiling(xs[i % SETS].data_ptr(), ys[i % SETS].data_ptr(), N, grid, wg, stream)
        torch.cuda.synchronize()
        cur = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        for i in range(reps):
            D.dsr_stream_ceiling(xs[i % SETS].data_ptr(), ys[i % SETS].data_ptr(), N, grid, wg, stream)
        e1.record(cur)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        out["grid_%dx%d" % (grid, wg)] = {"us_per_launch": us, "gbs": BYTES_PER_ELEM * N / (us * 1e-6) / 1e9}
    ok = bool(torch.equal(ys[(reps - 1) % SETS], xs[(reps - 1) % SETS].double()))
    out["verified"] = ok
    del xs, ys
    torch.cuda.empty_cache()
    return out


# ---- plain region -------------------------------------------------------------
def run_plain(torch, np, D, W, stream):
    from oracle import ref as R
    c = W.cfg1_inputs()
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=4096, hbm_slab_bytes=4096, max_teams=4)
    out = torch.zeros(1024, dtype=torch.int32, device="cuda")
    r = D.dsr_region_begin(ctx, 4)
    f = D.dsr_push(r, 24, D.affine_xor_frame(c.a, c.b, c.c, c.d))
    D.dsr_publish(r, f, D.DSR_BODY_AFFINE_XOR, 1024, out=out.data_ptr())
    D.dsr_pop(r, f)
    for _ in range(20):
        D.dsr_launch(r, stream)
        D.dsr_region_sync(r)
    lat = []
    for _ in range(200):
        t = time.perf_counter()
        D.dsr_launch(r, stream)
        D.dsr_region_sync(r)
        lat.append((time.perf_counter() - t) * 1e6)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(1000):
        D.dsr_launch(r, stream)
    torch.cuda.synchronize()
    rate = 1000 / (time.perf_counter() - t)
    ro, rs = R.affine_xor(c.a, c.b, c.c, c.d, 0, 1024)
    ok = D.dsr_region_sync(r) == 0 and D.dsr_region_reduction(r, 0)[0] == rs and \
        bool(np.array_equal(out.cpu().numpy(), ro))
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)
    return {"latency_us_p50": pct(lat, 50), "latency_us_p99": pct(lat, 99),
            "back_to_back_regions_per_s": rate, "verified": ok}


# ---- arrays + nesting -------------------------------------------------------
def run_arrays(torch, np, D, W, stream, reps=6, shapes=None):
    from oracle import ref as R
    n, teams = 1 << 26, 2048
    lds_max = 163840 - D.dsr_control_bytes(WG)
    outs = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(2)]
    res = {}
    for A, length in (shapes or [(a, l) for a in W.CFG3_AS for l in W.CFG3_LENS]):
        if True:
            arrs = W.cfg3_arrays(A, length)
            frame = 4 * A * length
            row = {"frame_bytes": frame}
            for mode in ("lds", "hbm_only"):
                slab = 0 if (mode == "hbm_only" or frame > lds_max) else (frame + 15) // 16 * 16
                ctx = D.dsr_init(wg_size=256, lds_slab_bytes=slab,
                                 hbm_slab_bytes=(frame + 15) // 16 * 16, max_teams=teams,
                                 master_joins=1)
                regs = []
                for o in outs:
                    r = D.dsr_region_begin(ctx, teams)
                    f = D.dsr_push(r, frame, D.gather_frame(arrs))
                    D.dsr_publish(r, f, D.DSR_BODY_GATHER_NESTED, n, out=o.data_ptr(), arrays=A,
                                  length=length)
                    D.dsr_pop(r, f)
                    regs.append(r)
                for k in range(2):
                    D.dsr_launch(regs[k % 2], stream)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for k in range(reps):
                    D.dsr_launch(regs[k % 2], stream)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                occ = D.dsr_region_occupancy(ctx, 0)
                row[mode] = {"ms": ms, "gbs": 4.0 * n / (ms * 1e-3) / 1e9,
                             "frame_in": "lds" if slab else "hbm", "lds_bytes_per_team": D.dsr_control_bytes(WG) + slab,
                             # array reads: 4 B per array per element, from LDS or from L2/HBM
                             "array_read_gbs": 4.0 * A * n / (ms * 1e-3) / 1e9,
                             "teams_per_cu": occ["teams_per_cu"], "occupancy_limiter": occ["limiter"]}
                if mode == "lds":
                    ok = D.dsr_region_sync(regs[(reps - 1) % 2]) == 0
                    idx = np.random.default_rng(A * 7 + length).integers(0, n, 256)
                    got = outs[(reps - 1) % 2].cpu().numpy()[idx]
                    want = np.array([int(R.gather(arrs, int(i), int(i) + 1)[0]) for i in idx])
                    row["verified_sample"] = bool(ok and np.array_equal(got, want))
                for r in regs:
                    D.dsr_region_free(r)
                D.dsr_destroy(ctx)
            row["lds_speedup"] = row["hbm_only"]["ms"] / row["lds"]["ms"]
            res["A%d_len%d" % (A, length)] = row
            say("arrays", A, length, round(row["lds"]["gbs"]), round(row["hbm_only"]["gbs"]))
    del outs
    torch.cuda.empty_cache()
    return res


# ---- batched -------------------------------------------------------------------
def instance_pool(W, n, seed, lcap=None):
    import numpy as np
    Ls, Fs = W.cfg4_descriptors(n, seed=seed)
    if lcap:
        Ls = np.minimum(Ls, lcap)
    offs = np.zeros(n + 1, np.int64)
    offs[1:] = np.cumsum((Ls + 63) // 64 * 64)
    return Ls, Fs, offs


def fill_x(torch, W, Ls, offs, seed, dev):
    """Generate every instance's x on the host in pieces of ~256 MB and
    upload them into one device buffer."""
    x = torch.empty(int(offs[-1]), dtype=torch.float32, device=dev)
    n, r = len(Ls), 0
    while r < n:
        r1, tot = r, 0
        while r1 < n and tot < (1 << 26):
            tot += int(offs[r1 + 1] - offs[r1])
            r1 += 1
        host = torch.empty(int(offs[r1] - offs[r]), dtype=torch.float32).pin_memory()
        hn = host.numpy()
        for q in range(r, r1):
            a = int(offs[q] - offs[r])
            hn[a:a + int(Ls[q])] = W.instance_x(q, int(Ls[q]), seed=seed)
        x[int(offs[r]):int(offs[r1])].copy_(host)
        r = r1
    return x


def build_programs(D, W, ctx, Ls, Fs, offs, seed, x_ptr, y_ptr, chunk):
    regs, insts = [], []
    for q in range(len(Ls)):
        ins = W.cfg4_instance(q, int(Ls[q]), int(Fs[q]), seed=seed)
        teams = max(1, -(-int(Ls[q]) // chunk))
        regs.append(D.fma_chain_region(ctx, teams, ins.s_i32, ins.s_f64, ins.arr, int(Ls[q]),
                                       x_ptr + 4 * int(offs[q]), y_ptr + 8 * int(offs[q])))
        insts.append(ins)
    return regs, insts


def run_batched(torch, np, D, W, stream, n_inst=10000, seed=3, sample=64, each=True):
    from oracle import ref as R
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    Ls, Fs, offs = instance_pool(W, n_inst, seed)
    x = fill_x(torch, W, Ls, offs, seed, dev)
    y = torch.empty(int(offs[-1]), dtype=torch.float64, device=dev)
    say("batched inputs", round(time.perf_counter() - t0, 1), "s")
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=65536, hbm_slab_bytes=65536, max_teams=4096)
    chunk = 65536
    regs, insts = build_programs(D, W, ctx, Ls, Fs, offs, seed, x.data_ptr(), y.data_ptr(), chunk)
    b = D.dsr_batch_create(ctx, regs)
    for r in regs:
        D.dsr_region_free(r)
    torch.cuda.synchronize()
    total_elems = int(Ls.sum())
    algo = 12.0 * total_elems
    # candidates from the footprint/occupancy model: LDS slabs sized to the
    # batch's stacks, pruned per predicted residency
    cands = D.dsr_autotune_plan(b)
    best, ms = D.dsr_autotune(b, cands, reps=2, stream=stream)
    say("autotune best", best)

    def measure(launch, reps):
        secs, lats = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            launch(b, stream)
            st = D.dsr_batch_sync(b)
            secs.append(time.perf_counter() - t)
            lats.append(D.dsr_batch_times(b, n_inst))
            assert st == 0, st
        mid = int(np.argsort(secs)[len(secs) // 2])
        s = secs[mid]
        lat = lats[mid]
        return {"ms": s * 1e3, "instances_per_s": n_inst / s, "gbs": algo / s / 1e9,
                "p50_completion_us": pct(lat, 50), "p99_completion_us": pct(lat, 99),
                "device_ms": D.dsr_batch_elapsed(b)}

    pers = measure(D.dsr_batch_launch, 5)
    rng = np.random.default_rng(1)
    pick = rng.choice(n_inst, sample, replace=False)
    ok = True
    for q in pick:
        ins = insts[q]
        lo, hi = int(offs[q]), int(offs[q]) + ins.L
        yr = R.fma_chain(x[lo:hi].cpu().numpy(), ins.s_i32, ins.s_f64, ins.arr)
        _, f64, fixed, stq = D.dsr_batch_result(b, int(q))
        ok &= (stq == 0 and f64 == R.exact_sum(yr) and fixed == R.fixed75_sum(yr))
        ok &= bool(np.array_equal(y[lo:hi].cpu().numpy(), yr))
    # one launch per region, under the tuned configuration and under plain
    # 256-thread teams; the comparison takes the faster of the two (skipped
    # when profiling the persistent launch: 40,000 launches)
    each_res = None
    if each:
        each_tuned = measure(D.dsr_batch_launch_each, 2)
        each_tuned["tune"] = "tuned"
        D.dsr_batch_tune(b, wg_size=256, lds_slab_bytes=65536, master_joins=1, use_graph=0)
        each_256 = measure(D.dsr_batch_launch_each, 2)
        each_256["tune"] = "256 threads, 64 KiB LDS stack, master joins"
        each_res = min((each_tuned, each_256), key=lambda e: e["ms"])
    D.dsr_batch_tune(b, **{k: best[k] for k in ("wg_size", "lds_slab_bytes", "overflow_threshold",
                                                 "master_joins", "grid")}, use_graph=0)
    plain = measure(D.dsr_batch_launch, 3)
    D.dsr_batch_free(b)
    D.dsr_destroy(ctx)
    del x, y
    torch.cuda.empty_cache()
    return {"instances": n_inst, "elements": total_elems, "algorithmic_bytes": algo,
            "tuned": best, "autotune_candidates": len(cands),
            "autotune_ms": {"%d/%d/%d" % (c["wg_size"], c["lds_slab_bytes"], c["master_joins"]): m
                            for c, m in zip(cands, ms)},
            "persistent_graph": pers, "persistent_no_graph": plain,
            "one_launch_per_region": each_res,
            "one_launch_per_region_ms": {"tuned": each_tuned["ms"], "256": each_256["ms"]} if each else None,
            "speedup_vs_one_launch": each_res["ms"] / pers["ms"] if each else None,
            "verified_sample": {"instances": sample, "ok": bool(ok)}}


# ---- served ----------------------------------------------------------------------
def run_served(torch, np, D, W, stream, rates, seconds, pool=1000, seed=4, slots=256, check=192,
               serial_seconds=10.0):
    """Poisson arrivals at each rate for `seconds`.  Request q runs instance
    prog[q] drawn uniformly (seeded) from a pool of `pool` instances of the
    seed-4 table (sizes log-uniform as in the batched workload), writing its
    y into a recycled slot buffer.  Every request's exact sum is checked
    against the oracle's.  Then `check` requests drawn from the pool are
    submitted back to back, each with its own output buffer, so that they
    overlap on the device, and every element of their y is checked.  The
    comparison form (one launch and synchronisation per request) replays
    the first `serial_seconds` of each schedule: where it cannot keep up
    its backlog only grows, and a longer replay would only take longer."""
    from oracle import ref as R
    dev = torch.device("cuda:0")
    Ls, Fs, offs = instance_pool(W, pool, seed)
    x = fill_x(torch, W, Ls, offs, seed, dev)
    y = torch.empty(int(offs[-1]), dtype=torch.float64, device=dev)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=32768, hbm_slab_bytes=65536, max_teams=4096)
    # a request's teams: one per 16384 elements (up to 64), for latency
    chunk = 16384
    regs, insts = build_programs(D, W, ctx, Ls, Fs, offs, seed, x.data_ptr(), y.data_ptr(), chunk)
    # the templates' frame images resident in HBM, as the batch's are
    for r in regs:
        D.dsr_region_freeze(r)
    slot_y = [torch.empty(1 << 20, dtype=torch.float64, device=dev) for _ in range(slots)]
    torch.cuda.synchronize()
    def oracle_y(q):
        ins = insts[q]
        lo = int(offs[q])
        return R.fma_chain(x[lo:lo + ins.L].cpu().numpy(), ins.s_i32, ins.s_f64, ins.arr)

    want = [R.exact_sum(oracle_y(q)) for q in range(pool)]
    b = D.dsr_batch_create(ctx, regs)
    res = {"pool_instances": pool, "seconds_per_rate": seconds, "slots": slots,
           "templates": "frozen before the server starts (frame images over 1 KiB read from HBM)",
           "request_to_instance": "request q runs instance prog[q], drawn uniformly from the pool "
                                  "(seeded per rate)"}
    rng = np.random.default_rng(seed)
    for rate in rates:
        arr = W.poisson_schedule(rate, seconds, seed=seed)
        prog = rng.integers(0, pool, len(arr)).astype(np.int32)
        srv = D.dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=32768, slots=slots, slot_bytes=40960,
                                max_teams=64, idle_ms=30000)
        try:
            lat, done = D.dsr_serve_replay(srv, regs, prog, arr, [t.data_ptr() for t in slot_y], 1,
                                           timeout_s=60.0)
        finally:
            D.dsr_serve_stop(srv)
        bad = sum(1 for q, d in enumerate(done) if d["status"] != 0 or d["f64"] != [want[int(prog[q])]])
        span = max(float(arr[-1]), 1e-9) if len(arr) else 1e-9
        fin = float((arr + lat * 1e-6).max()) if len(arr) else 0.0
        served = {"requests": int(len(arr)), "p50_us": pct(lat, 50), "p99_us": pct(lat, 99),
                  "instances_per_s": len(arr) / max(fin, span), "sums_checked": int(len(arr)),
                  "sums_wrong": int(bad)}
        say("served", rate, served)
        cut = arr < serial_seconds
        arr2, prog2 = arr[cut], prog[cut]
        span2 = max(float(arr2[-1]), 1e-9) if len(arr2) else 1e-9
        lat2 = D.dsr_batch_replay_serial(b, prog2, arr2)
        fin2 = float((arr2 + lat2 * 1e-6).max()) if len(arr2) else 0.0
        serial = {"seconds": float(min(seconds, serial_seconds)), "requests": int(len(arr2)),
                  "p50_us": pct(lat2, 50), "p99_us": pct(lat2, 99),
                  "instances_per_s": len(arr2) / max(fin2, span2)}
        res["%dk_per_s" % (rate // 1000)] = {"served": served, "serial_launch_sync": serial}
        say("served", rate, served, serial)
    # outputs in the mix: requests submitted back to back, each with its own y
    picks = rng.integers(0, pool, check)
    outs = [torch.full((insts[int(q)].L,), -1.0, dtype=torch.float64, device=dev) for q in picks]
    srv = D.dsr_serve_start(ctx, wg_size=256, lds_slab_bytes=32768, slots=slots, slot_bytes=40960,
                            max_teams=64, idle_ms=30000)
    got, tickets = [], {}
    try:
        for k, q in enumerate(picks):
            while True:
                try:
                    tickets[D.dsr_serve_submit(srv, regs[int(q)], [outs[k].data_ptr()])] = k
                    break
                except D.DsrError as e:
                    if e.code != D.DSR_E_BUSY:
                        raise
                    got += D.dsr_serve_poll(srv)
        t0 = time.time()
        while len(got) < check and time.time() - t0 < 30:
            got += D.dsr_serve_poll(srv)
    finally:
        D.dsr_serve_stop(srv)
    ok = len(got) == check
    for d in got:
        k = tickets[d["ticket"]]
        q = int(picks[k])
        ok &= d["status"] == 0 and d["f64"] == [want[q]]
        ok &= bool(np.array_equal(outs[k].cpu().numpy().view(np.uint64), oracle_y(q).view(np.uint64)))
    res["outputs_in_mix"] = {"requests": int(check), "y_elements_checked": int(sum(insts[int(q)].L for q in picks)),
                             "ok": bool(ok)}
    D.dsr_batch_free(b)
    for r in regs:
        D.dsr_region_free(r)
    D.dsr_destroy(ctx)
    del x, y, slot_y, outs
    torch.cuda.empty_cache()
    return res


# ---- CPU baseline ---------------------------------------------------------------
def cpu_baseline(W, runs=5, one_core_elems=1 << 22):
    """The oracle on the host's cores.  One run computes, for each K of the
    sweep, y with the oracle's fma chain and its exact 2^-75 fixed-point
    total (oracle/ref.c), over slices of the range in a pool of threads
    (the C calls release the interpreter lock); the slices' exact integer
    totals are added and rounded once (Python's int / int is correctly
    rounded).  All-core: whole 2^24-element regions on every thread the
    host gives this process; one core: the first 2^22 elements of each
    region on one thread, scaled to whole regions.  Medians of `runs`."""
    import statistics
    from concurrent.futures import ThreadPoolExecutor
    from oracle import ref as R
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = max(1, min(ncpu, int(os.environ.get("OMP_NUM_THREADS") or ncpu), 16))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    _, x = W.cfg2_inputs(1, n=N)
    scal = {K: W.cfg2_inputs(K, n=N, with_x=False)[0] for K in W.CFG2_KS}

    def piece(K, lo, hi):
        y = R.fma_chain(x[lo:hi], scal[K].s_i32, scal[K].s_f64)
        return R.fixed75_sum(y)

    def sweep(n, nthreads, pool):
        step = -(-n // nthreads)
        out = {}
        for K in W.CFG2_KS:
            parts = [pool.submit(piece, K, lo, min(n, lo + step)) for lo in range(0, n, step)]
            out[K] = sum(p.result() for p in parts) / (1 << 75)
        return out

    def timed(n, nthreads):
        secs = []
        with ThreadPoolExecutor(nthreads) as pool:
            for _ in range(runs):
                t0 = time.perf_counter()
                sweep(n, nthreads, pool)
                secs.append(time.perf_counter() - t0)
        return statistics.median(secs)

    t1 = timed(one_core_elems, 1)
    tn = timed(N, threads)
    one = len(W.CFG2_KS) * (one_core_elems / N) / t1
    allc = len(W.CFG2_KS) / tn
    return {"value": allc, "unit": "region instances/s", "cores": threads, "kind": "oracle",
            "sample": "the K sweep (7 regions of 2^24 elements: fma chain + exact fixed-point sum, "
                      "oracle/ref.c): all-core median of %d runs over whole regions on %d threads "
                      "(%.2f s per run); one-core median of %d runs over the first 2^22 elements of "
                      "each region, scaled (%.2f s per run)" % (runs, threads, tn, runs, t1),
            "cpu_model": model, "nproc": ncpu, "one_core_value": one, "all_core_value": allc,
            "runs": runs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--parts", default="sweep,ceiling,plain,arrays,lists,batched,served,cpu",
                    help="comma list of: sweep ceiling plain arrays lists batched served cpu calib")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-batched-each", action="store_true",
                    help="skip the one-launch-per-region leg of the batched part (for profiling)")
    ap.add_argument("--no-hbm-only", action="store_true")
    ap.add_argument("--no-phases", action="store_true",
                    help="skip the traced launches that measure the loop phase")
    ap.add_argument("--master-joins", type=int, default=1,
                    help="1: the master wave runs loop iterations too (four streaming waves per team)")
    ap.add_argument("--schedule", choices=["static", "dynamic"], default="static")
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="length of each served arrival schedule (the full workload is 60)")
    ap.add_argument("--serve-rates", default="1000,10000,50000")
    ap.add_argument("--serve-serial-seconds", type=float, default=10.0,
                    help="schedule seconds the launch-per-request comparison replays")
    ap.add_argument("--arrays-shapes", default="",
                    help="comma list of AxLEN array shapes for the arrays part (default: all 16)")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "FETCH_CMD", "WRITE_CMD"),
                    help="write the HBM traffic summary from two counter runs and exit")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from_counters(*args.traffic_from)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a region would "
              "split by team blocks with one exact partial exchanged per GPU)", file=sys.stderr)
        sys.exit(2)
    parts = set(args.parts.split(","))

    import numpy as np
    import torch
    import dsr_workloads as W
    from paper_1711_10413_amd import dsr as D

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    # a stream of its own: launches on the null stream pay for its implicit
    # synchronisation with other streams (about 6 us per region launch)
    work_stream = torch.cuda.Stream()
    torch.cuda.set_stream(work_stream)
    stream = torch.cuda.current_stream().cuda_stream
    out = {"metric": "region instances/sec (scalar-sharing sweep, LDS team stack)",
           "value": None, "unit": "region instances/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded splitmix64 inputs, resident in HBM)",
           "config": {"workload": "scalar sweep: 512 teams x 256 threads, K in {1,2,4,8,16,32,64} "
                                  "shared scalars, 2^24 fp32 x -> fp64 y, exact fp64 sum",
                      "teams": TEAMS, "wg_size": WG, "elements": N, "regions_per_step": 7,
                      "buffer_sets": SETS, "master_joins": args.master_joins,
                      "schedule": args.schedule}}
    if "sweep" in parts:
        say("sweep")
        sw = run_sweep(torch, np, D, W, args, stream)
        out["value"] = sw["value"]
        out["ms_per_step"] = sw["secs"] * 1e3 / args.steps
        # the dominant kernel: the region kernel's lean instances of the
        # HBM-bound chains (K <= 16: five of the step's seven regions, one
        # template specialised per chain length)
        avg_ms = sum(sw["per_k_kernel_ms"][K] for K in STREAM_KS) / len(STREAM_KS)
        achieved = sw["algo_bytes"] / (avg_ms * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": measured_traffic(DOMINANT),
                           "kernel": DOMINANT, "regions": "K in %s" % list(STREAM_KS),
                           "algorithmic_bytes_per_launch": sw["algo_bytes"],
                           "avg_launch_ms": avg_ms}
        # the 64-scalar chain is bound by fp64 FMA: 2 * 64 flop per element
        ms64 = sw["per_k_kernel_ms"].get(64)
        if ms64:
            tf = 2.0 * 64 * N / (ms64 * 1e-3) / 1e12
            out["roofline_k64"] = {"bound": "fp64 valu", "achieved": tf, "peak": 78.6, "unit": "TFLOP/s",
                                   "frac": tf / 78.6, "kernel": "dsr_region_kernel<256, %d>" % kernel_variant(64),
                                   "avg_launch_ms": ms64}
        for k in ("per_k_kernel_ms", "per_k_gbs", "loop_phase_us", "loop_phase_gbs",
                  "team_phases_us", "occupancy", "lds_bytes_per_team", "hbm_only_stack", "verified"):
            out[k] = sw[k]
    if "ceiling" in parts:
        say("ceiling")
        ce = run_ceiling(torch, D, stream)
        out["streaming_ceiling"] = ce
        if "roofline" in out:
            a = out["roofline"]["achieved"]
            out["roofline"]["frac_of_ceiling_same_shape"] = a / ce["grid_%dx%d" % (TEAMS, WG)]["gbs"]
            out["roofline"]["frac_of_ceiling_full_grid"] = a / ce["grid_4096x%d" % WG]["gbs"]
    if "lists" in parts:
        say("lists")
        out["reference_lists"] = run_lists(torch, np, D, W, stream)
    if "calib" in parts:
        say("calib")
        out["calibration_copy"] = run_calib(torch)
    if "plain" in parts:
        say("plain")
        out["plain_region"] = run_plain(torch, np, D, W, stream)
    if "arrays" in parts:
        say("arrays")
        shapes = [tuple(int(v) for v in t.split("x")) for t in args.arrays_shapes.split(",")] \
            if args.arrays_shapes else None
        out["arrays_nested"] = run_arrays(torch, np, D, W, stream, shapes=shapes)
    if "batched" in parts:
        say("batched")
        out["batched"] = run_batched(torch, np, D, W, stream, each=not args.no_batched_each)
    if "served" in parts:
        say("served")
        rates = [int(v) for v in args.serve_rates.split(",") if v]
        out["served"] = run_served(torch, np, D, W, stream, rates, args.serve_seconds,
                                   serial_seconds=args.serve_serial_seconds)
    if "cpu" in parts:
        say("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
