"""Pins the CPU oracle to facts outside itself: a published generator test
vector, closed forms, exact rational arithmetic, Python's math.fsum, brute
force and the paper's own example programs."""
import json
import math
import os
import random
import struct
from fractions import Fraction

import numpy as np
import pytest

import dsr_workloads as W
from oracle import ref as R
from oracle import sim as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---- generator ----------------------------------------------------------
def test_splitmix64_published_vector():
    want = [int(l) for l in open(os.path.join(GOLD, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    assert W.splitmix64_sequence(1234567, 5) == want


def test_counter_draws_match_sequential_generator():
    for seed, stream in [(0, 0), (1, 2), (3, 513), (2**63 + 5, 17)]:
        base = int(W.stream_base(seed, stream))
        seq = W.splitmix64_sequence(base, 40)
        assert [int(v) for v in W.draws(seed, stream, 0, 40)] == seq
        assert [int(v) for v in W.draws(seed, stream, 17, 5)] == seq[17:22]


def test_fast_fp32_path_matches_numpy_path():
    for seed, stream, start, count in [(1, 2, 0, 100000), (3, 515, 12345, 3 << 20), (4, 9, 7, 1)]:
        a = W.uniform_f32(W.draws(seed, stream, start, count))
        b = W.uniform_f32_draws(seed, stream, start, count)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_value_maps_are_exact_and_in_range():
    u = W.draws(9, 2, 0, 200000)
    x = W.uniform_f32(u)
    assert x.min() >= -1.0 and x.max() < 1.0
    assert np.all((x.astype(np.float64) * 2**23) == np.round(x.astype(np.float64) * 2**23))
    f = W.uniform_f64(u)
    assert f.min() >= -1.0 and f.max() < 1.0
    assert np.all(f * 2.0**52 == np.round(f * 2.0**52))
    k = W.uniform_int(u, -1000, 1000)
    assert k.min() == -1000 and k.max() == 1000


# ---- Figure 1b pattern with four shared scalars ---------------------------
def closed_form_sum(a, b, c, d, n=1024):
    # sum_i a*i = a*n(n-1)/2; c XOR i over i < 1024 keeps c's bits above
    # bit 9 and permutes the low 10 bits through 0..1023.
    assert n == 1024
    return 523776 * a + 1024 * (b + d) - 1024 * (c & ~1023) - 523776


def test_affine_xor_closed_form_random_draws():
    rng = np.random.default_rng(0)
    for a, b, c, d in rng.integers(-1000, 1001, size=(20000, 4)):
        _, s = R.affine_xor(int(a), int(b), int(c), int(d), 0, 1024)
        assert s == closed_form_sum(int(a), int(b), int(c), int(d))


def test_affine_xor_brute_force_and_wrap():
    rng = random.Random(1)
    for _ in range(50):
        a, b, c, d = (rng.randint(-2**31, 2**31 - 1) for _ in range(4))
        lo = rng.randint(0, 5000)
        hi = lo + rng.randint(0, 40)
        out, s = R.affine_xor(a, b, c, d, lo, hi)
        want = []
        for i in range(lo, hi):
            v = (a * i + b - (c ^ i) + d) % 2**32      # exact integers, then wrap
            want.append(v - 2**32 if v >= 2**31 else v)
        assert list(out) == want and s == sum(want)


# ---- Figure 5 pattern: fma chain over the shared scalars --------------------
def frac_fma_chain(xi, si, sf, acc=0.0):
    for s in list(si) + list(sf):
        acc = float(Fraction(float(s)) * Fraction(float(xi)) + Fraction(acc))
    return acc


def test_fma_chain_single_int_scalar_is_exact_product():
    cf, x = W.cfg2_inputs(1, n=4096)
    y = R.fma_chain(x, cf.s_i32, cf.s_f64)
    assert np.array_equal(y, float(cf.s_i32[0]) * x.astype(np.float64))


@pytest.mark.parametrize("K", [2, 4, 8, 16, 64])
def test_fma_chain_matches_exact_rational_fma(K):
    cf, x = W.cfg2_inputs(K, n=1 << 12)
    y = R.fma_chain(x, cf.s_i32, cf.s_f64)
    for i in range(0, 1 << 12, 97):
        assert y[i] == frac_fma_chain(x[i], cf.s_i32, cf.s_f64)


def test_fma_chain_order_and_fusion_matter():
    # the pins above would catch a reordered chain: on the workload the
    # reversed order changes some results
    cf, x = W.cfg2_inputs(16, n=2000)
    y = R.fma_chain(x, cf.s_i32, cf.s_f64)
    rev = np.array([frac_fma_chain(v, list(cf.s_f64)[::-1], list(cf.s_i32)[::-1]) for v in x])
    assert np.any(rev != y)
    # ... and an unfused multiply-add: with x = 1 + 2**-23, s_i = -1 and
    # s_f = 1 + 2**-52 the fused chain keeps the 2**-75 bit of the product
    x1 = np.array([1 + 2.0**-23], np.float32)
    y1 = R.fma_chain(x1, [-1], [1 + 2.0**-52])
    assert y1[0] == 2.0**-52 + 2.0**-75
    unfused = (1 + 2.0**-52) * float(x1[0]) - float(x1[0])
    assert unfused == 2.0**-52 != y1[0]


def test_fma_chain_array_term():
    inst = W.cfg4_instance(5, 1000, 4096)
    x = W.instance_x(5, 1000)
    y = R.fma_chain(x, inst.s_i32, inst.s_f64, inst.arr)
    alen = len(inst.arr)
    for i in range(0, 1000, 37):
        assert y[i] == frac_fma_chain(x[i], inst.s_i32, inst.s_f64, float(inst.arr[i % alen]))


def test_products_lie_on_exact_sum_grid():
    # every y of these workloads is a multiple of 2**-75 below 2**32: the
    # exact-sum window of the fp64 reduction
    for K in (1, 8, 64):
        cf, x = W.cfg2_inputs(K, n=1 << 14)
        y = R.fma_chain(x, cf.s_i32, cf.s_f64)
        assert R.fixed75_sum(y) is not None
        assert np.all(np.abs(y) < 2.0**32)


# ---- exact summation ------------------------------------------------------
def test_exact_sum_against_fsum():
    rng = np.random.default_rng(3)
    cases = [rng.standard_normal(10000),
             rng.standard_normal(5000) * np.exp(rng.uniform(-300, 300, 5000)),
             np.array([1e100, 1.0, -1e100]),
             np.array([1.0, 2.0**-53]),                     # tie: even stays
             np.array([1.0 + 2**-52, 2.0**-53]),            # tie: rounds up
             np.array([1.0, 2.0**-53, 2.0**-106]),          # sticky breaks tie
             np.array([5e-324, 5e-324, -1e-320]),           # subnormals
             np.array([]), np.array([-0.0])]
    for v in cases:
        assert R.exact_sum(v) == math.fsum(v), v[:4]
    # a partial sum beyond the double range (math.fsum gives up here)
    v = np.array([1.7e308, 1.7e308, -1.7e308])
    assert R.exact_sum(v) == float(sum(Fraction(t) for t in v)) == 1.7e308
    assert R.exact_sum(np.array([1.7e308, 1.7e308])) == float("inf")


def test_exact_sum_matches_rational_on_workload():
    cf, x = W.cfg2_inputs(8, n=1 << 15)
    y = R.fma_chain(x, cf.s_i32, cf.s_f64)
    exact = sum((Fraction(float(v)) for v in y), Fraction(0))
    assert R.exact_sum(y) == float(exact) == math.fsum(y)
    assert Fraction(R.fixed75_sum(y), 2**75) == exact


def test_fixed75_rejects_off_grid():
    assert R.fixed75_sum(np.array([2.0**-76])) is None
    assert R.fixed75_sum(np.array([2.0**-75, 3.0])) == 1 + 3 * 2**75


# ---- Figure 6 pattern: shared arrays ---------------------------------------
@pytest.mark.parametrize("A,length", [(1, 16), (2, 256), (4, 4096), (3, 16384)])
def test_gather_periodic_and_brute(A, length):
    arrs = W.cfg3_arrays(A, length)
    n = 3 * length + 5
    out = R.gather(arrs, 0, n)
    d = out.astype(np.int64) - np.arange(n)
    assert np.array_equal(d[length:], d[:-length])               # period len
    for i in range(0, n, max(1, n // 200)):
        assert out[i] == sum(int(a[i % length]) for a in arrs) + i


# ---- contention-group simulator -------------------------------------------
def cfg1_program(c):
    out = np.zeros(1024, np.int64)
    prog = [S.Push(24, S.affine_xor_init(c.a, c.b, c.c, c.d)),
            S.Publish(0, "affine_xor", {"n": 1024, "out": out}), S.Pop(0)]
    return prog, out


@pytest.mark.parametrize("sched", ["block", "cyclic", "reverse", "random"])
@pytest.mark.parametrize("order", ["canonical", "roundrobin", "random"])
def test_sim_cfg1_every_schedule(sched, order):
    c = W.cfg1_inputs()
    prog, out = cfg1_program(c)
    tr, red = S.run_region(prog, 4, S.Config(workers=3, schedule=sched, interleave=order, seed=7))
    ro, rs = R.affine_xor(c.a, c.b, c.c, c.d, 0, 1024)
    assert red == [rs] == [closed_form_sum(c.a, c.b, c.c, c.d)]
    assert np.array_equal(out, ro)
    for t in tr:
        # section 5.3.1 aligns the stack to 8 bytes: the 24-byte frame takes 24
        assert t.error is None and t.placements == [("lds", 0, 24)]
        # Figures 2 and 3: two barriers per parallel region, one to end
        assert t.master_barriers == 3 and t.worker_barriers == [3, 3, 3]


def test_sim_exhaustive_interleavings_tiny():
    c = W.cfg1_inputs()
    for W_ in (1, 2, 3):
        for n in range(0, 7):
            out = np.zeros(n, np.int64)
            prog = [S.Push(24, S.affine_xor_init(c.a, c.b, c.c, c.d)),
                    S.Publish(0, "affine_xor", {"n": n, "out": out}), S.Pop(0)]
            want_out, want = R.affine_xor(c.a, c.b, c.c, c.d, 0, n)
            cfg = S.Config(workers=W_, schedule="cyclic")
            q = S.assign(range(n), W_, "cyclic", None)
            seen = 0
            for il in S.all_interleavings(q):
                if seen > 400:
                    break
                seen += 1
                out[:] = 0
                tr, red = S.run_region(prog, 1, cfg, interleaving=lambda qs, il=il: iter(il))
                assert red == [want] and np.array_equal(out, want_out)


def test_sim_fma_chain_exact_reduction():
    cf, x = W.cfg2_inputs(8, n=257)
    y = np.zeros(257)
    size, _ = S.fma_chain_layout(4, 4, 0)
    prog = [S.Push(size, S.fma_chain_init(cf.s_i32, cf.s_f64)),
            S.Publish(0, "fma_chain", {"n": 257, "x": x, "y": y, "ni": 4, "nf": 4}),
            S.Pop(0)]
    for teams in (1, 3, 5):
        tr, red = S.run_region(prog, teams, S.Config(workers=3, schedule="random", interleave="random"))
        yr = R.fma_chain(x, cf.s_i32, cf.s_f64)
        assert np.array_equal(y, yr)
        assert red == [R.exact_sum(yr)] == [math.fsum(yr)]


def test_sim_gather_nested_and_spill():
    arrs = W.cfg3_arrays(2, 16)
    n = 500
    out = np.zeros(n, np.int64)
    prog = [S.Push(2 * 16 * 4, S.gather_init(arrs)),
            S.Publish(0, "gather_nested", {"n": n, "out": out, "A": 2, "length": 16}), S.Pop(0)]
    for lds in (0, 64, 256):                      # 0 and 64: the frame spills
        out[:] = 0
        tr, red = S.run_region(prog, 3, S.Config(lds_bytes=lds, hbm_bytes=1024))
        assert np.array_equal(out, R.gather(arrs, 0, n))
        want_space = "lds" if lds >= 128 else "hbm"
        assert all(t.placements == [(want_space, 0, 128)] for t in tr)
        # one 16-byte inner frame per worker, on chip at its own stack's base
        assert all(t.sub_placements == [(2, "w%d" % m, "nlds", 64 * m, 16) for m in range(3)] for t in tr)


def test_sim_runtime_errors():
    c = W.cfg1_inputs()
    init = S.affine_xor_init(c.a, c.b, c.c, c.d)
    out = np.zeros(8, np.int64)
    pub = S.Publish(0, "affine_xor", {"n": 8, "out": out})
    cases = [
        ([S.Push(24, init), pub], "LIVE"),
        ([S.Push(24, init), S.Push(8), S.Pop(0), S.Pop(1)], "ORDER"),
        # a pop with no live frame has nothing to release: the stack of
        # section 5.3.1 underflows (not a state error of a live frame)
        ([S.Pop(0)], "UNDERFLOW"),
        ([S.Push(24, init), S.Pop(0), S.Pop(0)], "UNDERFLOW"),
        ([S.Push(24, init), S.Pop(0), pub], "STATE"),
        ([S.Push(4096)], "NOMEM"),
    ]
    for prog, code in cases:
        tr, red = S.run_region(prog, 2, S.Config(lds_bytes=64, hbm_bytes=1024))
        assert red is None and all(t.error == code for t in tr), (prog, code)


def test_sim_exact_sum_has_no_window():
    # the reduction is the exact sum of the y, rounded once: values off the
    # kernel's 2**-75 grid, or beyond 2**32, are summed exactly all the same
    # (the kernel reports such values as a range error instead)
    x = np.array([2.0**-30, 1.5, -1.5, 2.0**-30, 3.0], np.float32)
    y = np.zeros(5)
    size, _ = S.fma_chain_layout(0, 2, 0)
    prog = [S.Push(size, S.fma_chain_init([], [2.0**-50, 2.0**40])),
            S.Publish(0, "fma_chain", {"n": 5, "x": x, "y": y, "ni": 0, "nf": 2}), S.Pop(0)]
    for teams in (1, 2, 5):
        tr, red = S.run_region(prog, teams, S.Config(workers=2, schedule="random", seed=teams))
        yr = R.fma_chain(x, [], [2.0**-50, 2.0**40])
        assert all(t.error is None for t in tr)
        assert np.array_equal(y, yr) and R.fixed75_sum(yr) is None
        assert red == [math.fsum(yr)] == [float(sum(Fraction(float(v)) for v in yr))]


def brute_programs(depth):
    """Every push/pop sequence of at most ``depth`` pushes (LIFO pops at
    arbitrary points), with sizes drawn from a small set."""
    sizes = (0, 8, 16, 24, 40)
    def rec(prog, live, pushes):
        yield list(prog)
        if pushes < depth:
            for s in sizes:
                yield from rec(prog + [S.Push(s)], live + [pushes], pushes + 1)
        if live:
            yield from rec(prog + [S.Pop(live[-1])], live[:-1], pushes)
    yield from rec([], [], 0)


def test_sim_stack_brute_force_properties():
    count = 0
    for C in (0, 16, 32, 64):
        for H in (0, 16, 64):
            for T in (16, 1 << 20):
                for prog in brute_programs(3):
                    count += 1
                    team = S.Team(0, S.Config(lds_bytes=C, hbm_bytes=H, threshold=T), 1)
                    tr = S.run_team(team, prog)
                    # replay from the outside: sizes, spaces, capacities
                    live, sp = [], {"lds": 0, "hbm": 0}
                    pushes = [op for op in prog]
                    k = 0
                    expect_err = None
                    for op in prog:
                        if isinstance(op, S.Push):
                            size = -(-op.nbytes // 8) * 8
                            fits_l = size <= T and sp["lds"] + size <= C
                            fits_h = sp["hbm"] + size <= H
                            if not (fits_l or fits_h):
                                expect_err = "NOMEM"
                                break
                            space, off, sz = tr.placements[k]
                            assert sz == size and off == sp[space]
                            assert space == ("lds" if fits_l else "hbm")
                            sp[space] += size
                            live.append((space, size))
                            k += 1
                        else:
                            space, size = live.pop()
                            sp[space] -= size
                    if expect_err is None and live:
                        expect_err = "LIVE"
                    assert tr.error == expect_err
    assert count > 1000


def test_paper_programs():
    gold = json.load(open(os.path.join(GOLD, "paper_programs.json")))
    # Figure 6: a[i] starts at i; each worker adds d1[tid] = 10
    g6 = gold["fig6"]
    n = 3 * g6["workers"]
    out = np.zeros(n, np.int64)
    arr = [np.full(g6["workers"], g6["fill"], np.int32)]
    prog = [S.Push(4 * g6["workers"], S.gather_init(arr)),
            S.Publish(0, "gather", {"n": n, "out": out, "A": 1, "length": g6["workers"],
                                    "chunk": g6["workers"]}), S.Pop(0)]
    tr, _ = S.run_region(prog, 3, S.Config(workers=g6["workers"]))
    assert np.array_equal(out - np.arange(n), np.full(n, g6["increment"]))
    # Figure 5 (reading c_k = k): each element gains c1 + ... + c7
    g5 = gold["fig5"]
    n = 2 * g5["workers"]
    x = np.ones(n, np.float32)
    y = np.zeros(n)
    size, _ = S.fma_chain_layout(7, 0, 0)
    prog = [S.Push(size, S.fma_chain_init(g5["c"], [])),
            S.Publish(0, "fma_chain", {"n": n, "x": x, "y": y, "ni": 7, "nf": 0}), S.Pop(0)]
    tr, red = S.run_region(prog, 2, S.Config(workers=g5["workers"]))
    assert np.all(y == g5["increment"]) and red == [g5["increment"] * n]
    # Figure 1b: every worker reads the master's c == 1
    g1 = gold["fig1b"]
    n = 64
    x = np.ones(n, np.float32)
    y = np.zeros(n)
    size, _ = S.fma_chain_layout(1, 0, 0)
    prog = [S.Push(size, S.fma_chain_init([g1["c"]], [])),
            S.Publish(0, "fma_chain", {"n": n, "x": x, "y": y, "ni": 1, "nf": 0}), S.Pop(0)]
    S.run_region(prog, 1, S.Config(workers=8))
    assert np.all(y == g1["c"])


def test_sim_detects_planted_race():
    # a body that writes the shared slot from every worker in the same
    # phase must be flagged by the race detector
    class Racy(S.Body):
        def iteration(self, team, f, who, i, loop):
            team.write(f, 0, struct.pack("<q", i), who)
            return 0
    S.BODIES["racy"] = Racy()
    try:
        prog = [S.Push(24), S.Publish(0, "racy", {"n": 8}), S.Pop(0)]
        with pytest.raises(S.Violation):
            S.run_region(prog, 1, S.Config(workers=2))
    finally:
        del S.BODIES["racy"]
