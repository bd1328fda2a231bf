"""The contention-group simulator as a checker: planted mistakes in the
model itself (on the CPU) must trip its invariants, and its nested levels,
member stacks and exact sums must agree with plain definitions.

Each mutation test changes one step of the simulator with monkeypatch and
asserts that a specific invariant fires; the unmodified run of the same
program passes.  This shows the invariants can fail, not only hold."""
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

import dsr_workloads as W
from oracle import ref as R
from oracle import sim as S


def cfg1_program():
    c = W.cfg1_inputs()
    out = np.zeros(1024, np.int64)
    prog = [S.Push(24, S.affine_xor_init(c.a, c.b, c.c, c.d)),
            S.Publish(0, "affine_xor", {"n": 1024, "out": out}), S.Pop(0)]
    return prog, out, c


def nested_program(A, length, n, depth, chunk=None):
    arrs = W.cfg3_arrays(A, length)
    out = np.zeros(n, np.int64)
    loop = {"n": n, "out": out, "A": A, "length": length, "depth": depth}
    if chunk:
        loop["chunk"] = chunk
    prog = [S.Push(4 * A * length, S.gather_init(arrs)), S.Publish(0, "gather_nested", loop), S.Pop(0)]
    return prog, out, arrs


# ---- I1: what a worker sees at its await ------------------------------------
def test_i1_holds_on_the_unmodified_model():
    prog, out, c = cfg1_program()
    tr, red = S.run_region(prog, 2, S.Config(workers=3))
    assert red == [R.affine_xor(c.a, c.b, c.c, c.d, 0, 1024)[1]]


def test_i1_fires_when_the_fork_does_not_release_the_masters_writes(monkeypatch):
    """A worker that reads the frame before the master's writes are
    released (as if it looked before the fork barrier) sees stale bytes."""
    prog, out, c = cfg1_program()
    real = S.Team.sync

    def no_release(self, scope):
        self.epoch[scope] = self.epoch.get(scope, 0) + 1     # a barrier that publishes nothing

    monkeypatch.setattr(S.Team, "sync", no_release)
    with pytest.raises(S.Violation, match="I1"):
        S.run_region(prog, 1, S.Config(workers=3))
    monkeypatch.setattr(S.Team, "sync", real)
    S.run_region(prog, 1, S.Config(workers=3))


def test_i1_fires_when_workers_look_before_the_fork(monkeypatch):
    """Workers take their view of the frame before the fork barrier instead
    of after it (the publish steps in the wrong order)."""
    prog, out, c = cfg1_program()
    real_check = S.check_views
    seen = {}

    def early_publish(team, f, op, rng, interleaving):
        early = {w: team.frame_view(f, "w%d" % w) for w in range(team.cfg.workers)}
        master_view = team.frame_view(f, "master")
        team.barrier("all")
        for w, v in early.items():
            if v != master_view:
                seen["fired"] = True
                raise S.Violation("I1: w%d sees a frame different from its master's" % w)

    monkeypatch.setattr(S, "publish", early_publish)
    with pytest.raises(S.Violation, match="I1"):
        S.run_region(prog, 1, S.Config(workers=2))
    assert seen["fired"] and real_check is S.check_views


def test_i1_fires_at_a_nested_level_without_the_inner_release(monkeypatch):
    """The member's barrier with its inner team releases the member's
    writes; without it the inner members see a stale inner frame."""
    prog, out, arrs = nested_program(2, 16, 300, 2)
    real = S.Team.sync

    def team_only(self, scope):
        if scope == S.TEAM:
            return real(self, scope)
        self.epoch[scope] = self.epoch.get(scope, 0) + 1

    monkeypatch.setattr(S.Team, "sync", team_only)
    with pytest.raises(S.Violation, match="I1"):
        S.run_region(prog, 1, S.Config(workers=4))


# ---- race detector with distinct inner identities -----------------------------
def test_inner_members_are_distinct_threads_for_the_race_detector(monkeypatch):
    """An inner member that writes into the inner frame its siblings read
    races with them: the detector tells inner members apart."""
    prog, out, arrs = nested_program(1, 16, 200, 2)
    real = S.read_nested

    def writing_read(team, f, who):
        v = real(team, f, who)
        team.write(f, 0, struct.pack("<I", v[0]), who)          # planted: a member writes
        return v

    monkeypatch.setattr(S, "read_nested", writing_read)
    with pytest.raises(S.Violation, match="race detector"):
        S.run_region(prog, 1, S.Config(workers=2))


def test_inner_member_reading_a_sibling_members_frame_races(monkeypatch):
    """A member of one inner team reading another member's inner frame has
    no barrier in common with its writer but the team's, which came before
    the write: flagged."""
    prog, out, arrs = nested_program(1, 16, 200, 2)
    real = S.read_nested
    frames = {}

    def snooping_read(team, f, who):
        frames[f.owner] = f
        if who.startswith("w1.") and "w0" in frames and frames["w0"].fid not in team.dead:
            team.read(frames["w0"], 0, 4, who)
        return real(team, f, who)

    def run_members_together(team, outer_frame, loop, lo, hi):
        # both members push and publish before either's inner team runs
        cfg = team.cfg
        f = []
        for m in range(cfg.workers):
            a, b = S.split(lo, hi, cfg.workers, m)
            fm, _ = S.nested_fork(team, team.wave_stack(m), "w%d" % m, a, b, outer_frame)
            frames["w%d" % m] = fm
            f.append(fm)
        for m in range(cfg.workers):
            for g in range(cfg.inner):
                S.read_nested(team, f[m], "w%d.g%d" % (m, g))

    monkeypatch.setattr(S, "read_nested", snooping_read)
    monkeypatch.setattr(S, "run_nested", run_members_together)
    with pytest.raises(S.Violation, match="race detector"):
        S.run_region(prog, 1, S.Config(workers=2))


# ---- nested levels: results, placement, overflow, errors ------------------------
@pytest.mark.parametrize("depth", [2, 3])
@pytest.mark.parametrize("A,length", [(1, 16), (2, 100), (3, 256)])
def test_nested_levels_match_plain_gather(depth, A, length):
    n = 1000
    prog, out, arrs = nested_program(A, length, n, depth)
    tr, _ = S.run_region(prog, 3, S.Config(workers=4))
    assert np.array_equal(out, R.gather(arrs, 0, n))
    for t in tr:
        assert t.error is None
        lv2 = [p for p in t.sub_placements if p[0] == 2]
        lv3 = [p for p in t.sub_placements if p[0] == 3]
        assert lv2 == [(2, "w%d" % m, "nlds", 64 * m, 16) for m in range(4)]
        if depth == 3:
            # lane-group stacks follow the four wave stacks
            assert lv3 == [(3, "w%d.g%d" % (m, g), "nlds", 4 * 64 + 16 * (4 * m + g), 16)
                           for m in range(4) for g in range(4)]
        else:
            assert lv3 == []


def test_nested_stacks_overflow_to_global_memory():
    """With no on-chip room for member stacks (section 7: the runtime's
    global-memory stack), every nested frame goes to global memory at the
    member's own base; results do not change."""
    n = 700
    prog, out, arrs = nested_program(2, 64, n, 3)
    cfg = S.Config(workers=4, wave_lds=0, group_lds=0, wave_hbm=32, group_hbm=16)
    tr, _ = S.run_region(prog, 2, cfg)
    assert np.array_equal(out, R.gather(arrs, 0, n))
    for t in tr:
        assert [p[2] for p in t.sub_placements] == ["nhbm"] * 20
        assert [p[3] for p in t.sub_placements if p[0] == 2] == [32 * m for m in range(4)]
        assert [p[3] for p in t.sub_placements if p[0] == 3] == [4 * 32 + 16 * k for k in range(16)]


def test_nested_partial_overflow_and_nomem():
    n = 300
    prog, out, arrs = nested_program(1, 16, n, 3)
    # wave stacks on chip, lane-group stacks in global memory
    tr, _ = S.run_region(prog, 1, S.Config(workers=2, group_lds=8, group_hbm=16))
    assert np.array_equal(out, R.gather(arrs, 0, n))
    assert {p[2] for p in tr[0].sub_placements if p[0] == 2} == {"nlds"}
    assert {p[2] for p in tr[0].sub_placements if p[0] == 3} == {"nhbm"}
    # a member stack that fits neither part: the region fails
    tr, red = S.run_region(prog, 2, S.Config(workers=2, group_lds=8, group_hbm=8))
    assert red is None and all(t.error == "NOMEM" for t in tr)
    tr, red = S.run_region(prog, 1, S.Config(workers=2, wave_lds=0, wave_hbm=0))
    assert red is None and tr[0].error == "NOMEM"


def test_member_stack_brute_force():
    """Every sequence of up to four nested pushes with LIFO pops on one
    member stack: spaces, offsets and errors follow the placement rule."""
    sizes = (0, 4, 8, 16, 24)

    def programs(depth):
        def rec(prog, live, k):
            yield list(prog)
            if k < depth:
                for s in sizes:
                    yield from rec(prog + [("push", s)], live + [k], k + 1)
            if live:
                yield from rec(prog + [("pop", live[-1])], live[:-1], k)
        yield from rec([], [], 0)

    count = 0
    for cap_l in (0, 8, 16, 32):
        for cap_h in (0, 16, 48):
            for prog in programs(4):
                count += 1
                team = S.Team(0, S.Config(workers=1, lds_bytes=0, hbm_bytes=0, wave_lds=cap_l,
                                          wave_hbm=cap_h, group_lds=0, group_hbm=0), 1)
                ms = team.wave_stack(0)
                live, frames, sp = [], {}, {"nlds": 0, "nhbm": 0}
                err = None
                for op, v in prog:
                    if op == "push":
                        size = -(-v // 8) * 8
                        want = ("nlds" if sp["nlds"] + size <= cap_l else
                                "nhbm" if sp["nhbm"] + size <= cap_h else None)
                        try:
                            f = ms.push(v)
                        except S.SimError as e:
                            err = e.code
                            assert want is None and err == "NOMEM"
                            break
                        assert f.space == want and f.size == size
                        assert f.off == sp[want]
                        sp[want] += size
                        frames[v, len(frames)] = f
                        live.append(f)
                    else:
                        f = live.pop()
                        ms.pop(f)
                        sp[f.space] -= f.size
                    assert ms.sp == sp
                if err is None and live:
                    # a non-top pop is refused (I2)
                    if len(live) > 1:
                        with pytest.raises(S.SimError, match="ORDER"):
                            ms.pop(live[0])
    assert count > 1000


def test_bad_nesting_depth():
    prog, out, arrs = nested_program(1, 16, 64, 4)
    tr, red = S.run_region(prog, 1)
    assert tr[0].error == "INVAL"


# ---- alignment and exact sums -----------------------------------------------------
def test_default_alignment_is_eight_bytes():
    tr, _ = S.run_region([S.Push(20), S.Push(4), S.Pop(1), S.Pop(0)], 1)
    assert tr[0].placements == [("lds", 0, 24), ("lds", 24, 8)]
    tr, _ = S.run_region([S.Push(20), S.Push(4), S.Pop(1), S.Pop(0)], 1, S.Config(align=16))
    assert tr[0].placements == [("lds", 0, 32), ("lds", 32, 16)]


def test_exact_sum_across_teams_is_one_rounding():
    """y = 1, 2**-53, 2**-53: adding them one by one in double gives 1 (each
    2**-53 is a tie that rounds to even), the exact sum is 1 + 2**-52.  The
    simulator's reduction is the exact one however teams and workers split
    the loop."""
    x = np.array([1.0, 2.0**-53, 2.0**-53, 0.0], np.float32)
    y = np.zeros(len(x))
    size, _ = S.fma_chain_layout(1, 0, 0)
    prog = [S.Push(size, S.fma_chain_init([1], [])),
            S.Publish(0, "fma_chain", {"n": len(x), "x": x, "y": y, "ni": 1, "nf": 0}), S.Pop(0)]
    naive = 0.0
    for v in x:
        naive += float(v)
    assert naive == 1.0
    for teams in (1, 2, 4):
        for sched in ("block", "cyclic", "reverse"):
            tr, red = S.run_region(prog, teams, S.Config(workers=2, schedule=sched))
            assert red == [1.0 + 2.0**-52] == [math.fsum(x.astype(np.float64))]
