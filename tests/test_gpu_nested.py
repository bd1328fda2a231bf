"""GPU parity of the nested levels (section 3.1.2 nesting; section 7's
sharing at worker level): every participating wave is the master of an
inner team of four 16-lane groups, and at depth 3 every group is the master
of four 4-lane groups.  Each member pushes its frame on its own member
stack (on chip, or the global part), its inner members reach the team's
arrays through the chain of frame references, and frames pop in LIFO
order.  Outputs are compared element by element with the plain gather;
the member stacks' placements with the contention-group simulator's."""
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


def sim_placements(members, depth, nest_global):
    """The simulator's member-stack placements for one team."""
    arrs = W.cfg3_arrays(1, 16)
    loop = {"n": 64, "out": np.zeros(64, np.int64), "A": 1, "length": 16, "depth": depth}
    cfg = S.Config(workers=members, align=16,
                   wave_lds=0 if nest_global else 64, group_lds=0 if nest_global else 16,
                   wave_hbm=256, group_hbm=64)
    tr, _ = S.run_region([S.Push(64, S.gather_init(arrs)), S.Publish(0, "gather_nested", loop), S.Pop(0)],
                         1, cfg)
    assert tr[0].error is None
    return tr[0].sub_placements


@pytest.mark.parametrize("depth", [2, 3])
@pytest.mark.parametrize("nest_global", [0, 1])
@pytest.mark.parametrize("joins", [0, 1])
@pytest.mark.parametrize("A,length", [(1, 16), (2, 256), (4, 4096), (3, 100), (2, 16384)])
def test_nested_levels(depth, nest_global, joins, A, length):
    say("nested depth", depth, "global", nest_global, "joins", joins, "A", A, "len", length)
    arrs = W.cfg3_arrays(A, length)
    n = (1 << 18) + 7
    teams = 16
    frame = 4 * A * length
    slab = (frame + 15) // 16 * 16
    flags = D.DSR_F_TRACE | (D.DSR_F_NESTED_GLOBAL if nest_global else 0)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=slab if slab <= 65536 else 0, hbm_slab_bytes=slab,
                     max_teams=teams, master_joins=joins, flags=flags)
    out = torch.zeros(n, dtype=torch.int32, device="cuda")
    r = D.dsr_region_begin(ctx, teams)
    f = D.dsr_push(r, frame, D.gather_frame(arrs))
    D.dsr_publish(r, f, D.DSR_BODY_GATHER_NESTED, n, out=out.data_ptr(), arrays=A, length=length,
                  depth=depth)
    D.dsr_pop(r, f)
    D.dsr_launch(r, stream())
    assert D.dsr_region_sync(r) == 0
    assert np.array_equal(out.cpu().numpy(), R.gather(arrs, 0, n))
    members = 4 if joins else 3
    want = sim_placements(members, depth, nest_global)
    for t in (0, teams - 1):
        tr = D.dsr_region_trace(r, t)
        got = []
        for m in range(members):
            nm = tr["nested"][m]
            assert nm["pop_error"] == 0 and nm["pushes"] == (1 if depth == 2 else 5), (m, nm)
            got.append((2, "w%d" % m) + nm["frame"] + (16,))
            if depth == 3:
                got += [(3, "w%d.g%d" % (m, g)) + nm["groups"][g] + (16,) for g in range(4)]
        assert sorted(got) == sorted(want), (got, want)
        assert tr["inner_pushes"][:members] == [1 if depth == 2 else 5] * members
    D.dsr_region_free(r)
    D.dsr_destroy(ctx)


@pytest.mark.parametrize("depth", [2, 3])
def test_nested_small_and_ragged_ranges(depth):
    """Loops shorter than the members (some members get empty pieces),
    odd lengths, and a team range that starts off a vector boundary."""
    arrs = W.cfg3_arrays(2, 12)
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=4096, hbm_slab_bytes=4096, max_teams=8, master_joins=1)
    for n, chunk in ((0, 0), (1, 0), (5, 0), (63, 0), (1001, 0), (1001, 130), (4099, 514)):
        teams = 8 if chunk == 0 else -(-n // chunk)
        out = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
        r = D.dsr_region_begin(ctx, teams)
        f = D.dsr_push(r, 96, D.gather_frame(arrs))
        D.dsr_publish(r, f, D.DSR_BODY_GATHER_NESTED, n, out=out.data_ptr(), arrays=2, length=12, depth=depth,
                      chunk=chunk)
        D.dsr_pop(r, f)
        D.dsr_launch(r, stream())
        assert D.dsr_region_sync(r) == 0, (n, chunk)
        if n:
            assert np.array_equal(out.cpu().numpy()[:n], R.gather(arrs, 0, n)), (n, chunk)
        D.dsr_region_free(r)
    D.dsr_destroy(ctx)
