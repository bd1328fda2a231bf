"""The launch that allocates nothing (dsr_launch_static): its outputs and
reductions against dsr_launch's for the same region programs, on calls in a
row through the one fixed workspace, the later ones smaller; and against the
oracle."""
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


def run_static(region):
    rec = torch.zeros(D.RESULT_REC_BYTES, dtype=torch.uint8, device="cuda")
    D.dsr_launch_static(region, rec.data_ptr(), stream())
    torch.cuda.synchronize()
    return D.result_rec(rec.cpu().numpy().tobytes())


def fma_region(ctx, K, n, teams, x, y, seed_k=None):
    cf, _ = W.cfg2_inputs(K, n=n, with_x=False)
    img, size = D.fma_chain_frame(cf.s_i32, cf.s_f64)
    r = D.dsr_region_begin(ctx, teams)
    f = D.dsr_push(r, size, img)
    D.dsr_publish(r, f, D.DSR_BODY_FMA_CHAIN, n, inp=x.data_ptr(), out=y.data_ptr(),
                  ni=len(cf.s_i32), nf=len(cf.s_f64))
    D.dsr_pop(r, f)
    return r, cf


@pytest.mark.parametrize("joins", [0, 1])
def test_static_matches_launch_on_calls_in_a_row(joins):
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=4096, hbm_slab_bytes=4096, max_teams=512,
                     master_joins=joins)
    # (K, elements, teams): the second and third calls are smaller than the
    # first, and the third takes the run-time chain
    for K, n, teams in ((8, 1 << 20, 512), (4, (1 << 16) + 37, 16), (5, 1000, 3)):
        say("static fma", joins, K, n, teams)
        _, x_np = W.cfg2_inputs(1, n=n)
        x = torch.from_numpy(x_np).cuda()
        y_a = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        y_b = torch.full((n,), -2.0, dtype=torch.float64, device="cuda")
        ra, cf = fma_region(ctx, K, n, teams, x, y_a)
        rb, _ = fma_region(ctx, K, n, teams, x, y_b)
        assert D.dsr_static_bytes(rb) <= D.DSR_STATIC_SCRATCH_BYTES
        D.dsr_launch(ra, stream())
        assert D.dsr_region_sync(ra) == 0
        rec = run_static(rb)
        assert rec["status"] == 0
        ya = y_a.cpu().numpy()
        yb = y_b.cpu().numpy()
        assert np.array_equal(ya.view(np.uint64), yb.view(np.uint64))
        yr = R.fma_chain(x_np, cf.s_i32, cf.s_f64)
        assert np.array_equal(yb.view(np.uint64), yr.view(np.uint64))
        _, f64, fixed = D.dsr_region_reduction(ra, 0)
        assert rec["f64"] == [f64] and rec["fixed"] == [fixed]
        assert f64 == R.exact_sum(yr) and fixed == R.fixed75_sum(yr)
        D.dsr_region_free(ra)
        D.dsr_region_free(rb)
    D.dsr_destroy(ctx)


def test_static_integer_and_spilled_nested_frames():
    """cfg1's region and a nested gather whose frame spills to the HBM stack
    (its nested members' stacks then also live in the workspace), then the
    cfg1 region again: every call matches dsr_launch and the oracle."""
    c = W.cfg1_inputs()
    ctx = D.dsr_init(wg_size=256, lds_slab_bytes=1024, hbm_slab_bytes=16384, max_teams=64,
                     master_joins=1)
    ro, rs = R.affine_xor(c.a, c.b, c.c, c.d, 0, 1024)

    def plain():
        out = torch.zeros(1024, dtype=torch.int32, device="cuda")
        r = D.dsr_region_begin(ctx, 4)
        f = D.dsr_push(r, 24, D.affine_xor_frame(c.a, c.b, c.c, c.d))
        D.dsr_publish(r, f, D.DSR_BODY_AFFINE_XOR, 1024, out=out.data_ptr())
        D.dsr_pop(r, f)
        return r, out

    ra, oa = plain()
    D.dsr_launch(ra, stream())
    assert D.dsr_region_sync(ra) == 0
    rb, ob = plain()
    rec = run_static(rb)
    assert rec["status"] == 0 and rec["i64"] == [rs] == [D.dsr_region_reduction(ra, 0)[0]]
    assert np.array_equal(ob.cpu().numpy(), ro) and np.array_equal(oa.cpu().numpy(), ro)
    D.dsr_region_free(rb)

    # nested members' frames forced to their global stacks, which the static
    # launch places in the workspace too
    ctx2 = D.dsr_init(wg_size=256, lds_slab_bytes=1024, hbm_slab_bytes=16384, max_teams=64,
                      master_joins=1, flags=D.DSR_F_NESTED_GLOBAL)
    arrs = W.cfg3_arrays(3, 1024)            # 12 KiB frame > the 1 KiB LDS slab
    n, teams = (1 << 18) + 12, 64
    outs = []
    for launch in ("launch", "static"):
        for depth in (2, 3):
            out = torch.full((n,), -7, dtype=torch.int32, device="cuda")
            r = D.dsr_region_begin(ctx2, teams)
            f = D.dsr_push(r, 4 * 3 * 1024, D.gather_frame(arrs))
            D.dsr_publish(r, f, D.DSR_BODY_GATHER_NESTED, n, out=out.data_ptr(), arrays=3, length=1024,
                          depth=depth)
            D.dsr_pop(r, f)
            if launch == "launch":
                D.dsr_launch(r, stream())
                assert D.dsr_region_sync(r) == 0
            else:
                assert run_static(r)["status"] == 0
            outs.append(out.cpu().numpy())
            D.dsr_region_free(r)
    want = R.gather(arrs, 0, n)
    for o in outs:
        assert np.array_equal(o, want)
    D.dsr_destroy(ctx2)

    rc, oc = plain()
    rec = run_static(rc)
    assert rec["status"] == 0 and rec["i64"] == [rs]
    assert np.array_equal(oc.cpu().numpy(), ro)
    D.dsr_region_free(rc)
    D.dsr_region_free(ra)
    D.dsr_destroy(ctx)
