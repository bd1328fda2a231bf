"""The region kernel's instances compile without scratch (no register
spills, no private arrays) and within the register budget their
workgroup size allows: 256 per lane up to 512 threads (two waves per SIMD),
128 for 1024-thread workgroups.  A device-only compile on the CPU."""
import shutil

import pytest

from paper_1711_10413_amd import build as B


@pytest.mark.skipif(not shutil.which(B.HIPCC) and not __import__("os").path.exists(B.HIPCC),
                    reason="hipcc not available")
def test_no_scratch_and_register_budget():
    res = B.kernel_resources()
    names = [n for n in res if "dsr_region_kernel" in n]
    assert len(names) == len(B.instances()), res
    for n in names:
        r = res[n]
        assert r["scratch"] == 0, (n, r)
        limit = 128 if "ILi1024E" in n else 256
        assert r["vgprs"] <= limit, (n, r)
        assert r["waves_per_simd"] >= (4 if "ILi1024E" in n else 2), (n, r)
