"""The footprint/occupancy model against the HIP runtime's own occupancy
for the region kernel on the device."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1711_10413_amd import dsr as D  # noqa: E402


# control block of a 4-wave team: header 64, frame table 16 x 16, reference
# list 20 x 8, reduction slots 4 x 32, nested area 4 x (64 + 4 x 16 + 48)
CB4 = 64 + 256 + 160 + 4 * 32 + 4 * (64 + 4 * 16 + 48)


@pytest.mark.parametrize("wg,lds,variant", [(256, 4096, 0), (256, 4096, 2), (256, 32768, 0),
                                            (256, 65536, 1), (256, 163840 - CB4, 0),
                                            (1024, 8192, 0), (128, 16384, 0), (64, 0, 0)])
def test_model_matches_runtime(wg, lds, variant):
    assert D.dsr_control_bytes(256) == CB4
    ctx = D.dsr_init(wg_size=wg, lds_slab_bytes=lds, hbm_slab_bytes=4096, max_teams=4)
    o = D.dsr_region_occupancy(ctx, variant)
    print(wg, lds, variant, o)
    assert o["teams_per_cu"] == o["hip_teams_per_cu"], o
    assert o["teams_per_cu"] >= 1
    D.dsr_destroy(ctx)
