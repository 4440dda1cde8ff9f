"""The kernels' tunable sizes come from the library (no GPU work), and the
fallback-path geometries of the GPU operator tests exceed them by the host
lower bounds, so those tests really take the global-memory paths."""

import sys
import os

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def test_kernel_config_is_sane():
    import paper_1002_3675_amd as cb
    cfg = cb.kernel_config()
    assert cfg["tile_u"] * cfg["tile_v"] == 256  # one lane per ray of a tile
    assert cfg["brick_x"] * cfg["brick_y"] * cfg["brick_z"] == 256  # one lane per cell
    assert cfg["tile_lds_floats"] > 0 and cfg["table_pixels"] > 0 and cfg["tile_chunk"] > 0


def test_fallback_geometries_exceed_the_staged_capacity():
    import paper_1002_3675_amd as cb
    from test_gpu_operators import fallback_margins
    pt, p = fallback_margins(cb.kernel_config())
    assert pt > 2.0, pt
    assert p > 2.0, p
