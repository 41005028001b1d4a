"""Host-side arithmetic of bench.py's roofline objects (no GPU): the
algorithmic bytes per launch of the radix scatter and the tile build."""
import os
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(__file__), ".."))
import bench  # noqa: E402


def _stats(items, tile, item_bytes=20, passes=2):
    return {"sort_items": items, "tile": tile, "sort_item_bytes": item_bytes, "sort_passes": passes}


def test_scatter_bytes_per_launch():
    # a narrow two-pass sort moves 12 + 8 = 20 bytes per item over its passes
    st = [_stats(1_000_000, 64)]
    r = bench.roofline_for("scatter", st, ms=2.0, n=2, workload="none", nverts=0)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(1_000_000 * 10.0)
    assert r["achieved"] == pytest.approx(1_000_000 * 10.0 / 1e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS)
    # three key + value passes, the last writing no keys: 16 + 16 + 12
    st = [_stats(1_000_000, 64, item_bytes=44, passes=3)]
    r = bench.roofline_for("scatter", st, ms=3.0, n=3, workload="none", nverts=0)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(1_000_000 * 44.0 / 3)


def test_tile_bytes_lazy_and_eager():
    tris, verts = 64 * 100_000, 3_000_000
    lazy = bench.roofline_for("tiles", [_stats(tris, 64)], ms=1.0, n=1, workload="none",
                              nverts=verts)
    ntiles = tris / 64
    assert ntiles >= bench.LAZY_COPY_MIN_TILES
    assert lazy["algorithmic_bytes_per_launch"] == pytest.approx(
        tris * bench.BYTES_TILE_TRI + verts * bench.BYTES_TILE_VTX + ntiles * bench.BYTES_TILE_META)
    # a call under the threshold also writes the 36-byte FP32 copy of every slot
    small = 128 * 100
    eager = bench.roofline_for("tiles", [_stats(small, 128)], ms=1.0, n=1, workload="none",
                               nverts=6000)
    assert eager["algorithmic_bytes_per_launch"] == pytest.approx(
        small * (bench.BYTES_TILE_TRI + bench.BYTES_TILE_COPY) + 6000 * bench.BYTES_TILE_VTX +
        (small / 128) * bench.BYTES_TILE_META)
