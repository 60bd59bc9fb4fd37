"""Host logic of bench.py: the raster's work units against closed forms, the
counter-summary stamp (measured traffic only for the library the summary measured),
the frame's VALU-issue floor from a summary, and the one-GPU rule."""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def table(rows):
    """[8][n] table from (cx, cy, angle, a, b, shape) tuples."""
    s = np.zeros((8, len(rows)), np.float32)
    for k, (cx, cy, ang, a, b, shape) in enumerate(rows):
        s[:, k] = [cx, cy, ang, a, b, 1.0, 0.03, shape]
    return s


def test_raster_work_closed_forms():
    H, W = 64, 48
    # square prism of half-width 5 centred on a pixel centre: binning box ext = 5 sqrt 2 + 1 = 8.07,
    # pixels 12..28 per axis; its four edges (perimeter 4 (a + b) = 40) cross 40 pixels when axis-aligned
    assert bench.raster_work(table([(20.5, 20.5, 0.0, 5, 5, 0)]), H, W) == (289.0, 40.0)
    # turned by 45 degrees: the same box, the edges cross sqrt 2 more pixels
    t, c = bench.raster_work(table([(20.5, 20.5, math.pi / 4, 5, 5, 0)]), H, W)
    assert t == 289.0 and c == pytest.approx(40.0 * math.sqrt(2.0), rel=1e-6)
    # an ellipsoid: ext = max(a, b) + 1 = 6, pixels 14..26, no clips
    assert bench.raster_work(table([(20.5, 20.5, 1.1, 5, 5, 1)]), H, W) == (169.0, 0.0)
    # clipped by the canvas corner: columns and rows 0..8
    assert bench.raster_work(table([(0.0, 0.0, 0.0, 5, 5, 0)]), H, W) == (81.0, 40.0)
    both = table([(20.5, 20.5, 0.0, 5, 5, 0), (0.0, 0.0, 0.0, 5, 5, 0), (20.5, 20.5, 1.1, 5, 5, 1)])
    assert bench.raster_work(both, H, W) == (539.0, 80.0)


def test_raster_flop_model_matches_the_frame():
    # the 2048^2 x 40k frame: 19.2 M candidate tests and 1.5 M clips, 0.50 GFLOP
    from paper_2606_21381_amd import workloads
    fr = workloads.config1()
    t, c = bench.raster_work(fr.soa, fr.H, fr.W)
    assert 1.90e7 < t < 1.94e7 and 1.4e6 < c < 1.6e6
    assert 0.48e9 < t * bench.RASTER_FLOP_PER_TEST + c * bench.RASTER_FLOP_PER_CLIP < 0.52e9


def summary(stamp, rows):
    head = "kernel                   fetch_MB   write_MB   total_MB   valu_winst  salu_inst  lanes    avg_us    valu%"
    lines = ["# test summary", "# kernel library: sha1 %s (test)" % stamp, head]
    for name, winst in rows:
        lines.append("%-24s %10.2f %10.2f %10.2f %12d %10d %6.3f %9.2f %8.1f" % (name, 1.0, 2.0, 3.0, winst, 0, 1.0,
                                                                                  10.0, 50.0))
    return "\n".join(lines) + "\n"


FRAME = [("k_bin", 1_000_000), ("k_bin_clear", 1_000), ("k_tile_scan", 2_000), ("k_emit", 300_000),
         ("k_pass1<11, 8>", 2_000_000), ("k_pass2<11, 8>", 500_000), ("k_pass3<11, 8>", 3_000_000),
         ("k_raster<false, false>", 10_000_000)]


@pytest.fixture
def lib_hash():
    try:
        return bench.kernel_hash()
    except OSError:
        pytest.skip("library not built")


def test_counter_stamp_and_valu_floor(tmp_path, monkeypatch, lib_hash):
    f = tmp_path / "counters.txt"
    monkeypatch.setattr(bench, "COUNTERS", str(f))
    f.write_text(summary(lib_hash, FRAME))
    c = bench.measured_counters("k_raster")
    assert c["traffic"] == 3.0e6 and c["fetch"] == 1.0e6 and c["write"] == 2.0e6
    assert c["valu_winst"] == 10_000_000 and c["valu_busy"] == 0.5
    # the pass names carry spaces; the bin counters must not be taken for the clear's
    assert bench.measured_counters("k_pass1<11")["valu_winst"] == 2_000_000
    total = sum(w for _, w in FRAME)
    assert bench.frame_valu_floor_us() == pytest.approx(total * 4.0 / (1024 * 2.4e3))
    # another build of the library: nothing is reported
    f.write_text(summary("0" * 40, FRAME))
    assert bench.measured_counters("k_raster") is None and bench.frame_valu_floor_us() is None
    # a summary missing one of the frame's kernels gives no floor
    f.write_text(summary(lib_hash, FRAME[:-1]))
    assert bench.frame_valu_floor_us() is None


def test_one_gpu_only():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "single MI355X" in r.stderr and r.stdout == ""
