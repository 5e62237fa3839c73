"""Host-side checks of bench.py's measurement contract (no GPU): the committed profile summaries
belong to the current kernel sources, and the roofline arithmetic."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (imports nothing from the GPU stack at module level)

C = bench.CSRC

# profile summary -> the sources whose digest it records (the same lists bench.py hashes)
PROFILES = {
    "batch_update_f32_rmat_s24": [C + "batch.hip", C + "batch.h", C + "internal.h"],
    "update_f64_rmat_s24": [C + "pull.hip", C + "device.h", C + "internal.h", C + "segment.hip"],
    "multi_64graphs": [C + "multi.hip", C + "multi.h", C + "device.h", C + "internal.h"],
}


@pytest.mark.parametrize("tag", sorted(PROFILES))
def test_committed_counters_belong_to_the_current_kernels(tag):
    # bench.py reports roofline.traffic only when the summary's digest matches the sources; a
    # kernel changed without a new rocprofv3 summary would silently report traffic = null
    traffic = bench.read_traffic(tag, bench.source_digest(PROFILES[tag]))
    assert traffic is not None and traffic > 0, "profiles/%s_traffic.txt was taken on other kernel sources" % tag
    assert os.path.exists(os.path.join(ROOT, "profiles", tag + ".md"))


def test_roofline_arithmetic():
    r = bench.roofline("k", alg_bytes=4e9, avg_s=2e-3, launches=7, traffic=1.2e10)
    assert r["achieved"] == pytest.approx(2000.0)
    assert r["frac"] == pytest.approx(2000.0 / bench.HBM_PEAK_GBS, abs=1e-4)
    assert r["traffic_GBps"] == pytest.approx(6000.0)
    assert r["traffic_frac_of_peak"] == pytest.approx(6000.0 / bench.HBM_PEAK_GBS, abs=1e-4)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["launches_timed"] == 7
    assert "traffic_GBps" not in bench.roofline("k", 1e9, 1e-3, 1, None)
