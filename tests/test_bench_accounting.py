"""The benchmark's roofline accounting, checked without a GPU: the algorithmic bytes of one
config-2 spectrum from its parts, and the committed HBM-traffic counters belonging to the
committed kernel source (so that the benchmark reports them) and lying just above those
bytes."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_config2_algorithmic_bytes():
    tables = 2 * 4 * 100 * 30000 * 4        # two temperature rows, 4 species, float32
    cia = 20 * 30000 * 8                    # every CIA temperature row, double
    out = 30000 * 8 + 1000 * 8              # depth and channel means, double
    assert bench.spectrum_bytes(4, 100, 30000, 20, 1000) == tables + cia + out == 101_048_000


def test_committed_traffic_matches_the_kernel_source():
    alg = bench.spectrum_bytes(4, 100, 30000, 20, 1000)
    one = bench.traffic_from_profile("config2_b1", 5)
    assert one is not None, "profiles/forward_traffic.json was taken on another kernel source"
    assert alg <= one <= 1.10 * alg
    many = bench.traffic_from_profile("config2_b256", 3)
    assert many is not None and many < 256 * alg      # samples of a tile share rows in L2
    assert bench.traffic_from_profile("config2_b1", 99) is None
