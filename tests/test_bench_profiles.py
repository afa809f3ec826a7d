"""The benchmark reads its counter figures from the committed rocprofv3
summaries by kernel name: every kernel it looks up is there."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2605_17222_amd import profiling  # noqa: E402


def test_profile_summaries_name_the_benchmarked_kernels():
    trace = profiling.read_block(bench.PROFILE_TRACE)
    hbm = profiling.read_block(bench.PROFILE_HBM)
    valu = profiling.read_block(bench.PROFILE_VALU)
    assert trace and hbm and valu
    for name in bench.TH444_KERNEL.values():
        assert name in trace["kernels"], name
        assert name in hbm["kernels"], name
        assert name in valu["kernels"], name
    # the trace covers the number of LTs the bench divides by
    assert trace["kernels"][bench.TH444_KERNEL["ksmac"]]["calls"] == bench.PROFILE_LTS
