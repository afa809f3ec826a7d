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


def test_profile_summaries_were_taken_from_the_current_sources():
    """Every summary the bench reads carries the digest of the library
    sources it was profiled from; a committed tree keeps them in step (the
    bench drops counter figures whose digest does not match)."""
    for path in (bench.PROFILE_TRACE, bench.PROFILE_HBM, bench.PROFILE_VALU):
        assert profiling.current_block(path) is not None, path


def test_keyswitch_phase_kernels_are_library_kernels():
    import paper_2605_17222_amd as H
    for name in bench.KEYSWITCH_KERNELS:
        assert name in H.KERNELS, name
