"""Host-side pieces of bench.py (no GPU): the work model behind the roofline
figures and the reader of the committed traffic summary."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_slot_model_is_consistent():
    for k in range(1, 7):
        # algorithmic slots: 12 + 2k (one add at k = 1) + 4 per transcendental,
        # one for the delay and one (k = 2) or two (k >= 3) for the root
        n_trans = 1 + (0 if k == 1 else 1 if k == 2 else 2)
        assert bench.ALGO_SLOTS[k] == 12 + (2 if k == 1 else 2 * k) + 4 * n_trans
        # a transcendental weighs four plain slots in the published-peak model
        assert bench.METHOD_SLOTS[k] == bench.NONTRANS[k] + 4 * bench.TRANS[k]
        # delay (sqrt, rcp) always; roots add 0 (k=1), 1 (k=2) or 2 transcendentals
        assert bench.TRANS[k] == 2 + {1: 0, 2: 1}.get(k, 2)
    # the all-orders kernel computes the delay once, so it costs less than the
    # per-order kernels together and at least the highest order alone
    for kmax in range(1, 7):
        assert bench.METHOD_SLOTS[kmax] <= bench.FUSED_SLOTS[kmax] <= \
            sum(bench.METHOD_SLOTS[k] for k in range(1, kmax + 1))
    # the fraction of the peak follows the algorithmic count
    assert abs(bench.frac_of_peak(6, 1e6, 36e6 / 78.64e12) - 1.0) < 1e-12


def test_profiled_traffic_reader():
    # present only while the committed summary matches the kernel source
    v = bench._profiled_traffic("hodmas_frame_kernel<6, f32, comp>")
    assert v is None or 1e6 < v < 1e9
    assert bench._profiled_traffic("no such kernel") is None
    assert bench._issued_slots("no such kernel", 1e6, 1e-3) is None
