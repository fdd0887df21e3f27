"""Host-side logic of bench.py (no GPU): the settled-time rule of the
time-to-tolerance figures."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402


def test_settled_time_overshoot():
    # passes through the window, overshoots, then comes back for good
    pts = [(1.0, -0.5), (2.0, -1.0000005), (3.0, -1.1), (4.0, -1.0000002), (5.0, -1.0)]
    assert bench.settled_time(pts, -1.0, 1e-6) == (4.0, 2.0)


def test_settled_time_monotone_and_edges():
    pts = [(0.1, 2.0), (0.2, 1.5), (0.3, 1.0 + 1e-12), (0.4, 1.0)]
    assert bench.settled_time(pts, 1.0, 1e-10) == (0.3, 0.3)
    # never within, or leaving the window at the end: no settled time
    assert bench.settled_time([(1.0, 3.0), (2.0, 2.0)], 1.0, 1e-6) == (None, None)
    assert bench.settled_time([(1.0, 1.0), (2.0, 2.0)], 1.0, 1e-6) == (None, 1.0)
    assert bench.settled_time([], 1.0, 1e-6) == (None, None)
    # the window is relative to |ref|
    assert bench.settled_time([(1.0, -2.0 - 1.8e-6)], -2.0, 1e-6) == (1.0, 1.0)
    assert bench.settled_time([(1.0, -2.0 - 2.2e-6)], -2.0, 1e-6) == (None, None)
