"""CPU checks of the work accounting that bench.py reports: the algorithmic
flops of the truncated convolution (10 flops per valid (k, m) pair, Sec. 3.2)
and the flops the mirror-halved kernel issues (10 per pair of each kept
line), each against a brute-force count over the index grids."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _valid_pairs_brute(N):
    """All (k, m) on the N^3 index cube with n = k - m + N/2 also on it."""
    c = N // 2
    idx = np.arange(N)
    k, m = np.meshgrid(idx, idx, indexing="ij")
    ok1 = ((k - m + c) >= 0) & ((k - m + c) < N)  # one dimension
    return int(ok1.sum()) ** 3, ok1


@pytest.mark.parametrize("N", [8, 16, 24, 32])
def test_algorithmic_flops_count_every_valid_pair(N):
    pairs, _ = _valid_pairs_brute(N)
    assert pairs == 27 * N ** 6 // 64
    assert bench.conv_flops_per_cell(N) == 10.0 * pairs


@pytest.mark.parametrize("N", [4, 8, 16])
def test_executed_flops_count_each_mirrored_line_once(N):
    """For every output row (k1, k2) the lines (m1, m2) and their mirrors
    (k1 - m1 + N/2, k2 - m2 + N/2) carry the same products, so one line of
    each mirrored couple (a self-mirror line once) is summed, with all of its
    3N^2/4 valid (k3, m3) pairs: brute-force count over the 2-D line grid."""
    c = N // 2
    kept = 0
    for k1 in range(N):
        for k2 in range(N):
            classes = set()
            for m1 in range(N):
                for m2 in range(N):
                    n1, n2 = k1 - m1 + c, k2 - m2 + c
                    if 0 <= n1 < N and 0 <= n2 < N:
                        classes.add(frozenset(((m1, m2), (n1, n2))))
            kept += len(classes)
    assert bench.conv_executed_flops_per_cell(N) == 10.0 * kept * (3 * N * N // 4)


def test_executed_flops_match_the_stored_table():
    """One stored weight per kept couple: 3 545 088 weights (28.4 MB in FP64)
    at N = 16, the packed table the one-cell convolution streams."""
    assert bench.conv_executed_flops_per_cell(16) == 10.0 * 3545088
    assert bench.conv_executed_flops_per_cell(16) / bench.conv_flops_per_cell(16) == pytest.approx(0.5009, abs=1e-4)
