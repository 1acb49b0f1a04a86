"""The Indexing step alone (stable counting sort building LCR, Sec. 1.1 and
1.4) on the GPU against the oracle's counting sort: bit-exact, including
empty and ragged inputs, one, two and three 11-bit passes."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


CASES = [
    # n, nbins, near_sorted, dead_fraction
    (0, 1, False, 0.0),
    (1, 1, False, 0.0),
    (63, 2, False, 0.3),
    (64, 5, False, 0.0),
    (65, 5, True, 0.0),
    (16384 + 17, 1025, True, 0.01),          # one tile plus a ragged tail
    (1_000_003, 1025, True, 0.02),           # many tiles, single pass
    (200_000, 2048, False, 0.0),             # largest single-pass bin count
    (200_000, 2049, False, 0.1),             # smallest two-pass bin count
    (500_000, 16385, True, 0.0),             # the channel grid's bins
    (300_000, 2_000_001, False, 0.0),        # the 3-D grid's bins, two passes
    (100_000, (1 << 22) + 1, False, 0.05),   # three passes
]


@pytest.mark.parametrize("n,nbins,near,dead", CASES)
def test_counting_sort_matches_oracle(dsmc_gpu, oracle_lib, n, nbins, near, dead):
    import torch
    keys = W.random_cells(n, nbins, seed=n + nbins, near_sorted=near, jump=40, dead_fraction=dead)
    if n:
        assert keys.max() < nbins
    lcr_ref, start_ref, _ = oracle_lib.counting_sort(keys, nbins)
    kt = torch.from_numpy(keys).cuda()
    lcr, start = dsmc_gpu.counting_sort(kt, nbins)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(lcr.cpu().numpy(), lcr_ref)
    np.testing.assert_array_equal(start.cpu().numpy().astype(np.int64), start_ref)


def test_counting_sort_repeatable(dsmc_gpu):
    import torch
    keys = torch.from_numpy(W.random_cells(777_777, 4097, seed=5)).cuda()
    a, sa = dsmc_gpu.counting_sort(keys, 4097)
    b, sb = dsmc_gpu.counting_sort(keys, 4097)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(sa, sb)
