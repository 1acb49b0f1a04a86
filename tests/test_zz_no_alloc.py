"""The allocation-free counting sort (dsmc_counting_sort_noalloc, workspace
in the library's static device array) against the same sort with a caller
workspace (dsmc_counting_sort) and the oracle's counting sort: bit-exact on
two calls in a row, the second smaller, so that the second runs over the
first call's leftovers in the shared array."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _with_workspace(P, kt, nbins):
    import torch
    n = kt.numel()
    lcr = torch.empty(max(n, 1), dtype=torch.int32, device=kt.device)
    start = torch.empty(nbins + 1, dtype=torch.int32, device=kt.device)
    wb = P.dsmc_counting_sort_bytes(n, nbins)
    work = torch.empty(wb + 256, dtype=torch.uint8, device=kt.device)
    wp = (work.data_ptr() + 255) & ~255
    P.dsmc_counting_sort(kt.data_ptr(), n, nbins, lcr.data_ptr(), start.data_ptr(), wp, wb,
                         torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return lcr[:n].cpu().numpy(), start.cpu().numpy()


def _no_alloc(P, kt, nbins):
    import torch
    n = kt.numel()
    # poisoned outputs: every entry must be written
    lcr = torch.full((max(n, 1),), -7, dtype=torch.int32, device=kt.device)
    start = torch.full((nbins + 1,), -7, dtype=torch.int32, device=kt.device)
    P.dsmc_counting_sort_noalloc(kt.data_ptr(), n, nbins, lcr.data_ptr(), start.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return lcr[:n].cpu().numpy(), start.cpu().numpy()


# (n, nbins, near_sorted, dead fraction): a two-pass sort of 1.5M keys (about
# 19 MB of the 32 MiB array), then a smaller single-pass sort
CALLS = [(1_500_000, 4097, True, 0.02), (70_001, 1025, False, 0.1)]


def test_no_alloc_sort_equals_workspace_sort_twice(dsmc_gpu, oracle_lib):
    import torch
    P = dsmc_gpu
    for n, nbins, near, dead in CALLS:
        assert P.dsmc_counting_sort_bytes(n, nbins) <= P.SORT_SCRATCH_BYTES
        keys = W.random_cells(n, nbins, seed=n + 3 * nbins, near_sorted=near, jump=40,
                              dead_fraction=dead)
        assert keys.min() >= 0 and keys.max() < nbins
        print(f"no-alloc sort: n={n} nbins={nbins}", flush=True)
        kt = torch.from_numpy(keys).cuda()
        lcr_w, start_w = _with_workspace(P, kt, nbins)
        lcr_s, start_s = _no_alloc(P, kt, nbins)
        np.testing.assert_array_equal(lcr_s, lcr_w)
        np.testing.assert_array_equal(start_s, start_w)
        lcr_o, start_o, _ = oracle_lib.counting_sort(keys, nbins)
        np.testing.assert_array_equal(lcr_s, lcr_o)
        np.testing.assert_array_equal(start_s.astype(np.int64), start_o)


def test_no_alloc_sort_rejects_oversize_before_launch(dsmc_gpu):
    import torch
    P = dsmc_gpu
    n, nbins = 4_000_000, 4097   # 12 B per key of multi-pass buffers alone: 48 MB
    assert P.dsmc_counting_sort_bytes(n, nbins) > P.SORT_SCRATCH_BYTES
    keys = torch.zeros(n, dtype=torch.int32, device="cuda")
    lcr = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    start = torch.full((nbins + 1,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(P.DsmcError) as e:
        P.dsmc_counting_sort_noalloc(keys.data_ptr(), n, nbins, lcr.data_ptr(), start.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
    assert e.value.status == -2
    torch.cuda.synchronize()
    assert int(lcr.min()) == -7 and int(lcr.max()) == -7   # nothing was launched
