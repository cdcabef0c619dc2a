"""tabnet_mask_stats_noalloc (the entry point for callers that cannot allocate) against
tabnet_mask_stats with a caller workspace: identical results, bit for bit, on two calls in
a row, the second with a smaller input, through the C ABI."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _masks(rows, D, seed):
    g = torch.Generator().manual_seed(seed)
    m = torch.rand((rows, D), generator=g, dtype=torch.float32)
    m = m / m.sum(1, keepdim=True)
    return m.cuda()


def _with_workspace(lib, m):
    B, D = m.shape
    mean = torch.empty(D, dtype=torch.float64, device=m.device)
    var = torch.empty(D, dtype=torch.float64, device=m.device)
    ws = torch.empty(lib.tabnet_mask_stats_workspace_bytes(B, D), dtype=torch.uint8, device=m.device)
    st = lib.tabnet_mask_stats(m.data_ptr(), B, D, mean.data_ptr(), var.data_ptr(), ws.data_ptr(), ws.numel(), None)
    assert st == 0
    return mean, var


def _noalloc(lib, m):
    B, D = m.shape
    mean = torch.full((D,), float("nan"), dtype=torch.float64, device=m.device)
    var = torch.full((D,), float("nan"), dtype=torch.float64, device=m.device)
    st = lib.tabnet_mask_stats_noalloc(m.data_ptr(), B, D, mean.data_ptr(), var.data_ptr(), None)
    assert st == 0, lib.tabnet_last_error()
    return mean, var


def test_noalloc_matches_workspace_entry_twice_second_smaller():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_19689_amd import tabnet
    lib = tabnet.lib()
    cases = [(65536, 108, 1), (1000, 35, 2)]       # the second call is smaller
    print("noalloc cases", cases, flush=True)
    for rows, D, seed in cases:
        m = _masks(rows, D, seed)
        assert lib.tabnet_mask_stats_workspace_bytes(rows, D) <= lib.tabnet_mask_stats_noalloc_max_bytes()
        a_mean, a_var = _noalloc(lib, m)
        b_mean, b_var = _with_workspace(lib, m)
        torch.cuda.synchronize()
        assert torch.equal(a_mean, b_mean) and torch.equal(a_var, b_var)
        ref = m.double().cpu()
        np.testing.assert_allclose(a_mean.cpu().numpy(), ref.mean(0).numpy(), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(a_var.cpu().numpy(), ref.var(0, unbiased=False).numpy(), rtol=1e-9, atol=1e-15)


def test_noalloc_rejects_oversize_and_null():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_19689_amd import tabnet
    lib = tabnet.lib()
    m = _masks(64, 8, 3)
    mean = torch.empty(8, dtype=torch.float64, device=m.device)
    var = torch.empty(8, dtype=torch.float64, device=m.device)
    # 1024 blocks x 2 x 4096 columns x 8 bytes = 64 MiB of partial sums: beyond the scratch
    big_rows, big_D = 1 << 22, 4096
    assert lib.tabnet_mask_stats_workspace_bytes(big_rows, big_D) > lib.tabnet_mask_stats_noalloc_max_bytes()
    assert lib.tabnet_mask_stats_noalloc(m.data_ptr(), big_rows, big_D, mean.data_ptr(), var.data_ptr(),
                                         None) == tabnet.E_INVALID
    assert b"exceeds" in lib.tabnet_last_error()
    assert lib.tabnet_mask_stats_noalloc(None, 64, 8, mean.data_ptr(), var.data_ptr(), None) == tabnet.E_INVALID
