"""The allocation-free POD projection (pcfv_pod_project_noalloc) against the
workspace entry point pcfv_pod_project: same kernels and split of the sum, so
the coefficients must agree bit for bit, on two calls in a row (the second
smaller, reusing the device-resident scratch the first one left behind)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(m, n, r, seed):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.randn((m, n), dtype=torch.float64, generator=g).to("cuda:0").contiguous()
    mean = torch.randn(n, dtype=torch.float64, generator=g).to("cuda:0").contiguous()
    basis = torch.randn((r, n), dtype=torch.float64, generator=g).to("cuda:0").contiguous()
    return X, mean, basis


def test_noalloc_projection_matches_workspace_entry_point():
    import torch
    from paper_2306_00165_amd import pcfv
    for (m, n, r, seed) in [(64, 100000, 32, 1), (16, 30000, 8, 2)]:
        print(f"[gpu] no-alloc POD projection m={m} n={n} r={r}", flush=True)
        assert 1 < pcfv._lib.pcfv_pod_project_scratch_bytes(m, n, r) <= pcfv.NOALLOC_SCRATCH_BYTES
        X, mean, basis = _case(m, n, r, seed)
        want = pcfv.pod_project(X, mean, basis)
        coef = torch.full((m, r), float("nan"), dtype=torch.float64, device="cuda:0")
        got = pcfv.pod_project_noalloc(X, mean, basis, coef)
        torch.cuda.synchronize()
        assert got.data_ptr() == coef.data_ptr()
        assert torch.equal(got, want)
        ref = ((X - mean).cpu().numpy() @ basis.cpu().numpy().T)
        assert np.abs(got.cpu().numpy() - ref).max() <= 1e-11 * np.abs(ref).max()


def test_noalloc_projection_rejects_sizes_beyond_its_scratch():
    import torch
    from paper_2306_00165_amd import pcfv
    m, n, r = 256, 1_000_000, 256
    assert pcfv._lib.pcfv_pod_project_scratch_bytes(m, n, r) > pcfv.NOALLOC_SCRATCH_BYTES
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    p = pcfv._ptr(dummy)
    st = pcfv._lib.pcfv_pod_project_noalloc(pcfv._cuda_stream_ptr(torch, dummy.device), p, m, n, r, p, p, p)
    assert st == pcfv.ENOMEM
    assert b"scratch" in pcfv._lib.pcfv_last_error(None)
