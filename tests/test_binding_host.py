"""Host-only checks of the Python binding's argument checks: a caller's
output or workspace of the wrong shape, dtype, device or layout is rejected
before anything reaches the library (CPU only; no launch happens)."""
import pytest
import torch

import paper_1012_2273_amd as G
from paper_1012_2273_amd import GemmArgError


def _ab(dtype, m=6, n=5, k=4):
    return torch.zeros((m, k), dtype=dtype), torch.zeros((k, n), dtype=dtype)


@pytest.mark.parametrize("dtype,out", [(torch.float64, torch.float64),
                                       (torch.float32, torch.float32),
                                       (torch.bfloat16, torch.float32)])
def test_plain_rejects_bad_output(dtype, out):
    A, B = _ab(dtype)
    with pytest.raises(GemmArgError, match="shape"):
        G.gemm_plain(A, B, torch.zeros((5, 6), dtype=out))
    with pytest.raises(GemmArgError, match="dtype"):
        # bf16 inputs write binary32: a bf16 C would be half the size written
        G.gemm_plain(A, B, torch.zeros((6, 5), dtype=torch.bfloat16 if out != torch.bfloat16
                                       else torch.float64))
    with pytest.raises(GemmArgError, match="shape"):
        G.gemm_plain_ksplit(A, B, torch.zeros((6, 4), dtype=out))


def test_plain_rejects_output_on_another_device():
    A, B = _ab(torch.float64)
    C = torch.zeros((6, 5), dtype=torch.float64, device="meta")
    with pytest.raises(GemmArgError, match="device|is on"):
        G.gemm_plain(A, B, C)


@pytest.mark.parametrize("fn", [G.gemm_split, G.gemm_split3])
def test_split_rejects_bad_output_and_workspace(fn):
    A, B = _ab(torch.float32)
    with pytest.raises(GemmArgError, match="shape"):
        fn(A, B, torch.zeros((6, 6), dtype=torch.float32))
    with pytest.raises(GemmArgError, match="dtype"):
        fn(A, B, torch.zeros((6, 5), dtype=torch.float64))
    # a host workspace (a host pointer must never reach the kernels)
    with pytest.raises(GemmArgError, match="workspace"):
        fn(A, B, torch.zeros((6, 5), dtype=torch.float32), torch.zeros(4096, dtype=torch.uint8))


def test_ksplit_rejects_host_workspace():
    A, B = _ab(torch.float64)
    with pytest.raises(GemmArgError, match="workspace"):
        G.gemm_plain_ksplit(A, B, torch.zeros((6, 5), dtype=torch.float64),
                            torch.zeros(64, dtype=torch.uint8))


def test_grouped_rejects_bad_outputs():
    A, B = _ab(torch.float64)
    with pytest.raises(GemmArgError, match="shape"):
        G.gemm_grouped([A], [B], [torch.zeros((5, 5), dtype=torch.float64)])
    with pytest.raises(GemmArgError, match="dtype"):
        G.GroupedPlan([A], [B], [torch.zeros((6, 5), dtype=torch.float32)])
