"""GPU parity of the transfer-inclusive path: operands that start in pinned
host memory, go host -> device, through gemm_plain, and back, all queued on
one stream (the one-GPU analogue of the paper's distribute / compute /
collect sequence, Section 3.1.1, Algorithms 2 and 3). The result must equal
the resident call bit for bit and the oracle within the binary64 tolerance.
"""
import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    yield G


@pytest.mark.parametrize("n", [10, 500, 2000])
def test_host_round_trip_matches_resident_and_oracle(G, n):
    import torch
    A, B = inputs.uniform_square(n, inputs.seed_for(1, n))
    Ah = torch.empty((n, n), dtype=torch.float64, pin_memory=True)
    Bh = torch.empty((n, n), dtype=torch.float64, pin_memory=True)
    Ch = torch.empty((n, n), dtype=torch.float64, pin_memory=True)
    Ah.copy_(torch.from_numpy(A))
    Bh.copy_(torch.from_numpy(B))
    Ad = torch.empty((n, n), dtype=torch.float64, device="cuda:0")
    Bd = torch.empty_like(Ad)
    Cd = torch.empty_like(Ad)
    say(f"transfer round trip n={n}")
    for _ in range(3):                     # repeated: later copies overwrite earlier ones
        Ad.copy_(Ah, non_blocking=True)
        Bd.copy_(Bh, non_blocking=True)
        G.gemm_plain(Ad, Bd, Cd)
        Ch.copy_(Cd, non_blocking=True)
    torch.cuda.synchronize()
    resident = G.gemm_plain(torch.from_numpy(A).to("cuda:0"), torch.from_numpy(B).to("cuda:0"))
    torch.cuda.synchronize()
    got = Ch.numpy().copy()
    assert np.array_equal(got, resident.cpu().numpy())
    ref = oracle.gemm_omp(A, B) if n > 500 else oracle.gemm(A, B)
    assert oracle.relerr_fro(got, ref) <= 1e-12
