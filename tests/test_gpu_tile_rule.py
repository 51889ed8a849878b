"""GPU parity at the sizes where the 16-bit tile rule takes the loader-wave
tile in more than one round of workgroups (N = 1200, 2600) or the 256 x 256
tile (N = 3000), or the three-way loader form beyond five tiles per CU: bf16
(kernel-only, against the binary64 oracle of the rounded inputs), the
two-way split and the three-way split (against the binary64 oracle of the
binary32 inputs), sampled entries."""
import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import dev, sample_idx, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    return G


def _torch():
    import torch
    return torch


@pytest.mark.parametrize("n", [1200, 2600, 3000])
def test_bf16_and_split_loader_tile_rounds(G, n):
    torch = _torch()
    A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    Ad, Bd = dev(A, torch), dev(B, torch)
    r, c = sample_idx(n, n, 800, n + 3)
    ref = oracle.gemm_entries(A, B, r, c)
    Ar = oracle.bf16_to_f32(oracle.bf16_rne(A))
    Br = oracle.bf16_to_f32(oracle.bf16_rne(B))
    ref_r = oracle.gemm_entries(Ar, Br, r, c)
    Cb = G.gemm_plain(Ad.to(torch.bfloat16), Bd.to(torch.bfloat16)).cpu().double().numpy()
    err_b = oracle.relerr_sampled(Cb[r, c], ref_r)
    Cs = G.gemm_split(Ad, Bd).cpu().double().numpy()
    err_s = oracle.relerr_sampled(Cs[r, c], ref)
    say(f"n={n} bf16 kernel-only relerr={err_b:.3e} split relerr={err_s:.3e}")
    assert err_b <= 1e-5
    assert err_s <= 1e-5


def test_split3_loader_form_n5000(G):
    torch = _torch()
    n = 5000
    A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    Ad, Bd = dev(A, torch), dev(B, torch)
    C = G.gemm_split3(Ad, Bd).cpu().double().numpy()
    r, c = sample_idx(n, n, 600, n + 5)
    err = oracle.relerr_sampled(C[r, c], oracle.gemm_entries(A, B, r, c))
    say(f"split3 n={n} relerr={err:.3e}")
    assert err <= 1e-5
