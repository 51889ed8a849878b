"""GPU test of gemm_plain_ksplit_noalloc, the allocation-free K split: through
the C ABI, its result must equal gemm_plain_ksplit's (same kernels, chunking
and summation order, so bit for bit) on two calls in a row, the second with a
smaller product that reuses the scratch array the first one filled, and stay
within the binary64 tolerance of the oracle on sampled entries. A product
whose K split needs more than the scratch array holds is refused before any
launch and leaves C untouched."""
import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs, _lib
from gpu_util import dev, say, sample_idx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    yield G
    G.force_ksplit(-1)
    G.force_tile_config(-1)


def _sampled_err(A, B, C, seed):
    r, c = sample_idx(A.shape[0], B.shape[1], 400, seed)
    ref = oracle.gemm_entries(A, B, r, c)
    return oracle.relerr_sampled(C[r, c], ref)


@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
def test_noalloc_matches_workspace_call_twice(G, tname):
    import torch
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[tname]
    code = {"f64": G.GEMM_F64, "f32": G.GEMM_F32, "bf16": G.GEMM_BF16}[tname]
    odt = torch.float64 if tname == "f64" else torch.float32
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}[tname]
    # first a larger split product, then a smaller one (fewer rows, columns
    # and K) on the scratch the first call left behind
    for i, (m, n, k) in enumerate([(512, 512, 16384), (200, 136, 8000)]):
        need = G.gemm_plain_ksplit_workspace_size(code, m, n, k)
        say(f"noalloc {tname} call {i}: {m}x{n}x{k}, split needs {need} bytes")
        assert 0 < need <= _lib.NOALLOC_SCRATCH_BYTES
        A, B = inputs.uniform_mnk(m, n, k, 7000 + 10 * i + len(tname))
        Ad, Bd = dev(A, torch, tdt), dev(B, torch, tdt)
        C_ws = G.gemm_plain_ksplit(Ad, Bd)
        C_na = torch.full((m, n), float("nan"), dtype=odt, device="cuda:0")
        G.gemm_plain_ksplit_noalloc(Ad, Bd, C_na)
        torch.cuda.synchronize()
        got, want = C_na.cpu().numpy(), C_ws.cpu().numpy()
        assert np.array_equal(got, want), f"call {i}: differs from the workspace call"
        # oracle on the exact inputs the device saw (bf16-rounded for bf16)
        Ah = Ad.double().cpu().numpy() if tname == "bf16" else A
        Bh = Bd.double().cpu().numpy() if tname == "bf16" else B
        if tname == "f32":
            Ah, Bh = A.astype(np.float32), B.astype(np.float32)
        err = _sampled_err(Ah, Bh, got.astype(np.float64), 31 + i)
        say(f"  sampled error against the oracle {err:.3e}")
        assert err <= (1e-5 if tname == "bf16" else tol)


def test_noalloc_refuses_products_beyond_the_scratch(G):
    import torch
    m, n, k = 1024, 1024, 8192
    G.force_ksplit(20)          # 18 planes of 1024 x 1024 binary64: 144 MiB
    try:
        need = G.gemm_plain_ksplit_workspace_size(G.GEMM_F64, m, n, k)
        assert need > _lib.NOALLOC_SCRATCH_BYTES
        Ad = torch.ones((m, k), dtype=torch.float64, device="cuda:0")
        Bd = torch.ones((k, n), dtype=torch.float64, device="cuda:0")
        C = torch.full((m, n), 5.0, dtype=torch.float64, device="cuda:0")
        with pytest.raises(ValueError, match="scratch"):
            G.gemm_plain_ksplit_noalloc(Ad, Bd, C)
        torch.cuda.synchronize()
        assert bool((C == 5.0).all())
    finally:
        G.force_ksplit(-1)


def test_noalloc_unsplit_products_run_as_plain(G):
    """A product with enough tiles runs unsplit and touches no scratch."""
    import torch
    A, B = inputs.integers((600, 300), 88, np.float64, 2)[0], inputs.integers((300, 700), 89, np.float64, 2)[1]
    Ad, Bd = dev(A, torch), dev(B, torch)
    C = torch.empty((600, 700), dtype=torch.float64, device="cuda:0")
    G.gemm_plain_ksplit_noalloc(Ad, Bd, C)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), oracle.gemm(A, B))
