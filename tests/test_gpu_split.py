"""GPU parity of the three-term bfloat16 split product.

The split step is bit-exact against the oracle's split (a rounding decision
taken in the same binary32 precision on both sides); the product is within
1e-5 normwise of the binary64 oracle; integer inputs are exact.
"""
import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import dev, sample_idx, say

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    return G


def _torch():
    import torch
    return torch


@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (64, 64), (65, 63), (130, 257), (1000, 37)])
@pytest.mark.parametrize("transpose", [False, True])
def test_split_convert_bit_exact(G, shape, transpose):
    torch = _torch()
    g = np.random.Generator(np.random.PCG64(sum(shape)))
    X = g.uniform(-1, 1, size=shape).astype(np.float32)
    # include values with many significant bits, ties and large/small magnitudes
    X.flat[:: 7] *= np.float32(1e-30)
    X.flat[1:: 11] *= np.float32(1e30)
    hi, lo = G.gemm_split_convert(dev(X, torch), transpose=transpose)
    torch.cuda.synchronize()
    ohi, olo = oracle.split_bf16(X.T.copy() if transpose else X)
    assert np.array_equal(hi.cpu().numpy().view(np.uint16), ohi)
    assert np.array_equal(lo.cpu().numpy().view(np.uint16), olo)


def test_split_convert_random_bit_patterns(G):
    torch = _torch()
    g = np.random.Generator(np.random.PCG64(99))
    bits = g.integers(0, 2 ** 32, size=(512, 384), dtype=np.uint64).astype(np.uint32)
    X = bits.view(np.float32)
    X[~np.isfinite(X)] = 1.0
    X[np.abs(X) > 3e38] = 1.0            # keep x - hi finite
    for transpose in (False, True):
        hi, lo = G.gemm_split_convert(dev(X, torch), transpose=transpose)
        torch.cuda.synchronize()
        ohi, olo = oracle.split_bf16(X.T.copy() if transpose else X)
        assert np.array_equal(hi.cpu().numpy().view(np.uint16), ohi)
        assert np.array_equal(lo.cpu().numpy().view(np.uint16), olo)


@pytest.mark.parametrize("n", [1, 7, 33, 100, 257, 500])
def test_split_small_full(G, n):
    torch = _torch()
    A, B = inputs.uniform_square(n, 4400 + n, dtype=np.float32)
    C = G.gemm_split(dev(A, torch), dev(B, torch))
    torch.cuda.synchronize()
    err = oracle.relerr_fro(C.cpu().double().numpy(), oracle.gemm(A, B))
    assert err <= TOL, (n, err)


@pytest.mark.parametrize("shape", [(37, 53, 71), (129, 1, 300), (1, 257, 19), (300, 200, 1), (70, 90, 0)])
def test_split_rectangular(G, shape):
    torch = _torch()
    m, n, k = shape
    A, B = inputs.uniform_mnk(m, n, k, 5 + m, dtype=np.float32)
    C = G.gemm_split(dev(A, torch), dev(B, torch))
    torch.cuda.synchronize()
    got = C.cpu().double().numpy()
    ref = oracle.gemm(A, B)
    if k == 0:
        assert np.count_nonzero(got) == 0
    else:
        assert oracle.relerr_fro(got, ref) <= TOL


def test_split_metric_size_n2000(G):
    """The headline size: full binary64 oracle comparison at N = 2000."""
    torch = _torch()
    n = 2000
    A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    C = G.gemm_split(dev(A, torch), dev(B, torch))
    torch.cuda.synchronize()
    err = oracle.relerr_fro(C.cpu().double().numpy(), oracle.gemm_omp(A, B))
    say(f"split n=2000 relerr={err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("n", [2048, 4096, 8192])
@pytest.mark.parametrize("variant", ["uniform", "row_scaled"])
def test_split_precision_config(G, n, variant):
    torch = _torch()
    if variant == "uniform":
        A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    else:
        A, B = inputs.row_scaled(n, inputs.seed_for(2, n, variant=True))
    C = G.gemm_split(dev(A, torch), dev(B, torch))
    torch.cuda.synchronize()
    Ch = C.cpu().double().numpy()
    r, c = sample_idx(n, n, 1500, n + 2)
    err = oracle.relerr_sampled(Ch[r, c], oracle.gemm_entries(A, B, r, c))
    say(f"split n={n} {variant} sampled relerr={err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("n", [100, 1000, 2048])
def test_split_integer_bit_exact(G, n):
    """Integers in -8..8 are bfloat16 values: lo = 0 and the sum is exact."""
    torch = _torch()
    A, B = inputs.integer_square(n, inputs.seed_for(1, n, variant=True), dtype=np.float32)
    C = G.gemm_split(dev(A, torch), dev(B, torch))
    torch.cuda.synchronize()
    got = C.cpu().double().numpy()
    r, c = sample_idx(n, n, 3000, n)
    assert np.array_equal(got[r, c], oracle.gemm_entries(A, B, r, c))
    if n <= 1000:
        assert np.array_equal(got, oracle.gemm_omp(A, B))


def test_split_beats_plain_bf16_accuracy(G):
    """The split recovers binary32-level accuracy that plain bfloat16 loses."""
    torch = _torch()
    n = 512
    A, B = inputs.uniform_square(n, 12, dtype=np.float32)
    Ad, Bd = dev(A, torch), dev(B, torch)
    ref = oracle.gemm(A, B)
    e_split = oracle.relerr_fro(G.gemm_split(Ad, Bd).cpu().double().numpy(), ref)
    e_bf16 = oracle.relerr_fro(G.gemm_plain(Ad.to(torch.bfloat16), Bd.to(torch.bfloat16)).cpu().double().numpy(), ref)
    assert e_split < 1e-5 < 1e-3 < e_bf16
