"""GPU parity of the three-way bfloat16 split product (six terms).

The split step is bit-exact against the oracle's three-way split (each
rounding decision taken in binary32 on both sides); the product is within
1e-5 normwise of the binary64 oracle and, because the dropped terms are
~2^-24 |A||B|, within a small factor of plain binary32 and well below the
two-way split; integer inputs are exact on every tile configuration.
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
    yield G
    G.force_tile_config(-1)


def _torch():
    import torch
    return torch


@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (64, 64), (65, 63), (130, 257), (1000, 37)])
@pytest.mark.parametrize("transpose", [False, True])
def test_split3_convert_bit_exact(G, shape, transpose):
    torch = _torch()
    g = np.random.Generator(np.random.PCG64(7 + sum(shape)))
    X = g.uniform(-1, 1, size=shape).astype(np.float32)
    X.flat[:: 7] *= np.float32(1e-30)
    X.flat[1:: 11] *= np.float32(1e30)
    got = G.gemm_split3_convert(dev(X, torch), transpose=transpose)
    torch.cuda.synchronize()
    ref = oracle.split3_bf16(X.T.copy() if transpose else X)
    for plane, r in zip(got, ref):
        assert np.array_equal(plane.cpu().numpy().view(np.uint16), r)


def test_split3_convert_random_bit_patterns(G):
    torch = _torch()
    g = np.random.Generator(np.random.PCG64(98))
    bits = g.integers(0, 2 ** 32, size=(384, 256), dtype=np.uint64).astype(np.uint32)
    X = bits.view(np.float32)
    X[~np.isfinite(X)] = 1.0
    X[np.abs(X) > 3e38] = 1.0
    for transpose in (False, True):
        got = G.gemm_split3_convert(dev(X, torch), transpose=transpose)
        torch.cuda.synchronize()
        ref = oracle.split3_bf16(X.T.copy() if transpose else X)
        for plane, r in zip(got, ref):
            assert np.array_equal(plane.cpu().numpy().view(np.uint16), r)


@pytest.mark.parametrize("n", [1, 7, 33, 100, 257, 500])
def test_split3_small_full(G, n):
    torch = _torch()
    A, B = inputs.uniform_square(n, 4500 + n, dtype=np.float32)
    C = G.gemm_split3(dev(A, torch), dev(B, torch))
    torch.cuda.synchronize()
    err = oracle.relerr_fro(C.cpu().double().numpy(), oracle.gemm(A, B))
    assert err <= TOL, (n, err)


@pytest.mark.parametrize("shape", [(37, 53, 71), (129, 1, 300), (1, 257, 19), (300, 200, 1), (70, 90, 0)])
def test_split3_rectangular(G, shape):
    torch = _torch()
    m, n, k = shape
    A, B = inputs.uniform_mnk(m, n, k, 15 + m, dtype=np.float32)
    C = G.gemm_split3(dev(A, torch), dev(B, torch))
    torch.cuda.synchronize()
    got = C.cpu().double().numpy()
    if k == 0:
        assert np.count_nonzero(got) == 0
    else:
        assert oracle.relerr_fro(got, oracle.gemm(A, B)) <= TOL


def test_split3_n2000_accuracy_ladder(G):
    """At the headline size: three-way split within 1e-5 of the binary64
    oracle, at most twice the plain binary32 error, and below the two-way
    split's error."""
    torch = _torch()
    n = 2000
    A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    Ad, Bd = dev(A, torch), dev(B, torch)
    ref = oracle.gemm_omp(A, B)
    e3 = oracle.relerr_fro(G.gemm_split3(Ad, Bd).cpu().double().numpy(), ref)
    e2 = oracle.relerr_fro(G.gemm_split(Ad, Bd).cpu().double().numpy(), ref)
    e32 = oracle.relerr_fro(G.gemm_plain(Ad, Bd).cpu().double().numpy(), ref)
    say(f"n=2000 relerr split3={e3:.3e} split={e2:.3e} fp32={e32:.3e}")
    assert e3 <= TOL
    assert e3 <= 2.0 * e32
    assert e3 < 0.5 * e2


@pytest.mark.parametrize("n", [2048, 4096, 8192])
@pytest.mark.parametrize("variant", ["uniform", "row_scaled"])
def test_split3_precision_config(G, n, variant):
    torch = _torch()
    if variant == "uniform":
        A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    else:
        A, B = inputs.row_scaled(n, inputs.seed_for(2, n, variant=True))
    C = G.gemm_split3(dev(A, torch), dev(B, torch))
    torch.cuda.synchronize()
    Ch = C.cpu().double().numpy()
    r, c = sample_idx(n, n, 1500, n + 3)
    err = oracle.relerr_sampled(Ch[r, c], oracle.gemm_entries(A, B, r, c))
    say(f"split3 n={n} {variant} sampled relerr={err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("n", [100, 1000])
def test_split3_integer_bit_exact_every_config(G, n):
    """Integers in -8..8 are bfloat16 values (mid = lo = 0): exact sums."""
    torch = _torch()
    A, B = inputs.integer_square(n, inputs.seed_for(1, n, variant=True), dtype=np.float32)
    Ad, Bd = dev(A, torch), dev(B, torch)
    ref = oracle.gemm_omp(A, B)
    for cfg, name in enumerate(G.tile_configs()):
        G.force_tile_config(cfg)
        try:
            got = G.gemm_split3(Ad, Bd).cpu().double().numpy()
        finally:
            G.force_tile_config(-1)
        assert np.array_equal(got, ref), (n, name)
