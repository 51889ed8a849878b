"""GPU parity at the largest operand sizes: a binary64 A of more than 4 GiB
(63 600 x 8 448, ragged against every tile height), so that row offsets
from the operand base pass 2^32 bytes on the direct-to-LDS path (tile bases
are 64-bit, offsets inside a tile 32-bit), through the NN product and the
backward's transposed reads (dB = A^T dC reduces over all 63 600 rows).

The entries are integers -8..8 from the addressable generator
(``inputs.hashed_integers``), so every product is exact in binary64 and
the sampled outputs are compared bit for bit with the oracle, which gets
only the rows (columns) of A that the samples need.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import say, sample_idx

pytestmark = pytest.mark.gpu

M, K, N = 63_600, 8_448, 72
SALT_A, SALT_B, SALT_DC = 11, 12, 13


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    return G


@pytest.fixture(scope="module")
def big_a(G):
    import torch
    assert M * K * 8 > 2 ** 32
    A = torch.empty((M, K), dtype=torch.float64, device="cuda:0")
    step = 2048
    starts = list(range(0, M, step))

    def block(r0):
        return r0, inputs.hashed_integers(np.arange(r0, min(r0 + step, M)), K, SALT_A)

    with cf.ThreadPoolExecutor(8) as ex:
        for r0, rows in ex.map(block, starts):
            A[r0:r0 + rows.shape[0]].copy_(torch.from_numpy(rows))
    torch.cuda.synchronize()
    say(f"A {M} x {K} binary64 ({M * K * 8 / 2 ** 30:.2f} GiB) on the device")
    yield A
    del A
    torch.cuda.empty_cache()


def test_nn_product_operand_over_4gib(G, big_a):
    import torch
    B = inputs.hashed_integers(np.arange(K), N, SALT_B)
    C = G.gemm_plain(big_a, torch.from_numpy(B).to("cuda:0"))
    torch.cuda.synchronize()
    r, c = sample_idx(M, N, 1500, 7)
    r = np.concatenate([r, [M - 1, M - 2, 2 ** 32 // (K * 8), 2 ** 32 // (K * 8) + 1]])
    c = np.concatenate([c, [N - 1, 0, 5, N - 1]])
    rows, inv = np.unique(r, return_inverse=True)
    A_rows = inputs.hashed_integers(rows, K, SALT_A)
    ref = oracle.gemm_entries(A_rows, B, inv, c)
    got = C.cpu().numpy()[r, c]
    say(f"NN over 4 GiB: {len(r)} sampled outputs, max |C| {np.abs(ref).max():.0f}")
    assert np.array_equal(got, ref)


def test_tn_backward_operand_over_4gib(G, big_a):
    """dB = A^T dC with the >4 GiB A read transposed (M-contiguous tiles)."""
    import torch
    B = torch.zeros((K, N), dtype=torch.float64, device="cuda:0")
    dC_h = inputs.hashed_integers(np.arange(M), N, SALT_DC)
    _, dB = G.gemm_backward(big_a, B, torch.from_numpy(dC_h).to("cuda:0"), need_dA=False)
    torch.cuda.synchronize()
    g = np.random.Generator(np.random.PCG64(8))
    p = np.concatenate([g.integers(0, K, 300), [K - 1, 0]])
    j = np.concatenate([g.integers(0, N, 300), [N - 1, N - 1]])
    cols, inv = np.unique(p, return_inverse=True)
    At_cols = np.ascontiguousarray(inputs.hashed_integers(np.arange(M), cols, SALT_A).T)
    ref = oracle.gemm_entries(At_cols, dC_h, inv, j)
    got = dB.cpu().numpy()[p, j]
    say(f"TN over 4 GiB: {len(p)} sampled outputs, max |dB| {np.abs(ref).max():.0f}")
    assert np.array_equal(got, ref)
