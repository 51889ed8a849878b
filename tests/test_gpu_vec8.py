"""GPU parity of the register path with 8-byte vector loads.

Operands whose rows are 8-byte but not 16-byte multiples (bfloat16 extents
that are multiples of 4 but not of 8, binary32 extents that are even but not
multiples of 4) cannot take the direct-to-LDS path; the register path then
moves them in 8-byte vectors (4 bfloat16 or 2 binary32 elements) instead of
single elements. Every layout (NN product, NT and TN backward) on every tile
configuration, integer inputs in [-8, 8] (exact in bfloat16, partial sums
below 2^24), compared bit for bit with the oracle; shapes ragged against the
tiles, K below and above the K-tile depths.
"""
import numpy as np
import pytest

import oracle
from gpu_util import dev, say

pytestmark = pytest.mark.gpu

# (m, n, k) with every dimension = 4 (mod 8) for bfloat16 and = 2 (mod 4)
# for binary32 (all three operands then use 8-byte vectors on every layout)
SHAPES = {"bf16": [(12, 20, 4), (132, 204, 68), (260, 100, 524)],
          "f32": [(10, 6, 2), (130, 202, 66), (258, 98, 522)]}


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    yield G
    G.force_tile_config(-1)


def _ints(shape, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    return g.integers(-8, 9, size=shape).astype(np.float64)


CASES = [(t, s) for t in ("bf16", "f32") for s in SHAPES[t]]


@pytest.mark.parametrize("tname,shape", CASES)
def test_vec8_every_layout_every_config(G, tname, shape):
    import torch
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16}[tname]
    m, n, k = shape
    A, B, W = _ints((m, k), 31 + m), _ints((k, n), 37 + n), _ints((m, n), 41 + k)
    ref = oracle.gemm(A, B)
    refA = oracle.gemm(W, np.ascontiguousarray(B.T))
    refB = oracle.gemm(np.ascontiguousarray(A.T), W)
    Ad, Bd, Wd = dev(A, torch, tdt), dev(B, torch, tdt), dev(W, torch, tdt)
    for cfg, name in enumerate(G.tile_configs()):
        say(f"vec8 {tname} {shape} cfg={name}")
        G.force_tile_config(cfg)
        try:
            C = G.gemm_plain(Ad, Bd)
            dA, dB = G.gemm_backward(Ad, Bd, Wd)
            torch.cuda.synchronize()
        finally:
            G.force_tile_config(-1)
        assert np.array_equal(C.cpu().double().numpy(), ref), (tname, shape, name)
        assert np.array_equal(dA.cpu().double().numpy(), refA), (tname, shape, name)
        assert np.array_equal(dB.cpu().double().numpy(), refB), (tname, shape, name)
