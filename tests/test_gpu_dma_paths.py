"""GPU parity of the direct-to-LDS data path on every tile configuration.

Operands whose base and row pitch are 16-byte aligned, and whose contiguous
extent is a whole number of 16-byte vectors, go global -> LDS with transfer
instructions (K-contiguous operands XOR-swizzled per row, MN-contiguous
binary64/binary32 operands shifted per row, MN-contiguous bfloat16 operands
read back with transposing LDS reads). Every shape here is a multiple of 8 in
every dimension (aligned for all three element sizes) but ragged against the
tiles, with K below, near and well above the K-tile depth so that short and
full transfer rings and their tail waits all run.

Inputs are integers in [-8, 8]: exact in bfloat16, and every partial sum is
an integer below 2^24, so each precision, summation order and layout must
reproduce the oracle bit for bit (Section 3.1, Algorithm 1 over integers).
"""
import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import dev, say

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8, 8), (136, 200, 72), (264, 136, 200), (200, 264, 520)]


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    yield G
    G.force_tile_config(-1)


def _torch():
    import torch
    return torch


def _ints(shape, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    return g.integers(-8, 9, size=shape).astype(np.float64)


def _tdt(tname):
    torch = _torch()
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[tname]


@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_plain_nn_every_config_bit_exact(G, tname, shape):
    torch = _torch()
    m, n, k = shape
    A, B = _ints((m, k), 11 + m), _ints((k, n), 13 + n)
    ref = oracle.gemm(A, B)
    Ad, Bd = dev(A, torch, _tdt(tname)), dev(B, torch, _tdt(tname))
    for cfg, name in enumerate(G.tile_configs()):
        say(f"dma plain {tname} {shape} cfg={name}")
        G.force_tile_config(cfg)
        try:
            C = G.gemm_plain(Ad, Bd)
            torch.cuda.synchronize()
        finally:
            G.force_tile_config(-1)
        got = C.cpu().double().numpy()
        assert np.array_equal(got, ref), (tname, shape, name, np.abs(got - ref).max())


@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_backward_nt_tn_every_config_bit_exact(G, tname, shape):
    """dA = dC B^T (B read K-contiguous) and dB = A^T dC (A read
    MN-contiguous) against the oracle on explicit transposes."""
    torch = _torch()
    m, n, k = shape
    A, B, W = _ints((m, k), 17 + m), _ints((k, n), 19 + n), _ints((m, n), 23 + k)
    refA = oracle.gemm(W, np.ascontiguousarray(B.T))
    refB = oracle.gemm(np.ascontiguousarray(A.T), W)
    t = _tdt(tname)
    Ad, Bd, Wd = dev(A, torch, t), dev(B, torch, t), dev(W, torch, t)
    for cfg, name in enumerate(G.tile_configs()):
        say(f"dma backward {tname} {shape} cfg={name}")
        G.force_tile_config(cfg)
        try:
            dA, dB = G.gemm_backward(Ad, Bd, Wd)
            torch.cuda.synchronize()
        finally:
            G.force_tile_config(-1)
        assert np.array_equal(dA.cpu().double().numpy(), refA), (tname, shape, name, "dA")
        assert np.array_equal(dB.cpu().double().numpy(), refB), (tname, shape, name, "dB")


@pytest.mark.parametrize("shape", SHAPES + [(72, 56, 1000), (130, 70, 33)])
def test_split_every_config_bit_exact(G, shape):
    """Integers are their own hi plane (lo = 0), so the three-term product
    is exact; the last two shapes also exercise unaligned user operands
    (split step) and a K that is not a multiple of 8 (zero plane padding)."""
    torch = _torch()
    m, n, k = shape
    A, B = _ints((m, k), 29 + m), _ints((k, n), 31 + n)
    ref = oracle.gemm(A, B)
    Ad, Bd = dev(A, torch, torch.float32), dev(B, torch, torch.float32)
    for cfg, name in enumerate(G.tile_configs()):
        say(f"dma split {shape} cfg={name}")
        G.force_tile_config(cfg)
        try:
            C = G.gemm_split(Ad, Bd)
            torch.cuda.synchronize()
        finally:
            G.force_tile_config(-1)
        assert np.array_equal(C.cpu().double().numpy(), ref), (shape, name)


@pytest.mark.parametrize("tname", ["f64", "f32"])
@pytest.mark.parametrize("coff,pad", [((0, 0), 8), ((1, 2), 8), ((0, 1), 8), ((0, 0), 1), ((3, 0), 5)])
def test_plain_nn_output_views_every_config(G, tname, coff, pad):
    """C as a view into a larger buffer with operands on the direct-to-LDS
    path: a 16-byte aligned base and pitch (interleaved neighbouring columns
    leave in one 16-byte store), and bases or pitches that are not (element
    stores). Every config is bit-exact against the oracle and the buffer's
    margin stays untouched."""
    torch = _torch()
    m, n, k = 200, 264, 136
    A, B = _ints((m, k), 41), _ints((k, n), 43)
    ref = oracle.gemm(A, B)
    Ad, Bd = dev(A, torch, _tdt(tname)), dev(B, torch, _tdt(tname))
    r0, c0 = coff
    for cfg, name in enumerate(G.tile_configs()):
        say(f"dma plain {tname} C view {coff} pad {pad} cfg={name}")
        Cbig = torch.zeros((m + r0 + 1, n + pad), dtype=_tdt(tname), device="cuda:0")
        Cv = Cbig[r0:r0 + m, c0:c0 + n]
        G.force_tile_config(cfg)
        try:
            G.gemm_plain(Ad, Bd, Cv)
            torch.cuda.synchronize()
        finally:
            G.force_tile_config(-1)
        got = Cv.cpu().double().numpy()
        assert np.array_equal(got, ref), (tname, coff, pad, name, np.abs(got - ref).max())
        mask = torch.ones_like(Cbig, dtype=torch.bool)
        mask[r0:r0 + m, c0:c0 + n] = False
        assert torch.count_nonzero(Cbig[mask]).item() == 0, (tname, coff, pad, name)
