"""GPU checks of the loader form of the split products.

From half a 128 x 128 output tile per CU to three, gemm_split3 runs as one
launch (gemm_split on request) whose loader waves read binary32 tiles of A
and B, split every
element into bfloat16 terms (the split step's rounding: hi = bf16(x),
lo = bf16(x - hi), each to nearest even) and write the terms into the LDS
planes the compute waves multiply. Nothing goes through the workspace. On
the same tile shape (128x128k2ld) the two-step form (split step into the
workspace, then the plane product) reads the same planes in the same order,
so the two forms must agree bit for bit; the two-step form is held to the
oracle elsewhere, plane by plane. Which form ran is visible in the workspace:
the loader form leaves it untouched.
"""
import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import dev, say

pytestmark = pytest.mark.gpu

K2LD = "128x128k2ld"


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    yield G
    G.force_tile_config(-1)
    G.force_split_form(-1)


def _torch():
    import torch
    return torch


def _operands(m, n, k, seed):
    """Uniform entries with tiny and huge magnitudes, negative zeros and
    bfloat16 ties, so that every term of the split is exercised."""
    A, B = inputs.uniform_mnk(m, n, k, seed, dtype=np.float32)
    A.flat[::13] *= np.float32(2.0 ** -60)
    B.flat[5::17] *= np.float32(2.0 ** 40)
    A.flat[3::29] = np.float32(-0.0)
    B.flat[7::31] = np.float32(1.0) + np.float32(2.0 ** -9)
    return A, B


def _run(G, fn, size_fn, Ad, Bd, form, fill=0x3C):
    torch = _torch()
    m, k = Ad.shape
    n = Bd.shape[1]
    ws = torch.full((size_fn(m, n, k),), fill, dtype=torch.uint8, device="cuda:0")
    G.force_split_form(form)
    try:
        C = fn(Ad, Bd, workspace=ws)
        torch.cuda.synchronize()
    finally:
        G.force_split_form(-1)
    return C.cpu().numpy(), ws


# the headline size, K not a multiple of the 64-deep K-tile, ragged tile
# edges in M and N (multiples of 4: 16-byte rows), a single K-tile and a
# K shorter than one 16-byte half of a chunk's neighbour
SHAPES = [(2000, 2000, 2000), (1000, 36, 1004), (130, 260, 68), (257, 124, 516),
          (64, 64, 4), (300, 8, 2052)]


@pytest.mark.parametrize("name", ["gemm_split", "gemm_split3"])
@pytest.mark.parametrize("shape", SHAPES)
def test_loader_form_equals_two_step(G, name, shape):
    torch = _torch()
    m, n, k = shape
    cfg = G.tile_configs().index(K2LD)
    A, B = _operands(m, n, k, 7100 + m + n + k)
    Ad, Bd = dev(A, torch), dev(B, torch)
    fn = getattr(G, name)
    size_fn = G.gemm_split_workspace_size if name == "gemm_split" else G.gemm_split3_workspace_size
    say(f"loader form {name} m={m} n={n} k={k}")
    G.force_tile_config(cfg)
    try:
        two, ws2 = _run(G, fn, size_fn, Ad, Bd, 0)
        lod, wsl = _run(G, fn, size_fn, Ad, Bd, 2)
    finally:
        G.force_tile_config(-1)
    # the loader form ran (the two-step form writes its planes)
    assert bool((wsl == 0x3C).all())
    assert not bool((ws2 == 0x3C).all())
    assert np.array_equal(lod.view(np.uint32), two.view(np.uint32))


@pytest.mark.parametrize("name", ["gemm_split", "gemm_split3"])
def test_loader_form_headline_size_against_oracle(G, name):
    """The loader form at N = 2000 (the three-way split takes it by itself,
    the two-way split when forced): normwise error against the oracle's
    binary64 product of the binary32 inputs within 1e-5 (two-way split
    ~3.8e-6, three-way ~7e-7)."""
    torch = _torch()
    n = 2000
    A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    Ad, Bd = dev(A, torch), dev(B, torch)
    fn = getattr(G, name)
    size_fn = G.gemm_split_workspace_size if name == "gemm_split" else G.gemm_split3_workspace_size
    C, ws = _run(G, fn, size_fn, Ad, Bd, -1 if name == "gemm_split3" else 2, fill=0x77)
    assert bool((ws == 0x77).all()), "N = 2000 did not take the loader form"
    err = oracle.relerr_fro(C.astype(np.float64), oracle.gemm_omp(A, B))
    say(f"{name} N=2000 loader form: error {err:.3e}")
    assert err <= (5e-6 if name == "gemm_split" else 1e-6)


@pytest.mark.parametrize("name", ["gemm_split", "gemm_split3"])
def test_loader_form_integers_bit_exact(G, name):
    """Integer entries in [-8, 8] are exact in bfloat16 (lo terms zero) and
    every partial sum is an integer below 2^24: the product is exact."""
    torch = _torch()
    m, n, k = 600, 520, 1500
    A, B = inputs.integers((m, k), 81, np.float32, 1)[0], inputs.integers((k, n), 82, np.float32, 1)[0]
    Ad, Bd = dev(A, torch), dev(B, torch)
    fn = getattr(G, name)
    size_fn = G.gemm_split_workspace_size if name == "gemm_split" else G.gemm_split3_workspace_size
    C, ws = _run(G, fn, size_fn, Ad, Bd, 2)
    assert bool((ws == 0x3C).all())
    assert np.array_equal(C.astype(np.float64), oracle.gemm(A, B))


def test_loader_form_zero_k_and_misaligned_fallback(G):
    torch = _torch()
    # k = 0: C = 0
    Ad = torch.empty((256, 0), dtype=torch.float32, device="cuda:0")
    Bd = torch.empty((0, 256), dtype=torch.float32, device="cuda:0")
    C, _ = _run(G, G.gemm_split, G.gemm_split_workspace_size, Ad, Bd, 2)
    assert not np.any(C)
    # rows that are not 16-byte multiples: the forced loader form falls back
    # to the two-step form (which writes the workspace) with the same result
    A, B = _operands(200, 120, 130, 7300)     # k = 130: 520-byte rows of A
    Ad, Bd = dev(A, torch), dev(B, torch)
    lod, wsl = _run(G, G.gemm_split, G.gemm_split_workspace_size, Ad, Bd, 2)
    two, _ = _run(G, G.gemm_split, G.gemm_split_workspace_size, Ad, Bd, 0)
    assert not bool((wsl == 0x3C).all())
    assert np.array_equal(lod.view(np.uint32), two.view(np.uint32))
