"""GPU parity of the hand-written backward dA = dC B^T, dB = A^T dC.

L = sum(W (.) (A B)) so dC = W. Checks: binary64 central differences at
N = 16 (step 1e-6; L is bilinear, so the difference quotient has no
truncation error), the oracle gradient at N = 512 (binary32) and sampled at
N = 2048, torch.autograd.gradcheck, the identities sum(A dA) = L = sum(B dB),
and bitwise equality of the transposed-operand kernels with the plain
kernel on explicitly transposed copies at the same tile shape.
"""
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
    yield G
    G.force_tile_config(-1)


def _torch():
    import torch
    return torch


def test_central_differences_fp64_n16(G):
    torch = _torch()
    n, h = 16, 1e-6
    A, B, W = inputs.uniform((n, n), inputs.seed_for(4, n), np.float64, 3)
    Ad = dev(A, torch).requires_grad_(True)
    Bd = dev(B, torch).requires_grad_(True)
    Wd = dev(W, torch)
    L = (Wd * G.matmul(Ad, Bd)).sum()
    L.backward()
    gA = Ad.grad.cpu().numpy()
    gB = Bd.grad.cpu().numpy()

    def loss(Ah, Bh):
        C = G.gemm_plain(dev(Ah, torch), dev(Bh, torch)).cpu().numpy()
        return float(np.sum(W * C))

    g = np.random.Generator(np.random.PCG64(1))
    for _ in range(10):
        i, j = (int(v) for v in g.integers(0, n, 2))
        for X, grad, which in ((A, gA, "A"), (B, gB, "B")):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, j] += h
            Xm[i, j] -= h
            if which == "A":
                fd = (loss(Xp, B) - loss(Xm, B)) / (2 * h)
            else:
                fd = (loss(A, Xp) - loss(A, Xm)) / (2 * h)
            assert abs(fd - grad[i, j]) < 1e-7, (which, i, j, fd, grad[i, j])
    _, dA, dB = oracle.loss_and_grads(A, B, W)
    assert oracle.relerr_fro(gA, dA) <= 1e-12
    assert oracle.relerr_fro(gB, dB) <= 1e-12


def test_gradcheck_fp64(G):
    torch = _torch()
    A = torch.rand((9, 7), dtype=torch.float64, device="cuda:0", requires_grad=True)
    B = torch.rand((7, 5), dtype=torch.float64, device="cuda:0", requires_grad=True)
    assert torch.autograd.gradcheck(G.matmul, (A, B), eps=1e-6, atol=1e-8)


def test_oracle_gradient_fp32_n512(G):
    torch = _torch()
    n = 512
    A, B, W = inputs.uniform((n, n), inputs.seed_for(4, n), np.float32, 3)
    dA, dB = G.gemm_backward(dev(A, torch), dev(B, torch), dev(W, torch))
    torch.cuda.synchronize()
    L, rA, rB = oracle.loss_and_grads(A, B, W)
    eA = oracle.relerr_fro(dA.cpu().double().numpy(), rA)
    eB = oracle.relerr_fro(dB.cpu().double().numpy(), rB)
    say(f"backward n=512 relerr dA={eA:.3e} dB={eB:.3e}")
    assert eA <= 1e-5 and eB <= 1e-5


def test_backward_n2048_sampled(G):
    torch = _torch()
    n = 2048
    A, B, W = inputs.uniform((n, n), inputs.seed_for(4, n), np.float32, 3)
    dA, dB = G.gemm_backward(dev(A, torch), dev(B, torch), dev(W, torch))
    torch.cuda.synchronize()
    r, c = sample_idx(n, n, 1000, 3)
    refA = oracle.gemm_entries(W, np.ascontiguousarray(B.T), r, c)
    refB = oracle.gemm_entries(np.ascontiguousarray(A.T), W, r, c)
    eA = oracle.relerr_sampled(dA.cpu().double().numpy()[r, c], refA)
    eB = oracle.relerr_sampled(dB.cpu().double().numpy()[r, c], refB)
    say(f"backward n=2048 sampled relerr dA={eA:.3e} dB={eB:.3e}")
    assert eA <= 1e-5 and eB <= 1e-5


@pytest.mark.parametrize("shape", [(33, 17, 65), (1, 40, 3), (130, 129, 1), (64, 1, 300)])
@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
def test_rectangular_and_integer_exact(G, shape, tname):
    torch = _torch()
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[tname]
    m, n, k = shape
    g = np.random.Generator(np.random.PCG64(m * n + k))
    A = g.integers(-8, 8, (m, k), endpoint=True).astype(np.float64)
    B = g.integers(-8, 8, (k, n), endpoint=True).astype(np.float64)
    W = g.integers(-8, 8, (m, n), endpoint=True).astype(np.float64)
    dA, dB = G.gemm_backward(dev(A, torch, tdt), dev(B, torch, tdt), dev(W, torch, tdt))
    torch.cuda.synchronize()
    _, rA, rB = oracle.loss_and_grads(A, B, W)
    assert np.array_equal(dA.cpu().double().numpy(), rA)
    assert np.array_equal(dB.cpu().double().numpy(), rB)


def test_skip_one_gradient(G):
    torch = _torch()
    A, B, W = inputs.uniform((40, 40), 5, np.float64, 3)
    dA, dB = G.gemm_backward(dev(A, torch), dev(B, torch), dev(W, torch), need_dB=False)
    assert dB is None and dA is not None
    dA, dB = G.gemm_backward(dev(A, torch), dev(B, torch), dev(W, torch), need_dA=False)
    assert dA is None and dB is not None


def test_euler_identities_fp64(G):
    torch = _torch()
    A, B, W = inputs.uniform((64, 64), 6, np.float64, 3)
    dA, dB = G.gemm_backward(dev(A, torch), dev(B, torch), dev(W, torch))
    L = float(np.sum(W * oracle.gemm(A, B)))
    assert abs(np.sum(A * dA.cpu().numpy()) - L) < 1e-10
    assert abs(np.sum(B * dB.cpu().numpy()) - L) < 1e-10


@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
def test_transposed_tiles_equal_plain_on_transposed_copies(G, tname):
    torch = _torch()
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[tname]
    n = 300
    A, B, W = inputs.uniform((n, n), 8, np.float64, 3)
    Ad, Bd, Wd = dev(A, torch, tdt), dev(B, torch, tdt), dev(W, torch, tdt)
    for cfg in range(len(G.tile_configs())):
        G.force_tile_config(cfg)
        dA, dB = G.gemm_backward(Ad, Bd, Wd)
        pA = G.gemm_plain(Wd, Bd.t().contiguous())
        pB = G.gemm_plain(Ad.t().contiguous(), Wd)
        torch.cuda.synchronize()
        G.force_tile_config(-1)
        assert torch.equal(dA, pA), cfg
        assert torch.equal(dB, pB), cfg


def test_backward_bf16_n3072_large_tiles(G):
    """bf16 backward where the 16-bit rule takes the 256 x 256 tile for the
    transposed-operand products (576 tiles of 128 x 128): sampled entries
    against the binary64 oracle of the rounded inputs."""
    torch = _torch()
    n = 3072
    A, B, W = inputs.uniform((n, n), inputs.seed_for(4, n), np.float32, 3)
    Ab, Bb, Wb = (dev(X, torch).to(torch.bfloat16) for X in (A, B, W))
    dA, dB = G.gemm_backward(Ab, Bb, Wb)
    torch.cuda.synchronize()
    Ar, Br, Wr = (oracle.bf16_to_f32(oracle.bf16_rne(X)) for X in (A, B, W))
    r, c = sample_idx(n, n, 600, 5)
    refA = oracle.gemm_entries(Wr, np.ascontiguousarray(Br.T), r, c)
    refB = oracle.gemm_entries(np.ascontiguousarray(Ar.T), Wr, r, c)
    eA = oracle.relerr_sampled(dA.cpu().double().numpy()[r, c], refA)
    eB = oracle.relerr_sampled(dB.cpu().double().numpy()[r, c], refB)
    say(f"bf16 backward n={n} sampled relerr dA={eA:.3e} dB={eB:.3e}")
    assert eA <= 1e-5 and eB <= 1e-5


def test_autograd_bf16_and_fp32_through_gemmfn(G):
    torch = _torch()
    n = 256
    A, B, W = inputs.uniform((n, n), 9, np.float32, 3)
    Ad = dev(A, torch).requires_grad_(True)
    Bd = dev(B, torch).requires_grad_(True)
    (dev(W, torch) * G.matmul(Ad, Bd)).sum().backward()
    _, rA, rB = oracle.loss_and_grads(A, B, W)
    assert oracle.relerr_fro(Ad.grad.cpu().double().numpy(), rA) <= 1e-5
    assert oracle.relerr_fro(Bd.grad.cpu().double().numpy(), rB) <= 1e-5
