"""GPU checks of the split products' one-launch form.

For small products whose A and B allow 16-byte direct-to-LDS transfers
(16-byte aligned base and row pitch, k and n multiples of 4, k <= 1024, at
most one 128 x 128 output tile per two CUs), gemm_split and gemm_split3
split each binary32 fragment into bfloat16 terms in registers, right before
the MFMAs, instead of writing the terms to planes in a separate split step.
Both forms take the same rounding decisions and run the same MFMAs in the
same order, so their results must agree bit for bit; operands with a row
pitch that is not a multiple of 16 bytes take the two-step form, which the
tests use as the reference (it is itself held to the oracle elsewhere).
Each case first asserts which form the library reports it will take.
"""
import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import dev, say

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


def _pitched(X, torch):
    """The same matrix with a row pitch of cols + 1 elements (not a multiple
    of 16 bytes when cols is a multiple of 4): forces the two-step form."""
    r, c = X.shape
    buf = torch.zeros((r, c + 1), dtype=torch.float32, device="cuda:0")
    buf[:, :c] = dev(X, torch)
    return buf[:, :c]


def _operands(m, n, k, seed):
    """Uniform entries with a sprinkling of very small and very large
    magnitudes and negative zeros (every term of the split nonzero for most
    elements, some exactly representable ones)."""
    A, B = inputs.uniform_mnk(m, n, k, seed, dtype=np.float32)
    A.flat[::13] *= np.float32(2.0 ** -60)
    B.flat[5::17] *= np.float32(2.0 ** 40)
    A.flat[3::29] = np.float32(-0.0)
    B.flat[7::31] = np.float32(0.75)
    return A, B


SHAPES = [(8, 8, 8), (64, 64, 64), (130, 260, 300), (257, 124, 516), (1000, 1000, 1000),
          (33, 2000, 68), (1024, 1024, 1024)]


@pytest.mark.parametrize("name", ["gemm_split", "gemm_split3"])
@pytest.mark.parametrize("shape", SHAPES)
def test_fused_equals_two_step(G, name, shape):
    torch = _torch()
    m, n, k = shape
    A, B = _operands(m, n, k, 900 + m + n + k)
    fn = getattr(G, name)
    Ad, Bd, Ap = dev(A, torch), dev(B, torch), _pitched(A, torch)
    assert G.split_one_launch(Ad, Bd) and not G.split_one_launch(Ap, Bd)
    fused = fn(Ad, Bd)
    two_step = fn(Ap, Bd)
    torch.cuda.synchronize()
    f, t = fused.cpu().numpy(), two_step.cpu().numpy()
    assert np.array_equal(f.view(np.uint32), t.view(np.uint32)), (name, shape)
    ref = oracle.gemm(A, B)
    err = oracle.relerr_fro(f.astype(np.float64), ref)
    assert err <= 1e-5, (name, shape, err)


@pytest.mark.parametrize("name", ["gemm_split", "gemm_split3"])
def test_fused_equals_two_step_every_config(G, name):
    torch = _torch()
    m, n, k = 200, 264, 520
    A, B = _operands(m, n, k, 77)
    fn = getattr(G, name)
    Ad, Bd, Ap = dev(A, torch), dev(B, torch), _pitched(A, torch)
    assert G.split_one_launch(Ad, Bd)
    for cfg, cname in enumerate(G.tile_configs()):
        G.force_tile_config(cfg)
        try:
            f = fn(Ad, Bd).cpu().numpy()
            t = fn(Ap, Bd).cpu().numpy()
        finally:
            G.force_tile_config(-1)
        assert np.array_equal(f.view(np.uint32), t.view(np.uint32)), (name, cname)


def test_form_rule(G):
    """Which form the library takes: one launch for aligned products with a
    short K loop that leave most CUs idle, and for aligned products from half
    a 128 x 128 tile per CU to one per CU (one round of the loader-wave tile)."""
    torch = _torch()
    z = lambda r, c: torch.zeros((r, c), dtype=torch.float32, device="cuda:0")
    assert G.split_one_launch(z(1000, 1000), z(1000, 1000))
    assert G.split_one_launch(z(1024, 1024), z(1024, 1024))
    assert not G.split_one_launch(z(1200, 1200), z(1200, 1200))      # long K, a few tiles
    assert G.split_one_launch(z(1500, 1500), z(1500, 1500))          # 144 tiles
    assert G.split_one_launch(z(2000, 2000), z(2000, 2000))          # 256 tiles
    assert G.split_one_launch(z(2048, 2048), z(2048, 2048))          # 256 tiles
    assert not G.split_one_launch(z(2200, 2200), z(2200, 2200))      # a second round
    assert not G.split_one_launch(z(64, 2048), z(2048, 64))          # long K loop
    assert not G.split_one_launch(z(64, 63), z(63, 64))              # k not a multiple of 4
    assert not G.split_one_launch(z(64, 64), z(64, 62))              # n not a multiple of 4
    assert not G.split_one_launch(z(64, 65)[:, 1:], z(64, 64))       # misaligned base


@pytest.mark.parametrize("name", ["gemm_split", "gemm_split3"])
def test_fused_largest_one_launch_size(G, name):
    """The largest square size of the one-launch form, on the headline input
    recipe, against the full binary64 oracle product."""
    torch = _torch()
    n = 1024
    A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    Ad, Bd = dev(A, torch), dev(B, torch)
    assert G.split_one_launch(Ad, Bd)
    f = getattr(G, name)(Ad, Bd).cpu().numpy().astype(np.float64)
    err = oracle.relerr_fro(f, oracle.gemm_omp(A, B))
    say(f"{name} one launch n={n} relerr={err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("n", [1500, 2000])
def test_fused_loader_tile(G, n):
    """The one-launch two-way split on the loader-wave tile (N = 1500, 144
    tiles; N = 2000, 256): bit for bit the two steps on the same tile, and the
    full binary64 oracle product within 1e-5."""
    torch = _torch()
    A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    Ad, Bd, Ap = dev(A, torch), dev(B, torch), _pitched(A, torch)
    assert G.split_one_launch(Ad, Bd) and not G.split_one_launch(Ap, Bd)
    f = G.gemm_split(Ad, Bd).cpu().numpy()
    t = G.gemm_split(Ap, Bd).cpu().numpy()
    assert np.array_equal(f.view(np.uint32), t.view(np.uint32))
    err = oracle.relerr_fro(f.astype(np.float64), oracle.gemm_omp(A, B))
    say(f"gemm_split one launch n={n} relerr={err:.3e}")
    assert err <= 1e-5


def test_fused_zero_k_and_empty(G):
    torch = _torch()
    A = torch.zeros((40, 0), dtype=torch.float32, device="cuda:0")
    B = torch.zeros((0, 36), dtype=torch.float32, device="cuda:0")
    C = torch.full((40, 36), 5.0, dtype=torch.float32, device="cuda:0")
    for fn in (G.gemm_split, G.gemm_split3):
        C.fill_(5.0)
        fn(A, B, C)
        torch.cuda.synchronize()
        assert int(torch.count_nonzero(C)) == 0


@pytest.mark.parametrize("name", ["gemm_split", "gemm_split3"])
def test_one_launch_leaves_workspace_untouched(G, name):
    """The one-launch form needs no planes: the caller's workspace keeps its
    contents; the two-step form writes its planes there."""
    torch = _torch()
    m, n, k = 96, 128, 200
    A, B = inputs.uniform_mnk(m, n, k, 31, dtype=np.float32)
    Ad, Bd = dev(A, torch), dev(B, torch)
    size = getattr(G, name + "_workspace_size")(m, n, k)
    ws = torch.full((size,), 0xA5, dtype=torch.uint8, device="cuda:0")
    assert G.split_one_launch(Ad, Bd)
    getattr(G, name)(Ad, Bd, None, ws)
    torch.cuda.synchronize()
    assert bool((ws == 0xA5).all())
    getattr(G, name)(_pitched(A, torch), Bd, None, ws)
    torch.cuda.synchronize()
    assert not bool((ws == 0xA5).all())
