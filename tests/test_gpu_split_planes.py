"""GPU parity of the split step the split products run (the operand planes).

gemm_split and gemm_split3 (two-step form) split both operands in one launch
into the caller's workspace and then multiply the planes. The header fixes the
workspace layout, so the planes can be read back and compared bit for bit with
the oracle's split of the same binary32 values (the rounding decision of each
term is taken in binary32 on both sides):

  kp  = k rounded up to 8, ldp = kp rounded up to 64 (elements of 2 bytes)
  A planes (hi, lo[, mid before lo]): m rows of ldp, row-major, A[r][c] at r*ldp + c
  B planes: n rows of ldp, B transposed, B[c][r] at r*ldp + c
  each plane starts on a 256-byte boundary, the A planes first
  columns [k, kp) of every plane row hold zeros

A misplaced lo element changes the product by ~2^-16 of one term and hides
below the 1e-5 normwise bar, which is why the planes are checked directly.
"""
import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import dev, say

pytestmark = pytest.mark.gpu

# (m, n, k): the headline size, and ragged shapes whose k is not a multiple
# of 8 (zero padding), whose n is not a multiple of the 64-wide split tile,
# and a single-column K
SHAPES = [(2000, 2000, 2000), (1000, 37, 1003), (130, 257, 61), (65, 9, 1)]


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    # the split step writes the planes only in the two-step form (larger
    # products otherwise split inside the product launch)
    G.force_split_form(0)
    yield G
    G.force_split_form(-1)


def _torch():
    import torch
    return torch


def _round_up(x, q):
    return (x + q - 1) // q * q


def _planes(ws, nplanes, m, n, k):
    """A and B plane views of the workspace bytes at the documented layout."""
    kp = _round_up(max(k, 1), 8)
    ldp = _round_up(kp, 64)
    a_bytes = _round_up(m * ldp * 2, 256)
    b_bytes = _round_up(n * ldp * 2, 256)
    a = [ws[p * a_bytes:p * a_bytes + m * ldp * 2].view(np.uint16).reshape(m, ldp)
         for p in range(nplanes)]
    base = nplanes * a_bytes
    b = [ws[base + p * b_bytes:base + p * b_bytes + n * ldp * 2].view(np.uint16).reshape(n, ldp)
         for p in range(nplanes)]
    return a, b, kp


def _operands(m, n, k, seed, wild):
    A, B = inputs.uniform_mnk(m, n, k, seed, dtype=np.float32)
    if wild:
        # values with many significant bits, tiny and huge magnitudes
        A.flat[::7] *= np.float32(1e-30)
        B.flat[1::11] *= np.float32(1e30)
        A.flat[3::13] = np.float32(1.0) + np.float32(2.0 ** -9)   # a bf16 tie
    return A, B


@pytest.mark.parametrize("nplanes", [2, 3])
@pytest.mark.parametrize("shape", SHAPES)
def test_split_step_planes_bit_exact(G, nplanes, shape):
    torch = _torch()
    m, n, k = shape
    A, B = _operands(m, n, k, 6100 + m + n + k, wild=True)
    say(f"split planes np={nplanes} m={m} n={n} k={k}")
    Ad, Bd = dev(A, torch), dev(B, torch)
    # the two-step form is the one that writes the planes
    assert not G.split_one_launch(Ad, Bd)
    if nplanes == 2:
        size, fn, split = G.gemm_split_workspace_size(m, n, k), G.gemm_split, oracle.split_bf16
    else:
        size, fn, split = G.gemm_split3_workspace_size(m, n, k), G.gemm_split3, oracle.split3_bf16
    # stale bytes in the workspace: the padding must be written, not inherited
    ws = torch.full((size,), 0xA5, dtype=torch.uint8, device="cuda:0")
    fn(Ad, Bd, workspace=ws)
    torch.cuda.synchronize()
    a, b, kp = _planes(ws.cpu().numpy(), nplanes, m, n, k)
    ra = split(A)
    rb = split(np.ascontiguousarray(B.T))
    for p in range(nplanes):
        assert np.array_equal(a[p][:, :k], ra[p]), ("A plane", p)
        assert np.array_equal(b[p][:, :k], rb[p]), ("B plane", p)
        assert not np.any(a[p][:, k:kp]), ("A padding", p)
        assert not np.any(b[p][:, k:kp]), ("B padding", p)


@pytest.mark.parametrize("nplanes", [2, 3])
def test_split_step_planes_random_bit_patterns(G, nplanes):
    """Every finite binary32 bit pattern class (normals, subnormals, both
    signs) at a ragged shape: the planes equal the oracle's split."""
    torch = _torch()
    m, n, k = 77, 45, 203
    g = np.random.Generator(np.random.PCG64(61))

    def draw(shape):
        bits = g.integers(0, 2 ** 32, size=shape, dtype=np.uint64).astype(np.uint32)
        X = bits.view(np.float32).copy()
        X[~np.isfinite(X)] = 1.0
        X[np.abs(X) > 3e38] = 1.0          # keep x - hi finite
        return X

    A, B = draw((m, k)), draw((k, n))
    Ad, Bd = dev(A, torch), dev(B, torch)
    assert not G.split_one_launch(Ad, Bd)
    if nplanes == 2:
        size, fn, split = G.gemm_split_workspace_size(m, n, k), G.gemm_split, oracle.split_bf16
    else:
        size, fn, split = G.gemm_split3_workspace_size(m, n, k), G.gemm_split3, oracle.split3_bf16
    ws = torch.full((size,), 0x5A, dtype=torch.uint8, device="cuda:0")
    with np.errstate(all="ignore"):
        fn(Ad, Bd, workspace=ws)
        torch.cuda.synchronize()
    a, b, kp = _planes(ws.cpu().numpy(), nplanes, m, n, k)
    ra = split(A)
    rb = split(np.ascontiguousarray(B.T))
    for p in range(nplanes):
        assert np.array_equal(a[p][:, :k], ra[p]), ("A plane", p)
        assert np.array_equal(b[p][:, :k], rb[p]), ("B plane", p)
        assert not np.any(a[p][:, k:kp]) and not np.any(b[p][:, k:kp])


def test_split_product_equals_plane_emulation_ragged(G):
    """At a ragged shape the two-step product is within binary32 accumulation
    error of the oracle's emulation (binary64 sum of the three plane
    products), elementwise: a wrong plane pairing would show here."""
    torch = _torch()
    m, n, k = 1000, 37, 1003
    A, B = _operands(m, n, k, 6200, wild=False)
    Ad, Bd = dev(A, torch), dev(B, torch)
    C = G.gemm_split(Ad, Bd).cpu().double().numpy()
    emul = oracle.split_emul_gemm(A, B)
    absAB = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    # binary32 accumulation of the 3k exact plane products (each at most
    # |a||b|): |error| <= 3k u |A||B| with u = 2^-24
    assert np.all(np.abs(C - emul) <= 3 * k * 2.0 ** -24 * absAB)
