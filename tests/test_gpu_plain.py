"""GPU parity of gemm_plain (binary64, binary32, bfloat16) against the CPU oracle.

Tolerances (normwise relative, ||C - C_ref||_F / ||C_ref||_F, binary64):
binary64 1e-12, binary32 1e-5, bfloat16 inputs 2e-2; integer-valued inputs
bit-exact on every path.
"""
import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import dev, full_or_sampled_ref, say, sample_idx

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}


@pytest.fixture(scope="module")
def G(gpu_device):
    import torch
    import paper_1012_2273_amd as G
    G.load()
    yield G
    G.force_tile_config(-1)


def _torch():
    import torch
    return torch


def _gpu_plain(G, A, B, tdtype, cfg=-1):
    torch = _torch()
    G.force_tile_config(cfg)
    try:
        C = G.gemm_plain(dev(A, torch, tdtype), dev(B, torch, tdtype))
        torch.cuda.synchronize()
    finally:
        G.force_tile_config(-1)
    return C.cpu().double().numpy()


@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
def test_identity_permutation_every_tile_config(G, tname):
    """Exact: I*B = B, A*I = A, P*A = row permutation (checks the MFMA
    operand and output lane layouts of every tile shape)."""
    torch = _torch()
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[tname]
    n = 77
    A, B = inputs.integer_square(n, 3)
    I = inputs.special("identity", n)
    P = inputs.special("permutation", n, 4)
    perm = np.argmax(P, axis=1)
    for cfg in range(len(G.tile_configs())):
        say(f"identity {tname} cfg={cfg}")
        assert np.array_equal(_gpu_plain(G, I, B, tdt, cfg), B)
        assert np.array_equal(_gpu_plain(G, A, I, tdt, cfg), A)
        assert np.array_equal(_gpu_plain(G, P, A, tdt, cfg), A[perm])


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 31, 33, 64, 127, 129, 255])
def test_f64_ragged_sizes_every_config(G, n):
    torch = _torch()
    A, B = inputs.uniform_square(n, 7000 + n)
    ref = oracle.gemm(A, B)
    for cfg in range(len(G.tile_configs())):
        C = _gpu_plain(G, A, B, torch.float64, cfg)
        err = oracle.relerr_fro(C, ref)
        assert err <= TOL["f64"], (n, cfg, err)


def test_f64_smallest_instance_n500(G):
    """N = 500 binary64, U[-1,1], the plain method's smallest configuration."""
    torch = _torch()
    n = 500
    A, B = inputs.uniform_square(n, inputs.seed_for(0, n))
    C = _gpu_plain(G, A, B, torch.float64)
    err = oracle.relerr_fro(C, oracle.gemm(A, B))
    say(f"f64 n=500 relerr={err:.3e}")
    assert err <= TOL["f64"]


@pytest.mark.parametrize("n", [10, 100, 500, 1000, 2000, 4096])
def test_f64_sweep(G, n):
    """The paper's sweep plus N = 4096 (full oracle up to 2000, sampled above)."""
    torch = _torch()
    A, B = inputs.uniform_square(n, inputs.seed_for(1, n))
    C = _gpu_plain(G, A, B, torch.float64)
    err, _ = full_or_sampled_ref(A, B, C, full_limit=2000, seed=n)
    say(f"f64 sweep n={n} relerr={err:.3e}")
    assert err <= TOL["f64"]


@pytest.mark.parametrize("n", [100, 500, 1000, 2000])
@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
def test_integer_inputs_bit_exact(G, n, tname):
    torch = _torch()
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[tname]
    A, B = inputs.integer_square(n, inputs.seed_for(1, n, variant=True))
    C = _gpu_plain(G, A, B, tdt)
    if n <= 1000:
        ref = oracle.gemm_omp(A, B) if n > 500 else oracle.gemm(A, B)
        assert np.array_equal(C, ref)
    else:
        r, c = sample_idx(n, n, 4000, n)
        assert np.array_equal(C[r, c], oracle.gemm_entries(A, B, r, c))


@pytest.mark.parametrize("shape", [(37, 53, 71), (129, 1, 300), (1, 257, 19), (300, 200, 1),
                                   (65, 130, 33), (200, 3, 1000), (5, 700, 9)])
@pytest.mark.parametrize("tname", ["f64", "f32"])
def test_rectangular(G, shape, tname):
    torch = _torch()
    tdt = torch.float64 if tname == "f64" else torch.float32
    m, n, k = shape
    A, B = inputs.uniform_mnk(m, n, k, 900 + m + n + k)
    A = A.astype(np.float32 if tname == "f32" else np.float64)
    B = B.astype(np.float32 if tname == "f32" else np.float64)
    for cfg in (-1, 0, 3):
        C = _gpu_plain(G, A, B, tdt, cfg)
        assert oracle.relerr_fro(C, oracle.gemm(A, B)) <= TOL[tname]


def test_k_zero_writes_zeros(G):
    torch = _torch()
    for tdt in (torch.float64, torch.float32, torch.bfloat16):
        A = torch.zeros((33, 0), dtype=tdt, device="cuda:0")
        B = torch.zeros((0, 17), dtype=tdt, device="cuda:0")
        C = torch.full((33, 17), 7.0, dtype=torch.float64 if tdt == torch.float64 else torch.float32,
                       device="cuda:0")
        G.gemm_plain(A, B, C)
        torch.cuda.synchronize()
        assert torch.count_nonzero(C).item() == 0


def test_empty_outputs_noop(G):
    torch = _torch()
    A = torch.ones((0, 5), dtype=torch.float64, device="cuda:0")
    B = torch.ones((5, 3), dtype=torch.float64, device="cuda:0")
    assert G.gemm_plain(A, B).shape == (0, 3)


@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
def test_leading_dims_and_unaligned(G, tname):
    """Views into larger buffers: ld > row length, and pointers/lds that
    defeat 16-byte vector loads (scalar path)."""
    torch = _torch()
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[tname]
    m, n, k = 131, 97, 203
    if tname == "bf16":
        A, B = inputs.integers((m + 3, k + 5), 31, np.float64, 1)[0], inputs.integers((k + 4, n + 7), 32, np.float64, 1)[0]
    else:
        A = inputs.uniform((m + 3, k + 5), 31, count=1)[0]
        B = inputs.uniform((k + 4, n + 7), 32, count=1)[0]
    Ad, Bd = dev(A, torch, tdt), dev(B, torch, tdt)
    Cbig = torch.zeros((m + 4, n + 9), dtype=torch.float64 if tname == "f64" else torch.float32,
                       device="cuda:0")
    for (ao, bo) in ((0, 0), (1, 1), (1, 0), (0, 3)):
        Av = Ad[ao:ao + m, ao:ao + k]
        Bv = Bd[bo:bo + k, bo:bo + n]
        Cv = Cbig[1:1 + m, 2:2 + n]
        G.gemm_plain(Av, Bv, Cv)
        torch.cuda.synchronize()
        ref = oracle.gemm(A[ao:ao + m, ao:ao + k].astype(np.float32).astype(np.float64) if tname != "f64" else A[ao:ao + m, ao:ao + k],
                          B[bo:bo + k, bo:bo + n].astype(np.float32).astype(np.float64) if tname != "f64" else B[bo:bo + k, bo:bo + n])
        got = Cv.cpu().double().numpy()
        tol = 0.0 if tname == "bf16" else TOL[tname]
        assert oracle.relerr_fro(got, ref) <= tol, (ao, bo)
        # the margin of the output buffer is untouched
        mask = torch.ones_like(Cbig, dtype=torch.bool)
        mask[1:1 + m, 2:2 + n] = False
        assert torch.count_nonzero(Cbig[mask]).item() == 0


def test_deterministic_bits(G):
    torch = _torch()
    A, B = inputs.uniform_square(700, 77)
    Ad, Bd = dev(A, torch), dev(B, torch)
    C1 = G.gemm_plain(Ad, Bd)
    C2 = G.gemm_plain(Ad, Bd)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("n", [2048, 4096, 8192])
@pytest.mark.parametrize("variant", ["uniform", "row_scaled"])
def test_f32_precision_config(G, n, variant):
    """Binary32 at the precision-study sizes, against binary64 oracle entries,
    plus the associativity invariant (A B) x = A (B x) over all rows."""
    torch = _torch()
    if variant == "uniform":
        A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    else:
        A, B = inputs.row_scaled(n, inputs.seed_for(2, n, variant=True))
    Ad, Bd = dev(A, torch), dev(B, torch)
    C = G.gemm_plain(Ad, Bd)
    torch.cuda.synchronize()
    Ch = C.cpu().double().numpy()
    r, c = sample_idx(n, n, 1500, n)
    err = oracle.relerr_sampled(Ch[r, c], oracle.gemm_entries(A, B, r, c))
    say(f"f32 n={n} {variant} sampled relerr={err:.3e}")
    assert err <= TOL["f32"]
    x = inputs.uniform((n, 1), 5, np.float32, 1)[0]
    xd = dev(x, torch)
    left = G.gemm_plain(C, xd).cpu().double().numpy()
    right = G.gemm_plain(Ad, G.gemm_plain(Bd, xd)).cpu().double().numpy()
    scale = np.abs(A.astype(np.float64)) @ (np.abs(B.astype(np.float64)) @ np.abs(x.astype(np.float64)))
    assert np.all(np.abs(left - right) <= 3 * n * 2.0 ** -24 * scale + 1e-30)


@pytest.mark.parametrize("n", [2048, 4096, 8192])
@pytest.mark.parametrize("variant", ["uniform", "row_scaled"])
def test_bf16_plain_precision_config(G, n, variant):
    """bfloat16 inputs (RNE of the binary32 data) at the precision-study sizes,
    uniform and row-scaled: whole-path error against the binary64 oracle of
    the binary32 inputs <= 2e-2; kernel-only error against the oracle of the
    rounded inputs <= 1e-5 (sampled entries)."""
    torch = _torch()
    if variant == "uniform":
        A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
    else:
        A, B = inputs.row_scaled(n, inputs.seed_for(2, n, variant=True))
    say(f"bf16 precision config n={n} {variant}")
    Ab = dev(A, torch).to(torch.bfloat16)
    Bb = dev(B, torch).to(torch.bfloat16)
    C = G.gemm_plain(Ab, Bb)
    torch.cuda.synchronize()
    Ch = C.cpu().double().numpy()
    del C
    r, c = sample_idx(n, n, 1500, n + 1)
    err = oracle.relerr_sampled(Ch[r, c], oracle.gemm_entries(A, B, r, c))
    Ar = oracle.bf16_to_f32(oracle.bf16_rne(A))
    Br = oracle.bf16_to_f32(oracle.bf16_rne(B))
    err_k = oracle.relerr_sampled(Ch[r, c], oracle.gemm_entries(Ar, Br, r, c))
    say(f"bf16 n={n} {variant} whole-path relerr={err:.3e} kernel-only={err_k:.3e}")
    assert err <= TOL["bf16"]
    assert err_k <= 1e-5
