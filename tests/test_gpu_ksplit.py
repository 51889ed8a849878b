"""GPU parity of gemm_plain_ksplit (the plain product with its K loop cut into
chunks that run as separate workgroups, partial products added in chunk
order) against the CPU oracle.

Tolerances as for gemm_plain (normwise relative to the binary64 oracle):
binary64 1e-12, binary32 1e-5, bfloat16 inputs 2e-2; integer-valued inputs
bit-exact (every partial sum is an integer below 2^24). Chunk counts and
tile shapes are forced to cover chunks whose K-ranges end inside a K-tile,
chunk counts the K loop cannot fill, both the direct-to-LDS and the
register paths (a row pitch that is not a multiple of 16 bytes), and the
automatic choice on the sizes it is meant for.
"""
import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import dev, say

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}
SHAPES_CFG = {"128x128": 0, "128x64": 1, "64x64": 2, "128x128w8": 4}


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    yield G
    G.force_tile_config(-1)
    G.force_ksplit(-1)


def _torch():
    import torch
    return torch


def _tdt(torch, tname):
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[tname]


def _code(G, tname):
    return {"f64": G.GEMM_F64, "f32": G.GEMM_F32, "bf16": G.GEMM_BF16}[tname]


def _run(G, A, B, tname, parts=-1, cfg=-1, pitched=False):
    torch = _torch()
    tdt = _tdt(torch, tname)
    Ad, Bd = dev(A, torch, tdt), dev(B, torch, tdt)
    if pitched:   # row pitch k + 1 elements: the register path
        buf = torch.zeros((A.shape[0], A.shape[1] + 1), dtype=tdt, device="cuda:0")
        buf[:, :A.shape[1]] = Ad
        Ad = buf[:, :A.shape[1]]
    G.force_tile_config(cfg)
    G.force_ksplit(parts)
    try:
        C = G.gemm_plain_ksplit(Ad, Bd)
        torch.cuda.synchronize()
    finally:
        G.force_tile_config(-1)
        G.force_ksplit(-1)
    return C.cpu().double().numpy()


@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("cname", list(SHAPES_CFG))
def test_forced_chunks_every_shape(G, tname, cname):
    """Ragged m, n and k (k not a multiple of any K-tile), 2, 3 and 5 chunks."""
    m, n, k = 300, 260, 1000
    np_dt = np.float32 if tname != "f64" else np.float64
    A, B = inputs.uniform_mnk(m, n, k, 4100 + m, dtype=np_dt)
    ref = oracle.gemm(A, B)
    for parts in (2, 3, 5):
        got = _run(G, A, B, tname, parts, SHAPES_CFG[cname])
        err = oracle.relerr_fro(got, ref)
        say(f"ksplit {tname} {cname} parts={parts} relerr={err:.2e}")
        assert err <= TOL[tname], (tname, cname, parts, err)


@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
def test_integer_inputs_bit_exact(G, tname):
    m, n, k = 130, 200, 2100
    A = inputs.integers((m, k), 21, count=1)[0]
    B = inputs.integers((k, n), 22, count=1)[0]
    ref = oracle.gemm(A, B)
    for parts, cfg in ((2, 0), (7, 2), (4, 4), (16, 1)):
        got = _run(G, A, B, tname, parts, cfg)
        assert np.array_equal(got, ref), (tname, parts, cfg)


@pytest.mark.parametrize("tname", ["f64", "f32", "bf16"])
def test_register_path_pitched_operand(G, tname):
    m, n, k = 200, 136, 700
    np_dt = np.float32 if tname != "f64" else np.float64
    A, B = inputs.uniform_mnk(m, n, k, 77, dtype=np_dt)
    ref = oracle.gemm(A, B)
    for parts in (2, 4):
        got = _run(G, A, B, tname, parts, 0, pitched=True)
        assert oracle.relerr_fro(got, ref) <= TOL[tname], (tname, parts)


def test_more_chunks_than_k_allows(G):
    """k = 100 holds two 64-index chunks: a request for 8 runs 2."""
    m, n, k = 64, 96, 100
    A, B = inputs.uniform_mnk(m, n, k, 5)
    got = _run(G, A, B, "f64", 8, 0)
    assert oracle.relerr_fro(got, oracle.gemm(A, B)) <= 1e-12
    G.force_ksplit(8)
    try:
        assert G.gemm_plain_ksplit_workspace_size(G.GEMM_F64, m, n, k) == 1 * m * n * 8
    finally:
        G.force_ksplit(-1)


@pytest.mark.parametrize("shape", [(1000, 1000, 1000), (256, 256, 65536), (800, 640, 1200),
                                   (1024, 1024, 8192)])
def test_automatic_split_binary64(G, shape):
    """The sizes the split is meant for: it splits them, and matches the
    oracle over the whole product."""
    m, n, k = shape
    assert G.gemm_plain_ksplit_workspace_size(G.GEMM_F64, m, n, k) > 0
    A, B = inputs.uniform_mnk(m, n, k, 900 + k)
    got = _run(G, A, B, "f64")
    err = oracle.relerr_fro(got, oracle.gemm_omp(A, B))
    say(f"ksplit auto {shape} relerr={err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("shape", [(256, 192, 20000), (1024, 1024, 4096), (1024, 1024, 8192)])
def test_automatic_split_binary32_deep_k(G, shape):
    m, n, k = shape
    assert G.gemm_plain_ksplit_workspace_size(G.GEMM_F32, m, n, k) > 0
    A, B = inputs.uniform_mnk(m, n, k, 31, dtype=np.float32)
    got = _run(G, A, B, "f32")
    assert oracle.relerr_fro(got, oracle.gemm_omp(A, B)) <= 1e-5


@pytest.mark.parametrize("shape", [(256, 192, 20000), (1024, 1024, 8192), (512, 512, 16384)])
def test_automatic_split_bf16_deep_k(G, shape):
    """bfloat16 inputs on the automatic rule's deep-K shapes (4-wave 128 x 128
    tiles, two per CU, chunks of at least 512): whole-path error against the
    oracle of the binary32 data <= 2e-2, kernel-only error against the
    oracle of the rounded inputs <= 1e-5."""
    m, n, k = shape
    assert G.gemm_plain_ksplit_workspace_size(G.GEMM_BF16, m, n, k) > 0
    A, B = inputs.uniform_mnk(m, n, k, 33, dtype=np.float32)
    got = _run(G, A, B, "bf16")
    Ar = oracle.bf16_to_f32(oracle.bf16_rne(A))
    Br = oracle.bf16_to_f32(oracle.bf16_rne(B))
    e_path = oracle.relerr_fro(got, oracle.gemm_omp(A, B))
    e_kernel = oracle.relerr_fro(got, oracle.gemm_omp(Ar, Br))
    say(f"bf16 ksplit {shape}: whole-path {e_path:.3e} kernel-only {e_kernel:.3e}")
    assert e_path <= TOL["bf16"]
    assert e_kernel <= 1e-5


def test_large_products_run_unsplit_and_leave_workspace(G):
    torch = _torch()
    n = 512
    assert G.gemm_plain_ksplit_workspace_size(G.GEMM_F64, 4096, 4096, 4096) == 0   # many tiles
    assert G.gemm_plain_ksplit_workspace_size(G.GEMM_F32, 1000, 1000, 1000) == 0
    assert G.gemm_plain_ksplit_workspace_size(G.GEMM_F64, n, n, 64) == 0   # K too short
    A, B = inputs.uniform_mnk(n, n, 64, 3)
    ws = torch.full((4096,), 0x5A, dtype=torch.uint8, device="cuda:0")
    Ad, Bd = dev(A, torch), dev(B, torch)
    C = G.gemm_plain_ksplit(Ad, Bd, workspace=ws)
    Cp = G.gemm_plain(Ad, Bd)
    torch.cuda.synchronize()
    assert bool((ws == 0x5A).all())
    assert torch.equal(C, Cp)


def test_workspace_errors_and_zero_k(G):
    torch = _torch()
    m, n, k = 500, 500, 1000
    need = G.gemm_plain_ksplit_workspace_size(G.GEMM_F64, m, n, k)
    assert need > 0
    A = torch.ones((m, k), dtype=torch.float64, device="cuda:0")
    B = torch.ones((k, n), dtype=torch.float64, device="cuda:0")
    small = torch.empty(need - 8, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(G.GemmArgError):
        G.gemm_plain_ksplit(A, B, workspace=small)
    odd = torch.empty(need + 16, dtype=torch.uint8, device="cuda:0")[8:]
    with pytest.raises(G.GemmArgError):
        G.gemm_plain_ksplit(A, B, workspace=odd)
    C = G.gemm_plain_ksplit(A, B)
    torch.cuda.synchronize()
    assert bool((C == float(k)).all())
    A0 = torch.zeros((40, 0), dtype=torch.float64, device="cuda:0")
    B0 = torch.zeros((0, 36), dtype=torch.float64, device="cuda:0")
    C0 = torch.full((40, 36), 5.0, dtype=torch.float64, device="cuda:0")
    G.gemm_plain_ksplit(A0, B0, C0)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(C0)) == 0


def test_repeatable(G):
    """The same sizes give the same chunks: two calls agree bit for bit."""
    torch = _torch()
    A, B = inputs.uniform_mnk(1000, 1000, 1000, 8)
    Ad, Bd = dev(A, torch), dev(B, torch)
    C1 = G.gemm_plain_ksplit(Ad, Bd)
    C2 = G.gemm_plain_ksplit(Ad, Bd)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
