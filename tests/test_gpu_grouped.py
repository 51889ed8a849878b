"""GPU parity of the persistent grouped product (captured hipGraph, tuned policy).

512 independent square products, N log-uniform in [10, 2000], in binary64
and binary32. Every problem equals the single-product kernel at the same
tile shape bit for bit (same tiles, same reduction order): problems whose
rows are whole 16-byte vectors against a launch on their own operands,
packed problems (the plan copies their operands into zero-padded 16-byte
rows) against a launch on padded copies, and with packing off against a
launch on their own operands again; the oracle checks every problem (full
product for N <= 256, sampled entries above).
"""
import os

import numpy as np
import pytest

import oracle
from paper_1012_2273_amd import inputs
from gpu_util import dev, sample_idx, say

pytestmark = pytest.mark.gpu
CLASS_EDGES = [48, 96, 192, 384, 768, 1536]


def size_class(m, n):
    s = max(m, n)
    return sum(1 for e in CLASS_EDGES if s >= e)


@pytest.fixture(scope="module")
def G(gpu_device):
    import paper_1012_2273_amd as G
    G.load()
    yield G
    G.force_tile_config(-1)


def _torch():
    import torch
    return torch


def _batch(count, dtype, seed=3_000_000):
    sizes = inputs.batch_sizes(count, seed)
    probs = [inputs.batch_problem(i, int(n), seed, dtype) for i, n in enumerate(sizes)]
    return sizes, probs


def _vec_ok(A, B):
    """Both operands allow 16-byte transfers (the plan's test)."""
    v = 16 // A.element_size()
    return (A.data_ptr() % 16 == 0 and B.data_ptr() % 16 == 0 and A.stride(0) % v == 0
            and B.stride(0) % v == 0 and A.shape[1] % v == 0 and B.shape[1] % v == 0)


def _single_like_plan(G, A, B, cfg, packed):
    """One gemm_plain launch at tile config `cfg` computing what the plan
    computes for (A, B): on the operands themselves, or on zero-padded
    copies with 16-byte rows (the packed form), keeping the first n columns."""
    torch = _torch()
    n = B.shape[1]
    if packed:
        v = 16 // A.element_size()
        m, k = A.shape
        kp, np_ = -(-k // v) * v, -(-n // v) * v
        Ap = torch.zeros((m, kp), dtype=A.dtype, device=A.device)
        Ap[:, :k] = A
        Bp = torch.zeros((kp, np_), dtype=B.dtype, device=B.device)
        Bp[:k, :n] = B
        A, B = Ap, Bp
    G.force_tile_config(cfg)
    try:
        C = G.gemm_plain(A, B)
    finally:
        G.force_tile_config(-1)
    return C[:, :n]


def _check_against_oracle(sizes, probs, Cs, tol, max_full=256):
    worst = 0.0
    for i, (n, (A, B)) in enumerate(zip(sizes, probs)):
        C = Cs[i].cpu().double().numpy()
        if n <= max_full:
            err = oracle.relerr_fro(C, oracle.gemm(A, B))
        else:
            r, c = sample_idx(n, n, 120, i)
            err = oracle.relerr_sampled(C[r, c], oracle.gemm_entries(A, B, r, c))
        worst = max(worst, err)
    assert worst <= tol, worst
    return worst


@pytest.mark.parametrize("tname", ["f64", "f32"])
def test_batch_512_graph_autotuned(G, tname, tmp_path):
    torch = _torch()
    dt = np.float64 if tname == "f64" else np.float32
    tol = 1e-12 if tname == "f64" else 1e-5
    sizes, probs = _batch(512, dt)
    say(f"grouped {tname}: sum 2N^3 = {sum(2 * int(n) ** 3 for n in sizes):.3e}")
    As = [dev(A, torch) for A, _ in probs]
    Bs = [dev(B, torch) for _, B in probs]
    cache = str(tmp_path / "tune.json")
    plan = G.GroupedPlan(As, Bs, autotune=True, tune_cache=cache)
    tiles, policy = plan.info()
    say(f"grouped {tname}: tiles={tiles} policy={policy}")
    assert os.path.exists(cache)
    Cs = plan.run()
    torch.cuda.synchronize()
    worst = _check_against_oracle(sizes, probs, Cs, tol)
    say(f"grouped {tname}: worst relerr={worst:.3e}")

    # bitwise equal to single-product launches at the policy's tile shape
    names = G.tile_configs()
    n_packed = 0
    for i in range(0, 512, 7):
        cfg = names.index(policy[size_class(int(sizes[i]), int(sizes[i]))])
        packed = not _vec_ok(As[i], Bs[i])
        n_packed += packed
        Ci = _single_like_plan(G, As[i], Bs[i], cfg, packed)
        torch.cuda.synchronize()
        assert torch.equal(Ci, Cs[i]), (i, packed)
    assert n_packed > 0

    # graph replays with eager work in between: every replay identical
    first = [C.clone() for C in Cs]
    for rep in range(6):
        for C in Cs:
            C.zero_()
        _ = G.gemm_plain(As[0], Bs[0])
        plan.run()
        torch.cuda.synchronize()
        for i in range(0, 512, 5):
            assert torch.equal(Cs[i], first[i]), (rep, i)

    # a second plan reads the tuned policy from the cache
    plan2 = G.GroupedPlan(As[:512], Bs[:512], autotune=True, tune_cache=cache)
    assert plan2.info()[1] == policy
    plan2.close()
    plan.close()

    # packing off: the problems without 16-byte rows run on the register
    # path, bit for bit as a single launch on their own operands
    plan3 = G.GroupedPlan(As, Bs, tune_cache=cache, autotune=True, pack=False)
    assert plan3.info()[1] == policy
    Cs3 = plan3.run()
    torch.cuda.synchronize()
    _check_against_oracle(sizes, probs, Cs3, tol)
    for i in range(0, 512, 11):
        cfg = names.index(policy[size_class(int(sizes[i]), int(sizes[i]))])
        Ci = _single_like_plan(G, As[i], Bs[i], cfg, False)
        torch.cuda.synchronize()
        assert torch.equal(Ci, Cs3[i]), i
    plan3.close()


def test_plan_update_new_pointers(G):
    torch = _torch()
    sizes, probs = _batch(40, np.float64, seed=77)
    As = [dev(A, torch) for A, _ in probs]
    Bs = [dev(B, torch) for _, B in probs]
    plan = G.GroupedPlan(As, Bs)
    plan.run()
    As2 = [A.flip(0).contiguous() for A in As]
    Cs2 = [torch.empty_like(C) for C in plan.Cs]
    plan.update(As2, Bs, Cs2)
    plan.run()
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(probs):
        ref = oracle.gemm(A[::-1].copy(), B) if sizes[i] <= 300 else None
        if ref is not None:
            assert oracle.relerr_fro(Cs2[i].cpu().numpy(), ref) <= 1e-12
    with pytest.raises(ValueError):
        plan.update(As2[:-1], Bs[:-1], Cs2[:-1])
    plan.close()


def test_plan_update_rejects_misaligned_views(G):
    """A problem planned with 16-byte aligned operands runs in the kernel of
    16-byte transfers: an update to an offset view (8-byte aligned binary64)
    is refused, the plan keeps its old pointers and still computes them."""
    torch = _torch()
    n = 64                                   # even: 16-byte rows, planned aligned
    A, B = inputs.uniform_square(n, 505)
    Ad, Bd = dev(A, torch), dev(B, torch)
    plan = G.GroupedPlan([Ad], [Bd])
    C0 = plan.Cs[0]
    # same shape and leading dimension, base 8 bytes past a 16-byte boundary
    flat = torch.zeros(n * n + 1, dtype=torch.float64, device="cuda:0")
    view = flat[1:].view(n, n)
    view.copy_(Ad)
    assert view.data_ptr() % 16 == 8 and view.stride() == Ad.stride()
    with pytest.raises(ValueError, match="16-byte"):
        plan.update([view], [Bd], [torch.empty_like(C0)])
    C0.zero_()
    plan.run()
    torch.cuda.synchronize()
    assert oracle.relerr_fro(C0.cpu().numpy(), oracle.gemm(A, B)) <= 1e-12
    # an odd-sized problem (packed, or on the register path) is planned for
    # any alignment and takes the view; a packed plan reads the new pointers
    # in its next run's copies
    m = 63
    A3, B3 = inputs.uniform_square(m, 506)
    A3d, B3d = dev(A3, torch), dev(B3, torch)
    flat3 = torch.zeros(m * m + 1, dtype=torch.float64, device="cuda:0")
    view3 = flat3[1:].view(m, m)
    for pack in (True, False):
        plan3 = G.GroupedPlan([A3d], [B3d], pack=pack)
        view3.copy_(2.0 * A3d)
        C3 = torch.empty((m, m), dtype=torch.float64, device="cuda:0")
        plan3.update([view3], [B3d], [C3])
        plan3.run()
        torch.cuda.synchronize()
        assert oracle.relerr_fro(C3.cpu().numpy(), oracle.gemm(2.0 * A3, B3)) <= 1e-12, pack
        view3.copy_(A3d)
        plan3.run()
        torch.cuda.synchronize()
        assert oracle.relerr_fro(C3.cpu().numpy(), oracle.gemm(A3, B3)) <= 1e-12, pack
        plan3.close()
    plan.close()


def test_uncaptured_and_edge_problems(G):
    torch = _torch()
    shapes = [(5, 7, 3), (0, 4, 4), (6, 0, 2), (9, 9, 0), (1, 1, 1), (130, 70, 257), (33, 600, 10)]
    As, Bs, hostA, hostB = [], [], [], []
    for m, n, k in shapes:
        A, B = inputs.uniform_mnk(m, n, k, m + n + k)
        hostA.append(A)
        hostB.append(B)
        As.append(dev(A, torch))
        Bs.append(dev(B, torch))
    Cs = [torch.full((m, n), 3.0, dtype=torch.float64, device="cuda:0") for m, n, _ in shapes]
    G.gemm_grouped(As, Bs, Cs)
    for (m, n, k), A, B, C in zip(shapes, hostA, hostB, Cs):
        got = C.cpu().numpy()
        if m == 0 or n == 0:
            assert got.size == 0
        elif k == 0:
            assert np.count_nonzero(got) == 0
        else:
            assert oracle.relerr_fro(got, oracle.gemm(A, B)) <= 1e-12
    # empty group
    G.gemm_grouped([], [], [])


def test_grouped_integer_bit_exact(G):
    torch = _torch()
    sizes = inputs.batch_sizes(64, 11, lo=10, hi=700)
    As, Bs, probs = [], [], []
    for i, n in enumerate(sizes):
        A, B = inputs.integers((int(n), int(n)), 100 + i, np.float32, 2)
        probs.append((A, B))
        As.append(dev(A, torch))
        Bs.append(dev(B, torch))
    plan = G.GroupedPlan(As, Bs)
    Cs = plan.run()
    torch.cuda.synchronize()
    for (A, B), C in zip(probs, Cs):
        assert np.array_equal(C.cpu().double().numpy(), oracle.gemm(A, B))
    plan.close()


def _offset_view(X, torch, lead_pad, base_elems):
    """X's values in a view with row pitch cols + lead_pad, starting
    base_elems elements past a 256-byte aligned allocation."""
    r, c = X.shape
    flat = torch.zeros(base_elems + r * (c + lead_pad), dtype=X.dtype, device=X.device)
    v = flat[base_elems:].view(r, c + lead_pad)[:, :c]
    v.copy_(X)
    return v


@pytest.mark.parametrize("pack", [True, False], ids=["pack", "nopack"])
@pytest.mark.parametrize("tname", ["f64", "f32"])
def test_grouped_unaligned_rows_every_edge(G, tname, pack):
    """Problems whose rows are not whole 16-byte vectors (odd binary64
    sizes, binary32 sizes not multiples of 4, offset views and padded
    pitches) are packed into 16-byte rows, or with packing off run in the
    persistent kernel's register path: ragged M, N and K edges, single rows
    and columns, K shorter than a K-tile; each against the oracle, and
    integer entries bit for bit."""
    torch = _torch()
    dt = np.float64 if tname == "f64" else np.float32
    tol = 1e-12 if tname == "f64" else 1e-5
    shapes = [(33, 65, 17), (129, 1, 3), (1, 127, 255), (257, 255, 129), (131, 67, 1001),
              (67, 133, 5), (255, 257, 258), (9, 7, 1), (130, 66, 200), (64, 128, 96)]
    # the last two have 16-byte rows; given as views they are not 16-byte
    # operands any more (base 1 element off, pitch padded by 3 elements)
    views = {8: (3, 1), 9: (0, 1)}
    As, Bs, host = [], [], []
    for i, (m, n, k) in enumerate(shapes):
        A, B = inputs.uniform_mnk(m, n, k, 880 + i, dtype=dt)
        host.append((A, B))
        Ad, Bd = dev(A, torch), dev(B, torch)
        if i in views:
            Ad = _offset_view(Ad, torch, *views[i])
        As.append(Ad)
        Bs.append(Bd)
    assert not any(_vec_ok(A, B) for A, B in zip(As, Bs))
    plan = G.GroupedPlan(As, Bs, pack=pack)
    Cs = plan.run()
    torch.cuda.synchronize()
    for (A, B), C in zip(host, Cs):
        assert oracle.relerr_fro(C.cpu().double().numpy(), oracle.gemm(A, B)) <= tol
    # replays recopy: new values in the same operands
    for A in As:
        A.mul_(-1.0)
    Cs = plan.run()
    torch.cuda.synchronize()
    for (A, B), C in zip(host, Cs):
        assert oracle.relerr_fro(C.cpu().double().numpy(), oracle.gemm(-A, B)) <= tol
    plan.close()
    # integer entries: exact
    As, Bs, host = [], [], []
    for i, (m, n, k) in enumerate(shapes):
        A = inputs.integers((m, k), 890 + i, dt, 1)[0]
        B = inputs.integers((k, n), 990 + i, dt, 1)[0]
        host.append((A, B))
        As.append(dev(A, torch))
        Bs.append(dev(B, torch))
    plan = G.GroupedPlan(As, Bs, pack=pack)
    Cs = plan.run()
    torch.cuda.synchronize()
    for (A, B), C in zip(host, Cs):
        assert np.array_equal(C.cpu().double().numpy(), oracle.gemm(A, B))
    plan.close()
