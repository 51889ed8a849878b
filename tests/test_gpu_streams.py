"""GPU checks of the asynchronous contract: every entry point runs on the
caller's stream (torch's current stream in the binding), in order with the
caller's other work on that stream, and calls on different streams or from
different host threads do not interfere (separate workspaces, thread-local
error state, locked caches). Results are held to the oracle or bit-exact.
"""
import threading

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
    return G


def test_every_entry_point_on_a_user_stream(G):
    import torch
    n = 300
    A, B = inputs.uniform_square(n, 61)
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        Ad, Bd = dev(A, torch), dev(B, torch)
        A32d, B32d = dev(A32, torch), dev(B32, torch)
        C64 = G.gemm_plain(Ad, Bd)
        Cs = G.gemm_split(A32d, B32d)
        C3 = G.gemm_split3(A32d, B32d)
        dA, dB = G.gemm_backward(Ad, Bd, Ad)
        plan = G.GroupedPlan([Ad, Bd], [Bd, Ad])
        Cg = plan.run()
    s.synchronize()
    ref = oracle.gemm(A, B)
    assert oracle.relerr_fro(C64.cpu().numpy(), ref) <= 1e-12
    ref32 = oracle.gemm(A32, B32)
    assert oracle.relerr_fro(Cs.cpu().double().numpy(), ref32) <= 1e-5
    assert oracle.relerr_fro(C3.cpu().double().numpy(), ref32) <= 1e-5
    _, gA, gB = oracle.loss_and_grads(A, B, A)
    assert oracle.relerr_fro(dA.cpu().numpy(), gA) <= 1e-12
    assert oracle.relerr_fro(dB.cpu().numpy(), gB) <= 1e-12
    assert oracle.relerr_fro(Cg[0].cpu().numpy(), ref) <= 1e-12
    assert oracle.relerr_fro(Cg[1].cpu().numpy(), oracle.gemm(B, A)) <= 1e-12
    plan.close()


def test_ordered_behind_earlier_work_on_the_stream(G):
    """The product reads its inputs only after the stream's earlier work
    (here: the operands are written by a copy queued behind a long product
    on a second stream that the first stream waits for)."""
    import torch
    n = 1024
    A, B = inputs.integer_square(n, 62)
    Ad, Bd = dev(A, torch), dev(B, torch)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    X = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    with torch.cuda.stream(s2):
        big = torch.from_numpy(inputs.uniform_square(3000, 63)[0]).to("cuda:0")
        for _ in range(3):
            G.gemm_plain(big, big)            # keeps s2 busy for a few ms
        X.copy_(Ad)                           # the operand lands only after that
        ev = torch.cuda.Event()
        ev.record(s2)
    with torch.cuda.stream(s1):
        s1.wait_event(ev)
        C = G.gemm_plain(X, Bd)
    s1.synchronize()
    assert np.array_equal(C.cpu().numpy(), oracle.gemm_omp(A, B))


def test_two_streams_concurrently(G):
    """Split products on two streams at once, each with its own workspace."""
    import torch
    n = 700
    probs = [inputs.uniform_square(n, 64 + i, dtype=np.float32) for i in range(2)]
    streams = [torch.cuda.Stream() for _ in range(2)]
    outs = []
    for (A, B), s in zip(probs, streams):
        with torch.cuda.stream(s):
            Ad, Bd = dev(A, torch), dev(B, torch)
            outs.append([G.gemm_split(Ad, Bd) for _ in range(4)])
    torch.cuda.synchronize()
    for (A, B), cs in zip(probs, outs):
        ref = oracle.gemm(A, B)
        first = cs[0].cpu().numpy()
        for c in cs:
            got = c.cpu().numpy()
            assert np.array_equal(got, first)          # deterministic, no cross-talk
            assert oracle.relerr_fro(got.astype(np.float64), ref) <= 1e-5


def test_host_threads_concurrently(G):
    """Several host threads, each with its own stream and problem sizes (so
    each also fills the library's occupancy cache); one thread also provokes
    an argument error, which must not leak into the others."""
    import torch
    results, errors = {}, []

    def worker(i):
        try:
            n = 200 + 37 * i
            A, B = inputs.integer_square(n, 70 + i)
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                Ad, Bd = dev(A, torch), dev(B, torch)
                lib = G._lib.load()
                if i == 0:   # an argument error (ld < k) in this thread only
                    assert lib.gemm_plain(0, 4, 4, 4, 16, 3, 16, 4, 16, 4, None) != 0
                    assert b"leading dimension" in lib.gemm_last_error()
                C = G.gemm_plain(Ad, Bd)
                C32 = G.gemm_plain(Ad.float(), Bd.float())
                assert lib.gemm_last_error() == b""
            s.synchronize()
            results[i] = (A, B, C.cpu().numpy(), C32.cpu().double().numpy())
        except Exception as e:               # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for i, (A, B, C, C32) in results.items():
        ref = oracle.gemm(A, B)
        assert np.array_equal(C, ref) and np.array_equal(C32, ref), i
    say("4 host threads ok")
