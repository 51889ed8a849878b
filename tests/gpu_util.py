"""Helpers for the GPU parity tests: device copies and sampled comparisons."""
import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, torch, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def host(t):
    return t.detach().float().cpu().numpy() if t.dtype not in (__import__("torch").float64,) \
        else t.detach().cpu().numpy()


def sample_idx(m, n, count, seed):
    """Sampled output positions: the four corners, the last row/column
    (ragged tile edges) and uniform random entries."""
    g = np.random.Generator(np.random.PCG64(seed))
    r = list(g.integers(0, m, count))
    c = list(g.integers(0, n, count))
    edge = [(0, 0), (0, n - 1), (m - 1, 0), (m - 1, n - 1)]
    for j in g.integers(0, n, 16):
        edge.append((m - 1, int(j)))
    for i in g.integers(0, m, 16):
        edge.append((int(i), n - 1))
    r += [e[0] for e in edge]
    c += [e[1] for e in edge]
    return np.array(r, dtype=np.int64), np.array(c, dtype=np.int64)


def full_or_sampled_ref(A, B, C_gpu, full_limit=1200, samples=3000, seed=0):
    """Relative normwise error of C_gpu against the oracle: full product up to
    ``full_limit`` (threaded oracle above 600), else on sampled entries."""
    m, k = A.shape
    n = B.shape[1]
    if max(m, n, k) <= full_limit:
        ref = oracle.gemm(A, B) if max(m, n, k) <= 600 else oracle.gemm_omp(A, B)
        return oracle.relerr_fro(C_gpu, ref), ref
    r, c = sample_idx(m, n, samples, seed)
    ref = oracle.gemm_entries(A, B, r, c)
    return oracle.relerr_sampled(C_gpu[r, c], ref), None
