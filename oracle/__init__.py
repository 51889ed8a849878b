"""Plain CPU oracle for C = A*B and everything the GPU path derives from it.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the product package.
It shares no code with the HIP library. The arithmetic lives in ``oracle.c``
(plain C, binary64, no FMA contraction); this module compiles it with gcc,
marshals NumPy arrays and adds the bookkeeping the paper states in words.

Source: Hasta and Mutiara, arXiv 1012.2273.
  * Section 3.1, Algorithm 1; Algorithms 3 and 4 (zeroed C): ``gemm``.
  * Section 3.1.2, Algorithm 4 (static row split over threads): ``gemm_omp``.
  * Section 3.1 (operation count N^2 (2N-1), about 2N^3): ``flops_paper``,
    ``flops_2n3``; Algorithm 2 / Algorithm 4 (rate = ops / t / 1e6).
  * Section 3.1.1, Algorithm 2 (averow / extra / offset row split): ``row_partition``.
The extensions that the paper does not contain (binary32 and bfloat16
inputs, the two- and three-term bfloat16 splits, batching, the backward
product) are
reduced here to the same binary64 definition applied to the exact values the
GPU receives, see the individual docstrings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-std=c11", "-shared", "-fPIC", "-Wall"]
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (next to it)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            i64, dp, fp = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
            lib.oracle_gemm_f64.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64]
            lib.oracle_gemm_f64.restype = None
            lib.oracle_gemm_f64_omp.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64,
                                                ctypes.c_int]
            lib.oracle_gemm_f64_omp.restype = None
            lib.oracle_gemm_entries_f64.argtypes = [i64, dp, i64, dp, i64, dp, dp, i64, dp]
            lib.oracle_gemm_entries_f64.restype = None
            lib.oracle_split_bf16.argtypes = [i64, fp, dp, dp]
            lib.oracle_split_bf16.restype = None
            lib.oracle_split3_bf16.argtypes = [i64, fp, dp, dp, dp]
            lib.oracle_split3_bf16.restype = None
            lib.oracle_bf16_rne_array.argtypes = [i64, fp, dp]
            lib.oracle_bf16_rne_array.restype = None
            lib.oracle_max_threads.argtypes = []
            lib.oracle_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _f64(x) -> np.ndarray:
    """Exact widening of binary32 / bfloat16-valued / integer data to binary64."""
    a = np.asarray(x)
    if a.dtype == np.float64 and a.flags.c_contiguous:
        return a
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _check2(A, B):
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError(f"shape mismatch {A.shape} x {B.shape}")


def gemm(A, B) -> np.ndarray:
    """C = A*B in binary64, each entry summed in ascending reduction order.

    Section 3.1, Algorithm 1 (loop nest), zeroed C as in Algorithms 3 and 4.
    Inputs of any real dtype are widened exactly to binary64 first.
    """
    A, B = _f64(A), _f64(B)
    _check2(A, B)
    m, k = A.shape
    n = B.shape[1]
    C = np.empty((m, n), dtype=np.float64)
    _load().oracle_gemm_f64(m, n, k, _ptr(A), k, _ptr(B), n, _ptr(C), n)
    return C


def gemm_omp(A, B, threads: int | None = None) -> np.ndarray:
    """Section 3.1.2, Algorithm 4: the rows of C split statically over threads.

    Bit-identical to :func:`gemm`; only the wall time differs.
    """
    A, B = _f64(A), _f64(B)
    _check2(A, B)
    m, k = A.shape
    n = B.shape[1]
    C = np.empty((m, n), dtype=np.float64)
    t = threads or max_threads()
    _load().oracle_gemm_f64_omp(m, n, k, _ptr(A), k, _ptr(B), n, _ptr(C), n, int(t))
    return C


def gemm_entries(A, B, rows, cols) -> np.ndarray:
    """Entries C[rows[t], cols[t]] of A*B, bit-identical to :func:`gemm`."""
    A, B = _f64(A), _f64(B)
    _check2(A, B)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    if r.shape != c.shape:
        raise ValueError("rows/cols length mismatch")
    if r.size and (r.min() < 0 or r.max() >= A.shape[0] or c.min() < 0 or c.max() >= B.shape[1]):
        raise IndexError("entry index out of range")
    out = np.empty(r.shape, dtype=np.float64)
    k = A.shape[1]
    _load().oracle_gemm_entries_f64(k, _ptr(A), k, _ptr(B), B.shape[1],
                                    _ptr(r), _ptr(c), r.size, _ptr(out))
    return out


def max_threads() -> int:
    return int(_load().oracle_max_threads())


# ---------------------------------------------------------------- bfloat16

def bf16_rne(x) -> np.ndarray:
    """binary32 -> bfloat16 bit patterns (uint16), round to nearest, ties even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.uint16)
    _load().oracle_bf16_rne_array(x.size, _ptr(x), _ptr(out))
    return out


def bf16_to_f32(h) -> np.ndarray:
    """bfloat16 bit patterns -> the binary32 values they denote (exact)."""
    h = np.asarray(h, dtype=np.uint16)
    return (h.astype(np.uint32) << 16).view(np.float32)


def split_bf16(x):
    """Two-term split: hi = bf16(x), lo = bf16(x - hi). Returns uint16 planes."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    hi = np.empty(x.shape, dtype=np.uint16)
    lo = np.empty(x.shape, dtype=np.uint16)
    _load().oracle_split_bf16(x.size, _ptr(x), _ptr(hi), _ptr(lo))
    return hi, lo


def split_emul_gemm(A, B) -> np.ndarray:
    """What the three-term split product computes, with exact binary64 sums.

    A_hi*B_hi + A_hi*B_lo + A_lo*B_hi (the lo*lo term is dropped). Each
    term is this module's binary64 product of bfloat16-valued operands, so
    the result isolates the representation error of the split from the
    accumulation error of the device.
    """
    ahi, alo = (bf16_to_f32(p) for p in split_bf16(A))
    bhi, blo = (bf16_to_f32(p) for p in split_bf16(B))
    return gemm(ahi, bhi) + gemm(ahi, blo) + gemm(alo, bhi)


def split3_bf16(x):
    """Three-term split: hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi -
    mid). Returns uint16 planes."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    hi = np.empty(x.shape, dtype=np.uint16)
    mid = np.empty(x.shape, dtype=np.uint16)
    lo = np.empty(x.shape, dtype=np.uint16)
    _load().oracle_split3_bf16(x.size, _ptr(x), _ptr(hi), _ptr(mid), _ptr(lo))
    return hi, mid, lo


def split3_emul_gemm(A, B) -> np.ndarray:
    """What the six-term split product computes, with exact binary64 sums.

    A_lo*B_hi + A_hi*B_lo + A_mid*B_mid + A_mid*B_hi + A_hi*B_mid + A_hi*B_hi
    (mid*lo, lo*mid and lo*lo dropped), each term this module's binary64
    product of bfloat16-valued operands.
    """
    ahi, amid, alo = (bf16_to_f32(p) for p in split3_bf16(A))
    bhi, bmid, blo = (bf16_to_f32(p) for p in split3_bf16(B))
    return (gemm(alo, bhi) + gemm(ahi, blo) + gemm(amid, bmid) + gemm(amid, bhi)
            + gemm(ahi, bmid) + gemm(ahi, bhi))


# ------------------------------------------------------------- backward

def loss_and_grads(A, B, W):
    """L = sum(W (.) (A*B)); dA = W*B^T; dB = A^T*W, all in binary64.

    L is bilinear, so these are its exact partial derivatives. The transposes
    are explicit copies and the products are :func:`gemm`.
    """
    A, B, W = _f64(A), _f64(B), _f64(W)
    C = gemm(A, B)
    L = float(np.sum(W * C))
    dA = gemm(W, np.ascontiguousarray(B.T))
    dB = gemm(np.ascontiguousarray(A.T), W)
    return L, dA, dB


# ------------------------------------------------------- error and counts

def relerr_fro(C, Cref) -> float:
    """Normwise relative error ||C - Cref||_F / ||Cref||_F in binary64."""
    C, Cref = _f64(C), _f64(Cref)
    den = float(np.sqrt(np.sum(Cref * Cref)))
    num = float(np.sqrt(np.sum((C - Cref) ** 2)))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den


def relerr_sampled(vals, ref) -> float:
    """Normwise relative error over a sample of entries (same definition)."""
    return relerr_fro(np.asarray(vals).reshape(-1, 1), np.asarray(ref).reshape(-1, 1))


def flops_paper(n: int) -> int:
    """Section 3.1: N multiplications and N-1 additions per entry, N^2 entries."""
    n = int(n)
    return n * n * (2 * n - 1)


def flops_2n3(n: int) -> int:
    """The large-N form 2N^3 of the Section 3.1 count (exact Python integer)."""
    n = int(n)
    return 2 * n * n * n


def flops_mnk(m: int, n: int, k: int) -> int:
    """2*m*n*k for a rectangular product (m x k times k x n)."""
    return 2 * int(m) * int(n) * int(k)


def mflops(ops: float, seconds: float) -> float:
    """Algorithm 2 / Algorithm 4: rate = ops / t / 10^6."""
    return float(ops) / float(seconds) / 1.0e6


def row_partition(rows: int, numworkers: int):
    """Section 3.1.1, Algorithm 2: row split of A over workers 1..numworkers.

    averow = rows / numworkers, extra = rows % numworkers; worker ``dest``
    gets averow + 1 rows when dest <= extra, else averow; offsets are the
    running sum. Returns a list of (dest, offset, rows) tuples.
    """
    if numworkers <= 0:
        raise ValueError("numworkers must be positive")
    averow, extra = divmod(int(rows), int(numworkers))
    out, offset = [], 0
    for dest in range(1, numworkers + 1):
        r = averow + 1 if dest <= extra else averow
        out.append((dest, offset, r))
        offset += r
    return out
