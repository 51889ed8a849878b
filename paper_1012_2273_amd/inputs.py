"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random matrices and problem lists and nothing else: it
holds none of the product's arithmetic. The paper fills A and B with RAND()
before the timer starts (Section 3.1.1 Algorithm 2, Section 3.1.2 Algorithm 4)
without naming a distribution; the recipes here are:

* ``uniform``: i.i.d. uniform [-1, 1], A drawn before B (then W), row-major.
* ``integers``: i.i.d. uniform over the integers -8..8 (exact in bfloat16,
  and every sum of N <= 8192 products stays below 2^24 in magnitude, so the
  product is exact in binary32 and binary64 whatever the summation order).
* ``row_scaled``: each row normalised to unit 2-norm and then scaled by
  10^u, u ~ U(-3, 3), in binary64 before rounding to binary32 (row norms
  spread log-uniformly over 1e-3 .. 1e3).
* ``batch_sizes``: N_i = rint(exp(U(ln 10, ln 2000))), clipped to [10, 2000].
* ``hashed_integers``: integers -8..8 addressed by (row, column): entry (i, j)
  is the SplitMix64 output function (Steele, Lea and Flood, 2014) of the
  counter salt * 0x9E3779B97F4A7C15 + i * 2^32 + j, reduced mod 17 and
  shifted by -8. Any set of rows or columns of an arbitrarily large matrix
  can be regenerated without drawing the rest (used for operands of several
  GiB whose sampled outputs are checked).

Seeds: ``seed_for(cfg, n, variant)`` = 1_000_000*cfg + n (+500_000 for the
variant); generator PCG64.
"""
from __future__ import annotations

import numpy as np


def seed_for(cfg: int, n: int, variant: bool = False) -> int:
    return 1_000_000 * int(cfg) + int(n) + (500_000 if variant else 0)


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(shape, seed, dtype=np.float64, count: int = 2):
    """``count`` arrays of i.i.d. U[-1, 1] values, drawn in order."""
    g = _rng(seed)
    return tuple(g.uniform(-1.0, 1.0, size=shape).astype(dtype) for _ in range(count))


def uniform_square(n: int, seed, dtype=np.float64):
    """A, B: n x n, U[-1, 1]."""
    return uniform((n, n), seed, dtype, 2)


def uniform_mnk(m: int, n: int, k: int, seed, dtype=np.float64):
    """A: m x k, B: k x n, U[-1, 1] (rectangular problems)."""
    g = _rng(seed)
    A = g.uniform(-1.0, 1.0, size=(m, k)).astype(dtype)
    B = g.uniform(-1.0, 1.0, size=(k, n)).astype(dtype)
    return A, B


def integers(shape, seed, dtype=np.float64, count: int = 2, lo: int = -8, hi: int = 8):
    """``count`` arrays with i.i.d. integer entries in [lo, hi], as floats."""
    g = _rng(seed)
    return tuple(g.integers(lo, hi, size=shape, endpoint=True).astype(dtype)
                 for _ in range(count))


def integer_square(n: int, seed, dtype=np.float64):
    return integers((n, n), seed, dtype, 2)


def row_scaled(n: int, seed, dtype=np.float32):
    """A, B: n x n with U[-1,1] directions and row norms 10^U(-3,3)."""
    g = _rng(seed)
    out = []
    for _ in range(2):
        X = g.uniform(-1.0, 1.0, size=(n, n))
        norms = np.sqrt(np.sum(X * X, axis=1, keepdims=True))
        scale = 10.0 ** g.uniform(-3.0, 3.0, size=(n, 1))
        out.append((X / norms * scale).astype(dtype))
    return tuple(out)


def batch_sizes(count: int, seed, lo: int = 10, hi: int = 2000) -> np.ndarray:
    """Square sizes log-uniform in [lo, hi]."""
    g = _rng(seed)
    u = g.uniform(np.log(lo), np.log(hi), size=count)
    return np.clip(np.rint(np.exp(u)), lo, hi).astype(np.int64)


def batch_problem(i: int, n: int, base_seed: int, dtype=np.float64):
    """A_i, B_i for problem i of a batch: U[-1,1], stream SeedSequence([base, i])."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(base_seed), int(i)])))
    A = g.uniform(-1.0, 1.0, size=(n, n)).astype(dtype)
    B = g.uniform(-1.0, 1.0, size=(n, n)).astype(dtype)
    return A, B


def special(kind: str, n: int, seed=0, dtype=np.float64):
    """Structured matrices for exactness checks: identity, permutation, diagonal."""
    g = _rng(seed)
    if kind == "identity":
        return np.eye(n, dtype=dtype)
    if kind == "permutation":
        P = np.zeros((n, n), dtype=dtype)
        P[np.arange(n), g.permutation(n)] = 1.0
        return P
    if kind == "diagonal":
        return np.diag(g.integers(-8, 8, size=n, endpoint=True).astype(dtype))
    raise ValueError(kind)


_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on uint64 arrays (wrapping arithmetic)."""
    z = z + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def hashed_integers(rows, cols, salt: int) -> np.ndarray:
    """Entries (rows[a], cols[b]) of the addressable integer matrix of the
    given salt (see the module docstring), as a len(rows) x len(cols)
    float64 array; ``cols`` may be an int n for columns 0..n-1."""
    r = np.asarray(rows, dtype=np.uint64).reshape(-1, 1)
    c = (np.arange(cols, dtype=np.uint64) if np.isscalar(cols) else
         np.asarray(cols, dtype=np.uint64)).reshape(1, -1)
    with np.errstate(over="ignore"):
        base = np.uint64(salt) * np.uint64(0x9E3779B97F4A7C15)
        z = _splitmix64(base + (r << np.uint64(32)) + c)
    return (z % np.uint64(17)).astype(np.int64).astype(np.float64) - 8.0
