"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module holds none of the method's arithmetic: it only draws random
matrices (numpy ``Generator(PCG64(seed))``) and builds test matrices with a
prescribed singular value decomposition, A = Q diag(s) V^T, so that the exact
polar factors U = Q V^T and H = V diag(s) V^T are known (eqs. SVD, SVDdef of
section III.D).  The paper does not say which matrices its benchmarks used, so
these recipes *are* the workloads:

* GEMM operands: i.i.d. N(0, 1) entries, drawn directly in float32.
* Polar inputs: Q, V Haar-distributed (QR of a seeded Gaussian, columns
  multiplied by the signs of diag(R)); s_1 = 1, s_n = lo, the rest i.i.d.
  log-uniform in [lo, 1], so cond(A) = 1/lo exactly before rounding to FP32.
* Serving stream: Poisson arrivals, n log-uniform in [128, 4096] rounded to a
  multiple of 64, cond = 10^U(1, 6).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian(shape, seed: int, dtype=np.float32) -> np.ndarray:
    """i.i.d. N(0, 1) entries of the given dtype."""
    return rng(seed).standard_normal(size=shape, dtype=dtype)


def integer_matrix(shape, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Small-integer float32 entries (products and sums stay exact in FP32)."""
    return rng(seed).integers(lo, hi + 1, size=shape).astype(np.float32)


def haar(n: int, seed: int) -> np.ndarray:
    """Haar-distributed n x n orthogonal matrix in float64."""
    return column_orthonormal(n, n, seed)


def column_orthonormal(m: int, n: int, seed: int) -> np.ndarray:
    """m x n matrix with Haar-distributed orthonormal columns (float64)."""
    g = rng(seed).standard_normal(size=(m, n))
    q, r = np.linalg.qr(g, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def singular_values(n: int, lo: float, seed: int) -> np.ndarray:
    """s_1 = 1, s_n = lo, the others i.i.d. log-uniform in [lo, 1], descending."""
    if n == 1:
        return np.ones(1)
    s = np.exp(rng(seed).uniform(np.log(lo), 0.0, size=n))
    s[0] = 1.0
    s[-1] = lo
    s[1:-1] = np.sort(s[1:-1])[::-1]
    return s


@dataclass
class PolarCase:
    """A = Q diag(s) V^T with its exact factors (float64) and A rounded to FP32."""

    A32: np.ndarray  # m x n float32, the actual input
    Q: np.ndarray    # m x n float64, orthonormal columns
    s: np.ndarray    # n float64
    V: np.ndarray    # n x n float64, orthogonal

    @property
    def U_exact(self) -> np.ndarray:
        return self.Q @ self.V.T

    @property
    def H_exact(self) -> np.ndarray:
        return (self.V * self.s[None, :]) @ self.V.T

    @property
    def A64(self) -> np.ndarray:
        return (self.Q * self.s[None, :]) @ self.V.T


def polar_case(m: int, n: int, lo: float, seeds=(103, 104, 105)) -> PolarCase:
    """Polar test matrix with prescribed singular values in [lo, 1]."""
    Q = column_orthonormal(m, n, seeds[0])
    V = haar(n, seeds[1])
    s = singular_values(n, lo, seeds[2])
    A = ((Q * s[None, :]) @ V.T).astype(np.float32)
    return PolarCase(A, Q, s, V)


@dataclass
class ServeRequest:
    t_arrival: float  # seconds after stream start
    n: int
    cond: float
    pool_index: int


def serve_sizes(count: int, seed: int, n_lo: int = 128, n_hi: int = 4096) -> np.ndarray:
    """n = 64 * round(exp(U(ln n_lo, ln n_hi)) / 64), clipped to [n_lo, n_hi]."""
    g = rng(seed)
    x = np.exp(g.uniform(np.log(n_lo), np.log(n_hi), size=count))
    n = 64 * np.rint(x / 64.0)
    return np.clip(n, n_lo, n_hi).astype(np.int64)


def serve_stream(rate: float, duration: float, seed: int, pool_size: int,
                 n_lo: int = 128, n_hi: int = 4096):
    """Poisson arrivals at `rate` req/s over `duration` s; each picks a pool entry."""
    g = rng(seed)
    t = 0.0
    out = []
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append(t)
    idx = g.integers(0, pool_size, size=len(out))
    return [(ti, int(ii)) for ti, ii in zip(out, idx)]


def serve_pool(pool_size: int, seed: int, n_lo: int = 128, n_hi: int = 4096):
    """Pool of square polar cases: sizes log-uniform, cond = 10^U(1, 6)."""
    g = rng(seed)
    sizes = serve_sizes(pool_size, seed + 1, n_lo, n_hi)
    conds = 10.0 ** g.uniform(1.0, 6.0, size=pool_size)
    cases = []
    for i, (n, c) in enumerate(zip(sizes, conds)):
        base = seed * 1000 + 3 * i
        cases.append(polar_case(int(n), int(n), 1.0 / float(c), (base, base + 1, base + 2)))
    return cases


def polar_case_torch(m: int, n: int, lo: float, seeds, device="cuda", progress=None):
    """Same recipe as polar_case (A = Q diag(s) V^T, Haar Q and V from the QR
    of seeded numpy Gaussians, sign-fixed), with the QR and the product done
    in float64 by torch on `device` so that large sizes are practical.
    progress, if given, is called with a short message after each factor.
    Returns (A32 host float32, Q dev float64, s host float64, V dev float64)."""
    import torch

    def done(what):
        if progress is not None:
            progress(what)

    def orth(rows, cols, seed):
        g = torch.from_numpy(rng(seed).standard_normal(size=(rows, cols))).to(device)
        q, r = torch.linalg.qr(g, mode="reduced")
        d = torch.sign(torch.diagonal(r))
        d[d == 0] = 1.0
        return q * d[None, :]

    Q = orth(m, n, seeds[0])
    done(f"Q {m}x{n}")
    V = orth(n, n, seeds[1])
    done(f"V {n}x{n}")
    s = singular_values(n, lo, seeds[2])
    sd = torch.from_numpy(s).to(device)
    A = ((Q * sd[None, :]) @ V.T.contiguous()).to(torch.float32).cpu().numpy()
    done(f"A {m}x{n}")
    return A, Q, s, V
