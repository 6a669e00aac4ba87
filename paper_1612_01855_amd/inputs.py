"""Seeded synthetic inputs for L X = B.

This module holds no arithmetic of the solver: it only draws matrices.  Both
the GPU tests/benchmark and the CPU oracle read the very same arrays produced
here.  Every generator takes an explicit seed and uses numpy's PCG64, drawing
in a fixed order so that one seed fixes every byte.

Workload families (the paper itself runs no experiments; these stand in for
its problem statement, an n x n lower-triangular L and a dense n x k B):

* ``easy_lower``  -- diagonal ~ U[1,2], strict lower ~ U[-1,1]/n.  Strictly
  row-diagonally dominant, so cond(L) is small (a handful).
* ``chol_lower``  -- L = chol(G G^T / m + I), G ~ N(0,1) of size n x m,
  m = 2n by default.  A well conditioned Cholesky factor.
* ``hard_lower``  -- L = chol(G G^T / m + eps I) with G of size n x n/2 (so
  G G^T has rank n/2) and eps = 1e-12 * ||G G^T / m||_2: cond_2(A) ~ 1e12,
  hence cond_2(L) ~ 1e6.
* ``spd`` / ``spd_on`` -- the symmetric positive definite A = G G^T / m + I
  (or + eps I) behind the Cholesky factors, the input of the factorization.
* ``diag_dominant`` -- nonsymmetric, strictly column diagonally dominant
  matrices: the input of the LU factorization without row exchanges.
* ``rhs``         -- B ~ N(0,1).
* closed-form matrices used as pins (identity, diagonal, bidiagonal,
  all-ones lower triangle, random integer unit-lower).
* ``serving_factors`` / ``request_stream`` -- the serving mix: factor sizes
  log-uniform in [64, 4096], request widths log-uniform in [1, 512], Poisson
  arrivals.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _fill_upper(L: np.ndarray, upper: Optional[float]) -> np.ndarray:
    """Write ``upper`` strictly above the diagonal (NaN proves it is unread)."""
    if upper is not None:
        for i in range(L.shape[0] - 1):
            L[i, i + 1:] = upper
    return L


def easy_lower(n: int, seed: int, upper: Optional[float] = 0.0) -> np.ndarray:
    """Diagonal ~ U[1,2], strict lower ~ U[-1,1]/n (float64, row-major)."""
    g = rng(seed)
    d = g.uniform(1.0, 2.0, size=n)
    L = g.uniform(-1.0, 1.0, size=(n, n))
    L *= 1.0 / max(n, 1)
    L = np.tril(L, -1)
    L[np.arange(n), np.arange(n)] = d
    return _fill_upper(L, upper)


def rhs(n: int, k: int, seed: int) -> np.ndarray:
    """B ~ N(0,1), n x k float64."""
    return rng(seed + 0x5EED).standard_normal(size=(n, k))


def easy_system(n: int, k: int, seed: int, upper: Optional[float] = 0.0):
    return easy_lower(n, seed, upper), rhs(n, k, seed)


def chol_lower(n: int, seed: int, m: Optional[int] = None,
               upper: Optional[float] = 0.0) -> np.ndarray:
    """L = chol(G G^T / m + I), G ~ N(0,1) n x m (m = 2n by default)."""
    m = 2 * n if m is None else m
    g = rng(seed)
    G = g.standard_normal(size=(n, m))
    A = G @ G.T
    A *= 1.0 / m
    A[np.arange(n), np.arange(n)] += 1.0
    del G
    L = np.linalg.cholesky(A)
    return _fill_upper(np.ascontiguousarray(L), upper)


def hard_lower(n: int, seed: int, upper: Optional[float] = 0.0,
               ratio: float = 1e-12) -> np.ndarray:
    """L = chol(G G^T / m + eps I), G ~ N(0,1) n x m, m = max(n//2, 1),
    eps = ratio * lambda_max(G G^T / m) (lambda_max by 50 seeded power
    iterations).  cond_2(L) ~ ratio^{-1/2}."""
    m = max(n // 2, 1)
    g = rng(seed)
    G = g.standard_normal(size=(n, m))
    A = G @ G.T
    A *= 1.0 / m
    v = g.standard_normal(size=n)
    lam = 0.0
    for _ in range(50):
        w = A @ v
        lam = float(np.linalg.norm(w))
        v = w / lam
    A[np.arange(n), np.arange(n)] += ratio * lam
    L = np.linalg.cholesky(A)
    return _fill_upper(np.ascontiguousarray(L), upper)


def chol_lower_on(torch, device, n: int, seed: int, m: Optional[int] = None,
                  ratio: Optional[float] = None):
    """The Cholesky-family factors at sizes where forming G G^T on the host is
    slow: the same seeded G as chol_lower / hard_lower (host generator), the
    product and the factorisation done by torch on `device`.  ratio=None gives
    chol_lower's A = G G^T / m + I (m = 2n by default); a ratio gives
    hard_lower's A = G G^T / m + ratio * lambda_max I (m = n/2 by default,
    lambda_max by 50 seeded power iterations).  Returns a float64 tensor on
    `device`, zeros above the diagonal.  The rounding of the product differs
    from the host versions, so the factor is not bit-identical to them."""
    if m is None:
        m = 2 * n if ratio is None else max(n // 2, 1)
    g = rng(seed)
    G = torch.from_numpy(g.standard_normal(size=(n, m))).to(device)
    A = G @ G.t().contiguous()
    del G
    A *= 1.0 / m
    if ratio is None:
        A.diagonal().add_(1.0)
    else:
        v = torch.from_numpy(g.standard_normal(size=n)).to(device)
        lam = 0.0
        for _ in range(50):
            w = A @ v
            lam = float(torch.linalg.norm(w).item())
            v = w / lam
        A.diagonal().add_(ratio * lam)
    L = torch.linalg.cholesky(A)
    del A
    return L.tril_().contiguous()


def spd(n: int, seed: int, m: Optional[int] = None) -> np.ndarray:
    """A = G G^T / m + I, G ~ N(0,1) n x m (m = 2n by default): the symmetric
    positive definite matrix whose Cholesky factor chol_lower returns (same
    seed, same G).  Full symmetric float64, row-major."""
    m = 2 * n if m is None else m
    g = rng(seed)
    G = g.standard_normal(size=(n, m))
    A = G @ G.T
    A *= 1.0 / m
    A[np.arange(n), np.arange(n)] += 1.0
    return np.ascontiguousarray(A)


def spd_on(torch, device, n: int, seed: int, m: Optional[int] = None,
           ratio: Optional[float] = None):
    """The symmetric positive definite matrices behind chol_lower_on, formed
    by torch on `device` from the same seeded G: A = G G^T / m + I
    (ratio=None, m = 2n by default) or A = G G^T / m + ratio * lambda_max I
    (m = n/2 by default; cond_2(A) ~ 1/ratio).  A float64 tensor, full
    symmetric (the product's two triangles are computed separately, so they
    may differ in the last bit)."""
    if m is None:
        m = 2 * n if ratio is None else max(n // 2, 1)
    g = rng(seed)
    G = torch.from_numpy(g.standard_normal(size=(n, m))).to(device)
    A = G @ G.t().contiguous()
    del G
    A *= 1.0 / m
    if ratio is None:
        A.diagonal().add_(1.0)
    else:
        v = torch.from_numpy(g.standard_normal(size=n)).to(device)
        lam = 0.0
        for _ in range(50):
            w = A @ v
            lam = float(torch.linalg.norm(w).item())
            v = w / lam
        A.diagonal().add_(ratio * lam)
    return A


def int_lower_positive(n: int, seed: int, lo: int = -2, hi: int = 2,
                       dmax: int = 3) -> np.ndarray:
    """Integer lower-triangular matrix: diagonal in {1..dmax}, strict lower
    entries in {lo..hi}, zeros above.  A = L L^T then has integer entries and
    L is its Cholesky factor exactly."""
    g = rng(seed)
    L = np.tril(g.integers(lo, hi + 1, size=(n, n)), -1).astype(np.float64)
    L[np.arange(n), np.arange(n)] = g.integers(1, dmax + 1, size=n)
    return L


def diag_dominant(n: int, seed: int, margin: float = 1.0) -> np.ndarray:
    """Nonsymmetric A with entries ~ U[-1, 1] off the diagonal and a_jj =
    sign * (margin + sum_{i != j} |a_ij|) (random sign): strictly column
    diagonally dominant, so elimination without row exchanges is stable and
    partial pivoting would not exchange any row."""
    g = rng(seed)
    A = g.uniform(-1.0, 1.0, size=(n, n))
    A[np.arange(n), np.arange(n)] = 0.0
    col = np.abs(A).sum(axis=0)
    sign = np.where(g.uniform(size=n) < 0.5, -1.0, 1.0)
    A[np.arange(n), np.arange(n)] = sign * (margin + col)
    return np.ascontiguousarray(A)


def diag_dominant_on(torch, device, n: int, seed: int, margin: float = 1.0):
    """diag_dominant's construction at sizes where the host generator is slow:
    off-diagonal entries ~ U[-1, 1] from torch's seeded generator on `device`,
    a_jj = margin + sum_{i != j} |a_ij| (positive diagonal).  A float64
    tensor; not bit-identical to the host version (a different stream of
    random numbers)."""
    g = torch.Generator(device=device).manual_seed(seed)
    A = torch.rand((n, n), generator=g, dtype=torch.float64, device=device) * 2.0 - 1.0
    A.diagonal().zero_()
    A.diagonal().add_(A.abs().sum(dim=0) + margin)
    return A


def int_unit_lower_small(n: int, seed: int, lo: int = -2, hi: int = 2) -> np.ndarray:
    """Unit lower-triangular integer matrix, strict lower entries in {lo..hi}."""
    g = rng(seed)
    L = np.tril(g.integers(lo, hi + 1, size=(n, n)), -1).astype(np.float64)
    L[np.arange(n), np.arange(n)] = 1.0
    return L


def int_upper_pow2(n: int, seed: int, lo: int = -2, hi: int = 2) -> np.ndarray:
    """Upper-triangular integer matrix with diagonal entries +-1, +-2 or +-4 and
    strict upper entries in {lo..hi}: A = L U for an integer unit-lower L is an
    integer matrix whose no-pivoting LU divisions are exact."""
    g = rng(seed)
    U = np.triu(g.integers(lo, hi + 1, size=(n, n)), 1).astype(np.float64)
    U[np.arange(n), np.arange(n)] = g.choice([-4.0, -2.0, -1.0, 1.0, 2.0, 4.0], size=n)
    return U


# ---- closed-form matrices (pins) -------------------------------------------

def identity(n: int) -> np.ndarray:
    return np.eye(n)


def diagonal(n: int, seed: int) -> np.ndarray:
    d = rng(seed).uniform(0.5, 4.0, size=n)
    return np.diag(d)


def bidiagonal_minus_one(n: int) -> np.ndarray:
    """Unit lower bidiagonal with -1 on the subdiagonal.  Its inverse is the
    all-ones lower triangle, so X is the column-wise prefix sum of B."""
    L = np.eye(n)
    if n > 1:
        L[np.arange(1, n), np.arange(n - 1)] = -1.0
    return L


def ones_lower(n: int) -> np.ndarray:
    """All-ones lower triangle.  Its inverse is unit lower bidiagonal with -1
    on the subdiagonal, so X_i = B_i - B_{i-1}."""
    return np.tril(np.ones((n, n)))


def int_unit_lower(n: int, seed: int, density: float = 0.5) -> np.ndarray:
    """Unit lower-triangular matrix with strict-lower entries in {-1, 0, 1}.
    det = 1, so the inverse is an integer matrix."""
    g = rng(seed)
    vals = g.choice(np.array([-1.0, 0.0, 1.0]), size=(n, n),
                    p=[density / 2, 1.0 - density, density / 2])
    L = np.tril(vals, -1)
    L[np.arange(n), np.arange(n)] = 1.0
    return L


def int_rhs(n: int, k: int, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    return rng(seed + 77).integers(lo, hi + 1, size=(n, k)).astype(np.float64)


# ---- serving mix -----------------------------------------------------------

def log_uniform_int(g: np.random.Generator, lo: int, hi: int, size=None):
    """round(exp(U(ln lo, ln hi))) clamped to [lo, hi]."""
    u = g.uniform(math.log(lo), math.log(hi), size=size)
    v = np.rint(np.exp(u)).astype(np.int64)
    return np.clip(v, lo, hi)


def serving_factor_sizes(count: int, seed: int, nmin: int = 64,
                         nmax: int = 4096) -> np.ndarray:
    return log_uniform_int(rng(seed), nmin, nmax, size=count)


@dataclass
class Request:
    t_arrival: float   # seconds after the stream starts
    factor: int        # index of the resident L
    k: int             # number of right-hand sides
    seed: int          # seed of its B


def request_stream(num: int, rate_hz: float, num_factors: int, seed: int,
                   kmin: int = 1, kmax: int = 512) -> List[Request]:
    """Poisson arrivals (exponential gaps with mean 1/rate), each request
    picks its factor uniformly and k log-uniform in [kmin, kmax]."""
    g = rng(seed + 991)
    gaps = g.exponential(1.0 / rate_hz, size=num)
    t = np.cumsum(gaps)
    fac = g.integers(0, num_factors, size=num)
    ks = log_uniform_int(g, kmin, kmax, size=num)
    return [Request(float(t[i]), int(fac[i]), int(ks[i]), seed * 1000003 + i)
            for i in range(num)]
