"""Seeded synthetic inputs for the log-determinant workloads.

This module is shared by the oracle side (tests, expected-value scripts) and
the GPU side (tests, bench).  It holds none of the condensation arithmetic:
only random draws and the Gram products that define the covariance inputs.

Workloads (sizes and distributions follow the paper's dense FP64 matrices of
Section 3, which leaves the distribution unstated, and the covariance use
named in the Abstract):

* ``uniform(n, seed)``   -- i.i.d. U[-1, 1] entries.
* ``normal(n, seed)``    -- i.i.d. N(0, 1) entries.
* ``wishart(n, rng)``    -- A = X^T X / m + 1e-3 I, X of shape (m, n) with
  i.i.d. N(0, 1) entries and m = 2n, symmetrised as (A + A^T)/2.
* ``wishart_batch``      -- sizes drawn uniformly in [lo, hi] from one
  generator, then one Wishart matrix per size from the same generator.

All generators use ``numpy.random.default_rng(seed)`` (PCG64).  Large draws
are made in row chunks, which yields the same stream as a single draw.
"""

from __future__ import annotations

import numpy as np

RIDGE = 1e-3


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform(n: int, seed: int) -> np.ndarray:
    """Dense n x n FP64 matrix, entries i.i.d. U[-1, 1]."""
    return rng(seed).uniform(-1.0, 1.0, size=(n, n))


def normal(n: int, seed: int) -> np.ndarray:
    """Dense n x n FP64 matrix, entries i.i.d. N(0, 1)."""
    g = rng(seed)
    out = np.empty((n, n), dtype=np.float64)
    chunk = max(1, (1 << 24) // max(n, 1))
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        out[r0:r1] = g.standard_normal((r1 - r0, n))
    return out


def wishart_from(g: np.random.Generator, n: int, m_factor: int = 2,
                 ridge: float = RIDGE, gram=None) -> np.ndarray:
    """A = X^T X / m + ridge * I with X (m x n) ~ N(0,1), m = m_factor * n.

    ``gram`` (optional) computes X^T X for a float64 array X; the default is
    numpy.  Only the product differs between callers, never the draws.
    """
    m = m_factor * n
    x = np.empty((m, n), dtype=np.float64)
    chunk = max(1, (1 << 24) // max(n, 1))
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        x[r0:r1] = g.standard_normal((r1 - r0, n))
    a = gram(x) if gram is not None else x.T @ x
    a = np.asarray(a, dtype=np.float64)
    a /= m
    a = 0.5 * (a + a.T)
    a[np.diag_indices(n)] += ridge
    return a


def wishart(n: int, seed: int, m_factor: int = 2, ridge: float = RIDGE,
            gram=None) -> np.ndarray:
    return wishart_from(rng(seed), n, m_factor, ridge, gram)


def wishart_batch(count: int, lo: int, hi: int, seed: int,
                  m_factor: int = 2, ridge: float = RIDGE, gram=None):
    """Sizes ~ U{lo..hi} then one Wishart matrix per size, one stream."""
    g = rng(seed)
    sizes = g.integers(lo, hi + 1, count)
    mats = [wishart_from(g, int(n), m_factor, ridge, gram) for n in sizes]
    return [int(n) for n in sizes], mats


def int_matrix(n: int, seed: int, lo: int = -9, hi: int = 9) -> np.ndarray:
    """Integer-valued matrix (stored as FP64) with entries in [lo, hi]."""
    return rng(seed).integers(lo, hi + 1, size=(n, n)).astype(np.float64)


def householder_qd(n: int, seed: int, reflectors: int, dlo: float = 0.5,
                   dhi: float = 2.0, neg_frac: float = 0.5):
    """A = H_1 ... H_r diag(d): a matrix with a closed-form determinant.

    Returns (A, d, r).  Each H = I - 2 v v^T / (v^T v) has determinant -1,
    so det A = (-1)^r * prod(d).  |d_i| ~ U[dlo, dhi], a fraction of the
    d_i negated.
    """
    g = rng(seed)
    d = g.uniform(dlo, dhi, n)
    d[g.random(n) < neg_frac] *= -1.0
    a = np.diag(d).astype(np.float64)
    for _ in range(reflectors):
        v = g.standard_normal(n)
        v /= np.linalg.norm(v)
        # H a = a - 2 v (v^T a)
        a -= 2.0 * np.outer(v, v @ a)
    return a, d, reflectors


# Workload table: the five benchmark configurations, by name.
CONFIGS = {
    "uniform_n1000": dict(kind="uniform", n=1000, seed=1),
    "normal_n8000": dict(kind="normal", n=8000, seed=2),
    "normal_n8192": dict(kind="normal", n=8192, seed=2),
    "wishart_n16384": dict(kind="wishart", n=16384, seed=3),
    "wishart_batch512": dict(kind="wishart_batch", count=512, lo=32, hi=1024, seed=4),
    "wishart_batch64": dict(kind="wishart_batch", count=64, lo=256, hi=2048, seed=5),
}


def make(name: str, **kw):
    c = dict(CONFIGS[name])
    c.update(kw)
    kind = c.pop("kind")
    if kind == "uniform":
        return uniform(c["n"], c["seed"])
    if kind == "normal":
        return normal(c["n"], c["seed"])
    if kind == "wishart":
        return wishart(c["n"], c["seed"], gram=c.get("gram"))
    if kind == "wishart_batch":
        return wishart_batch(c["count"], c["lo"], c["hi"], c["seed"],
                             gram=c.get("gram"))
    raise KeyError(kind)
