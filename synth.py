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
  i.i.d. N(0, 1) entries and m = 2n.  The draws are rounded to multiples of
  2^-12 (and clipped to |x| <= 8, which a draw passes with probability
  1 - 1e-15), so every product x_ki x_kj is a multiple of 2^-24 below 2^6
  and any sum of up to 2^15 of them is exact in FP64: X^T X comes out the
  same bytes on any host or device and in any summation order.  The
  division by m and the ridge are single IEEE operations.
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


GRID = 1.0 / 4096.0  # spacing of the Wishart draws (2^-12)
CLIP = 8.0


def wishart_from(g: np.random.Generator, n: int, m_factor: int = 2,
                 ridge: float = RIDGE, gram=None) -> np.ndarray:
    """A = X^T X / m + ridge * I with X (m x n) ~ N(0,1) on the 2^-12 grid,
    m = m_factor * n.

    ``gram`` (optional) computes X^T X for a float64 array X; the default is
    numpy.  On the grid the product is exact, so every caller gets the same
    bytes; only where it runs differs.
    """
    m = m_factor * n
    if m > (1 << 15):
        raise ValueError("the exact-Gram bound holds for m <= 2^15 rows")
    x = np.empty((m, n), dtype=np.float64)
    chunk = max(1, (1 << 24) // max(n, 1))
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        d = g.standard_normal((r1 - r0, n))
        np.clip(d, -CLIP, CLIP, out=d)
        x[r0:r1] = np.round(d / GRID) * GRID
    a = gram(x) if gram is not None else x.T @ x
    a = np.asarray(a, dtype=np.float64)
    a /= m
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


def unimodular_ties(n: int, seed: int, reach: int = 0) -> np.ndarray:
    """A totally unimodular n x n matrix with |det| = 1 and many exact ties.

    Built as D1 P U Q D2: U upper triangular with ones on the diagonal and
    row i holding ones on columns i .. r_i (an interval, r_i - i uniform in
    0 .. reach, reach = n // 4 by default), P and Q random permutations and
    D1, D2 random +-1 diagonals.  Interval matrices are totally unimodular,
    and permutations and sign changes keep that, as does pivoting on a +-1
    entry, so every condensed row holds only -1, 0 and 1: each pivot is +-1
    and is tied with every other non-zero of its row.  The arithmetic is
    exact in any floating-point format and any summation order.
    """
    g = rng(seed)
    reach = max(1, n // 4) if reach <= 0 else reach
    u = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        r = min(n - 1, i + int(g.integers(0, reach + 1)))
        u[i, i:r + 1] = 1.0
    p = g.permutation(n)
    q = g.permutation(n)
    d1 = np.where(g.random(n) < 0.5, -1.0, 1.0)
    d2 = np.where(g.random(n) < 0.5, -1.0, 1.0)
    return (d1[:, None] * u[p][:, q]) * d2[None, :]


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


def gmm(k: int, d: int, m: int, seed: int):
    """A Gaussian mixture and points to score (the model-mixture use of the
    Abstract): weights pi ~ U[0.5, 1.5] normalised, means ~ N(0, 4 I),
    covariances Wishart as above (m = 2d, 2^-12 grid, + 1e-3 I), then m
    points, each the mean of a component drawn by pi plus N(0, I) noise.
    Returns (weights (k,), means (k, d), covs: k arrays (d, d), x (m, d))."""
    g = rng(seed)
    w = g.uniform(0.5, 1.5, k)
    w /= w.sum()
    means = 2.0 * g.standard_normal((k, d))
    covs = [wishart_from(g, d) for _ in range(k)]
    comp = g.choice(k, size=m, p=w)
    x = means[comp] + g.standard_normal((m, d))
    return w, means, covs, x


# Workload table: the five benchmark configurations, by name.
CONFIGS = {
    "uniform_n1000": dict(kind="uniform", n=1000, seed=1),
    "normal_n8000": dict(kind="normal", n=8000, seed=2),
    "normal_n8192": dict(kind="normal", n=8192, seed=2),
    "wishart_n16384": dict(kind="wishart", n=16384, seed=3),
    "wishart_batch512": dict(kind="wishart_batch", count=512, lo=32, hi=1024, seed=4),
    "wishart_batch64": dict(kind="wishart_batch", count=64, lo=256, hi=2048, seed=5),
    # mixture log-likelihood: 16 components in 512 dimensions, 16384 points
    "gmm_k16_d512_m16384": dict(kind="gmm", k=16, d=512, m=16384, seed=6),
}


def sha256_of(mats) -> str:
    """SHA-256 of the C-ordered bytes of a matrix, or of a list of matrices
    one after another: the identity of a workload input."""
    import hashlib

    h = hashlib.sha256()
    for m in (mats if isinstance(mats, (list, tuple)) else [mats]):
        h.update(np.ascontiguousarray(m).tobytes())
    return h.hexdigest()


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
    if kind == "gmm":
        return gmm(c["k"], c["d"], c["m"], c["seed"])
    if kind == "wishart_batch":
        return wishart_batch(c["count"], c["lo"], c["hi"], c["seed"],
                             gram=c.get("gram"))
    raise KeyError(kind)
