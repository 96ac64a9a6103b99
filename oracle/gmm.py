"""Oracle of the mixture-model log-likelihood (plain numpy, FP64).

TEST INFRASTRUCTURE ONLY: the reference the GPU engine's mixture
log-likelihood is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may use it; it shares no code with the GPU
engine and never imports it.

The paper motivates the log-determinant by the log-likelihood of model
mixtures (Abstract): for a Gaussian mixture with weights pi_k, means mu_k
and covariances Sigma_k in dimension d, the log-likelihood of a point x is

    l(x) = log sum_k pi_k N(x; mu_k, Sigma_k)
    log N(x; mu, Sigma) = -(d log(2 pi) + log|Sigma| + (x-mu)^T Sigma^{-1} (x-mu)) / 2.

This module writes that definition out: log|Sigma_k| and its sign from the
condensation oracle (Figure 6, ``oracle.slogdet``), Sigma_k^{-1} from the
oracle's separate Gauss-Jordan inverse, the quadratic form as two plain
matrix-vector products, and the sum over components as a log-sum-exp
shifted by its largest term (the shift changes no value, only the range of
the exponentials).  A component whose determinant is not positive (sign
<= 0, or a failed condensation) makes every log-likelihood NaN.
"""

from __future__ import annotations

import math
from typing import NamedTuple

import numpy as np

from oracle import oracle as O

LOG_2PI = math.log(2.0 * math.pi)


class Components(NamedTuple):
    """What the log-likelihood needs of each component: log|Sigma_k|, the
    sign of det Sigma_k and Sigma_k^{-1}."""
    logdet: np.ndarray  # (K,)
    sign: np.ndarray    # (K,)
    inv: list           # K arrays (d, d)


def components(covs) -> Components:
    """log|Sigma_k| by condensation and Sigma_k^{-1} by Gauss-Jordan."""
    logdet, sign, inv = [], [], []
    for c in covs:
        r = O.slogdet(np.asarray(c, dtype=np.float64))
        logdet.append(r.logabsdet if r.info == 0 else math.nan)
        sign.append(r.sign if r.info == 0 else 0.0)
        inv.append(O.inverse(c) if r.info == 0 else None)
    return Components(np.array(logdet), np.array(sign), inv)


def mahalanobis(x: np.ndarray, mu: np.ndarray, inv: np.ndarray) -> np.ndarray:
    """(x_i - mu)^T Sigma^{-1} (x_i - mu) for every row x_i of x."""
    r = np.asarray(x, dtype=np.float64) - np.asarray(mu, dtype=np.float64)[None, :]
    return np.einsum("ij,ij->i", r, r @ inv.T)


def loglik(x, weights, means, covs, comp: Components = None) -> np.ndarray:
    """l(x_i) for every row of x (M x d); weights (K,), means (K x d),
    covs: K matrices (d x d).  comp: precomputed components(covs)."""
    x = np.asarray(x, dtype=np.float64)
    m, d = x.shape
    comp = comp or components(covs)
    k_count = len(covs)
    if any(s <= 0.0 for s in comp.sign):
        return np.full(m, math.nan)
    terms = np.empty((k_count, m))
    for k in range(k_count):
        q = mahalanobis(x, means[k], comp.inv[k])
        terms[k] = math.log(weights[k]) - 0.5 * (d * LOG_2PI + comp.logdet[k] + q)
    top = terms.max(axis=0)
    return top + np.log(np.exp(terms - top[None, :]).sum(axis=0))
