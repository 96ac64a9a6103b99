"""Pins of the mixture log-likelihood oracle (oracle/gmm.py) against
closed forms and a library routine (the Abstract's use of log-determinants:
the log-likelihood of model mixtures).

* one component with a diagonal covariance: the sum of univariate normal
  log-densities, written out;
* isotropic components s_k^2 I with unequal weights: the closed form of
  each density, summed directly (no log-sum-exp shift);
* random SPD covariances: scipy.stats.multivariate_normal.logpdf per
  component and scipy.special.logsumexp over components;
* K identical components: the single-component value, whatever the weights;
* a component with det <= 0: NaN.
"""

import math

import numpy as np
import pytest

import synth
from oracle import gmm as G

stats = pytest.importorskip("scipy.stats")
special = pytest.importorskip("scipy.special")


def test_single_diagonal_component():
    g = np.random.default_rng(1)
    d = 7
    sig2 = g.uniform(0.2, 3.0, d)
    mu = g.standard_normal(d)
    x = g.standard_normal((20, d)) * 2
    got = G.loglik(x, np.array([1.0]), mu[None, :], [np.diag(sig2)])
    ref = np.array([sum(-0.5 * (math.log(2 * math.pi * s) + (xi - m) ** 2 / s)
                        for xi, m, s in zip(row, mu, sig2)) for row in x])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_isotropic_mixture_closed_form():
    g = np.random.default_rng(2)
    k, d = 3, 5
    w = np.array([0.2, 0.5, 0.3])
    s2 = np.array([0.5, 1.0, 2.5])
    mu = g.standard_normal((k, d))
    covs = [s * np.eye(d) for s in s2]
    x = g.standard_normal((30, d))
    got = G.loglik(x, w, mu, covs)
    ref = []
    for row in x:
        dens = sum(w[j] * (2 * math.pi * s2[j]) ** (-d / 2)
                   * math.exp(-0.5 * float(((row - mu[j]) ** 2).sum()) / s2[j])
                   for j in range(k))
        ref.append(math.log(dens))
    assert np.abs(got - np.array(ref)).max() <= 1e-12


@pytest.mark.parametrize("d", [3, 16, 40])
def test_random_spd_against_scipy(d):
    w, means, covs, x = synth.gmm(4, d, 50, 10 + d)
    got = G.loglik(x, w, means, covs)
    per = np.stack([np.log(w[j]) + stats.multivariate_normal.logpdf(x, means[j], covs[j])
                    for j in range(len(covs))])
    ref = special.logsumexp(per, axis=0)
    assert np.abs(got - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


def test_identical_components_reduce_to_one():
    w, means, covs, x = synth.gmm(1, 12, 40, 3)
    one = G.loglik(x, np.array([1.0]), means, covs)
    many = G.loglik(x, np.array([0.1, 0.6, 0.3]), np.repeat(means, 3, axis=0), covs * 3)
    assert np.abs(one - many).max() <= 1e-12 * np.abs(one).max()


def test_non_positive_determinant_gives_nan():
    d = 4
    bad = -np.eye(d)  # det = +1 but negative definite: not a covariance...
    bad[0, 0] = 1.0   # ... det < 0 now
    x = np.zeros((3, d))
    out = G.loglik(x, np.array([0.5, 0.5]), np.zeros((2, d)), [np.eye(d), bad])
    assert np.isnan(out).all()
    sing = np.zeros((d, d))
    out = G.loglik(x, np.array([1.0]), np.zeros((1, d)), [sing])
    assert np.isnan(out).all()
