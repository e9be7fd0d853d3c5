"""Pins of the host work analysis: Bennett's acceptance ratio recovers mu
from Crooks-consistent work distributions, Eq. (21) gives the hybrid-MC
acceptance erfc(sqrt(beta <dH>) / 2) for Gaussian work, and alpha_2 tells
Gaussian from fat-tailed distributions."""
import math

import numpy as np
import pytest
from scipy.special import erfc

from paper_2307_11447_amd import analysis as A


def crooks_gaussian(mu, sigma, beta, n, seed):
    # insertion-signed work with P_ins(x) / P_del(x) = exp(beta (x - mu)):
    # Gaussians of equal width sigma at mu +- beta sigma^2 / 2
    rng = np.random.default_rng(seed)
    d = 0.5 * beta * sigma * sigma
    return rng.normal(mu + d, sigma, n), rng.normal(mu - d, sigma, n)


@pytest.mark.parametrize("mu,sigma,beta", [(-9.5, 2.0, 1.0), (3.0, 1.0, 2.0), (-120.0, 2.0, 1.0 / 0.59)])
def test_bar_recovers_mu_from_crooks_distributions(mu, sigma, beta):
    ins, dele = crooks_gaussian(mu, sigma, beta, 200000, 1)
    est = A.bar_beta_mu(ins, dele, beta)
    assert est / beta == pytest.approx(mu, abs=0.05 * max(1.0, sigma))


def test_bar_with_unequal_sample_sizes():
    ins, dele = crooks_gaussian(-2.0, 1.5, 1.0, 200000, 2)
    est = A.bar_beta_mu(ins, dele[:40000], 1.0)
    assert est == pytest.approx(-2.0, abs=0.05)


def test_predicted_acceptance_is_the_hybrid_mc_erfc_for_gaussian_work():
    # at beta mu = beta mu_F, beta (dM - mu) ~ N(d, 2 d) for insertions with
    # d = beta^2 sigma^2 / 2 = beta <dH>: P_acc = erfc(sqrt(d) / 2)
    beta, mu, sigma = 1.0, -4.0, 1.7
    ins, dele = crooks_gaussian(mu, sigma, beta, 400000, 3)
    p_ins, p_del = A.pacc_predicted(ins, dele, beta, beta * mu)
    d = 0.5 * (beta * sigma) ** 2
    assert p_ins == pytest.approx(erfc(0.5 * math.sqrt(d)), abs=3e-3)
    assert p_del == pytest.approx(erfc(0.5 * math.sqrt(d)), abs=3e-3)


def test_alpha2():
    rng = np.random.default_rng(4)
    assert abs(A.alpha2(rng.normal(0.0, 3.0, 400000), 1.0)) < 0.02
    assert A.alpha2(rng.exponential(2.0, 400000), 1.0) == pytest.approx(2.0, abs=0.1)   # kurtosis 9 -> 9/3 - 1


def test_overlap_ratio_of_gaussian_crooks_pair():
    # at mu: the insertion work N(mu + d, sigma) lies below mu with
    # probability Phi(-beta sigma / 2), and symmetrically for deletions
    from scipy.stats import norm
    beta, mu, sigma = 2.0, 1.0, 0.8
    ins, dele = crooks_gaussian(mu, sigma, beta, 400000, 6)
    r_ins, r_del = A.overlap_ratio(ins, dele, beta * mu, beta)
    assert r_ins == pytest.approx(norm.cdf(-0.5 * beta * sigma), abs=3e-3)
    assert r_del == pytest.approx(norm.cdf(-0.5 * beta * sigma), abs=3e-3)
    p_ins, _ = A.pacc_predicted(ins, dele, beta, beta * mu)
    assert p_ins > r_ins


def test_work_summary_brackets_mu():
    beta, mu, sigma = 1.0, -9.5, 1.5
    ins, dele = crooks_gaussian(mu, sigma, beta, 5000, 7)
    s = A.work_summary(ins, dele, beta, -9.5, boot=100)
    lo, hi = s["beta_mu_bar_bootstrap90"]
    assert lo - 0.05 < beta * mu < hi + 0.05
    assert s["beta_dM_var_ins"] == pytest.approx((beta * sigma) ** 2, rel=0.1)
    assert abs(s["alpha2_ins"]) < 0.2
