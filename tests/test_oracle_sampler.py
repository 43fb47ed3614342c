"""Pins of the oracle's sampling chain (Algorithm of Sec. III).

The chain's ingredients are checked against facts that do not go through it:
heterodyne draws reproduce the Husimi mean and covariance; conditioning leaves
uncorrelated modes unchanged; averaging the conditional photon-number
probability over heterodyne outcomes recovers the (pinned) marginal, which is
the identity the algorithm rests on; coherent product states give exact
per-mode Poisson draws; and a small version of the total-variation-distance
experiment of Fig. 1 compares the chain's samples with the exact distribution,
judged against exact samplers drawing the same number of samples.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import sampler
from paper_2010_15595_amd import workloads


def test_heterodyne_moments():
    st = workloads.pure_state(3, 0.6, 0.4, seed=2)
    Q, al = st["Q"], st["alpha_vec"]
    rng = np.random.default_rng(0)
    modes = [1, 2]
    draws = np.array([sampler.heterodyne_sample(Q, al, modes, rng.standard_normal(4)) for _ in range(20000)])
    aug = np.concatenate([draws, np.conj(draws)], axis=1)
    idx = [1, 2, 4, 5]
    mean = aug.mean(axis=0)
    cov = (aug - mean).T @ np.conj(aug - mean) / len(aug)
    assert np.abs(mean - al[idx]).max() < 0.03
    assert np.abs(cov - Q[np.ix_(idx, idx)]).max() < 0.04


def test_conditioning_leaves_uncorrelated_modes_unchanged():
    s1 = workloads.pure_state(1, 0.5, 0.3, seed=1)
    s2 = workloads.pure_state(1, 0.7, 0.2, seed=2)
    Q = np.zeros((4, 4), dtype=complex)
    Q[np.ix_([0, 2], [0, 2])] = s1["Q"]
    Q[np.ix_([1, 3], [1, 3])] = s2["Q"]
    al = np.array([s1["alpha_vec"][0], s2["alpha_vec"][0], s1["alpha_vec"][1], s2["alpha_vec"][1]])
    QA, aA = sampler.conditional_state(Q, al, [0], [1], np.array([0.3 - 0.7j]))
    assert np.abs(QA - s1["Q"]).max() < 1e-14
    assert np.abs(aA - s1["alpha_vec"]).max() < 1e-14


def test_heterodyne_average_of_conditional_probability_is_the_marginal():
    """p(s_1) = E_beta [ p(s_1 | beta_2) ]: the identity behind the algorithm."""
    st = workloads.pure_state(2, 0.5, 0.3, seed=4)
    Q, al = st["Q"], st["alpha_vec"]
    rng = np.random.default_rng(1)
    K = 6000
    acc = np.zeros(4)
    for _ in range(K):
        b = sampler.heterodyne_sample(Q, al, [1], rng.standard_normal(2))
        QA, aA = sampler.conditional_state(Q, al, [0], [1], b)
        acc += [oracle.probability(QA, aA, [s], prec="d")[0] for s in range(4)]
    acc /= K
    marg = [sum(oracle.probability(Q, al, [s, t], prec="d")[0] for t in range(30)) for s in range(4)]
    for s in range(4):
        assert acc[s] == pytest.approx(marg[s], rel=0.04, abs=2e-3)


def test_coherent_product_state_gives_poisson_draws():
    a = np.array([0.8 + 0.3j, -0.5j, 1.1 + 0.0j])
    M = 3
    Q = np.eye(2 * M, dtype=complex)
    al = np.concatenate([a, np.conj(a)])
    rng = np.random.default_rng(3)
    for _ in range(20):
        u = rng.random(M)
        s = sampler.sample_chain(Q, al, 12, rng.standard_normal(2 * (M - 1)), u)
        for k in range(M):
            lam = abs(a[k]) ** 2
            cdf = np.cumsum([math.exp(-lam) * lam ** j / math.factorial(j) for j in range(13)])
            cdf /= cdf[-1]
            assert s[k] == int(np.searchsorted(cdf, u[k], side="right"))


def test_total_variation_distance_small_state():
    """Fig. 1 in miniature: 3 modes, r = 0.5, cutoff 6 (as in Fig. 1), 2000 samples."""
    st = workloads.pure_state(3, 0.5, 0.2, seed=5)
    Q, al = st["Q"], st["alpha_vec"]
    cutoff = 6
    pats, probs = sampler.exact_distribution(Q, al, cutoff)
    assert probs.sum() > 0.998  # the truncated tail is far below the statistical resolution
    probs_n = probs / probs.sum()
    rng = np.random.default_rng(11)
    n = 2000
    counts = {}
    for _ in range(n):
        s = tuple(sampler.sample_chain(Q, al, cutoff, rng.standard_normal(4), rng.random(3)))
        counts[s] = counts.get(s, 0) + 1
    key = {tuple(p): i for i, p in enumerate(pats)}
    emp = np.zeros(len(pats))
    for s, c in counts.items():
        emp[key[s]] = c / n
    tvd = 0.5 * np.abs(emp - probs_n).sum()
    # TVD of exact samplers with the same number of samples
    ref = [0.5 * np.abs(rng.multinomial(n, probs_n) / n - probs_n).sum() for _ in range(1000)]
    assert tvd <= np.quantile(ref, 0.995), (tvd, np.quantile(ref, [0.5, 0.995]))
