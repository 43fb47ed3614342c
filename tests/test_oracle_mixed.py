"""Pins of the oracle's mixed-state probability, Eq. (11) of the paper:
  p(S) = p(vac) lhaf(filldiag(A_S, gamma_S)) / prod s_i!,  A = X (I - Q^-1),
with A_S repeating rows/columns i and i + M s_i times.

The pins do not go through the formula: closed forms for thermal and displaced
thermal states, a brute-force Fock-space computation of a displaced, squeezed,
beam-split two-mode state with thermal inputs (Q and the mean vector measured
from the density operator), marginals of pinned pure states, products of
independent modes, normalisation, and the reduction to the pure-state formula.
The Fock-space test also fixes the loop-weight convention (reading R11): gamma
is X Q^-1 alpha, i.e. each index of A takes the entry of Q^-1 alpha of its
partner index; the unswapped vector disagrees.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import expm_multiply
from scipy.special import eval_laguerre

import oracle
from paper_2010_15595_amd import workloads


def thermal_q(nbar):
    """Q of independent thermal modes: Sigma = diag(nbar + 1/2) in the (a, a^dag) basis."""
    nb = np.asarray(nbar, dtype=float)
    return np.diag(np.concatenate([nb, nb]) + 1.0).astype(complex)


def test_thermal_single_mode_closed_form():
    for nbar in (0.3, 1.7):
        Q = thermal_q([nbar])
        for n in range(9):
            p, lh = oracle.probability_mixed(Q, None, [n])
            ref = nbar ** n / (1 + nbar) ** (n + 1)
            assert p == pytest.approx(ref, rel=1e-12)
            assert abs(complex(lh).imag) <= 1e-12 * abs(complex(lh))


def test_displaced_thermal_closed_form():
    """p(n) = nbar^n / (1+nbar)^(n+1) exp(-|a|^2/(1+nbar)) L_n(-|a|^2 / (nbar (1+nbar)))."""
    nbar, a = 0.6, 0.8 * np.exp(1.1j)
    Q = thermal_q([nbar])
    al = np.array([a, np.conj(a)])
    x = abs(a) ** 2
    for n in range(9):
        p, _ = oracle.probability_mixed(Q, al, [n])
        ref = nbar ** n / (1 + nbar) ** (n + 1) * math.exp(-x / (1 + nbar)) * eval_laguerre(n, -x / (nbar * (1 + nbar)))
        assert p == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_reduces_to_pure_state_formula(seed):
    st = workloads.pure_state(4, 0.7, 0.3, seed=seed)
    r = np.random.default_rng(seed)
    for _ in range(4):
        pat = r.integers(0, 3, 4)
        if pat.sum() > 6:
            continue
        p_mix, lh = oracle.probability_mixed(st["Q"], st["alpha_vec"], pat)
        p_pure, _ = oracle.probability(st["Q"], st["alpha_vec"], pat)
        assert p_mix == pytest.approx(p_pure, rel=1e-11)
        assert abs(complex(lh).imag) <= 1e-11 * abs(complex(lh))


def test_marginal_of_a_two_mode_pure_state():
    """Tracing out mode 2 of a pinned pure state leaves a mixed state whose
    distribution is the marginal sum over mode 2."""
    st = workloads.pure_state(2, 0.3, 0.3, seed=7)  # tanh r = 0.29: terms beyond t = 20 are < 1e-20
    Q, al = st["Q"], st["alpha_vec"]
    keep = [0, 2]  # a_1 and a_1^dag
    Qa = Q[np.ix_(keep, keep)]
    ala = al[keep]
    for s in range(5):
        marg = sum(oracle.probability(Q, al, [s, t], prec="d")[0] for t in range(21))
        p, _ = oracle.probability_mixed(Qa, ala, [s])
        assert p == pytest.approx(marg, rel=1e-9)


def test_independent_modes_factorise():
    st1 = workloads.pure_state(1, 0.5, 0.3, seed=3)
    nbar = 0.4
    Q1, a1 = st1["Q"], st1["alpha_vec"]
    Q2 = thermal_q([nbar])
    # modes (1, 2): Q in (a1, a2, a1^dag, a2^dag) order
    Q = np.zeros((4, 4), dtype=complex)
    Q[np.ix_([0, 2], [0, 2])] = Q1
    Q[np.ix_([1, 3], [1, 3])] = Q2
    al = np.array([a1[0], 0.0, a1[1], 0.0])
    for s1, s2 in itertools.product(range(4), range(3)):
        p, _ = oracle.probability_mixed(Q, al, [s1, s2])
        ref = oracle.probability(Q1, a1, [s1])[0] * nbar ** s2 / (1 + nbar) ** (s2 + 1)
        assert p == pytest.approx(ref, rel=1e-11)


def test_normalisation_of_a_small_mixed_state():
    st = workloads.pure_state(2, 0.3, 0.2, seed=11)
    # add thermal noise: Q_mixed = Q + diag(noise) keeps the (a, a^dag) form
    Q = st["Q"] + np.diag([0.05, 0.08, 0.05, 0.08])
    total = 0.0
    for s1, s2 in itertools.product(range(14), range(14)):
        if s1 + s2 < 14:
            total += oracle.probability_mixed(Q, st["alpha_vec"], [s1, s2], prec="d")[0]
    assert total == pytest.approx(1.0, abs=1e-6)


# --------------------------------------------------------------------------
# Fock-space pin (two modes, thermal inputs, truncated number basis)
# --------------------------------------------------------------------------

CUT = 30
KMAX = 14
NBAR = (0.12, 0.07)


def _mixed_fock():
    a1 = sp.diags(np.sqrt(np.arange(1, CUT)), 1, format="csr")
    Idn = sp.identity(CUT, format="csr")
    A1 = sp.kron(a1, Idn, format="csr").astype(complex)
    A2 = sp.kron(Idn, a1, format="csr").astype(complex)
    z = 0.3 * np.exp(0.5j)  # two-mode squeezer exp(z* a1 a2 - z a1^dag a2^dag)
    th, ph = 0.55, -0.3     # beamsplitter
    al = (0.25 - 0.2j, 0.15 + 0.3j)
    gens = [
        np.conj(z) * (A1 @ A2) - z * (A1.T @ A2.T),
        th * (np.exp(1j * ph) * (A1 @ A2.T) - np.exp(-1j * ph) * (A1.T @ A2)),
        al[0] * A1.T - np.conj(al[0]) * A1 + al[1] * A2.T - np.conj(al[1]) * A2,
    ]
    states, weights = [], []
    for k1, k2 in itertools.product(range(KMAX), range(KMAX)):
        w = 1.0
        for k, nb in ((k1, NBAR[0]), (k2, NBAR[1])):
            w *= nb ** k / (1 + nb) ** (k + 1)
        psi = np.zeros(CUT * CUT, dtype=complex)
        psi[k1 * CUT + k2] = 1.0
        for g in gens:
            psi = expm_multiply(g, psi)
        states.append(psi)
        weights.append(w)
    weights = np.array(weights)
    return states, weights / weights.sum(), (A1, A2)


def _mixed_moments(states, weights, ops):
    M = len(ops)
    ex = lambda O: sum(w * np.vdot(psi, O @ psi) for psi, w in zip(states, weights))
    mean = np.array([ex(a) for a in ops])
    xi = list(ops) + [a.T for a in ops]
    mu = np.concatenate([mean, np.conj(mean)])
    Idn = sp.identity(states[0].size, format="csr")
    d = [x - m * Idn for x, m in zip(xi, mu)]
    dag = [d[M + i] if i < M else d[i - M] for i in range(2 * M)]
    S = np.zeros((2 * M, 2 * M), dtype=complex)
    for k in range(2 * M):
        for l in range(2 * M):
            S[k, l] = 0.5 * (ex(d[k] @ dag[l]) + ex(dag[l] @ d[k]))
    return S + 0.5 * np.eye(2 * M), mu


@pytest.fixture(scope="module")
def mixed_fock():
    states, weights, ops = _mixed_fock()
    Q, al = _mixed_moments(states, weights, ops)
    pf = lambda s1, s2: float(sum(w * abs(psi[s1 * CUT + s2]) ** 2 for psi, w in zip(states, weights)))
    return Q, al, pf


def test_fock_space_mixed_state_is_mixed(mixed_fock):
    """A = X (I - Q^-1) of the test state is not of the pure form B (+) conj(B)."""
    Q, al, _ = mixed_fock
    A, _, _ = oracle.mixed_state_params(Q, al)
    assert np.abs(A[:2, 2:]).max() > 1e-3


def test_fock_space_mixed_probabilities(mixed_fock):
    Q, al, pf = mixed_fock
    worst = 0.0
    for s1 in range(5):
        for s2 in range(5 - s1):
            p_fock = pf(s1, s2)
            p, lh = oracle.probability_mixed(Q, al, [s1, s2])
            worst = max(worst, abs(p - p_fock) / p_fock)
            assert abs(complex(lh).imag) <= 1e-9 * abs(complex(lh))
    assert worst < 1e-7


def test_fock_space_rules_out_unswapped_loop_weights(mixed_fock):
    """Loop weights Q^-1 alpha without the half swap (the literal Eq. (9)
    vector placed on the diagonal) give wrong probabilities."""
    Q, al, pf = mixed_fock
    literal = lambda Q_, a_: np.linalg.inv(Q_) @ a_
    worst = 0.0
    for s1, s2 in [(2, 1), (1, 2), (3, 0), (1, 1)]:
        p_lit, _ = oracle.probability_mixed(Q, al, [s1, s2], gamma_fn=literal)
        worst = max(worst, abs(p_lit - pf(s1, s2)) / pf(s1, s2))
    assert worst > 1e-2
