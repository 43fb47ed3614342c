"""Mixed-state probabilities (Eq. (11)) on the GPU against the oracle.

The library builds the 2N x 2N matrix filldiag(A_S, gamma_S) on the host and
evaluates its loop hafnian with the same kernels as every other entry point;
the oracle builds it independently in numpy and evaluates it in long double.
"""
import numpy as np
import pytest

import oracle
from paper_2010_15595_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gbs():
    import paper_2010_15595_amd as g

    g.init(0)
    return g


def noisy_state(M, r, sigma, noise, seed):
    """A pure state plus independent thermal noise (Q + noise I keeps the (a, a^dag) form)."""
    st = workloads.pure_state(M, r, sigma, seed=seed)
    return st["Q"] + noise * np.eye(2 * M), st["alpha_vec"]


def _check(gbs, Q, al, pat, tol_rel=1e-10):
    p, lh, d = gbs.probability_mixed(Q, al, pat, with_lhaf=True, with_diag=True)
    p_ref, lh_ref = oracle.probability_mixed(Q, al, pat)
    lh_ref = complex(lh_ref)
    err = abs(lh - lh_ref)
    tol = max(tol_rel * abs(lh_ref), 2e-14 * d["abs_sum"])
    print(f"[mixed {list(pat)}] N={2 * int(np.sum(pat))} p={p:.6e} ref={p_ref:.6e} |dlhaf|={err:.2e} tol={tol:.2e} "
          f"kappa={d['kappa']:.2e}", flush=True)
    assert err <= tol
    assert abs(p - p_ref) <= max(tol_rel * abs(p_ref), 2e-14 * d["abs_sum"] * abs(p_ref) / max(abs(lh_ref), 1e-300))
    return p


def test_thermal_and_displaced_thermal(gbs):
    nbar = 0.6
    Q = np.diag([nbar + 1, nbar + 1]).astype(complex)
    for n in range(7):
        p = gbs.probability_mixed(Q, None, [n])
        assert p == pytest.approx(nbar ** n / (1 + nbar) ** (n + 1), rel=1e-12)
    a = 0.8 * np.exp(1.1j)
    al = np.array([a, np.conj(a)])
    for n in range(5):
        _check(gbs, Q, al, [n])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_noisy_states_small(gbs, seed):
    Q, al = noisy_state(4, 0.8, 0.3, 0.15, seed)
    r = np.random.default_rng(100 + seed)
    for _ in range(3):
        pat = r.integers(0, 3, 4)
        _check(gbs, Q, al, pat)


def test_pure_state_agrees_with_pure_entry_point(gbs):
    st = workloads.pure_state(5, 0.7, 0.25, seed=21)
    pat = [1, 2, 0, 1, 1]
    p_mix = gbs.probability_mixed(st["Q"], st["alpha_vec"], pat)
    p_pure = gbs.probability(st["Q"], st["alpha_vec"], pat)
    assert p_mix == pytest.approx(p_pure, rel=1e-9)


def test_larger_mixed_state(gbs):
    """16 photons on 10 modes: a 32 x 32 loop hafnian (2^16 subset terms)."""
    Q, al = noisy_state(10, 0.9, 0.2, 0.1, 31)
    pat = [2, 1, 2, 1, 2, 2, 1, 2, 1, 2]
    _check(gbs, Q, al, pat)


def test_vacuum_pattern_is_p_vac(gbs):
    Q, al = noisy_state(3, 0.6, 0.3, 0.2, 5)
    _, _, pvac = oracle.mixed_state_params(Q, al)
    assert gbs.probability_mixed(Q, al, [0, 0, 0]) == pytest.approx(pvac, rel=1e-13)
