"""Pins of the CPU oracle's loop hafnian against facts fixed by the definition
and by mathematics (not by the oracle itself).

Each test names what would break it: a dropped loop term, a wrong sign of the
inclusion-exclusion, a wrong pairing, a broken Hessenberg/La Budde/Newton chain
or a wrong exponential recurrence all fail at least one of these.
"""
import itertools
import math

import numpy as np
import pytest

import oracle

rng = np.random.default_rng(12345)


def gauss_int_sym(N, lo=-3, hi=4, seed=None):
    r = np.random.default_rng(seed)
    R = r.integers(lo, hi, (N, N)) + 1j * r.integers(lo, hi, (N, N))
    return np.triu(R) + np.triu(R, 1).T


def rel(a, b):
    return abs(complex(a) - complex(b)) / max(abs(complex(b)), 1e-300)


# ---------------------------------------------------------------- definition

@pytest.mark.parametrize("N", range(0, 11))
def test_dp_equals_exact_enumeration(N):
    """Memoised DP == exact enumeration of single-pair matchings (Gaussian
    integers, exact in binary64)."""
    A = gauss_int_sym(N, seed=100 + N)
    exact = oracle.lhaf_enumerate(A.tolist(), loops=True) if N else 1
    assert oracle.lhaf_dp(A, prec="d") == exact
    assert oracle.to_complex(oracle.lhaf_dp(A, prec="ld")) == exact


@pytest.mark.parametrize("N", range(1, 13))
def test_powertrace_equals_definition_integer(N):
    """Power-trace sum (long double) reproduces the exact integer lhaf."""
    A = gauss_int_sym(N, seed=200 + N)
    exact = complex(oracle.lhaf_enumerate(A.tolist(), loops=True))
    got = oracle.to_complex(oracle.lhaf_pt(A, prec="ld"))
    assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact))


@pytest.mark.parametrize("N", [1, 2, 3, 5, 8, 11, 14, 17, 20])
def test_powertrace_equals_dp_random(N):
    A = oracle_normal(N, seed=300 + N)
    ref = oracle.to_complex(oracle.lhaf_dp(A, prec="ld"))
    got_ld, abs_ld = oracle.lhaf_pt(A, prec="ld", with_abs=True)
    got_d, abs_d = oracle.lhaf_pt(A, prec="d", with_abs=True)
    # long double: per-term rounding ~ 1e-19 * sum|t_S|
    assert abs(oracle.to_complex(got_ld) - ref) <= 1e-16 * float(abs_ld) + 1e-300
    # double: per-term rounding ~ 1e-16 * sum|t_S|
    assert abs(got_d - ref) <= 1e-13 * abs_d + 1e-300


def oracle_normal(N, seed):
    r = np.random.default_rng(seed)
    R = r.standard_normal((N, N)) + 1j * r.standard_normal((N, N))
    return (R + R.T) / 2


@pytest.mark.parametrize("N", [4, 7, 10, 12])
def test_powertrace_vs_mpmath_definition(N):
    """50-digit evaluation of the definition vs the long-double power-trace sum."""
    A = oracle_normal(N, seed=400 + N)
    ref = oracle.lhaf_mpmath(A, dps=40)
    got, ab = oracle.lhaf_pt(A, prec="ld", with_abs=True)
    assert abs(oracle.to_complex(got) - ref) <= 2e-18 * float(ab)


def test_haf_is_lhaf_of_zero_diagonal():
    A = gauss_int_sym(8, seed=7)
    A0 = A - np.diag(np.diag(A))
    exact = oracle.lhaf_enumerate(A.tolist(), loops=False)
    assert oracle.to_complex(oracle.lhaf_pt(A0, prec="ld")) == pytest.approx(exact, abs=1e-9)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", range(1, 25))
def test_telephone_numbers(n):
    """lhaf(1_n) = T(n), the number of involutions (caption of Fig. 2)."""
    T = oracle.telephone(n)
    got, ab = oracle.lhaf_pt(oracle_ones(n), prec="ld", with_abs=True)
    got = oracle.to_complex(got)
    assert abs(got.imag) == 0
    # rounding grows with the cancellation sum_S |t_S| / T(n) (cf. Fig. 2)
    assert abs(got.real - T) <= 1e-17 * float(ab)
    got_d, ab_d = oracle.lhaf_pt(oracle_ones(n), prec="d", with_abs=True)
    assert abs(got_d.real - T) <= 1e-14 * ab_d


def oracle_ones(n):
    return np.ones((n, n), dtype=complex)


def test_telephone_sequence_values():
    # OEIS A000085 start: independent listing of the involution numbers
    assert [oracle.telephone(n) for n in range(12)] == [1, 1, 2, 4, 10, 26, 76, 232, 764, 2620, 9496, 35696]


@pytest.mark.parametrize("n", range(1, 11))
def test_hafnian_all_ones_double_factorial(n):
    """haf(1_{2n}) = (2n-1)!!: number of perfect matchings of K_2n."""
    A = oracle_ones(2 * n)
    np.fill_diagonal(A, 0)
    got, ab = oracle.lhaf_pt(A, prec="ld", with_abs=True)
    assert abs(oracle.to_complex(got) - oracle.double_factorial(2 * n - 1)) <= 1e-17 * float(ab)


@pytest.mark.parametrize("n", range(1, 8))
def test_hafnian_bipartite_is_permanent(n):
    """haf([[0, B], [B^T, 0]]) = perm(B) (Ryser, exact integers)."""
    r = np.random.default_rng(500 + n)
    B = r.integers(-3, 4, (n, n)) + 1j * r.integers(-3, 4, (n, n))
    A = np.zeros((2 * n, 2 * n), dtype=complex)
    A[:n, n:] = B
    A[n:, :n] = B.T
    perm = oracle.ryser_permanent(B.tolist())
    got = oracle.to_complex(oracle.lhaf_pt(A, prec="ld"))
    assert abs(got - perm) <= 1e-12 * max(1, abs(perm))


@pytest.mark.parametrize("N", [3, 6, 9, 14, 20])
def test_rank_one(N):
    """lhaf(filldiag(v v^T, v)) = T(N) prod v_i and haf(v v^T) = (N-1)!! prod v_i."""
    r = np.random.default_rng(600 + N)
    v = r.standard_normal(N) * 0.7 + 1j * r.standard_normal(N) * 0.7
    A = np.outer(v, v)
    np.fill_diagonal(A, v)
    prod = np.prod(v)
    got = oracle.to_complex(oracle.lhaf_pt(A, prec="ld"))
    assert rel(got, oracle.telephone(N) * prod) <= 1e-14
    if N % 2 == 0:
        A2 = np.outer(v, v)
        np.fill_diagonal(A2, 0)
        got2 = oracle.to_complex(oracle.lhaf_pt(A2, prec="ld"))
        assert rel(got2, oracle.double_factorial(N - 1) * prod) <= 1e-14


def single_mode_closed_form(N, b, g):
    """lhaf of an N x N matrix with every off-diagonal entry b and diagonal g:
    sum_k N! / (k! (N-2k)! 2^k) b^k g^(N-2k) (choose k pairs, the rest loops)."""
    import mpmath

    with mpmath.workdps(40):
        b = mpmath.mpc(b.real, b.imag)
        g = mpmath.mpc(g.real, g.imag)
        tot = mpmath.mpc(0)
        for k in range(N // 2 + 1):
            tot += mpmath.factorial(N) / (mpmath.factorial(k) * mpmath.factorial(N - 2 * k) * 2**k) * b**k * g ** (N - 2 * k)
        return complex(tot)


@pytest.mark.parametrize("N", [5, 8, 11, 16, 21, 24])
def test_single_mode_repeated(N):
    b, g = 0.43 - 0.21j, -0.3 + 0.55j
    A = np.full((N, N), b)
    np.fill_diagonal(A, g)
    got, ab = oracle.lhaf_pt(A, prec="ld", with_abs=True)
    assert abs(oracle.to_complex(got) - single_mode_closed_form(N, b, g)) <= 1e-17 * float(ab)


def test_block_diagonal_product():
    """lhaf of a permuted block-diagonal matrix = product of the blocks' lhafs
    (matchings never cross blocks)."""
    sizes = [3, 4, 5, 6]
    blocks = [oracle_normal(k, seed=700 + k) for k in sizes]
    N = sum(sizes)
    A = np.zeros((N, N), dtype=complex)
    o = 0
    for Bk in blocks:
        A[o:o + len(Bk), o:o + len(Bk)] = Bk
        o += len(Bk)
    perm = np.random.default_rng(7).permutation(N)
    Ap = A[np.ix_(perm, perm)]
    expect = np.prod([oracle.to_complex(oracle.lhaf_dp(Bk, prec="ld")) for Bk in blocks])
    got, ab = oracle.lhaf_pt(Ap, prec="ld", with_abs=True)
    assert abs(oracle.to_complex(got) - expect) <= 1e-16 * float(ab)


def test_homogeneity_and_similarity():
    """lhaf(t^2 A0 + t diag(d)) = t^N lhaf(A); lhaf(D A0 D + diag(D d)) = det(D) lhaf(A)."""
    N = 12
    A = oracle_normal(N, seed=800)
    base = oracle.to_complex(oracle.lhaf_pt(A, prec="ld"))
    t = 0.8 + 0.3j
    A0 = A - np.diag(np.diag(A))
    At = t * t * A0 + t * np.diag(np.diag(A))
    assert rel(oracle.to_complex(oracle.lhaf_pt(At, prec="ld")), t**N * base) <= 1e-13
    dvec = np.random.default_rng(9).uniform(0.5, 1.5, N) * np.exp(1j * np.random.default_rng(10).uniform(0, 6.28, N))
    AD = np.diag(dvec) @ A0 @ np.diag(dvec) + np.diag(dvec * np.diag(A))
    assert rel(oracle.to_complex(oracle.lhaf_pt(AD, prec="ld")), np.prod(dvec) * base) <= 1e-13


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_permutation_invariance(seed):
    """The pairing (i, i+n) is a free choice: a simultaneous permutation of rows
    and columns changes the subsets but not the value."""
    N = 14
    A = oracle_normal(N, seed=900 + seed)
    p = np.random.default_rng(seed).permutation(N)
    a1, ab1 = oracle.lhaf_pt(A, prec="ld", with_abs=True)
    a2, _ = oracle.lhaf_pt(A[np.ix_(p, p)], prec="ld", with_abs=True)
    assert abs(oracle.to_complex(a1) - oracle.to_complex(a2)) <= 1e-16 * float(ab1)


@pytest.mark.parametrize("N", [1, 3, 7, 13])
def test_odd_dimension_padding(N):
    A = oracle_normal(N, seed=1000 + N)
    ref = oracle.to_complex(oracle.lhaf_dp(A, prec="ld"))
    got, ab = oracle.lhaf_pt(A, prec="ld", with_abs=True)
    assert abs(oracle.to_complex(got) - ref) <= 1e-16 * float(ab)


def test_empty_matrix():
    assert oracle.to_complex(oracle.lhaf_pt(np.zeros((0, 0)), prec="ld")) == 1
    assert oracle.lhaf_dp(np.zeros((0, 0)), prec="d") == 1


def test_terms_sum_to_lhaf_and_empty_subset_zero():
    N = 10
    A = oracle_normal(N, seed=1100)
    n = N // 2
    terms = [oracle.term(A, mask, prec="ld") for mask in range(1 << n)]
    assert terms[0] == 0
    ref = oracle.to_complex(oracle.lhaf_pt(A, prec="ld"))
    assert abs(sum(terms) - ref) <= 1e-13 * sum(abs(t) for t in terms)


def test_thread_count_does_not_change_result():
    A = oracle_normal(30, seed=1200)
    a = oracle.lhaf_pt(A, prec="d", nthreads=1)
    b = oracle.lhaf_pt(A, prec="d", nthreads=4)
    assert a == b


# ---------------------------------------------------------------- power traces

@pytest.mark.parametrize("m", [1, 2, 3, 8, 17, 32, 50])
def test_power_traces_vs_eigenvalues(m):
    """Hessenberg + La Budde + Newton == sum of powers of numpy eigenvalues."""
    r = np.random.default_rng(1300 + m)
    M = (r.standard_normal((m, m)) + 1j * r.standard_normal((m, m))) / np.sqrt(2 * m)
    K = 26
    got = oracle.power_traces(M, K, prec="ld")
    lam = np.linalg.eigvals(M)
    for k in range(1, K + 1):
        ref = np.sum(lam**k)
        scale = np.sum(np.abs(lam) ** k)
        assert abs(got[k - 1] - ref) <= 1e-11 * scale, (k, got[k - 1], ref)


@pytest.mark.parametrize("m", [1, 4, 9, 20])
def test_charpoly_vs_numpy_poly(m):
    r = np.random.default_rng(1400 + m)
    M = r.standard_normal((m, m)) + 1j * r.standard_normal((m, m))
    got = oracle.charpoly(M, prec="ld")           # coefficient of x^t at index t
    ref = np.poly(M)[::-1]                         # numpy: highest power first
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_power_traces_direct_matrix_powers():
    M = oracle_normal(12, seed=1500) / 4
    got = oracle.power_traces(M, 20, prec="ld")
    P = np.eye(12, dtype=complex)
    for k in range(1, 21):
        P = P @ M
        assert abs(got[k - 1] - np.trace(P)) <= 1e-12 * max(1, abs(np.trace(P)))


# ---------------------------------------------------------------- accuracy report

def test_allones_accuracy_in_line_with_paper():
    """Long-double oracle error on 1_30 is of the order the paper reports for
    its long-double La Budde code in Fig. 2 (3.6e-12 at n = 30)."""
    T = oracle.telephone(30)
    got = oracle.to_complex(oracle.lhaf_pt(oracle_ones(30), prec="ld"))
    err = abs(got.real - T) / T
    assert err < 1e-9
