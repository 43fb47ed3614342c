"""CPU oracle for the loop-hafnian path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library (the HIP kernels and
the C ABI under ``paper_2010_15595_amd``) never imports, links or calls it, and
shares no code with it.

Everything here is written from Quesada et al., "Quadratic speedup for
simulating Gaussian boson sampling" (the paper):

* ``lhaf_dp`` / ``lhaf_pt`` / ``term`` wrap the C oracle (lhaf_oracle.c): the
  single-pair-matching definition (Sec. II, after Eq. (11)) by memoised brute
  force, and the power-trace subset sum benchmarked in Sec. IV, in double or
  x87 long double.
* ``expand`` builds filldiag(B_S, gamma_S) (Sec. II: rows/columns repeated s_i
  times, deleted when s_i = 0, diagonal replaced; Eqs. (2), (11), (12)).
* ``pure_state_params`` / ``probability`` assemble the pure-state displaced
  probability of Eq. (12) with p(vac) of Eq. (10) and A of Eq. (4), using
  numpy's inverse and determinant as library steps.  The loop-weight vector is
  the half of Q^-1 alpha that pairs with B (reading R1 of the design notes: the
  literal block order of Eq. (9) pairs it with B*, which the Fock-space test in
  tests/test_oracle_probability.py rules out).
* Exact references used as pins: telephone numbers, double factorials, Ryser's
  permanent over the integers, exact enumeration of matchings, and an mpmath
  evaluation of the definition.

parity pins: every function above is pinned by tests/test_oracle_*.py.
"""
import ctypes
import functools
import math
import os

import numpy as np

from . import build as _build

_LIB = None
DP_MAX_N = 26
PT_MAX_N = 64


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        for sfx, real in (("d", ctypes.c_double), ("ld", ctypes.c_longdouble)):
            rp = ctypes.POINTER(real)
            getattr(lib, f"oracle_lhaf_dp_{sfx}").argtypes = [dp, ctypes.c_int, rp]
            getattr(lib, f"oracle_lhaf_pt_{sfx}").argtypes = [dp, ctypes.c_int, ctypes.c_int, rp, rp]
            getattr(lib, f"oracle_term_{sfx}").argtypes = [dp, ctypes.c_int, ctypes.c_ulonglong, rp]
            getattr(lib, f"oracle_terms_{sfx}").argtypes = [dp, ctypes.c_int, ctypes.POINTER(ctypes.c_ulonglong),
                                                            ctypes.c_longlong, ctypes.c_int, rp]
            getattr(lib, f"oracle_charpoly_{sfx}").argtypes = [dp, ctypes.c_int, rp]
            getattr(lib, f"oracle_power_traces_{sfx}").argtypes = [dp, ctypes.c_int, ctypes.c_int, rp]
            for name in ("lhaf_dp", "lhaf_pt", "term", "terms", "charpoly", "power_traces"):
                getattr(lib, f"oracle_{name}_{sfx}").restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _prec(prec):
    if prec in ("d", "double", "fp64"):
        return "d", ctypes.c_double, np.float64
    if prec in ("ld", "longdouble"):
        return "ld", ctypes.c_longdouble, np.longdouble
    raise ValueError(f"unknown precision {prec!r}")


def _as_input(A):
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    return A, A.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _out(n, prec):
    _, ct, nt = _prec(prec)
    buf = np.zeros(n, dtype=nt)
    return buf, buf.ctypes.data_as(ctypes.POINTER(ct))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def max_threads():
    return _lib().oracle_max_threads()


def lhaf_dp(A, prec="ld"):
    """lhaf by memoised enumeration of single-pair matchings (the definition)."""
    A, ap = _as_input(A)
    N = A.shape[0]
    sfx = _prec(prec)[0]
    out, op = _out(2, prec)
    _check(getattr(_lib(), f"oracle_lhaf_dp_{sfx}")(ap, N, op), "lhaf_dp")
    return complex(float(out[0]), float(out[1])) if sfx == "d" else (out[0], out[1])


def lhaf_pt(A, prec="ld", nthreads=0, with_abs=False):
    """lhaf by the power-trace subset sum (Sec. IV).  Returns complex for
    prec='d' and an (re, im) pair of np.longdouble for prec='ld'; with
    with_abs=True also sum_S |t_S|."""
    A, ap = _as_input(A)
    N = A.shape[0]
    sfx = _prec(prec)[0]
    out, op = _out(2, prec)
    ab, abp = _out(1, prec)
    _check(getattr(_lib(), f"oracle_lhaf_pt_{sfx}")(ap, N, int(nthreads), op, abp), "lhaf_pt")
    val = complex(float(out[0]), float(out[1])) if sfx == "d" else (out[0], out[1])
    return (val, ab[0]) if with_abs else val


def term(A, mask, prec="ld"):
    """One signed subset term t_S of the power-trace sum for pair subset ``mask``
    (bit i set = pair (i, i+n) kept; n = ceil(N/2))."""
    A, ap = _as_input(A)
    N = A.shape[0]
    sfx = _prec(prec)[0]
    out, op = _out(2, prec)
    _check(getattr(_lib(), f"oracle_term_{sfx}")(ap, N, ctypes.c_ulonglong(int(mask)), op), "term")
    return complex(float(out[0]), float(out[1]))


def terms(A, masks, prec="ld", nthreads=0):
    """Signed subset terms for an array of masks (threads over the list)."""
    A, ap = _as_input(A)
    N = A.shape[0]
    sfx = _prec(prec)[0]
    mk = np.ascontiguousarray(masks, dtype=np.uint64)
    out, op = _out(2 * mk.shape[0], prec)
    _check(getattr(_lib(), f"oracle_terms_{sfx}")(ap, N, mk.ctypes.data_as(ctypes.POINTER(ctypes.c_ulonglong)),
                                                  mk.shape[0], int(nthreads), op), "terms")
    o = out.astype(np.float64)
    return o[0::2] + 1j * o[1::2]


def charpoly(M, prec="ld"):
    """Coefficients c[t] of x^t in det(xI - M) (Hessenberg + La Budde)."""
    M, mp = _as_input(M)
    m = M.shape[0]
    sfx = _prec(prec)[0]
    out, op = _out(2 * (m + 1), prec)
    _check(getattr(_lib(), f"oracle_charpoly_{sfx}")(mp, m, op), "charpoly")
    o = out.astype(np.float64)
    return o[0::2] + 1j * o[1::2]


def power_traces(M, K, prec="ld"):
    """tr(M^k), k = 1..K (Hessenberg + La Budde + Newton's identities)."""
    M, mp = _as_input(M)
    m = M.shape[0]
    sfx = _prec(prec)[0]
    out, op = _out(2 * K, prec)
    _check(getattr(_lib(), f"oracle_power_traces_{sfx}")(mp, m, int(K), op), "power_traces")
    o = out.astype(np.float64)
    return o[0::2] + 1j * o[1::2]


def to_complex(val):
    """(re, im) long-double pair or complex -> Python complex."""
    if isinstance(val, tuple):
        return complex(float(val[0]), float(val[1]))
    return complex(val)


# ---------------------------------------------------------------------------
# pattern expansion and the pure-state probability (Sec. II)
# ---------------------------------------------------------------------------

def expand(B, gamma, pattern):
    """filldiag(B_S, gamma_S): row/column i of B repeated pattern[i] times
    (dropped when 0), then the main diagonal replaced by gamma repeated the same
    way.  gamma=None keeps B's own diagonal."""
    B = np.asarray(B, dtype=np.complex128)
    idx = [i for i, s in enumerate(pattern) for _ in range(int(s))]
    A = B[np.ix_(idx, idx)].copy()
    if gamma is not None:
        g = np.asarray(gamma, dtype=np.complex128)
        A[np.diag_indices(len(idx))] = g[idx]
    return A


def pure_state_params(Q, alpha_vec):
    """(B, gamma, p_vac) of a pure Gaussian state from Q = Sigma + I/2 and the
    mean vector alpha = [a; conj(a)]:
      A = X (I - Q^-1)                     Eq. (4), B = A[:M, :M]
      gamma = (Q^-1 alpha)[M:] = conj(a) - B a   (reading R1)
      p(vac) = exp(-alpha^H Q^-1 alpha / 2) / sqrt(det Q)   Eq. (10)"""
    Q = np.asarray(Q, dtype=np.complex128)
    al = np.asarray(alpha_vec, dtype=np.complex128)
    M2 = Q.shape[0]
    M = M2 // 2
    Qinv = np.linalg.inv(Q)
    X = np.block([[np.zeros((M, M)), np.eye(M)], [np.eye(M), np.zeros((M, M))]])
    A = X @ (np.eye(M2) - Qinv)
    B = A[:M, :M]
    gamma = (Qinv @ al)[M:]
    detQ = np.linalg.det(Q)
    quad = np.vdot(al, Qinv @ al)
    p_vac = float(np.exp(-0.5 * quad.real) / math.sqrt(detQ.real))
    return B, gamma, p_vac


def probability(Q, alpha_vec, pattern, prec="ld", lhaf_fn=None):
    """p(S) = p(vac) |lhaf(filldiag(B_S, gamma_S))|^2 / prod s_i!   (Eq. (12))."""
    B, gamma, p_vac = pure_state_params(Q, alpha_vec)
    Aexp = expand(B, gamma, pattern)
    if lhaf_fn is None:
        lh = to_complex(lhaf_pt(Aexp, prec=prec)) if Aexp.shape[0] else 1.0
    else:
        lh = lhaf_fn(Aexp)
    fact = 1
    for s in pattern:
        fact *= math.factorial(int(s))
    return p_vac * abs(lh) ** 2 / fact, lh


def mixed_state_params(Q, alpha_vec=None):
    """(A, gamma, p_vac) of a general (mixed) Gaussian state:
      A = X (I - Q^-1)                                      Eq. (4), 2M x 2M
      gamma = X Q^-1 alpha: entry k is the loop weight of index k of A (the
              half of Q^-1 alpha that pairs with each block, as in reading R1;
              for a pure state its first half is the pure-state gamma)
      p(vac) = exp(-alpha^H Q^-1 alpha / 2) / sqrt(det Q)   Eq. (10)"""
    Q = np.asarray(Q, dtype=np.complex128)
    M2 = Q.shape[0]
    M = M2 // 2
    al = np.zeros(M2, dtype=np.complex128) if alpha_vec is None else np.asarray(alpha_vec, dtype=np.complex128)
    Qinv = np.linalg.inv(Q)
    X = np.block([[np.zeros((M, M)), np.eye(M)], [np.eye(M), np.zeros((M, M))]])
    A = X @ (np.eye(M2) - Qinv)
    gamma = X @ (Qinv @ al)
    detQ = np.linalg.det(Q)
    quad = np.vdot(al, Qinv @ al)
    p_vac = float(np.exp(-0.5 * quad.real) / math.sqrt(detQ.real))
    return A, gamma, p_vac


def expand_mixed(A, gamma, pattern):
    """filldiag(A_S, gamma_S) of Eq. (11): rows and columns i and i + M of the
    2M x 2M matrix A repeated s_i times (copies of first-half indices, then of
    second-half indices), the diagonal replaced by gamma repeated the same way."""
    M = len(pattern)
    idx = [i for i, s in enumerate(pattern) for _ in range(int(s))]
    idx = idx + [i + M for i in idx]
    As = np.asarray(A, dtype=np.complex128)[np.ix_(idx, idx)].copy()
    As[np.diag_indices(len(idx))] = np.asarray(gamma, dtype=np.complex128)[idx]
    return As


def probability_mixed(Q, alpha_vec, pattern, prec="ld", gamma_fn=None):
    """p(S) = p(vac) lhaf(filldiag(A_S, gamma_S)) / prod s_i!   (Eq. (11)).
    Returns (p, lhaf); p is the real part (the loop hafnian of a valid state is
    real and non-negative).  gamma_fn(Q, alpha) overrides the loop weights (used
    by tests of alternative readings)."""
    A, gamma, p_vac = mixed_state_params(Q, alpha_vec)
    if gamma_fn is not None:
        gamma = gamma_fn(Q, alpha_vec)
    As = expand_mixed(A, gamma, pattern)
    lh = to_complex(lhaf_pt(As, prec=prec)) if As.shape[0] else 1.0
    fact = 1
    for s in pattern:
        fact *= math.factorial(int(s))
    return p_vac * complex(lh).real / fact, lh


# ---------------------------------------------------------------------------
# exact references (pins)
# ---------------------------------------------------------------------------

def telephone(n):
    """Number of involutions of n elements = lhaf of the n x n all-ones matrix
    (caption of Fig. 2): T(0) = T(1) = 1, T(n) = T(n-1) + (n-1) T(n-2)."""
    a, b = 1, 1
    for k in range(2, n + 1):
        a, b = b, b + (k - 1) * a
    return b if n >= 1 else 1


def double_factorial(k):
    out = 1
    while k > 1:
        out *= k
        k -= 2
    return out


def ryser_permanent(B):
    """perm(B) over the integers (or Python complex) by Ryser's formula."""
    B = [list(row) for row in B]
    n = len(B)
    total = 0
    for sub in range(1, 1 << n):
        cols = [j for j in range(n) if sub >> j & 1]
        prod = 1
        for i in range(n):
            prod *= sum(B[i][j] for j in cols)
        total += (-1) ** len(cols) * prod
    return (-1) ** n * total


def lhaf_enumerate(A, loops=True):
    """Exact enumeration of single-pair matchings (loops=True) or perfect
    matchings (loops=False) with Python arithmetic -- exact for integer or
    Gaussian-integer entries of moderate size.  Tiny N only."""
    A = [list(row) for row in A]
    N = len(A)

    @functools.lru_cache(maxsize=None)
    def rec(rem):
        if not rem:
            return 1
        i = rem[0]
        rest = rem[1:]
        tot = A[i][i] * rec(rest) if loops else 0
        for k, j in enumerate(rest):
            tot += A[i][j] * rec(rest[:k] + rest[k + 1:])
        return tot

    return rec(tuple(range(N)))


def lhaf_mpmath(A, dps=50, exact=False):
    """The definition evaluated in mpmath at ``dps`` digits (memoised over
    vertex subsets), for accuracy references at N <= 16.  Returns a Python
    complex (rounded to double), or with exact=True the mpmath value itself."""
    import mpmath

    A = np.asarray(A, dtype=np.complex128)
    N = A.shape[0]
    with mpmath.workdps(dps):
        M = [[mpmath.mpc(A[i, j].real, A[i, j].imag) for j in range(N)] for i in range(N)]
        f = [mpmath.mpc(0)] * (1 << N)
        f[0] = mpmath.mpc(1)
        for mask in range(1, 1 << N):
            i = (mask & -mask).bit_length() - 1
            rest = mask & ~(1 << i)
            tot = M[i][i] * f[rest]
            r = rest
            while r:
                j = (r & -r).bit_length() - 1
                tot += M[i][j] * f[rest & ~(1 << j)]
                r &= r - 1
            f[mask] = tot
        return f[(1 << N) - 1] if exact else complex(f[(1 << N) - 1])
