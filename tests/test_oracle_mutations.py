"""The oracle's pins must catch plausible mistakes.

Each case copies the oracle source to a temporary directory, plants one
mistake by text substitution, compiles it on the CPU and checks that the pin
set (definition by brute force, telephone numbers, rank-one closed form,
eigenvalue power traces) rejects it.  Nothing here touches the GPU.
"""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

SRC = os.path.dirname(oracle.__file__)

MUTATIONS = {
    "drop_loop_term": ("ws->c[k] = ws->p[k] / (REAL)(2 * k) + ws->q[k] / (REAL)2;",
                       "ws->c[k] = ws->p[k] / (REAL)(2 * k);"),
    "no_inclusion_exclusion_sign": ("return ((n - s) & 1) ? -ws->e[n] : ws->e[n];",
                                    "return ws->e[n];"),
    "no_pair_swap": ("int xr = r < s ? r + s : r - s;", "int xr = r;"),
    "labudde_transposed_entry": ("CPLX beta = HH(i - k, i) * prod;", "CPLX beta = HH(i, i - k) * prod;"),
    "newton_sign": ("for (int j = 1; j <= k - 1 && j <= m; ++j) acc -= coef[m - j] * p[k - j];",
                    "for (int j = 1; j <= k - 1 && j <= m; ++j) acc += coef[m - j] * p[k - j];"),
    "exp_recurrence_weight": ("acc += (REAL)j * ws->c[j] * ws->e[k - j];", "acc += ws->c[j] * ws->e[k - j];"),
    "householder_missing_conj": ("w += ZCONJ(v[r]) * H[r * m + c];", "w += v[r] * H[r * m + c];"),
    "loop_vector_unswapped": ("ws->zS[r] = Ap[idx[xr] * Np + idx[xr]];", "ws->zS[r] = Ap[idx[r] * Np + idx[r]];"),
}


def build_mutant(name, tmp):
    old, new = MUTATIONS[name]
    for f in ("lhaf_oracle.c", "lhaf_body.h"):
        shutil.copy(os.path.join(SRC, f), os.path.join(tmp, f))
    body = open(os.path.join(tmp, "lhaf_body.h")).read()
    assert body.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    open(os.path.join(tmp, "lhaf_body.h"), "w").write(body.replace(old, new))
    lib = os.path.join(tmp, "libmut.so")
    subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-o", lib,
                    os.path.join(tmp, "lhaf_oracle.c"), "-lm"], check=True)
    L = ctypes.CDLL(lib)
    rp = ctypes.POINTER(ctypes.c_longdouble)
    L.oracle_lhaf_pt_ld.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int, rp, rp]
    L.oracle_power_traces_ld.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int, rp]
    return L


def mut_lhaf(L, A):
    A = np.ascontiguousarray(A, dtype=np.complex128)
    out = np.zeros(2, dtype=np.longdouble)
    ab = np.zeros(1, dtype=np.longdouble)
    rc = L.oracle_lhaf_pt_ld(A.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), A.shape[0], 1,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_longdouble)),
                             ab.ctypes.data_as(ctypes.POINTER(ctypes.c_longdouble)))
    assert rc == 0
    return complex(float(out[0]), float(out[1])), float(ab[0])


def pins_pass(L):
    """True when every pin holds for library L."""
    r = np.random.default_rng(5)
    for N in (5, 8, 11):
        R = r.standard_normal((N, N)) + 1j * r.standard_normal((N, N))
        A = (R + R.T) / 2
        got, ab = mut_lhaf(L, A)
        if abs(got - oracle.to_complex(oracle.lhaf_dp(A, prec="ld"))) > 1e-16 * ab:
            return False
    for n in (6, 9):
        got, ab = mut_lhaf(L, np.ones((n, n), dtype=complex))
        if abs(got - oracle.telephone(n)) > 1e-17 * ab:
            return False
    v = r.standard_normal(7) + 1j * r.standard_normal(7)
    A = np.outer(v, v)
    np.fill_diagonal(A, v)
    got, ab = mut_lhaf(L, A)
    if abs(got - oracle.telephone(7) * np.prod(v)) > 1e-16 * ab:
        return False
    M = (r.standard_normal((9, 9)) + 1j * r.standard_normal((9, 9))) / 3
    p = np.zeros(2 * 12, dtype=np.longdouble)
    L.oracle_power_traces_ld(np.ascontiguousarray(M).view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             9, 12, p.ctypes.data_as(ctypes.POINTER(ctypes.c_longdouble)))
    lam = np.linalg.eigvals(M)
    for k in range(1, 13):
        got = complex(float(p[2 * k - 2]), float(p[2 * k - 1]))
        if abs(got - np.sum(lam**k)) > 1e-10 * np.sum(np.abs(lam) ** k):
            return False
    return True


def test_unmutated_copy_passes():
    with tempfile.TemporaryDirectory() as tmp:
        for f in ("lhaf_oracle.c", "lhaf_body.h"):
            shutil.copy(os.path.join(SRC, f), os.path.join(tmp, f))
        lib = os.path.join(tmp, "libmut.so")
        subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-o", lib,
                        os.path.join(tmp, "lhaf_oracle.c"), "-lm"], check=True)
        L = ctypes.CDLL(lib)
        rp = ctypes.POINTER(ctypes.c_longdouble)
        L.oracle_lhaf_pt_ld.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int, rp, rp]
        L.oracle_power_traces_ld.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int, rp]
        assert pins_pass(L)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    with tempfile.TemporaryDirectory() as tmp:
        L = build_mutant(name, tmp)
        assert not pins_pass(L), f"mutation {name} survived the pins"
