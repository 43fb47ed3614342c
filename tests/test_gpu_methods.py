"""La Budde against diagonalisation (Sec. IV) on the LDS-resident reference
kernels: both methods take the same bordered Hessenberg matrices and feed the
same series; only the characteristic polynomials differ.  Both must agree with
the oracle; the double-double path through the same entry point must equal
gbs_lhaf with GBS_DD.
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


def _matrix(N, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    return (A + A.T) / 2


@pytest.mark.parametrize("N,seed", [(1, 0), (6, 1), (11, 2), (16, 3), (24, 4)])
def test_both_methods_match_the_oracle(gbs, N, seed):
    A = _matrix(N, seed)
    ld, ab = oracle.lhaf_pt(A, prec="ld", with_abs=True)
    ref = oracle.to_complex(ld)
    ab = float(ab)
    lb = gbs.lhaf_method(A, gbs.GBS_CHARPOLY_LABUDDE)
    ev = gbs.lhaf_method(A, gbs.GBS_CHARPOLY_EIGEN)
    e_lb, e_ev = abs(lb - ref) / ab, abs(ev - ref) / ab
    print(f"[methods N={N}] |labudde-ld|/sum|t| {e_lb:.2e}, |eigen-ld|/sum|t| {e_ev:.2e}", flush=True)
    assert e_lb <= 2e-14
    assert e_ev <= 1e-11


def test_benchmark_family(gbs):
    """N = 32 of the benchmark family against the double-double value."""
    st = workloads.config3(32)
    A = gbs.expand(st["B"], st["gamma"], st["pattern"])
    ref, d = gbs.lhaf(A, prec=gbs.GBS_DD, with_diag=True)
    lb = gbs.lhaf_method(A, gbs.GBS_CHARPOLY_LABUDDE)
    ev = gbs.lhaf_method(A, gbs.GBS_CHARPOLY_EIGEN)
    prod = gbs.lhaf(A)
    e = {k: abs(v - ref) / d["abs_sum"] for k, v in (("labudde", lb), ("eigen", ev), ("production", prod))}
    print(f"[methods N=32] kappa {d['kappa']:.2e}: " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()), flush=True)
    assert e["labudde"] <= 2e-14 and e["production"] <= 2e-14
    assert e["eigen"] <= 1e-11


def test_allones_matrices(gbs):
    """Degenerate spectra: subsets of the all-ones matrix."""
    for n in (8, 13, 20):
        T = oracle.telephone(n)
        for method in (gbs.GBS_CHARPOLY_LABUDDE, gbs.GBS_CHARPOLY_EIGEN):
            v, d = gbs.lhaf_method(np.ones((n, n), dtype=complex), method, with_diag=True)
            assert abs(v - T) <= 1e-11 * d["abs_sum"], (n, method, v, T)


def test_double_double_through_the_method_entry(gbs):
    A = _matrix(14, 9)
    a, da = gbs.lhaf_method(A, gbs.GBS_CHARPOLY_LABUDDE, prec=gbs.GBS_DD, with_diag=True)
    b, db = gbs.lhaf(A, prec=gbs.GBS_DD, with_diag=True)
    assert a == b and da["lhaf_lo"] == db["lhaf_lo"]
