"""The conditional sampling chain (Sec. III) on the GPU against the oracle.

Both sides take the same normals and uniforms.  The oracle conditions each
state in numpy and evaluates every probability with its own loop hafnian; the
library conditions the covariance once on the host and runs every per-sample
step (outcomes, loop weights, matrices, loop hafnians, draws) in its kernels.
Draws must agree exactly unless a uniform falls within rounding of a CDF
boundary; the normalised probabilities behind every draw must agree to 1e-10.
"""
import math

import numpy as np
import pytest

from oracle import sampler as osampler
import oracle
from paper_2010_15595_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gbs():
    import paper_2010_15595_amd as g

    g.init(0)
    return g


def _compare(gbs, Q, al, cutoff, z, u, idx=None, tol=1e-10):
    s, pr, info = gbs.sample_pure(Q, al, cutoff, z, u, with_probs=True, with_info=True)
    M = Q.shape[0] // 2
    assert s.shape == (u.shape[0], M)
    idx = range(u.shape[0]) if idx is None else idx
    worst = 0.0
    for b in idx:
        ref, rp = osampler.sample_chain(Q, al, cutoff, z[b], u[b], return_probs=True)
        for k in range(M):
            worst = max(worst, np.abs(pr[b, k] - rp[k]).max())
            assert np.abs(pr[b, k] - rp[k]).max() <= tol, (b, k, pr[b, k], rp[k])
            if s[b, k] != ref[k]:
                # a draw may differ only when u lies within rounding of a CDF boundary
                cdf = np.cumsum(rp[k])
                assert np.abs(cdf - u[b, k]).min() < 1e-9, (b, k, s[b], ref)
                break
    print(f"[sampler M={M} cutoff={cutoff} n={u.shape[0]}] max |dp|={worst:.2e} info={info}", flush=True)
    return s, pr, info


@pytest.mark.parametrize("M,r,sigma,cutoff,seed", [(2, 0.6, 0.3, 5, 1), (3, 0.5, 0.0, 6, 2), (4, 0.7, 0.4, 4, 3),
                                                   (5, 0.5, 0.2, 3, 4)])
def test_chain_matches_oracle(gbs, M, r, sigma, cutoff, seed):
    st = workloads.pure_state(M, r, sigma, seed=seed)
    rng = np.random.default_rng(100 + seed)
    n = 40
    z, u = rng.standard_normal((n, 2 * (M - 1))), rng.random((n, M))
    _compare(gbs, st["Q"], st["alpha_vec"], cutoff, z, u)


def test_single_mode_needs_no_normals(gbs):
    st = workloads.pure_state(1, 0.8, 0.5, seed=7)
    u = np.random.default_rng(1).random((30, 1))
    s, pr = gbs.sample_pure(st["Q"], st["alpha_vec"], 8, np.zeros((30, 0)), u, with_probs=True)
    ref = [oracle.probability(st["Q"], st["alpha_vec"], [j])[0] for j in range(9)]
    ref = np.array(ref) / np.sum(ref)
    assert np.abs(pr[:, 0, :] - ref[None, :]).max() < 1e-12
    for b in range(30):
        assert s[b, 0] == min(int(np.searchsorted(np.cumsum(ref), u[b, 0], side="right")), 8)


def test_coherent_product_state_gives_poisson_draws(gbs):
    """Closed form, independent of the oracle: a coherent product state has
    independent Poisson photon numbers, whatever the heterodyne outcomes."""
    a = np.array([0.8 + 0.3j, -0.5j, 1.1 + 0.0j, 0.2 - 0.4j])
    M = len(a)
    Q = np.eye(2 * M, dtype=complex)
    al = np.concatenate([a, np.conj(a)])
    rng = np.random.default_rng(3)
    n, cutoff = 200, 12
    z, u = rng.standard_normal((n, 2 * (M - 1))), rng.random((n, M))
    s, pr = gbs.sample_pure(Q, al, cutoff, z, u, with_probs=True)
    for k in range(M):
        lam = abs(a[k]) ** 2
        p = np.array([math.exp(-lam) * lam ** j / math.factorial(j) for j in range(cutoff + 1)])
        p /= p.sum()
        assert np.abs(pr[:, k, :] - p[None, :]).max() < 1e-13
        cdf = np.cumsum(p)
        for b in range(n):
            assert s[b, k] == min(int(np.searchsorted(cdf, u[b, k], side="right")), cutoff)


def test_cutoff_zero_and_empty(gbs):
    st = workloads.pure_state(3, 0.5, 0.2, seed=5)
    rng = np.random.default_rng(2)
    s, pr = gbs.sample_pure(st["Q"], st["alpha_vec"], 0, rng.standard_normal((5, 4)), rng.random((5, 3)),
                            with_probs=True)
    assert (s == 0).all() and np.allclose(pr, 1.0)
    s = gbs.sample_pure(st["Q"], st["alpha_vec"], 4, np.zeros((0, 4)), np.zeros((0, 3)))
    assert s.shape == (0, 3)


def test_groups_of_samples(gbs):
    """More samples than one lockstep group (8192): samples on both sides of
    the group boundary follow the oracle."""
    st = workloads.pure_state(3, 0.5, 0.3, seed=8)
    rng = np.random.default_rng(4)
    n = 8192 + 300
    z, u = rng.standard_normal((n, 4)), rng.random((n, 3))
    _, _, info = _compare(gbs, st["Q"], st["alpha_vec"], 5, z, u,
                          idx=[0, 1, 8190, 8191, 8192, 8193, n - 2, n - 1])
    assert info["groups"] == 2
    assert info["loop_hafnians"] == n * 3 * 6


def test_too_many_photons_is_an_error(gbs):
    """Bright coherent light (mean 33.6 photons per mode): photons so far plus
    the cutoff exceed 64 at mode 2 for some of the samples."""
    a = np.array([5.8 + 0.0j, 5.8 + 0.0j])
    Q = np.eye(4, dtype=complex)
    al = np.concatenate([a, np.conj(a)])
    rng = np.random.default_rng(5)
    with pytest.raises(gbs.GbsError) as e:
        gbs.sample_pure(Q, al, 34, rng.standard_normal((16, 2)), rng.random((16, 2)))
    assert e.value.code == -4


def test_fp32_path_probabilities(gbs):
    st = workloads.pure_state(4, 0.6, 0.3, seed=9)
    rng = np.random.default_rng(6)
    z, u = rng.standard_normal((30, 6)), rng.random((30, 4))
    _, p64 = gbs.sample_pure(st["Q"], st["alpha_vec"], 5, z, u, with_probs=True)
    s32, p32 = gbs.sample_pure(st["Q"], st["alpha_vec"], 5, z, u, prec=gbs.GBS_FP32_COMP, with_probs=True)
    s64 = gbs.sample_pure(st["Q"], st["alpha_vec"], 5, z, u)
    same = (s32 == s64).all(axis=1)
    # where the draws agree the conditional probabilities agree to FP32 accuracy
    assert same.mean() > 0.9
    assert np.abs(p32[same] - p64[same]).max() < 1e-4


def test_total_variation_distance(gbs):
    """Fig. 1 in miniature on the GPU: 4 modes, r = 0.5, cutoff 6, 40000
    samples against the exact distribution, judged against exact samplers
    drawing as many samples."""
    M, cutoff, n = 4, 6, 40000
    st = workloads.pure_state(M, 0.5, 0.0, seed=12)
    Q, al = st["Q"], st["alpha_vec"]
    pats, probs = osampler.exact_distribution(Q, al, cutoff)
    probs = probs / probs.sum()
    rng = np.random.default_rng(21)
    s = gbs.sample_pure(Q, al, cutoff, rng.standard_normal((n, 2 * (M - 1))), rng.random((n, M)))
    codes = s @ ((cutoff + 1) ** np.arange(M - 1, -1, -1))
    emp = np.bincount(codes, minlength=(cutoff + 1) ** M) / n
    pcode = pats @ ((cutoff + 1) ** np.arange(M - 1, -1, -1))
    ref = np.zeros_like(emp)
    ref[pcode] = probs
    tvd = 0.5 * np.abs(emp - ref).sum()
    exact = [0.5 * np.abs(rng.multinomial(n, ref) / n - ref).sum() for _ in range(400)]
    q = np.quantile(exact, [0.5, 0.995])
    print(f"[tvd] M={M} cutoff={cutoff} n={n}: tvd={tvd:.4f} exact-sampler median {q[0]:.4f}, 99.5% {q[1]:.4f}",
          flush=True)
    assert tvd <= q[1]
