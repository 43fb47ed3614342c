"""Seeded synthetic workloads (inputs only).

This module builds the inputs that both the tests/benchmark (through the HIP
library) and the CPU oracle consume.  It holds none of the loop-hafnian or
probability arithmetic: it draws random states and photon patterns following
the workload recipes and returns arrays.

State recipe (pure Gaussian state, Sec. II of the paper):
  * U Haar-random M x M unitary (QR of a complex Ginibre matrix, phases fixed),
  * B = U diag(tanh r) U^T  (the "A = B (+) B*" block of a pure state),
  * displacement a_i ~ CN(0, sigma^2): Re, Im i.i.d. N(0, sigma^2 / 2),
  * loop weights gamma = conj(a) - B a (the diagonal that replaces B's in the
    loop-hafnian matrix of the displaced pure state),
  * Q = (I - X (B (+) conj B))^-1 and alpha = [a; conj(a)] for the probability
    interface (the inverse of A = X (I - Q^-1), Eq. (4)).

Photon patterns:
  * C1  M=16, r=1.0, sigma=0.3, one photon in every mode           -> N=16
  * C2  M=64, r=0.8, sigma=0.2, 20 modes, 1 + Multinomial(12)       -> N=32
  * C3  M=100, r=1.2, sigma=0.1, N distinct modes (N = 40, 44, 50)
  * C4  M=100, r=1.0, sigma=0.2, 4096 chain-like patterns, N in 2*U{5..18}
  * E2  all-ones n x n matrix (accuracy figure of the paper)
  * E3  Re, Im ~ U[0, 1), symmetrised (R + R^T)/2 (timing figure of the paper)
"""
import numpy as np


def haar_unitary(M, rng):
    Z = (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))) / np.sqrt(2.0)
    Qm, Rm = np.linalg.qr(Z)
    ph = np.diag(Rm)
    ph = ph / np.abs(ph)
    return Qm * ph[None, :]


def pure_state(M, r, sigma, seed=0):
    """Random pure displaced squeezed state.  Returns a dict with B (M x M),
    a (M,), gamma (M,), Q (2M x 2M) and alpha_vec (2M,)."""
    rng = np.random.default_rng(seed)
    U = haar_unitary(M, rng)
    rs = np.full(M, float(r)) if np.isscalar(r) else np.asarray(r, dtype=float)
    B = U @ np.diag(np.tanh(rs)) @ U.T
    B = (B + B.T) / 2
    a = (rng.standard_normal(M) + 1j * rng.standard_normal(M)) * (sigma / np.sqrt(2.0))
    gamma = np.conj(a) - B @ a
    Z = np.zeros((M, M))
    X = np.block([[Z, np.eye(M)], [np.eye(M), Z]])
    Afull = np.block([[B, Z], [Z, np.conj(B)]])
    Q = np.linalg.inv(np.eye(2 * M) - X @ Afull)
    alpha_vec = np.concatenate([a, np.conj(a)])
    return dict(B=B, a=a, gamma=gamma, Q=Q, alpha_vec=alpha_vec, U=U, r=rs)


def config1(seed=0):
    st = pure_state(16, 1.0, 0.3, seed)
    st["pattern"] = np.ones(16, dtype=np.int32)
    st["name"] = "lhaf N=16 (M=16, r=1.0, one photon per mode)"
    return st


def config2(seed=0):
    st = pure_state(64, 0.8, 0.2, seed)
    rng = np.random.default_rng(seed + 1000)
    modes = rng.choice(64, size=20, replace=False)
    mult = 1 + rng.multinomial(12, np.full(20, 1 / 20))
    pat = np.zeros(64, dtype=np.int32)
    pat[modes] = mult
    st["pattern"] = pat
    st["name"] = "lhaf N=32 (M=64, r=0.8, 32 photons on 20 modes)"
    return st


def config3(N, seed=0):
    st = pure_state(100, 1.2, 0.1, seed)
    rng = np.random.default_rng(seed + 2000 + N)
    modes = rng.choice(100, size=N, replace=False)
    pat = np.zeros(100, dtype=np.int32)
    pat[modes] = 1
    st["pattern"] = pat
    st["name"] = f"lhaf N={N} (M=100, r=1.2, {N} distinct modes)"
    return st


def config4_patterns(count=4096, M=100, cutoff=6):
    """Chain-like patterns: for item i (seed i), N_i = 2*U{5..18}, k_i ~
    U{N_i..M}, N_i photons placed i.i.d. uniformly on modes 0..k_i-1, any draw
    that would put more than ``cutoff`` photons in a mode is redrawn."""
    pats = []
    for i in range(count):
        rng = np.random.default_rng(i)
        N = 2 * int(rng.integers(5, 19))
        k = int(rng.integers(N, M + 1))
        pat = np.zeros(M, dtype=np.int32)
        placed = 0
        while placed < N:
            j = int(rng.integers(0, k))
            if pat[j] < cutoff:
                pat[j] += 1
                placed += 1
        pats.append(pat)
    return pats


def config4(count=4096, seed=0):
    st = pure_state(100, 1.0, 0.2, seed)
    st["patterns"] = config4_patterns(count)
    st["name"] = f"batched {count} lhafs, N in [10,36] (M=100, r=1.0)"
    return st


def allones(n):
    return np.ones((n, n), dtype=np.complex128)


def random_uniform_symmetric(N, seed=0):
    """Re, Im ~ U[0, 1), then (R + R^T)/2 (the paper's timing inputs)."""
    rng = np.random.default_rng(seed)
    R = rng.random((N, N)) + 1j * rng.random((N, N))
    return (R + R.T) / 2


def random_normal_symmetric(N, seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    R = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * scale
    return (R + R.T) / 2
