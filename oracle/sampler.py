"""Oracle of the paper's sampling algorithm (Sec. III, Algorithm): test
infrastructure only, plain numpy on top of the oracle's pure-state probability.

Complex basis throughout: a state of M modes is (Q, alpha) with Q = Sigma + I/2
(2M x 2M, (a, a^dag) ordering) and alpha = [a; conj(a)].  Q is also the
covariance of the augmented heterodyne outcome [beta; conj(beta)]
(Husimi function), and heterodyne conditioning on modes B gives
  Sigma_A|B = Sigma_AA - Sigma_AB Q_BB^-1 Sigma_BA,
  alpha_A|B = alpha_A + Sigma_AB Q_BB^-1 ([beta; conj(beta)]_B - alpha_B),
the complex-basis form of the conditional covariance and mean of Sec. II.

Random numbers are inputs: per sample, 2 (M - 1) standard normals for the
heterodyne outcomes of modes 2..M and M uniforms for the photon numbers.
"""
import numpy as np

from . import probability


def _aug(modes, M):
    """Indices of (a_i, a_i^dag) for the given modes in the 2M space."""
    modes = list(modes)
    return modes + [i + M for i in modes]


def heterodyne_sample(Q, alpha_vec, modes, normals):
    """beta_B ~ complex normal with mean a_B and augmented covariance Q[B, B]
    (Husimi distribution of a heterodyne measurement, Sec. II).  `normals`: 2|B|
    standard normals.  Returns the complex outcomes of `modes`."""
    M = Q.shape[0] // 2
    idx = _aug(modes, M)
    C = np.asarray(Q, dtype=complex)[np.ix_(idx, idx)]
    mu = np.asarray(alpha_vec, dtype=complex)[idx]
    b = len(modes)
    # (Re beta, Im beta) = T [beta; conj(beta)], T = [[I, I], [-iI, iI]] / 2
    T = 0.5 * np.block([[np.eye(b), np.eye(b)], [-1j * np.eye(b), 1j * np.eye(b)]])
    R = (T @ C @ T.conj().T).real
    m = (T @ mu).real
    x = m + np.linalg.cholesky(R) @ np.asarray(normals, dtype=float)
    return x[:b] + 1j * x[b:]


def conditional_state(Q, alpha_vec, A, B, beta_B):
    """(Q_A|B, alpha_A|B) of modes A after heterodyne outcome beta_B on modes B."""
    Q = np.asarray(Q, dtype=complex)
    al = np.asarray(alpha_vec, dtype=complex)
    M = Q.shape[0] // 2
    ia, ib = _aug(A, M), _aug(B, M)
    S = Q - 0.5 * np.eye(2 * M)
    if len(B) == 0:
        return Q[np.ix_(ia, ia)], al[ia]
    G = S[np.ix_(ia, ib)] @ np.linalg.inv(Q[np.ix_(ib, ib)])
    S_A = S[np.ix_(ia, ia)] - G @ S[np.ix_(ib, ia)]
    bt = np.concatenate([beta_B, np.conj(beta_B)])
    a_A = al[ia] + G @ (bt - al[ib])
    return S_A + 0.5 * np.eye(len(ia)), a_A


def sample_chain(Q, alpha_vec, cutoff, normals, uniforms, prec="d", return_probs=False):
    """One sample of the Algorithm of Sec. III for a pure state: heterodyne
    outcomes for modes 2..M, then for k = 1..M the conditional pure state of
    modes 1..k, the probabilities of s_k = 0..cutoff (Eq. (12)) and an
    inverse-CDF draw.  Returns the photon pattern (M ints), and with
    return_probs also the (M, cutoff + 1) normalised probabilities drawn from."""
    M = np.asarray(Q).shape[0] // 2
    beta = heterodyne_sample(Q, alpha_vec, range(1, M), normals) if M > 1 else np.zeros(0, complex)
    s, probs = [], []
    for k in range(1, M + 1):
        A = list(range(k))
        B = list(range(k, M))
        QA, aA = conditional_state(Q, alpha_vec, A, B, beta[k - 1:])
        p = np.array([probability(QA, aA, s + [j], prec=prec)[0] for j in range(cutoff + 1)])
        probs.append(p / p.sum())
        cdf = np.cumsum(probs[-1])
        j = int(np.searchsorted(cdf, uniforms[k - 1], side="right"))
        s.append(min(j, cutoff))
    return (s, np.array(probs)) if return_probs else s


def exact_distribution(Q, alpha_vec, cutoff, prec="d"):
    """All patterns with s_i <= cutoff and their probabilities (Eq. (12))."""
    M = np.asarray(Q).shape[0] // 2
    pats = np.array(np.meshgrid(*[np.arange(cutoff + 1)] * M, indexing="ij")).reshape(M, -1).T
    probs = np.array([probability(Q, alpha_vec, list(p), prec=prec)[0] for p in pats])
    return pats, probs
