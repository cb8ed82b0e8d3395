"""Brute-force references for tiny N (numpy, dense matrices).

Independent of the oracle: the basis is built here from the generator
definitions (Sec. 2, Eqs. (3)-(5), with D^l read as Hermitian and
orthonormal), and Q, K are obtained by projecting the matrix-form
Lindbladian (Eqs. (1), (2)) onto the basis:

    Q_sn = Tr(F_s L(F_n)),   K_s = Tr(F_s L(1/N)),

which follows from rho = 1/N + sum_n v_n F_n (Eq. (7)) and Tr(F_s F_n) = delta.
"""
import numpy as np


def basis(N):
    """F_0..F_{M-1}: S^(j,k) for j<k row-major, then J^(j,k), then D^1..D^{N-1}."""
    pairs = [(j, k) for j in range(N) for k in range(j + 1, N)]
    F = []
    for j, k in pairs:
        X = np.zeros((N, N), complex)
        X[j, k] = X[k, j] = 1 / np.sqrt(2)
        F.append(X)
    for j, k in pairs:
        X = np.zeros((N, N), complex)
        X[j, k] = -1j / np.sqrt(2)
        X[k, j] = 1j / np.sqrt(2)
        F.append(X)
    for l in range(1, N):
        d = np.zeros(N)
        d[:l] = 1.0
        d[l] = -l
        F.append(np.diag(d / np.sqrt(l * (l + 1))).astype(complex))
    return np.array(F)


def structure_constants(N):
    """f_mns = -i Tr(F_s [F_m, F_n]) and d_mns = Tr(F_s {F_m, F_n}) for all triples."""
    F = basis(N)
    T = np.einsum("mab,nbc,sca->mns", F, F, F)   # Tr(F_m F_n F_s)
    Tt = np.einsum("nab,mbc,sca->mns", F, F, F)  # Tr(F_n F_m F_s)
    f = (-1j * (T - Tt))
    d = (T + Tt)
    return f, d


def lindblad_apply(X, H, gamma=None, F=None, jumps=()):
    """L(X) = -i[H, X] + sum_jk gamma_jk (F_j X F_k - 1/2 {F_k F_j, X})
              + sum_p g_p (L_p X L_p^+ - 1/2 {L_p^+ L_p, X})."""
    out = -1j * (H @ X - X @ H)
    if gamma is not None:
        M = len(F)
        for j in range(M):
            FjX = F[j] @ X
            for k in range(M):
                g = gamma[j, k]
                if g == 0:
                    continue
                FkFj = F[k] @ F[j]
                out += g * (FjX @ F[k] - 0.5 * (FkFj @ X + X @ FkFj))
    for g, L in jumps:
        LdL = L.conj().T @ L
        out += g * (L @ X @ L.conj().T - 0.5 * (LdL @ X + X @ LdL))
    return out


def project(H, gamma=None, jumps=()):
    """Q (M x M) and K (M) by projection of the matrix-form Lindbladian."""
    N = H.shape[0]
    F = basis(N)
    M = len(F)
    Q = np.zeros((M, M), complex)
    for n in range(M):
        Y = lindblad_apply(F[n], H, gamma, F, jumps)
        Q[:, n] = np.einsum("sab,ba->s", F, Y)
    Y0 = lindblad_apply(np.eye(N) / N, H, gamma, F, jumps)
    K = np.einsum("sab,ba->s", F, Y0)
    return Q, K


def coherence_vector(rho):
    F = basis(rho.shape[0])
    return np.einsum("sab,ba->s", F, rho)
