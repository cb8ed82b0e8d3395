"""Pins of the oracle's RK4 integration (Eq. (10), Table 1 step 3.1)."""
import numpy as np
import pytest
import scipy.linalg

import brute
from paper_1912_01491_amd import workloads as wl


def exact_affine(Q, K, v0, T):
    """v(T) of dv/dt = Qv + K from the exponential of the augmented matrix."""
    M = len(K)
    A = np.zeros((M + 1, M + 1))
    A[:M, :M] = Q
    A[:M, M] = K
    E = scipy.linalg.expm(A * T)
    return E[:M, :M] @ v0 + E[:M, M]


def test_bloch_rk4_vs_exponential(oracle):
    omega, g = 1.3, 0.4
    Q = np.array([[-g / 2, -omega, 0], [omega, -g / 2, 0], [0, 0, -g]])
    K = np.array([0, 0, g / np.sqrt(2)])
    v0 = np.array([0.3, -0.2, 0.5])
    v = oracle.rk4_dense(Q, K, v0, 1e-3, 1000)[0]
    assert np.abs(v - exact_affine(Q, K, v0, 1.0)).max() < 1e-13


@pytest.mark.parametrize("N", [3, 4])
def test_rk4_fourth_order(oracle, N):
    H, gamma = wl.random_lindbladian(N, 11)
    Q, K = oracle.prepare_dense(H, gamma)
    psi = wl.random_pure_state(N, 2)
    v0 = oracle.expand(np.outer(psi, psi.conj())).real
    ref = exact_affine(Q, K, v0, 0.5)
    e1 = np.abs(oracle.rk4_dense(Q, K, v0, 0.05, 10)[0] - ref).max()
    e2 = np.abs(oracle.rk4_dense(Q, K, v0, 0.025, 20)[0] - ref).max()
    assert e1 / e2 > 12  # 2^4 = 16 for a fourth-order method


def test_rk4_many_states_and_csr(oracle):
    N = 4
    H, gamma = wl.random_lindbladian(N, 12)
    Q, K = oracle.prepare_dense(H, gamma)
    psis = wl.random_pure_states(N, 3, 5)
    V0 = np.array([oracle.expand(np.outer(p, p.conj())).real for p in psis])
    V = oracle.rk4_dense(Q, K, V0, 1e-3, 200)
    for b in range(3):
        assert np.array_equal(V[b], oracle.rk4_dense(Q, K, V0[b], 1e-3, 200)[0])
    nz = Q != 0
    rowptr = np.concatenate([[0], np.cumsum(nz.sum(1))])
    r, c = np.nonzero(nz)
    Vc = oracle.rk4_csr(rowptr, c, Q[r, c], K, V0, 1e-3, 200)
    assert np.abs(Vc - V).max() < 1e-14


def test_trajectory_stays_a_density_matrix(oracle):
    N = 4
    H, gamma = wl.random_lindbladian(N, 13)
    Q, K = oracle.prepare_dense(H, gamma)
    psi = wl.random_pure_state(N, 1)
    v = oracle.expand(np.outer(psi, psi.conj())).real
    for _ in range(10):
        v = oracle.rk4_dense(Q, K, v, 1e-2, 20)[0]
        rho = oracle.reconstruct(N, v)
        assert abs(np.trace(rho) - 1) < 1e-14
        assert np.abs(rho - rho.conj().T).max() < 1e-15
        assert np.linalg.eigvalsh(rho).min() > -1e-10


def test_unital_purity_decreases(oracle):
    N = 3
    M = N * N - 1
    Q, K = oracle.prepare_dense(np.diag([0.1, 0.5, -0.3]).astype(complex), 0.2 * np.eye(M))
    psi = wl.random_pure_state(N, 4)
    v = oracle.expand(np.outer(psi, psi.conj())).real
    pur = [1 / N + v @ v]
    for _ in range(5):
        v = oracle.rk4_dense(Q, K, v, 1e-2, 10)[0]
        pur.append(1 / N + v @ v)
    assert all(b < a for a, b in zip(pur, pur[1:]))
    # depolarizing closed form: |v(t)| = |v0| exp(-cN t)
    assert pur[-1] - 1 / N == pytest.approx((pur[0] - 1 / N) * np.exp(-2 * 0.2 * N * 0.5), rel=1e-9)
