"""Pins of the oracle's driven integrator (the periodically rocked dimer of
Sec. 3, Eq. (16)): dv/dt = (Q0 + eps(t) Q1) v + K with the square wave
eps(t) = E + A Theta(t), Theta = +1 on [0, T/2) and -1 on [T/2, T).

The drive is piecewise constant, so over one period the exact solution is the
product of two affine exponentials; RK4 must converge to it. The inputs of the
rocked dimer are checked against an independent two-mode construction."""
import numpy as np
import pytest
from scipy.linalg import expm

import brute
from paper_1912_01491_amd import workloads as wl


def _system(oracle, N, seed):
    g = wl.rng(seed)
    H0 = wl.hermitize(wl.ginibre(g, N))
    H1 = wl.hermitize(wl.ginibre(g, N))
    L = wl.ginibre(g, N)
    Q0, K = oracle.prepare_factored(H0, [0.3], [L], np.arange(N * N - 1))
    Q1, K1 = oracle.prepare_factored(H1, [0.0], [np.zeros((N, N))], np.arange(N * N - 1))
    return Q0, Q1, K, K1


def test_drive_square_wave(oracle):
    E, A, T = -1.0, -1.5, 2.0
    assert oracle.drive(0.0, E, A, T) == E + A
    assert oracle.drive(0.999, E, A, T) == E + A
    assert oracle.drive(1.0, E, A, T) == E - A          # Theta = -1 from T/2 on
    assert oracle.drive(1.999, E, A, T) == E - A
    assert oracle.drive(2.0, E, A, T) == E + A          # periodic
    assert oracle.drive(4.25, E, A, T) == E + A
    assert oracle.drive(5.25, E, A, T) == E - A
    assert oracle.drive(-0.5, E, A, T) == E - A         # t < 0 folds into [T/2, T)
    # limits from the left: at a switch, the half period that ends there
    assert oracle.drive_left(1.0, E, A, T) == E + A
    assert oracle.drive_left(1.001, E, A, T) == E - A
    assert oracle.drive_left(2.0, E, A, T) == E - A
    assert oracle.drive_left(0.5, E, A, T) == E + A


def test_hamiltonian_part_is_linear_and_k_free(oracle):
    """Q of (H0 + e H1) = Q0 + e Q1 and the drive term adds nothing to K."""
    N = 3
    Q0, Q1, K, K1 = _system(oracle, N, 1)
    assert np.abs(K1).max() == 0.0
    g = wl.rng(1)
    H0 = wl.hermitize(wl.ginibre(g, N))
    H1 = wl.hermitize(wl.ginibre(g, N))
    L = wl.ginibre(g, N)
    Qe, Ke = oracle.prepare_factored(H0 + 0.7 * H1, [0.3], [L], np.arange(N * N - 1))
    assert np.abs(Qe - (Q0 + 0.7 * Q1)).max() < 1e-13 * np.abs(Qe).max()
    assert np.abs(Ke - K).max() < 1e-15


def test_zero_drive_is_the_static_integrator(oracle):
    N = 3
    Q0, Q1, K, _ = _system(oracle, N, 2)
    V0 = wl.rng(3).standard_normal((2, N * N - 1)) * 0.1
    a = oracle.rk4_drive(Q0, Q1, K, V0, 1e-2, 50, 0.0, 0.0, 0.0, 2.0)
    b = oracle.rk4_dense(Q0, K, V0, 1e-2, 50)
    assert np.array_equal(a, b)


def test_constant_drive(oracle):
    N = 3
    Q0, Q1, K, _ = _system(oracle, N, 4)
    V0 = wl.rng(5).standard_normal((1, N * N - 1)) * 0.1
    a = oracle.rk4_drive(Q0, Q1, K, V0, 1e-2, 40, 0.3, 0.8, 0.0, 2.0)
    b = oracle.rk4_dense(Q0 + 0.8 * Q1, K, V0, 1e-2, 40)
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()


def _affine_expm(Q, K, t):
    M = Q.shape[0]
    G = np.zeros((M + 1, M + 1))
    G[:M, :M] = Q
    G[:M, M] = K
    return expm(G * t)


@pytest.mark.parametrize("N", [2, 3])
def test_one_period_against_piecewise_exponential(oracle, N):
    Q0, Q1, K, _ = _system(oracle, N, 10 + N)
    M = N * N - 1
    E, A, T = -1.0, -1.5, 2.0
    psi = wl.random_pure_state(N, 7)
    V0 = brute.coherence_vector(np.outer(psi, psi.conj())).real[None, :]
    x = np.concatenate([V0[0], [1.0]])
    x = _affine_expm(Q0 + (E + A) * Q1, K, T / 2) @ x   # Theta = +1 on [0, T/2)
    x = _affine_expm(Q0 + (E - A) * Q1, K, T / 2) @ x
    exact = x[:M]
    # dt = 2^-10, 2^-11, 2^-12: the stage times and T/2 are exact; fourth order
    errs = []
    for steps in (2048, 4096, 8192):
        got = oracle.rk4_drive(Q0, Q1, K, V0, T / steps, steps, 0.0, E, A, T)[0]
        errs.append(np.abs(got - exact).max())
    assert errs[2] < 1e-10 * np.abs(exact).max()
    assert 10.0 < errs[0] / errs[1] < 24.0
    # the opposite phase convention is far away
    y = np.concatenate([V0[0], [1.0]])
    y = _affine_expm(Q0 + (E - A) * Q1, K, T / 2) @ y
    y = _affine_expm(Q0 + (E + A) * Q1, K, T / 2) @ y
    assert np.abs(got - y[:M]).max() > 1e-4 * np.abs(exact).max()


def _two_mode(N):
    """b1, b2 on the two-mode Fock space with n1, n2 < N, and the projector onto
    n1 + n2 = N - 1 ordered by n1 (the library's basis |n, N-1-n>)."""
    a = np.diag(np.sqrt(np.arange(1, N)), 1)  # annihilation on one mode, dimension N
    I = np.eye(N)
    b1 = np.kron(a, I)
    b2 = np.kron(I, a)
    idx = [n1 * N + (N - 1 - n1) for n1 in range(N)]
    Pm = np.zeros((N, N * N))
    Pm[np.arange(N), idx] = 1.0
    return b1, b2, Pm


@pytest.mark.parametrize("N", [2, 4, 7])
def test_rocked_dimer_inputs(N):
    b1, b2, Pm = _two_mode(N)
    n1, n2 = b1.T @ b1, b2.T @ b2
    J, U = -1.0, 2.2
    H0 = -J * (b1.T @ b2 + b2.T @ b1) + (2 * U / (N - 1)) * (n1 @ (n1 - np.eye(N * N)) + n2 @ (n2 - np.eye(N * N)))
    L = (b1.T + b2.T) @ (b1 - b2)
    h0, h1, rates, Ls = wl.rocked_dimer_model(N)
    assert np.abs(h0 - Pm @ H0 @ Pm.T).max() < 1e-12
    assert np.abs(h1 - Pm @ (n2 - n1) @ Pm.T).max() < 1e-12
    assert np.abs(Ls[0] - Pm @ L @ Pm.T).max() < 1e-12
    assert rates[0] == pytest.approx(0.1 / (N - 1))
    assert abs(np.trace(Ls[0])) < 1e-12 and np.abs(Ls[0] - Ls[0].conj().T).max() > 0.1
