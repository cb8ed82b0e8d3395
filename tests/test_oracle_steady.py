"""Pins of the oracle's steady state v_inf (Qv = -K, the asymptotic state
rho_inf with L(rho_inf) = 0 of Sec. 3) against what the physics fixes:
closed forms (a detailed-balance chain, the driven two-level atom, depolarising
noise), the null vector of the matrix-form Lindbladian built independently of
the generator basis, and the long-time limit of the integrator."""
import numpy as np
import pytest

import brute
from paper_1912_01491_amd import workloads as wl


def rho_of(oracle, N, v):
    return oracle.reconstruct(N, v)  # 1/N + sum_n v_n F_n


@pytest.mark.parametrize("N", [2, 5, 9])
def test_detailed_balance_chain(oracle, N):
    """Diagonal H; jumps |n><n+1| at rate a_n and |n+1><n| at rate b_n. The
    unique steady state is diagonal with p_{n+1} / p_n = b_n / a_n."""
    g = wl.rng(40 + N)
    h = g.standard_normal(N)
    a = 0.2 + g.random(N - 1)
    b = 0.2 + g.random(N - 1)
    Ls, rates = [], []
    for n in range(N - 1):
        down = np.zeros((N, N), complex)
        down[n, n + 1] = 1.0
        Ls += [down, down.T.copy()]
        rates += [a[n], b[n]]
    M = N * N - 1
    Q, K = oracle.prepare_factored(np.diag(h).astype(complex), rates, Ls, np.arange(M))
    v = oracle.steady_state(Q, K)
    p = np.concatenate([[1.0], np.cumprod(b / a)])
    p /= p.sum()
    assert np.abs(rho_of(oracle, N, v) - np.diag(p)).max() < 1e-13


@pytest.mark.parametrize("Om,De,ga", [(1.0, 0.0, 1.0), (0.7, 0.4, 0.3), (3.0, -1.2, 0.5)])
def test_driven_two_level_atom(oracle, Om, De, ga):
    """H = De |1><1| + (Om/2) sigma_x, L = |0><1| at rate ga: the excited
    population is (Om^2/4) / (De^2 + ga^2/4 + Om^2/2) (resonance fluorescence)."""
    H = np.array([[0.0, Om / 2], [Om / 2, De]], complex)
    L = np.array([[0.0, 1.0], [0.0, 0.0]], complex)
    Q, K = oracle.prepare_factored(H, [ga], [L], np.arange(3))
    rho = rho_of(oracle, 2, oracle.steady_state(Q, K))
    want = (Om**2 / 4) / (De**2 + ga**2 / 4 + Om**2 / 2)
    assert abs(rho[1, 1].real - want) < 1e-14
    assert abs(np.trace(rho) - 1) < 1e-15 and np.abs(rho - rho.conj().T).max() < 1e-15


@pytest.mark.parametrize("N", [3, 6])
def test_depolarising_fixes_the_maximally_mixed_state(oracle, N):
    """gamma = c 1 is unital, so rho_inf = 1/N whatever H is: v_inf = 0."""
    M = N * N - 1
    H = wl.gue_hamiltonian(N, N)
    Q, K = oracle.prepare_dense(H, 0.4 * np.eye(M, dtype=complex))
    v = oracle.steady_state(Q, K)
    assert np.abs(K).max() < 1e-15
    assert np.abs(v).max() < 1e-15


@pytest.mark.parametrize("N", [3, 4])
def test_null_vector_of_the_matrix_form_lindbladian(oracle, N):
    """The N^2 x N^2 superoperator of the matrix-form Lindbladian (tests/brute.py,
    standard matrix units E_ab, no generator basis) has rho_inf as its null vector."""
    H, gamma = wl.random_lindbladian(N, 10 + N)
    F = brute.basis(N)
    S = np.zeros((N * N, N * N), complex)
    for a in range(N):
        for b in range(N):
            E = np.zeros((N, N), complex)
            E[a, b] = 1.0
            S[:, a * N + b] = brute.lindblad_apply(E, H, gamma, F).reshape(-1)
    _, sv, Vh = np.linalg.svd(S)
    assert sv[-1] < 1e-12 * sv[0] and sv[-2] > 1e-3 * sv[0]  # one-dimensional null space
    rho_null = Vh[-1].conj().reshape(N, N)
    rho_null /= np.trace(rho_null)
    Q, K = oracle.prepare_dense(H, gamma)
    rho = rho_of(oracle, N, oracle.steady_state(Q, K))
    assert np.abs(rho - rho_null).max() < 1e-12
    assert np.linalg.eigvalsh(rho).min() > 0


def test_long_time_limit_of_the_integrator(oracle):
    """Integrated long enough, any initial state relaxes onto v_inf."""
    N = 3
    H, gamma = wl.random_lindbladian(N, 21)
    Q, K = oracle.prepare_dense(H, gamma)
    v = oracle.steady_state(Q, K)
    gap = -np.max(np.linalg.eigvals(Q).real)
    T = 40.0 / gap
    steps = int(np.ceil(T / 1e-2))
    psi = wl.random_pure_state(N, 3)
    v0 = oracle.expand(np.outer(psi, psi.conj())).real[None, :]
    vT = oracle.rk4_dense(Q, K, v0, T / steps, steps)[0]
    assert np.abs(vT - v).max() < 1e-12
    assert np.abs(Q @ v + K).max() < 1e-14 * np.abs(Q).max()
