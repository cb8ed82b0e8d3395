"""Pins of the oracle's data preparation (Eqs. (13)-(15), Table 1 steps 2.1-2.5).

The references are independent of the oracle's formulas: projection of the
matrix-form Lindbladian (tests/brute.py), the single-qubit Bloch equations,
and closed forms that follow from completeness of the basis.
"""
import numpy as np
import pytest

import brute
from paper_1912_01491_amd import workloads as wl


@pytest.mark.parametrize("N,seed", [(2, 0), (3, 1), (4, 2), (5, 3)])
def test_dense_matches_projection(oracle, N, seed):
    H, gamma = wl.random_lindbladian(N, seed)
    Q, K, maximag = oracle.prepare_dense(H, gamma, with_imag=True)
    Qb, Kb = brute.project(H, gamma)
    assert np.abs(Qb.imag).max() < 1e-13 and np.abs(Kb.imag).max() < 1e-14
    assert np.abs(Q - Qb.real).max() < 1e-13 * max(1.0, np.abs(Qb).max())
    assert np.abs(K - Kb.real).max() < 1e-14
    assert maximag < 1e-13


def test_dense_matches_projection_zero_h(oracle):
    N = 4
    H, gamma = wl.random_lindbladian(N, 9, hamiltonian="zero")
    Q, K = oracle.prepare_dense(H, gamma)
    Qb, Kb = brute.project(H, gamma)
    assert np.abs(Q - Qb.real).max() < 1e-13


def test_sampled_rows_equal_full(oracle):
    N = 6
    H, gamma = wl.random_lindbladian(N, 4)
    Q, K = oracle.prepare_dense(H, gamma)
    rows = np.array([34, 0, 17, N * N - 2, 5])
    Qr, Kr = oracle.prepare_dense(H, gamma, rows=rows)
    assert np.array_equal(Qr, Q[rows]) and np.array_equal(Kr, K)


@pytest.mark.parametrize("N", [3, 4, 6])
def test_factored_matches_matrix_form_with_trace_part(oracle, N):
    H, rates, Ls = wl.dimer_model(N)
    g = wl.rng(N)
    # a second jump operator with a nonzero trace and complex entries
    L2 = wl.ginibre(g, N) + (0.7 - 0.2j) * np.eye(N)
    rates = np.array([rates[0], 0.05])
    Ls = [Ls[0], L2]
    M = N * N - 1
    Q, K = oracle.prepare_factored(H, rates, Ls, np.arange(M))
    Qb, Kb = brute.project(H, jumps=list(zip(rates, Ls)))
    assert np.abs(Q - Qb.real).max() < 1e-13 * max(1.0, np.abs(Qb).max())
    assert np.abs(K - Kb.real).max() < 1e-13


@pytest.mark.parametrize("N", [3, 5])
def test_factored_equals_dense_gamma(oracle, N):
    """gamma = sum_p g_p l_p l_p^dagger built densely gives the same Q and K."""
    H, rates, Ls = wl.dimer_model(N)
    M = N * N - 1
    Heff, l = oracle.jump_setup(H, rates, Ls)
    gamma = sum(r * np.outer(lp, lp.conj()) for r, lp in zip(rates, l))
    Qd, Kd = oracle.prepare_dense(Heff, gamma)
    Qf, Kf = oracle.prepare_factored(H, rates, Ls, np.arange(M))
    assert np.abs(Qd - Qf).max() < 1e-13 and np.abs(Kd - Kf).max() < 1e-14


@pytest.mark.parametrize("omega,g", [(1.3, 0.4), (0.0, 1.0), (2.0, 0.0)])
def test_single_qubit_bloch_equations(oracle, omega, g):
    """N = 2: H = (omega/2) sigma_z, L = sqrt(g) |0><1| gives the Bloch equations
    dr/dt = omega z x r with T1 = 1/g, T2 = 2/g (Sec. 1); in the orthonormal basis
    v = r / sqrt2, so Q = [[-g/2, -omega, 0], [omega, -g/2, 0], [0, 0, -g]] and
    K = (0, 0, g/sqrt2)."""
    H = np.diag([omega / 2, -omega / 2]).astype(complex)
    L = np.array([[0, 1], [0, 0]], complex)
    Qw = np.array([[-g / 2, -omega, 0], [omega, -g / 2, 0], [0, 0, -g]])
    Kw = np.array([0, 0, g / np.sqrt(2)])
    Qf, Kf = oracle.prepare_factored(H, [g], [L], np.arange(3))
    assert np.abs(Qf - Qw).max() < 1e-15 and np.abs(Kf - Kw).max() < 1e-15
    # the same through a dense Kossakowski matrix gamma = g l l^dagger
    l = np.array([np.trace(brute.basis(2)[j] @ L) for j in range(3)])
    Qd, Kd = oracle.prepare_dense(H, g * np.outer(l, l.conj()))
    assert np.abs(Qd - Qw).max() < 1e-15 and np.abs(Kd - Kw).max() < 1e-15


@pytest.mark.parametrize("N", [2, 3, 5])
def test_depolarizing_closed_form(oracle, N):
    """gamma = c 1: sum_j F_j X F_j = Tr(X) 1 - X/N gives Q = -cN 1, K = 0."""
    M = N * N - 1
    c = 0.37
    Q, K = oracle.prepare_dense(np.zeros((N, N)), c * np.eye(M))
    assert np.abs(Q + c * N * np.eye(M)).max() < 1e-14 and np.abs(K).max() < 1e-15


@pytest.mark.parametrize("N,seed", [(3, 5), (4, 6), (6, 7)])
def test_invariants(oracle, N, seed):
    H, gamma = wl.random_lindbladian(N, seed)
    M = N * N - 1
    Q, K = oracle.prepare_dense(H, gamma)
    # Tr Q = -N Tr gamma for any H
    assert abs(np.trace(Q) + N * np.trace(gamma).real) < 1e-12 * N * N
    # Hamiltonian part alone is skew-symmetric and gives K = 0
    QH, KH = oracle.prepare_dense(H, np.zeros((M, M)))
    assert np.abs(QH + QH.T).max() < 1e-14 and np.abs(KH).max() == 0
    # real symmetric gamma: K = 0 and the dissipator part is symmetric
    gs = gamma.real
    QD, KD = oracle.prepare_dense(np.zeros((N, N)), gs)
    assert np.abs(KD).max() < 1e-15 and np.abs(QD - QD.T).max() < 1e-14
    # the full generator is linear in (H, gamma)
    assert np.abs(Q - QH - oracle.prepare_dense(np.zeros((N, N)), gamma)[0]).max() < 1e-14
    # spectrum of a GKSL generator: Re lambda <= 0
    assert np.linalg.eigvals(Q).real.max() < 1e-12


def test_diagonal_h_rotates_pairs(oracle):
    """Diagonal H = diag(e): the (S_jk, J_jk) planes rotate with frequency e_j - e_k."""
    N = 5
    e = np.array([0.3, -1.1, 2.0, 0.5, -0.2])
    M = N * N - 1
    Q, _ = oracle.prepare_dense(np.diag(e).astype(complex), np.zeros((M, M)))
    P = N * (N - 1) // 2
    for j in range(N):
        for k in range(j + 1, N):
            s = oracle.index_of(N, 0, j, k)
            a = oracle.index_of(N, 1, j, k)
            # -i[H, J_jk] = -(e_j - e_k) S_jk and -i[H, S_jk] = (e_j - e_k) J_jk
            assert Q[s, a] == pytest.approx(-(e[j] - e[k]), abs=1e-14)
            assert Q[a, s] == pytest.approx(e[j] - e[k], abs=1e-14)
    Q[np.arange(P), np.arange(P, 2 * P)] = 0
    Q[np.arange(P, 2 * P), np.arange(P)] = 0
    assert np.abs(Q).max() < 1e-14
