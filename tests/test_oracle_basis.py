"""Pins of the oracle's basis (Sec. 2, Eqs. (3)-(5)) against definitions and textbook matrices."""
import numpy as np
import pytest

import brute


@pytest.mark.parametrize("N", [2, 3, 4, 7, 12, 40])
def test_index_roundtrip(oracle, N):
    M = N * N - 1
    P = N * (N - 1) // 2
    seen = set()
    for i in range(M):
        c, j, k = oracle.class_of(N, i)
        if c < 2:
            assert 0 <= j < k < N
            assert oracle.index_of(N, c, j, k) == i
        else:
            assert 1 <= j <= N - 1 and i == 2 * P + j - 1
            assert oracle.index_of(N, 2, j) == i
        seen.add((c, j, k))
    assert len(seen) == M


@pytest.mark.parametrize("N", [2, 3, 5])
def test_basis_orthonormal_hermitian_traceless(oracle, N):
    M = N * N - 1
    F = np.array([oracle.basis_dense(N, i) for i in range(M)])
    assert np.allclose(F, np.conj(np.transpose(F, (0, 2, 1))), atol=0)
    assert np.abs(np.einsum("iaa->i", F)).max() < 1e-15
    G = np.einsum("iab,jba->ij", F, F)
    assert np.abs(G - np.eye(M)).max() < 1e-15
    # completeness: sum_i F_i (x) F_i = SWAP - 1/N (1 (x) 1) on C^N (x) C^N
    S = np.einsum("iab,icd->acbd", F, F).reshape(N * N, N * N)
    swap = np.zeros((N, N, N, N))
    for a in range(N):
        for b in range(N):
            swap[a, b, b, a] = 1.0
    assert np.abs(S - (swap.reshape(N * N, N * N) - np.eye(N * N) / N)).max() < 1e-14


def test_basis_matches_independent_construction(oracle):
    for N in (2, 3, 4, 6):
        F = brute.basis(N)
        for i in range(N * N - 1):
            assert np.abs(oracle.basis_dense(N, i) - F[i]).max() <= 4e-16


def test_su2_is_pauli(oracle):
    s = 1 / np.sqrt(2)
    sx = np.array([[0, 1], [1, 0]], complex)
    sy = np.array([[0, -1j], [1j, 0]])
    sz = np.array([[1, 0], [0, -1]], complex)
    for i, P in enumerate((sx, sy, sz)):
        assert np.allclose(oracle.basis_dense(2, i), s * P, atol=1e-16)


def test_su3_is_gellmann(oracle):
    s3 = np.sqrt(3)
    lam = {
        1: [[0, 1, 0], [1, 0, 0], [0, 0, 0]],
        2: [[0, -1j, 0], [1j, 0, 0], [0, 0, 0]],
        3: [[1, 0, 0], [0, -1, 0], [0, 0, 0]],
        4: [[0, 0, 1], [0, 0, 0], [1, 0, 0]],
        5: [[0, 0, -1j], [0, 0, 0], [1j, 0, 0]],
        6: [[0, 0, 0], [0, 0, 1], [0, 1, 0]],
        7: [[0, 0, 0], [0, 0, -1j], [0, 1j, 0]],
        8: [[1 / s3, 0, 0], [0, 1 / s3, 0], [0, 0, -2 / s3]],
    }
    pos = {1: 0, 2: 3, 3: 6, 4: 1, 5: 4, 6: 2, 7: 5, 8: 7}
    for a, L in lam.items():
        assert np.allclose(oracle.basis_dense(3, pos[a]), np.array(L, complex) / np.sqrt(2), atol=1e-15)


@pytest.mark.parametrize("N", [2, 3, 6])
def test_expand_reconstruct_roundtrip(oracle, N):
    from paper_1912_01491_amd import workloads as wl
    psi = wl.random_pure_state(N, 3)
    rho = np.outer(psi, psi.conj())
    v = oracle.expand(rho)
    assert np.abs(v.imag).max() < 1e-15
    v = v.real
    assert np.allclose(v, brute.coherence_vector(rho).real, atol=1e-15)
    # purity of a pure state: Tr rho^2 = 1/N + |v|^2 = 1
    assert abs(1.0 / N + v @ v - 1.0) < 1e-13
    assert np.abs(oracle.reconstruct(N, v) - rho).max() < 1e-14
