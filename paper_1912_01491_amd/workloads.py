"""Seeded synthetic inputs shaped like the paper's two test-bed models (Sec. 3).

This module only draws and assembles inputs: it holds none of the method's
arithmetic (no basis expansion, no structure constants, no Q/K contraction,
no integration). Both the GPU path and the CPU oracle receive exactly the
arrays produced here.

Models:
  * Random Lindbladian (Sec. 3, second model): a Kossakowski matrix drawn from
    the complex Wishart ensemble, gamma = N W W^dagger / Tr(W W^dagger) with W
    an M x M complex Ginibre matrix (M = N^2 - 1), given directly in the
    generator basis. A GUE Hamiltonian is added (the paper's model has H = 0;
    ``hamiltonian="zero"`` reproduces that).
  * Bosonic dimer (Sec. 3, first model, static drive): N-1 bosons on two
    sites in the Fock basis |n, N-1-n>, n = 0..N-1. Hopping -J(b1^+ b2 + h.c.),
    on-site interaction 2U/(N-1) sum_j n_j(n_j - 1), static offset eps(n2 - n1),
    and one jump operator.

Conventions: complex Gaussians have Re, Im ~ N(0, 1/2) (E|z|^2 = 1). Host
draws use numpy's PCG64 ``default_rng(seed)``. The largest Kossakowski
matrices (N = 200, 25.6 GB) are drawn on the device with torch's seeded
generator; they are exactly Hermitian (gamma_kj == conj(gamma_jk) bit for bit),
which the GPU library relies on.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def ginibre(g: np.random.Generator, n: int, m: int | None = None) -> np.ndarray:
    m = n if m is None else m
    return (g.standard_normal((n, m)) + 1j * g.standard_normal((n, m))) * np.sqrt(0.5)


def hermitize(A: np.ndarray) -> np.ndarray:
    """(A + A^dagger)/2, exactly Hermitian elementwise."""
    return (A + A.conj().T) * 0.5


def gue_hamiltonian(N: int, seed: int) -> np.ndarray:
    """H = (G + G^dagger)/sqrt(2N): E|H_ij|^2 = 1/N, spectrum on [-2, 2]."""
    G = ginibre(rng(seed), N)
    return hermitize(G) * np.sqrt(2.0 / N)


def plain_hamiltonian(N: int, seed: int) -> np.ndarray:
    """H = (G + G^dagger)/2 with G an N x N complex Gaussian matrix."""
    return hermitize(ginibre(rng(seed), N))


def wishart_kossakowski(N: int, seed: int) -> np.ndarray:
    """gamma = N W W^dagger / Tr(W W^dagger), W an M x M complex Ginibre matrix."""
    M = N * N - 1
    W = ginibre(rng(seed), M)
    A = hermitize(W @ W.conj().T)
    return A * (N / np.trace(A).real)


def random_lindbladian(N: int, seed: int, hamiltonian: str = "gue"):
    """(H, gamma) for the dense random model. Seeds: H from seed, gamma from seed + 1."""
    if hamiltonian == "gue":
        H = gue_hamiltonian(N, seed)
    elif hamiltonian == "plain":
        H = plain_hamiltonian(N, seed)
    elif hamiltonian == "zero":
        H = np.zeros((N, N), np.complex128)
    else:
        raise ValueError(hamiltonian)
    return H, wishart_kossakowski(N, seed + 1)


def random_pure_state(N: int, seed: int) -> np.ndarray:
    g = rng(seed)
    psi = (g.standard_normal(N) + 1j * g.standard_normal(N)) * np.sqrt(0.5)
    return psi / np.linalg.norm(psi)


def random_pure_states(N: int, B: int, seed: int) -> np.ndarray:
    """(B, N) complex128, each row a normalised complex Gaussian vector."""
    g = rng(seed)
    psi = (g.standard_normal((B, N)) + 1j * g.standard_normal((B, N))) * np.sqrt(0.5)
    return psi / np.linalg.norm(psi, axis=1, keepdims=True)


# ---------------------------------------------------------------------------
# Bosonic dimer (Sec. 3, first model)
# ---------------------------------------------------------------------------

def dimer_hamiltonian(N: int, J: float = 1.0, U: float = 0.5, eps: float = 0.0) -> np.ndarray:
    """N-1 bosons on two sites; basis |n1 = n, n2 = N-1-n>. Tridiagonal, real."""
    nb = N - 1
    n1 = np.arange(N, dtype=np.float64)
    n2 = nb - n1
    H = np.zeros((N, N), np.complex128)
    diag = (2.0 * U / max(nb, 1)) * (n1 * (n1 - 1) + n2 * (n2 - 1)) + eps * (n2 - n1)
    H[np.arange(N), np.arange(N)] = diag
    # b1^+ b2 |n1, n2> = sqrt((n1+1) n2) |n1+1, n2-1>
    amp = np.sqrt((n1[:-1] + 1) * n2[:-1])
    H[np.arange(1, N), np.arange(N - 1)] += -J * amp
    H[np.arange(N - 1), np.arange(1, N)] += -J * amp
    return H


def dimer_jump_a1dag_a2(N: int) -> np.ndarray:
    """L = b1^+ b2: L_{n+1, n} = sqrt((n+1)(N-1-n)). Traceless, non-Hermitian."""
    nb = N - 1
    n = np.arange(N - 1, dtype=np.float64)
    L = np.zeros((N, N), np.complex128)
    L[np.arange(1, N), np.arange(N - 1)] = np.sqrt((n + 1) * (nb - n))
    return L


def dimer_model(N: int, J: float = 1.0, U: float = 0.5, eps: float = 0.0, gamma: float = 0.1):
    """(H, rates, [L]) for the static dimer with one jump operator b1^+ b2 at rate gamma/(N-1)."""
    H = dimer_hamiltonian(N, J, U, eps)
    L = dimer_jump_a1dag_a2(N)
    return H, np.array([gamma / max(N - 1, 1)]), [L]


def dimer_jump_sync(N: int) -> np.ndarray:
    """L = (b1^+ + b2^+)(b1 - b2) = n1 - n2 + b2^+ b1 - b1^+ b2 on |n, N-1-n>:
    traceless and not Hermitian (the synchronising jump of the rocked dimer)."""
    nb = N - 1
    n = np.arange(N, dtype=np.float64)
    L = np.zeros((N, N), np.complex128)
    L[np.arange(N), np.arange(N)] = n - (nb - n)
    # b1^+ b2 |n, nb-n> = sqrt((n+1)(nb-n)) |n+1, nb-n-1>
    up = np.sqrt((n[:-1] + 1) * (nb - n[:-1]))
    L[np.arange(1, N), np.arange(N - 1)] -= up
    # b2^+ b1 |n, nb-n> = sqrt(n (nb-n+1)) |n-1, nb-n+1>
    L[np.arange(N - 1), np.arange(1, N)] += up
    return L


def rocked_dimer_model(N: int, J: float = -1.0, U: float = 2.2, gamma: float = 0.1):
    """The periodically rocked dimer of the sparse test model with its published
    parameters: (H0, H1, rates, [L]) with H(t) = H0 + eps(t) H1, H0 the hopping
    and interaction part, H1 = n2 - n1, one jump L = (b1^+ + b2^+)(b1 - b2) at
    rate gamma/(N-1). The drive eps(t) (E = -1, A = -1.5, T = 2 pi) is applied
    by the integrator."""
    H0 = dimer_hamiltonian(N, J, U, 0.0)
    n1 = np.arange(N, dtype=np.float64)
    H1 = np.diag((N - 1 - n1) - n1).astype(np.complex128)
    return H0, H1, np.array([gamma / max(N - 1, 1)]), [dimer_jump_sync(N)]


def to_csr(A: np.ndarray):
    """Dense N x N complex -> (rowptr int64, col int64, val complex128), zeros dropped."""
    A = np.asarray(A)
    nz = A != 0
    rowptr = np.zeros(A.shape[0] + 1, np.int64)
    rowptr[1:] = np.cumsum(nz.sum(axis=1))
    r, c = np.nonzero(nz)
    return rowptr, c.astype(np.int64), A[r, c].astype(np.complex128)


# ---------------------------------------------------------------------------
# Device-side draw for the largest Kossakowski matrices
# ---------------------------------------------------------------------------

def wishart_kossakowski_device(N: int, seed: int, device="cuda", block: int = 4096):
    """gamma = N W W^dagger / Tr(W W^dagger) drawn on the GPU (torch), complex128.

    W is drawn in complex128 and W W^dagger is formed in complex128 by torch's
    GEMM: input synthesis only, never the library under test, so the oracle's
    inputs do not come from the path it checks. FP64 keeps gamma positive
    semidefinite to FP64 rounding: a square complex Ginibre W has eigenvalues of
    W W^dagger down to about 1/M of its mean, which FP32 rounding would push
    below zero at N = 200. The product is made exactly Hermitian in place, block
    by block (X = (A_ij + A_ji^dagger)/2 stored at (i, j) and X^dagger at (j, i)),
    and scaled by a real factor, which keeps gamma_kj == conj(gamma_jk) bit for
    bit. Deterministic for a given seed and device.
    """
    import torch

    M = N * N - 1
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    W = torch.randn(M, M, dtype=torch.complex128, device=device, generator=gen)
    Wh = W.mH.contiguous()  # materialized conjugate transpose as the right operand
    A = W @ Wh
    del W, Wh
    for i0 in range(0, M, block):
        i1 = min(M, i0 + block)
        for j0 in range(i0, M, block):
            j1 = min(M, j0 + block)
            X = (A[i0:i1, j0:j1] + A[j0:j1, i0:i1].mH) * 0.5
            A[i0:i1, j0:j1] = X
            if j0 != i0:
                A[j0:j1, i0:i1] = X.mH
            del X
    tr = A.diagonal().real.sum()
    A *= (N / tr)
    return A


def random_dense_device(M: int, ldq: int, seed: int, scale: float = 1.0, device="cuda"):
    """A dense M x ldq FP64 matrix with N(0, scale^2 / M) entries in columns < M
    and zeros in the padding columns, drawn on the GPU (torch) for a given seed:
    a stand-in operand for integrator tests at full size (the integrator does not
    depend on Q being a Lindbladian)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    Q = torch.zeros(M, ldq, dtype=torch.float64, device=device)
    Q[:, :M] = torch.randn(M, M, dtype=torch.float64, device=device, generator=gen) * (scale / M ** 0.5)
    return Q
