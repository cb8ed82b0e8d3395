"""Pins of the oracle's spectrum of Q (the eigenvalues histogrammed in Fig. 5) and
of its grid counts, against what the physics and the definitions fix: the
two-level Bloch equations, the depolarising channel (its spectrum is the
Hamiltonian's Bohr frequencies shifted by -cN), the spectrum of the
matrix-form Lindbladian built without the generator basis (tests/brute.py),
and the invariants of a real generator of a contraction semigroup."""
import numpy as np
import pytest

import brute
import spectra
from paper_1912_01491_amd import workloads as wl


def close_as_sets(a, b, tol):
    _, _, d = spectra.pair_up(a, b)
    return d.max() <= tol


@pytest.mark.parametrize("w,ga,ka", [(1.0, 0.3, 0.0), (2.5, 0.7, 0.2), (-0.8, 1.1, 0.05)])
def test_two_level_bloch_equations(oracle, w, ga, ka):
    """H = (w/2) sigma_z, decay |0><1| at rate ga, dephasing sigma_z at rate ka: the
    Bloch equations relax the population at -ga and the coherences at
    -(ga/2 + 2 ka) +- i w."""
    H = np.diag([w / 2, -w / 2]).astype(complex)
    down = np.array([[0, 1], [0, 0]], complex)
    sz = np.diag([1.0, -1.0]).astype(complex)
    rates, Ls = [ga], [down]
    if ka:
        rates.append(ka)
        Ls.append(sz)
    Q, _ = oracle.prepare_factored(H, rates, Ls, np.arange(3))
    want = [-ga, complex(-(ga / 2 + 2 * ka), w), complex(-(ga / 2 + 2 * ka), -w)]
    assert close_as_sets(oracle.spectrum(Q), want, 1e-14)


@pytest.mark.parametrize("N,c", [(3, 0.4), (5, 0.15), (7, 1.0)])
def test_depolarising_channel(oracle, N, c):
    """gamma = c 1 gives D(rho) = c (1 - N rho) on unit-trace rho (completeness of
    the orthonormal generators), so Q = Q_H - cN 1 and the spectrum is
    {-cN - i(E_a - E_b) : a != b} with -cN once more for each of the N - 1
    traceless diagonal directions."""
    M = N * N - 1
    H = wl.gue_hamiltonian(N, 70 + N)
    E = np.linalg.eigvalsh(H)
    Q, _ = oracle.prepare_dense(H, c * np.eye(M, dtype=complex))
    want = [complex(-c * N, -(E[a] - E[b])) for a in range(N) for b in range(N) if a != b]
    want += [complex(-c * N, 0.0)] * (N - 1)
    assert close_as_sets(oracle.spectrum(Q), want, 1e-12 * (1 + np.abs(E).max()))


@pytest.mark.parametrize("N", [3, 4])
def test_spectrum_of_the_matrix_form_lindbladian(oracle, N):
    """The N^2 x N^2 superoperator of the matrix-form Lindbladian (standard matrix
    units, no generator basis) has the spectrum of Q together with one zero."""
    H, gamma = wl.random_lindbladian(N, 20 + N)
    F = brute.basis(N)
    S = np.zeros((N * N, N * N), complex)
    for a in range(N):
        for b in range(N):
            E = np.zeros((N, N), complex)
            E[a, b] = 1.0
            S[:, a * N + b] = brute.lindblad_apply(E, H, gamma, F).reshape(-1)
    Q, _ = oracle.prepare_dense(H, gamma)
    lam = oracle.spectrum(Q)
    assert close_as_sets(np.linalg.eigvals(S), np.concatenate([[0.0], lam]), 1e-11 * np.linalg.norm(S))


@pytest.mark.parametrize("N", [5, 8])
def test_invariants_of_a_random_lindbladian(oracle, N):
    """Sum of the eigenvalues = trace of Q; the set is closed under conjugation (Q is
    real); every eigenvalue has a negative real part (a contraction semigroup with a
    unique steady state)."""
    H, gamma = wl.random_lindbladian(N, 30 + N)
    Q, _ = oracle.prepare_dense(H, gamma)
    lam = oracle.spectrum(Q)
    assert len(lam) == N * N - 1
    assert abs(lam.sum() - np.trace(Q)) < 1e-12 * np.abs(Q).sum()
    assert close_as_sets(lam, lam.conj(), 1e-12 * np.linalg.norm(Q))
    assert lam.real.max() < 0


def test_histogram_cell_centres_and_edges(oracle):
    """Points at cell centres with known multiplicities; the left and lower edges
    count, the right and upper edges and NaN do not."""
    re0, re1, im0, im1, nx, ny = -2.0, 2.0, -1.0, 3.0, 8, 4
    dx, dy = (re1 - re0) / nx, (im1 - im0) / ny
    want = np.zeros((ny, nx), np.int64)
    pts = []
    g = np.random.default_rng(5)
    for _ in range(60):
        ix, iy, m = g.integers(nx), g.integers(ny), g.integers(1, 4)
        pts += [complex(re0 + (ix + 0.5) * dx, im0 + (iy + 0.5) * dy)] * int(m)
        want[iy, ix] += m
    pts += [complex(re0, im0)]
    want[0, 0] += 1
    pts += [complex(re1, 0.0), complex(0.0, im1), complex(-5.0, 0.0), complex(np.nan, 0.0), complex(0.0, -1.5)]
    assert np.array_equal(oracle.histogram(pts, re0, re1, im0, im1, nx, ny), want)


def test_histogram_against_numpy_away_from_edges(oracle):
    """Random points kept off the cell edges land where numpy.histogram2d puts them."""
    g = np.random.default_rng(6)
    z = g.standard_normal(4000) + 1j * g.standard_normal(4000)
    re0, re1, im0, im1, nx, ny = -2.5, 2.0, -3.0, 3.0, 30, 20
    tx = (z.real - re0) / ((re1 - re0) / nx)
    ty = (z.imag - im0) / ((im1 - im0) / ny)
    keep = (np.abs(tx - np.round(tx)) > 1e-6) & (np.abs(ty - np.round(ty)) > 1e-6)
    z = z[keep]
    ref, _, _ = np.histogram2d(z.imag, z.real, bins=[ny, nx], range=[[im0, im1], [re0, re1]])
    assert np.array_equal(oracle.histogram(z, re0, re1, im0, im1, nx, ny), ref.astype(np.int64))
