"""Pins of the oracle's Q and K against exact rows (tests/exact_rows.py): the
adjoint generator applied to F_s and expanded in the basis, in rational
arithmetic on the same FP64 inputs. Unlike the brute-force projection, this
reaches the sizes of the sparse model (Sec. 3) and takes jump operators with
trace parts as given, so it also checks the oracle's move of those parts into H.

The oracle sums Eq. (15)'s terms, which cancel heavily for the rocked dimer's
jump operator; its error against the exact rows grows with N (about 2e-13 of
the row's largest entry at N = 100, 3e-12 at N = 1000). The bounds here leave
room for that and none for a wrong term."""
import numpy as np
import pytest

from exact_rows import exact_row, row_error
from paper_1912_01491_amd import workloads as wl


def sampled_rows(N, extra, seed):
    M = N * N - 1
    P = N * (N - 1) // 2
    rows = {0, 1, N - 2, P - 1, P, P + 1, 2 * P - 1, 2 * P, 2 * P + N // 2, M - 1}
    rows |= set(int(r) for r in wl.rng(seed).integers(0, M, extra))
    return np.array(sorted(rows))


def check(oracle, N, H, rates, Ls, rows, tol):
    Q, K = oracle.prepare_factored(H, rates, Ls, rows)
    for t, s in enumerate(rows):
        ex, Kx = exact_row(N, H, rates, Ls, int(s))
        assert row_error(Q[t], ex) < tol, (N, s)
        assert abs(K[t] - float(Kx)) <= tol * max(1.0, abs(float(Kx))), (N, s)


@pytest.mark.parametrize("N", [3, 12, 40, 100])
def test_rocked_dimer_rows(oracle, N):
    H0, H1, rates, Ls = wl.rocked_dimer_model(N)
    rows = sampled_rows(N, 6, N)
    check(oracle, N, H0, rates, Ls, rows, 1e-11)
    # the drive term: Q of H1 = n2 - n1 without dissipation
    check(oracle, N, H1, [0.0], [np.zeros((N, N))], rows, 1e-13)


@pytest.mark.parametrize("N", [5, 60])
def test_static_dimer_rows(oracle, N):
    H, rates, Ls = wl.dimer_model(N)
    check(oracle, N, H, rates, Ls, sampled_rows(N, 6, 100 + N), 1e-12)


@pytest.mark.parametrize("N", [4, 9])
def test_dense_complex_inputs_with_traced_jumps_rows(oracle, N):
    """Complex H and two complex jump operators with nonzero traces: the exact
    side uses them as given, the oracle after moving the trace parts into H."""
    g = wl.rng(7 + N)
    H = wl.hermitize(wl.ginibre(g, N))
    Ls = [wl.ginibre(g, N) + (0.7 - 0.4j) * np.eye(N), wl.ginibre(g, N) + 1.3j * np.eye(N)]
    assert min(abs(np.trace(L)) for L in Ls) > 1.0
    M = N * N - 1
    check(oracle, N, H, [0.3, 0.05], Ls, np.arange(M), 1e-12)


def test_exact_rows_match_brute_projection():
    """The exact construction itself against the dense projection of the
    matrix-form Lindbladian (tests/brute.py) at N = 3."""
    import brute
    N = 3
    g = wl.rng(3)
    H = wl.hermitize(wl.ginibre(g, N))
    L = wl.ginibre(g, N)
    Q, K = brute.project(H, jumps=[(0.4, L)])
    assert np.abs(Q.imag).max() < 1e-13 and np.abs(K.imag).max() < 1e-13
    for s in range(N * N - 1):
        ex, Kx = exact_row(N, H, [0.4], [L], s)
        assert row_error(Q[s].real, ex) < 1e-13
        assert abs(K[s].real - float(Kx)) < 1e-13
