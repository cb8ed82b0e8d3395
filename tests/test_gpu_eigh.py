"""The device Hermitian eigensolver (Jacobi), which gives the energy eigenbasis
for the steady-state preconditioner, against LAPACK's eigenvalues (numpy) and
against its own residual and orthogonality."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1912_01491_amd import workloads as wl  # noqa: E402


@pytest.fixture(scope="module")
def lb():
    import paper_1912_01491_amd as lb
    lb.load()
    return lb


@pytest.fixture(scope="module")
def ctx(lb):
    c = lb.Context(0)
    yield c
    c.close()


def check(lb, ctx, A, tol=1e-12):
    w, Z, sweeps = lb.lb_eigh(ctx, torch.from_numpy(A).cuda())
    w, Z = w.cpu().numpy(), Z.cpu().numpy()
    N = A.shape[0]
    scale = max(1.0, np.abs(np.linalg.eigvalsh(A)).max())
    assert np.abs(np.sort(w) - np.linalg.eigvalsh(A)).max() < tol * scale
    assert np.abs(A @ Z - Z * w[None, :]).max() < tol * scale
    assert np.abs(Z.conj().T @ Z - np.eye(N)).max() < tol
    return sweeps


@pytest.mark.parametrize("N", [1, 2, 3, 16, 65, 200])
def test_random_hermitian(lb, ctx, N):
    print("[gpu] eigh GUE N=%d" % N, flush=True)
    check(lb, ctx, wl.gue_hamiltonian(N, 3 + N))


def test_rocked_dimer_hamiltonian_doublets(lb, ctx):
    """H0 + (E + A)(n2 - n1) of the rocked dimer at N = 300: strong interaction,
    nearly degenerate pairs of levels."""
    N = 300
    print("[gpu] eigh rocked dimer N=%d" % N, flush=True)
    H0, H1, _, _ = wl.rocked_dimer_model(N)
    check(lb, ctx, H0 + (-2.5) * H1)
    check(lb, ctx, H0)


def test_degenerate_spectrum(lb, ctx):
    g = wl.rng(4)
    Qm, _ = np.linalg.qr(wl.ginibre(g, 12))
    A = Qm @ np.diag([1.0] * 5 + [2.0] * 4 + [-3.0] * 3) @ Qm.conj().T
    check(lb, ctx, (A + A.conj().T) / 2)


def test_diagonal_input_takes_no_sweep(lb, ctx):
    A = np.diag(np.arange(7, dtype=float)).astype(complex)
    assert check(lb, ctx, A) == 0


def test_bad_arguments(lb, ctx):
    A = torch.zeros((3, 3), dtype=torch.complex128, device="cuda")
    L = lb.load()
    w = torch.zeros(3, dtype=torch.float64, device="cuda")
    assert L.lb_eigh(ctx.handle, 0, lb._ptr(A), 3, lb._ptr(w), lb._ptr(A), 3, None) == -1
    assert L.lb_eigh(ctx.handle, 3, lb._ptr(A), 2, lb._ptr(w), lb._ptr(A), 3, None) == -1
