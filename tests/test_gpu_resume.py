"""Resuming an integration: a run split in two (the state carried over, the
drive's step offset given) is bit-identical to the uninterrupted run, on the
dense one-state and block paths, the sparse path and the driven sparse path
(every step is deterministic; stage times are formed from t0 and the global
step index)."""
import math

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


def dcsr(A):
    return tuple(torch.from_numpy(x).cuda() for x in wl.to_csr(A))


@pytest.mark.parametrize("B", [1, 16])
def test_dense_resume(lb, ctx, B):
    N = 12
    H, gamma = wl.random_lindbladian(N, 4)
    Q, K = lb.lindblad_prepare(ctx, torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda())
    V0 = torch.from_numpy(wl.rng(5).standard_normal((B, N * N - 1)) * 0.05).cuda()
    a, b = V0.clone(), V0.clone()
    lb.lindblad_propagate(ctx, Q, K, a, 1e-3, 100)
    lb.lindblad_propagate(ctx, Q, K, b, 1e-3, 37)
    lb.lindblad_propagate(ctx, Q, K, b, 1e-3, 63)
    assert torch.equal(a, b)


def test_sparse_resume(lb, ctx):
    N = 40
    H, rates, Ls = wl.dimer_model(N)
    rp, col, val, K = lb.lindblad_prepare_sparse(ctx, N, dcsr(H), rates, [dcsr(L) for L in Ls])
    V0 = torch.from_numpy(wl.rng(6).standard_normal((3, N * N - 1)) * 0.01).cuda()
    a, b = V0.clone(), V0.clone()
    lb.lindblad_propagate_csr(ctx, rp, col, val, K, a, 1e-3, 90)
    lb.lindblad_propagate_csr(ctx, rp, col, val, K, b, 1e-3, 50)
    lb.lindblad_propagate_csr(ctx, rp, col, val, K, b, 1e-3, 40)
    assert torch.equal(a, b)


def test_driven_resume_across_a_switch(lb, ctx):
    """dt = T/200, split at step 97 so that the second part starts three steps
    before the switch at T/2 (a stage time exactly on it)."""
    N = 20
    H0, H1, rates, Ls = wl.rocked_dimer_model(N)
    rp0, c0, v0, K = lb.lindblad_prepare_sparse(ctx, N, dcsr(H0), rates, [dcsr(L) for L in Ls])
    rp1, c1, v1, _ = lb.lindblad_prepare_sparse(ctx, N, dcsr(H1), [], [])
    Q0, Q1 = (rp0, c0, v0), (rp1, c1, v1)
    E, A, T = -1.0, -1.5, 2 * math.pi
    dt, t0 = T / 200, 0.0
    V0 = torch.from_numpy(wl.rng(7).standard_normal((2, N * N - 1)) * 0.01).cuda()
    a, b = V0.clone(), V0.clone()
    lb.lindblad_propagate_csr_drive(ctx, Q0, Q1, K, a, dt, 160, t0, E, A, T)
    lb.lindblad_propagate_csr_drive(ctx, Q0, Q1, K, b, dt, 97, t0, E, A, T)
    lb.lindblad_propagate_csr_drive(ctx, Q0, Q1, K, b, dt, 63, t0, E, A, T, k0=97)
    assert torch.equal(a, b)
    with pytest.raises(lb.LindbladError):
        lb.lindblad_propagate_csr_drive(ctx, Q0, Q1, K, b, dt, 1, t0, E, A, T, k0=-1)
