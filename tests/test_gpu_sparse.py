"""GPU parity of the sparse path (jump operators, CSR Q) against the CPU oracle.

Q is compared densely row by row (explicit zeros in the CSR are allowed);
normwise tolerance 1e-10 as for the dense path.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1912_01491_amd import workloads as wl  # noqa: E402

RTOL = 1e-10


def rel(x, ref):
    den = np.abs(ref).max()
    return np.abs(np.asarray(x) - np.asarray(ref)).max() / (den if den > 0 else 1.0)


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
    rp, c, v = wl.to_csr(A)
    return (torch.from_numpy(rp).cuda(), torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda())


def gpu_sparse(lb, ctx, H, rates, Ls):
    N = H.shape[0]
    rp, col, val, K = lb.lindblad_prepare_sparse(ctx, N, dcsr(H), rates, [dcsr(L) for L in Ls])
    return rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy(), K.cpu().numpy()


def csr_rows_dense(rp, col, val, rows, M):
    out = np.zeros((len(rows), M))
    for t, r in enumerate(rows):
        e0, e1 = rp[r], rp[r + 1]
        cols = col[e0:e1]
        assert np.all(np.diff(cols) > 0), "columns must be sorted and unique within a row"
        out[t, cols] = val[e0:e1]
    return out


def random_sparse_model(N, seed):
    """A banded complex Hamiltonian and two jump operators (one with a trace part)."""
    g = wl.rng(seed)
    H = np.zeros((N, N), complex)
    for k in range(3):
        d = wl.ginibre(g, 1, N - k)[0]
        H += np.diag(d, k)
    H = wl.hermitize(H)
    L1 = np.diag(wl.ginibre(g, 1, N - 1)[0], -1)
    L2 = np.diag(wl.ginibre(g, 1, N)[0]) + 0.3 * np.diag(wl.ginibre(g, 1, N - 2)[0], 2)
    return H, np.array([0.07, 0.02]), [L1, L2]


@pytest.mark.parametrize("N", [2, 3, 5, 8, 13])
def test_dimer_full(lb, ctx, oracle, N):
    print("[gpu] sparse dimer N=%d" % N, flush=True)
    H, rates, Ls = wl.dimer_model(N)
    M = N * N - 1
    rp, col, val, K = gpu_sparse(lb, ctx, H, rates, Ls)
    Qg = csr_rows_dense(rp, col, val, range(M), M)
    Qo, Ko = oracle.prepare_factored(H, rates, Ls, np.arange(M))
    assert rel(Qg, Qo) < RTOL and rel(K, Ko) < RTOL


@pytest.mark.parametrize("N,seed", [(4, 1), (9, 2), (17, 3)])
def test_random_sparse_model_full(lb, ctx, oracle, N, seed):
    print("[gpu] sparse random model N=%d" % N, flush=True)
    H, rates, Ls = random_sparse_model(N, seed)
    M = N * N - 1
    rp, col, val, K = gpu_sparse(lb, ctx, H, rates, Ls)
    Qg = csr_rows_dense(rp, col, val, range(M), M)
    Qo, Ko = oracle.prepare_factored(H, rates, Ls, np.arange(M))
    assert rel(Qg, Qo) < RTOL and rel(K, Ko) < RTOL


def test_dimer_large_sampled_rows(lb, ctx, oracle):
    """The dimer at N = 1000 (M = 999999): sampled rows of every class, incl. the
    first/last pairs and the D rows, against the oracle."""
    N = 1000
    print("[gpu] sparse dimer N=%d" % N, flush=True)
    H, rates, Ls = wl.dimer_model(N)
    M = N * N - 1
    P = N * (N - 1) // 2
    rp, col, val, K = gpu_sparse(lb, ctx, H, rates, Ls)
    nnz = len(col)
    print("[gpu] nnz(Q) = %d (%.2f N^2)" % (nnz, nnz / N**2), flush=True)
    g = wl.rng(5)
    rows = np.unique(np.concatenate([
        [0, 1, 2, N - 2, N - 1, P - 1, P, P + 1, 2 * P - 1, 2 * P, 2 * P + 1, 2 * P + 500, M - 1],
        g.integers(0, 2 * P, 24), 2 * P + g.integers(0, N - 1, 8)]))
    Qo, Ko = oracle.prepare_factored(H, rates, Ls, rows)
    Qg = csr_rows_dense(rp, col, val, rows, M)
    assert rel(Qg, Qo) < RTOL
    assert rel(K[rows], Ko) < RTOL


@pytest.mark.parametrize("N,B,steps", [(7, 1, 200), (12, 3, 100)])
def test_csr_rk4(lb, ctx, oracle, N, B, steps):
    print("[gpu] csr rk4 N=%d" % N, flush=True)
    H, rates, Ls = wl.dimer_model(N)
    M = N * N - 1
    Qo, Ko = oracle.prepare_factored(H, rates, Ls, np.arange(M))
    psis = wl.random_pure_states(N, B, 3)
    V0 = np.array([oracle.expand(np.outer(p, p.conj())).real for p in psis])
    Vo = oracle.rk4_dense(Qo, Ko, V0, 1e-3, steps)
    rp, col, val, K = lb.lindblad_prepare_sparse(ctx, N, dcsr(H), rates, [dcsr(L) for L in Ls])
    V = torch.from_numpy(V0).cuda()
    lb.lindblad_propagate_csr(ctx, rp, col, val, K, V, 1e-3, steps)
    assert rel(V.cpu().numpy(), Vo) < RTOL


def test_sparse_rejects_dense_operators(lb, ctx):
    N = 40
    H = wl.gue_hamiltonian(N, 0)
    with pytest.raises(lb.LindbladError) as e:
        lb.lindblad_prepare_sparse(ctx, N, dcsr(H), [0.1], [dcsr(wl.ginibre(wl.rng(1), N))])
    assert e.value.code == -5


def test_csr_rk4_long_rows(lb, ctx, oracle):
    """N = 70: rows of the diagonal generators hold more than 64 entries and go
    through the one-wavefront-per-row kernel."""
    N, B, steps = 70, 2, 60
    print("[gpu] csr rk4 long rows N=%d" % N, flush=True)
    H, rates, Ls = wl.dimer_model(N)
    M = N * N - 1
    rp, col, val, K = lb.lindblad_prepare_sparse(ctx, N, dcsr(H), rates, [dcsr(L) for L in Ls])
    lens = np.diff(rp.cpu().numpy())
    assert lens.max() > 64
    Qo, Ko = oracle.prepare_factored(H, rates, Ls, np.arange(M))
    psis = wl.random_pure_states(N, B, 4)
    V0 = np.array([oracle.expand(np.outer(p, p.conj())).real for p in psis])
    Vo = oracle.rk4_dense(Qo, Ko, V0, 1e-3, steps)
    V = torch.from_numpy(V0).cuda()
    lb.lindblad_propagate_csr(ctx, rp, col, val, K, V, 1e-3, steps)
    assert rel(V.cpu().numpy(), Vo) < RTOL


@pytest.mark.parametrize("N", [5, 8, 12])
def test_dimer_csr_stores_no_zeros(lb, ctx, oracle, N):
    """Entries that are exactly zero (the S or J half of a pair for real H and
    real L) are not stored: nnz equals the number of nonzero entries of the
    oracle's Q (threshold 1e-13 of the largest), and no stored value is zero."""
    H, rates, Ls = wl.dimer_model(N)
    M = N * N - 1
    rp, col, val, K = gpu_sparse(lb, ctx, H, rates, Ls)
    Qo, _ = oracle.prepare_factored(H, rates, Ls, np.arange(M))
    assert np.all(val != 0.0)
    assert len(val) == int((np.abs(Qo) > 1e-13 * np.abs(Qo).max()).sum())
