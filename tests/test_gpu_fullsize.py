"""GPU parity at the full sizes of the benchmark configurations, in the launch
configuration bench.py times, on outputs the oracle can compute one by one or
through properties that hold at any size.

* dense N = 200 (M = 39999): the benchmark's realization-0 inputs (GUE H,
  device-drawn Wishart gamma); sampled rows of Q from every index class and all
  of K against the oracle;
* the RK4 stage GEMM at N = 200 in the benchmark's batched configuration (8
  systems x 16 states, default tile, LDS-staged kernel): a seeded stand-in Q
  from the input generators, two RK4 steps against the oracle's RK4;
* sparse N = 1000 dimer: the 1000-step CSR integration is deterministic and
  keeps rho(T) Hermitian with unit trace, and the integrator converges with
  fourth order at this size.
Normwise tolerance 1e-10 as everywhere else.
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


def test_dense_n200_sampled_rows(lb, ctx, oracle):
    N = 200
    M = N * N - 1
    P = N * (N - 1) // 2
    print("[gpu] full size: dense N=%d assembly" % N, flush=True)
    H = wl.gue_hamiltonian(N, 0)
    gamma = wl.wishart_kossakowski_device(N, 1000, device="cuda")
    Q, K = lb.lindblad_prepare(ctx, torch.from_numpy(H).cuda(), gamma)
    torch.cuda.synchronize()
    g = wl.rng(17)
    rows = np.unique(np.concatenate([[0, 1, N - 2, P - 1, P, P + 1, 2 * P - 1, 2 * P, 2 * P + 1, M - 1],
                                     g.integers(0, 2 * P, 10), 2 * P + g.integers(0, N - 1, 4)]))
    Qg = Q[torch.from_numpy(rows).cuda(), :M].cpu().numpy()
    Kg = K.cpu().numpy()
    gh = gamma.cpu().numpy()
    del gamma, Q
    torch.cuda.empty_cache()
    print("[gpu] oracle on %d sampled rows" % len(rows), flush=True)
    Qo, Ko = oracle.prepare_dense(H, gh, rows)
    assert rel(Qg, Qo) < RTOL
    assert rel(Kg, Ko) < RTOL


def test_stage_gemm_n200_batched_configuration(lb, ctx, oracle):
    N, R, B, steps = 200, 8, 16, 2
    M = N * N - 1
    ldq = lb.default_ldq(M)
    print("[gpu] full size: RK4 N=%d, %d systems x %d states" % (N, R, B), flush=True)
    Q = wl.random_dense_device(M, ldq, 5, scale=1.0)
    Kv = torch.from_numpy(wl.rng(6).standard_normal(M) * 1e-2).cuda()
    V0 = [wl.rng(7 + r).standard_normal((B, M)) * 1e-2 for r in range(R)]
    Vs = [torch.from_numpy(v).cuda() for v in V0]
    tile = lb.lindblad_tile_info(ctx, M, B)
    lb.lindblad_propagate_batched(ctx, [Q] * R, [Kv] * R, Vs, 1e-3, steps)
    torch.cuda.synchronize()
    assert Q.data_ptr() % 128 == 0 and (ldq * 8) % 128 == 0  # the staged kernel ran
    Qh = Q[:, :M].cpu().numpy()
    Kh = Kv.cpu().numpy()
    del Q
    torch.cuda.empty_cache()
    print("[gpu] oracle RK4 (tile %s)" % tile, flush=True)
    for r in (0, R - 1):
        Vo = oracle.rk4_dense(Qh, Kh, V0[r], 1e-3, steps)
        assert rel(Vs[r].cpu().numpy(), Vo) < RTOL


def test_csr_n1000_dimer_properties(lb, ctx):
    """Full-size sparse integration (1000 steps of dt = 1e-3 as benchmarked):
    deterministic, rho(T) Hermitian with unit trace; and fourth-order convergence
    of the integrator at this size: with dt = 5e-4, 2.5e-4, 1.25e-4 to the same
    T the successive differences shrink by about 2^4. (Classic RK4 does not keep
    rho positive: at N = 1000 the on-site term puts coherence frequencies near
    1000, so omega dt ~ 1 at dt = 1e-3 and rho(T) has small negative
    eigenvalues, which shrink with dt like the truncation error.)"""
    N = 1000
    print("[gpu] full size: sparse dimer N=%d, 1000 RK4 steps" % N, flush=True)
    H, rates, Ls = wl.dimer_model(N)
    Hc = tuple(torch.from_numpy(x).cuda() for x in wl.to_csr(H))
    Lc = [tuple(torch.from_numpy(x).cuda() for x in wl.to_csr(L)) for L in Ls]
    rp, col, val, K = lb.lindblad_prepare_sparse(ctx, N, Hc, rates, Lc)
    psi = torch.from_numpy(wl.random_pure_state(N, 0)[None, :]).cuda()
    V0 = lb.lb_expand_pure(ctx, psi)
    outs = []
    for _ in range(2):
        V = V0.clone()
        lb.lindblad_propagate_csr(ctx, rp, col, val, K, V, 1e-3, 1000)
        outs.append(V)
    assert torch.equal(outs[0], outs[1])
    rho = lb.lb_reconstruct(ctx, outs[0], N)[0].cpu().numpy()
    assert abs(np.trace(rho) - 1) < 1e-12
    assert np.abs(rho - rho.conj().T).max() < 1e-14
    vs, mins = [], []
    for dt, S in ((5e-4, 2000), (2.5e-4, 4000), (1.25e-4, 8000)):
        V = V0.clone()
        lb.lindblad_propagate_csr(ctx, rp, col, val, K, V, dt, S)
        vs.append(V.cpu().numpy()[0])
        mins.append(np.linalg.eigvalsh(lb.lb_reconstruct(ctx, V, N)[0].cpu().numpy()).min())
    d1 = np.abs(vs[0] - vs[1]).max()
    d2 = np.abs(vs[1] - vs[2]).max()
    print("[gpu] differences %.3e %.3e (ratio %.2f); min eig %s" % (d1, d2, d1 / d2, mins), flush=True)
    assert 8.0 < d1 / d2 < 32.0
    assert min(mins[2], 0.0) > 8.0 * min(mins[0], 0.0)
