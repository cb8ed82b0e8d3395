"""Serving: results in a concurrent mix equal the same requests run alone, the
memory budget is respected, and served results match the oracle."""
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


def dcsr(A):
    rp, c, v = wl.to_csr(A)
    return (torch.from_numpy(rp).cuda(), torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda())


def make_mix(lb, n_req=30, seed=0):
    g = wl.rng(seed)
    ctx = lb.Context(0)
    pool = {}
    reqs = []
    for i in range(n_req):
        N = int(g.choice([4, 6, 9, 12, 18]))
        B = int(g.choice([1, 2]))
        steps = int(g.choice([40, 60]))
        psis = wl.random_pure_states(N, B, 100 + i)
        V0 = lb.lb_expand_pure(ctx, torch.from_numpy(psis).cuda())
        if g.random() < 0.6:
            key = (N, int(g.integers(0, 2)))
            if key not in pool:
                H, gamma = wl.random_lindbladian(N, 10 * N + key[1])
                pool[key] = (torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda(), H, gamma)
            reqs.append(("dense", N, pool[key], V0, steps))
        else:
            H, rates, Ls = wl.dimer_model(N)
            reqs.append(("sparse", N, (dcsr(H), rates, [dcsr(L) for L in Ls], H, Ls), V0, steps))
    torch.cuda.synchronize()
    return ctx, reqs


def run_alone(lb, ctx, req, dt=1e-3):
    kind, N, sysd, V0, steps = req
    V = V0.clone()
    if kind == "dense":
        Q, K = lb.lindblad_prepare(ctx, sysd[0], sysd[1])
        lb.lindblad_propagate(ctx, Q, K, V, dt, steps)
    else:
        rp, col, val, K = lb.lindblad_prepare_sparse(ctx, N, sysd[0], sysd[1], sysd[2])
        lb.lindblad_propagate_csr(ctx, rp, col, val, K, V, dt, steps)
    ctx.sync()
    return V


def submit(srv, req, dt=1e-3):
    kind, N, sysd, V0, steps = req
    if kind == "dense":
        return srv.submit_dense(sysd[0], sysd[1], V0, dt, steps)
    return srv.submit_sparse(N, sysd[0], sysd[1], sysd[2], V0, dt, steps)


def test_mix_equals_alone(lb):
    print("[gpu] serving mix vs alone", flush=True)
    ctx, reqs = make_mix(lb)
    alone = [run_alone(lb, ctx, r) for r in reqs]
    srv = lb.Server(0, budget_bytes=1 << 30, slots=3, max_batch=4, max_N=32)
    tickets = [submit(srv, r) for r in reqs]
    for t, _ in tickets:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs)
    for (t, Vout), ref in zip(tickets, alone):
        assert torch.equal(Vout, ref)
    print("[gpu] serving stats %s" % st, flush=True)
    ctx.close()


def test_served_results_match_oracle(lb, oracle):
    ctx, reqs = make_mix(lb, n_req=8, seed=3)
    srv = lb.Server(0, budget_bytes=1 << 30, slots=2, max_batch=4, max_N=32)
    tickets = [submit(srv, r) for r in reqs]
    for (t, Vout), req in zip(tickets, reqs):
        srv.wait(t)
        kind, N, sysd, V0, steps = req
        M = N * N - 1
        if kind == "dense":
            Qo, Ko = oracle.prepare_dense(sysd[2], sysd[3])
        else:
            Qo, Ko = oracle.prepare_factored(sysd[3], sysd[1], sysd[4], np.arange(M))
        Vo = oracle.rk4_dense(Qo, Ko, V0.cpu().numpy(), 1e-3, steps)
        err = np.abs(Vout.cpu().numpy() - Vo).max() / np.abs(Vo).max()
        assert err < 1e-10, (kind, N, err)
    srv.close()
    ctx.close()


def test_budget_respected_and_admission(lb):
    ctx, reqs = make_mix(lb, n_req=16, seed=5)
    # room for about two of the largest dense requests at a time
    N = 18
    M = N * N - 1
    ldq = lb.default_ldq(M)
    budget = 2 * (8 * M * ldq + 8 * M) + 1024
    srv = lb.Server(0, budget_bytes=budget, slots=4, max_batch=2, max_N=32)
    tickets = [submit(srv, r) for r in reqs if r[0] == "dense"]
    for t, _ in tickets:
        srv.wait(t)
    st = srv.stats()
    assert st["peak_bytes"] <= budget
    # a request that can never fit is refused at submission
    H, gamma = wl.random_lindbladian(30, 1)
    V0 = torch.zeros((1, 899), dtype=torch.float64, device="cuda")
    with pytest.raises(lb.LindbladError) as e:
        srv.submit_dense(torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda(), V0, 1e-3, 10)
    assert e.value.code == -6
    srv.close()
    ctx.close()


def _resident_setup(lb, seed=0):
    g = wl.rng(seed)
    ctx = lb.Context(0)
    srv = lb.Server(0, budget_bytes=1 << 30, slots=3, max_batch=16, max_N=32)
    systems = []  # (sid, kind, N, oracle inputs)
    for N in (6, 12, 18):
        H, gamma = wl.random_lindbladian(N, 300 + N)
        sid = srv.register_dense(torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda())
        systems.append((sid, "dense", N, (H, gamma)))
    for N in (9, 14):
        H, rates, Ls = wl.dimer_model(N)
        sid = srv.register_sparse(N, dcsr(H), rates, [dcsr(L) for L in Ls])
        systems.append((sid, "sparse", N, (H, rates, Ls)))
    reqs = []
    for i in range(40):
        sid, kind, N, _ = systems[int(g.integers(0, len(systems)))]
        B = int(g.choice([1, 1, 2, 3]))
        psis = wl.random_pure_states(N, B, 700 + i)
        reqs.append((sid, N, lb.lb_expand_pure(ctx, torch.from_numpy(psis).cuda())))
    torch.cuda.synchronize()
    return ctx, srv, systems, reqs


def test_resident_systems_mix_equals_alone(lb, oracle):
    """Requests on registered systems: each result is the same bit for bit
    whether it ran alone or packed with others into one pass over Q, and
    matches the oracle (normwise 1e-10)."""
    print("[gpu] resident systems: mix vs alone", flush=True)
    ctx, srv, systems, reqs = _resident_setup(lb)
    alone = []
    for sid, N, V0 in reqs:
        t, Vout = srv.submit_system(sid, V0, 1e-3, 40)
        srv.wait(t)
        alone.append(Vout)
    tickets = [srv.submit_system(sid, V0, 1e-3, 40) for sid, N, V0 in reqs]
    for t, _ in tickets:
        srv.wait(t)
    st = srv.stats()
    assert st["batched_requests"] > 0
    for (t, Vout), ref in zip(tickets, alone):
        assert torch.equal(Vout, ref)
    info = {sid: (kind, N, inp) for sid, kind, N, inp in systems}
    checked = set()
    for (sid, N, V0), (t, Vout) in zip(reqs, tickets):
        if sid in checked:
            continue
        checked.add(sid)
        kind, N, inp = info[sid]
        M = N * N - 1
        if kind == "dense":
            Qo, Ko = oracle.prepare_dense(*inp)
        else:
            Qo, Ko = oracle.prepare_factored(inp[0], inp[1], inp[2], np.arange(M))
        Vo = oracle.rk4_dense(Qo, Ko, V0.cpu().numpy(), 1e-3, 40)
        err = np.abs(Vout.cpu().numpy() - Vo).max() / np.abs(Vo).max()
        assert err < 1e-10, (kind, N, err)
    print("[gpu] resident stats %s" % st, flush=True)
    for sid, _, _, _ in systems:
        srv.release(sid)
    with pytest.raises(lb.LindbladError):
        srv.submit_system(systems[0][0], reqs[0][2], 1e-3, 5)
    srv.close()
    ctx.close()


def test_resident_release_while_queued_and_admission(lb):
    ctx = lb.Context(0)
    N = 18
    M = N * N - 1
    H, gamma = wl.random_lindbladian(N, 5)
    one = 8 * M * lb.default_ldq(M) + 8 * M
    stage = 2 * 16 * M * 8  # state staging of one pass
    srv = lb.Server(0, budget_bytes=one + 2 * stage, slots=1, max_batch=16, max_N=32)
    sid = srv.register_dense(torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda())
    # a second system of the same size cannot fit next to the first
    with pytest.raises(lb.LindbladError) as e:
        srv.register_dense(torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda())
    assert e.value.code == -6
    V0 = torch.zeros((1, M), dtype=torch.float64, device="cuda")
    tickets = [srv.submit_system(sid, V0, 1e-3, 20) for _ in range(6)]
    srv.release(sid)  # freed once the queued requests have run
    for t, _ in tickets:
        srv.wait(t)
    sid2 = srv.register_dense(torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda())
    t, V = srv.submit_system(sid2, V0, 1e-3, 20)
    srv.wait(t)
    assert torch.equal(V, tickets[0][1])
    srv.close()
    ctx.close()
