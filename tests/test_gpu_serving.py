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


FP32_TOL = 2e-5  # served FP32 requests against the FP64 oracle, normwise relative


def make_mix(lb, n_req=30, seed=0, fp32_share=0.0):
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
            prec = lb.FP32 if g.random() < fp32_share else lb.FP64
            reqs.append(("dense", N, pool[key], V0, steps, prec))
        else:
            H, rates, Ls = wl.dimer_model(N)
            reqs.append(("sparse", N, (dcsr(H), rates, [dcsr(L) for L in Ls], H, Ls), V0, steps, lb.FP64))
    torch.cuda.synchronize()
    return ctx, reqs


def submit(srv, req, dt=1e-3):
    kind, N, sysd, V0, steps, prec = req
    if kind == "dense":
        return srv.submit_dense(sysd[0], sysd[1], V0, dt, steps, precision=prec)
    return srv.submit_sparse(N, sysd[0], sysd[1], sysd[2], V0, dt, steps)


def run_each_alone(lb, reqs):
    """Every request through a one-slot server without batching, one at a time."""
    srv = lb.Server(0, budget_bytes=1 << 30, slots=1, max_batch=1, max_N=32)
    outs = []
    for r in reqs:
        t, V = submit(srv, r)
        srv.wait(t)
        outs.append(V)
    srv.close()
    return outs


def oracle_result(oracle, req, dt=1e-3):
    kind, N, sysd, V0, steps, _ = req
    M = N * N - 1
    if kind == "dense":
        Qo, Ko = oracle.prepare_dense(sysd[2], sysd[3])
    else:
        Qo, Ko = oracle.prepare_factored(sysd[3], sysd[1], sysd[4], np.arange(M))
    return oracle.rk4_dense(Qo, Ko, V0.cpu().numpy(), dt, steps)


def test_mix_equals_alone(lb):
    """FP64 and FP32 (30 %) dense and sparse requests: each result is the same
    bit for bit in a concurrent mix (requests on the same inputs sharing one
    preparation and one pass, several systems per launch) as run alone."""
    print("[gpu] serving mix vs alone", flush=True)
    ctx, reqs = make_mix(lb, fp32_share=0.3)
    alone = run_each_alone(lb, reqs)
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


def test_same_inputs_share_one_preparation(lb, oracle):
    """Requests on the same (H, gamma) queued together are prepared once and
    integrated in one pass (up to 16 states); results equal the requests run
    alone and the oracle."""
    ctx = lb.Context(0)
    N = 9
    H, gamma = wl.random_lindbladian(N, 77)
    Hd, gd = torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda()
    reqs = []
    for i in range(10):
        V0 = lb.lb_expand_pure(ctx, torch.from_numpy(wl.random_pure_states(N, 1 + i % 3, 900 + i)).cuda())
        reqs.append(("dense", N, (Hd, gd, H, gamma), V0, 50, lb.FP64))
    torch.cuda.synchronize()
    alone = run_each_alone(lb, reqs)
    srv = lb.Server(0, budget_bytes=1 << 30, slots=1, max_batch=4, max_N=32)
    tickets = [submit(srv, r) for r in reqs]
    for t, _ in tickets:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    assert st["batched_requests"] >= 2 and st["batches"] < len(reqs)
    for (t, Vout), ref, req in zip(tickets, alone, reqs):
        assert torch.equal(Vout, ref)
        Vo = oracle_result(oracle, req)
        assert np.abs(Vout.cpu().numpy() - Vo).max() / np.abs(Vo).max() < 1e-10
    ctx.close()


def test_served_results_match_oracle(lb, oracle):
    """FP64 requests within 1e-10 of the oracle, FP32 opt-in requests within
    FP32_TOL (normwise relative)."""
    ctx, reqs = make_mix(lb, n_req=10, seed=3, fp32_share=0.4)
    srv = lb.Server(0, budget_bytes=1 << 30, slots=2, max_batch=4, max_N=32)
    tickets = [submit(srv, r) for r in reqs]
    nfp32 = 0
    for (t, Vout), req in zip(tickets, reqs):
        srv.wait(t)
        Vo = oracle_result(oracle, req)
        err = np.abs(Vout.cpu().numpy() - Vo).max() / np.abs(Vo).max()
        if req[5] == lb.FP32:
            nfp32 += 1
            assert err < FP32_TOL, (req[0], req[1], err)
        else:
            assert err < 1e-10, (req[0], req[1], err)
    assert nfp32 > 0
    srv.close()
    ctx.close()


def test_budget_respected_and_admission(lb):
    ctx, reqs = make_mix(lb, n_req=16, seed=5)
    # room for about two of the largest dense requests at a time (Q, K and a
    # 16-state block each)
    N = 18
    M = N * N - 1
    ldq = lb.default_ldq(M)
    budget = 2 * (8 * M * ldq + 8 * M + 16 * 8 * M) + 1024
    srv = lb.Server(0, budget_bytes=budget, slots=4, max_batch=2, max_N=32)
    tickets = [submit(srv, r) for r in reqs if r[0] == "dense"]  # FP64 only (fp32_share 0)
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
