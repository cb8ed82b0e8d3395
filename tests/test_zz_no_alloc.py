"""The allocation-free propagate (lindblad_propagate_noalloc) against
lindblad_propagate through the C ABI: the same kernels and tile on the static
per-GPU array, so the results agree bit for bit; two calls in a row, the
second on a smaller input, on each integration path (matrix-core block, one
state, one workgroup), FP64 and FP32; sizes beyond the array are refused; a
fresh context's call allocates no device memory."""
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


def _system(lb, ctx, N, seed):
    H, gamma = wl.random_lindbladian(N, seed)
    Q, K = lb.lindblad_prepare(ctx, torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda())
    return Q, K


def _states(lb, ctx, N, B, seed):
    return lb.lb_expand_pure(ctx, torch.from_numpy(wl.random_pure_states(N, B, seed)).cuda())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("sizes", [((40, 16), (20, 16)), ((40, 1), (21, 1)), ((30, 16), (9, 3))])
def test_noalloc_equals_propagate_twice(lb, sizes, precision):
    """(N, B) pairs: matrix-core path then a smaller one; one-state GEMV path
    twice; matrix-core path then the one-workgroup path (M = 80)."""
    ctx = lb.Context(0)
    prec = lb.FP32 if precision == "fp32" else lb.FP64
    for i, (N, B) in enumerate(sizes):
        if prec == lb.FP32 and B == 1:
            pytest.skip("the one-state path is FP64 only")
        print("[gpu] noalloc %s call %d: N=%d B=%d" % (precision, i, N, B), flush=True)
        Q, K = _system(lb, ctx, N, 40 + N)
        Q32 = lb.lindblad_q_to_f32(ctx, Q) if prec == lb.FP32 else None
        V0 = _states(lb, ctx, N, B, 90 + N)
        a = V0.clone()
        lb.lindblad_propagate(ctx, Q if prec == lb.FP64 else None, K, a, 1e-3, 37, precision=prec, Q32=Q32)
        b = V0.clone()
        lb.lindblad_propagate_noalloc(ctx, Q if prec == lb.FP64 else None, K, b, 1e-3, 37, precision=prec, Q32=Q32)
        ctx.sync()
        assert torch.isfinite(a).all()
        assert torch.equal(a, b), (N, B, float((a - b).abs().max()))
    ctx.close()


def test_noalloc_refuses_sizes_beyond_its_array(lb):
    ctx = lb.Context(0)
    N, B = 100, 16  # split-K partials of 16 states at M = 9999 exceed 16 MiB
    M = N * N - 1
    ldq = lb.default_ldq(M)
    Q = torch.zeros((M, ldq), dtype=torch.float64, device="cuda")
    K = torch.zeros(M, dtype=torch.float64, device="cuda")
    V = torch.ones((B, M), dtype=torch.float64, device="cuda")
    before = V.clone()
    with pytest.raises(lb.LindbladError) as e:
        lb.lindblad_propagate_noalloc(ctx, Q, K, V, 1e-3, 2)
    assert e.value.code == -5
    ctx.sync()
    assert torch.equal(V, before)
    ctx.close()


def test_noalloc_allocates_nothing(lb):
    """A fresh context (empty workspace) runs the allocation-free propagate
    without changing the device's free memory, and agrees with
    lindblad_propagate run afterwards on the same context."""
    warm = lb.Context(0)
    N, B = 24, 16
    Q, K = _system(lb, warm, N, 7)
    V = _states(lb, warm, N, B, 8)
    lb.lindblad_propagate_noalloc(warm, Q, K, V.clone(), 1e-3, 3)  # loads every kernel once
    warm.sync()
    torch.cuda.synchronize()
    ctx = lb.Context(0)
    W = V.clone()
    X = V.clone()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    lb.lindblad_propagate_noalloc(ctx, Q, K, W, 1e-3, 5)
    ctx.sync()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0
    lb.lindblad_propagate(ctx, Q, K, X, 1e-3, 5)
    ctx.sync()
    print("[gpu] free device memory: %d before, %d after the allocation-free call, %d after the workspace one"
          % (free0, free1, torch.cuda.mem_get_info()[0]), flush=True)
    assert torch.equal(W, X)
    ctx.close()
    warm.close()
    assert np.isfinite(W.cpu().numpy()).all()
