"""The FP64 matrix-core products (lb_gemm_f64, lb_gemm_c128) against numpy's
float64 / complex128 products on the host: every transposition, ragged sizes
that leave partial 64 x 64 tiles and partial k steps, the tall-skinny form
(n <= 32, k >= 2048: split k over the waves, ragged last quad), leading dimensions above
the stored rows, alpha/beta, beta = 0 over a C full of NaN (C must not be read),
empty sizes and rejected arguments. Normwise relative tolerance 1e-13."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1912_01491_amd import workloads as wl  # noqa: E402

RTOL = 1e-13


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


def colmajor(A, ld, dtype):
    """Device tensor whose memory is the column-major A (rows x cols) with leading dimension ld."""
    rows, cols = A.shape
    buf = np.zeros((cols, ld), dtype=dtype)
    buf[:, :rows] = A.T
    return torch.from_numpy(buf).cuda()


def back(T, rows):
    return T.cpu().numpy()[:, :rows].T


def test_binding_refuses_storage_smaller_than_the_matrix(lb, ctx):
    """The shape checks run before any device call: a buffer one element short
    of the column-major matrix it is said to hold is refused."""
    A = torch.zeros(4 * 3 - 1, dtype=torch.float64, device="cuda")
    B = torch.zeros(3 * 2, dtype=torch.float64, device="cuda")
    C = torch.zeros(4 * 2, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        lb.gemm_f64(ctx, 4, 2, 3, A, 4, B, 3, C, 4)
    with pytest.raises(ValueError):
        lb.gemm_f64(ctx, 4, 2, 3, torch.zeros(12, dtype=torch.float64, device="cuda"), 3, B, 3, C, 4)


def rel(x, ref):
    den = np.abs(ref).max()
    return np.abs(x - ref).max() / (den if den > 0 else 1.0)


@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (64, 64, 16), (70, 33, 17), (129, 200, 45), (300, 32, 517),
                                   (300, 32, 5000), (130, 20, 2049)])
def test_gemm_f64(lb, ctx, ta, tb, m, n, k):
    print("[gpu] gemm_f64 ta=%d tb=%d m=%d n=%d k=%d" % (ta, tb, m, n, k), flush=True)
    g = wl.rng(7 * m + 3 * n + k + 2 * ta + tb)
    A = g.standard_normal((k, m) if ta else (m, k))
    B = g.standard_normal((n, k) if tb else (k, n))
    C0 = g.standard_normal((m, n))
    alpha, beta = -0.75, 1.25
    lda, ldb, ldc = A.shape[0] + 3, B.shape[0] + 5, m + 1
    dA = colmajor(A, lda, np.float64)
    dB = colmajor(B, ldb, np.float64)
    dC = colmajor(C0, ldc, np.float64)
    lb.gemm_f64(ctx, m, n, k, dA, lda, dB, ldb, dC, ldc, alpha=alpha, beta=beta, trans_a=ta, trans_b=tb)
    ref = alpha * ((A.T if ta else A) @ (B.T if tb else B)) + beta * C0
    assert rel(back(dC, m), ref) < RTOL
    # beta = 0 must not read C
    dC.fill_(float("nan"))
    lb.gemm_f64(ctx, m, n, k, dA, lda, dB, ldb, dC, ldc, alpha=1.0, beta=0.0, trans_a=ta, trans_b=tb)
    out = back(dC, m)
    assert np.isfinite(out).all()
    assert rel(out, (A.T if ta else A) @ (B.T if tb else B)) < RTOL


@pytest.mark.parametrize("ca", [False, True])
@pytest.mark.parametrize("cb", [False, True])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (64, 64, 8), (70, 33, 9), (130, 97, 200)])
def test_gemm_c128(lb, ctx, ca, cb, m, n, k):
    print("[gpu] gemm_c128 ca=%d cb=%d m=%d n=%d k=%d" % (ca, cb, m, n, k), flush=True)
    g = wl.rng(11 * m + 5 * n + k + 2 * ca + cb)
    def cplx(shape):
        return g.standard_normal(shape) + 1j * g.standard_normal(shape)
    A = cplx((k, m) if ca else (m, k))
    B = cplx((n, k) if cb else (k, n))
    lda, ldb, ldc = A.shape[0] + 2, B.shape[0], m + 3
    dA = colmajor(A, lda, np.complex128)
    dB = colmajor(B, ldb, np.complex128)
    dC = colmajor(np.full((m, n), np.nan + 0j), ldc, np.complex128)
    lb.gemm_c128(ctx, m, n, k, dA, lda, dB, ldb, dC, ldc, conj_a=ca, conj_b=cb)
    ref = (A.conj().T if ca else A) @ (B.conj().T if cb else B)
    assert rel(back(dC, m), ref) < RTOL


@pytest.mark.parametrize("ca,cb", [(False, False), (True, False), (False, True)])
@pytest.mark.parametrize("slots", [8, 3, 1])
def test_gemm_c128_split_k(lb, ctx, ca, cb, slots):
    """A small tile grid with a long k: with scratch for `slots` partial products
    k is split into that many slices (at most 8), summed in order; the result
    agrees with numpy's product and with the unsplit call to rounding."""
    m, n, k = 100, 90, 1000
    print("[gpu] gemm_c128 split k: ca=%d cb=%d slots=%d" % (ca, cb, slots), flush=True)
    g = wl.rng(500 + 2 * ca + cb + slots)
    def cplx(shape):
        return g.standard_normal(shape) + 1j * g.standard_normal(shape)
    A = cplx((k, m) if ca else (m, k))
    B = cplx((n, k) if cb else (k, n))
    lda, ldb, ldc = A.shape[0], B.shape[0] + 1, m
    dA = colmajor(A, lda, np.complex128)
    dB = colmajor(B, ldb, np.complex128)
    dC = colmajor(np.zeros((m, n), dtype=np.complex128), ldc, np.complex128)
    work = torch.full((slots * m * n,), complex("nan"), dtype=torch.complex128, device="cuda")
    lb.gemm_c128(ctx, m, n, k, dA, lda, dB, ldb, dC, ldc, conj_a=ca, conj_b=cb, work=work)
    ref = (A.conj().T if ca else A) @ (B.conj().T if cb else B)
    split = back(dC, m)
    assert rel(split, ref) < RTOL
    lb.gemm_c128(ctx, m, n, k, dA, lda, dB, ldb, dC, ldc, conj_a=ca, conj_b=cb)
    assert rel(split, back(dC, m)) < RTOL


def test_gemm_zero_k_scales_c(lb, ctx):
    C0 = np.arange(12.0).reshape(4, 3)
    dC = colmajor(C0, 4, np.float64)
    dA = torch.zeros((1, 4), dtype=torch.float64, device="cuda")
    dB = torch.zeros((3, 1), dtype=torch.float64, device="cuda")
    lb.load().lb_gemm_f64(ctx.handle, 0, 0, 4, 3, 0, 1.0, dA.data_ptr(), 4, dB.data_ptr(), 1, 2.0, dC.data_ptr(), 4)
    ctx.sync()
    assert np.array_equal(back(dC, 4), 2.0 * C0)


def test_gemm_rejects_bad_arguments(lb, ctx):
    L = lb.load()
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    p = d.data_ptr()
    for args in [(0, 0, -1, 2, 2, 1.0, p, 1, p, 2, 0.0, p, 1),   # negative m
                 (0, 0, 4, 2, 2, 1.0, p, 3, p, 2, 0.0, p, 4),    # lda < m
                 (1, 0, 4, 2, 3, 1.0, p, 2, p, 3, 0.0, p, 4),    # A^T stored k x m: lda < k
                 (0, 0, 4, 2, 2, 1.0, p, 4, p, 2, 0.0, p, 3),    # ldc < m
                 (0, 0, 4, 2, 2, 1.0, None, 4, p, 2, 0.0, p, 4)]:  # null A
        rc = L.lb_gemm_f64(ctx.handle, *args)
        assert rc == -1, args
    rc = L.lb_gemm_c128(ctx.handle, 0, 1, 4, 2, 2, p, 4, p, 1, p, 4, None, 0)  # B^H stored n x k: ldb < n
    assert rc == -1
    rc = L.lb_gemm_c128(ctx.handle, 0, 0, 4, 2, 2, p, 4, p, 2, p, 4, None, 16)  # work elements without work
    assert rc == -1
    # empty products are accepted and touch nothing
    assert L.lb_gemm_f64(ctx.handle, 0, 0, 0, 5, 3, 1.0, p, 1, p, 3, 0.0, p, 1) == 0
