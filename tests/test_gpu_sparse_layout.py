"""Edge cases of the sliced sparse layout behind lindblad_propagate_csr[_drive]
and the sparse steady-state operator: rows are regrouped into slices of 64
(one row per lane) and rows of more than 32 entries are taken by whole blocks.
Synthetic CSR matrices whose shapes sit on those boundaries (ragged last
slices, rows of exactly 32 and 33 entries, empty rows, all-long matrices,
states in groups of four with a ragged rest, a drive matrix whose long rows
differ from Q0's) are integrated on the GPU and by the oracle's CSR / dense
RK4 (classic RK4, Table 1 step 3.1), normwise tolerance 1e-12."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1912_01491_amd import workloads as wl  # noqa: E402

RTOL = 1e-12


def rel(x, ref):
    return float(np.abs(np.asarray(x) - ref).max() / np.abs(ref).max())


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


def rand_csr(M, lens, seed):
    """Row r holds lens[r] distinct sorted columns with N(0, 1)/sqrt(len) values."""
    g = wl.rng(seed)
    rowptr = np.zeros(M + 1, np.int64)
    rowptr[1:] = np.cumsum(lens)
    cols, vals = [], []
    for r in range(M):
        c = np.sort(g.choice(M, size=int(lens[r]), replace=False))
        cols.append(c)
        vals.append(g.standard_normal(len(c)) / math.sqrt(max(len(c), 1)))
    col = np.concatenate(cols).astype(np.int64) if M else np.zeros(0, np.int64)
    val = np.concatenate(vals) if M else np.zeros(0)
    return rowptr, col, val


def dense(M, csr):
    rp, c, v = csr
    D = np.zeros((M, M))
    for r in range(M):
        D[r, c[rp[r]:rp[r + 1]]] = v[rp[r]:rp[r + 1]]
    return D


def dev(*xs):
    return tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs)


def lens_for(name, M, seed):
    return np.minimum(_lens(name, M, seed), M)


def _lens(name, M, seed):
    g = wl.rng(seed)
    if name == "random":
        return g.integers(0, 13, M)
    if name == "threshold":  # rows of exactly 32 and 33 entries next to short and empty ones
        L = g.integers(0, 9, M)
        L[::5] = 32
        L[1::5] = 33
        L[2::7] = 0
        L[3::11] = min(60, M)
        return L
    if name == "all_long":
        return np.full(M, M)
    raise ValueError(name)


CASES = [(3, "random"), (63, "random"), (64, "random"), (65, "random"), (130, "threshold"), (40, "all_long"),
         (200, "threshold")]


@pytest.mark.parametrize("M,kind", CASES)
@pytest.mark.parametrize("B", [1, 5])
def test_csr_propagate_layout_edges(lb, ctx, oracle, M, kind, B):
    print("[gpu] sliced layout M=%d %s B=%d" % (M, kind, B), flush=True)
    lens = lens_for(kind, M, M)
    csr = rand_csr(M, lens, 7 + M)
    K = wl.rng(1).standard_normal(M) * 0.1
    V0 = wl.rng(2).standard_normal((B, M))
    dt, steps = 1e-2, 7
    Vo = oracle.rk4_csr(*csr, K, V0, dt, steps)
    rp, c, v, Kd, V = dev(*csr, K, V0)
    lb.lindblad_propagate_csr(ctx, rp, c, v, Kd, V, dt, steps)
    assert rel(V.cpu().numpy(), Vo) < RTOL


@pytest.mark.parametrize("B", [3, 4])
def test_csr_propagate_state_groups(lb, ctx, oracle, B):
    """States go through a slice four at a time: B = 3 (one partial group) and 4 (one full)."""
    M = 130
    csr = rand_csr(M, lens_for("threshold", M, 3), 11)
    K = wl.rng(3).standard_normal(M) * 0.1
    V0 = wl.rng(4).standard_normal((B, M))
    Vo = oracle.rk4_csr(*csr, K, V0, 1e-2, 5)
    rp, c, v, Kd, V = dev(*csr, K, V0)
    lb.lindblad_propagate_csr(ctx, rp, c, v, Kd, V, 1e-2, 5)
    assert rel(V.cpu().numpy(), Vo) < RTOL


def test_drive_with_long_rows_in_either_matrix(lb, ctx, oracle):
    """Q1 has long rows where Q0's rows are short (they stay in the slices, the
    slice widens) and short rows where Q0's are long (taken by the row's block)."""
    M = 130
    L0 = lens_for("threshold", M, 5)
    L1 = np.where(L0 > 32, 2, 0)
    L1[4::9] = 45
    L1[L0 > 32] = 3
    Q0, Q1 = rand_csr(M, L0, 21), rand_csr(M, L1, 22)
    K = wl.rng(5).standard_normal(M) * 0.1
    V0 = wl.rng(6).standard_normal((2, M))
    E, A, T = -1.0, -1.5, 0.4
    dt, steps, t0 = 0.01, 60, 0.13
    Vo = oracle.rk4_drive(dense(M, Q0), dense(M, Q1), K, V0, dt, steps, t0, E, A, T)
    a, b = dev(*Q0), dev(*Q1)
    Kd, V = dev(K, V0)
    lb.lindblad_propagate_csr_drive(ctx, a, b, Kd, V, dt, steps, t0, E, A, T)
    assert rel(V.cpu().numpy(), Vo) < RTOL


@pytest.mark.parametrize("M,kind", [(65, "threshold"), (40, "all_long")])
def test_steady_state_operator_layout_edges(lb, ctx, oracle, M, kind):
    """The sliced operator inside GMRES: a stable synthetic Q (shifted so that
    its spectrum lies in the left half plane) against the oracle's dense solve."""
    csr = rand_csr(M, lens_for(kind, M, 9), 31)
    D = dense(M, csr)
    shift = np.abs(np.linalg.eigvals(D)).max() + 1.0
    rp, c, v = csr
    v = v.copy()
    for r in range(M):  # Q = D - shift 1 (the diagonal entry stored or added)
        row = slice(rp[r], rp[r + 1])
        hit = np.nonzero(c[row] == r)[0]
        if len(hit):
            v[rp[r] + hit[0]] -= shift
    extra = [r for r in range(M) if not np.any(c[rp[r]:rp[r + 1]] == r)]
    if extra:  # rebuild with the missing diagonal entries
        Dq = dense(M, (rp, c, v))
        Dq[extra, extra] -= shift
        rp, c, v = wl.to_csr(Dq)
        v = v.real.copy()
    Qd = dense(M, (rp, c, v))
    K = wl.rng(8).standard_normal(M)
    vo = oracle.steady_state(Qd, K)
    rpd, cd, vd, Kd = dev(rp, c, v, K)
    x, info = lb.lindblad_steady_state_csr(ctx, rpd, cd, vd, Kd, tol=1e-13)
    assert info["converged"] == 1
    assert rel(x.cpu().numpy(), vo) < 1e-10
