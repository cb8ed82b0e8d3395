"""Saved systems on the device: bit-exact round trips of dense and CSR systems,
the same integration from a loaded system, the payload hash as documented
(recomputed here in Python), and corrupt or mismatched files rejected."""
import struct

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1912_01491_amd import workloads as wl  # noqa: E402

MASK = (1 << 64) - 1


def mix64(z):
    z = ((z ^ (z >> 30)) * 0xbf58476d1ce4e5b9) & MASK
    z = ((z ^ (z >> 27)) * 0x94d049bb133111eb) & MASK
    return z ^ (z >> 31)


def payload_hash(words):
    h = 0
    for i, w in enumerate(words):
        h = (h + mix64(int(w) ^ ((i * 0x9E3779B97F4A7C15) & MASK))) & MASK
    return h


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


def dense_system(lb, ctx, N, seed):
    H, gamma = wl.random_lindbladian(N, seed)
    return lb.lindblad_prepare(ctx, torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda())


def dcsr(A):
    return tuple(torch.from_numpy(x).cuda() for x in wl.to_csr(A))


@pytest.mark.parametrize("N", [2, 8, 20])
def test_dense_round_trip(lb, ctx, tmp_path, N):
    Q, K = dense_system(lb, ctx, N, 40 + N)
    M = N * N - 1
    p = str(tmp_path / "d.bin")
    lb.save_system(ctx, p, N, K, Q=Q)
    assert lb.load_system_info(p) == (lb.SYSTEM_DENSE, N, 0)
    Q2, K2 = lb.load_system(ctx, p)
    assert torch.equal(Q2[:, :M], Q[:, :M]) and torch.equal(K2, K)
    Q3, K3 = lb.load_system(ctx, p, ldq=M + 5)  # another leading dimension: padding zeroed
    assert torch.equal(Q3[:, :M], Q[:, :M]) and float(Q3[:, M:].abs().max()) == 0.0


def test_csr_round_trip_and_integration(lb, ctx, tmp_path):
    N = 30
    H, rates, Ls = wl.dimer_model(N)
    rp, col, val, K = lb.lindblad_prepare_sparse(ctx, N, dcsr(H), rates, [dcsr(L) for L in Ls])
    p = str(tmp_path / "s.bin")
    lb.save_system(ctx, p, N, K, csr=(rp, col, val))
    assert lb.load_system_info(p) == (lb.SYSTEM_CSR, N, col.numel())
    (rp2, col2, val2), K2 = lb.load_system(ctx, p)
    assert torch.equal(rp2, rp) and torch.equal(col2, col) and torch.equal(val2, val) and torch.equal(K2, K)
    V0 = torch.from_numpy(wl.rng(1).standard_normal((2, N * N - 1)) * 0.01).cuda()
    a, b = V0.clone(), V0.clone()
    lb.lindblad_propagate_csr(ctx, rp, col, val, K, a, 1e-3, 20)
    lb.lindblad_propagate_csr(ctx, rp2, col2, val2, K2, b, 1e-3, 20)
    assert torch.equal(a, b)


def test_file_layout_and_hash(lb, ctx, tmp_path):
    """The header fields and the payload (Q compact, then K) as documented, and
    the hash recomputed from the payload words."""
    N = 3
    Q, K = dense_system(lb, ctx, N, 7)
    M = N * N - 1
    p = tmp_path / "h.bin"
    lb.save_system(ctx, str(p), N, K, Q=Q)
    raw = p.read_bytes()
    assert raw[:8] == b"LBSYSTEM"
    version, kind, n_, m_, nnz, h = struct.unpack("<IIqqqQ", raw[8:48])
    assert (version, kind, n_, m_, nnz) == (1, 0, N, M, 0)
    body = np.frombuffer(raw[80:], dtype=np.float64)
    assert body.size == M * M + M
    assert np.array_equal(body[:M * M].reshape(M, M), Q[:, :M].cpu().numpy())
    assert np.array_equal(body[M * M:], K.cpu().numpy())
    assert payload_hash(np.frombuffer(raw[80:], dtype=np.uint64)) == h


def test_corrupt_file_is_rejected(lb, ctx, tmp_path):
    N = 6
    Q, K = dense_system(lb, ctx, N, 3)
    p = tmp_path / "c.bin"
    lb.save_system(ctx, str(p), N, K, Q=Q)
    raw = bytearray(p.read_bytes())
    raw[80 + 8 * 17 + 3] ^= 0x10  # one bit of one entry of Q
    p.write_bytes(bytes(raw))
    with pytest.raises(lb.LindbladError) as e:
        lb.load_system(ctx, str(p))
    assert e.value.code == -8
    p.write_bytes(bytes(raw[:len(raw) // 2]))  # truncated
    with pytest.raises(lb.LindbladError) as e:
        lb.load_system(ctx, str(p))
    assert e.value.code == -8


def test_mismatched_buffers_are_rejected(lb, ctx, tmp_path):
    import ctypes
    N = 4
    Q, K = dense_system(lb, ctx, N, 2)
    p = str(tmp_path / "m.bin")
    lb.save_system(ctx, p, N, K, Q=Q)
    s = lb._System()
    s.kind, s.N, s.nnz = lb.SYSTEM_CSR, N, 10
    rp = torch.zeros(N * N, dtype=torch.int64, device="cuda")
    s.rowptr, s.col, s.val, s.K = rp.data_ptr(), rp.data_ptr(), K.data_ptr(), K.data_ptr()
    assert lb.load().lindblad_load_system(ctx.handle, p.encode(), ctypes.byref(s)) == -1
    s.kind, s.N, s.ldq, s.Q = lb.SYSTEM_DENSE, N + 1, 100, Q.data_ptr()
    assert lb.load().lindblad_load_system(ctx.handle, p.encode(), ctypes.byref(s)) == -1
