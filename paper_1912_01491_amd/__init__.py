"""Python binding of the gfx950 GKSL -> real-ODE library (liblindblad.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/lindblad.h``. torch provides
device memory and streams. The binding raises ``LibraryMissing`` when the
shared library has not been built; there is no fallback implementation.

Typical use::

    import torch, paper_1912_01491_amd as lb
    ctx = lb.Context()                        # torch's current stream
    Q, K = lb.lindblad_prepare(ctx, H, gamma) # H: (N,N) c128, gamma: (M,M) c128 on cuda
    V = lb.lb_expand_pure(ctx, psi)           # (B, M) coherence vectors
    lb.lindblad_propagate(ctx, Q, K, V, dt=1e-3, steps=1000)
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "LibraryMissing", "LindbladError", "Context", "library_path", "load",
    "lb_basis_index", "lb_basis_table", "lb_fd_count", "lb_fd_enumerate",
    "lb_expand", "lb_expand_pure", "lb_reconstruct",
    "lindblad_prepare", "lindblad_q_to_f32", "lindblad_propagate", "lindblad_propagate_noalloc",
    "lindblad_propagate_batched",
    "lindblad_propagate_graph", "lindblad_graph_clear", "lindblad_propagate_csr", "lindblad_prepare_sparse",
    "lindblad_propagate_csr_drive", "lb_eigh", "Secular", "read_bandwidth", "gemm_f64", "gemm_c128", "lb_hessenberg", "lindblad_spectrum",
    "lindblad_spectrum_histogram", "save_system", "load_system", "load_system_info", "lindblad_steady_state", "lindblad_steady_state_csr", "lindblad_autotune", "lindblad_tile_info", "lindblad_set_tile", "lindblad_time_stage", "Server",
    "FP64", "FP32", "CHECK_HERMITIAN",
]

FP64 = 0
FP32 = 1
CHECK_HERMITIAN = 1
MAX_N = 2048

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liblindblad.so")
_lib = None

_ERRORS = {-1: "invalid argument", -2: "not Hermitian", -3: "out of memory", -4: "device error",
           -5: "unsupported", -6: "admission", -7: "no convergence", -8: "i/o", -9: "cancelled"}


class LibraryMissing(RuntimeError):
    pass


class LindbladError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_ERRORS.get(code, "error"), code, msg))
        self.code = code


def library_path() -> str:
    return _LIB_PATH


class _CSR(ctypes.Structure):
    _fields_ = [("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("nnz", ctypes.c_int64)]


def load():
    """Loads liblindblad.so (built by ``paper_1912_01491_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise LibraryMissing("%s is not built; run `python -m paper_1912_01491_amd.build` "
                             "or __graft_entry__.build()" % _LIB_PATH)
    lib = ctypes.CDLL(_LIB_PATH)
    for name, args in signatures().items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name == "lb_last_error" else ctypes.c_int
    _lib = lib
    return lib


def signatures():
    """ctypes argument types of every C entry point."""
    V, I, I64, D, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_uint
    return {
        "lb_last_error": [],
        "lb_create": [ctypes.POINTER(ctypes.c_void_p), I, V],
        "lb_destroy": [V],
        "lb_set_stream": [V, V],
        "lb_sync": [V],
        "lb_version": [],
        "lb_set_progress": [V, V, V],
        "lb_basis_index": [I, I64, V, V, V],
        "lb_basis_table": [V, I, V],
        "lb_fd_count": [V, I, I, V],
        "lb_fd_enumerate": [V, I, I, V, V, I64, V],
        "lb_expand": [V, I, I, V, V],
        "lb_expand_pure": [V, I, I, V, V],
        "lb_reconstruct": [V, I, I, V, V],
        "lindblad_prepare": [V, I, V, V, V, I64, V, U],
        "lindblad_prepare_sparse_count": [V, I, V, I, V, V, V],
        "lindblad_prepare_sparse_fill": [V, I, V, I, V, V, I64, V, V, V, V],
        "lindblad_propagate": [V, I64, V, V, I64, V, V, I, D, I64, I],
        "lindblad_propagate_noalloc": [V, I64, V, V, I64, V, V, I, D, I64, I],
        "lindblad_q_to_f32": [V, I64, V, I64, V],
        "lindblad_propagate_csr": [V, I64, V, V, V, V, V, I, D, I64],
        "lindblad_propagate_csr_drive": [V, I64, V, V, V, V, V, V, V, V, I, D, I64, D, I64, D, D, D],
        "lb_eigh": [V, I, V, I, V, V, I, V],
        "lb_read_bandwidth": [V, ctypes.c_size_t, V],
        "lindblad_graph_clear": [V, V],
        "lb_gemm_f64": [V, I, I, I64, I64, I64, D, V, I64, V, I64, D, V, I64],
        "lb_gemm_c128": [V, I, I, I64, I64, I64, V, I64, V, I64, V, I64, V, I64],
        "lb_hessenberg": [V, I64, V, I64],
        "lindblad_spectrum": [V, I64, V, I64, V, V],
        "lindblad_spectrum_histogram": [V, I64, V, D, D, D, D, I, I, V],
        "lindblad_save_system": [V, ctypes.c_char_p, V],
        "lindblad_load_system_info": [ctypes.c_char_p, V],
        "lindblad_load_system": [V, ctypes.c_char_p, V],
        "lindblad_steady_state": [V, I64, V, I64, V, V, V, D, I64, I64, V],
        "lindblad_steady_state_csr": [V, I64, V, V, V, V, V, V, D, I64, I64, V],
        "lindblad_secular_create": [V, I, V, I, V, V, ctypes.POINTER(ctypes.c_void_p)],
        "lindblad_secular_destroy": [V],
        "lindblad_propagate_batched": [V, I, I64, V, V, I64, V, V, I, D, I64, I],
        "lindblad_propagate_graph": [V, I64, V, V, I64, V, V, I, D, I64, I],
        "lindblad_autotune": [V, I64, V, V, I64, V, V, I, I],
        "lindblad_tile_info": [V, I64, I, I, V, V, V, V],
        "lindblad_set_tile": [V, I64, I, I, I, I, I],
        "lindblad_time_stage": [V, I, I64, V, V, I64, V, V, I, I, I, V],
        "lindblad_server_create": [I, ctypes.c_size_t, I, I, I, ctypes.POINTER(ctypes.c_void_p)],
        "lindblad_server_submit": [V, V, V],
        "lindblad_server_poll": [V, I64, V],
        "lindblad_server_wait": [V, I64],
        "lindblad_server_times": [V, I64, V, V, V],
        "lindblad_server_stats": [V, V, V, V, V],
        "lindblad_server_destroy": [V],
        "lindblad_server_register": [V, V, V],
        "lindblad_server_release": [V, I64],
    }


def _check(rc: int):
    if rc != 0:
        raise LindbladError(rc, load().lb_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) torch tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.is_complex() and t.is_conj():
        raise ValueError("%s is a lazy conjugate view (its memory is not conjugated); call resolve_conj()" % name)


_PROGRESS = ctypes.CFUNCTYPE(None, ctypes.c_char_p, ctypes.c_double, ctypes.c_void_p)


class Context:
    """A library context bound to a device and a stream (default: torch's
    current stream on that device)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        h = ctypes.c_void_p()
        _check(lib.lb_create(ctypes.byref(h), int(device), ctypes.c_void_p(handle or None)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def set_stream(self, stream):
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(load().lb_set_stream(self._h, ctypes.c_void_p(handle or None)))

    def sync(self):
        _check(load().lb_sync(self._h))

    def set_progress(self, fn=None):
        """fn(stage: str, fraction: float) is called during long calls (the spectrum),
        at most about every two seconds; None turns it off."""
        if fn is None:
            self._progress = None
            _check(load().lb_set_progress(self._h, None, None))
            return
        cb = _PROGRESS(lambda stage, frac, user: fn(stage.decode(), frac))
        self._progress = cb  # kept alive while set
        _check(load().lb_set_progress(self._h, ctypes.cast(cb, ctypes.c_void_p), None))

    def close(self):
        if self._h:
            load().lb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _dev(ctx):
    import torch
    return torch.device("cuda", ctx.device)


# ---------------------------------------------------------------------------
# basis and structure constants
# ---------------------------------------------------------------------------

def lb_basis_index(N: int, i: int):
    c, j, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().lb_basis_index(int(N), int(i), ctypes.byref(c), ctypes.byref(j), ctypes.byref(k)))
    return c.value, j.value, k.value


def lb_basis_table(ctx: Context, N: int):
    import torch
    M = N * N - 1
    t = torch.empty((M, 3), dtype=torch.int32, device=_dev(ctx))
    _check(load().lb_basis_table(ctx.handle, int(N), _ptr(t)))
    return t


def lb_fd_count(ctx: Context, N: int, which: str) -> int:
    n = ctypes.c_int64()
    _check(load().lb_fd_count(ctx.handle, int(N), {"f": 0, "d": 1}[which], ctypes.byref(n)))
    return n.value


def lb_fd_enumerate(ctx: Context, N: int, which: str):
    """(mns int32 (count, 3), val float64 (count,)) on the device."""
    import torch
    cnt = lb_fd_count(ctx, N, which)
    mns = torch.empty((max(cnt, 1), 3), dtype=torch.int32, device=_dev(ctx))
    val = torch.empty(max(cnt, 1), dtype=torch.float64, device=_dev(ctx))
    n = ctypes.c_int64()
    _check(load().lb_fd_enumerate(ctx.handle, int(N), {"f": 0, "d": 1}[which], _ptr(mns), _ptr(val),
                                  cnt, ctypes.byref(n)))
    return mns[:n.value], val[:n.value]


# ---------------------------------------------------------------------------
# expansion
# ---------------------------------------------------------------------------

def lb_expand(ctx: Context, A):
    """A: (B, N, N) or (N, N) complex128 Hermitian -> (B, M) or (M,) float64."""
    import torch
    squeeze = A.dim() == 2
    A3 = A.unsqueeze(0) if squeeze else A
    _need(A3, torch.complex128, "A")
    B, N = A3.shape[0], A3.shape[1]
    out = torch.empty((B, N * N - 1), dtype=torch.float64, device=A.device)
    _check(load().lb_expand(ctx.handle, N, B, _ptr(A3), _ptr(out)))
    return out[0] if squeeze else out


def lb_expand_pure(ctx: Context, psi):
    """psi: (B, N) or (N,) complex128 -> coherence vectors (B, M) float64."""
    import torch
    psi2 = psi.unsqueeze(0) if psi.dim() == 1 else psi
    _need(psi2, torch.complex128, "psi")
    B, N = psi2.shape
    out = torch.empty((B, N * N - 1), dtype=torch.float64, device=psi.device)
    _check(load().lb_expand_pure(ctx.handle, N, B, _ptr(psi2), _ptr(out)))
    return out


def lb_reconstruct(ctx: Context, V, N: int):
    import torch
    V2 = V.unsqueeze(0) if V.dim() == 1 else V
    _need(V2, torch.float64, "V")
    B = V2.shape[0]
    rho = torch.empty((B, N, N), dtype=torch.complex128, device=V.device)
    _check(load().lb_reconstruct(ctx.handle, N, B, _ptr(V2), _ptr(rho)))
    return rho


# ---------------------------------------------------------------------------
# data preparation
# ---------------------------------------------------------------------------

def default_ldq(M: int) -> int:
    """Leading dimension used by default: M rounded up to 32 elements, so that
    rows of Q (FP64) and of Q32 (FP32) start on 128-byte boundaries, which the
    LDS-staged stage GEMMs need."""
    return (M + 31) // 32 * 32


def lindblad_prepare(ctx: Context, H, gamma, ldq: int | None = None, Q=None, K=None,
                     check_hermitian: bool = False):
    """Dense Q (M x ldq, columns >= M zero) and K (M) for H (N,N) and gamma (M,M), complex128."""
    import torch
    _need(H, torch.complex128, "H")
    _need(gamma, torch.complex128, "gamma")
    N = H.shape[0]
    M = N * N - 1
    if gamma.shape != (M, M):
        raise ValueError("gamma must be (%d, %d)" % (M, M))
    ldq = default_ldq(M) if ldq is None else int(ldq)
    if Q is None:
        Q = torch.empty((M, ldq), dtype=torch.float64, device=H.device)
    if K is None:
        K = torch.empty(M, dtype=torch.float64, device=H.device)
    _need(Q, torch.float64, "Q")
    _need(K, torch.float64, "K")
    if Q.shape != (M, ldq) or K.shape != (M,):
        raise ValueError("Q must be (M, ldq) and K (M,)")
    _check(load().lindblad_prepare(ctx.handle, N, _ptr(H), _ptr(gamma), _ptr(Q), ldq, _ptr(K),
                                   CHECK_HERMITIAN if check_hermitian else 0))
    return Q, K


def _csr_struct(rowptr, col, val):
    import torch
    _need(rowptr, torch.int64, "rowptr")
    _need(col, torch.int64, "col")
    _need(val, torch.complex128, "val")
    return _CSR(rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), int(col.numel()))


def lindblad_prepare_sparse(ctx: Context, N: int, H_csr, rates, L_csrs):
    """Sparse Q (CSR: rowptr, col, val) and K for H and jump operators L_p with
    rates g_p. Each CSR is a tuple (rowptr int64, col int64, val complex128) on
    the device."""
    import torch
    lib = load()
    M = N * N - 1
    Hs = _csr_struct(*H_csr)
    P = len(L_csrs)
    Ls = (_CSR * max(P, 1))(*[_csr_struct(*l) for l in L_csrs])
    r = (ctypes.c_double * max(P, 1))(*[float(x) for x in rates])
    nnz = ctypes.c_int64()
    _check(lib.lindblad_prepare_sparse_count(ctx.handle, N, ctypes.byref(Hs), P, r, Ls, ctypes.byref(nnz)))
    dev = _dev(ctx)
    rowptr = torch.empty(M + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(nnz.value, 1), dtype=torch.int64, device=dev)
    val = torch.empty(max(nnz.value, 1), dtype=torch.float64, device=dev)
    K = torch.empty(M, dtype=torch.float64, device=dev)
    _check(lib.lindblad_prepare_sparse_fill(ctx.handle, N, ctypes.byref(Hs), P, r, Ls, nnz.value,
                                            _ptr(rowptr), _ptr(col), _ptr(val), _ptr(K)))
    return rowptr, col[:nnz.value], val[:nnz.value], K


# ---------------------------------------------------------------------------
# propagation
# ---------------------------------------------------------------------------

def lindblad_q_to_f32(ctx: Context, Q):
    import torch
    _need(Q, torch.float64, "Q")
    Q32 = torch.empty(Q.shape, dtype=torch.float32, device=Q.device)
    _check(load().lindblad_q_to_f32(ctx.handle, Q.shape[0], _ptr(Q), Q.shape[1], _ptr(Q32)))
    return Q32


def _prop_args(Q, Q32, K, V, precision):
    import torch
    if precision == FP64:
        _need(Q, torch.float64, "Q")
        M, ldq = Q.shape
    else:
        _need(Q32, torch.float32, "Q32")
        M, ldq = Q32.shape
    _need(K, torch.float64, "K")
    _need(V, torch.float64, "V")
    if V.dim() != 2 or V.shape[1] != M or K.shape != (M,):
        raise ValueError("V must be (B, M) and K (M,) with M = %d" % M)
    return M, ldq


def lindblad_propagate(ctx: Context, Q, K, V, dt: float, steps: int, precision: int = FP64, Q32=None):
    """In place: V (B, M) <- RK4 solution after `steps` steps of size dt."""
    M, ldq = _prop_args(Q, Q32, K, V, precision)
    _check(load().lindblad_propagate(ctx.handle, M, _ptr(Q) if Q is not None else None,
                                     _ptr(Q32) if Q32 is not None else None, ldq, _ptr(K), _ptr(V),
                                     V.shape[0], float(dt), int(steps), int(precision)))
    return V


def lindblad_propagate_noalloc(ctx: Context, Q, K, V, dt: float, steps: int, precision: int = FP64, Q32=None):
    """lindblad_propagate without any allocation: the buffers live in the
    library's static per-GPU array (calls on one GPU must not overlap)."""
    M, ldq = _prop_args(Q, Q32, K, V, precision)
    _check(load().lindblad_propagate_noalloc(ctx.handle, M, _ptr(Q) if Q is not None else None,
                                             _ptr(Q32) if Q32 is not None else None, ldq, _ptr(K), _ptr(V),
                                             V.shape[0], float(dt), int(steps), int(precision)))
    return V


def lindblad_propagate_graph(ctx: Context, Q, K, V, dt: float, steps: int, precision: int = FP64, Q32=None):
    M, ldq = _prop_args(Q, Q32, K, V, precision)
    _check(load().lindblad_propagate_graph(ctx.handle, M, _ptr(Q) if Q is not None else None,
                                           _ptr(Q32) if Q32 is not None else None, ldq, _ptr(K), _ptr(V),
                                           V.shape[0], float(dt), int(steps), int(precision)))
    return V


def lindblad_propagate_batched(ctx: Context, Qs, Ks, Vs, dt: float, steps: int, precision: int = FP64,
                               Q32s=None):
    """R systems of the same M; Vs[r] is (B, M), updated in place."""
    R = len(Ks)
    for r in range(R):
        M, ldq = _prop_args(Qs[r] if Qs else None, Q32s[r] if Q32s else None, Ks[r], Vs[r], precision)
    B = Vs[0].shape[0]
    arr = ctypes.c_void_p * R
    qa = arr(*[q.data_ptr() for q in Qs]) if Qs else None
    q32a = arr(*[q.data_ptr() for q in Q32s]) if Q32s else None
    ka = arr(*[k.data_ptr() for k in Ks])
    va = arr(*[v.data_ptr() for v in Vs])
    _check(load().lindblad_propagate_batched(ctx.handle, R, M, qa, q32a, ldq, ka, va, B, float(dt), int(steps),
                                             int(precision)))
    return Vs


def lindblad_propagate_csr(ctx: Context, rowptr, col, val, K, V, dt: float, steps: int):
    import torch
    _need(rowptr, torch.int64, "rowptr")
    _need(val, torch.float64, "val")
    _need(K, torch.float64, "K")
    _need(V, torch.float64, "V")
    M = rowptr.numel() - 1
    _check(load().lindblad_propagate_csr(ctx.handle, M, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(K), _ptr(V),
                                         V.shape[0], float(dt), int(steps)))
    return V


def lb_eigh(ctx: Context, A):
    """Eigenvalues w (unsorted) and eigenvectors Z (columns) of the Hermitian
    complex128 matrix A (device), A = Z diag(w) Z^H, by Jacobi on the device.
    Returns (w, Z, sweeps); A is not modified."""
    import torch
    _need(A, torch.complex128, "A")
    N = A.shape[0]
    # the library works column-major: pass the memory of A^T, read Z back transposed
    work = A.resolve_conj().transpose(0, 1).contiguous()
    w = torch.empty(N, dtype=torch.float64, device=A.device)
    Zc = torch.empty((N, N), dtype=torch.complex128, device=A.device)
    sw = ctypes.c_int()
    _check(load().lb_eigh(ctx.handle, N, _ptr(work), N, _ptr(w), _ptr(Zc), N, ctypes.byref(sw)))
    return w, Zc.transpose(0, 1), sw.value


class SpectrumInfo(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("chain_steps", ctypes.c_int64), ("updates", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("product_flops", ctypes.c_int64)]


def lb_hessenberg(ctx: Context, A):
    """Reduces the square float64 matrix A (device, rows of M, or a column slice of
    wider rows) in place to upper Hessenberg form by an orthogonal similarity."""
    import torch
    if not isinstance(A, torch.Tensor) or not A.is_cuda or A.dtype != torch.float64:
        raise ValueError("A must be a float64 CUDA (HIP) tensor")
    M = A.shape[0]
    if A.dim() != 2 or A.shape[1] != M or A.stride(1) != 1:
        raise ValueError("A must be M x M with unit column stride")
    _check(load().lb_hessenberg(ctx.handle, M, _ptr(A), A.stride(0)))
    return A


def lindblad_spectrum(ctx: Context, Q):
    """Eigenvalues of the generator Q (float64 M x M on the device, rows may be
    padded: Q = buffer[:, :M]). Returns (lam, info): lam complex128 (M,) on the
    device, conjugate pairs adjacent; info = {sweeps, chain_steps, updates, rounds,
    product_flops}."""
    import torch
    if not isinstance(Q, torch.Tensor) or not Q.is_cuda or Q.dtype != torch.float64:
        raise ValueError("Q must be a float64 CUDA (HIP) tensor")
    M = Q.shape[0]
    if Q.dim() != 2 or Q.shape[1] != M or Q.stride(1) != 1:
        raise ValueError("Q must be M x M with unit column stride")
    lam = torch.empty(2 * M, dtype=torch.float64, device=Q.device)
    info = SpectrumInfo()
    _check(load().lindblad_spectrum(ctx.handle, M, _ptr(Q), Q.stride(0), _ptr(lam), ctypes.byref(info)))
    return torch.view_as_complex(lam.view(M, 2)), {"sweeps": info.sweeps, "chain_steps": info.chain_steps,
                                                   "updates": info.updates, "rounds": info.rounds,
                                                   "product_flops": info.product_flops}


def lindblad_spectrum_histogram(ctx: Context, lam, re0: float, re1: float, im0: float, im1: float, nx: int, ny: int):
    """Counts of the complex128 values lam (device) per cell of the nx x ny grid
    over [re0, re1) x [im0, im1); int64 (ny, nx), row = imaginary cell."""
    import torch
    _need(lam, torch.complex128, "lam")
    counts = torch.empty((ny, nx), dtype=torch.int64, device=lam.device)
    _check(load().lindblad_spectrum_histogram(ctx.handle, lam.numel(), _ptr(torch.view_as_real(lam)), float(re0),
                                              float(re1), float(im0), float(im1), int(nx), int(ny), _ptr(counts)))
    return counts


def _need_cover(t, dtype, name, rows, cols, ld):
    """t must be a contiguous device tensor holding a column-major rows x cols
    matrix with leading dimension ld."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype:
        raise ValueError("%s must be a CUDA (HIP) %s tensor" % (name, dtype))
    if not t.is_contiguous() or (t.is_complex() and t.is_conj()):
        raise ValueError("%s must be contiguous (and not a lazily conjugated view)" % name)
    if ld < max(1, rows):
        raise ValueError("%s: leading dimension %d below its %d rows" % (name, ld, rows))
    if rows > 0 and cols > 0 and t.numel() < (cols - 1) * ld + rows:
        raise ValueError("%s holds %d elements, fewer than a %d x %d matrix with leading dimension %d"
                         % (name, t.numel(), rows, cols, ld))


def gemm_f64(ctx: Context, m: int, n: int, k: int, A, lda: int, B, ldb: int, C, ldc: int, alpha: float = 1.0,
             beta: float = 0.0, trans_a: bool = False, trans_b: bool = False):
    """C = alpha op(A) op(B) + beta C (lb_gemm_f64): float64 device tensors
    holding column-major matrices with leading dimensions; C is m x n, op(A)
    m x k, op(B) k x n, op the transpose when trans_a / trans_b (A then stored
    k x m, B n x k)."""
    import torch
    _need_cover(A, torch.float64, "A", k if trans_a else m, m if trans_a else k, lda)
    _need_cover(B, torch.float64, "B", n if trans_b else k, k if trans_b else n, ldb)
    _need_cover(C, torch.float64, "C", m, n, ldc)
    _check(load().lb_gemm_f64(ctx.handle, int(trans_a), int(trans_b), m, n, k, float(alpha), _ptr(A), lda,
                              _ptr(B), ldb, float(beta), _ptr(C), ldc))
    return C


def gemm_c128(ctx: Context, m: int, n: int, k: int, A, lda: int, B, ldb: int, C, ldc: int, conj_a: bool = False,
              conj_b: bool = False, work=None):
    """C = op(A) op(B) (lb_gemm_c128) on complex128 device tensors holding
    column-major matrices (leading dimensions in complex elements); op is the
    conjugate transpose when conj_a / conj_b. work: optional complex128 device
    scratch for splitting k (see lb_gemm_c128)."""
    import torch
    _need_cover(A, torch.complex128, "A", k if conj_a else m, m if conj_a else k, lda)
    _need_cover(B, torch.complex128, "B", n if conj_b else k, k if conj_b else n, ldb)
    _need_cover(C, torch.complex128, "C", m, n, ldc)
    wp, wn = None, 0
    if work is not None:
        _need_cover(work, torch.complex128, "work", work.numel(), 1, work.numel())
        wp, wn = _ptr(work), work.numel()
    _check(load().lb_gemm_c128(ctx.handle, int(conj_a), int(conj_b), m, n, k, _ptr(A), lda, _ptr(B), ldb, _ptr(C),
                               ldc, wp, wn))
    return C


def read_bandwidth(ctx: Context, nbytes: int = 4 << 30) -> float:
    """The device's read-stream bandwidth in GB/s (lb_read_bandwidth)."""
    g = ctypes.c_double()
    _check(load().lb_read_bandwidth(ctx.handle, int(nbytes), ctypes.byref(g)))
    return g.value


class _System(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("N", ctypes.c_int), ("ldq", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("Q", ctypes.c_void_p), ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("K", ctypes.c_void_p)]


SYSTEM_DENSE = 0
SYSTEM_CSR = 1


def save_system(ctx: Context, path: str, N: int, K, Q=None, csr=None):
    """Writes a prepared system to `path`: dense Q (M x ldq) or csr = (rowptr,
    col, val) as written by lindblad_prepare_sparse, and K (device tensors)."""
    import torch
    _need(K, torch.float64, "K")
    s = _System()
    s.N = N
    s.K = K.data_ptr()
    if Q is not None:
        _need(Q, torch.float64, "Q")
        s.kind, s.ldq, s.Q = SYSTEM_DENSE, Q.stride(0), Q.data_ptr()
    else:
        rp, col, val = csr
        _need(rp, torch.int64, "rowptr")
        _need(val, torch.float64, "val")
        s.kind, s.nnz, s.rowptr, s.col, s.val = SYSTEM_CSR, col.numel(), rp.data_ptr(), col.data_ptr(), val.data_ptr()
    _check(load().lindblad_save_system(ctx.handle, path.encode(), ctypes.byref(s)))


def load_system_info(path: str):
    """(kind, N, nnz) from the file's header (host only)."""
    s = _System()
    _check(load().lindblad_load_system_info(path.encode(), ctypes.byref(s)))
    return s.kind, s.N, s.nnz


def load_system(ctx: Context, path: str, ldq: int | None = None):
    """Loads a saved system into new device tensors: (Q, K) for a dense file
    (Q of shape (M, ldq), default ldq as lindblad_prepare), ((rowptr, col,
    val), K) for a CSR file."""
    import torch
    kind, N, nnz = load_system_info(path)
    M = N * N - 1
    dev = _dev(ctx)
    s = _System()
    s.kind, s.N, s.nnz = kind, N, nnz
    K = torch.empty(M, dtype=torch.float64, device=dev)
    s.K = K.data_ptr()
    if kind == SYSTEM_DENSE:
        ldq = default_ldq(M) if ldq is None else int(ldq)
        Q = torch.empty((M, ldq), dtype=torch.float64, device=dev)
        s.ldq, s.Q = ldq, Q.data_ptr()
        _check(load().lindblad_load_system(ctx.handle, path.encode(), ctypes.byref(s)))
        return Q, K
    rp = torch.empty(M + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(nnz, 1), dtype=torch.int64, device=dev)
    val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
    s.rowptr, s.col, s.val = rp.data_ptr(), col.data_ptr(), val.data_ptr()
    _check(load().lindblad_load_system(ctx.handle, path.encode(), ctypes.byref(s)))
    return (rp, col[:nnz], val[:nnz]), K


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("restarts", ctypes.c_int64), ("residual", ctypes.c_double),
                ("converged", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _steady_call(fn, args, check):
    info = SolveInfo()
    rc = fn(*args, ctypes.byref(info))
    if rc != 0 and not (rc == -7 and not check):
        _check(rc)
    return info.as_dict()


class Secular:
    """Steady-state preconditioner (secular approximation in the energy
    eigenbasis of H) for the system of H and jump operators L_p (device CSR
    tuples as for lindblad_prepare_sparse). Release with close()."""

    def __init__(self, ctx: Context, N: int, H_csr, rates, L_csrs):
        lib = load()
        Hs = _csr_struct(*H_csr)
        P = len(L_csrs)
        Ls = (_CSR * max(P, 1))(*[_csr_struct(*l) for l in L_csrs])
        r = (ctypes.c_double * max(P, 1))(*[float(x) for x in rates])
        self._keep = (H_csr, L_csrs)
        h = ctypes.c_void_p()
        _check(lib.lindblad_secular_create(ctx.handle, N, ctypes.byref(Hs), P, r, Ls, ctypes.byref(h)))
        self.handle = h
        self.N = N

    def close(self):
        if self.handle:
            load().lindblad_secular_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lindblad_steady_state(ctx: Context, Q, K, tol: float = 1e-12, maxit: int = 4000, restart: int | None = None,
                          check: bool = True, pre: Secular | None = None):
    """v with Q v = -K (dense Q, M x ldq), by FP64 GMRES on the device (right-
    preconditioned by pre, if given). Returns (v, info) with info = {iterations,
    restarts, residual, converged}; a solve that stops at maxit raises unless
    check is False."""
    import torch
    _need(Q, torch.float64, "Q")
    _need(K, torch.float64, "K")
    M = K.numel()
    v = torch.empty(M, dtype=torch.float64, device=K.device)
    info = _steady_call(load().lindblad_steady_state,
                        (ctx.handle, M, _ptr(Q), Q.stride(0), _ptr(K), pre.handle if pre else None, _ptr(v),
                         float(tol), int(maxit),
                         int(restart or min(maxit, 8192))), check)
    return v, info


def lindblad_steady_state_csr(ctx: Context, rowptr, col, val, K, tol: float = 1e-12, maxit: int = 4000,
                              restart: int | None = None, check: bool = True, pre: Secular | None = None):
    """As lindblad_steady_state for Q in CSR form."""
    import torch
    _need(rowptr, torch.int64, "rowptr")
    _need(val, torch.float64, "val")
    _need(K, torch.float64, "K")
    M = rowptr.numel() - 1
    v = torch.empty(M, dtype=torch.float64, device=K.device)
    info = _steady_call(load().lindblad_steady_state_csr,
                        (ctx.handle, M, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(K), pre.handle if pre else None,
                         _ptr(v), float(tol), int(maxit),
                         int(restart or min(maxit, 8192))), check)
    return v, info


def lindblad_propagate_csr_drive(ctx: Context, Q0, Q1, K, V, dt: float, steps: int, t0: float, E: float, A: float,
                                 T: float, k0: int = 0):
    """In place: RK4 of dv/dt = (Q0 + eps(t) Q1) v + K with the square-wave
    drive eps(t) = E + A Theta(t) over steps k0 .. k0 + steps - 1 of the grid
    t0 + k dt; Q0, Q1 are (rowptr, col, val) CSR triples."""
    import torch
    for name, (rp, c, v) in (("Q0", Q0), ("Q1", Q1)):
        _need(rp, torch.int64, name + " rowptr")
        _need(c, torch.int64, name + " col")
        _need(v, torch.float64, name + " val")
    _need(K, torch.float64, "K")
    _need(V, torch.float64, "V")
    M = Q0[0].numel() - 1
    if Q1[0].numel() != M + 1:
        raise ValueError("Q0 and Q1 must have the same number of rows")
    _check(load().lindblad_propagate_csr_drive(ctx.handle, M, _ptr(Q0[0]), _ptr(Q0[1]), _ptr(Q0[2]), _ptr(Q1[0]),
                                               _ptr(Q1[1]), _ptr(Q1[2]), _ptr(K), _ptr(V), V.shape[0], float(dt),
                                               int(steps), float(t0), int(k0), float(E), float(A), float(T)))
    return V


def lindblad_autotune(ctx: Context, Q, K, B: int, precision: int = FP64, Q32=None):
    import torch
    M = (Q if precision == FP64 else Q32).shape[0]
    ldq = (Q if precision == FP64 else Q32).shape[1]
    V = torch.zeros((B, M), dtype=torch.float64, device=K.device)
    _check(load().lindblad_autotune(ctx.handle, M, _ptr(Q) if Q is not None else None,
                                    _ptr(Q32) if Q32 is not None else None, ldq, _ptr(K), _ptr(V), B, precision))


def lindblad_graph_clear(ctx: Context) -> int:
    """Frees the context's captured graphs; returns how many there were."""
    n = ctypes.c_int()
    _check(load().lindblad_graph_clear(ctx.handle, ctypes.byref(n)))
    return n.value


def lindblad_set_tile(ctx: Context, M: int, B: int, rows: int, kslab: int, waves: int, precision: int = FP64):
    _check(load().lindblad_set_tile(ctx.handle, int(M), int(B), int(precision), int(rows), int(kslab), int(waves)))


def lindblad_tile_info(ctx: Context, M: int, B: int, precision: int = FP64):
    r, k, w, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().lindblad_tile_info(ctx.handle, int(M), int(B), int(precision), ctypes.byref(r),
                                     ctypes.byref(k), ctypes.byref(w), ctypes.byref(t)))
    return {"rows": r.value, "kslab": k.value, "waves": w.value, "tuned": bool(t.value)}


def lindblad_time_stage(ctx: Context, Qs, Ks, Vs, iters: int = 10, precision: int = FP64, Q32s=None) -> float:
    """Average duration (ms) of one launch of the dominant RK4 stage kernel over
    the R systems (HIP events on the context stream)."""
    R = len(Ks)
    for r in range(R):
        M, ldq = _prop_args(Qs[r] if Qs else None, Q32s[r] if Q32s else None, Ks[r], Vs[r], precision)
    arr = ctypes.c_void_p * R
    qa = arr(*[q.data_ptr() for q in Qs]) if Qs else None
    q32a = arr(*[q.data_ptr() for q in Q32s]) if Q32s else None
    ka = arr(*[k.data_ptr() for k in Ks])
    va = arr(*[v.data_ptr() for v in Vs])
    ms = ctypes.c_double()
    _check(load().lindblad_time_stage(ctx.handle, R, M, qa, q32a, ldq, ka, va, Vs[0].shape[0], int(precision),
                                      int(iters), ctypes.byref(ms)))
    return ms.value


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

MAX_JUMPS = 8


class _Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("N", ctypes.c_int), ("H", ctypes.c_void_p), ("gamma", ctypes.c_void_p),
                ("Hs", _CSR), ("P", ctypes.c_int), ("rates", ctypes.c_double * MAX_JUMPS),
                ("L", _CSR * MAX_JUMPS), ("V0", ctypes.c_void_p), ("Vout", ctypes.c_void_p), ("B", ctypes.c_int),
                ("dt", ctypes.c_double), ("steps", ctypes.c_int64), ("precision", ctypes.c_int),
                ("system", ctypes.c_int64)]


class Server:
    """Continuous-batching server over the library (see lindblad_server_* in
    include/lindblad.h). Submitted tensors are kept referenced until the
    request's completion has been observed through wait()."""

    def __init__(self, device: int = 0, budget_bytes: int = 16 << 30, slots: int = 4, max_batch: int = 8,
                 max_N: int = 128):
        h = ctypes.c_void_p()
        _check(load().lindblad_server_create(int(device), int(budget_bytes), int(slots), int(max_batch),
                                             int(max_N), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit_dense(self, H, gamma, V0, dt: float, steps: int, precision: int = FP64):
        import torch
        _need(H, torch.complex128, "H")
        _need(gamma, torch.complex128, "gamma")
        _need(V0, torch.float64, "V0")
        Vout = torch.empty_like(V0)
        r = _Request()
        r.kind, r.N = 0, H.shape[0]
        r.H, r.gamma = H.data_ptr(), gamma.data_ptr()
        r.V0, r.Vout, r.B = V0.data_ptr(), Vout.data_ptr(), V0.shape[0]
        r.dt, r.steps, r.precision = float(dt), int(steps), int(precision)
        return self._submit(r, (H, gamma, V0, Vout), Vout)

    def submit_sparse(self, N: int, H_csr, rates, L_csrs, V0, dt: float, steps: int):
        import torch
        _need(V0, torch.float64, "V0")
        if len(L_csrs) > MAX_JUMPS:
            raise ValueError("at most %d jump operators" % MAX_JUMPS)
        Vout = torch.empty_like(V0)
        r = _Request()
        r.kind, r.N = 1, int(N)
        r.Hs = _csr_struct(*H_csr)
        r.P = len(L_csrs)
        for p, (g, l) in enumerate(zip(rates, L_csrs)):
            r.rates[p] = float(g)
            r.L[p] = _csr_struct(*l)
        r.V0, r.Vout, r.B = V0.data_ptr(), Vout.data_ptr(), V0.shape[0]
        r.dt, r.steps, r.precision = float(dt), int(steps), FP64
        return self._submit(r, (H_csr, L_csrs, V0, Vout), Vout)

    def register_dense(self, H, gamma, precision: int = FP64) -> int:
        """Prepares Q and K of a dense Lindbladian once and keeps them resident;
        returns the system id for submit_system()."""
        import torch
        _need(H, torch.complex128, "H")
        _need(gamma, torch.complex128, "gamma")
        r = _Request()
        r.kind, r.N = 0, H.shape[0]
        r.H, r.gamma, r.precision = H.data_ptr(), gamma.data_ptr(), int(precision)
        sid = ctypes.c_int64()
        _check(load().lindblad_server_register(self._h, ctypes.byref(r), ctypes.byref(sid)))
        return sid.value

    def register_sparse(self, N: int, H_csr, rates, L_csrs) -> int:
        if len(L_csrs) > MAX_JUMPS:
            raise ValueError("at most %d jump operators" % MAX_JUMPS)
        r = _Request()
        r.kind, r.N = 1, int(N)
        r.Hs = _csr_struct(*H_csr)
        r.P = len(L_csrs)
        for p, (g, l) in enumerate(zip(rates, L_csrs)):
            r.rates[p] = float(g)
            r.L[p] = _csr_struct(*l)
        r.precision = FP64
        sid = ctypes.c_int64()
        _check(load().lindblad_server_register(self._h, ctypes.byref(r), ctypes.byref(sid)))
        return sid.value

    def submit_system(self, system: int, V0, dt: float, steps: int, precision: int = FP64):
        """Integrates the states V0 (B, M) on a registered system."""
        import torch
        _need(V0, torch.float64, "V0")
        Vout = torch.empty_like(V0)
        r = _Request()
        r.kind, r.system = 2, int(system)
        r.V0, r.Vout, r.B = V0.data_ptr(), Vout.data_ptr(), V0.shape[0]
        r.dt, r.steps, r.precision = float(dt), int(steps), int(precision)
        return self._submit(r, (V0, Vout), Vout)

    def release(self, system: int):
        _check(load().lindblad_server_release(self._h, int(system)))

    def _submit(self, r, keep, Vout):
        t = ctypes.c_int64()
        _check(load().lindblad_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value, Vout

    def wait(self, ticket: int):
        rc = load().lindblad_server_wait(self._h, int(ticket))
        self._keep.pop(ticket, None)
        _check(rc)

    def done(self, ticket: int) -> bool:
        d = ctypes.c_int()
        _check(load().lindblad_server_poll(self._h, int(ticket), ctypes.byref(d)))
        return bool(d.value)

    def times(self, ticket: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(load().lindblad_server_times(self._h, int(ticket), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def stats(self):
        c, b, n, m = ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().lindblad_server_stats(self._h, ctypes.byref(c), ctypes.byref(b), ctypes.byref(n),
                                            ctypes.byref(m)))
        return {"completed": c.value, "peak_bytes": b.value, "batches": n.value, "batched_requests": m.value}

    def close(self):
        if self._h:
            load().lindblad_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
