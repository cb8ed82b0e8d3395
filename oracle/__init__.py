"""CPU FP64 oracle for the GKSL -> real linear ODE transformation (TEST INFRASTRUCTURE).

This package is test infrastructure: a plain, slow, obviously-correct
implementation of what the GPU library computes, written from the paper
(Meyerov et al., arXiv:1912.01491, Sec. 2 and Table 1). Only the test suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
it. The GPU library never imports it and shares no code with it.

The arithmetic lives in ``lindblad_oracle.c`` (plain C, FP64, OpenMP over
output rows); this module only marshals numpy arrays through ctypes.

Functions (all arrays numpy, complex matrices as complex128):
  index_of, class_of          basis order (S block, J block, D block; 0-based)
  basis_dense                 F_i as an N x N matrix (Eqs. (3)-(5))
  fd_count, fd_enumerate      nonzero structure constants (Eq. (11), step 2.2)
  expand, reconstruct         Eqs. (6), (7) (steps 2.1, 2.6, 3.2)
  prepare_dense               Q = Q_H + Q_D rows and K (Eqs. (13)-(15))
  jump_setup, prepare_factored   the same for gamma = sum_p g_p l_p l_p^dagger
  rk4_dense, rk4_csr          classic RK4 for dv/dt = Qv + K (Eq. (10), step 3.1)
  drive, drive_left, rk4_drive   the rocked dimer's square-wave drive and its RK4 (Sec. 3)
  steady_state                Qv = -K, the asymptotic state rho_inf of Sec. 3 (dense solve)
  spectrum, histogram         eigenvalues of Q and their counts on a grid (Sec. 5, Fig. 5)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lindblad_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liblindblad_oracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp). Returns the library path."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_long
        lib.or_index_of.restype = i64
        lib.or_index_of.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.or_class_of.restype = None
        lib.or_class_of.argtypes = [ctypes.c_int, i64, P, P, P]
        lib.or_basis_dense.restype = None
        lib.or_basis_dense.argtypes = [ctypes.c_int, i64, P]
        lib.or_fd_count.restype = None
        lib.or_fd_count.argtypes = [ctypes.c_int, P, P]
        lib.or_fd_enumerate.restype = i64
        lib.or_fd_enumerate.argtypes = [ctypes.c_int, ctypes.c_int, P, P, i64]
        lib.or_expand.restype = None
        lib.or_expand.argtypes = [ctypes.c_int, P, P]
        lib.or_reconstruct.restype = None
        lib.or_reconstruct.argtypes = [ctypes.c_int, P, P]
        lib.or_prepare_dense.restype = None
        lib.or_prepare_dense.argtypes = [ctypes.c_int, P, P, P, i64, P, P, P]
        lib.or_jump_setup.restype = None
        lib.or_jump_setup.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, P, P]
        lib.or_prepare_factored.restype = None
        lib.or_prepare_factored.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, P, i64, P, P]
        lib.or_rk4_dense.restype = None
        lib.or_rk4_dense.argtypes = [i64, P, P, P, ctypes.c_int, ctypes.c_double, i64]
        lib.or_rk4_csr.restype = None
        lib.or_rk4_csr.argtypes = [i64, P, P, P, P, P, ctypes.c_int, ctypes.c_double, i64]
        D = ctypes.c_double
        lib.or_drive.restype = D
        lib.or_drive.argtypes = [D, D, D, D]
        lib.or_drive_left.restype = D
        lib.or_drive_left.argtypes = [D, D, D, D]
        lib.or_rk4_drive.restype = None
        lib.or_rk4_drive.argtypes = [i64, P, P, P, P, ctypes.c_int, D, i64, D, D, D, D]
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_num_threads.argtypes = []
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(_L().or_num_threads())


def n_gen(N: int) -> int:
    return N * N - 1


def index_of(N: int, cls: int, j: int, k: int = 0) -> int:
    """Basis position of S^(j,k) (cls 0), J^(j,k) (cls 1) or D^j (cls 2); 0-based j<k."""
    return int(_L().or_index_of(N, cls, j, k))


def class_of(N: int, i: int):
    c, j, k = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _L().or_class_of(N, i, ctypes.byref(c), ctypes.byref(j), ctypes.byref(k))
    return c.value, j.value, k.value


def basis_dense(N: int, i: int) -> np.ndarray:
    F = np.zeros((N, N), dtype=np.complex128)
    _L().or_basis_dense(N, i, _p(F))
    return F


def fd_count(N: int):
    nf, nd = ctypes.c_long(), ctypes.c_long()
    _L().or_fd_count(N, ctypes.byref(nf), ctypes.byref(nd))
    return nf.value, nd.value


def fd_enumerate(N: int, which: str):
    """All ordered (m, n, s) with f_mns != 0 (which='f') or d_mns != 0 ('d').
    Returns (int32 array (count, 3), float64 values)."""
    w = {"f": 0, "d": 1}[which]
    lib = _L()
    dummy_i = np.zeros((1, 3), np.int32)
    dummy_v = np.zeros(1, np.float64)
    cnt = lib.or_fd_enumerate(N, w, _p(dummy_i), _p(dummy_v), 0)
    mns = np.zeros((cnt, 3), np.int32)
    val = np.zeros(cnt, np.float64)
    lib.or_fd_enumerate(N, w, _p(mns), _p(val), cnt)
    return mns, val


def expand(A: np.ndarray) -> np.ndarray:
    """a_j = Tr(F_j A), j < M (Eq. (6)). Complex result; real part for Hermitian A."""
    A = _c(A, np.complex128)
    N = A.shape[0]
    a = np.zeros(n_gen(N), np.complex128)
    _L().or_expand(N, _p(A), _p(a))
    return a


def reconstruct(N: int, v: np.ndarray) -> np.ndarray:
    v = _c(v, np.float64)
    rho = np.zeros((N, N), np.complex128)
    _L().or_reconstruct(N, _p(v), _p(rho))
    return rho


def prepare_dense(H: np.ndarray, gamma: np.ndarray, rows=None, with_imag: bool = False):
    """Rows of Q (default: all) and K for dense H (N x N) and gamma (M x M)."""
    H = _c(H, np.complex128)
    gamma = _c(gamma, np.complex128)
    N = H.shape[0]
    M = n_gen(N)
    assert gamma.shape == (M, M)
    rows = np.arange(M, dtype=np.int64) if rows is None else _c(rows, np.int64)
    Q = np.zeros((len(rows), M), np.float64)
    K = np.zeros(M, np.float64)
    mi = ctypes.c_double(0.0)
    _L().or_prepare_dense(N, _p(H), _p(gamma), _p(rows), len(rows), _p(Q), _p(K), ctypes.byref(mi))
    if with_imag:
        return Q, K, mi.value
    return Q, K


def jump_setup(H: np.ndarray, rates, Ls):
    """Moves jump-operator trace parts into H; returns (H_eff, l (P x M complex))."""
    H = _c(H, np.complex128)
    N = H.shape[0]
    rates = _c(rates, np.float64)
    Ls = _c(np.stack([np.asarray(L) for L in Ls]), np.complex128)
    P = Ls.shape[0]
    Heff = np.zeros((N, N), np.complex128)
    l = np.zeros((P, n_gen(N)), np.complex128)
    _L().or_jump_setup(N, _p(H), P, _p(rates), _p(Ls), _p(Heff), _p(l))
    return Heff, l


def prepare_factored(H: np.ndarray, rates, Ls, rows):
    """Rows of Q and the matching entries of K for gamma = sum_p g_p l_p l_p^dagger,
    with l_p the expansion of the jump operators Ls (trace parts moved into H)."""
    Heff, l = jump_setup(H, rates, Ls)
    N = Heff.shape[0]
    M = n_gen(N)
    rows = _c(rows, np.int64)
    Q = np.zeros((len(rows), M), np.float64)
    K = np.zeros(len(rows), np.float64)
    _L().or_prepare_factored(N, _p(Heff), l.shape[0], _p(_c(rates, np.float64)), _p(l),
                             _p(rows), len(rows), _p(Q), _p(K))
    return Q, K


def rk4_dense(Q: np.ndarray, K: np.ndarray, V: np.ndarray, dt: float, steps: int) -> np.ndarray:
    """Classic RK4 on dv/dt = Qv + K; V is (B, M); returns the updated copy."""
    Q = _c(Q, np.float64)
    K = _c(K, np.float64)
    V = np.array(V, dtype=np.float64, order="C", copy=True)
    if V.ndim == 1:
        V = V[None, :]
    M = Q.shape[0]
    _L().or_rk4_dense(M, _p(Q), _p(K), _p(V), V.shape[0], float(dt), int(steps))
    return V


def drive(t: float, E: float, A: float, T: float) -> float:
    """The square-wave modulation eps(t) = E + A Theta(t) of the driven dimer."""
    return float(_L().or_drive(float(t), float(E), float(A), float(T)))


def drive_left(t: float, E: float, A: float, T: float) -> float:
    """eps(t-), the limit from the left (at a switch: the half period ending there)."""
    return float(_L().or_drive_left(float(t), float(E), float(A), float(T)))


def rk4_drive(Q0, Q1, K, V, dt: float, steps: int, t0: float, E: float, A: float, T: float) -> np.ndarray:
    """Classic RK4 on dv/dt = (Q0 + eps(t) Q1) v + K (dense Q0, Q1); V is (B, M)."""
    Q0 = _c(Q0, np.float64)
    Q1 = _c(Q1, np.float64)
    K = _c(K, np.float64)
    V = np.array(V, dtype=np.float64, order="C", copy=True)
    if V.ndim == 1:
        V = V[None, :]
    M = Q0.shape[0]
    _L().or_rk4_drive(M, _p(Q0), _p(Q1), _p(K), _p(V), V.shape[0], float(dt), int(steps), float(t0), float(E),
                      float(A), float(T))
    return V


def rk4_csr(rowptr, col, val, K, V, dt: float, steps: int) -> np.ndarray:
    rowptr = _c(rowptr, np.int64)
    col = _c(col, np.int64)
    val = _c(val, np.float64)
    K = _c(K, np.float64)
    V = np.array(V, dtype=np.float64, order="C", copy=True)
    if V.ndim == 1:
        V = V[None, :]
    M = len(rowptr) - 1
    _L().or_rk4_csr(M, _p(rowptr), _p(col), _p(val), _p(K), _p(V), V.shape[0], float(dt), int(steps))
    return V


def steady_state(Q: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Stationary point of dv/dt = Qv + K (Eq. (10) with dv/dt = 0): the v with
    Qv = -K, i.e. the expansion (Eq. (7)) of the asymptotic state rho_inf with
    L(rho_inf) = 0 of Sec. 3. A dense LU solve (LAPACK through numpy)."""
    Q = _c(Q, np.float64)
    K = _c(K, np.float64)
    return np.linalg.solve(Q, -K)


def spectrum(Q: np.ndarray) -> np.ndarray:
    """Eigenvalues of the real generator Q of Eq. (10). With rho = 1/N + sum_n v_n F_n
    (Eq. (7)) the Lindbladian acts on the coordinates (1, v) as the block matrix
    [[0, 0], [K, Q]], so its spectrum is 0 together with the M = N^2 - 1 eigenvalues
    of Q: the values histogrammed in Fig. 5. LAPACK's nonsymmetric eigenvalue
    routine through numpy (a library primitive), complex128 in LAPACK's order."""
    return np.linalg.eigvals(_c(Q, np.float64))


def histogram(lam, re0: float, re1: float, im0: float, im1: float, nx: int, ny: int) -> np.ndarray:
    """Eigenvalue counts on the nx x ny grid of Fig. 5 (100 x 100 cells there; the
    figure divides each count by the cell area). A value lands in column
    ix = floor((Re - re0) / dx), dx = (re1 - re0) / nx, and row iy = floor((Im - im0) / dy),
    dy = (im1 - im0) / ny; it is counted when 0 <= (Re - re0) / dx < nx and
    0 <= (Im - im0) / dy < ny (so the left and lower edges belong to the grid, the
    right and upper ones do not, and NaN is never counted). Returns int64 (ny, nx)."""
    dx = (float(re1) - float(re0)) / nx
    dy = (float(im1) - float(im0)) / ny
    out = np.zeros((ny, nx), np.int64)
    for z in np.asarray(lam, np.complex128).ravel():
        tx = (float(z.real) - float(re0)) / dx
        ty = (float(z.imag) - float(im0)) / dy
        if 0.0 <= tx < nx and 0.0 <= ty < ny:
            out[int(math.floor(ty)), int(math.floor(tx))] += 1
    return out
