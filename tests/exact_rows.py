"""Exact rows of Q and entries of K for sparse H and jump operators (tests only).

Independent of the oracle and of the library. With rho = 1/N + sum_n v_n F_n
(Eq. (7)) and Tr(F_s F_n) = delta, Q_sn = Tr(F_s L(F_n)) and
K_s = Tr(F_s L(1/N)). Moving L onto F_s (the adjoint, Heisenberg-picture
generator of Eqs. (1), (2)),

    A_s = i[H, F_s] + sum_p g_p (L_p^+ F_s L_p - 1/2 {L_p^+ L_p, F_s}),

row s of Q is the expansion of A_s in the basis, Q_sn = Tr(F_n A_s), and
K_s = Tr(A_s) / N. For sparse H and L_p (a dimer: tridiagonal) A_s has O(N)
entries, so a row costs O(N) operations whatever M is.

The arithmetic is exact: the FP64 inputs are taken as exact rationals, the
generators without their normalisation have integer entries (Eqs. (3)-(5),
D^l read as Hermitian, R1), and the two normalisations of F_s and F_n
(1/sqrt 2 or 1/sqrt(l(l+1))) are applied at the end in 50-digit arithmetic.
Jump operators are used as given, trace parts included (the oracle and the
library move those into H first). Basis order: S^(j,k) for j<k row-major, then
J^(j,k), then D^1..D^{N-1}; J^(j,k) has -i/sqrt 2 at (j,k).
"""
from fractions import Fraction as Fr

import mpmath
import numpy as np

mpmath.mp.dps = 50
_ZERO = Fr(0)


class _C:
    """Exact complex number: a pair of rationals."""
    __slots__ = ("re", "im")

    def __init__(self, re=_ZERO, im=_ZERO):
        self.re, self.im = re, im

    def __add__(a, b):
        return _C(a.re + b.re, a.im + b.im)

    def __sub__(a, b):
        return _C(a.re - b.re, a.im - b.im)

    def __mul__(a, b):
        return _C(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re)

    def conj(a):
        return _C(a.re, -a.im)

    def scale(a, f):
        return _C(a.re * f, a.im * f)


_I = _C(_ZERO, Fr(1))


def _sparse(A):
    """Dense complex array -> {row: {col: exact value}} over the nonzeros."""
    out = {}
    for r, c in zip(*np.nonzero(A)):
        v = complex(A[r, c])
        out.setdefault(int(r), {})[int(c)] = _C(Fr(v.real), Fr(v.imag))
    return out


def _mul(A, B):
    out = {}
    for r, row in A.items():
        acc = out.setdefault(r, {})
        for k, a in row.items():
            for c, b in B.get(k, {}).items():
                acc[c] = acc.get(c, _C()) + a * b
    return out


def _add(A, B, f=Fr(1)):
    out = {r: dict(row) for r, row in A.items()}
    for r, row in B.items():
        acc = out.setdefault(r, {})
        for c, b in row.items():
            acc[c] = acc.get(c, _C()) + b.scale(f)
    return out


def _dagger(A):
    out = {}
    for r, row in A.items():
        for c, a in row.items():
            out.setdefault(c, {})[r] = a.conj()
    return out


def _generator(N, s):
    """Unnormalised F_s (integer entries) and its normalisation."""
    P = N * (N - 1) // 2
    if s < 2 * P:
        cls, q = divmod(s, P)
        j = 0
        while q >= N - 1 - j:
            q -= N - 1 - j
            j += 1
        k = j + 1 + q
        if cls == 0:
            F = {j: {k: _C(Fr(1))}, k: {j: _C(Fr(1))}}
        else:
            F = {j: {k: _C(_ZERO, Fr(-1))}, k: {j: _C(_ZERO, Fr(1))}}
        return F, 1 / mpmath.sqrt(2)
    l = s - 2 * P + 1
    F = {x: {x: _C(Fr(1))} for x in range(l)}
    F[l] = {l: _C(Fr(-l))}
    return F, 1 / mpmath.sqrt(l * (l + 1))


def _real(v, what):
    assert v.im == 0, "%s is not real: %r" % (what, v.im)
    return mpmath.mpf(v.re.numerator) / v.re.denominator


def exact_row(N, H, rates, Ls, s):
    """Row s of Q as {column: mpf} (nonzeros only) and K_s as an mpf."""
    F, cs = _generator(N, s)
    Hs = _sparse(np.asarray(H))
    comm = _add(_mul(Hs, F), _mul(F, Hs), Fr(-1))
    A = {r: {c: v * _I for c, v in row.items()} for r, row in comm.items()}
    for g, L in zip(rates, Ls):
        Lp = _sparse(np.asarray(L))
        Ld = _dagger(Lp)
        LdL = _mul(Ld, Lp)
        D = _add(_mul(_mul(Ld, F), Lp), _add(_mul(LdL, F), _mul(F, LdL)), Fr(-1, 2))
        A = _add(A, D, Fr(float(g)))
    P = N * (N - 1) // 2
    row = {}

    def put(n, val, cn):
        x = _real(val, "Q[%d, %d]" % (s, n))
        if x != 0:
            row[n] = cs * cn * x

    done = set()
    for r, entries in A.items():
        for c in entries:
            if r == c:
                continue
            j, k = min(r, c), max(r, c)
            if (j, k) in done:
                continue
            done.add((j, k))
            ajk = A.get(j, {}).get(k, _C())
            akj = A.get(k, {}).get(j, _C())
            pos = j * N - j * (j + 1) // 2 + k - j - 1
            put(pos, akj + ajk, 1 / mpmath.sqrt(2))                 # Tr(S^(j,k) A)
            put(P + pos, ajk * _I - akj * _I, 1 / mpmath.sqrt(2))  # Tr(J^(j,k) A)
    diag = [A.get(x, {}).get(x, _C()) for x in range(N)]
    pref = _C()
    tr = _C()
    for x in range(N):
        tr = tr + diag[x]
    for l in range(1, N):
        pref = pref + diag[l - 1]
        put(2 * P + l - 1, pref - diag[l].scale(Fr(l)), 1 / mpmath.sqrt(l * (l + 1)))
    K = cs * _real(tr, "Tr A_%d" % s) / N
    return row, K


def row_error(row, exact):
    """Largest |row - exact| over the union of their nonzeros, relative to the
    largest |exact| (normwise per row). `row` is a dense vector or {col: value}."""
    if isinstance(row, np.ndarray):
        row = {int(c): float(row[c]) for c in np.nonzero(row)[0]}
    mx = max((abs(v) for v in exact.values()), default=mpmath.mpf(0))
    err = mpmath.mpf(0)
    for c in set(exact) | set(row):
        err = max(err, abs(mpmath.mpf(row.get(c, 0.0)) - exact.get(c, 0)))
    return float(err / mx) if mx > 0 else float(err)
