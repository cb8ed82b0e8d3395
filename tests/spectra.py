"""Comparison of two spectra given as unordered multisets of complex values.

``pair_up`` pairs the entries of ``a`` and ``b`` one to one so that the largest
distance between partners is small (minimum-cost assignment on |a_i - b_j|),
which does not depend on the order either side lists its eigenvalues in.
``condition`` gives each eigenvalue's condition number 1 / |y^H x| (unit left
and right eigenvectors y, x): by first-order perturbation theory a backward
error E moves that eigenvalue by at most kappa ||E||, so two backward-stable
computations on the same M x M matrix agree to about kappa max(M, 16) eps ||Q||_F."""
import numpy as np
import scipy.linalg as sl
from scipy.optimize import linear_sum_assignment


def pair_up(a, b):
    """Index arrays (i, j) pairing a[i] with b[j], and the distances |a_i - b_j|."""
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    assert a.shape == b.shape
    C = np.abs(a[:, None] - b[None, :])
    i, j = linear_sum_assignment(C)
    return i, j, C[i, j]


def condition(Q):
    """Eigenvalues of Q and their condition numbers (LAPACK, left and right vectors)."""
    w, yl, xr = sl.eig(np.asarray(Q, float), left=True, right=True)
    yl = yl / np.linalg.norm(yl, axis=0)
    xr = xr / np.linalg.norm(xr, axis=0)
    return w, 1.0 / np.abs(np.einsum("ij,ij->j", yl.conj(), xr))


def bound(Q, kappa):
    """Per-eigenvalue tolerance kappa_i * max(M, 16) * eps * ||Q||_F: the backward
    error of a Householder reduction and QR iteration grows like M eps ||Q|| with a
    fixed constant of order ten that dominates for the smallest matrices."""
    M = np.asarray(Q).shape[0]
    return kappa * max(M, 16) * np.finfo(float).eps * np.linalg.norm(Q)
