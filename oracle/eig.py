"""Oracle: the small dense eigenproblem eig(C) (test infrastructure only).

Sec. 1 (end) defines [zr, zl, D] = eig(C): right eigenvectors, left
eigenvectors and eigenvalues sorted by a user-chosen criterion; Sec. 2 names
"smallest absolute value" as the example criterion.  Here the solver is
LAPACK through scipy.linalg.eig.

Readings (the paper is silent on both):
* sort: |lambda| ascending; values whose moduli agree to 1e-12 relative are
  ordered by imaginary part descending (the + then - order of Table 1).
* normalisation: ||y_i||_2 = 1 and z_i^+ y_i = 1 (so that Z^+ Y = I for
  distinct eigenvalues), one of the normalisations Sec. 2 allows.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.linalg as sla


def sort_order(lam, tie_rel=1e-12):
    """Indices of lam ordered by |lambda| ascending, ties by Im descending."""
    lam = np.asarray(lam)

    def cmp(i, j):
        ai, aj = abs(lam[i]), abs(lam[j])
        if abs(ai - aj) > tie_rel * max(ai, aj, 1e-300):
            return -1 if ai < aj else 1
        if lam[i].imag != lam[j].imag:
            return -1 if lam[i].imag > lam[j].imag else 1
        return -1 if i < j else (1 if i > j else 0)

    return sorted(range(len(lam)), key=functools.cmp_to_key(cmp))


def eig(C):
    """[y, z, lam] = eig(C): right vectors y, left vectors z (z_i^+ C = lam_i z_i^+).

    Columns are normalised to ||y_i|| = 1 and z_i^+ y_i = 1, sorted by
    :func:`sort_order`.
    """
    C = np.asarray(C, dtype=np.complex128)
    lam, zl, yr = sla.eig(C, left=True, right=True)
    idx = sort_order(lam)
    lam, zl, yr = lam[idx], zl[:, idx], yr[:, idx]
    yr = yr / np.linalg.norm(yr, axis=0)
    d = np.einsum("ij,ij->j", zl.conj(), yr)  # z_i^+ y_i
    zl = zl / d.conj()
    return yr, zl, lam
