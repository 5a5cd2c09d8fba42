"""Oracle: the small dense eigenproblem eig(C) (test infrastructure only).

Sec. 1 (end) defines [zr, zl, D] = eig(C): right eigenvectors, left
eigenvectors and eigenvalues sorted by a user-chosen criterion; Sec. 2 names
"smallest absolute value" as the example criterion.  Here the solver is
LAPACK through scipy.linalg.eig.

Readings (the paper is silent on both):
* sort: three criteria, chosen by ``which``.  "SM" (the default, the
  criterion Sec. 2 names): |lambda| ascending.  "SR": real part ascending
  (the eigenvalues nearest the left edge of the Wilson-Dirac spectrum).
  "LM": |lambda| descending.  Keys that agree to 1e-12 relative (to the
  larger modulus) are ordered by imaginary part descending (the + then - order
  of Table 1).
* normalisation: ||y_i||_2 = 1 and z_i^+ y_i = 1 (so that Z^+ Y = I for
  distinct eigenvalues), one of the normalisations Sec. 2 allows.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.linalg as sla


SORT_KEYS = ("SM", "SR", "LM")


def sort_order(lam, which="SM", tie_rel=1e-12):
    """Indices of lam ordered by the criterion ``which`` (ascending key), ties by Im descending."""
    lam = np.asarray(lam)
    if which not in SORT_KEYS:
        raise ValueError(f"unknown sort criterion {which!r}")

    def key(i):
        if which == "SM":
            return abs(lam[i])
        if which == "SR":
            return lam[i].real
        return -abs(lam[i])

    def cmp(i, j):
        ki, kj = key(i), key(j)
        if abs(ki - kj) > tie_rel * max(abs(lam[i]), abs(lam[j]), 1e-300):
            return -1 if ki < kj else 1
        if lam[i].imag != lam[j].imag:
            return -1 if lam[i].imag > lam[j].imag else 1
        return -1 if i < j else (1 if i > j else 0)

    return sorted(range(len(lam)), key=functools.cmp_to_key(cmp))


def eig(C, which="SM"):
    """[y, z, lam] = eig(C): right vectors y, left vectors z (z_i^+ C = lam_i z_i^+).

    Columns are normalised to ||y_i|| = 1 and z_i^+ y_i = 1, sorted by
    :func:`sort_order` with the criterion ``which``.
    """
    C = np.asarray(C, dtype=np.complex128)
    lam, zl, yr = sla.eig(C, left=True, right=True)
    idx = sort_order(lam, which)
    lam, zl, yr = lam[idx], zl[:, idx], yr[:, idx]
    yr = yr / np.linalg.norm(yr, axis=0)
    d = np.einsum("ij,ij->j", zl.conj(), yr)  # z_i^+ y_i
    zl = zl / d.conj()
    return yr, zl, lam
