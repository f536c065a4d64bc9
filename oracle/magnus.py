"""Iterated stochastic Magnus scheme.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 2, "Iterated Magnus expansion": split [0, T] into K sub-intervals of
length h = T/K and evaluate the truncated Magnus expansion on each one, using
the terminal value of one sub-interval as the initial value of the next:

  u_{k+1} = exp(Y^{(order)}_{h; k}) u_k,   k = 0..K-1,

where Y_{h;k} = sum_l c_{k,l} M_l is eq. (MagnusFormulas) on the k-th
sub-interval, M = (B, A, A^2, [B,A], [[B,A],A], [[B,A],B]) and the weights
c_{k,l} come from integrals.path_coefficients.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
import scipy.sparse as sp

from .expmv import expmv_series
from .integrals import path_coefficients


def magnus_log(basis: Sequence[sp.spmatrix], c: np.ndarray) -> sp.csr_matrix:
    """Y = sum_l c_l M_l for one sub-interval (zero weights are skipped)."""
    Y = None
    for cl, Ml in zip(c, basis):
        if cl == 0.0:
            continue
        Y = cl * Ml if Y is None else Y + cl * Ml
    if Y is None:
        Y = sp.csr_matrix(basis[0].shape)
    return sp.csr_matrix(Y)


def iterated_magnus(basis: Sequence[sp.spmatrix], coef: np.ndarray, u0: np.ndarray,
                    terms: int = 20) -> np.ndarray:
    """Terminal value of one path.

    coef: weights [K][6] of that path; u0: initial vector (vec order)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    for k in range(coef.shape[0]):
        u = expmv_series(magnus_log(basis, coef[k]), u, terms=terms)
    return u


def iterated_magnus_paths(basis: Sequence[sp.spmatrix], coef: np.ndarray, u0: np.ndarray,
                          terms: int = 20) -> np.ndarray:
    """All paths: coef [P][K][6], u0 [N] (shared) or [P][N] -> uT [P][N]."""
    P = coef.shape[0]
    u0 = np.asarray(u0, dtype=np.float64)
    out = np.empty((P, basis[0].shape[0]))
    for p in range(P):
        start = u0 if u0.ndim == 1 else u0[p]
        out[p] = iterated_magnus(basis, coef[p], start, terms=terms)
    return out


def piecewise_magnus_paths(pieces, dW: np.ndarray, u0: np.ndarray, order: int,
                           terms: int = 20) -> np.ndarray:
    """Coefficients that are deterministic and piecewise constant in time
    (Remark piecewise): [0, T] is cut where the coefficients change and the
    constant-coefficient scheme runs on each piece, its terminal value being
    the initial value of the next piece.

    pieces: (basis, T_piece, K_piece, Nf_piece) in time order, the basis of
    that piece's coefficients and its length, Magnus steps and fine
    increments; dW [P][sum of Nf_piece], the fine increments of the whole
    interval; u0 [N] (shared) or [P][N]."""
    u = np.asarray(u0, dtype=np.float64)
    start = 0
    for basis, Tp, Kp, Nfp in pieces:
        coef = path_coefficients(dW[:, start:start + Nfp], Tp, Kp, order)
        u = iterated_magnus_paths(basis, coef, u, terms=terms)
        start += Nfp
    if start != dW.shape[1]:
        raise ValueError("the pieces do not cover the fine increments")
    return u
