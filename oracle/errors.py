"""Error norms of Section 3 ("Error and notations"), eq. (meanErr).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For kappa = 0, 1, ... only the central 2^-kappa part of the d x d solution
matrix is compared.  The printed index set I^kappa has floor(d/2^kappa)+1
entries for a floor(d/2^kappa)-wide matrix; the reading used here keeps the
stated width: 0-based indices i0, ..., i0 + floor(d/2^kappa) - 1 with
i0 = floor(d/2 - d/2^(kappa+1)).  kappa = 0 is the whole grid.
"""
from __future__ import annotations

import math

import numpy as np


def window(d: int, kappa: int) -> np.ndarray:
    """0-based indices of I^kappa (see module doc)."""
    w = d // (2 ** kappa)
    i0 = int(math.floor(d / 2.0 - d / 2.0 ** (kappa + 1)))
    return np.arange(i0, i0 + w)


def central_part(U: np.ndarray, kappa: int) -> np.ndarray:
    """U^{d,kappa}: U is a grid function [n_v][n_x] (or a vec-order vector of a
    square grid); returns the central window [w][w]."""
    U = np.asarray(U)
    if U.ndim == 1:
        d = int(round(math.sqrt(U.size)))
        U = U.reshape(d, d)
    wv = window(U.shape[0], kappa)
    wx = window(U.shape[1], kappa)
    return U[np.ix_(wv, wx)]


def relative_error(ref: np.ndarray, app: np.ndarray, kappa: int = 0) -> float:
    """||U_ref - U_app||_F / ||U_ref||_F on the kappa window, one path."""
    R = central_part(ref, kappa)
    A = central_part(app, kappa)
    return float(np.linalg.norm(R - A) / np.linalg.norm(R))


def err(refs, apps, kappa: int = 0) -> float:
    """Err_t^{d,kappa}: mean over paths of the relative Frobenius error."""
    return float(np.mean([relative_error(r, a, kappa) for r, a in zip(refs, apps)]))


def mean_abs_error(refs, apps, kappa: int = 0) -> np.ndarray:
    """ME_t^{d,kappa}: pointwise mean absolute error over paths (a matrix)."""
    return np.mean([np.abs(central_part(r, kappa) - central_part(a, kappa))
                    for r, a in zip(refs, apps)], axis=0)


def average_mean_error(refs, apps, kappa: int = 0) -> float:
    """AME_t^{d,kappa}: average of ME over the window."""
    return float(np.mean(mean_abs_error(refs, apps, kappa)))
