"""Step-size selection by comparing the Magnus orders 2 and 3.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Remark "stepSizeControl": orders 2 and 3 of the iterated scheme stay close for
step sizes inside the convergence range, so their distance tells whether a
step size is small enough: accept it when the two results agree within a
tolerance, else shrink the step by a given factor.  The order-3 logarithm
contains the order-2 one, and with many trajectories the test may run on a
sample of them.

Reading used here (uniform steps for a batch): h = T/K with
K = K0, K0 f, K0 f^2, ... (each K must divide the number of fine increments
and stay <= Kmax).  For a sample of paths the distance at K is

    gap(K) = max_p ||u3_p - u2_p||_F / ||u3_p||_F,

u2, u3 the terminal values of the iterated scheme of orders 2 and 3 with the
same K (the same paths, eq. (MagnusFormulas) for the weights).  The first K
with gap(K) <= tol is selected; if none qualifies the last K tried is
returned, marked as not accepted.

Per-path reading (select_steps_per_path): the same rule applied to each
trajectory on its own, so that every path gets its own step size.

Per-step reading (adaptive_path): the rule applied to each step of a path as
the path is integrated.  The horizon is cut into K0 coarse steps of length
h = T/K0.  From the state u at the start of coarse step k the step is taken
as factor^l uniform sub-steps (l = 0, 1, ..., max_level) of orders 2 and 3
with the same weights; the first l whose distance
||u3 - u2||_F / ||u3||_F is <= tol is accepted (at l = max_level the step
is accepted whatever its distance), the state moves on with u3, and a
rejected level is redone from the same state with the step shortened by the
factor.  A non-finite distance counts as +inf.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

from . import errors, integrals, magnus


def order_gap(basis: Sequence[sp.spmatrix], dW: np.ndarray, T: float, K: int,
              u0: np.ndarray, nx: int, nv: int) -> np.ndarray:
    """||u3 - u2||_F / ||u3||_F per sample path at K uniform steps."""
    c2 = integrals.path_coefficients(dW, T, K, 2)
    c3 = integrals.path_coefficients(dW, T, K, 3)
    u2 = magnus.iterated_magnus_paths(basis, c2, u0)
    u3 = magnus.iterated_magnus_paths(basis, c3, u0)
    return np.array([errors.relative_error(u3[p].reshape(nv, nx), u2[p].reshape(nv, nx))
                     for p in range(u2.shape[0])])


def select_steps(basis: Sequence[sp.spmatrix], dW: np.ndarray, T: float, u0: np.ndarray,
                 nx: int, nv: int, K0: int, factor: int, Kmax: int,
                 tol: float) -> Tuple[int, float, bool, List[Tuple[int, float]]]:
    """(K, gap(K), accepted, [(K, gap), ...] of every K tried)."""
    dW = np.atleast_2d(dW)
    Nf = dW.shape[1]
    history: List[Tuple[int, float]] = []
    K = K0
    while K <= Kmax and Nf % K == 0:
        g = float(np.max(order_gap(basis, dW, T, K, u0, nx, nv)))
        history.append((K, g))
        if g <= tol:
            return K, g, True, history
        K *= factor
    if not history:
        raise ValueError("K0 must divide the fine increments and not exceed Kmax")
    K, g = history[-1]
    return K, g, False, history


def select_steps_per_path(basis: Sequence[sp.spmatrix], dW: np.ndarray, T: float,
                          u0: np.ndarray, nx: int, nv: int, K0: int, factor: int, Kmax: int,
                          tol: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray,
                                              List[List[Tuple[int, float]]]]:
    """Per path p: (K[p], gap[p], accepted[p], history[p]) of select_steps
    run on that path alone."""
    dW = np.atleast_2d(dW)
    K = np.zeros(dW.shape[0], dtype=np.int64)
    gap = np.zeros(dW.shape[0])
    acc = np.zeros(dW.shape[0], dtype=bool)
    hist = []
    for p in range(dW.shape[0]):
        K[p], gap[p], acc[p], h = select_steps(basis, dW[p:p + 1], T, u0, nx, nv, K0, factor,
                                               Kmax, tol)
        hist.append(h)
    return K, gap, acc, hist


def padded_coefficients(dW: np.ndarray, T: float, K: Sequence[int], Kmax: int,
                        order: int) -> np.ndarray:
    """Weights of path p with K[p] uniform steps in rows 0 .. K[p]-1 of
    [P][Kmax][6], zero rows after them (a zero step is the identity)."""
    dW = np.atleast_2d(dW)
    out = np.zeros((dW.shape[0], Kmax, 6))
    for p in range(dW.shape[0]):
        out[p, :K[p]] = integrals.path_coefficients(dW[p:p + 1], T, int(K[p]), order)[0]
    return out


def adaptive_path(basis: Sequence[sp.spmatrix], dW: np.ndarray, T: float, u0: np.ndarray,
                  nx: int, nv: int, K0: int, factor: int, max_level: int,
                  tol: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """One path (fine increments dW [Nf]): (uT, level [K0], gap [K0]) of the
    per-step rule above."""
    dW = np.asarray(dW, dtype=np.float64).reshape(-1)
    Nf = dW.shape[0]
    if K0 < 1 or Nf % K0 != 0 or factor < 2 or max_level < 0:
        raise ValueError("K0 must divide the fine increments, factor >= 2, max_level >= 0")
    n = Nf // K0
    if n % factor ** max_level != 0:
        raise ValueError("the finest sub-steps must divide a coarse step's increments")
    h = T / K0
    u = np.array(u0, dtype=np.float64, copy=True)
    levels = np.zeros(K0, dtype=np.int64)
    gaps = np.zeros(K0)
    for k in range(K0):
        seg = dW[k * n:(k + 1) * n][None, :]
        for lev in range(max_level + 1):
            m = factor ** lev
            u2 = magnus.iterated_magnus(basis, integrals.path_coefficients(seg, h, m, 2)[0], u)
            u3 = magnus.iterated_magnus(basis, integrals.path_coefficients(seg, h, m, 3)[0], u)
            g = errors.relative_error(u3.reshape(nv, nx), u2.reshape(nv, nx))
            if not np.isfinite(g):
                g = np.inf
            if g <= tol or lev == max_level:
                levels[k], gaps[k] = lev, g
                u = u3
                break
    return u, levels, gaps


def adaptive_paths(basis: Sequence[sp.spmatrix], dW: np.ndarray, T: float, u0: np.ndarray,
                   nx: int, nv: int, K0: int, factor: int, max_level: int,
                   tol: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """adaptive_path for every path: dW [P][Nf], u0 [N] (shared) or [P][N]."""
    dW = np.atleast_2d(dW)
    u0 = np.asarray(u0, dtype=np.float64)
    P = dW.shape[0]
    uT = np.empty((P, nx * nv))
    lv = np.zeros((P, K0), dtype=np.int64)
    gp = np.zeros((P, K0))
    for p in range(P):
        uT[p], lv[p], gp[p] = adaptive_path(basis, dW[p], T, u0 if u0.ndim == 1 else u0[p],
                                            nx, nv, K0, factor, max_level, tol)
    return uT, lv, gp
