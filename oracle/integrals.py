"""Lebesgue integrals of the Brownian path and the Magnus coefficients.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. (MagnusFormulas) needs, on each Magnus sub-interval, the increment W_t
and the Lebesgue integrals int W ds, int W^2 ds and int s W ds; Section 3
("Implementation") computes them for all paths with simple sums on a fine
grid of step delta.  Readings used here:

* Each sub-interval (t_k, t_k + h] restarts the path: the local path is
  W~_r = W_{t_k + r} - W_{t_k}, r in [0, h], because the formulas are stated
  for an interval starting at 0 with W_0 = 0 (Section 2, "Iterated Magnus
  expansion").
* "Simple Riemann sums" are read as the exact integrals of the piecewise
  linear interpolant of the fine path (trapezoid family); these make
  int_0^T W ds equal to the sum of the per-step pieces exactly.
"""
from __future__ import annotations

import numpy as np


def local_integrals(dW_seg: np.ndarray, h: float):
    """Increment and integrals of one sub-interval of length h.

    dW_seg: the n fine increments of the sub-interval (delta = h/n).
    Returns (DW, I1, I2, J) with I1 = int W~, I2 = int W~^2, J = int r W~ (dr),
    each the exact integral of the piecewise-linear path through the nodes."""
    dW_seg = np.asarray(dW_seg, dtype=np.float64)
    n = dW_seg.shape[-1]
    delta = h / n
    W = np.concatenate([np.zeros(dW_seg.shape[:-1] + (1,)), np.cumsum(dW_seg, axis=-1)], axis=-1)
    r = delta * np.arange(n + 1)
    Wl, Wr = W[..., :-1], W[..., 1:]
    rl, rr = r[:-1], r[1:]
    DW = W[..., -1]
    I1 = np.sum(delta * (Wl + Wr) / 2.0, axis=-1)
    I2 = np.sum(delta * (Wl * Wl + Wl * Wr + Wr * Wr) / 3.0, axis=-1)
    J = np.sum(delta * (rl * (2.0 * Wl + Wr) + rr * (Wl + 2.0 * Wr)) / 6.0, axis=-1)
    return DW, I1, I2, J


def magnus_coefficients(order: int, h: float, DW, I1, I2, J) -> np.ndarray:
    """Scalar weights of the six matrices B, A, A^2, [B,A], [[B,A],A], [[B,A],B]
    in Y_h of eq. (MagnusFormulas) with t = h:

      order 1: Y = B h + A W_h
      order 2: + (-h/2) A^2 + (int W - h W_h / 2) [B,A]
      order 3: + (1/2 int W^2 - 1/2 W_h int W + h W_h^2 / 12) [[B,A],A]
               + (int s W - h/2 int W - h^2 W_h / 12) [[B,A],B]
    """
    DW = np.asarray(DW, dtype=np.float64)
    c = np.zeros(DW.shape + (6,))
    c[..., 0] = h
    c[..., 1] = DW
    if order >= 2:
        c[..., 2] = -0.5 * h
        c[..., 3] = I1 - 0.5 * h * DW
    if order >= 3:
        c[..., 4] = 0.5 * I2 - 0.5 * DW * I1 + h * DW * DW / 12.0
        c[..., 5] = J - 0.5 * h * I1 - h * h * DW / 12.0
    return c


def path_coefficients(dW: np.ndarray, T: float, K: int, order: int) -> np.ndarray:
    """Magnus weights for every path and step: shape [P][K][6].

    dW: fine increments [P][Nf]; requires Nf % K == 0."""
    dW = np.atleast_2d(np.asarray(dW, dtype=np.float64))
    P, Nf = dW.shape
    if Nf % K != 0:
        raise ValueError("the number of fine increments must be a multiple of K")
    h = T / K
    seg = dW.reshape(P, K, Nf // K)
    DW, I1, I2, J = local_integrals(seg, h)
    return magnus_coefficients(order, h, DW, I1, I2, J)


def path_statistics(dW: np.ndarray, T: float) -> np.ndarray:
    """(W_T, int_0^T W ds) per path, shape [P][2]; the integral is exact for
    the piecewise-linear path (same reading as local_integrals)."""
    dW = np.atleast_2d(np.asarray(dW, dtype=np.float64))
    P, Nf = dW.shape
    delta = T / Nf
    W = np.concatenate([np.zeros((P, 1)), np.cumsum(dW, axis=1)], axis=1)
    out = np.empty((P, 2))
    out[:, 0] = W[:, -1]
    out[:, 1] = np.sum(delta * (W[:, :-1] + W[:, 1:]) / 2.0, axis=1)
    return out


def euler_increments(dW: np.ndarray, NE: int) -> np.ndarray:
    """Increments Delta W_{t_k} of eq. (EulerMaruyama) on NE equal steps:
    sums of Nf/NE consecutive fine increments (requires Nf % NE == 0)."""
    dW = np.atleast_2d(np.asarray(dW, dtype=np.float64))
    P, Nf = dW.shape
    if Nf % NE != 0:
        raise ValueError("the number of fine increments must be a multiple of the Euler steps")
    return dW.reshape(P, NE, Nf // NE).sum(axis=2)
