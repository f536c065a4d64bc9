"""Euler-Maruyama scheme for the discretised SPDE.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. (EulerMaruyama), written in vectorised form with the same B and A as the
Magnus scheme (Section 2, "Euler-Maruyama"):

  U_{k+1} = U_k + (B U_k) dt + (A U_k) Delta W_k,   dt = T / NE,

with Delta W_k the sum of the fine increments inside step k
(integrals.euler_increments).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def euler_path(B: sp.spmatrix, A: sp.spmatrix, u0: np.ndarray, dWE: np.ndarray,
               dt: float) -> np.ndarray:
    """Terminal value of one path; dWE: the NE Euler increments of that path."""
    u = np.array(u0, dtype=np.float64, copy=True)
    for dw in dWE:
        u = u + (B @ u) * dt + (A @ u) * dw
    return u


def euler_paths(B: sp.spmatrix, A: sp.spmatrix, u0: np.ndarray, dWE: np.ndarray,
                dt: float) -> np.ndarray:
    """All paths: dWE [P][NE]; u0 [N] or [P][N] -> [P][N]."""
    dWE = np.atleast_2d(dWE)
    u0 = np.asarray(u0, dtype=np.float64)
    out = np.empty((dWE.shape[0], B.shape[0]))
    for p in range(dWE.shape[0]):
        out[p] = euler_path(B, A, u0 if u0.ndim == 1 else u0[p], dWE[p], dt)
    return out
