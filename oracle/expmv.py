"""exp(Omega) u for the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper applies the matrix exponential to a vector without forming it
(Section 2, "Space discretization and Magnus expansion"; Section 3,
"Implementation").  The result exp(Omega) u is unique, so the oracle simply
evaluates the definition, the exponential power series, made safe by two
exact identities:

  exp(Omega) = e^mu exp(Omega - mu I)           (mu = trace(Omega)/N commutes)
  exp(M)     = (exp(M / s))^s                   (s a positive integer)

With s = ceil(||Omega - mu I||_1) every factor has 1-norm argument <= 1, and
the series is cut after the degree-``terms`` term.  The remainder is then at
most 2/(terms+1)! relative to ||u||_1 (about 4e-20 for terms = 20), far below
FP64 rounding, independently of any (m, s) choice made by the GPU path.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
import scipy.sparse as sp


def norm1(M) -> float:
    """Matrix 1-norm: maximum absolute column sum."""
    if sp.issparse(M):
        return float(abs(M).sum(axis=0).max()) if M.shape[0] else 0.0
    return float(np.abs(M).sum(axis=0).max())


def expmv_series(Omega, u: np.ndarray, terms: int = 20, shift: bool = True) -> np.ndarray:
    """exp(Omega) @ u by the scaled, shifted power series (see module doc)."""
    Omega = sp.csr_matrix(Omega)
    N = Omega.shape[0]
    mu = Omega.diagonal().sum() / N if shift else 0.0
    M = (Omega - mu * sp.identity(N, format="csr")).tocsr()
    s = max(1, int(math.ceil(norm1(M))))
    u = np.array(u, dtype=np.float64, copy=True)
    for _ in range(s):
        term = u.copy()
        F = u.copy()
        for j in range(1, terms + 1):
            term = (M @ term) / (j * s)
            F += term
        u = math.exp(mu / s) * F
    return u


def expmv_dense(Omega, u: np.ndarray) -> np.ndarray:
    """Brute force: the full matrix exponential (scipy.linalg.expm, a
    Pade scaling-and-squaring method) times u.  For small N only."""
    M = Omega.toarray() if sp.issparse(Omega) else np.asarray(Omega)
    return scipy.linalg.expm(M) @ np.asarray(u, dtype=np.float64)
