"""Space discretisation of the general SPDE (Section 2 of the paper).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The SPDE eq. (generalSPDE) is discretised in (x, v) on homogeneous grids
eq. (xGrid)/(vGrid) with central differences and zero boundary values
(Section 2, "Computation of A and B"), then vectorised by column stacking so
that the matrix SDE eq. (SPDEvec) dU = B U dt + A U dW holds with

  B = diag(vec H) + diag(vec F^x)(I_v (x) D^x) + diag(vec F^v)(D^v (x) I_x)
      + 1/2 diag(vec G^xx)(I_v (x) D^xx) + diag(vec G^xv)(D^v (x) D^x)
      + 1/2 diag(vec G^vv)(D^vv (x) I_x)
  A = diag(vec Sigma) + diag(vec Sigma^x)(I_v (x) D^x) + diag(vec Sigma^v)(D^v (x) I_x)

The Magnus logarithm of eq. (MagnusFormulas) uses B, A, A^2 and the
commutators [B,A], [[B,A],A], [[B,A],B] with [X,Y] = XY - YX; these are
products of the truncated N x N matrices (no continuous-symbol shortcut).

Reading of the garbled grid definition: x_i = a_x + i*dx, i = 0..n_x+1,
dx = (b_x - a_x)/(n_x + 1); unknowns are i = 1..n_x, zero at i = 0, n_x + 1.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True)
class Grid:
    """Homogeneous grids of eq. (xGrid) and eq. (vGrid)."""

    nx: int
    nv: int
    ax: float
    bx: float
    av: float
    bv: float

    @property
    def dx(self) -> float:
        return (self.bx - self.ax) / (self.nx + 1)

    @property
    def dv(self) -> float:
        return (self.bv - self.av) / (self.nv + 1)

    def x(self) -> np.ndarray:
        """Interior x nodes x_i = a_x + i dx, i = 1..n_x."""
        return self.ax + self.dx * np.arange(1, self.nx + 1)

    def v(self) -> np.ndarray:
        """Interior v nodes v_j = a_v + j dv, j = 1..n_v."""
        return self.av + self.dv * np.arange(1, self.nv + 1)

    def mesh(self):
        """Coefficient sample points as matrices indexed [i, j] = (x_i, v_j),
        the convention of the matrices Z^w and Sigma^w in Section 2."""
        return np.meshgrid(self.x(), self.v(), indexing="ij")

    @property
    def N(self) -> int:
        return self.nx * self.nv


def vec(Z: np.ndarray) -> np.ndarray:
    """Column stacking of an (n_x x n_v) matrix, Section 2: entry (i, j) goes to
    position i + n_x * j (x fastest)."""
    return np.asarray(Z).reshape(-1, order="F")


def unvec(u: np.ndarray, nx: int, nv: int) -> np.ndarray:
    """Inverse of vec: returns the (n_x x n_v) matrix."""
    return np.asarray(u).reshape((nx, nv), order="F")


def first_difference(n: int, d: float) -> sp.csr_matrix:
    """D = (1/(2d)) tridiag(-1, 0, 1): -1 on the sub-diagonal, +1 on the
    super-diagonal, zero boundary values (Section 2)."""
    off = np.ones(n - 1)
    return (sp.diags([-off, off], [-1, 1], shape=(n, n)) / (2.0 * d)).tocsr()


def second_difference(n: int, d: float) -> sp.csr_matrix:
    """D2 = (1/d^2) tridiag(1, -2, 1), zero boundary values (Section 2)."""
    off = np.ones(n - 1)
    return (sp.diags([off, -2.0 * np.ones(n), off], [-1, 0, 1], shape=(n, n)) / (d * d)).tocsr()


def _diag_of(values: Optional[np.ndarray], N: int) -> sp.csr_matrix:
    if values is None:
        return sp.csr_matrix((N, N))
    return sp.diags(vec(values)).tocsr()


def coefficient_matrices(grid: Grid, coeffs) -> Dict[str, Optional[np.ndarray]]:
    """Sample the coefficient functions on the interior grid as (n_x x n_v)
    matrices Z^w(i, j) = z^w(x_i, v_j) (Section 2).  ``coeffs`` is a
    ``workloads.Coefficients`` (callables of (x, v)) or a dict of grid arrays
    stored [n_v][n_x] (x fastest)."""
    X, V = grid.mesh()
    out = {}
    for name in ("h", "fx", "fv", "gxx", "gxv", "gvv", "sig", "sx", "sv"):
        f = coeffs.get(name) if isinstance(coeffs, dict) else getattr(coeffs, name)
        if f is None:
            out[name] = None
        elif callable(f):
            out[name] = np.broadcast_to(np.asarray(f(X, V), dtype=np.float64), X.shape).copy()
        else:
            out[name] = np.asarray(f, dtype=np.float64).reshape(grid.nv, grid.nx).T.copy()
    return out


def drift_and_noise(grid: Grid, coeffs):
    """The matrices B (drift, dt part) and A (noise, dW part) of eq. (SPDEvec),
    built term by term as in Section 2, "Computation of A and B"."""
    Z = coefficient_matrices(grid, coeffs)
    N = grid.N
    Dx = first_difference(grid.nx, grid.dx)
    Dxx = second_difference(grid.nx, grid.dx)
    Dv = first_difference(grid.nv, grid.dv)
    Dvv = second_difference(grid.nv, grid.dv)
    Ix = sp.identity(grid.nx, format="csr")
    Iv = sp.identity(grid.nv, format="csr")

    B = (_diag_of(Z["h"], N)
         + _diag_of(Z["fx"], N) @ sp.kron(Iv, Dx)
         + _diag_of(Z["fv"], N) @ sp.kron(Dv, Ix)
         + 0.5 * _diag_of(Z["gxx"], N) @ sp.kron(Iv, Dxx)
         + _diag_of(Z["gxv"], N) @ sp.kron(Dv, Dx)
         + 0.5 * _diag_of(Z["gvv"], N) @ sp.kron(Dvv, Ix))
    A = (_diag_of(Z["sig"], N)
         + _diag_of(Z["sx"], N) @ sp.kron(Iv, Dx)
         + _diag_of(Z["sv"], N) @ sp.kron(Dv, Ix))
    return B.tocsr(), A.tocsr()


def commutator(X: sp.spmatrix, Y: sp.spmatrix) -> sp.csr_matrix:
    """[X, Y] = XY - YX (definition after eq. (MagnusFormulas))."""
    return (X @ Y - Y @ X).tocsr()


def magnus_basis(B: sp.spmatrix, A: sp.spmatrix) -> List[sp.csr_matrix]:
    """The six matrices of eq. (MagnusFormulas), in this fixed order:
    B, A, A^2, [B,A], [[B,A],A], [[B,A],B]."""
    BA = commutator(B, A)
    return [B.tocsr(), A.tocsr(), (A @ A).tocsr(), BA, commutator(BA, A), commutator(BA, B)]


def nonzero_diagonals(M: sp.spmatrix, tol: float = 0.0) -> List[int]:
    """Offsets of the diagonals of M holding at least one entry with
    |value| > tol (the count used in Remark 'sparsity', Section 2)."""
    C = sp.coo_matrix(M)
    keep = np.abs(C.data) > tol
    return sorted(set((C.col[keep] - C.row[keep]).tolist()))
