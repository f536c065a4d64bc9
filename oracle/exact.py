"""Closed-form solution of the constant-coefficient stochastic Langevin SPDE.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 3.1 gives, for f^x = -v, g^vv = a, sigma^v = sigma with
0 < sigma < sqrt(a) (eq. (coeffsLangevinConst)), the fundamental solution

  Gamma(t, z; 0, zeta) = Gamma_0(t, z - m_t(zeta)),
  m_t(xi, eta) = (xi + t eta - sigma int_0^t W, eta - sigma W_t),

with Gamma_0 the Gaussian kernel of the Kolmogorov operator with diffusion
c = a - sigma^2, and u_t(z) = int Gamma(t, z; 0, zeta) phi(zeta) d zeta.  The
paper leaves the final formula out.  For a Gaussian initial density
phi = N(0, s0^2 I) the integral is the density of y = M zeta + noise with
M = [[1, t], [0, 1]], i.e. a Gaussian evaluated at

  y = (x + sigma int_0^t W, v + sigma W_t),
  Sigma_t = s0^2 M M^T + c [[t^3/3, t^2/2], [t^2/2, t]],
  u_t(x, v) = exp(-y^T Sigma_t^{-1} y / 2) / (2 pi sqrt(det Sigma_t)).

(The paper's unnormalised phi = exp(-(xi^2+eta^2)/2) is s0 = 1 times 2 pi.)
gamma0 below is the printed kernel itself, used by the pins to check the
closed form by quadrature.
"""
from __future__ import annotations

import math

import numpy as np


def gamma0(t: float, x, v, a: float, sigma: float):
    """Gamma_0(t, (x, v)) exactly as printed in Section 3.1."""
    c = a - sigma * sigma
    return (math.sqrt(3.0) / (math.pi * t * t * c)
            * np.exp(-2.0 / c * (v * v / t - 3.0 * v * x / (t * t) + 3.0 * x * x / t ** 3)))


def mean_shift(t: float, xi, eta, sigma: float, W_t: float, I_t: float):
    """m_t(zeta) of Section 3.1 (I_t = int_0^t W ds)."""
    return xi + t * eta - sigma * I_t, eta - sigma * W_t


def covariance(t: float, a: float, sigma: float, s0sq: float) -> np.ndarray:
    """Sigma_t of the module docstring."""
    c = a - sigma * sigma
    return np.array([[s0sq * (1.0 + t * t) + c * t ** 3 / 3.0, s0sq * t + c * t * t / 2.0],
                     [s0sq * t + c * t * t / 2.0, s0sq + c * t]])


def solution(t: float, x, v, a: float, sigma: float, s0sq: float, W_t: float, I_t: float):
    """u_t(x, v) for the normalised Gaussian initial density N(0, s0sq I)."""
    S = covariance(t, a, sigma, s0sq)
    det = S[0, 0] * S[1, 1] - S[0, 1] * S[1, 0]
    y1 = np.asarray(x) + sigma * I_t
    y2 = np.asarray(v) + sigma * W_t
    q = (S[1, 1] * y1 * y1 - 2.0 * S[0, 1] * y1 * y2 + S[0, 0] * y2 * y2) / det
    return np.exp(-0.5 * q) / (2.0 * math.pi * math.sqrt(det))


def solution_on_grid(grid, t: float, a: float, sigma: float, s0sq: float,
                     W_t: float, I_t: float) -> np.ndarray:
    """Closed form at the interior nodes, as a vector in vec order (x fastest)."""
    X, V = grid.mesh()          # [i, j] = (x_i, v_j)
    U = solution(t, X, V, a, sigma, s0sq, W_t, I_t)
    return U.reshape(-1, order="F")
