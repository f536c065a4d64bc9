"""Seeded synthetic inputs for the stochastic Langevin workloads.

This module is shared by the CPU oracle (``oracle/``), the tests and the
benchmark.  It holds NO arithmetic of the numerical method: it only names the
workloads (grid sizes, domains, coefficient choices, path counts, seeds) and
draws their random and initial data.

* Brownian increments: ``dW[p, i] = sqrt(T / Nf) * Z[p, i]`` with ``Z`` drawn by
  ``numpy.random.default_rng(seed).standard_normal((P, Nf))`` (C order, so path
  ``p`` is row ``p`` and does not depend on ``P``).  The paper draws its paths
  with MATLAB's generator (Section 3, "Implementation"); any i.i.d. N(0, delta)
  increments are an equally valid stand-in.
* Initial datum: the normalised Gaussian density N(0, s0^2 I) sampled at the
  interior grid nodes.  The paper uses the unnormalised Gaussian of
  eq. (initialdatum); the workloads below use s0^2 = 0.25 with unit mass.
* Coefficients of the general SPDE, eq. (generalSPDE), as functions of (x, v).

Array layout everywhere: a grid function is stored ``[n_v][n_x]`` in C order,
i.e. x fastest, which is the column stacking ``vec`` of Section 2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Callable, Dict, Optional, Tuple

import numpy as np

CoefFn = Optional[Callable[[np.ndarray, np.ndarray], np.ndarray]]


@dataclass(frozen=True)
class Coefficients:
    """Coefficient functions of eq. (generalSPDE); ``None`` means identically 0."""

    h: CoefFn = None
    fx: CoefFn = None
    fv: CoefFn = None
    gxx: CoefFn = None
    gxv: CoefFn = None
    gvv: CoefFn = None
    sig: CoefFn = None
    sx: CoefFn = None
    sv: CoefFn = None

    NAMES = ("h", "fx", "fv", "gxx", "gxv", "gvv", "sig", "sx", "sv")

    def sample(self, X: np.ndarray, V: np.ndarray) -> Dict[str, Optional[np.ndarray]]:
        out = {}
        for name in self.NAMES:
            f = getattr(self, name)
            out[name] = None if f is None else np.broadcast_to(
                np.asarray(f(X, V), dtype=np.float64), X.shape).copy()
        return out


def langevin_constant(a: float, sigma: float) -> Coefficients:
    """Constant-coefficient stochastic Langevin SPDE, eq. (coeffsLangevinConst):
    f^x = -v, g^vv = a, sigma^v = sigma, every other coefficient 0."""
    return Coefficients(fx=lambda x, v: -v,
                        gvv=lambda x, v: np.full_like(x, a),
                        sv=lambda x, v: np.full_like(x, sigma))


def langevin_variable_sigma_beta() -> Coefficients:
    """Variable-coefficient Langevin workload: diffusion g^vv = s(x,v)^2 with
    s(x,v) = 1 + 0.3 sin(pi x / 5) exp(-v^2 / 8), noise sigma^v = b(v) =
    0.5 + 0.2 tanh(v), transport f^x = -v.  Same structure as
    eq. (coeffsLangevinVar) with other coefficient functions."""
    def s(x, v):
        return 1.0 + 0.3 * np.sin(np.pi * x / 5.0) * np.exp(-v * v / 8.0)
    return Coefficients(fx=lambda x, v: -v,
                        gvv=lambda x, v: s(x, v) ** 2,
                        sv=lambda x, v: 0.5 + 0.2 * np.tanh(v) + 0.0 * x)


def langevin_paper_variable(a: float, sigma: float) -> Coefficients:
    """The paper's own variable coefficients, eq. (coeffsLangevinVar)."""
    return Coefficients(fx=lambda x, v: -v,
                        gvv=lambda x, v: a * (1.0 + 1.0 / (x * x + 1.0)) + 0.0 * v,
                        sv=lambda x, v: sigma * np.sqrt(1.0 + 1.0 / (x * x + 1.0)) + 0.0 * v)


@dataclass(frozen=True)
class Workload:
    """One batch of the iterated-Magnus hot path."""

    name: str
    n: int                      # n_x = n_v
    lo: float                   # domain [lo, hi]^2
    hi: float
    paths: int
    K: int                      # Magnus steps
    order: int                  # Magnus order 1..3
    Nf: int                     # fine Brownian increments per path
    seed: int
    T: float = 1.0
    s0sq: float = 0.25          # variance of the Gaussian initial density
    a: float = 1.0              # g^vv (constant case)
    sigma: float = 0.5          # sigma^v (constant case)
    euler_steps: int = 0        # Euler-Maruyama steps of the baseline (0: none)
    ref_paths: int = 0          # leading paths given the fine Euler reference (0: all)
    euler_time_paths: int = 0   # paths the Euler baseline is timed on (0: all)
    precision: str = "fp64"     # "fp64" or "fp32c"
    variable: bool = False      # variable-coefficient workload
    extra: Tuple = field(default_factory=tuple)

    def coefficients(self) -> Coefficients:
        if self.variable:
            return langevin_variable_sigma_beta()
        return langevin_constant(self.a, self.sigma)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The workloads.  Names say what they are.  Constant case: g^vv = a = 1 (unit
# diffusion in v), sigma^v = 0.5 (noise through d/dv), so a - sigma^2 = 0.75 > 0
# and the explicit solution of Section 3.1 applies.
WORKLOADS: Dict[str, Workload] = {
    "const-32-p1-m2-k8": Workload("const-32-p1-m2-k8", 32, -5.0, 5.0, 1, 8, 2, 2 ** 12, 0,
                                   euler_steps=2 ** 12),
    "const-128-p1024-m2-k16": Workload("const-128-p1024-m2-k16", 128, -6.0, 6.0, 1024, 16, 2,
                                        2 ** 14, 2, euler_steps=2 ** 14),
    # The largest single-GPU constant-coefficient batch (the cooperative
    # kernel: several workgroups per path), run in FP64 and in the FP32 form.
    # The Euler baseline of this workload is timed on 64 paths (one per group
    # of workgroups the GPU holds at once) and scaled to paths/s.
    "const-256-p4096-m3-k32": Workload("const-256-p4096-m3-k32", 256, -5.0, 5.0, 4096,
                                        32, 3, 2 ** 14, 3, euler_time_paths=64),
    # The variable-coefficient workload at 512^2.  K = 256: the order-2
    # logarithm (its c3 [B,A] term) has an unbounded exponential at K = 64 on
    # this grid, as in the constant case, and at K = 128 two of the first 16
    # paths still end far from the reference (errors 0.75 and 1.7e-2); from
    # K = 256 on every path sits at the level of the fine Euler reference
    # itself.  That reference (2^18 steps) is formed on the first 16 paths, and
    # the Euler baseline is timed on 16 paths (one path per group of
    # workgroups that the GPU holds at once) and scaled to paths/s.
    "var-512-p512-m2-k256": Workload("var-512-p512-m2-k256", 512, -5.0, 5.0, 512, 256, 2, 2 ** 18,
                                      4, variable=True, euler_steps=2 ** 14, ref_paths=16,
                                      euler_time_paths=16),
    # the variable-coefficient workload on a 128^2 grid (the x-dependent
    # operator runs on one workgroup per path up to 128 points per axis)
    "var-128-p512-m2-k64": Workload("var-128-p512-m2-k64", 128, -5.0, 5.0, 512, 64, 2, 2 ** 18, 4,
                                     variable=True, euler_steps=2 ** 14),
    # groups (n, paths, K, seed).  The order-2 logarithm contains c3 [B,A],
    # whose norm grows like 1/(dv^2 dx), so its exponential stays bounded only
    # for steps h of order dx^2: the 1024^2 group takes K = 512 (K = 64 and 256
    # blow up, in FP64 as in FP32), the others keep the steps of their grids.
    "mixed-64-256-1024-m2-fp32c": Workload("mixed-64-256-1024-m2-fp32c", 64, -5.0, 5.0, 2048, 16, 2,
                                            2 ** 14, 5, precision="fp32c",
                                            extra=((64, 2048, 16, 5), (256, 512, 32, 6),
                                                   (1024, 64, 512, 7))),
}


def grid_nodes(n: int, lo: float, hi: float) -> np.ndarray:
    """Interior nodes lo + i*(hi-lo)/(n+1), i = 1..n (needed to sample the
    initial datum and the coefficients)."""
    d = (hi - lo) / (n + 1)
    return lo + d * np.arange(1, n + 1, dtype=np.float64)


def mesh(n_x: int, n_v: int, ax: float, bx: float, av: float, bv: float):
    """(X, V) sample points, each shaped [n_v][n_x] (x fastest)."""
    x = grid_nodes(n_x, ax, bx)
    v = grid_nodes(n_v, av, bv)
    V, X = np.meshgrid(v, x, indexing="ij")
    return X, V


def gaussian_density(n_x: int, n_v: int, ax: float, bx: float, av: float, bv: float,
                     s0sq: float) -> np.ndarray:
    """N(0, s0sq * I) density at the interior nodes, shape [n_v][n_x]."""
    X, V = mesh(n_x, n_v, ax, bx, av, bv)
    return np.exp(-(X * X + V * V) / (2.0 * s0sq)) / (2.0 * math.pi * s0sq)


def brownian_increments(seed: int, paths: int, Nf: int, T: float = 1.0,
                        first: int = 0, count: Optional[int] = None) -> np.ndarray:
    """Fine Brownian increments dW[p, i], shape [paths][Nf], float64.

    ``first``/``count`` select a sub-range of paths without changing the values
    of the selected rows (rows are drawn in order from one stream)."""
    if count is None:
        count = paths - first
    rng = np.random.default_rng(seed)
    scale = math.sqrt(T / Nf)
    out = np.empty((count, Nf), dtype=np.float64)
    # draw row by row so that a sub-range equals the same rows of the full draw
    if first > 0:
        rng.standard_normal((first, Nf))
    rng.standard_normal(out=out)
    out *= scale
    return out


def sample_coefficients(coeffs: Coefficients, n_x: int, n_v: int, ax: float, bx: float,
                        av: float, bv: float) -> Dict[str, Optional[np.ndarray]]:
    """Coefficient grids, each [n_v][n_x] float64 or None."""
    X, V = mesh(n_x, n_v, ax, bx, av, bv)
    return coeffs.sample(X, V)
