"""CPU FP64 oracle for the iterated stochastic Magnus scheme (arXiv 2207.09776).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path: it builds the
operators with explicit sparse Kronecker products exactly as printed in
Section 2, computes the Magnus logarithm of eq. (MagnusFormulas) with sparse
matrix sums, and applies exp(Omega) with a conservative power series.

Modules
  operators  grids, finite-difference matrices, drift B / noise A, commutators
  integrals  Lebesgue integrals of the Brownian path per Magnus step
  expmv      exp(Omega) u by the scaled power series; dense expm brute force
  magnus     iterated Magnus scheme (Section 2, "Iterated Magnus expansion")
  euler      Euler-Maruyama scheme, eq. (EulerMaruyama)
  exact      closed-form solution of the constant-coefficient Langevin SPDE
  errors     error norms ME, AME, Err with the kappa window, eq. (meanErr)
  step_control  uniform step size from the order-2/order-3 distance
                (Remark "stepSizeControl")

Pins (tests/test_oracle_*.py) tie every function to facts fixed by the paper
or by mathematics, not to this code.  Functions without such a pin say
"parity unpinned" in their docstring.
"""
from . import operators, integrals, expmv, magnus, euler, exact, errors  # noqa: F401
from . import step_control  # noqa: F401
