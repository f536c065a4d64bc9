"""The per-row non-zero counts bench.py uses for its algorithmic flop count
equal those of the matrices the oracle assembles (interior rows)."""
import math

import numpy as np
import scipy.sparse as sp

import bench
import workloads as wl
from oracle import magnus, operators


def interior_row_nnz(M, n):
    M = sp.csr_matrix(M)
    i = j = n // 2
    row = M.getrow(i + n * j)
    return int(np.count_nonzero(np.abs(row.data) > 1e-12 * abs(M).max()))


def test_nonzeros_per_interior_row():
    n = 20
    g = operators.Grid(n, n, -5, 5, -5, 5)
    B, A = operators.drift_and_noise(g, wl.langevin_constant(1.0, 0.5))
    basis = operators.magnus_basis(B, A)
    c = np.array([0.1, 0.3, -0.05, 0.02, 0.004, -0.003])
    for order, k in ((1, 2), (2, 4), (3, 6)):
        cc = c.copy()
        cc[k:] = 0.0
        assert interior_row_nnz(magnus.magnus_log(basis, cc), n) == bench.NNZ_ROW[order]
    assert interior_row_nnz(0.01 * B + 0.2 * A, n) * 2 + 1 == bench.EULER_FLOPS_PT
