"""Step size controlled step by step along each path (Remark
"stepSizeControl"): every coarse step of h = T/K0 is taken with orders 2 and
3 from the current state; if the two differ by more than the tolerance the
step is redone from the same state as `factor` times as many sub-steps, up to
max_level refinements, and the path moves on with the order-3 result.

CPU pins of the oracle (oracle/step_control.adaptive_path):
  * a tolerance no distance exceeds accepts every coarse step at once: the
    result is the uniform order-3 scheme with K0 steps;
  * a tolerance every distance exceeds refines every step to max_level: the
    uniform order-3 scheme with K0 factor^max_level steps;
  * without noise the orders agree to rounding, so nothing is refined;
  * with mixed decisions the result is the order-3 scheme on the partition
    the decisions describe, evaluated in one pass over the weights of its
    sub-steps.
GPU: mg_magnus_adaptive against the oracle, the level of every step equal
and the terminal values within 1e-10, with the tolerance placed away from
every distance the oracle sees.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import integrals, magnus, operators, step_control

N_GRID = 12
T = 1.0


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def problem(n, sigma=0.5, lo=-4.0, hi=4.0):
    coeffs = wl.langevin_constant(1.0, sigma)
    g = operators.Grid(n, n, lo, hi, lo, hi)
    B, A = operators.drift_and_noise(g, coeffs)
    return coeffs, g, operators.magnus_basis(B, A)


def u0_of(n):
    return wl.gaussian_density(n, n, -4, 4, -4, 4, 0.5).reshape(-1)


def test_adaptive_with_loose_tolerance_is_the_uniform_scheme():
    _, g, basis = problem(N_GRID)
    dW = wl.brownian_increments(11, 2, 64, T=T)
    u0 = u0_of(N_GRID)
    uT, lv, gp = step_control.adaptive_paths(basis, dW, T, u0, N_GRID, N_GRID, 4, 2, 2, 1e300)
    assert np.all(lv == 0)
    want = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW, T, 4, 3), u0)
    for p in range(2):
        assert rel(uT[p], want[p]) <= 1e-14


def test_adaptive_with_tight_tolerance_refines_every_step():
    _, g, basis = problem(N_GRID)
    dW = wl.brownian_increments(12, 2, 64, T=T)
    u0 = u0_of(N_GRID)
    uT, lv, gp = step_control.adaptive_paths(basis, dW, T, u0, N_GRID, N_GRID, 4, 2, 2, 1e-300)
    assert np.all(lv == 2)
    want = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW, T, 16, 3), u0)
    for p in range(2):
        assert rel(uT[p], want[p]) <= 1e-14


def test_adaptive_without_noise_refines_nothing():
    """sigma^v = 0: both orders are exp(h B) per step."""
    _, g, basis = problem(N_GRID, sigma=0.0)
    dW = wl.brownian_increments(13, 2, 64, T=T)
    uT, lv, gp = step_control.adaptive_paths(basis, dW, T, u0_of(N_GRID), N_GRID, N_GRID, 4, 2,
                                             3, 1e-10)
    assert np.all(lv == 0) and gp.max() <= 1e-13


def test_adaptive_mixed_decisions_follow_the_partition():
    """Steps of different levels in one path: the result is the order-3
    scheme over the partition (each coarse step cut into factor^level
    sub-steps), evaluated in one pass over the weights of all sub-steps."""
    _, g, basis = problem(N_GRID, sigma=0.9)
    dW = wl.brownian_increments(14, 3, 128, T=T)
    u0 = u0_of(N_GRID)
    K0, f, L = 4, 2, 2
    # distances at level 0 of every coarse step on the uniform trajectory,
    # and a tolerance inside their range
    g0 = step_control.adaptive_paths(basis, dW, T, u0, N_GRID, N_GRID, K0, f, 0, 1e300)[2]
    tol = float(np.median(g0))
    uT, lv, gp = step_control.adaptive_paths(basis, dW, T, u0, N_GRID, N_GRID, K0, f, L, tol)
    assert lv.min() == 0 and lv.max() >= 1, lv
    n = 128 // K0
    for p in range(3):
        rows = [integrals.path_coefficients(dW[p:p + 1, k * n:(k + 1) * n], T / K0, f ** lv[p, k],
                                            3)[0] for k in range(K0)]
        coef = np.concatenate(rows, axis=0)
        assert rel(uT[p], magnus.iterated_magnus(basis, coef, u0)) <= 1e-14
        # every accepted level is within tol unless it is the last level
        assert np.all((gp[p] <= tol) | (lv[p] == L))


def test_adaptive_argument_checks():
    _, g, basis = problem(N_GRID)
    dW = wl.brownian_increments(15, 1, 64, T=T)
    u0 = u0_of(N_GRID)
    with pytest.raises(ValueError):
        step_control.adaptive_path(basis, dW[0], T, u0, N_GRID, N_GRID, 3, 2, 1, 1e-3)
    with pytest.raises(ValueError):
        step_control.adaptive_path(basis, dW[0], T, u0, N_GRID, N_GRID, 4, 2, 5, 1e-3)
