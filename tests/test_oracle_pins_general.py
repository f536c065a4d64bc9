"""Pins of the oracle's general-coefficient branches (Section 2, "Computation
of A and B"; eq. (generalSPDE) -> eq. (SPDEvec)).

Every coefficient of eq. (generalSPDE) enters B or A as diag(vec Z) times a
Kronecker product of 1-D difference matrices.  Each test below switches on a
subset of the coefficients for which the space-discrete problem splits into
independent 1-D problems (one per x column or one per v row), or diagonalises
through the eigenvectors of the 1-D factors, and compares the oracle's whole
path (drift_and_noise -> magnus_basis -> iterated_magnus) with that
reduction.  The reductions use 1-D difference matrices written out here with
NumPy and dense scipy.linalg.expm / numpy.linalg.eig, never the oracle's 2-D
sparse assembly.  The grids are rectangular (nx != nv) and the coefficients
are not symmetric in (x, v), so a transposed coefficient grid, a swapped
Kronecker order or a wrong factor (1/2 on the second derivatives) fails.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import integrals, magnus, operators

NX, NV = 7, 9
AX, BX, AV, BV = -2.0, 3.0, -4.0, 2.5
T = 0.3


def _grid():
    return operators.Grid(NX, NV, AX, BX, AV, BV)


def _nodes():
    dx = (BX - AX) / (NX + 1)
    dv = (BV - AV) / (NV + 1)
    return AX + dx * np.arange(1, NX + 1), AV + dv * np.arange(1, NV + 1), dx, dv


def _d1(n, d):
    """(1/(2d)) tridiag(-1, 0, 1), dense, zero boundary values."""
    D = np.zeros((n, n))
    for i in range(n):
        if i > 0:
            D[i, i - 1] = -1.0
        if i + 1 < n:
            D[i, i + 1] = 1.0
    return D / (2.0 * d)


def _d2(n, d):
    """(1/d^2) tridiag(1, -2, 1), dense, zero boundary values."""
    D = -2.0 * np.eye(n)
    for i in range(n - 1):
        D[i, i + 1] = D[i + 1, i] = 1.0
    return D / (d * d)


def _grid_array(f):
    """Coefficient grid [nv][nx] (x fastest), the layout the library takes."""
    x, v, _, _ = _nodes()
    V, X = np.meshgrid(v, x, indexing="ij")
    return np.asarray(f(X, V), dtype=np.float64)


def _u0():
    """A smooth non-symmetric initial field [nv][nx] that is O(1) at the edges."""
    x, v, _, _ = _nodes()
    V, X = np.meshgrid(v, x, indexing="ij")
    return 1.0 + 0.4 * np.sin(1.3 * X + 0.2) * np.cos(0.7 * V - 0.5) + 0.1 * X * V


def _oracle_path(coeffs, order, K=3, Nf=12, seed=5):
    """Oracle terminal value [nv][nx] and the path's (W_T, dW)."""
    g = _grid()
    B, A = operators.drift_and_noise(g, coeffs)
    basis = operators.magnus_basis(B, A)
    dW = np.random.default_rng(seed).standard_normal((1, Nf)) * math.sqrt(T / Nf)
    coef = integrals.path_coefficients(dW, T, K, order)
    uT = magnus.iterated_magnus(basis, coef[0], _u0().reshape(-1))
    return uT.reshape(NV, NX), float(dW.sum())


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("order", [1, 2, 3])
def test_v_terms_split_into_columns(order):
    """A = 0 and B = diag(vec H) + diag(vec F^v)(D^v (x) I) + 1/2 diag(vec G^vv)(D^vv (x) I)
    with H, F^v, G^vv depending on x and v: each x column i evolves alone by
    exp(T (diag h_i + diag f_i D^v + 1/2 diag g_i D^vv)) (Remark
    'determLangevin': without noise every order gives exp(T B)).  Pins the
    x-dependent diag(vec Z) of the H, f^v and g^vv branches."""
    h = lambda x, v: 0.3 * np.sin(x) - 0.2 * v
    fv = lambda x, v: 0.5 + 0.3 * x - 0.1 * v * v
    gvv = lambda x, v: 1.0 + 0.4 * np.cos(x) * np.exp(-0.1 * v * v)
    coeffs = {"h": _grid_array(h), "fv": _grid_array(fv), "gvv": _grid_array(gvv)}
    got, _ = _oracle_path(coeffs, order)
    x, v, dx, dv = _nodes()
    u0 = _u0()
    want = np.empty_like(u0)
    for i in range(NX):
        L = (np.diag(h(x[i], v)) + np.diag(fv(x[i], v)) @ _d1(NV, dv)
             + 0.5 * np.diag(gvv(x[i], v)) @ _d2(NV, dv))
        want[:, i] = scipy.linalg.expm(T * L) @ u0[:, i]
    assert _rel(got, want) <= 1e-12


@pytest.mark.parametrize("order", [1, 2])
def test_x_terms_split_into_rows(order):
    """A = 0 and B = diag(vec F^x)(I (x) D^x) + 1/2 diag(vec G^xx)(I (x) D^xx):
    each v row j evolves alone by exp(T (diag f_j D^x + 1/2 diag g_j D^xx)).
    Pins the f^x and g^xx branches and the x-fast column stacking."""
    fx = lambda x, v: -v + 0.2 * x
    gxx = lambda x, v: 0.8 + 0.3 * np.sin(v) + 0.1 * x
    coeffs = {"fx": _grid_array(fx), "gxx": _grid_array(gxx)}
    got, _ = _oracle_path(coeffs, order)
    x, v, dx, dv = _nodes()
    u0 = _u0()
    want = np.empty_like(u0)
    for j in range(NV):
        L = np.diag(fx(x, v[j])) @ _d1(NX, dx) + 0.5 * np.diag(gxx(x, v[j])) @ _d2(NX, dx)
        want[j, :] = scipy.linalg.expm(T * L) @ u0[j, :]
    assert _rel(got, want) <= 1e-12


def test_mixed_derivative_by_eigenvectors():
    """A = 0 and B = diag(vec G^xv)(D^v (x) D^x) with G^xv = b(v) a(x):
    B = (diag b D^v) (x) (diag a D^x) = Bv (x) Bx, so with Bv = Qv Lv Qv^-1 and
    Bx = Qx Lx Qx^-1 (1-D eigendecompositions) exp(T B) acts on the field
    U [nv][nx] as Qv (E o (Qv^-1 U Qx^-T)) Qx^T with E_jk = exp(T lv_j lx_k).
    Pins the g^xv branch: its Kronecker order and its factor (1, not 1/2)."""
    a = lambda x: 1.0 + 0.3 * x
    b = lambda v: 0.7 - 0.2 * v
    coeffs = {"gxv": _grid_array(lambda X, V: a(X) * b(V))}
    got, _ = _oracle_path(coeffs, 2)
    x, v, dx, dv = _nodes()
    Bx = np.diag(a(x)) @ _d1(NX, dx)
    Bv = np.diag(b(v)) @ _d1(NV, dv)
    lx, Qx = np.linalg.eig(Bx)
    lv, Qv = np.linalg.eig(Bv)
    U = _u0().astype(complex)
    C = np.linalg.solve(Qv, U) @ np.linalg.inv(Qx).T
    C *= np.exp(T * np.outer(lv, lx))
    want = (Qv @ C @ Qx.T).real
    assert _rel(got, want) <= 1e-10


@pytest.mark.parametrize("order", [1, 2, 3])
def test_zeroth_order_noise_is_pointwise(order):
    """B = 0 and A = diag(vec Sigma) with Sigma depending on x and v: every
    matrix of the basis is diagonal and commutes, so the scheme gives exactly
    u_T = exp(Sigma W_T - Sigma^2 T / 2) u_0 pointwise for orders 2 and 3 (the
    Ito correction c2 A^2) and exp(Sigma W_T) u_0 for order 1 (no correction).
    Pins the sigma branch, its vec order, and the Ito term."""
    sig = lambda x, v: 0.4 + 0.3 * np.sin(x + 0.5 * v)
    got, WT = _oracle_path({"sig": _grid_array(sig)}, order)
    S = _grid_array(sig)
    want = np.exp(S * WT - (0.0 if order == 1 else 0.5 * S * S * T)) * _u0()
    assert _rel(got, want) <= 1e-12


@pytest.mark.parametrize("order", [1, 2, 3])
def test_x_derivative_noise_splits_into_rows(order):
    """B = 0 and A = diag(vec Sigma^x)(I (x) D^x): the basis matrices are
    A and A^2 (commutators with B vanish), which commute, so row j evolves by
    exp(W_T A_j - (T/2) A_j^2) (orders 2, 3) or exp(W_T A_j) (order 1) with
    A_j = diag(sigma^x(., v_j)) D^x.  Pins the sigma^x branch."""
    sx = lambda x, v: 0.5 + 0.2 * v + 0.1 * np.cos(x)
    got, WT = _oracle_path({"sx": _grid_array(sx)}, order)
    x, v, dx, dv = _nodes()
    u0 = _u0()
    want = np.empty_like(u0)
    for j in range(NV):
        Aj = np.diag(sx(x, v[j])) @ _d1(NX, dx)
        L = WT * Aj - (0.0 if order == 1 else 0.5 * T * Aj @ Aj)
        want[j, :] = scipy.linalg.expm(L) @ u0[j, :]
    assert _rel(got, want) <= 1e-12


@pytest.mark.parametrize("order", [2, 3])
def test_v_derivative_noise_with_x_dependence_splits_into_columns(order):
    """B = 0 and A = diag(vec Sigma^v)(D^v (x) I) with sigma^v depending on x
    and v (the paper's variable noise depends on x): column i evolves by
    exp(W_T A_i - (T/2) A_i^2), A_i = diag(sigma^v(x_i, .)) D^v."""
    sv = lambda x, v: 0.5 * np.sqrt(1.0 + 1.0 / (x * x + 1.0)) + 0.05 * v
    got, WT = _oracle_path({"sv": _grid_array(sv)}, order)
    x, v, dx, dv = _nodes()
    u0 = _u0()
    want = np.empty_like(u0)
    for i in range(NX):
        Ai = np.diag(sv(x[i], v)) @ _d1(NV, dv)
        want[:, i] = scipy.linalg.expm(WT * Ai - 0.5 * T * Ai @ Ai) @ u0[:, i]
    assert _rel(got, want) <= 1e-12


@pytest.mark.parametrize("order", [1, 2, 3])
def test_x_dependent_x_terms_with_v_noise_factor_exactly(order):
    """B = I (x) L_x with L_x = diag(h(x)) + diag(f^x(x)) D^x + 1/2 diag(g^xx(x)) D^xx
    and A = A_v (x) I with A_v = diag(sigma^v(v)) D^v: x-dependent coefficients
    of x derivatives and noise through d/dv in one problem.  B and A act on
    different factors, so they commute, every commutator of the Magnus basis
    vanishes and the step exponentials multiply to one: orders 2 and 3 give
    exp(T B + W_T A - (T/2) A^2) = exp(W_T A_v - (T/2) A_v^2) (x) exp(T L_x),
    order 1 (exponent B h + A W_h per step, no A^2 term) exp(W_T A_v) (x)
    exp(T L_x); on the [nv][nx] grid (x fastest) U_T = E_v U_0 E_x^T.
    Pins the H, f^x and g^xx branches with x dependence
    together with the sigma^v branch: their Kronecker slots, the x-fast
    stacking of x-dependent grids, and that no cross terms enter the basis."""
    h = lambda x, v: 0.2 * np.sin(x) + 0 * v
    fx = lambda x, v: 0.5 + 0.3 * np.cos(x) + 0 * v
    gxx = lambda x, v: 0.8 + 0.2 * np.sin(1.7 * x) + 0 * v
    sv = lambda x, v: 0.4 + 0.1 * v + 0 * x
    coeffs = {"h": _grid_array(h), "fx": _grid_array(fx), "gxx": _grid_array(gxx),
              "sv": _grid_array(sv)}
    got, WT = _oracle_path(coeffs, order)
    x, v, dx, dv = _nodes()
    Lx = (np.diag(h(x, 0.0)) + np.diag(fx(x, 0.0)) @ _d1(NX, dx)
          + 0.5 * np.diag(gxx(x, 0.0)) @ _d2(NX, dx))
    Av = np.diag(sv(0.0, v)) @ _d1(NV, dv)
    Ev = scipy.linalg.expm(WT * Av - (0.5 * T * Av @ Av if order >= 2 else 0.0))
    Ex = scipy.linalg.expm(T * Lx)
    want = Ev @ _u0() @ Ex.T
    assert _rel(got, want) <= 1e-12


def test_constant_potential_is_a_scalar_factor():
    """H = h constant commutes with every matrix: the Langevin path with H
    added equals e^{hT} times the path without it (catches a sign or a factor
    on the H term and its entry into the commutators)."""
    g = _grid()
    base = {"fx": _grid_array(lambda x, v: -v), "gvv": _grid_array(lambda x, v: 1.0 + 0 * x),
            "sv": _grid_array(lambda x, v: 0.5 + 0 * x)}
    with_h = dict(base, h=_grid_array(lambda x, v: -0.7 + 0 * x))
    u_base, _ = _oracle_path(base, 3)
    u_h, _ = _oracle_path(with_h, 3)
    assert _rel(u_h, math.exp(-0.7 * T) * u_base) <= 1e-12


def test_coefficient_callables_and_grids_agree():
    """The oracle takes coefficient functions of (x, v) or grids [nv][nx]: both
    give the same operators (pins the transpose in the grid path)."""
    g = _grid()
    f = {"fx": lambda x, v: -v + 0.1 * x, "gvv": lambda x, v: 1.0 + 0.2 * x * x,
         "sv": lambda x, v: 0.5 + 0.1 * np.tanh(x - v)}
    import workloads as wl
    fn = wl.Coefficients(**f)
    B1, A1 = operators.drift_and_noise(g, fn)
    B2, A2 = operators.drift_and_noise(g, {k: _grid_array(v) for k, v in f.items()})
    assert abs(B1 - B2).max() == 0.0 and abs(A1 - A2).max() == 0.0
