"""Pins of the CPU oracle against facts fixed by the paper or by mathematics.

Each test names what it pins and which plausible mistake it would catch.
None of them compares the oracle with itself or with the GPU path.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

from oracle import errors, euler, exact, expmv, integrals, magnus, operators
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _langevin(n, lo, hi, a, sigma):
    g = operators.Grid(n, n, lo, hi, lo, hi)
    B, A = operators.drift_and_noise(g, wl.langevin_constant(a, sigma))
    return g, B, A


# --------------------------------------------------------------------- P1
def test_sparsity_counts_match_remark():
    """Remark 'sparsity': 2/5/5/8/10 non-zero diagonals at d = 50.  Catches a
    swapped role of A and B, a wrong Kronecker order, a zeroth-order reading of
    the noise, or commutators built from untruncated stencils."""
    with open(os.path.join(GOLDEN, "sparsity_d50.json")) as f:
        gold = json.load(f)
    g, B, A = _langevin(gold["d"], gold["lo"], gold["hi"], gold["a"], gold["sigma"])
    basis = operators.magnus_basis(B, A)
    names = {"B": basis[0], "A": basis[1], "[B,A]": basis[3], "[[B,A],A]": basis[4],
             "[[B,A],B]": basis[5]}
    for name, want in gold["nonzero_diagonals"].items():
        assert len(operators.nonzero_diagonals(names[name])) == want, name


def test_sparsity_offsets_fix_layout():
    """x is the fast index (column stacking, Section 2): the transport
    f^x d/dx couples neighbours at offset +-1, d/dv at +-d."""
    d = 50
    g, B, A = _langevin(d, -4.0, 4.0, 1.1, 1 / math.sqrt(10))
    assert operators.nonzero_diagonals(B) == [-d, -1, 0, 1, d]
    assert operators.nonzero_diagonals(A) == [-d, d]
    # [B,A] has a main diagonal only on the v boundary rows (truncated products)
    BA = operators.magnus_basis(B, A)[3]
    diag = BA.diagonal()
    nz = np.nonzero(np.abs(diag) > 1e-9 * np.abs(diag).max())[0]
    assert set(nz // d) == {0, d - 1}


def test_exact_structure_of_double_commutators():
    """In exact arithmetic the +-(2d+-1) diagonals of the double commutators
    are cancellation residues of size ~1e-16 relative."""
    d = 50
    g, B, A = _langevin(d, -4.0, 4.0, 1.1, 1 / math.sqrt(10))
    basis = operators.magnus_basis(B, A)
    for M, want in ((basis[4], [-d, -1, 1, d]), (basis[5], [-d - 2, -d, -d + 2, d - 2, d, d + 2])):
        tol = 1e-13 * abs(M).max()
        assert operators.nonzero_diagonals(M, tol) == want


# --------------------------------------------------------------------- P2
def test_exact_solution_initial_limit():
    """u_t -> phi as t -> 0 (Section 3.1: u solves the Cauchy problem)."""
    x = np.linspace(-2, 2, 9)
    X, V = np.meshgrid(x, x)
    u = exact.solution(1e-9, X, V, 1.0, 0.5, 0.25, 0.0, 0.0)
    phi = np.exp(-(X ** 2 + V ** 2) / 0.5) / (2 * math.pi * 0.25)
    np.testing.assert_allclose(u, phi, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("t,Wt,It", [(1.0, 0.7, -0.3), (0.5, -1.1, 0.4)])
def test_exact_solution_matches_printed_kernel(t, Wt, It):
    """The closed form equals the integral of the printed Gamma_0 and m_t
    against the Gaussian initial density (tensor Gauss-Hermite quadrature).
    Catches a wrong sign of sigma*W or sigma*int W, a wrong covariance or a
    wrong normalisation."""
    a, sigma, s0sq = 1.0, 0.5, 0.25
    nodes, weights = np.polynomial.hermite_e.hermegauss(300)   # weight exp(-z^2/2)
    weights = weights / math.sqrt(2 * math.pi)                 # expectation under N(0,1)
    s0 = math.sqrt(s0sq)
    XI, ETA = np.meshgrid(s0 * nodes, s0 * nodes, indexing="ij")
    WW = np.outer(weights, weights)
    for (x, v) in [(0.0, 0.0), (0.8, -0.4), (-1.3, 0.9)]:
        mx, mv = exact.mean_shift(t, XI, ETA, sigma, Wt, It)
        quad = np.sum(WW * exact.gamma0(t, x - mx, v - mv, a, sigma))
        closed = exact.solution(t, x, v, a, sigma, s0sq, Wt, It)
        assert abs(quad - closed) <= 1e-9 * max(abs(closed), 1e-3)


def test_magnus_converges_to_exact_at_second_order_in_space():
    """Magnus m2 against the closed form: the error is the space
    discretisation floor and falls about 4x when the grid spacing halves
    (central differences).  A wrong transport sign gives O(1) error."""
    dW = wl.brownian_increments(0, 1, 2 ** 10)
    ps = integrals.path_statistics(dW, 1.0)
    errs = []
    for n in (31, 63):
        g, B, A = _langevin(n, -5.0, 5.0, 1.0, 0.5)
        basis = operators.magnus_basis(B, A)
        coef = integrals.path_coefficients(dW, 1.0, 8, 2)
        u0 = wl.gaussian_density(n, n, -5, 5, -5, 5, 0.25).reshape(-1)
        uT = magnus.iterated_magnus(basis, coef[0], u0)
        uex = exact.solution_on_grid(g, 1.0, 1.0, 0.5, 0.25, ps[0, 0], ps[0, 1])
        errs.append(errors.relative_error(uex, uT))
    assert errs[1] < 0.03
    assert 3.0 < errs[0] / errs[1] < 5.0


# --------------------------------------------------------------------- P3
@pytest.mark.parametrize("order", [1, 2, 3])
def test_drift_only_is_exact(order):
    """Remark 'determLangevin': with A = 0 the scheme is exact at every order:
    u_T = exp(T B) u_0 (dense expm as brute force)."""
    n = 10
    g = operators.Grid(n, n, -3, 3, -3, 3)
    B, A = operators.drift_and_noise(g, wl.Coefficients(fx=lambda x, v: -v,
                                                        gvv=lambda x, v: 1.0 + 0 * x))
    assert A.nnz == 0
    basis = operators.magnus_basis(B, A)
    dW = wl.brownian_increments(3, 1, 64)
    coef = integrals.path_coefficients(dW, 0.7, 4, order)
    u0 = wl.gaussian_density(n, n, -3, 3, -3, 3, 0.25).reshape(-1)
    got = magnus.iterated_magnus(basis, coef[0], u0)
    want = scipy.linalg.expm(0.7 * B.toarray()) @ u0
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


# --------------------------------------------------------------------- P4
@pytest.mark.parametrize("order,ito", [(1, False), (2, True), (3, True)])
def test_commuting_noise_closed_form(order, ito):
    """A = beta I commutes with B: the Ito solution is
    exp(beta W_T - beta^2 T/2) exp(T B) u_0.  Orders 2 and 3 reproduce it
    exactly; order 1 lacks the Ito correction -A^2 t/2 and gives
    exp(beta W_T) exp(T B) u_0 (eq. (MagnusFormulas))."""
    n, beta, T = 9, 0.6, 1.0
    g = operators.Grid(n, n, -3, 3, -3, 3)
    B, A = operators.drift_and_noise(g, wl.Coefficients(fx=lambda x, v: -v,
                                                        gvv=lambda x, v: 1.0 + 0 * x,
                                                        sig=lambda x, v: beta + 0 * x))
    basis = operators.magnus_basis(B, A)
    dW = wl.brownian_increments(5, 1, 96)
    coef = integrals.path_coefficients(dW, T, 6, order)
    u0 = wl.gaussian_density(n, n, -3, 3, -3, 3, 0.25).reshape(-1)
    got = magnus.iterated_magnus(basis, coef[0], u0)
    WT = dW.sum()
    scale = math.exp(beta * WT - (0.5 * beta * beta * T if ito else 0.0))
    want = scale * (scipy.linalg.expm(T * B.toarray()) @ u0)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


# --------------------------------------------------------------------- P5
def test_linear_path_gives_zero_commutator_weights():
    """If the path is linear on every Magnus step (one fine increment per
    step), int W = h W_h/2, int W^2 = h W_h^2/3, int s W = h^2 W_h/3, so the
    weights of [B,A], [[B,A],A] and [[B,A],B] in eq. (MagnusFormulas) vanish."""
    dW = wl.brownian_increments(7, 3, 16)
    c = integrals.path_coefficients(dW, 1.0, 16, 3)
    assert np.max(np.abs(c[..., 3:])) < 1e-15
    assert np.allclose(c[..., 1], dW)


def test_brownian_scaling_of_weights():
    """Scaling the path by lam scales the [B,A] and [[B,A],B] weights by lam
    and the [[B,A],A] weight by lam^2."""
    dW = wl.brownian_increments(8, 2, 256)
    c1 = integrals.path_coefficients(dW, 1.0, 4, 3)
    c2 = integrals.path_coefficients(2.5 * dW, 1.0, 4, 3)
    np.testing.assert_allclose(c2[..., 3], 2.5 * c1[..., 3], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(c2[..., 5], 2.5 * c1[..., 5], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(c2[..., 4], 6.25 * c1[..., 4], rtol=1e-12, atol=1e-15)


# --------------------------------------------------------------------- P6
def test_weight_moments():
    """Moments over Brownian paths: E[c3] = 0 and Var[c3] = h^3/12 (c3 is the
    area under the Brownian bridge), E[c4] = h^2/12, E[c5] = 0."""
    h, P = 1.0, 40000
    dW = wl.brownian_increments(11, P, 128, T=h)
    c = integrals.path_coefficients(dW, h, 1, 3)[:, 0, :]
    se = lambda x: x.std() / math.sqrt(P)
    assert abs(c[:, 3].mean()) < 4 * se(c[:, 3])
    var_c3 = c[:, 3].var()
    assert abs(var_c3 - h ** 3 / 12) < 4 * (h ** 3 / 12) * math.sqrt(2.0 / P)
    assert abs(c[:, 4].mean() - h * h / 12) < 4 * se(c[:, 4])
    assert abs(c[:, 5].mean()) < 4 * se(c[:, 5])


# --------------------------------------------------------------------- P7
def test_integrals_satisfy_ito_product_identities():
    """Lemma 'Ito1' (eq. (Ito1a)) applied to the piecewise-linear path, for
    which dW_r = (Delta W_i / delta) dr on each fine interval:
      int_0^h W dr   = h W_h - int r dW_r
      int_0^h r W dr = h^2 W_h / 2 - int r^2/2 dW_r
      int_0^h W^2 dr = h W_h^2 - int 2 r W dW_r
    with the right-hand sides evaluated interval by interval in closed form."""
    h, n = 0.37, 50
    dW = wl.brownian_increments(12, 1, n, T=h)[0]
    DW, I1, I2, J = integrals.local_integrals(dW, h)
    delta = h / n
    r = delta * np.arange(n + 1)
    W = np.concatenate([[0.0], np.cumsum(dW)])
    slope = dW / delta
    int_r_dW = np.sum(slope * (r[1:] ** 2 - r[:-1] ** 2) / 2)
    int_r2_dW = np.sum(slope * (r[1:] ** 3 - r[:-1] ** 3) / 6)
    # int r W(r) dW = sum slope * int_{r_i}^{r_i+1} r (W_i + slope (r - r_i)) dr
    rl, rr = r[:-1], r[1:]
    int_rW_dW = np.sum(slope * (W[:-1] * (rr ** 2 - rl ** 2) / 2
                                + slope * ((rr ** 3 - rl ** 3) / 3 - rl * (rr ** 2 - rl ** 2) / 2)))
    assert abs(I1 - (h * DW - int_r_dW)) < 1e-14
    assert abs(J - (h * h * DW / 2 - int_r2_dW)) < 1e-14
    assert abs(I2 - (h * DW * DW - 2 * int_rW_dW)) < 1e-14


def test_weights_linear_in_noise_match_dexp_series():
    """Independent derivation of the [B,A] and [[B,A],B] weights.  To first
    order in A, X_t = e^{Bt}(I + G), G = int e^{-Bs} A e^{Bs} dW_s
    = sum_n (-1)^n ad_B^n(A) I_n / n!,  I_n = int_0^t s^n dW_s, and
    log X_t = Bt + (x/(1-e^{-x}))|_{x = t ad_B} G + O(A^2), with
    x/(1-e^{-x}) = 1 + x/2 + x^2/12 + ...  Collecting ad_B(A) = [B,A] and
    ad_B^2(A) = -[[B,A],B]:
        w[B,A]     = -I_1 + t W_t / 2
        w[[B,A],B] = -(I_2/2 - t I_1/2 + t^2 W_t/12)
    (no Ito correction enters terms linear in A).  I_n is evaluated on the
    piecewise-linear path interval by interval.  Catches a sign or factor
    error in the c3 or c5 weight."""
    h, n = 0.61, 40
    for seed in (14, 15, 16):
        dW = wl.brownian_increments(seed, 1, n, T=h)[0]
        DW, I1, I2, J = integrals.local_integrals(dW, h)
        c = integrals.magnus_coefficients(3, h, DW, I1, I2, J)
        r = (h / n) * np.arange(n + 1)
        slope = dW / (h / n)
        In = [np.sum(slope * (r[1:] ** (k + 1) - r[:-1] ** (k + 1)) / (k + 1)) for k in range(3)]
        assert abs(In[0] - DW) < 1e-14
        assert abs(c[3] - (-In[1] + h * DW / 2)) < 1e-14
        assert abs(c[5] - (-(In[2] / 2 - h * In[1] / 2 + h * h * DW / 12))) < 1e-14


def test_step_integrals_add_up_to_path_integral():
    """int_0^T W = sum_k (W_{t_k} h + int W~ over step k): the per-step restart
    (Markov property) loses nothing."""
    dW = wl.brownian_increments(13, 2, 512)
    K, T = 8, 1.0
    h = T / K
    c = integrals.path_coefficients(dW, T, K, 2)
    I1 = c[..., 3] + 0.5 * h * c[..., 1]
    Wk = np.concatenate([np.zeros((2, 1)), np.cumsum(c[..., 1], axis=1)[:, :-1]], axis=1)
    total = np.sum(Wk * h + I1, axis=1)
    np.testing.assert_allclose(total, integrals.path_statistics(dW, T)[:, 1], rtol=1e-12)


# --------------------------------------------------------------------- P8
def _magnus_dense(Bm, Am, dW, T, K, order):
    coef = integrals.path_coefficients(dW[None, :], T, K, order)[0]
    BA = Bm @ Am - Am @ Bm
    basis = [Bm, Am, Am @ Am, BA, BA @ Am - Am @ BA, BA @ Bm - Bm @ BA]
    X = np.eye(Bm.shape[0])
    for k in range(K):
        Y = sum(c * M for c, M in zip(coef[k], basis))
        X = scipy.linalg.expm(Y) @ X
    return X


def test_strong_convergence_orders_on_small_matrices():
    """Theorem 'convergence' and eq. (MagnusFormulas) on random 4x4 A, B:
    against a Milstein solution on the fine grid, order 2 converges with
    strong order about 1 and order 3 faster; order 1 does not converge to the
    Ito solution.  Catches sign errors in the [B,A] weight and wrong order-3
    weights."""
    rng = np.random.default_rng(1)
    Bm = 0.7 * rng.standard_normal((4, 4))
    Am = 0.7 * rng.standard_normal((4, 4))
    T, Nf, P = 1.0, 2 ** 14, 12
    dW = wl.brownian_increments(21, P, Nf, T=T)
    delta = T / Nf
    # Milstein reference, all paths at once: X <- X + B X dt + A X dW + A^2 X (dW^2 - dt)/2
    X = np.broadcast_to(np.eye(4), (P, 4, 4)).copy()
    A2 = Am @ Am
    for i in range(Nf):
        w = dW[:, i][:, None, None]
        X = X + delta * (Bm @ X) + w * (Am @ X) + 0.5 * (w * w - delta) * (A2 @ X)
    Ks = [16, 32, 64, 128]
    slopes = {}
    final = {}
    for order in (1, 2, 3):
        e = []
        for K in Ks:
            errs = [np.linalg.norm(_magnus_dense(Bm, Am, dW[p], T, K, order) - X[p]) ** 2
                    for p in range(P)]
            e.append(math.sqrt(np.mean(errs)))
        slopes[order] = np.polyfit(np.log(Ks), np.log(e), 1)[0]
        final[order] = e[-1]
    assert slopes[2] < -0.8
    assert slopes[3] < -1.3
    assert final[3] < final[2]
    assert slopes[1] > -0.3          # stalls at the Stratonovich solution


# --------------------------------------------------------------------- P9
def test_euler_converges_towards_magnus():
    """Euler-Maruyama, eq. (EulerMaruyama), on the same paths approaches the
    Magnus solution as dt -> 0, with strong order about 1/2."""
    n = 12
    g, B, A = _langevin(n, -5.0, 5.0, 1.0, 0.5)
    basis = operators.magnus_basis(B, A)
    P, Nf, T = 4, 2 ** 13, 1.0
    dW = wl.brownian_increments(31, P, Nf)
    u0 = wl.gaussian_density(n, n, -5, 5, -5, 5, 0.25).reshape(-1)
    ref = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW, T, 128, 3), u0)
    NEs = [2 ** 7, 2 ** 9, 2 ** 11, 2 ** 13]
    e = []
    for NE in NEs:
        uE = euler.euler_paths(B, A, u0, integrals.euler_increments(dW, NE), T / NE)
        e.append(np.mean([np.linalg.norm(uE[p] - ref[p]) / np.linalg.norm(ref[p])
                          for p in range(P)]))
    slope = np.polyfit(np.log(NEs), np.log(e), 1)[0]
    assert -0.85 < slope < -0.35
    assert e[-1] < e[0] / 4


# --------------------------------------------------------------------- P10
@pytest.mark.parametrize("n,seed", [(8, 0), (12, 1)])
def test_series_expmv_matches_dense_expm(n, seed):
    """The oracle's power series against scipy's dense expm (Pade)."""
    g, B, A = _langevin(n, -4.0, 4.0, 1.1, 1 / math.sqrt(10))
    basis = operators.magnus_basis(B, A)
    rng = np.random.default_rng(seed)
    c = np.array([0.2, 0.4, -0.1, 0.05, 0.01, -0.02]) * (1 + 0.2 * rng.standard_normal(6))
    Om = magnus.magnus_log(basis, c)
    u = rng.standard_normal(g.N)
    got = expmv.expmv_series(Om, u)
    want = expmv.expmv_dense(Om, u)
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)
    got2 = expmv.expmv_series(Om, u, shift=False)
    assert np.linalg.norm(got2 - want) <= 1e-13 * np.linalg.norm(want)


# --------------------------------------------------------------------- P11
def test_mass_and_reflection_symmetry():
    """The density keeps unit mass up to boundary losses, and the scheme is
    symmetric under (x, v, W) -> (-x, -v, -W)."""
    n = 40
    g, B, A = _langevin(n, -5.0, 5.0, 1.0, 0.5)
    basis = operators.magnus_basis(B, A)
    dW = wl.brownian_increments(41, 1, 256)
    u0 = wl.gaussian_density(n, n, -5, 5, -5, 5, 0.25).reshape(-1)
    up = magnus.iterated_magnus(basis, integrals.path_coefficients(dW, 1.0, 8, 3)[0], u0)
    um = magnus.iterated_magnus(basis, integrals.path_coefficients(-dW, 1.0, 8, 3)[0], u0)
    assert abs(up.sum() * g.dx * g.dv - 1.0) < 1e-3
    flipped = um.reshape(n, n)[::-1, ::-1].reshape(-1)
    assert np.linalg.norm(up - flipped) <= 1e-12 * np.linalg.norm(up)


# --------------------------------------------------------------------- norms
def test_kappa_window_indices():
    """Central windows of eq. (meanErr), with the width floor(d/2^kappa)."""
    assert list(errors.window(8, 0)) == list(range(8))
    assert list(errors.window(8, 1)) == [2, 3, 4, 5]
    assert list(errors.window(8, 2)) == [3, 4]
    w = errors.window(300, 4)
    assert len(w) == 18 and w[0] == 140


def test_error_norms_on_hand_values():
    ref = np.ones((4, 4))
    app = np.ones((4, 4))
    app[1, 2] = 1.5            # inside the kappa=1 window (indices 1..2)
    app[0, 0] = 3.0            # outside it
    assert abs(errors.relative_error(ref, app, 1) - 0.5 / 2.0) < 1e-15
    assert abs(errors.relative_error(ref, app, 0) - math.sqrt(0.25 + 4.0) / 4.0) < 1e-15
    me = errors.mean_abs_error([ref, ref], [app, ref], 1)
    assert me.shape == (2, 2) and abs(me[0, 1] - 0.25) < 1e-15
    assert abs(errors.average_mean_error([ref], [app], 1) - 0.5 / 4) < 1e-15


def test_brownian_subrange_equals_full_draw():
    full = wl.brownian_increments(3, 10, 64)
    part = wl.brownian_increments(3, 10, 64, first=4, count=3)
    np.testing.assert_array_equal(part, full[4:7])


# ------------------------------------------------- Remark "stepSizeControl"
def _langevin_small(n, sig=None):
    g = operators.Grid(n, n, -4, 4, -4, 4)
    c = wl.langevin_constant(1.0, 0.5) if sig is None else wl.Coefficients(
        fx=lambda x, v: -v, gvv=lambda x, v: 1.0 + 0 * x, sig=sig)
    B, A = operators.drift_and_noise(g, c)
    return operators.magnus_basis(B, A), A


@pytest.mark.parametrize("case", ["drift_only", "commuting"])
def test_step_control_accepts_first_step_when_orders_agree(case):
    """With A = 0 (Remark 'determLangevin') or A = beta I (commuting noise)
    every commutator vanishes and orders 2 and 3 are the same exact scheme:
    the order gap is rounding only and the first step size is accepted."""
    n = 10
    if case == "drift_only":
        g = operators.Grid(n, n, -4, 4, -4, 4)
        B, A = operators.drift_and_noise(g, wl.Coefficients(fx=lambda x, v: -v,
                                                            gvv=lambda x, v: 1.0 + 0 * x))
        basis = operators.magnus_basis(B, A)
    else:
        basis, A = _langevin_small(n, sig=lambda x, v: 0.6 + 0 * x)
    dW = wl.brownian_increments(9, 2, 64)
    u0 = wl.gaussian_density(n, n, -4, 4, -4, 4, 0.25).reshape(-1)
    from oracle import step_control
    gap = step_control.order_gap(basis, dW, 1.0, 2, u0, n, n)
    assert gap.max() <= 1e-12
    K, g0, ok, hist = step_control.select_steps(basis, dW, 1.0, u0, n, n, 2, 2, 64, 1e-10)
    assert (K, ok, len(hist)) == (2, True, 1)


def test_step_control_gap_shrinks_at_first_order_or_faster():
    """Non-commuting Langevin noise: the order-2/order-3 distance is the size
    of the order-3 terms, c4 [[B,A],A] + c5 [[B,A],B] summed over the steps,
    which falls at least like h (c4 has mean h^2/12 per step, c5 zero mean and
    size h^(3/2)): every halving of h cuts the sample's largest gap by at
    least 1.5x, and 16x smaller steps by at least 16x."""
    n = 12
    basis, _ = _langevin_small(n)
    dW = wl.brownian_increments(7, 3, 256)
    u0 = wl.gaussian_density(n, n, -4, 4, -4, 4, 0.25).reshape(-1)
    from oracle import step_control
    g = [step_control.order_gap(basis, dW, 1.0, K, u0, n, n).max() for K in (2, 4, 8, 16, 32)]
    for a, b in zip(g, g[1:]):
        assert b <= a / 1.5, g
    assert g[-1] <= g[0] / 16, g


def test_step_control_selection_rule():
    """The selection walks K0, f K0, ... and stops at the first gap <= tol;
    without one it returns the last K tried (within Kmax and dividing Nf),
    not accepted."""
    n = 12
    basis, _ = _langevin_small(n)
    dW = wl.brownian_increments(7, 3, 256)
    u0 = wl.gaussian_density(n, n, -4, 4, -4, 4, 0.25).reshape(-1)
    from oracle import step_control
    gaps = {K: step_control.order_gap(basis, dW, 1.0, K, u0, n, n).max() for K in (2, 4, 8)}
    tol = 0.5 * (gaps[4] + gaps[8])       # between the gaps at K = 4 and 8
    K, g, ok, hist = step_control.select_steps(basis, dW, 1.0, u0, n, n, 2, 2, 64, tol)
    assert (K, ok) == (8, True) and g == gaps[8] and [k for k, _ in hist] == [2, 4, 8]
    K, g, ok, hist = step_control.select_steps(basis, dW, 1.0, u0, n, n, 2, 2, 8, 1e-12)
    assert (K, ok) == (8, False) and [k for k, _ in hist] == [2, 4, 8]
    K, g, ok, hist = step_control.select_steps(basis, dW, 1.0, u0, n, n, 4, 4, 64, 1e-12)
    assert (K, ok) == (64, False) and [k for k, _ in hist] == [4, 16, 64]
    # one fine increment per step: the path is linear on every step, c3 = c4 =
    # c5 = 0, and the two orders coincide (the gap is exactly zero)
    K, g, ok, hist = step_control.select_steps(basis, dW, 1.0, u0, n, n, 4, 4, 256, 1e-12)
    assert (K, ok, g) == (256, True, 0.0) and [k for k, _ in hist] == [4, 16, 64, 256]
    with pytest.raises(ValueError):
        step_control.select_steps(basis, dW, 1.0, u0, n, n, 3, 2, 64, 1.0)
