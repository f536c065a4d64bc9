"""GPU parity on inputs that reach the domain boundary, for every kernel
family, through the C ABI against the CPU FP64 oracle.

The workloads start from a Gaussian whose values at the edge rows and columns
are tiny, so an error confined to the boundary would not show in a relative
norm there.  The method's own special cases sit exactly at that boundary:
the truncated products give [B,A] and the double commutators extra diagonals
only on the boundary rows (Remark 'sparsity'), the kernels keep guard rows at
the first and last slab and zero-fill the lane shifts at the x edges.  These
cases start every path from a seeded uniform field in [0.5, 1.5] (O(1) on
every edge) over a horizon short enough that the edge values stay O(1), and
check both the relative Frobenius error per path and the largest pointwise
difference against the largest oracle value:

  FP64 Magnus: 1e-10;  FP32C: 1e-5;  Euler: 1e-12.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2207_09776_amd as mg
import workloads as wl
from oracle import euler, integrals, magnus, operators

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
LO, HI = -5.0, 5.0


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def random_field(nx, nv, P, seed):
    """Seeded uniform [0.5, 1.5] initial values, one field per path."""
    return np.random.default_rng(seed).uniform(0.5, 1.5, size=(P, nx * nv))


def check(got, want, nx, nv, tol, what):
    """Relative Frobenius and max-norm bounds; also asserts that the oracle's
    edge rows and columns are O(1), i.e. that the case reaches the boundary."""
    for p in range(want.shape[0]):
        w = want[p].reshape(nv, nx)
        g = got[p].reshape(nv, nx)
        edge = max(np.abs(w[0]).max(), np.abs(w[-1]).max(), np.abs(w[:, 0]).max(),
                   np.abs(w[:, -1]).max())
        assert edge >= 1e-2 * np.abs(w).max(), (what, p, "edges not reached")
        fro = np.linalg.norm(g - w) / np.linalg.norm(w)
        mx = np.abs(g - w).max() / np.abs(w).max()
        assert fro <= tol and mx <= tol, (what, p, fro, mx)


def setup(nx, nv, coeffs, order):
    g = operators.Grid(nx, nv, LO, HI, LO, HI)
    B, A = operators.drift_and_noise(g, coeffs)
    basis = operators.magnus_basis(B, A)
    ops = mg.build_operators(nx, nv, LO, HI, LO, HI,
                             wl.sample_coefficients(coeffs, nx, nv, LO, HI, LO, HI), order)
    return B, A, basis, ops


def run_magnus(nx, nv, coeffs, order, P, K, Nf, T, prec, tol, seed, what):
    B, A, basis, ops = setup(nx, nv, coeffs, order)
    dW = wl.brownian_increments(seed, P, Nf, T=T)
    u0 = random_field(nx, nv, P, seed + 1)
    coef, _ = mg.iterated_integrals(to_dev(dW), T, K, order)
    uT, flags, _ = mg.magnus_expmv(ops, coef, to_dev(u0), precision=prec)
    torch.cuda.synchronize()
    assert int(flags.abs().sum()) == 0, (what, flags.cpu().numpy())
    want = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW, T, K, order), u0)
    check(uT.cpu().numpy(), want, nx, nv, tol, what)


CONST_CASES = [
    # (name, nx, nv, order, P, K, Nf, T, precision)
    # register-resident kernel (nx, nv <= 128): one and two points per lane,
    # ragged last wave
    ("res-40x36-m1-f64", 40, 36, 1, 2, 2, 64, 0.08, "fp64"),
    ("res-40x36-m2-f64", 40, 36, 2, 2, 2, 64, 0.08, "fp64"),
    ("res-40x36-m3-f64", 40, 36, 3, 2, 2, 64, 0.08, "fp64"),
    ("res-40x36-m2-f32c", 40, 36, 2, 2, 2, 64, 0.08, "fp32c"),
    ("res-40x36-m3-f32c", 40, 36, 3, 2, 2, 64, 0.08, "fp32c"),
    ("res-64x64-m3-f64", 64, 64, 3, 2, 2, 64, 0.02, "fp64"),
    ("res-128x100-m1-f64", 128, 100, 1, 2, 2, 64, 0.008, "fp64"),
    ("res-128x100-m2-f64", 128, 100, 2, 2, 2, 64, 0.008, "fp64"),
    ("res-128x100-m3-f64", 128, 100, 3, 2, 2, 64, 0.008, "fp64"),
    ("res-128x100-m2-f32c", 128, 100, 2, 2, 2, 64, 0.008, "fp32c"),
    ("res-128x100-m3-f32c", 128, 100, 3, 2, 2, 64, 0.008, "fp32c"),
    # cooperative kernel (nx > 128): several slabs per path, ragged last slab
    ("coop-200x150-m2-f64", 200, 150, 2, 2, 2, 64, 0.008, "fp64"),
    ("coop-200x150-m3-f64", 200, 150, 3, 2, 2, 64, 0.008, "fp64"),
    ("coop-256x256-m3-f64", 256, 256, 3, 1, 2, 64, 0.004, "fp64"),
    ("coop-256x256-m2-f32c", 256, 256, 2, 2, 2, 64, 0.004, "fp32c"),
    ("coop-300x200-m3-f32c", 300, 200, 3, 1, 2, 64, 0.004, "fp32c"),
    ("coop-512x130-m2-f64", 512, 130, 2, 1, 2, 64, 0.002, "fp64"),
    ("coop-512x130-m3-f32c", 512, 130, 3, 1, 2, 64, 0.002, "fp32c"),
    # 24-row workgroups (nx > 512), ragged in x and in the last slab
    ("coop-520x40-m2-f32c", 520, 40, 2, 2, 2, 64, 0.002, "fp32c"),
    ("coop-1024x60-m3-f32c", 1024, 60, 3, 1, 2, 64, 0.0008, "fp32c"),
    ("coop-1024x60-m3-f64", 1024, 60, 3, 1, 2, 64, 0.0008, "fp64"),
    ("coop-600x45-m2-f64", 600, 45, 2, 1, 2, 64, 0.0008, "fp64"),
    ("coop-1000x50-m2-f32c", 1000, 50, 2, 1, 2, 64, 0.0008, "fp32c"),
]


@pytest.mark.parametrize("case", CONST_CASES, ids=[c[0] for c in CONST_CASES])
def test_edges_constant_coefficients(case):
    name, nx, nv, order, P, K, Nf, T, prec = case
    say(f"edges {name}")
    run_magnus(nx, nv, wl.langevin_constant(1.0, 0.5), order, P, K, Nf, T, prec,
               1e-10 if prec == "fp64" else 1e-5, 61, name)


def four_factor_coefficients():
    base = wl.langevin_variable_sigma_beta()
    return wl.Coefficients(fx=base.fx, gvv=base.gvv, sv=base.sv,
                           h=lambda x, v: 0.05 * np.cos(np.pi * x / 5.0) * np.exp(-v * v / 4.0))


VAR_CASES = [
    # (name, nx, nv, factors, order, T, precision): three- and four-factor
    # x-dependent builds, resident and cooperative
    ("var3-40x36-m1-f64", 40, 36, 3, 1, 0.02, "fp64"),
    ("var3-40x36-m2-f64", 40, 36, 3, 2, 0.02, "fp64"),
    ("var3-100x90-m2-f32c", 100, 90, 3, 2, 0.004, "fp32c"),
    ("var4-64x64-m2-f64", 64, 64, 4, 2, 0.005, "fp64"),
    ("var4-64x64-m2-f32c", 64, 64, 4, 2, 0.005, "fp32c"),
    ("var3-200x150-m2-f64", 200, 150, 3, 2, 0.002, "fp64"),
    ("var3-300x200-m2-f32c", 300, 200, 3, 2, 0.001, "fp32c"),
    ("var4-200x150-m2-f64", 200, 150, 4, 2, 0.002, "fp64"),
    ("var3-512x130-m1-f64", 512, 130, 3, 1, 0.0005, "fp64"),
]


@pytest.mark.parametrize("case", VAR_CASES, ids=[c[0] for c in VAR_CASES])
def test_edges_x_dependent_factors(case):
    name, nx, nv, nd, order, T, prec = case
    say(f"edges {name}")
    coeffs = wl.langevin_variable_sigma_beta() if nd == 3 else four_factor_coefficients()
    run_magnus(nx, nv, coeffs, order, 2, 2, 64, T, prec, 1e-10 if prec == "fp64" else 1e-5,
               71, name)


def general_v_coefficients(which):
    """The Langevin operator plus v-dependent coefficients of eq. (generalSPDE)
    that the workloads leave at zero: a potential H, a v-transport f^v, a
    mixed second derivative g^xv (corner entries) and a zeroth-order noise
    sigma."""
    extra = {"h": lambda x, v: -0.3 + 0.1 * v + 0 * x,
             "fv": lambda x, v: 0.2 * np.sin(v) + 0 * x,
             "gxv": lambda x, v: 0.1 * (1.0 + 0.1 * v) + 0 * x,
             "sig": lambda x, v: 0.3 + 0.1 * np.cos(v) + 0 * x}
    kw = {"fx": lambda x, v: -v, "gvv": lambda x, v: 1.0 + 0 * x,
          "sv": lambda x, v: 0.5 + 0 * x}
    for k in (extra if which == "all" else [which]):
        kw[k] = extra[k]
    return wl.Coefficients(**kw)


GEN_CASES = [
    # (name, nx, nv, which, order, T, precision)
    ("h-40x36-m3-f64", 40, 36, "h", 3, 0.02, "fp64"),
    ("fv-40x36-m3-f64", 40, 36, "fv", 3, 0.02, "fp64"),
    ("gxv-40x36-m2-f64", 40, 36, "gxv", 2, 0.02, "fp64"),
    ("gxv-40x36-m3-f64", 40, 36, "gxv", 3, 0.02, "fp64"),
    ("sig-40x36-m3-f64", 40, 36, "sig", 3, 0.02, "fp64"),
    ("all-40x36-m1-f64", 40, 36, "all", 1, 0.02, "fp64"),
    ("all-40x36-m2-f32c", 40, 36, "all", 2, 0.02, "fp32c"),
    ("all-128x100-m3-f64", 128, 100, "all", 3, 0.002, "fp64"),
    ("all-200x150-m2-f64", 200, 150, "all", 2, 0.002, "fp64"),
    ("all-256x200-m3-f32c", 256, 200, "all", 3, 0.001, "fp32c"),
]


@pytest.mark.parametrize("case", GEN_CASES, ids=[c[0] for c in GEN_CASES])
def test_general_v_dependent_coefficients(case):
    """v-dependent H, f^v, g^xv and sigma (the build accepts them): the
    factored tables carry them exactly, resident and cooperative kernels."""
    name, nx, nv, which, order, T, prec = case
    say(f"general coefficients {name}")
    run_magnus(nx, nv, general_v_coefficients(which), order, 2, 2, 64, T, prec,
               1e-10 if prec == "fp64" else 1e-5, 81, name)


EULER_CASES = [
    # (name, nx, nv, coefficients, NE, T): resident (nx <= 128) and cooperative
    ("euler-40x36", 40, 36, "const", 32, 0.02),
    ("euler-128x100", 128, 100, "const", 32, 0.002),
    ("euler-var-100x90", 100, 90, "var", 32, 0.004),
    ("euler-200x150", 200, 150, "const", 32, 0.002),
    ("euler-512x130", 512, 130, "const", 32, 0.0005),
    ("euler-var-300x200", 300, 200, "var", 32, 0.001),
    ("euler-gen-200x150", 200, 150, "gen", 32, 0.002),
]


@pytest.mark.parametrize("case", EULER_CASES, ids=[c[0] for c in EULER_CASES])
def test_edges_euler(case):
    name, nx, nv, kind, NE, T = case
    say(f"edges {name}")
    coeffs = {"const": wl.langevin_constant(1.0, 0.5),
              "var": wl.langevin_variable_sigma_beta(),
              "gen": general_v_coefficients("all")}[kind]
    B, A, basis, ops = setup(nx, nv, coeffs, 2)
    P = 2
    dW = wl.brownian_increments(91, P, NE * 2, T=T)
    dWE = integrals.euler_increments(dW, NE)
    u0 = random_field(nx, nv, P, 92)
    u = to_dev(u0)
    flags = mg.euler_step(ops, u, to_dev(dWE), T / NE)
    torch.cuda.synchronize()
    assert int(flags.abs().sum()) == 0
    want = np.stack([euler.euler_paths(B, A, u0[p], dWE[p:p + 1], T / NE)[0] for p in range(P)])
    check(u.cpu().numpy(), want, nx, nv, 1e-12, name)
