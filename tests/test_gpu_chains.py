"""The paper's variable coefficients, eq. (coeffsLangevinVar): diffusion
a (1 + 1/(x^2+1)) and noise sigma sqrt(1 + 1/(x^2+1)) through d/dv, both
depending on x, with the transport -v d/dx.  In [B, A] the x derivative meets
the x-dependent noise once, in [[B,A],B] twice, so the Magnus basis holds
x-terms C (x) diag(x_0) D^x diag(x_1) (order 2) and
C (x) diag(x_0) D^x diag(x_1) D^x diag(x_2) (order 3) besides the powers of
D^x and the diagonal x-factors (order 3: 14 x-terms over 7 x vectors).  GPU
(FP64) against the CPU oracle, which assembles B and A as printed in
Section 2 (sparse Kronecker products with diag(vec Z)) and forms the basis by
sparse products:

  Magnus FP64: 1e-10 relative (Frobenius) and max-norm, orders 1 to 3,
  register-resident (nx <= 128) and cooperative (nx <= 512) kernels;
  Euler: 1e-12.
FP32C is reported unsupported for x-terms.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2207_09776_amd as mg
import workloads as wl
from oracle import euler, integrals, magnus, operators

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
LO, HI = -4.0, 4.0          # the paper's domain
COEFFS = wl.langevin_paper_variable(1.1, 1.0 / math.sqrt(10.0))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def check(got, want, tol, what):
    for p in range(want.shape[0]):
        fro = np.linalg.norm(got[p] - want[p]) / np.linalg.norm(want[p])
        mx = np.abs(got[p] - want[p]).max() / np.abs(want[p]).max()
        assert fro <= tol and mx <= tol, (what, p, fro, mx)


def setup(nx, nv, order):
    g = operators.Grid(nx, nv, LO, HI, LO, HI)
    B, A = operators.drift_and_noise(g, COEFFS)
    basis = operators.magnus_basis(B, A)
    ops = mg.build_operators(nx, nv, LO, HI, LO, HI,
                             wl.sample_coefficients(COEFFS, nx, nv, LO, HI, LO, HI), order)
    return B, A, basis, ops


CASES = [
    # (name, nx, nv, order, P, K, Nf, T): resident and cooperative, edge-reaching
    ("res-40x36-m1", 40, 36, 1, 2, 2, 64, 0.02),
    ("res-40x36-m2", 40, 36, 2, 2, 2, 64, 0.02),
    ("res-100x90-m2", 100, 90, 2, 2, 2, 64, 0.004),
    ("res-128x128-m2", 128, 128, 2, 2, 3, 96, 0.003),
    ("coop-200x150-m2", 200, 150, 2, 2, 2, 64, 0.002),
    ("coop-256x256-m2", 256, 256, 2, 1, 2, 64, 0.001),
    ("coop-300x200-m2", 300, 200, 2, 1, 2, 64, 0.001),
    ("res-40x36-m3", 40, 36, 3, 2, 2, 64, 0.02),
    ("res-100x90-m3", 100, 90, 3, 2, 2, 64, 0.004),
    ("res-128x128-m3", 128, 128, 3, 2, 3, 96, 0.003),
    ("coop-200x150-m3", 200, 150, 3, 2, 2, 64, 0.002),
    ("coop-256x256-m3", 256, 256, 3, 1, 2, 64, 0.001),
    ("coop-300x200-m3", 300, 200, 3, 1, 2, 64, 0.001),
    ("coop-350x120-m3", 350, 120, 3, 1, 2, 64, 0.001),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_paper_variable_coefficients_match_oracle(case):
    name, nx, nv, order, P, K, Nf, T = case
    say(f"chains {name}")
    B, A, basis, ops = setup(nx, nv, order)
    dW = wl.brownian_increments(121, P, Nf, T=T)
    u0 = np.random.default_rng(122).uniform(0.5, 1.5, size=(P, nx * nv))
    coef, _ = mg.iterated_integrals(to_dev(dW), T, K, order)
    uT, flags, _ = mg.magnus_expmv(ops, coef, to_dev(u0))
    torch.cuda.synchronize()
    assert int(flags.abs().sum()) == 0, flags.cpu().numpy()
    want = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW, T, K, order), u0)
    check(uT.cpu().numpy(), want, 1e-10, name)
    ops.close()


@pytest.mark.parametrize("order", [2, 3])
def test_paper_variable_coefficients_full_horizon_gaussian(order):
    """The paper's setting at d = 40: Gaussian datum, T = 1, h = 0.05
    (K = 20), against the oracle."""
    say(f"chains 40x40 T=1 order {order}")
    n, K, Nf, T = 40, 20, 2000, 1.0
    B, A, basis, ops = setup(n, n, order)
    dW = wl.brownian_increments(123, 2, Nf, T=T)
    u0 = wl.gaussian_density(n, n, LO, HI, LO, HI, 1.0).reshape(-1)
    coef, _ = mg.iterated_integrals(to_dev(dW), T, K, order)
    uT, flags, _ = mg.magnus_expmv(ops, coef, to_dev(u0))
    torch.cuda.synchronize()
    assert int(flags.abs().sum()) == 0
    want = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW, T, K, order), u0)
    check(uT.cpu().numpy(), want, 1e-10, "40x40 T=1")
    ops.close()


@pytest.mark.parametrize("nx,nv", [(40, 36), (200, 150)])
def test_paper_variable_euler_matches_oracle(nx, nv):
    say(f"chains euler {nx}x{nv}")
    B, A, basis, ops = setup(nx, nv, 2)
    P, NE, T = 2, 32, 0.004
    dW = wl.brownian_increments(124, P, 2 * NE, T=T)
    dWE = integrals.euler_increments(dW, NE)
    u0 = np.random.default_rng(125).uniform(0.5, 1.5, size=(P, nx * nv))
    u = to_dev(u0)
    flags = mg.euler_step(ops, u, to_dev(dWE), T / NE)
    torch.cuda.synchronize()
    assert int(flags.abs().sum()) == 0
    want = np.stack([euler.euler_paths(B, A, u0[p], dWE[p:p + 1], T / NE)[0] for p in range(P)])
    check(u.cpu().numpy(), want, 1e-12, "euler")
    ops.close()


@pytest.mark.parametrize("order", [2, 3])
def test_chains_unsupported_forms_are_reported(order):
    say(f"chains unsupported, order {order}")
    ops = mg.build_operators(40, 36, LO, HI, LO, HI,
                             wl.sample_coefficients(COEFFS, 40, 36, LO, HI, LO, HI), order)
    coef = torch.zeros((1, 1, 6), dtype=torch.float64, device=DEV)
    u0 = torch.zeros(40 * 36, dtype=torch.float64, device=DEV)
    with pytest.raises(mg.MagnusError) as ex:
        mg.magnus_expmv(ops, coef, u0, precision="fp32c")
    assert ex.value.code == mg.MG_EUNSUPPORTED
    ops.close()
