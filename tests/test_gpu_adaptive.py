"""mg_magnus_adaptive (Remark "stepSizeControl", step by step along each
path) against the oracle's adaptive_path on the same paths: the accepted
level of every coarse step equal, and the terminal values within 1e-10
(FP64) or 1e-5 (FP32C) of the oracle, on the register-resident and the
cooperative kernels.  The tolerance is placed where the oracle's decisions
do not change when it moves by a relative 1e-3, so that rounding cannot flip
a level; the noise-free case refines nothing, and a tolerance above every
distance gives the uniform launch."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2207_09776_amd as mg
import workloads as wl
from oracle import integrals, magnus, operators, step_control

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
T = 1.0
LO, HI = -4.0, 4.0


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def setup(nx, nv, sigma):
    coeffs = wl.langevin_constant(1.0, sigma)
    g = operators.Grid(nx, nv, LO, HI, LO, HI)
    basis = operators.magnus_basis(*operators.drift_and_noise(g, coeffs))
    arrays = wl.sample_coefficients(coeffs, nx, nv, LO, HI, LO, HI)
    ops2 = mg.build_operators(nx, nv, LO, HI, LO, HI, arrays, 2)
    ops3 = mg.build_operators(nx, nv, LO, HI, LO, HI, arrays, 3)
    return basis, ops2, ops3


def stable_tolerance(basis, dW, u0, nx, nv, K0, f, L, margin, T):
    """A tolerance with some steps refined and some not, whose decisions stay
    the same when it moves by the relative margin either way."""
    g0 = np.sort(step_control.adaptive_paths(basis, dW, T, u0, nx, nv, K0, f, 0, 1e300)[2]
                 .reshape(-1))
    for i in range(len(g0) // 2, len(g0) - 1):
        tol = float(np.sqrt(g0[i] * g0[i + 1]))
        runs = [step_control.adaptive_paths(basis, dW, T, u0, nx, nv, K0, f, L, tol * s)
                for s in (1.0 - margin, 1.0, 1.0 + margin)]
        lv = [r[1] for r in runs]
        if all(np.array_equal(lv[0], x) for x in lv) and lv[1].max() > lv[1].min():
            return tol, runs[1]
    pytest.skip("no tolerance with stable mixed decisions for these paths")


CASES = [
    # (nx, nv, P, Nf, T, K0, factor, max_level, precision, tol, margin); the
    # horizon keeps every coarse step inside the convergence range
    (24, 24, 3, 128, 1.0, 4, 2, 2, "fp64", 1e-10, 1e-3),
    (24, 24, 3, 128, 1.0, 4, 2, 2, "fp32c", 1e-5, 1e-2),
    (200, 150, 2, 64, 0.02, 2, 2, 1, "fp64", 1e-10, 1e-3),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[8]}" for c in CASES])
def test_adaptive_matches_oracle(case):
    nx, nv, P, Nf, T, K0, f, L, prec, tol_u, margin = case
    say(f"adaptive {nx}x{nv} {prec}")
    basis, ops2, ops3 = setup(nx, nv, 0.9)
    dW = wl.brownian_increments(41, P, Nf, T=T)
    u0 = wl.gaussian_density(nx, nv, LO, HI, LO, HI, 0.5).reshape(-1)
    tol, (want, lv_o, gp_o) = stable_tolerance(basis, dW, u0, nx, nv, K0, f, L, margin, T)
    uT, lv, gp = mg.magnus_adaptive(ops2, ops3, to_dev(dW), T, to_dev(u0), K0, f, L, tol,
                                    precision=prec)
    torch.cuda.synchronize()
    assert np.array_equal(lv, lv_o), (lv, lv_o)
    got = uT.cpu().numpy()
    for p in range(P):
        assert rel(got[p], want[p]) <= tol_u, (p, rel(got[p], want[p]))
    fin = np.isfinite(gp_o)
    assert np.allclose(gp[fin], gp_o[fin], rtol=1e-3 if prec == "fp32c" else 1e-6, atol=1e-14)
    ops2.close()
    ops3.close()


def test_adaptive_special_cases():
    say("adaptive special cases")
    n, P, Nf, K0 = 24, 2, 64, 4
    # no noise: nothing is refined
    basis, ops2, ops3 = setup(n, n, 0.0)
    dW = wl.brownian_increments(43, P, Nf, T=T)
    u0 = wl.gaussian_density(n, n, LO, HI, LO, HI, 0.5).reshape(-1)
    uT, lv, gp = mg.magnus_adaptive(ops2, ops3, to_dev(dW), T, to_dev(u0), K0, 2, 3, 1e-10)
    assert np.all(lv == 0) and gp.max() <= 1e-12
    ops2.close()
    ops3.close()
    # a tolerance above every distance: the uniform order-3 launch
    basis, ops2, ops3 = setup(n, n, 0.9)
    uT, lv, gp = mg.magnus_adaptive(ops2, ops3, to_dev(dW), T, to_dev(u0), K0, 2, 2, 1e300)
    assert np.all(lv == 0)
    coef, _ = mg.iterated_integrals(to_dev(dW), T, K0, 3)
    ref, flags, _ = mg.magnus_expmv(ops3, coef, to_dev(u0))
    torch.cuda.synchronize()
    assert rel(uT.cpu().numpy(), ref.cpu().numpy()) <= 1e-13
    # argument checks
    with pytest.raises(mg.MagnusError) as ex:
        mg.magnus_adaptive(ops2, ops3, to_dev(dW), T, to_dev(u0), 3, 2, 1, 1e-3)   # 3 !| 64
    assert ex.value.code == mg.MG_EINVAL
    with pytest.raises(mg.MagnusError) as ex:
        mg.magnus_adaptive(ops2, ops3, to_dev(dW), T, to_dev(u0), 4, 2, 5, 1e-3)   # 32 !| 16
    assert ex.value.code == mg.MG_EINVAL
    with pytest.raises(mg.MagnusError) as ex:
        mg.magnus_adaptive(ops3, ops3, to_dev(dW), T, to_dev(u0), 4, 2, 1, 1e-3)   # orders
    assert ex.value.code == mg.MG_EINVAL
    ops2.close()
    ops3.close()
