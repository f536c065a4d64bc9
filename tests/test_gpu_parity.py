"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle on
the same seeded inputs.

Tolerances (relative Frobenius per path, over the full grid):
  * Magnus FP64: 1e-10 (the target for the FP64 form);
  * Euler FP64 and the error norm: 1e-12 (same operations, other order);
  * integral weights: 1e-12 of the natural scale of each weight.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2207_09776_amd as mg
import workloads as wl
from oracle import errors, euler, exact, expmv, integrals, magnus, operators

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def setup_problem(nx, nv, lo, hi, coeffs, order):
    g = operators.Grid(nx, nv, lo, hi, lo, hi)
    B, A = operators.drift_and_noise(g, coeffs)
    basis = operators.magnus_basis(B, A)
    arrays = wl.sample_coefficients(coeffs, nx, nv, lo, hi, lo, hi)
    ops = mg.build_operators(nx, nv, lo, hi, lo, hi, arrays, order)
    return g, B, A, basis, ops


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


# ------------------------------------------------------------------ a2
@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("P,Nf,K", [(5, 768, 6), (3, 4096, 16), (2, 7, 7), (1, 3 * 1021, 3)])
def test_iterated_integrals_match_oracle(order, P, Nf, K):
    say(f"integrals order={order} P={P} Nf={Nf} K={K}")
    dW = wl.brownian_increments(100 + order, P, Nf)
    coef, ps = mg.iterated_integrals(to_dev(dW), 1.0, K, order)
    torch.cuda.synchronize()
    want = integrals.path_coefficients(dW, 1.0, K, order)
    h = 1.0 / K
    scale = np.array([h, math.sqrt(h), h, h ** 1.5, h * h, h ** 2.5])
    got = coef.cpu().numpy()
    assert np.all(np.abs(got - want) <= 1e-12 * scale + 1e-15)
    wps = integrals.path_statistics(dW, 1.0)
    np.testing.assert_allclose(ps.cpu().numpy(), wps, rtol=1e-12, atol=1e-13)


# ------------------------------------------------------------------ a3-a6
CASES = [
    # (name, nx, nv, lo, hi, order, P, K, Nf)
    ("ragged-24x24-m1", 24, 24, -5.0, 5.0, 1, 3, 4, 256),
    ("ragged-24x24-m2", 24, 24, -5.0, 5.0, 2, 3, 4, 256),
    ("ragged-24x24-m3", 24, 24, -5.0, 5.0, 3, 3, 4, 256),
    ("rect-40x56-m2", 40, 56, -5.0, 5.0, 2, 2, 3, 192),
    ("full-64x64-m3", 64, 64, -5.0, 5.0, 3, 2, 4, 512),
    ("ragged-100x100-m2", 100, 100, -6.0, 6.0, 2, 2, 4, 512),
    ("ragged-100x90-m3", 100, 90, -6.0, 6.0, 3, 1, 4, 512),
    ("c1-32x32-m1", 32, 32, -5.0, 5.0, 1, 1, 8, 2 ** 12),
    ("c1-32x32-m2", 32, 32, -5.0, 5.0, 2, 1, 8, 2 ** 12),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_magnus_expmv_matches_oracle(case):
    name, nx, nv, lo, hi, order, P, K, Nf = case
    say(f"magnus {name}")
    coeffs = wl.langevin_constant(1.0, 0.5)
    g, B, A, basis, ops = setup_problem(nx, nv, lo, hi, coeffs, order)
    dW = wl.brownian_increments(7, P, Nf)
    u0 = wl.gaussian_density(nx, nv, lo, hi, lo, hi, 0.25).reshape(-1)
    coef, _ = mg.iterated_integrals(to_dev(dW), 1.0, K, order)
    uT, flags, stats = mg.magnus_expmv(ops, coef, to_dev(u0), want_stats=True)
    torch.cuda.synchronize()
    got = uT.cpu().numpy()
    want = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW, 1.0, K, order), u0)
    for p in range(P):
        assert rel(got[p], want[p]) <= 1e-10, (name, p, rel(got[p], want[p]))
    assert int(flags.abs().sum()) == 0
    st = stats.cpu().numpy()
    assert np.all(st[..., 1] >= 1) and np.all(st[..., 0] >= 1)


def test_full_size_128_sampled_paths():
    """The 128x128 workload (1024 paths, m2, 16 steps, 2^14 increments) in the
    launch configuration the benchmark times; paths 0, 517 and 1023 are
    checked against the oracle one by one."""
    w = wl.WORKLOADS["const-128-p1024-m2-k16"]
    say(f"magnus full {w.name}")
    g, B, A, basis, ops = setup_problem(w.n, w.n, w.lo, w.hi, w.coefficients(), w.order)
    dW = wl.brownian_increments(w.seed, w.paths, w.Nf)
    u0 = wl.gaussian_density(w.n, w.n, w.lo, w.hi, w.lo, w.hi, w.s0sq).reshape(-1)
    coef, ps = mg.iterated_integrals(to_dev(dW), w.T, w.K, w.order)
    uT, flags, _ = mg.magnus_expmv(ops, coef, to_dev(u0))
    torch.cuda.synchronize()
    assert int(flags.abs().sum()) == 0
    for p in (0, 517, 1023):
        c = integrals.path_coefficients(dW[p:p + 1], w.T, w.K, w.order)[0]
        want = magnus.iterated_magnus(basis, c, u0)
        assert rel(uT[p].cpu().numpy(), want) <= 1e-10, p


def test_per_path_initial_values_and_single_step():
    say("magnus per-path u0, K=1")
    nx = nv = 20
    coeffs = wl.langevin_constant(1.0, 0.5)
    g, B, A, basis, ops = setup_problem(nx, nv, -4.0, 4.0, coeffs, 2)
    rng = np.random.default_rng(3)
    u0 = rng.random((2, nx * nv))
    dW = wl.brownian_increments(9, 2, 64)
    coef, _ = mg.iterated_integrals(to_dev(dW), 0.3, 1, 2)
    uT, _, _ = mg.magnus_expmv(ops, coef, to_dev(u0))
    torch.cuda.synchronize()
    c = integrals.path_coefficients(dW, 0.3, 1, 2)
    for p in range(2):
        want = expmv.expmv_dense(magnus.magnus_log(basis, c[p, 0]), u0[p])
        assert rel(uT[p].cpu().numpy(), want) <= 1e-10


def test_drift_only_equals_dense_exponential():
    """A = 0 (sigma^v = 0): exp(T B) u0 exactly (Remark 'determLangevin')."""
    say("magnus drift only")
    n = 16
    coeffs = wl.Coefficients(fx=lambda x, v: -v, gvv=lambda x, v: 1.0 + 0 * x)
    g, B, A, basis, ops = setup_problem(n, n, -3.0, 3.0, coeffs, 3)
    dW = wl.brownian_increments(4, 1, 128)
    u0 = wl.gaussian_density(n, n, -3, 3, -3, 3, 0.25).reshape(-1)
    coef, _ = mg.iterated_integrals(to_dev(dW), 0.7, 4, 3)
    uT, _, _ = mg.magnus_expmv(ops, coef, to_dev(u0))
    torch.cuda.synchronize()
    want = expmv.expmv_dense(0.7 * B, u0)
    assert rel(uT[0].cpu().numpy(), want) <= 1e-10


def test_zero_paths_is_noop_and_nonfinite_path_is_flagged():
    say("magnus P=0 and NaN path")
    n = 16
    coeffs = wl.langevin_constant(1.0, 0.5)
    g, B, A, basis, ops = setup_problem(n, n, -4.0, 4.0, coeffs, 2)
    empty = torch.empty((0, 4, 6), dtype=torch.float64, device=DEV)
    uT, flags, _ = mg.magnus_expmv(ops, empty, torch.ones(n * n, dtype=torch.float64, device=DEV))
    assert uT.shape == (0, n * n)
    dW = wl.brownian_increments(5, 3, 64)
    dW[1, 10] = np.nan
    u0 = wl.gaussian_density(n, n, -4, 4, -4, 4, 0.25).reshape(-1)
    coef, _ = mg.iterated_integrals(to_dev(dW), 1.0, 4, 2)
    uT, flags, _ = mg.magnus_expmv(ops, coef, to_dev(u0))
    torch.cuda.synchronize()
    f = flags.cpu().numpy()
    assert f[1] & mg.MG_FLAG_NONFINITE and f[0] == 0 and f[2] == 0
    good = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW[[0, 2]], 1.0, 4, 2), u0)
    assert rel(uT[0].cpu().numpy(), good[0]) <= 1e-10
    assert rel(uT[2].cpu().numpy(), good[1]) <= 1e-10


def test_unaligned_workspace_is_rejected():
    """A workspace must start on a 16-byte boundary (tables are read in
    16-byte units, the cooperative exchange uses 32- and 64-bit atomics): one
    that does not fails with MG_EINVAL before anything runs, for the resident
    and the cooperative Taylor kernels and for the cooperative Euler kernel;
    the output is left untouched."""
    say("unaligned workspace")
    coeffs = wl.langevin_constant(1.0, 0.5)
    for n in (32, 160):
        g, B, A, basis, ops = setup_problem(n, n, -4.0, 4.0, coeffs, 2)
        dW = wl.brownian_increments(5, 2, 64)
        coef, _ = mg.iterated_integrals(to_dev(dW), 1.0, 4, 2)
        u0 = torch.ones(n * n, dtype=torch.float64, device=DEV)
        need = mg.workspace_bytes(ops, 2, 4)
        ws = torch.empty(need + 64, dtype=torch.uint8, device=DEV)
        uT = torch.full((2, n * n), 7.0, dtype=torch.float64, device=DEV)
        with pytest.raises(mg.MagnusError) as ei:
            mg.magnus_expmv(ops, coef, u0, uT=uT, ws=ws[8:])
        assert ei.value.code == mg.MG_EINVAL, (n, ei.value)
        torch.cuda.synchronize()
        assert bool((uT == 7.0).all())
        # the aligned slice of the same buffer runs
        mg.magnus_expmv(ops, coef, u0, uT=uT, ws=ws[16:])
        torch.cuda.synchronize()
        assert bool(torch.isfinite(uT).all())
        if n > 128:
            ew = mg.euler_workspace_bytes(ops, 2)
            wse = torch.empty(ew + 64, dtype=torch.uint8, device=DEV)
            u = torch.ones((2, n * n), dtype=torch.float64, device=DEV)
            dWE = torch.zeros((2, 4), dtype=torch.float64, device=DEV)
            with pytest.raises(mg.MagnusError) as ei:
                mg.euler_step(ops, u, dWE, 1e-5, ws=wse[8:])
            assert ei.value.code == mg.MG_EINVAL


def test_repeat_runs_are_bitwise_identical():
    say("magnus determinism")
    n = 64
    coeffs = wl.langevin_constant(1.0, 0.5)
    g, B, A, basis, ops = setup_problem(n, n, -5.0, 5.0, coeffs, 2)
    dW = wl.brownian_increments(6, 8, 1024)
    u0 = to_dev(wl.gaussian_density(n, n, -5, 5, -5, 5, 0.25).reshape(-1))
    coef, _ = mg.iterated_integrals(to_dev(dW), 1.0, 8, 2)
    a, _, _ = mg.magnus_expmv(ops, coef, u0)
    b, _, _ = mg.magnus_expmv(ops, coef, u0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


# ------------------------------------------------------------------ a7
@pytest.mark.parametrize("nx,nv,NE,T,P", [(24, 24, 256, 1.0, 2), (100, 100, 256, 1.0, 2),
                                          (32, 32, 2 ** 12, 1.0, 2),
                                          # cooperative Euler (nx > 128); 9 groups are
                                          # not aligned to the 8 XCDs
                                          (200, 150, 128, 0.1, 2), (256, 256, 64, 0.02, 9),
                                          (512, 512, 32, 0.002, 1)])
def test_euler_matches_oracle(nx, nv, NE, T, P):
    """Step counts respect the explicit stability limit dt <~ dv^2 / a."""
    say(f"euler {nx}x{nv} NE={NE} P={P}")
    coeffs = wl.langevin_constant(1.0, 0.5)
    g, B, A, basis, ops = setup_problem(nx, nv, -5.0, 5.0, coeffs, 2)
    dW = wl.brownian_increments(8, P, NE * 2, T=T)
    dWE = integrals.euler_increments(dW, NE)
    u0 = wl.gaussian_density(nx, nv, -5, 5, -5, 5, 0.25).reshape(-1)
    u = to_dev(np.tile(u0, (P, 1)))
    flags = mg.euler_step(ops, u, to_dev(dWE), T / NE)
    torch.cuda.synchronize()
    want = euler.euler_paths(B, A, u0, dWE, T / NE)
    for p in range(P):
        assert rel(u[p].cpu().numpy(), want[p]) <= 1e-12
    assert int(flags.abs().sum()) == 0


# ------------------------------------------------------------------ a8
@pytest.mark.parametrize("kappa", [0, 1, 2])
def test_error_vs_exact_matches_oracle(kappa):
    say(f"error kappa={kappa}")
    n = 48
    g = operators.Grid(n, n, -5.0, 5.0, -5.0, 5.0)
    P = 3
    rng = np.random.default_rng(kappa)
    ps = np.stack([rng.normal(size=P), 0.3 * rng.normal(size=P)], axis=1)
    u = np.stack([exact.solution_on_grid(g, 1.0, 1.0, 0.5, 0.25, ps[p, 0], ps[p, 1])
                  * (1 + 0.01 * rng.normal(size=n * n)) for p in range(P)])
    err = mg.error_vs_exact(mg.mg_grid(n, n, -5.0, 5.0, -5.0, 5.0), to_dev(u), pathstat=to_dev(ps),
                            a=1.0, sigma=0.5, s0sq=0.25, T=1.0, kappa=kappa)
    ref = to_dev(u[::-1].copy())
    err2 = mg.error_vs_exact(mg.mg_grid(n, n, -5.0, 5.0, -5.0, 5.0), to_dev(u), uref=ref,
                             kappa=kappa)
    torch.cuda.synchronize()
    for p in range(P):
        uex = exact.solution_on_grid(g, 1.0, 1.0, 0.5, 0.25, ps[p, 0], ps[p, 1])
        assert abs(err[p].item() - errors.relative_error(uex.reshape(n, n), u[p].reshape(n, n), kappa)) <= 1e-12
        want2 = errors.relative_error(u[P - 1 - p].reshape(n, n), u[p].reshape(n, n), kappa)
        assert abs(err2[p].item() - want2) <= 1e-12 * max(want2, 1e-3)


# ------------------------------------------------------------------ FP32C
F32_CASES = [
    ("f32c-24x24-m2", 24, 24, -5.0, 5.0, 2, 3, 4, 256),
    ("f32c-64x64-m3", 64, 64, -5.0, 5.0, 3, 2, 8, 512),
    ("f32c-100x90-m2", 100, 90, -6.0, 6.0, 2, 2, 8, 512),
    ("f32c-128x128-m2", 128, 128, -6.0, 6.0, 2, 2, 16, 2 ** 14),
]


@pytest.mark.parametrize("case", F32_CASES, ids=[c[0] for c in F32_CASES])
def test_fp32c_matches_oracle(case):
    """Compensated FP32 form: within 1e-5 relative of the FP64 oracle."""
    name, nx, nv, lo, hi, order, P, K, Nf = case
    say(f"magnus {name}")
    coeffs = wl.langevin_constant(1.0, 0.5)
    g, B, A, basis, ops = setup_problem(nx, nv, lo, hi, coeffs, order)
    dW = wl.brownian_increments(17, P, Nf)
    u0 = wl.gaussian_density(nx, nv, lo, hi, lo, hi, 0.25).reshape(-1)
    coef, _ = mg.iterated_integrals(to_dev(dW), 1.0, K, order)
    uT, flags, stats = mg.magnus_expmv(ops, coef, to_dev(u0), precision="fp32c", want_stats=True)
    u64, _, st64 = mg.magnus_expmv(ops, coef, to_dev(u0), want_stats=True)
    torch.cuda.synchronize()
    want = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW, 1.0, K, order), u0)
    for p in range(P):
        assert rel(uT[p].cpu().numpy(), want[p]) <= 1e-5, (name, p, rel(uT[p].cpu().numpy(), want[p]))
    assert int(flags.abs().sum()) == 0
    # the 2^-24 tolerance needs no more Taylor terms than 2^-53
    assert int(stats[..., 0].sum()) <= int(st64[..., 0].sum())


# ------------------------------------------------------------------ cooperative (nx > 128)
COOP_CASES = [
    # (name, nx, nv, lo, hi, order, P, K, Nf, T, precision, tol)
    ("coop-256x256-m2-f64", 256, 256, -5.0, 5.0, 2, 3, 2, 256, 0.25, "fp64", 1e-10),
    ("coop-256x256-m3-f64", 256, 256, -5.0, 5.0, 3, 2, 2, 256, 0.25, "fp64", 1e-10),
    ("coop-200x150-m2-f64", 200, 150, -5.0, 5.0, 2, 2, 2, 256, 0.25, "fp64", 1e-10),
    # FP64 between 256 and 384 points per row: 5 and 6 points per lane, the
    # last lane partly empty; order 3 and a ragged last slab
    ("coop-300x100-m3-f64", 300, 100, -5.0, 5.0, 3, 2, 2, 256, 0.05, "fp64", 1e-10),
    ("coop-350x90-m2-f64", 350, 90, -5.0, 5.0, 2, 2, 2, 256, 0.05, "fp64", 1e-10),
    ("coop-384x70-m3-f64", 384, 70, -5.0, 5.0, 3, 2, 2, 256, 0.05, "fp64", 1e-10),
    ("coop-256x256-m2-f32c", 256, 256, -5.0, 5.0, 2, 3, 2, 256, 0.25, "fp32c", 1e-5),
    ("coop-512x512-m2-f32c", 512, 512, -5.0, 5.0, 2, 1, 1, 64, 0.05, "fp32c", 1e-5),
    # nx > 512: workgroups of 24 rows; 520 leaves most of the last lane's 16
    # points empty, and 40 and 60 rows leave the last slab part empty
    ("coop-520x40-m2-f32c", 520, 40, -5.0, 5.0, 2, 2, 2, 256, 0.05, "fp32c", 1e-5),
    ("coop-1024x60-m3-f32c", 1024, 60, -5.0, 5.0, 3, 2, 2, 256, 0.02, "fp32c", 1e-5),
    # FP64 above 512 points: workgroups of 2 rows x 4 waves, up to 128 per path
    ("coop-520x40-m2-f64", 520, 40, -5.0, 5.0, 2, 2, 2, 256, 0.05, "fp64", 1e-10),
    ("coop-1024x60-m3-f64", 1024, 60, -5.0, 5.0, 3, 2, 2, 256, 0.02, "fp64", 1e-10),
    ("coop-700x1021-m2-f64", 700, 1021, -5.0, 5.0, 2, 1, 1, 64, 0.002, "fp64", 1e-10),
    # 8 paths: the plan places 8 groups, each on one XCD, and the members
    # exchange through that XCD's L2 (the other cases use agent scope)
    ("coop-256x256-m2-f64-p8", 256, 256, -5.0, 5.0, 2, 8, 2, 256, 0.05, "fp64", 1e-10),
    ("coop-256x256-m2-f32c-p8", 256, 256, -5.0, 5.0, 2, 8, 2, 256, 0.05, "fp32c", 1e-5),
]


@pytest.mark.parametrize("case", COOP_CASES, ids=[c[0] for c in COOP_CASES])
def test_coop_matches_oracle(case):
    name, nx, nv, lo, hi, order, P, K, Nf, T, prec, tol = case
    say(f"magnus {name}")
    coeffs = wl.langevin_constant(1.0, 0.5)
    g, B, A, basis, ops = setup_problem(nx, nv, lo, hi, coeffs, order)
    dW = wl.brownian_increments(23, P, Nf, T=T)
    u0 = wl.gaussian_density(nx, nv, lo, hi, lo, hi, 0.25).reshape(-1)
    coef, _ = mg.iterated_integrals(to_dev(dW), T, K, order)
    uT, flags, stats = mg.magnus_expmv(ops, coef, to_dev(u0), precision=prec, want_stats=True)
    torch.cuda.synchronize()
    assert int(flags.abs().sum()) == 0, flags.cpu().numpy()
    want = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW, T, K, order), u0)
    for p in range(P):
        e = rel(uT[p].cpu().numpy(), want[p])
        assert e <= tol, (name, p, e)


def test_full_size_256_fp32c_sampled_path():
    """The 256x256 workload (4096 paths, m3, 32 steps, compensated FP32) in
    the configuration the benchmark would run; path 1234 is checked against
    the FP64 oracle (1e-5)."""
    w = wl.WORKLOADS["const-256-p4096-m3-k32"]
    say(f"magnus full {w.name}")
    g, B, A, basis, ops = setup_problem(w.n, w.n, w.lo, w.hi, w.coefficients(), w.order)
    dW = wl.brownian_increments(w.seed, w.paths, w.Nf)
    u0 = wl.gaussian_density(w.n, w.n, w.lo, w.hi, w.lo, w.hi, w.s0sq).reshape(-1)
    coef, _ = mg.iterated_integrals(to_dev(dW), w.T, w.K, w.order)
    uT, flags, _ = mg.magnus_expmv(ops, coef, to_dev(u0), precision="fp32c")
    torch.cuda.synchronize()
    # no path is non-finite or aborted; the one whose last step leaves the
    # convergence region (path 3119, tests/test_negative_flag.py) is flagged
    f = flags.cpu().numpy()
    assert np.all((f & ~mg.MG_FLAG_NEGATIVE) == 0)
    assert np.nonzero(f)[0].tolist() == [3119]
    p = 1234
    c = integrals.path_coefficients(dW[p:p + 1], w.T, w.K, w.order)[0]
    want = magnus.iterated_magnus(basis, c, u0)
    assert rel(uT[p].cpu().numpy(), want) <= 1e-5


# ------------------------------------------------------------------ several batches in one call
def test_multi_job_call_matches_single_calls_and_oracle():
    """Three batches of different sizes and forms in one mg_magnus_expmv_multi
    call: each equals its own mg_magnus_expmv call bitwise and the oracle
    within the tolerance of its form."""
    say("magnus multi-job")
    specs = [  # (nx, nv, order, P, K, Nf, T, precision, tol)
        (32, 32, 2, 2, 4, 256, 1.0, "fp64", 1e-10),
        (64, 64, 3, 3, 8, 512, 1.0, "fp32c", 1e-5),
        (200, 150, 2, 1, 2, 256, 0.25, "fp64", 1e-10),
    ]
    coeffs = wl.langevin_constant(1.0, 0.5)
    jobs, refs = [], []
    for i, (nx, nv, order, P, K, Nf, T, prec, tol) in enumerate(specs):
        g, B, A, basis, ops = setup_problem(nx, nv, -5.0, 5.0, coeffs, order)
        dW = wl.brownian_increments(40 + i, P, Nf, T=T)
        u0 = wl.gaussian_density(nx, nv, -5, 5, -5, 5, 0.25).reshape(-1)
        coef, _ = mg.iterated_integrals(to_dev(dW), T, K, order)
        jobs.append({"ops": ops, "coef": coef, "u0": to_dev(u0), "precision": prec,
                     "want_stats": True})
        want = magnus.iterated_magnus_paths(basis, integrals.path_coefficients(dW, T, K, order), u0)
        single, _, _ = mg.magnus_expmv(ops, coef, to_dev(u0), precision=prec)
        refs.append((want, single, tol))
    out = mg.magnus_expmv_multi(jobs)
    torch.cuda.synchronize()
    for (uT, flags, stats), (want, single, tol) in zip(out, refs):
        assert int(flags.abs().sum()) == 0
        assert torch.equal(uT, single)
        for p in range(uT.shape[0]):
            assert rel(uT[p].cpu().numpy(), want[p]) <= tol


def test_multi_job_invalid_job_launches_nothing():
    say("magnus multi-job invalid")
    coeffs = wl.langevin_constant(1.0, 0.5)
    g, B, A, basis, ops = setup_problem(24, 24, -5.0, 5.0, coeffs, 2)
    dW = wl.brownian_increments(3, 2, 64)
    coef, _ = mg.iterated_integrals(to_dev(dW), 1.0, 4, 2)
    u0 = to_dev(wl.gaussian_density(24, 24, -5, 5, -5, 5, 0.25).reshape(-1))
    sentinel = torch.full((2, 24 * 24), float("nan"), dtype=torch.float64, device=DEV)
    bad = torch.zeros((2, 4, 6), dtype=torch.float64, device=DEV)
    jobs = [{"ops": ops, "coef": coef, "u0": u0, "uT": sentinel},
            {"ops": ops, "coef": bad, "u0": u0, "precision": "fp64", "tol": 2.0}]   # tol >= 1
    with pytest.raises(mg.MagnusError) as ei:
        mg.magnus_expmv_multi(jobs)
    torch.cuda.synchronize()
    assert ei.value.code == mg.MG_EINVAL and "job 1" in str(ei.value)
    assert bool(torch.isnan(sentinel).all())


def test_full_size_mixed_groups():
    """The mixed-size workload (64^2 x 2048, 256^2 x 512, 1024^2 x 64 paths,
    FP32C) in one mg_magnus_expmv_multi call, as the benchmark runs it.
    Sampled 64^2 paths against the oracle (1e-5); the larger grids, whose
    paths the oracle cannot afford, through properties: finite results and a
    median error against the closed form below a few times the second-order
    discretisation error of the grid (the oracle gives 9.2e-4 at 256^2; scaled
    by dx^2, 5.8e-5 at 1024^2), far below the O(1) error of a wrong operator
    or sum.  (The median: single rough paths can have larger Magnus errors.)"""
    w = wl.WORKLOADS["mixed-64-256-1024-m2-fp32c"]
    say(f"magnus full {w.name}")
    coeffs = w.coefficients()
    jobs, groups = [], []
    for (n, paths, K, seed) in w.extra:
        g, B, A, basis, ops = setup_problem(n, n, w.lo, w.hi, coeffs, w.order)
        dW = wl.brownian_increments(seed, paths, w.Nf)
        u0 = wl.gaussian_density(n, n, w.lo, w.hi, w.lo, w.hi, w.s0sq).reshape(-1)
        coef, ps = mg.iterated_integrals(to_dev(dW), w.T, K, w.order)
        jobs.append({"ops": ops, "coef": coef, "u0": to_dev(u0), "precision": "fp32c"})
        groups.append((n, K, dW, u0, basis, ops, ps))
    out = mg.magnus_expmv_multi(jobs)
    torch.cuda.synchronize()
    bounds = {256: 2e-3, 1024: 2e-4}
    for (n, K, dW, u0, basis, ops, ps), (uT, flags, _) in zip(groups, out):
        assert int(flags.abs().sum()) == 0, n
        assert bool(torch.isfinite(uT).all()), n
        if n == 64:
            for p in (0, 1000, 2047):
                c = integrals.path_coefficients(dW[p:p + 1], w.T, K, w.order)[0]
                want = magnus.iterated_magnus(basis, c, u0)
                assert rel(uT[p].cpu().numpy(), want) <= 1e-5, p
        else:
            err = mg.error_vs_exact(ops, uT, pathstat=ps, a=w.a, sigma=w.sigma, s0sq=w.s0sq, T=w.T)
            torch.cuda.synchronize()
            med = float(err.median())
            say(f"  {n}^2 median error vs closed form {med:.3e}, mean {float(err.mean()):.3e}")
            assert med <= bounds[n], (n, med)
