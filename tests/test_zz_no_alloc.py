"""mg_magnus_expmv_noalloc (the entry point for callers that cannot allocate
device memory) against mg_magnus_expmv through the C ABI.

Both calls run the same kernels on the same inputs, so the results, Taylor
statistics and flags must agree bit for bit (stronger than the 1e-10 / 1e-5
parity bar).  Two calls in a row share the library's scratch array, the
second with a smaller input, for a grid of the register-resident kernel and
one of the cooperative kernel; a call whose workspace exceeds the array is
refused before anything runs.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2207_09776_amd as mg
import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ops(n, m, order):
    lo, hi = -5.0, 5.0
    coeffs = wl.sample_coefficients(wl.langevin_constant(1.0, 0.5), n, m, lo, hi, lo, hi)
    return mg.build_operators(n, m, lo, hi, lo, hi, coeffs, order)


def _inputs(n, m, P, K, order, seed, per_path):
    dW = torch.from_numpy(wl.brownian_increments(seed, P, 8 * K, T=0.02)).to(DEV)
    coef, _ = mg.iterated_integrals(dW, 0.02, K, order)
    if per_path:
        u0 = np.random.default_rng(seed + 1).uniform(0.5, 1.5, size=(P, n * m))
    else:
        u0 = wl.gaussian_density(n, m, -5.0, 5.0, -5.0, 5.0, 0.25).reshape(-1)
    return coef, torch.from_numpy(np.ascontiguousarray(u0)).to(DEV)


def _compare(ops, coef, u0, precision, what):
    P, K, _ = coef.shape
    N = ops.grid.nx * ops.grid.nv
    want, wflags, wstats = mg.magnus_expmv(ops, coef, u0, precision=precision, want_stats=True)
    uT = torch.full((P, N), float("nan"), dtype=torch.float64, device=DEV)
    flags = torch.full((P,), -1, dtype=torch.int32, device=DEV)
    stats = torch.full((P, K, 2), -1, dtype=torch.int32, device=DEV)
    mg.magnus_expmv_noalloc(ops, coef, u0, uT, flags=flags, stats=stats, precision=precision)
    torch.cuda.synchronize()
    assert int(wflags.abs().sum()) == 0, what
    assert torch.equal(uT, want), (what, float((uT - want).abs().max()))
    assert torch.equal(flags, wflags), what
    assert torch.equal(stats, wstats), what


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_noalloc_resident_two_calls(precision):
    """48x40 then 24x20 (register-resident kernel): the second call is smaller
    and reuses the scratch array the first one filled."""
    say(f"noalloc resident {precision}")
    ops1 = _ops(48, 40, 2)
    coef1, u01 = _inputs(48, 40, 6, 4, 2, 301, True)
    _compare(ops1, coef1, u01, precision, "48x40")
    ops2 = _ops(24, 20, 3)
    coef2, u02 = _inputs(24, 20, 3, 2, 3, 302, False)
    _compare(ops2, coef2, u02, precision, "24x20")
    ops1.close()
    ops2.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_noalloc_cooperative_two_calls(precision):
    """200x150 then 160x136 (cooperative kernel, exchange area in the scratch
    array; its counters are cleared by each launch)."""
    say(f"noalloc cooperative {precision}")
    ops1 = _ops(200, 150, 2)
    coef1, u01 = _inputs(200, 150, 4, 2, 2, 311, True)
    _compare(ops1, coef1, u01, precision, "200x150")
    ops2 = _ops(160, 136, 2)
    coef2, u02 = _inputs(160, 136, 2, 2, 2, 312, False)
    _compare(ops2, coef2, u02, precision, "160x136")
    ops1.close()
    ops2.close()


def test_noalloc_refuses_a_workspace_beyond_the_scratch_array():
    """128^2 with 1024 paths x 16 steps needs about 135 MB of tables: refused
    with MG_ENOMEM on the host, the output left untouched."""
    say("noalloc limit")
    ops = _ops(128, 128, 2)
    P, K = 1024, 16
    need = mg.workspace_bytes(ops, P, K)
    assert need > mg.NOALLOC_SCRATCH_BYTES
    coef = torch.zeros((P, K, 6), dtype=torch.float64, device=DEV)
    u0 = torch.zeros(128 * 128, dtype=torch.float64, device=DEV)
    uT = torch.full((P, 128 * 128), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(mg.MagnusError) as ex:
        mg.magnus_expmv_noalloc(ops, coef, u0, uT)
    assert ex.value.code == mg.MG_ENOMEM
    assert "scratch" in str(ex.value)
    torch.cuda.synchronize()
    assert bool((uT == 7.0).all())
    ops.close()
