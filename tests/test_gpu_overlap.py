"""The cooperative Taylor kernel with the overlapped group exchange (bit 1 of
the cooperative kernel variants the autotuner times; the library's default
for operators without x-terms where it spills no more than the two-barrier
kernel): each wave bumps its own
counter and polls its group while it computes the rows that read no halo
row, then loads the halo rows and the norms; the rows are computed in the
segmented order (rows RH .. RJ-1 first).  The arithmetic per point and the
stop decisions are those of variant 0 (the two-barrier exchange), so the
results must be equal bit for bit, and within 1e-10 (FP64) or 1e-5 (FP32C)
of the CPU oracle.

The data reach every edge (uniform random u0, short horizons), so an error in
the halo rows, in the kept rows of the segmented order or in the stop rule
shows in the max-norm.  The variants are selected the way a serving process
would: the autotuner's choice is written to a cache file, edited, loaded and
applied by mg_build_operators.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2207_09776_amd as mg
import workloads as wl
from oracle import integrals, magnus, operators

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
OVL = 2   # the overlapped-exchange bit of the cooperative variants

SETS = {
    "const": lambda: wl.langevin_constant(1.0, 0.5),
    "xfactors": wl.langevin_variable_sigma_beta,           # x-dependent factors
    "xterms": lambda: wl.langevin_paper_variable(1.1, 0.3),  # x-terms at order 3
}

CASES = [
    # (name, nx, nv, set, order, P, K, Nf, T, precision, tol)
    ("256x256-m3-f64", 256, 256, "const", 3, 2, 2, 256, 0.02, "fp64", 1e-10),
    ("200x150-m2-f64", 200, 150, "const", 2, 2, 2, 256, 0.02, "fp64", 1e-10),
    ("300x100-m3-f64", 300, 100, "const", 3, 2, 2, 256, 0.01, "fp64", 1e-10),
    ("384x70-m2-f64", 384, 70, "const", 2, 2, 2, 256, 0.01, "fp64", 1e-10),
    ("450x64-m2-f64", 450, 64, "const", 2, 2, 2, 256, 0.01, "fp64", 1e-10),
    ("520x40-m2-f32c", 520, 40, "const", 2, 2, 2, 256, 0.005, "fp32c", 1e-5),
    ("1024x60-m3-f32c", 1024, 60, "const", 3, 1, 2, 256, 0.002, "fp32c", 1e-5),
    ("200x150-xfactors-m2-f64", 200, 150, "xfactors", 2, 2, 2, 256, 0.01, "fp64", 1e-10),
    ("200x150-xterms-m3-f64", 200, 150, "xterms", 3, 2, 2, 256, 0.005, "fp64", 1e-10),
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def set_cached_variant(path, nx, nv, prec, order, variant):
    """Edit the cooperative entries of (nx, nv, precision, order) in a saved
    cache (operators of other coefficient forms with this key included)."""
    lines = path.read_text().splitlines()
    out, hits = [lines[0]], 0
    for ln in lines[1:]:
        f = ln.split()
        if (len(f) == 18 and int(f[1]) == nx and int(f[2]) == nv and
                int(f[3]) == mg.PRECISIONS[prec] and int(f[4]) == order and f[14] == "1"):
            f[15] = str(variant)
            hits += 1
        out.append(" ".join(f))
    path.write_text("\n".join(out) + "\n")
    return hits


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_overlapped_exchange_matches_default_and_oracle(case, tmp_path):
    name, nx, nv, cset, order, P, K, Nf, T, prec, tol = case
    say(f"overlapped exchange {name}")
    lo, hi = -5.0, 5.0
    coeffs = SETS[cset]()
    arrays = wl.sample_coefficients(coeffs, nx, nv, lo, hi, lo, hi)

    def build():
        return mg.build_operators(nx, nv, lo, hi, lo, hi, arrays, order)

    dW = wl.brownian_increments(301, P, Nf, T=T)
    u0 = np.random.default_rng(302).uniform(0.5, 1.5, size=(P, nx * nv))
    coef, _ = mg.iterated_integrals(to_dev(dW), T, K, order)
    u0d = to_dev(u0)
    ops = build()
    # the autotuner times every variant and excludes any that differs bitwise
    # from the default-shape kernel without the overlapped exchange
    rep = mg.autotune_expmv(ops, coef, u0d, precision=prec, reps=1)
    say(f"  {rep}")
    assert f"variant {OVL} " in rep, rep
    assert "differs" not in rep, rep
    ops.close()
    cache = tmp_path / "cache.txt"
    mg.autotune_cache_save(str(cache))
    try:
        # the reference: variant 0 (the kernel with the two-barrier exchange)
        assert set_cached_variant(cache, nx, nv, prec, order, 0) >= 1
        mg.autotune_cache_load(str(cache))
        ops = build()
        ref, rflags, rstats = mg.magnus_expmv(ops, coef, u0d, precision=prec, want_stats=True)
        torch.cuda.synchronize()
        # rough data may dip below zero (the positivity flag); nothing else
        assert int((rflags & ~mg.MG_FLAG_NEGATIVE).abs().sum()) == 0
        ops.close()
        set_cached_variant(cache, nx, nv, prec, order, OVL)
        mg.autotune_cache_load(str(cache))
        ops = build()
        uT, flags, stats = mg.magnus_expmv(ops, coef, u0d, precision=prec, want_stats=True)
        torch.cuda.synchronize()
        assert torch.equal(flags, rflags)
        got, want0 = uT.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want0.view(np.uint64)), name
        assert torch.equal(stats, rstats)
        want = magnus.iterated_magnus_paths(
            operators.magnus_basis(*operators.drift_and_noise(
                operators.Grid(nx, nv, lo, hi, lo, hi), coeffs)),
            integrals.path_coefficients(dW, T, K, order), u0)
        for p in range(P):
            fro = np.linalg.norm(got[p] - want[p]) / np.linalg.norm(want[p])
            mx = np.abs(got[p] - want[p]).max() / np.abs(want[p]).max()
            assert fro <= tol and mx <= tol, (name, p, fro, mx)
        ops.close()
    finally:
        # later operators of this key take the overlapped exchange only
        # where it is the default (no x-dependent parts)
        set_cached_variant(cache, nx, nv, prec, order, OVL if cset == "const" else 0)
        mg.autotune_cache_load(str(cache))
