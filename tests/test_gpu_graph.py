"""The hot path captured in a HIP graph (torch.cuda.CUDAGraph over the C ABI
calls, as the benchmark replays it): every replay, with eager work of the
program between replays, reproduces the eager result bit for bit."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2207_09776_amd as mg
import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def test_graph_replays_match_eager():
    print("graph replay 64x64 P=8 K=4", flush=True)
    sys.stdout.flush()
    n, P, K, Nf = 64, 8, 4, 256
    c = wl.langevin_constant(1.0, 0.5)
    ops = mg.build_operators(n, n, -5, 5, -5, 5, wl.sample_coefficients(c, n, n, -5, 5, -5, 5), 2)
    u0 = torch.from_numpy(wl.gaussian_density(n, n, -5, 5, -5, 5, 0.25).reshape(-1)).to(DEV)
    dW = torch.from_numpy(wl.brownian_increments(41, P, Nf)).to(DEV)
    coef = torch.empty((P, K, 6), dtype=torch.float64, device=DEV)
    ps = torch.empty((P, 2), dtype=torch.float64, device=DEV)
    uT = torch.empty((P, n * n), dtype=torch.float64, device=DEV)
    err = torch.empty(P, dtype=torch.float64, device=DEV)
    ws = torch.empty(mg.workspace_bytes(ops, P, K), dtype=torch.uint8, device=DEV)

    def step():
        mg.iterated_integrals(dW, 1.0, K, 2, coef=coef, pathstat=ps)
        mg.magnus_expmv(ops, coef, u0, uT=uT, ws=ws)
        mg.error_vs_exact(ops, uT, pathstat=ps, a=1.0, sigma=0.5, s0sq=0.25, T=1.0, err=err)

    step()
    torch.cuda.synchronize()
    want_u, want_e = uT.clone(), err.clone()
    assert bool(torch.isfinite(want_u).all())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    other = torch.from_numpy(wl.brownian_increments(43, P, Nf)).to(DEV)
    for r in range(3):
        uT.zero_()
        err.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(uT, want_u), r
        assert torch.equal(err, want_e), r
        # eager work between replays: another batch through the same library
        cf, _ = mg.iterated_integrals(other, 1.0, K, 2)
        u2, fl, _ = mg.magnus_expmv(ops, cf, u0)
        torch.cuda.synchronize()
        assert int(fl.abs().sum()) == 0


@pytest.mark.parametrize("n,prec", [(128, "fp64"), (128, "fp32c"), (64, "fp64"), (64, "fp32c"),
                                    (256, "fp64"), (400, "fp32c")])
def test_autotune_keeps_results(n, prec):
    """mg_autotune_expmv times the kernel shapes of the grid (register-resident
    shapes up to 128^2, cooperative workgroup shapes above) and records one;
    results after tuning equal those before bit for bit (every shape applies
    the same operations in the same order; the tuner's own bitwise check
    excludes a shape that does not)."""
    print(f"autotune {n}^2 {prec}", flush=True)
    # cooperative grids: a horizon inside the convergence region of two
    # Magnus steps (T = 1 would overflow on the finer grids)
    P, K, Nf, T = (32, 4, 256, 1.0) if n <= 128 else (8, 2, 256, 0.01)
    c = wl.langevin_constant(1.0, 0.5)
    ops = mg.build_operators(n, n, -5, 5, -5, 5, wl.sample_coefficients(c, n, n, -5, 5, -5, 5), 2)
    u0 = torch.from_numpy(wl.gaussian_density(n, n, -5, 5, -5, 5, 0.25).reshape(-1)).to(DEV)
    dW = torch.from_numpy(wl.brownian_increments(47, P, Nf, T=T)).to(DEV)
    coef, _ = mg.iterated_integrals(dW, T, K, 2)
    before, fl, _ = mg.magnus_expmv(ops, coef, u0, precision=prec)
    torch.cuda.synchronize()
    before = before.clone()
    rep = mg.autotune_expmv(ops, coef, u0, precision=prec, reps=2)
    print(rep, flush=True)
    assert "chosen" in rep and "differs" not in rep, rep
    after, fl2, _ = mg.magnus_expmv(ops, coef, u0, precision=prec)
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    assert int(fl.abs().sum()) == 0 and int(fl2.abs().sum()) == 0


def test_autotune_cache_records_the_choice(tmp_path):
    """The shape the autotuner picks enters the library's cache, which save
    writes out and load reads back."""
    print("autotune cache", flush=True)
    n, P, K = 256, 8, 2
    c = wl.langevin_constant(1.0, 0.5)
    ops = mg.build_operators(n, n, -5, 5, -5, 5, wl.sample_coefficients(c, n, n, -5, 5, -5, 5), 3)
    u0 = torch.from_numpy(wl.gaussian_density(n, n, -5, 5, -5, 5, 0.25).reshape(-1)).to(DEV)
    dW = torch.from_numpy(wl.brownian_increments(48, P, 256, T=0.05)).to(DEV)
    coef, _ = mg.iterated_integrals(dW, 0.05, K, 3)
    rep = mg.autotune_expmv(ops, coef, u0, precision="fp64", reps=2)
    print(rep, flush=True)
    assert "chosen variant" in rep, rep
    chosen = int(rep.rsplit("chosen variant", 1)[1].split()[0])
    path = tmp_path / "cache.txt"
    assert mg.autotune_cache_save(str(path)) >= 1
    lines = path.read_text().splitlines()
    assert lines[0] == "mg-autotune-cache 1"
    key = f" {n} {n} 0 3 "
    mine = [l for l in lines[1:] if key in l]
    assert mine and mine[-1].split()[-4:] == ["1", str(chosen), "0", "0"], (mine, chosen)
    assert mg.autotune_cache_load(str(path)) == len(lines) - 1
    ops.close()


def test_graph_replays_cooperative_and_multi_job():
    """Cooperative launches (256^2, FP32C) and a multi-job call (a resident
    and a cooperative batch) captured in one graph: every replay, with eager
    work between replays, equals the eager result bit for bit."""
    print("graph replay cooperative + multi-job", flush=True)
    c = wl.langevin_constant(1.0, 0.5)
    batches = []
    for (n, P, K, T) in ((256, 8, 2, 0.05), (64, 16, 4, 1.0)):
        ops = mg.build_operators(n, n, -5, 5, -5, 5, wl.sample_coefficients(c, n, n, -5, 5, -5, 5),
                                 2)
        u0 = torch.from_numpy(wl.gaussian_density(n, n, -5, 5, -5, 5, 0.25).reshape(-1)).to(DEV)
        dW = torch.from_numpy(wl.brownian_increments(51, P, 256, T=T)).to(DEV)
        coef, _ = mg.iterated_integrals(dW, T, K, 2)
        uT = torch.empty((P, n * n), dtype=torch.float64, device=DEV)
        batches.append(dict(ops=ops, coef=coef, u0=u0, uT=uT, precision="fp32c"))
    b0 = batches[0]
    ws0 = torch.empty(mg.workspace_bytes(b0["ops"], 8, 2, "fp32c"), dtype=torch.uint8, device=DEV)
    uT_m = [torch.empty_like(b["uT"]) for b in batches]
    jobs = [dict(b, uT=u) for b, u in zip(batches, uT_m)]
    # the multi-job workspace: each job's slice rounded up to 256 bytes
    need = sum((mg.workspace_bytes(j["ops"], j["coef"].shape[0], j["coef"].shape[1], "fp32c")
                + 255) // 256 * 256 for j in jobs)
    wsm = torch.empty(need, dtype=torch.uint8, device=DEV)

    def step():
        mg.magnus_expmv(b0["ops"], b0["coef"], b0["u0"], precision="fp32c", uT=b0["uT"], ws=ws0)
        mg.magnus_expmv_multi(jobs, ws=wsm)

    step()
    torch.cuda.synchronize()
    want = [b0["uT"].clone()] + [u.clone() for u in uT_m]
    assert all(bool(torch.isfinite(x).all()) for x in want)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for r in range(3):
        for x in [b0["uT"]] + uT_m:
            x.zero_()
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip([b0["uT"]] + uT_m, want):
            assert torch.equal(x, y), r
        # eager work between replays
        u2, fl, _ = mg.magnus_expmv(b0["ops"], b0["coef"], b0["u0"], precision="fp32c")
        torch.cuda.synchronize()
        assert int(fl.abs().sum()) == 0


def test_graph_replays_per_path_step_counts():
    """The per-path batch (weights with a step count per path, zero steps
    after it, one Taylor launch at K = Kmax) captured in a graph: every
    replay equals the eager result bit for bit, on a resident and a
    cooperative grid."""
    print("graph replay per-path step counts", flush=True)
    P, Nf, Kmax = 4, 256, 16
    Kp = torch.tensor([4, 16, 2, 8], dtype=torch.int32, device=DEV)
    dW = torch.from_numpy(wl.brownian_increments(53, P, Nf)).to(DEV)
    c = wl.langevin_constant(1.0, 0.5)
    for n, prec, T in ((48, "fp64", 1.0), (160, "fp32c", 0.05)):
        ops = mg.build_operators(n, n, -4, 4, -4, 4, wl.sample_coefficients(c, n, n, -4, 4, -4, 4), 2)
        u0 = torch.from_numpy(wl.gaussian_density(n, n, -4, 4, -4, 4, 0.25).reshape(-1)).to(DEV)
        coef = torch.empty((P, Kmax, 6), dtype=torch.float64, device=DEV)
        ps = torch.empty((P, 2), dtype=torch.float64, device=DEV)
        uT = torch.empty((P, n * n), dtype=torch.float64, device=DEV)
        ws = torch.empty(mg.workspace_bytes(ops, P, Kmax, prec), dtype=torch.uint8, device=DEV)

        def step():
            mg.iterated_integrals_steps(dW, T, Kp, Kmax, 2, coef=coef, pathstat=ps)
            mg.magnus_expmv(ops, coef, u0, precision=prec, uT=uT, ws=ws)

        step()
        torch.cuda.synchronize()
        want = uT.clone()
        assert bool(torch.isfinite(want).all())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        for r in range(3):
            uT.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(uT, want), (n, r)
            # eager work between replays
            cf, _ = mg.iterated_integrals(dW, T, 4, 2)
            _, fl, _ = mg.magnus_expmv(ops, cf, u0, precision=prec)
            torch.cuda.synchronize()
            assert int(fl.abs().sum()) == 0
