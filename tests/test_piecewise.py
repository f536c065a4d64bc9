"""Coefficients piecewise constant in time (Remark piecewise): the time
interval is cut where the coefficients change and the constant-coefficient
scheme runs on each piece, the terminal value of one piece being the initial
value of the next.

On the GPU a piece is one mg_iterated_integrals call on that piece's fine
increments and one mg_magnus_expmv call with that piece's operators, its uT
passed as the next call's u0.  The CPU tests pin the oracle's composition:
with no noise each piece is exactly exp(T_piece B_piece) (Remark
determLangevin), so the whole run is the ordered product of dense matrix
exponentials, and pieces with equal coefficients reproduce the unsplit run.
"""
import sys

import numpy as np
import pytest
import scipy.linalg

import workloads as wl
from oracle import integrals, magnus, operators


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


# (g^vv, sigma^v) of each piece and its share of [0, T]: (length, Magnus steps, fine increments)
PIECES = [((1.0, 0.5), (0.25, 2, 256)), ((0.6, 0.3), (0.5, 4, 512)), ((1.4, 0.6), (0.25, 2, 256))]


def oracle_pieces(g, spec):
    out = []
    for (a, sig), (Tp, Kp, Nfp) in spec:
        B, A = operators.drift_and_noise(g, wl.langevin_constant(a, sig))
        out.append((operators.magnus_basis(B, A), Tp, Kp, Nfp))
    return out


@pytest.mark.parametrize("order", [1, 2, 3])
def test_piecewise_without_noise_is_the_ordered_product(order):
    """sigma^v = 0: each piece is exp(T_p B_p) at any order and step count,
    so the run equals exp(T_3 B_3) exp(T_2 B_2) exp(T_1 B_1) u0 (dense, 16x12
    grid).  The B_p do not commute (different g^vv against the transport
    term), and the reversed product is far off, so a piece applied out of
    order fails."""
    g = operators.Grid(16, 12, -4.0, 4.0, -4.0, 4.0)
    spec = [((a, 0.0), t) for (a, _), t in PIECES]
    pieces = oracle_pieces(g, spec)
    dW = wl.brownian_increments(41, 2, sum(t[2] for _, t in spec))
    u0 = wl.gaussian_density(16, 12, -4, 4, -4, 4, 0.5).reshape(-1)
    got = magnus.piecewise_magnus_paths(pieces, dW, u0, order)
    want = u0.copy()
    Bs = []
    for (a, _), (Tp, _, _) in spec:
        B, _ = operators.drift_and_noise(g, wl.langevin_constant(a, 0.0))
        Bs.append((B.toarray(), Tp))
        want = scipy.linalg.expm(Tp * B.toarray()) @ want
    for p in range(2):
        assert rel(got[p], want) <= 1e-12, (order, p, rel(got[p], want))
    rev = u0.copy()
    for B, Tp in reversed(Bs):
        rev = scipy.linalg.expm(Tp * B) @ rev
    assert rel(rev, want) > 1e-6


def test_piecewise_with_equal_pieces_is_the_unsplit_run():
    """Pieces that all carry the same coefficients give the unsplit scheme on
    the same fine path and the same steps (every Magnus step restarts its
    local path), so the results agree to rounding; a piece reading the wrong
    slice of the fine increments would not."""
    g = operators.Grid(12, 10, -4.0, 4.0, -4.0, 4.0)
    spec = [((1.0, 0.5), t) for _, t in PIECES]
    pieces = oracle_pieces(g, spec)
    Nf = sum(t[2] for _, t in spec)
    K = sum(t[1] for _, t in spec)
    dW = wl.brownian_increments(43, 3, Nf)
    u0 = wl.gaussian_density(12, 10, -4, 4, -4, 4, 0.5).reshape(-1)
    got = magnus.piecewise_magnus_paths(pieces, dW, u0, 2)
    want = magnus.iterated_magnus_paths(pieces[0][0], integrals.path_coefficients(dW, 1.0, K, 2), u0)
    for p in range(3):
        assert rel(got[p], want[p]) <= 1e-13
    shifted = np.roll(dW, 64, axis=1)
    bad = magnus.piecewise_magnus_paths(pieces, shifted, u0, 2)
    assert rel(bad[0], want[0]) > 1e-6


PIECE_GPU_CASES = [
    # (name, nx, nv, P, precision, tol); nx > 128 runs the cooperative kernel
    ("pw-40x36-f64", 40, 36, 3, "fp64", 1e-10),
    ("pw-40x36-f32c", 40, 36, 3, "fp32c", 1e-5),
    ("pw-160x136-f64", 160, 136, 2, "fp64", 1e-10),
    ("pw-160x136-f32c", 160, 136, 2, "fp32c", 1e-5),
]


@pytest.mark.gpu
@pytest.mark.parametrize("case", PIECE_GPU_CASES, ids=[c[0] for c in PIECE_GPU_CASES])
def test_piecewise_gpu_matches_oracle(case):
    """Three pieces with different diffusion and noise, chained through the C
    ABI, against the oracle's piecewise scheme on the same fine path."""
    torch = pytest.importorskip("torch")
    import paper_2207_09776_amd as mg

    name, nx, nv, P, prec, tol = case
    say(f"piecewise {name}")
    lo, hi = -5.0, 5.0
    if nx > 128:
        # short pieces keep the oracle's Taylor sums cheap on the wider grid
        spec = [(c, (t[0] / 10, t[1], t[2])) for c, t in PIECES]
    else:
        spec = PIECES
    g = operators.Grid(nx, nv, lo, hi, lo, hi)
    Nf = sum(t[2] for _, t in spec)
    dW = wl.brownian_increments(47, P, Nf, T=sum(t[0] for _, t in spec))
    u0 = wl.gaussian_density(nx, nv, lo, hi, lo, hi, 0.25).reshape(-1)
    dev = "cuda:0"
    dW_d = torch.from_numpy(dW).to(dev)
    u = torch.from_numpy(u0).to(dev)
    start = 0
    for (a, sig), (Tp, Kp, Nfp) in spec:
        arrays = wl.sample_coefficients(wl.langevin_constant(a, sig), nx, nv, lo, hi, lo, hi)
        ops = mg.build_operators(nx, nv, lo, hi, lo, hi, arrays, 2)
        coef, _ = mg.iterated_integrals(dW_d[:, start:start + Nfp].contiguous(), Tp, Kp, 2)
        u, flags, _ = mg.magnus_expmv(ops, coef, u, precision=prec)
        torch.cuda.synchronize()
        assert int(flags.abs().sum()) == 0, flags.cpu().numpy()
        start += Nfp
    want = magnus.piecewise_magnus_paths(oracle_pieces(g, spec), dW, u0, 2)
    got = u.cpu().numpy()
    for p in range(P):
        e = rel(got[p], want[p])
        assert e <= tol, (name, p, e)
