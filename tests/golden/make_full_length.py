"""Writes the oracle's terminal values for single paths of the full-length
workloads, for the GPU parity tests of those launches (tests/test_gpu_full_length.py).

Each record is the FP64 oracle (oracle/: operators built as printed in
Section 2, weights of eq. (MagnusFormulas), exp by the scaled power series)
run over the whole horizon of the workload, on the seeded inputs of
workloads/ -- nothing here comes from the GPU path.  Output per record:
  full/<name>.npy   uT [nv][nx] float64 (np.save, no pickle)
  full/<name>.json  workload, path index, seed, grid, K, order, Nf, T and the
                    oracle's series length.

Usage: python tests/golden/make_full_length.py [name ...]   (default: all;
one process per record; the 1024^2 path takes about an hour and a quarter
of one core).
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "full")

# name -> (workload, group index in a mixed workload or None, path index)
RECORDS = {
    "const-256-p4096-m3-k32_p0": ("const-256-p4096-m3-k32", None, 0),
    "const-256-p4096-m3-k32_p4095": ("const-256-p4096-m3-k32", None, 4095),
    "var-512-p512-m2-k256_p0": ("var-512-p512-m2-k256", None, 0),
    "var-512-p512-m2-k256_p511": ("var-512-p512-m2-k256", None, 511),
    "mixed-1024-p64-m2-k512_p0": ("mixed-64-256-1024-m2-fp32c", 2, 0),
}


def describe(name):
    """Shape of one record: (n, lo, hi, paths, K, order, Nf, T, seed, s0sq,
    coefficients, path index)."""
    import workloads as wl
    wname, group, p = RECORDS[name]
    w = wl.WORKLOADS[wname]
    if group is None:
        n, paths, K, seed = w.n, w.paths, w.K, w.seed
    else:
        n, paths, K, seed = w.extra[group]
    return dict(workload=wname, group=group, path=p, n=n, lo=w.lo, hi=w.hi, paths=paths, K=K,
                order=w.order, Nf=w.Nf, T=w.T, seed=seed, s0sq=w.s0sq,
                coefficients=("variable (g^vv = s(x,v)^2, sigma^v = b(v), f^x = -v)"
                              if w.variable else f"constant (a = {w.a}, sigma = {w.sigma})"))


def make(name):
    import numpy as np
    import workloads as wl
    from oracle import integrals, magnus, operators
    d = describe(name)
    w = wl.WORKLOADS[d["workload"]]
    t0 = time.time()
    n = d["n"]
    g = operators.Grid(n, n, d["lo"], d["hi"], d["lo"], d["hi"])
    B, A = operators.drift_and_noise(g, w.coefficients())
    basis = operators.magnus_basis(B, A)
    dW = wl.brownian_increments(d["seed"], d["paths"], d["Nf"], d["T"], first=d["path"], count=1)
    coef = integrals.path_coefficients(dW, d["T"], d["K"], d["order"])[0]
    u0 = wl.gaussian_density(n, n, d["lo"], d["hi"], d["lo"], d["hi"], d["s0sq"]).reshape(-1)
    uT = magnus.iterated_magnus(basis, coef, u0, terms=20)
    os.makedirs(OUT, exist_ok=True)
    np.save(os.path.join(OUT, name + ".npy"), uT.reshape(n, n))
    d.update(oracle="oracle.magnus.iterated_magnus, power series of 20 terms per scaled factor",
             seconds=round(time.time() - t0, 1), norm2=float(np.linalg.norm(uT)),
             max=float(np.abs(uT).max()))
    with open(os.path.join(OUT, name + ".json"), "w") as f:
        json.dump(d, f, indent=1)
    return name, d["seconds"]


def main(argv):
    names = argv or list(RECORDS)
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    with ProcessPoolExecutor(max_workers=min(len(names), 5)) as ex:
        for name, sec in ex.map(make, names):
            print(f"{name}: {sec:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
