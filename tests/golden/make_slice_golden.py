"""Writes slice_random5d_n200_nnz10m.json: oracle values of the bond-2 Gram slice on the
5-way 200^5 tensor with 10^7 seeded N(0,1) nonzeros, at seeded sample positions.

    python tests/golden/make_slice_golden.py

Calls only the oracle (oracle/, oracle/slice.py) and the seeded input generator.
The tensor is regenerated from its seed by the tests; the stored checksum confirms it
is the same one.  Sample positions are drawn with NumPy PCG64(seed 41).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

WORKLOAD = "random5d_n200_nnz10m"
OUT = os.path.join(HERE, "slice_random5d_n200_nnz10m.json")


def main():
    import oracle
    from oracle import slice as osl
    from paper_1908_02721_amd import synth

    oracle.build(force=False)
    t0 = time.time()
    idx, val, dims, eps = synth.workload(WORKLOAD)
    res = oracle.decompose(idx, val, dims, eps, do_round=False)
    print(f"sparse stage {time.time() - t0:.1f} s, betas {res.betas}", flush=True)
    sl = osl.Slice(res)
    b1 = sl.b1
    m, n2 = sl.m, sl.n2
    rng = np.random.Generator(np.random.PCG64(41))
    # R_1 at 1024 uniform positions
    r_a = rng.integers(0, m, 1024)
    r_g = rng.integers(0, b1.R1.shape[1], 1024)
    # X_2 at 4096 positions on its support: a uniform entry of N_2 gives (j, i)
    L2 = res.levels[1]
    e = rng.integers(0, len(L2.n_row), 4096)
    x_j = np.searchsorted(L2.n_colptr, e, side="right") - 1
    x_i = np.asarray(L2.n_row)[e] % n2
    x_a = rng.integers(0, m, 4096)
    # Gamma at 3072 uniform upper-block positions and 1024 in diagonal blocks
    q1 = rng.integers(0, m * n2, 3072)
    q2 = rng.integers(0, m * n2, 3072)
    swap = (q1 // m) > (q2 // m)
    q1[swap], q2[swap] = q2[swap].copy(), q1[swap].copy()
    di = rng.integers(0, n2, 1024)
    gq1 = np.concatenate([q1, di * m + rng.integers(0, m, 1024)])
    gq2 = np.concatenate([q2, di * m + rng.integers(0, m, 1024)])
    t0 = time.time()
    xv = [sl.x2(a, i, j) for a, i, j in zip(x_a, x_i, x_j)]
    # error scales of each X_2 sample: sum |c| and sum |c R_1[a, g]| over its block's entries
    rho_all = np.asarray(L2.n_row, dtype=np.int64)
    absc, xsc = [], []
    for a, i, j in zip(x_a, x_i, x_j):
        lo, hi = L2.n_colptr[j], L2.n_colptr[j + 1]
        rr, cc = rho_all[lo:hi], np.asarray(L2.n_val[lo:hi])
        sel = rr % n2 == i
        absc.append(float(np.sum(np.abs(cc[sel]))))
        xsc.append(float(np.sum(np.abs(cc[sel] * b1.R1[a, rr[sel] // n2]))))
    gv = [sl.gram(a, b) for a, b in zip(gq1, gq2)]
    # Cauchy-Schwarz scale of each Gram sample: sqrt(Gamma_qq Gamma_q2q2)
    diag = {}
    for q in np.unique(np.concatenate([gq1, gq2])):
        diag[int(q)] = sl.gram(q, q)
    gs = [float(np.sqrt(diag[int(a)] * diag[int(b)])) for a, b in zip(gq1, gq2)]
    bt = sl.block_traces()
    print(f"samples {time.time() - t0:.1f} s", flush=True)
    out = {
        "what": "oracle values of the bond-2 Gram slice (oracle/slice.py) at seeded positions",
        "workload": WORKLOAD,
        "checksum": synth.checksum(idx, val, dims),
        "dims": list(dims),
        "betas": [int(b) for b in res.betas],
        "nnz_n": [int(len(L.n_row)) for L in res.levels],
        "norm2": float(res.norm) ** 2,
        "m": int(m),
        "sigma1": [float(x) for x in b1.sigma],
        "r1": {"a": r_a.tolist(), "g": r_g.tolist(), "v": [float(b1.R1[a, g]) for a, g in zip(r_a, r_g)]},
        "x2": {"a": x_a.tolist(), "i": x_i.tolist(), "j": x_j.tolist(), "v": xv, "absc": absc, "scale": xsc},
        "gram": {"q": gq1.tolist(), "q2": gq2.tolist(), "v": gv, "scale": gs},
        "block_traces": [float(x) for x in bt],
        "weighted_norm2": float(np.sum(bt)),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
