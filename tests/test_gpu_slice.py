"""GPU parity of the bond-2 Gram slice (tt_sparse_gram_slice) against the oracle.

The slice's gauge (Q_1 = left singular vectors of X_1) is unique up to round-off
amplified by singular value gaps: a left singular vector moves by about
u sigma_max / gap.  FP64 bars: sigma within 1e-12 sigma_max; row a of R_1 (column a
of Q_1) within eps_a = 1e-12 + 64 u sigma_max / gap_a (relative to sigma_max); an
X_2 entry of row (i, a) within eps_a sigma_max sum|c| over its block's entries; a
Gram entry within (eps_a + eps_a2 + 1e-12) sqrt(Gamma_qq Gamma_q2q2); the
gauge-free quantities (diagonal block traces, their sum = ||A||_F^2) within 1e-12
relative.  The FP32 and BF16 forms carry the same gauge term plus their operand
rounding, gated at 1e-5 and 2e-2 of each entry's scale (sum |c R_1[a, g]| for X_2,
the Cauchy-Schwarz bound for the Gram, ||A||_F^2 for the traces).
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_1908_02721_amd import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "slice_random5d_n200_nnz10m.json")
GATE = {"fp64": None, "fp32": 1e-5, "bf16": 2e-2}


def _tts():
    import paper_1908_02721_amd as tts

    return tts


def _gpu(idx, val):
    return (torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(val, dtype=np.float64)).cuda())


def _eps_rows(sigma):
    s = np.asarray(sigma)
    d = np.abs(np.diff(s))
    gap = np.minimum(np.r_[np.inf, d], np.r_[d, np.inf])
    gap = np.where(np.isfinite(gap), gap, s[0])
    return 1e-12 + 64.0 * U * s[0] / np.maximum(gap, 1e-300)


CASES = [
    ("m12", (12, 6, 7, 8), 1500, 11),
    ("m40", (40, 5, 6, 7, 8), 8000, 12),
    ("m70_d3", (70, 9, 40), 6000, 13),
    ("m130", (130, 4, 20, 25), 20000, 14),
    ("m200", (200, 6, 8, 7, 9), 30000, 15),
    ("split_items", (20, 2, 60, 70), 30000, 16),  # slots with more than 2048 blocks
]


def _check_small(oracle_mod, name, dims, nnz, seed, precision):
    from oracle import slice as osl

    tts = _tts()
    print(f"[slice parity] {name} dims={dims} nnz={nnz} precision={precision}", flush=True)
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    res = oracle_mod.decompose(idx, val, dims, 0.0, do_round=False)
    sl = osl.Slice(res)
    gi, gv = _gpu(idx, val)
    gs = tts.gram_slice(gi, gv, dims, precision=precision)
    assert gs.betas == res.betas
    assert gs.m == sl.m
    m, n2 = sl.m, dims[1]
    so = sl.b1.sigma
    smax = so[0]
    eps = _eps_rows(so)
    nrm2 = res.norm ** 2
    assert np.max(np.abs(gs.sigma1 - so)) <= 1e-12 * smax
    # bond 1 (FP64 in every precision)
    Q = gs.q1().cpu().numpy()
    R = gs.r1().cpu().numpy()
    assert np.max(np.abs(Q - sl.b1.Q1) / eps[None, :]) <= 1.0, "Q_1"
    assert np.max(np.abs(R - sl.b1.R1) / (eps[:, None] * smax)) <= 1.0, "R_1"
    # X_2: GPU blocks scattered to the oracle's dense slot-major layout
    X = gs.x2_view().double().cpu().numpy()
    sp = gs.slot_ptr().cpu().numpy()
    bc = gs.blk_col().cpu().numpy()
    assert gs.nblocks == X.shape[0] and sp[-1] == gs.nblocks
    Xg = np.zeros((n2 * m, res.betas[2]))
    for i in range(n2):
        Xg[i * m:(i + 1) * m, bc[sp[i]:sp[i + 1]]] = X[sp[i]:sp[i + 1]].T
    Xo = sl.dense_x2()
    # scale of each X_2 entry: sigma_max * sum |c| over its block's entries
    L2 = res.levels[1]
    col = np.repeat(np.arange(L2.beta), np.diff(L2.n_colptr))
    csum = np.zeros((n2, L2.beta))
    np.add.at(csum, (np.asarray(L2.n_row) % n2, col), np.abs(L2.n_val))
    scale = np.repeat(csum, m, axis=0) * smax  # rows q = i m + a: the FP64 bound's scale
    G2 = res.exact_cores()[1]
    absx = np.einsum("ag,gib->iab", np.abs(sl.b1.R1), np.abs(G2)).reshape(n2 * m, -1)  # sum |c R_1[a, g]|
    erow = np.tile(eps, n2)[:, None]
    nzx = absx > 0
    assert np.all(Xg[~nzx] == 0.0)
    ex = np.max(np.abs(Xg - Xo)[nzx] / absx[nzx])
    # Gram, dense from the packed blocks
    gp = gs.gram_view().cpu().numpy()
    Go = sl.dense_gram()
    N = n2 * m
    Gg = np.zeros((N, N))
    for i in range(n2):
        for i2 in range(i, n2):
            off = (i * n2 - i * (i - 1) // 2 + (i2 - i)) * m * m
            B = gp[off:off + m * m].reshape(m, m)
            Gg[i * m:(i + 1) * m, i2 * m:(i2 + 1) * m] = B
            Gg[i2 * m:(i2 + 1) * m, i * m:(i + 1) * m] = B.T
    dg = np.sqrt(np.maximum(np.diag(Go), 0.0))
    cs = np.maximum(np.outer(dg, dg), 1e-300)
    eg = np.max(np.abs(Gg - Go) / cs)
    traces_g = np.array([np.trace(Gg[i * m:(i + 1) * m, i * m:(i + 1) * m]) for i in range(n2)])
    et = np.max(np.abs(traces_g - sl.block_traces())) / nrm2
    ew = abs(gs.wnorm2 - nrm2) / nrm2
    print(f"  m={m} nblocks={gs.nblocks} npairs={gs.npairs}: X_2 {ex:.2e}, Gram {eg:.2e}, block traces {et:.2e}, "
          f"wnorm2 {ew:.2e} (relative to their scales)", flush=True)
    gate = GATE[precision] or 1e-12
    eg_rows = np.tile(eps, n2)
    assert np.all(np.abs(Xg - Xo) <= erow * scale + gate * absx), "X_2"
    assert np.all(np.abs(Gg - Go) <= (eg_rows[:, None] + eg_rows[None, :] + gate) * cs), "Gram"
    assert et <= gate and ew <= gate
    return gs


@pytest.mark.parametrize("name,dims,nnz,seed", CASES)
def test_slice_fp64(oracle_mod, name, dims, nnz, seed):
    _check_small(oracle_mod, name, dims, nnz, seed, "fp64")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("name,dims,nnz,seed", [CASES[1], CASES[4]])
def test_slice_reduced_precision(oracle_mod, name, dims, nnz, seed, precision):
    gs = _check_small(oracle_mod, name, dims, nnz, seed, precision)
    assert gs.x2_dtype == torch.float32


def test_slice_argument_errors():
    tts = _tts()
    from paper_1908_02721_amd._lib import TTError

    idx, val, dims = synth.random_sparse((30, 4, 5), 300, 3)  # beta_1 <= 20 < n_1: tall bond-1 unfolding
    gi, gv = _gpu(idx, val)
    with pytest.raises(TTError, match="wide"):
        tts.gram_slice(gi, gv, dims)
    idx, val, dims = synth.random_sparse((6, 7), 30, 3)  # d = 2
    gi, gv = _gpu(idx, val)
    with pytest.raises(TTError, match="TT_ERR_ARG"):
        tts.gram_slice(gi, gv, dims)
    idx, val, dims = synth.random_sparse((209, 4, 5, 6), 3000, 3)  # n_1 above 208
    gi, gv = _gpu(idx, val)
    with pytest.raises(TTError, match="208"):
        tts.gram_slice(gi, gv, dims)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_slice_random5d_full_size(precision):
    """The 5-way 200^5 tensor with 10^7 N(0,1) nonzeros, against oracle values stored by
    tests/golden/make_slice_golden.py at seeded positions."""
    tts = _tts()
    with open(GOLDEN) as f:
        gold = json.load(f)
    idx, val, dims, _ = synth.workload(gold["workload"])
    assert synth.checksum(idx, val, dims) == gold["checksum"]
    print(f"[slice full size] {gold['workload']} precision={precision}", flush=True)
    gi, gv = _gpu(idx, val)
    gs = tts.gram_slice(gi, gv, dims, precision=precision)
    assert gs.betas == gold["betas"]
    m, n2 = gold["m"], dims[1]
    assert gs.m == m
    so = np.asarray(gold["sigma1"])
    smax = so[0]
    eps = _eps_rows(so)
    assert np.max(np.abs(gs.sigma1 - so)) <= 1e-12 * smax
    r = gold["r1"]
    ra, rg = np.asarray(r["a"]), np.asarray(r["g"])
    R = gs.r1()
    got = R[torch.from_numpy(ra).cuda(), torch.from_numpy(rg).cuda()].cpu().numpy()
    assert np.all(np.abs(got - np.asarray(r["v"])) <= eps[ra] * smax), "R_1"
    # X_2 samples: block of (j, i) found by searching column j in slot i
    x = gold["x2"]
    xa, xi, xj = (np.asarray(x[k]) for k in ("a", "i", "j"))
    sp = gs.slot_ptr().cpu().numpy()
    bc = gs.blk_col().cpu().numpy()
    b = np.array([sp[i] + np.searchsorted(bc[sp[i]:sp[i + 1]], j) for i, j in zip(xi, xj)])
    assert np.all(bc[b] == xj)
    X = gs.x2_view()
    xv = X[torch.from_numpy(b).cuda(), torch.from_numpy(xa).cuda()].double().cpu().numpy()
    xo = np.asarray(x["v"])
    xabsc, xsc = np.asarray(x["absc"]), np.asarray(x["scale"])
    ex = np.abs(xv - xo) / xsc
    # Gram samples
    g = gold["gram"]
    off = gs.gram_offset(np.asarray(g["q"]), np.asarray(g["q2"]))
    gv_ = gs.gram_view()[torch.from_numpy(off).cuda()].cpu().numpy()
    go, gsc = np.asarray(g["v"]), np.asarray(g["scale"])
    eg = np.abs(gv_ - go) / gsc
    # gauge-free: diagonal block traces and their sum
    gp = gs.gram_view()
    tr = []
    for i in range(n2):
        o = (i * n2 - i * (i - 1) // 2) * m * m
        tr.append(float(torch.diagonal(gp[o:o + m * m].view(m, m)).sum().item()))
    nrm2 = gold["norm2"]
    et = np.max(np.abs(np.asarray(tr) - np.asarray(gold["block_traces"]))) / nrm2
    ew = abs(gs.wnorm2 - nrm2) / nrm2
    tf = gs.gram_flops / (gs.slice_ms["gram"] * 1e-3) / 1e12
    print(f"  X_2 max {np.max(ex):.2e} (median {np.median(ex):.2e}); Gram {np.max(eg):.2e}; block traces "
          f"{et:.2e}; wnorm2 {ew:.2e} (relative to their scales); stages {gs.slice_ms}; Gram {tf:.1f} TFLOP/s",
          flush=True)
    # every precision carries the FP64 gauge term of the bond-1 factors; the reduced
    # ones add their operand rounding, at most `gate` of the entry's scale
    gate = GATE[precision] or 1e-12
    q1, q2 = np.asarray(g["q"]) % m, np.asarray(g["q2"]) % m
    assert np.all(np.abs(xv - xo) <= eps[xa] * smax * xabsc + gate * xsc), "X_2"
    assert np.all(np.abs(gv_ - go) <= (eps[q1] + eps[q2] + gate) * gsc), "Gram"
    assert et <= gate and ew <= gate
