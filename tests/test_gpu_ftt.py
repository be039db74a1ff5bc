"""GPU parity of the fiber-trie FastTT (Algorithms 4-7 and 9) against oracle/ftt.py.

Bar: the exact TT of Algorithm 4 bit for bit (ranks r~, R, every core: indicator
cores and the value core, same numbering); after Algorithm 6 identical ranks,
singular values per bond within 1e-12 ||A||_F, and the represented tensors within
1e-12 ||A||_F (stable TT-difference norm); Algorithm 9 the same p and costs.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import ftt as oftt
from paper_1908_02721_amd import synth
from tests import _brute

pytestmark = pytest.mark.gpu

TOL = 1e-12
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_fdm_ranks.json")


def _tts():
    import paper_1908_02721_amd as tts

    return tts


def _gpu(idx, val):
    return torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda(), \
        torch.from_numpy(np.ascontiguousarray(val, dtype=np.float64)).cuda()


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.int64)


def check_exact(idx, val, dims, p, label):
    tts = _tts()
    print(f"[ftt exact] {label} dims={tuple(dims)} nnz={len(val)} p={p}", flush=True)
    ex = oftt.exact_tt(idx, val, dims, p)
    gi, gv = _gpu(idx, val)
    tt = tts.fasttt_decompose(gi, gv, dims, 0.0, p=p, sparse_only=True)
    assert tt.ftt_p == p and tt.fibers == ex.R
    assert tt.betas == ex.ranks, (tt.betas, ex.ranks)
    assert abs(tt.norm - ex.norm) <= 1e-13 * ex.norm
    for k, (cg, co) in enumerate(zip(tt.cores, ex.cores)):
        assert tuple(cg.shape) == co.shape, k
        assert np.array_equal(_bits(cg.cpu().numpy()), _bits(co)), f"core {k + 1}"
    return tt


def check_round(oracle_mod, idx, val, dims, eps, p, label, max_rank=0, dense=False, dynamic=False):
    tts = _tts()
    print(f"[ftt round] {label} dims={tuple(dims)} nnz={len(val)} eps={eps} p={p} max_rank={max_rank} "
          f"dynamic={dynamic}", flush=True)
    res = oftt.decompose(idx, val, dims, eps, p=p, max_rank=max_rank, dynamic_delta=dynamic)
    gi, gv = _gpu(idx, val)
    tt = tts.fasttt_decompose(gi, gv, dims, eps, p=p, max_rank=max_rank, dynamic_delta=dynamic)
    nrm = res.norm
    assert tt.ftt_p == res.p
    assert tt.betas == res.exact_ranks
    assert tt.ranks == res.ranks, (tt.ranks, res.ranks)
    for b in range(1, len(dims)):
        sg, _ = tt.sigma(b)
        so = res.sigma[b - 1]
        mm = min(len(sg), len(so))
        assert np.max(np.abs(sg[:mm] - so[:mm])) <= TOL * nrm, f"bond {b} sigma"
        assert np.all(sg[mm:] <= TOL * nrm) and np.all(so[mm:] <= TOL * nrm)
        assert abs(tt.bond_delta(b) ** 2 - res.bond_delta[b - 1] ** 2) <= TOL * nrm * nrm
    cores = [c.cpu().numpy() for c in tt.cores]
    diff = oracle_mod.tt_diff_norm(cores, [np.ascontiguousarray(c) for c in res.cores])
    assert diff <= TOL * nrm, f"||B_gpu - B_oracle|| = {diff / nrm:.3e} ||A||"
    if dense and max_rank == 0:  # fixed-rank truncation ignores eps
        A = _brute.dense_tensor(idx, val, dims)
        assert np.linalg.norm(_brute.tt_full(cores) - A) <= eps * nrm + TOL * nrm
    return tt, res


TINY = [((4, 3, 5, 2), 40, 1), ((3, 4, 2, 3, 2), 60, 2), ((6, 5), 12, 3), ((2, 3, 4), 24, 4), ((5, 1, 4, 3), 30, 5)]


@pytest.mark.parametrize("dims,nnz,seed", TINY)
def test_exact_tiny_every_p(dims, nnz, seed):
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    for p in range(1, len(dims) + 1):
        check_exact(idx, val, dims, p, f"tiny {seed}")


def test_exact_ragged_and_large_keys():
    # several radix-sort tiles and a ragged tail; wide modes
    idx, val, dims = synth.random_sparse((300, 7, 5, 200), 20000 + 37, 11)
    for p in (1, 2):
        check_exact(idx, val, dims, p, "random 300x7x5x200")


def test_exact_fdm_table2():
    g = json.load(open(GOLDEN))
    for case in g["ftt"]:
        for coeff in ("pattern", "random"):
            idx, val, dims = synth.fdm3d_mpo(case["n"], coeff, seed=1)
            tt = check_exact(idx, val, dims, 2, f"fdm n={case['n']} {coeff}")
            assert tt.fibers == case["R"] and tt.betas[1:3] == case["r_tilde"]


@pytest.mark.parametrize("eps", [1e-14, 0.05, 0.3])
@pytest.mark.parametrize("dims,nnz,seed", TINY)
def test_round_tiny_every_p(oracle_mod, dims, nnz, seed, eps):
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    for p in range(1, len(dims) + 1):
        check_round(oracle_mod, idx, val, dims, eps, p, f"tiny {seed}", dense=True)


@pytest.mark.parametrize("max_rank", [1, 3])
def test_round_fixed_rank(oracle_mod, max_rank):
    idx, val, dims = synth.random_sparse((5, 6, 4, 5), 200, 31)
    for p in (1, 2, 4):
        check_round(oracle_mod, idx, val, dims, 0.5, p, "fixed rank", max_rank=max_rank, dense=True)


def test_round_fdm_table2_final_ranks(oracle_mod):
    g = json.load(open(GOLDEN))
    for c in g["cases"]:
        if c["n"] > 30:
            continue
        idx, val, dims = synth.fdm3d_mpo(c["n"], c["coeff"], seed=1)
        tt, _ = check_round(oracle_mod, idx, val, dims, 1e-14, 2, f"fdm n={c['n']} {c['coeff']}")
        assert tt.ranks[1:3] == c["final_ranks"]


@pytest.mark.parametrize("c", [65, 66, 97, 117, 127, 128])
@pytest.mark.parametrize("eps", [1e-14, 0.3])
def test_round_bond_widths_65_to_128(oracle_mod, c, eps):
    """Bonds of 65..128 columns (odd and even): the SVD of every bond is the
    register-resident Jacobi of that width, with and without truncation."""
    idx, val, dims = synth.random_sparse((c, 3, c), int(1.5 * c * c), 40 + c)
    tt, res = check_round(oracle_mod, idx, val, dims, eps, 2, f"bond width {c}")
    assert tt.betas == [1, c, c, 1]
    if eps < 1e-10:
        assert tt.ranks == [1, c, c, 1]


@pytest.mark.parametrize("dims,eps", [((120, 2, 40), 0.2), ((124, 2, 60), 0.4)])
def test_round_left_svd_wide_transpose(oracle_mod, dims, eps):
    """After the right sweep truncates bond 2, the left SVD's matrix has fewer rows
    (n_2 r_2 = 78, 106) than columns (120, 124): the Jacobi runs on its transpose,
    with more rows than columns, in the register-resident kernel."""
    idx, val, dims = synth.random_sparse(dims, int(0.6 * dims[0] * dims[1] * dims[2]), 7)
    tt, res = check_round(oracle_mod, idx, val, dims, eps, 2, "left SVD on a wide matrix")
    assert 64 < 2 * tt.ranks[2] < dims[0]


@pytest.mark.timeout(400)
def test_round_fdm_n40_random(oracle_mod):
    idx, val, dims = synth.fdm3d_mpo(40, "random", seed=1)
    tt, _ = check_round(oracle_mod, idx, val, dims, 1e-14, 2, "fdm n=40 random")
    assert tt.fibers == 7840 and tt.betas[1:3] == [118, 118] and tt.ranks[1:3] == [118, 118]


def test_select_p_matches_oracle():
    tts = _tts()
    for idx, val, dims in (synth.fdm3d_mpo(20, "random", seed=1), synth.random_sparse((6, 5, 7, 4), 300, 3),
                           synth.random_sparse((30, 2, 2, 2, 40), 500, 4)):
        p, costs = oftt.select_p(idx, dims)
        gi, gv = _gpu(idx, val)
        pg, cg = tts.fasttt_select_p(gi, gv, dims)
        assert pg == p and cg == costs
        tt = tts.fasttt_decompose(gi, gv, dims, 1e-10, p=0)
        assert tt.ftt_p == p


def test_same_ranks_as_column_parallel_path(oracle_mod):
    """At small eps both variants give the TT-SVD ranks (the remark after Algorithm 7)."""
    tts = _tts()
    idx, val, dims = synth.kronecker_sum(5, 6, 4, 2, seed=3)
    gi, gv = _gpu(idx, val)
    a = tts.decompose(gi, gv, dims, 1e-12)
    for p in range(1, 6):
        b = tts.fasttt_decompose(gi, gv, dims, 1e-12, p=p)
        assert a.ranks == b.ranks
        ca = [c.cpu().numpy() for c in a.cores]
        cb = [c.cpu().numpy() for c in b.cores]
        assert oracle_mod.tt_diff_norm(ca, cb) <= 1e-11 * a.norm


def test_device_detected_errors():
    tts = _tts()
    idx = np.array([[0, 1, 2], [1, 1, 1], [0, 1, 2]], dtype=np.int32)
    for case, ix, v, code in (
            ("duplicate", idx, [1.0, 2.0, 3.0], "TT_ERR_DUPLICATE"),
            ("index", np.array([[0, 4, 0]], dtype=np.int32), [1.0], "TT_ERR_INDEX"),
            ("nonfinite", idx[:2], [1.0, np.nan], "TT_ERR_NONFINITE"),
            ("zeros", idx[:2], [0.0, -0.0], "TT_ERR_EMPTY")):
        print(f"[ftt errors] {case}", flush=True)
        gi, gv = _gpu(ix, np.array(v))
        for p in (1, 2, 3):
            with pytest.raises(tts.TTError) as ei:
                tts.fasttt_decompose(gi, gv, (3, 3, 3), 0.1, p=p)
            assert ei.value.status == code, (case, p, ei.value.status)
    # an exact rank above the one-device limit (about 31,000 distinct i_2 here) is
    # refused before its core is allocated
    idx, val, dims = synth.random_sparse((40000, 40000), 60000, 7)
    assert len(np.unique(idx[:, 1])) > 16384
    gi, gv = _gpu(idx, val)
    with pytest.raises(tts.TTError) as ei:
        tts.fasttt_decompose(gi, gv, dims, 0.1, p=1, sparse_only=True)
    assert ei.value.status == "TT_ERR_TOO_LARGE"


@pytest.mark.parametrize("eps", [0.1, 0.3, 0.6])
@pytest.mark.parametrize("dims,nnz,seed", TINY[:4])
def test_round_dynamic_thresholds(oracle_mod, dims, nnz, seed, eps):
    """Algorithm 8 in the fiber-trie rounding, every p, against the oracle."""
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    for p in range(1, len(dims) + 1):
        check_round(oracle_mod, idx, val, dims, eps, p, f"tiny {seed}", dense=True, dynamic=True)
