"""Pins of the fiber-trie FastTT oracle (Algorithms 4-7 and 9, oracle/ftt.py).

References independent of the oracle: dense reconstruction of tiny tensors, brute
force sets of prefixes and suffixes, the rank bounds of Algorithm 4, orthonormality
of the indicator cores (corollary on left/right orthonormality), dense TT-SVD ranks
with LAPACK at eps -> 0 (the remark after Algorithm 7), the error bound of
Algorithm 6's correctness theorem, the FDM numbers R and r~ printed in Table 2, and
the worked FLOP examples of the complexity analysis.
"""
import json
import os

import numpy as np
import pytest

from oracle import ftt
from paper_1908_02721_amd import synth
from tests import _brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_fdm_ranks.json")

TINY = [((4, 3, 5, 2), 40, 1), ((3, 4, 2, 3, 2), 60, 2), ((6, 5), 12, 3), ((2, 3, 4), 24, 4), ((5, 1, 4, 3), 30, 5)]


@pytest.mark.parametrize("dims,nnz,seed", TINY)
def test_exact_tt_reconstructs_and_counts(dims, nnz, seed):
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    A = _brute.dense_tensor(idx, val, dims)
    d = len(dims)
    for p in range(1, d + 1):
        ex = ftt.exact_tt(idx, val, dims, p)
        assert np.array_equal(_brute.tt_full(ex.cores), A)
        for k in range(1, d):
            if k < p:
                want = len({tuple(r[:k]) for r in idx.tolist()})
            else:
                want = len({tuple(r[k:]) for r in idx.tolist()})
            assert ex.ranks[k] == want
        R = len({tuple(r[:p - 1] + r[p:]) for r in idx.tolist()})
        assert ex.R == R
        rb = ftt.rank_bounds(dims, p, R)
        assert all(a <= b for a, b in zip(ex.ranks, rb))
        # indicator cores: spl_2 orthonormal left of p, spl_1^T orthonormal right of p
        for k in range(1, d + 1):
            G = ex.cores[k - 1]
            if k < p:
                M = G.reshape(-1, G.shape[2])
                assert np.array_equal(M.T @ M, np.eye(G.shape[2]))
            elif k > p:
                M = G.reshape(G.shape[0], -1)
                assert np.array_equal(M @ M.T, np.eye(G.shape[0]))


@pytest.mark.parametrize("dims,nnz,seed", TINY)
def test_rounding_ranks_equal_ttsvd_at_small_eps(dims, nnz, seed):
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    A = _brute.dense_tensor(idx, val, dims)
    d = len(dims)
    for p in range(1, d + 1):
        res = ftt.decompose(idx, val, dims, 1e-14, p=p)
        for k in range(1, d):
            assert res.ranks[k] == np.linalg.matrix_rank(A.reshape(int(np.prod(dims[:k])), -1))
        assert np.linalg.norm(_brute.tt_full(res.cores) - A) <= 1e-13 * np.linalg.norm(A)


@pytest.mark.parametrize("eps", [0.05, 0.2, 0.5])
@pytest.mark.parametrize("dims,nnz,seed", TINY[:3])
def test_rounding_error_bound(dims, nnz, seed, eps):
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    A = _brute.dense_tensor(idx, val, dims)
    nrm = np.linalg.norm(A)
    d = len(dims)
    for p in range(1, d + 1):
        res = ftt.decompose(idx, val, dims, eps, p=p)
        err = np.linalg.norm(_brute.tt_full(res.cores) - A)
        # the proof's bound: first-sweep and second-sweep errors add as two Pythagorean sums
        first = np.sqrt(sum(res.tail[k - 1] for k in range(p, d)))
        second = np.sqrt(sum(res.tail[k - 2] for k in range(2, p + 1)))
        assert err <= first + second + 1e-13 * nrm
        assert err <= eps * nrm + 1e-13 * nrm
        # every core right of the last SVD sweep's end is right-orthonormal, left of p left-orthonormal
        for k in range(2, d + 1):
            G = res.cores[k - 1]
            M = G.reshape(G.shape[0], -1)
            assert np.max(np.abs(M @ M.T - np.eye(G.shape[0]))) <= 1e-12


def test_table2_fdm_R_and_ranks():
    g = json.load(open(GOLDEN))
    for case in g["ftt"]:
        n = case["n"]
        for coeff in ("pattern", "random"):
            idx, val, dims = synth.fdm3d_mpo(n, coeff, seed=1)
            ex = ftt.exact_tt(idx, val, dims, 2)
            assert ex.R == case["R"]
            assert ex.ranks[1:3] == case["r_tilde"]
        if n == 20:
            for c in g["cases"]:
                if c["n"] == 20:
                    idx, val, dims = synth.fdm3d_mpo(20, c["coeff"], seed=1)
                    res = ftt.decompose(idx, val, dims, 1e-14, p=2)
                    assert res.ranks[1:3] == c["final_ranks"]


def test_select_p_fdm():
    idx, val, dims = synth.fdm3d_mpo(20, "random", seed=1)
    p, costs = ftt.select_p(idx, dims)
    assert p == 2 and costs[1] < min(costs[0], costs[2])


def test_flop_examples_of_the_complexity_analysis():
    # 7-way 10x20x20x10x15x20x3, p = 7, fixed rank r = 10: with R <= 12000 nonzero
    # fibers the bounds are {10, 200, 4000, 12000, 12000, 12000} and the estimate is
    # about 8e8 (in units of the SVD constant); with R <= 120000 it is about 5.7e9
    dims = (10, 20, 20, 10, 15, 20, 3)
    r = [1] + [10] * 6 + [1]
    rb = ftt.rank_bounds(dims, 7, 12000)
    assert rb == [1, 10, 200, 4000, 12000, 12000, 12000, 1]
    f = ftt.flop_estimate(dims, 7, rb, r)
    assert abs(f - 8e8) <= 0.01 * 8e8
    rb = ftt.rank_bounds(dims, 7, 120000)
    assert rb == [1, 10, 200, 4000, 40000, 120000, 120000, 1]
    f = ftt.flop_estimate(dims, 7, rb, r)
    assert abs(f - 5.7e9) <= 0.02 * 5.7e9
    assert ftt.f_svd(3, 12000) == 1.08e5 and ftt.f_svd(12000, 3) == 1.08e5


# ---- Algorithm 8 in the fiber-trie rounding ----

@pytest.mark.parametrize("eps", [0.1, 0.3, 0.6])
@pytest.mark.parametrize("dims,nnz,seed", TINY[:4])
def test_dynamic_thresholds_theorem10(dims, nnz, seed, eps):
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    A = _brute.dense_tensor(idx, val, dims)
    nrm = np.linalg.norm(A)
    d = len(dims)
    for p in range(1, d + 1):
        st = ftt.decompose(idx, val, dims, eps, p=p)
        dy = ftt.decompose(idx, val, dims, eps, p=p, dynamic_delta=True)
        den = np.sqrt(p - 1) + np.sqrt(d - p)
        right, left = np.sqrt(d - p) / den * eps * nrm, np.sqrt(p - 1) / den * eps * nrm
        # loop invariants: each sweep's discarded sums stay within its budget
        assert sum(dy.tail[k - 1] for k in range(p, d)) <= right ** 2 * (1 + 1e-12) + 1e-28
        assert sum(dy.tail[k - 2] for k in range(2, p + 1)) <= left ** 2 * (1 + 1e-12) + 1e-28
        # the correctness theorem of Algorithm 8
        assert np.linalg.norm(_brute.tt_full(dy.cores) - A) <= eps * nrm + 1e-13 * nrm
        # the first bond of each sweep sees the static threshold
        if p < d:
            assert abs(dy.bond_delta[p - 1] - st.delta) <= 1e-14 * nrm
        if p > 1:
            assert abs(dy.bond_delta[p - 2] - st.delta) <= 1e-14 * nrm


@pytest.mark.parametrize("dims,nnz,seed", TINY[:4])
def test_dynamic_thresholds_at_p_d_match_dense_ttsvd(dims, nnz, seed):
    # at p = d the first sweep and the QR sweep are empty, and the second sweep is the
    # right-to-left TT-SVD of the whole tensor with Algorithm 8's thresholds
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    A = _brute.dense_tensor(idx, val, dims)
    for eps in (0.2, 0.5):
        dy = ftt.decompose(idx, val, dims, eps, p=len(dims), dynamic_delta=True)
        ranks, _ = _brute.tt_svd_right_to_left(A, eps, dynamic=True)
        assert dy.ranks == ranks


def test_exact_tt_numbering_worked_example():
    # Alg 5 keeps each nonzero row of a quasi-permutation matrix once, numbered by
    # increasing row index: a prefix's bond index is its rank among the distinct
    # prefixes (lexicographic), a suffix's its rank among the distinct suffixes with
    # its first mode most significant.  Three nonzeros of a 2 x 3 x 3 tensor, the
    # expected cores written out by hand from that rule.
    idx = np.array([[0, 1, 2], [1, 0, 0], [0, 2, 2]], dtype=np.int32)
    val = np.array([3.0, -5.0, 7.0])
    dims = (2, 3, 3)
    # p = 2: prefixes (i_1) = {0, 1} -> ids 0, 1; suffixes (i_3) = {0, 2} -> ids 0, 1
    ex = ftt.exact_tt(idx, val, dims, 2)
    assert ex.ranks == [1, 2, 2, 1]
    g1 = np.zeros((1, 2, 2)); g1[0, 0, 0] = g1[0, 1, 1] = 1.0
    g2 = np.zeros((2, 3, 2)); g2[0, 1, 1] = 3.0; g2[1, 0, 0] = -5.0; g2[0, 2, 1] = 7.0
    g3 = np.zeros((2, 3, 1)); g3[0, 0, 0] = g3[1, 2, 0] = 1.0
    for got, want in zip(ex.cores, (g1, g2, g3)):
        assert np.array_equal(got, want)
    # p = 3: prefixes (i_1, i_2) = (0,1), (0,2), (1,0) -> ids 0, 1, 2
    ex = ftt.exact_tt(idx, val, dims, 3)
    assert ex.ranks == [1, 2, 3, 1]
    g2 = np.zeros((2, 3, 3)); g2[0, 1, 0] = g2[0, 2, 1] = g2[1, 0, 2] = 1.0
    g3 = np.zeros((3, 3, 1)); g3[0, 2, 0] = 3.0; g3[1, 2, 0] = 7.0; g3[2, 0, 0] = -5.0
    for got, want in zip(ex.cores, (g1, g2, g3)):
        assert np.array_equal(got, want)
    # p = 1: suffixes (i_2, i_3) = (0,0), (1,2), (2,2) -> ids 0, 1, 2; (i_3) as above
    ex = ftt.exact_tt(idx, val, dims, 1)
    assert ex.ranks == [1, 3, 2, 1]
    h1 = np.zeros((1, 2, 3)); h1[0, 0, 1] = 3.0; h1[0, 1, 0] = -5.0; h1[0, 0, 2] = 7.0
    h2 = np.zeros((3, 3, 2)); h2[0, 0, 0] = h2[1, 1, 1] = h2[2, 2, 1] = 1.0
    h3 = np.zeros((2, 3, 1)); h3[0, 0, 0] = h3[1, 2, 0] = 1.0
    for got, want in zip(ex.cores, (h1, h2, h3)):
        assert np.array_equal(got, want)
