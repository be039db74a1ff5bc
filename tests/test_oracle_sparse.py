"""Pins of the oracle's sparse stage (parallel-vector rounding on sparse unfoldings).

Each test checks the oracle against something other than itself: a literal
Deparallelisation (Algorithm 3) in exact rational arithmetic, closed forms
(Lemma 1, Lemma 2, quasi-permutation columns, Lemma 6), and exact reconstruction.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_1908_02721_amd import synth
from tests import _brute


def _tiny(seed, dims, density, kind):
    rng = np.random.Generator(np.random.PCG64(seed))
    total = int(np.prod(dims))
    nnz = max(1, int(density * total))
    lin = rng.choice(total, nnz, replace=False)
    if kind == "int":
        val = rng.integers(1, 4, nnz) * rng.choice([-1, 1], nnz)
    elif kind == "dyadic":
        val = rng.integers(16, 49, nnz) / 32.0
    else:
        val = rng.standard_normal(nnz)
    return synth.unravel(lin, dims), val.astype(np.float64), dims


def _check_against_brute(oracle_mod, idx, val, dims):
    res = oracle_mod.decompose(idx, val, dims, 0.0, do_round=False)
    levels, last = _brute.cps_exact(idx, val, dims)
    d = len(dims)
    for k in range(1, d):
        L = res.levels[k - 1]
        B = levels[k - 1]
        assert L.beta == B["beta"], f"level {k}: beta"
        # numbering: group of each column, in row-major column order
        assert len(L.col) == len(B["T"])
        assert list(L.col) == sorted(B["T"].keys())
        for c, g, s in zip(L.col, L.g, L.s):
            bg, pf = B["T"][int(c)]
            assert int(g) == bg, f"level {k} col {c}: group"
            assert Fraction(float(s)) == pf, f"level {k} col {c}: prefactor"
        # distinct columns: rows and correctly rounded canonical values
        for gi in range(L.beta):
            rows = L.n_row[L.n_colptr[gi]:L.n_colptr[gi + 1]]
            vals = L.n_val[L.n_colptr[gi]:L.n_colptr[gi + 1]]
            ref = B["N"][gi]
            assert list(rows) == sorted(ref.keys())
            for r_, v_ in zip(rows, vals):
                assert float(v_) == float(ref[int(r_)])
    nd = dims[-1]
    le = res.last_exact.reshape(-1, nd)
    for (g, j), pf in last.items():
        assert Fraction(float(le[g, j])) == pf
    assert np.count_nonzero(le) == len(last)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("kind", ["int", "dyadic", "normal"])
def test_grouping_matches_literal_deparallelisation(oracle_mod, seed, kind):
    dims = [(3, 4, 2, 3), (2, 3, 3, 2, 2), (5, 4, 6)][seed % 3]
    idx, val, dims = _tiny(seed, dims, 0.35 if seed % 2 else 0.15, kind)
    _check_against_brute(oracle_mod, idx, val, dims)


@pytest.mark.parametrize("seed", range(3))
def test_grouping_with_structured_parallel_columns(oracle_mod, seed):
    # sum of a few rank-1 terms with small integer factors plus noise entries:
    # many exactly parallel columns, some mixed ones
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    dims = (4, 3, 4, 3)
    A = np.zeros(dims)
    for _ in range(3):
        fs = [rng.integers(-2, 3, n) for n in dims]
        A += np.einsum("a,b,c,d->abcd", *fs)
    for _ in range(4):
        A[tuple(rng.integers(0, n) for n in dims)] += rng.integers(1, 3)
    nz = np.argwhere(A != 0)
    _check_against_brute(oracle_mod, nz.astype(np.int32), A[tuple(nz.T)], dims)


def test_single_nonzero_all_ranks_one(oracle_mod):
    idx = np.array([[2, 0, 5, 1]], dtype=np.int32)
    res = oracle_mod.decompose(idx, np.array([-3.25]), (4, 3, 7, 2), 0.0, do_round=False)
    assert res.betas == [1, 1, 1, 1, 1]
    for L in res.levels:
        assert list(L.n_val) == [1.0]


def test_rank1_sparse_outer_product_lemma1(oracle_mod):
    # Lemma 1: an outer product of sparse vectors has TT rank 1; every unfolding
    # column is a multiple of the first factor(s).
    rng = np.random.Generator(np.random.PCG64(7))
    dims = (6, 5, 7, 4, 3)
    us = []
    for n in dims:
        u = np.zeros(n)
        pos = rng.choice(n, 3, replace=False)
        u[pos] = rng.integers(16, 49, 3) / 32.0
        us.append(u)
    A = np.einsum("a,b,c,d,e->abcde", *us)
    nz = np.argwhere(A != 0)
    res = oracle_mod.decompose(nz.astype(np.int32), A[tuple(nz.T)], dims, 0.0, do_round=False)
    assert res.betas == [1] * 6


def test_disjoint_rank1_terms_lemma2(oracle_mod):
    # Lemma 2: K rank-1 terms whose supports are pairwise disjoint in every mode
    # give an exact TT whose ranks are K (block-diagonal cores); Deparallelisation
    # keeps exactly K columns at every level.
    rng = np.random.Generator(np.random.PCG64(8))
    K, dims = 4, (8, 12, 8, 8)
    A = np.zeros(dims)
    for t in range(K):
        fs = []
        for n in dims:
            u = np.zeros(n)
            blk = np.arange(t * (n // K), (t + 1) * (n // K))
            # dyadic factors: products are exact, so columns of one term stay
            # exactly parallel in binary64
            u[rng.choice(blk, 2, replace=False)] = rng.integers(16, 49, 2) / 32.0
            fs.append(u)
        A += np.einsum("a,b,c,d->abcd", *fs)
    nz = np.argwhere(A != 0)
    res = oracle_mod.decompose(nz.astype(np.int32), A[tuple(nz.T)], dims, 0.0, do_round=False)
    assert res.betas == [1, K, K, K, 1]


def test_diagonal_tensor(oracle_mod):
    n = 9
    idx = np.repeat(np.arange(n, dtype=np.int32)[:, None], 4, axis=1)
    val = np.arange(1, n + 1, dtype=np.float64) * 0.5
    res = oracle_mod.decompose(idx, val, (n,) * 4, 0.0, do_round=False)
    assert res.betas == [1, n, n, n, 1]


def test_single_entry_columns_give_distinct_unit_columns(oracle_mod):
    # Quasi-permutation case (Corollary 4, Lemma 6): when every unfolding column has
    # one entry, N_k is a duplicate-free selection of unit vectors, so it is
    # orthonormal.
    idx, val, dims = synth.random_sparse((30, 30, 30, 30), 40, seed=3)
    res = oracle_mod.decompose(idx, val, dims, 0.0, do_round=False)
    for L in res.levels:
        lens = np.diff(L.n_colptr)
        if np.all(lens == 1):
            assert np.all(L.n_val == 1.0)
            assert len(set(L.n_row.tolist())) == L.beta


@pytest.mark.parametrize("name,dims,nnz,seed", [("a", (5, 6, 4, 5), 60, 11), ("b", (3, 3, 3, 3, 3, 3), 200, 12),
                                                 ("c", (20, 20, 20, 20), 1000, 1)])
def test_exact_reconstruction_and_bounds(oracle_mod, name, dims, nnz, seed):
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    res = oracle_mod.decompose(idx, val, dims, 0.0, do_round=False)
    d = len(dims)
    # invariants: beta_k <= nnz_{k+1} <= prod_{j>k} n_j, beta_{d-1} <= n_d
    for k in range(1, d):
        L = res.levels[k - 1]
        assert L.beta <= len(L.col) <= int(np.prod(dims[k:]))
    assert res.levels[-1].beta <= dims[-1]
    # exact TT reproduces every entry to 2(d-1) roundings; zero elsewhere
    A = _brute.dense_tensor(idx, val, dims)
    B = _brute.tt_full(res.exact_cores())
    tol = 2 * (d - 1) * np.finfo(float).eps
    assert np.all(np.abs(B - A) <= tol * np.abs(A))


def test_laplacian_exact_bitwise(oracle_mod):
    # every canonical ratio of the Laplacian (+-1, -1/4, -4) is exact, so the exact
    # TT reproduces the matrix bit for bit
    idx, val, dims = synth.laplacian_qtt(3)
    res = oracle_mod.decompose(idx, val, dims, 0.0, do_round=False)
    B = _brute.tt_full(res.exact_cores())
    A = _brute.dense_tensor(idx, val, dims)
    assert np.array_equal(A, B)


def test_permutation_invariance_and_zero_dropping(oracle_mod):
    idx, val, dims = synth.random_sparse((6, 7, 5, 6), 150, 21)
    r1 = oracle_mod.decompose(idx, val, dims, 1e-12)
    rng = np.random.Generator(np.random.PCG64(5))
    p = rng.permutation(len(val))
    extra_idx = np.array([[0, 0, 0, 0]], dtype=np.int32)
    if any((idx == extra_idx).all(1)):
        extra_idx = np.array([[5, 6, 4, 5]], dtype=np.int32)
    idx2 = np.concatenate([idx[p], extra_idx])
    val2 = np.concatenate([val[p], [0.0]])
    r2 = oracle_mod.decompose(idx2, val2, dims, 1e-12)
    assert r1.betas == r2.betas and r1.ranks == r2.ranks
    for c1, c2 in zip(r1.cores, r2.cores):
        assert np.array_equal(c1, c2)


def test_error_codes(oracle_mod):
    E = oracle_mod.OracleError
    ok_idx = np.array([[0, 1], [1, 0]], dtype=np.int32)
    with pytest.raises(E) as e:
        oracle_mod.decompose(np.array([[0, 2]], dtype=np.int32), np.array([1.0]), (2, 2), 0.1)
    assert e.value.name == "INDEX"
    with pytest.raises(E) as e:
        oracle_mod.decompose(ok_idx, np.array([1.0, np.nan]), (2, 2), 0.1)
    assert e.value.name == "NONFINITE"
    with pytest.raises(E) as e:
        oracle_mod.decompose(np.array([[0, 1], [0, 1]], dtype=np.int32), np.array([1.0, 2.0]), (2, 2), 0.1)
    assert e.value.name == "DUPLICATE"
    with pytest.raises(E) as e:
        oracle_mod.decompose(ok_idx, np.array([0.0, -0.0]), (2, 2), 0.1)
    assert e.value.name == "EMPTY"
    with pytest.raises(E) as e:
        oracle_mod.decompose(ok_idx, np.array([1.0, 2.0]), (2, 2), 1.5)
    assert e.value.name == "ARG"
    with pytest.raises(E) as e:
        oracle_mod.decompose(np.array([[0]], dtype=np.int32), np.array([1.0]), (2,), 0.1)
    assert e.value.name == "ARG"
