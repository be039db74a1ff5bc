"""Pins of the oracle's TT-rounding (QR sweep, truncated-SVD sweep).

The references are independent of the oracle: dense TT-SVD (Algorithm 1) with
LAPACK SVDs on densified tiny tensors, the error bound of Theorem 9 and the
Pythagorean error identity from its proof, orthonormality of the swept cores,
TT-ranks equal to the unfolding ranks at small eps (Sec. 3.3), the known QTT
ranks of the 2D Dirichlet Laplacian and the FDM matrix ranks printed in Table 2.
"""
import numpy as np
import pytest

from paper_1908_02721_amd import synth
from tests import _brute


def _sparse(seed, dims, nnz, kind="normal"):
    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    if kind == "lowrank":
        # sum of two rank-1 terms restricted to the sampled support: low rank mixes
        rng = np.random.Generator(np.random.PCG64(seed + 1000))
        fs = [rng.standard_normal((2, n)) for n in dims]
        val = np.zeros(len(val))
        for t in range(2):
            v = np.ones(len(val))
            for k, f in enumerate(fs):
                v *= f[t][idx[:, k]]
            val += v
    return idx, val, dims


CASES = [
    ("r4", 1, (6, 5, 4, 6), 200, "normal", 1e-12),
    ("r4b", 2, (5, 6, 7, 3), 120, "normal", 1e-3),
    ("r5", 3, (4, 3, 5, 4, 3), 300, "normal", 0.3),
    ("lr", 4, (7, 6, 5, 6), 500, "lowrank", 1e-10),
    ("r3", 5, (9, 8, 7), 150, "normal", 0.1),
]


@pytest.mark.parametrize("name,seed,dims,nnz,kind,eps", CASES)
def test_ranks_and_spectra_match_dense_ttsvd(oracle_mod, name, seed, dims, nnz, kind, eps):
    idx, val, dims = _sparse(seed, dims, nnz, kind)
    res = oracle_mod.decompose(idx, val, dims, eps)
    A = _brute.dense_tensor(idx, val, dims)
    nrm = np.linalg.norm(A)
    ranks, sig = _brute.tt_svd_right_to_left(A, eps)
    assert res.ranks == ranks
    assert abs(res.norm - nrm) <= 1e-14 * nrm
    for b in range(len(dims) - 1):
        s_o, s_r = res.sigma[b], sig[b]
        m = min(len(s_o), len(s_r))
        assert np.max(np.abs(s_o[:m] - s_r[:m])) <= 1e-12 * nrm
        assert np.all(s_o[m:] <= 1e-12 * nrm) and np.all(s_r[m:] <= 1e-12 * nrm)


@pytest.mark.parametrize("name,seed,dims,nnz,kind,eps", CASES)
def test_error_bound_pythagoras_orthonormality(oracle_mod, name, seed, dims, nnz, kind, eps):
    idx, val, dims = _sparse(seed, dims, nnz, kind)
    res = oracle_mod.decompose(idx, val, dims, eps)
    A = _brute.dense_tensor(idx, val, dims)
    nrm = np.linalg.norm(A)
    B = _brute.tt_full(res.cores)
    err = np.linalg.norm(A - B)
    # Theorem 9 / Algorithm 2 ENSURE: ||A - B|| <= eps ||A||  (plus round-off)
    assert err <= eps * nrm + 1e-13 * nrm
    # proof of Theorem 9: the error is the root of the discarded sigma^2 sums
    assert abs(err ** 2 - sum(res.tail)) <= 1e-13 * nrm ** 2
    # cores 2..d are right-orthonormal after the right-to-left sweep
    for G in res.cores[1:]:
        M = G.reshape(G.shape[0], -1)
        assert np.max(np.abs(M @ M.T - np.eye(G.shape[0]))) <= 1e-13
    # stable error measure (TT sum + QR sweep) agrees with dense subtraction
    exact = res.exact_cores()
    e2 = oracle_mod.tt_diff_norm(exact, res.cores)
    assert abs(e2 - err) <= 1e-13 * nrm


def test_qr_sweep_keeps_tensor_and_orthonormalises(oracle_mod):
    # eps = 0 keeps every nonzero singular value: the result equals the input up
    # to round-off and its ranks are the unfolding ranks (Sec. 3.3)
    idx, val, dims = _sparse(9, (5, 6, 5, 4), 180)
    res = oracle_mod.decompose(idx, val, dims, 0.0)
    A = _brute.dense_tensor(idx, val, dims)
    B = _brute.tt_full(res.cores)
    assert np.linalg.norm(A - B) <= 1e-13 * np.linalg.norm(A)
    assert res.qr_ranks[1] <= dims[0]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_small_eps_ranks_equal_unfolding_ranks(oracle_mod, seed):
    idx, val, dims = _sparse(seed, (6, 5, 6, 5), 150, "lowrank" if seed == 2 else "normal")
    res = oracle_mod.decompose(idx, val, dims, 1e-14)
    A = _brute.dense_tensor(idx, val, dims)
    for k in range(1, len(dims)):
        M = A.reshape(int(np.prod(dims[:k])), -1)
        assert res.ranks[k] == np.linalg.matrix_rank(M)


@pytest.mark.parametrize("max_rank", [1, 2, 5])
def test_fixed_rank_matches_dense_ttsvd(oracle_mod, max_rank):
    idx, val, dims = _sparse(31, (5, 6, 4, 5), 200)
    res = oracle_mod.decompose(idx, val, dims, 0.5, max_rank=max_rank)
    A = _brute.dense_tensor(idx, val, dims)
    ranks, sig = _brute.tt_svd_right_to_left(A, ranks_fixed=max_rank)
    assert res.ranks == ranks
    B = _brute.tt_full(res.cores)
    assert abs(np.linalg.norm(A - B) ** 2 - sum(res.tail)) <= 1e-12 * np.linalg.norm(A) ** 2


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_laplacian_qtt_ranks(oracle_mod, L):
    # QTT ranks of the 2D Dirichlet Laplacian, x bits then y bits:
    # [3]*(L-1), 2, [4]*(L-2), 3 -- re-derived here by dense TT-SVD (LAPACK)
    idx, val, dims = synth.laplacian_qtt(L)
    res = oracle_mod.decompose(idx, val, dims, 1e-10)
    expect = [1] + [3] * (L - 1) + [2] + [4] * (L - 2) + [3] + [1]
    assert res.ranks == expect
    if L <= 4:
        A = _brute.dense_tensor(idx, val, dims)
        ranks, _ = _brute.tt_svd_right_to_left(A, 1e-10)
        assert ranks == expect
    assert len(val) == 5 * 4 ** L - 4 * 2 ** L


def _table2():
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "table2_fdm_ranks.json")) as f:
        return [c for c in json.load(f)["cases"] if c["n"] <= 30]


@pytest.mark.parametrize("case", _table2(), ids=lambda c: f"n{c['n']}-{c['coeff']}")
def test_fdm_mpo_ranks_table2(oracle_mod, case):
    # Table 2: final TT-ranks of the 3D FDM matrix as an MPO, eps = 1e-14
    idx, val, dims = synth.fdm3d_mpo(case["n"], case["coeff"], seed=1)
    assert len(val) == case["nnz"]
    res = oracle_mod.decompose(idx, val, dims, 1e-14)
    assert res.ranks == [1] + case["final_ranks"] + [1]


# ---- dynamic truncation thresholds (Algorithm 8, Theorem 10) ----

def test_dynamic_delta_superdiagonal_closed_form(oracle_mod):
    # A = e0 x e0 x e0 + 0.5 e1 x e1 x e1 + 0.1 e2 x e2 x e2: both unfoldings have
    # singular values (1, 0.5, 0.1), ||A||^2 = 1.26.  With eps^2 = 0.012 the fixed
    # threshold delta^2 = eps^2 ||A||^2 / 2 = 0.00756 keeps 0.1 (0.01 > 0.00756) at
    # both bonds.  The dynamic one keeps it at bond 2 as well (same threshold first),
    # discards nothing there, and so offers the whole budget eps^2 ||A||^2 = 0.01512
    # to bond 1, which then drops 0.1 (0.01 <= 0.01512) but not 0.5.
    idx = np.array([[0, 0, 0], [1, 1, 1], [2, 2, 2]], dtype=np.int32)
    val = np.array([1.0, 0.5, 0.1])
    eps = np.sqrt(0.012)
    st = oracle_mod.decompose(idx, val, (3, 3, 3), eps)
    dy = oracle_mod.decompose(idx, val, (3, 3, 3), eps, dynamic_delta=True)
    assert st.ranks == [1, 3, 3, 1]
    assert dy.ranks == [1, 2, 3, 1]
    assert dy.tail[1] == 0.0 and abs(dy.tail[0] - 0.01) <= 1e-15
    assert abs(dy.bond_delta[1] ** 2 - 0.00756) <= 1e-15
    assert abs(dy.bond_delta[0] ** 2 - 0.01512) <= 1e-15
    B = _brute.tt_full(dy.cores)
    A = _brute.dense_tensor(idx, val, (3, 3, 3))
    assert abs(np.linalg.norm(A - B) - 0.1) <= 1e-14


@pytest.mark.parametrize("name,seed,dims,nnz,kind,eps", CASES)
def test_dynamic_delta_matches_dense_and_theorem10(oracle_mod, name, seed, dims, nnz, kind, eps):
    idx, val, dims = _sparse(seed, dims, nnz, kind)
    st = oracle_mod.decompose(idx, val, dims, eps)
    dy = oracle_mod.decompose(idx, val, dims, eps, dynamic_delta=True)
    A = _brute.dense_tensor(idx, val, dims)
    nrm = np.linalg.norm(A)
    ranks, _ = _brute.tt_svd_right_to_left(A, eps, dynamic=True)
    assert dy.ranks == ranks
    d = len(dims)
    # the first bond truncated (bond d-1) sees the same threshold in both modes
    assert dy.ranks[d - 1] == st.ranks[d - 1]
    assert abs(dy.bond_delta[d - 2] - st.delta) <= 1e-15 * nrm
    # every later threshold is at least the fixed one (loop invariant of Theorem 10)
    assert all(x >= st.delta * (1 - 1e-14) for x in dy.bond_delta)
    # Theorem 10: ||A - B|| <= eps ||A||; the discarded sums stay within the budget
    B = _brute.tt_full(dy.cores)
    err = np.linalg.norm(A - B)
    assert err <= eps * nrm + 1e-13 * nrm
    assert sum(dy.tail) <= (eps * nrm) ** 2 * (1 + 1e-12) + 1e-26
    assert abs(err ** 2 - sum(dy.tail)) <= 1e-13 * nrm ** 2


def test_dynamic_delta_two_modes_is_static(oracle_mod):
    # d = 2: one bond, whose threshold is eps ||A|| in both modes
    idx, val, dims = _sparse(12, (9, 11), 60)
    for eps in (1e-12, 0.2, 0.5):
        st = oracle_mod.decompose(idx, val, dims, eps)
        dy = oracle_mod.decompose(idx, val, dims, eps, dynamic_delta=True)
        assert st.ranks == dy.ranks
        for a, b in zip(st.cores, dy.cores):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("kappa", [10.0, 60.0, 1000.0, 1e9])
def test_known_spectrum_of_orthogonal_terms(oracle_mod, kappa):
    # Rank-1 terms with pairwise disjoint supports in every mode are orthogonal in
    # every unfolding: bond b has exactly the singular values w_t q^(d/2) (Sec. 3.3:
    # TT-ranks are the unfolding ranks), whatever the spread of the weights.
    d, T, q = 4, 12, 2
    idx, val, dims = synth.orthogonal_terms(d, T, q, kappa, seed=3)
    res = oracle_mod.decompose(idx, val, dims, 1e-14)
    expect = np.sort(kappa ** (np.arange(T) / (T - 1)))[::-1] * q ** (d / 2)
    assert abs(res.norm - np.sqrt(np.sum(expect ** 2))) <= 1e-14 * res.norm
    assert res.ranks == [1] + [T] * (d - 1) + [1]
    for b in range(d - 1):
        s = np.asarray(res.sigma[b])
        assert np.max(np.abs(s[:T] - expect)) <= 1e-14 * res.norm, b
        assert np.all(s[T:] <= 1e-14 * res.norm)


@pytest.mark.parametrize("case", ["kron", "random"])
def test_sign_rule_gauge_of_the_rounded_cores(oracle_mod, case):
    # The right-to-left SVD sweep leaves core k (k >= 2) as U^T of its bond's SVD, so
    # the rows of unfold_1(core k) are the kept left singular vectors: orthonormal, and
    # each with its entry of largest magnitude positive (the SVD gauge; it pins the
    # sign choice, which the represented tensor does not see).
    if case == "kron":
        idx, val, dims = synth.kronecker_sum(5, 8, 6, 3, seed=2)
    else:
        idx, val, dims = synth.random_sparse((6, 7, 5, 6), 400, 11)
    res = oracle_mod.decompose(idx, val, dims, 1e-10)
    for k, core in enumerate(res.cores[1:], start=2):
        u = core.reshape(core.shape[0], -1)
        assert np.allclose(u @ u.T, np.eye(u.shape[0]), atol=1e-12), k
        top = u[np.arange(u.shape[0]), np.argmax(np.abs(u), axis=1)]
        assert np.all(top > 0), (k, top)
