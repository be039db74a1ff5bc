"""Pins of the bond-2 Gram slice oracle (oracle/slice.py).

References independent of the slice code: dense reshapes and matrix products of the
exact TT's cores (X_1, X_2 = R_1 x_1 G^(2), the right part P_2), NumPy's LAPACK
singular values of the dense bond-2 unfolding of the tensor (the eigenvalues of the
weighted Gram), and ||A||_F^2 (its trace).
"""
import numpy as np
import pytest

from paper_1908_02721_amd import synth
from tests import _brute

CASES = [
    ("d5", (5, 6, 7, 4, 5), 300, 1),
    ("d5b", (6, 4, 5, 6, 3), 900, 2),   # denser: multi-entry columns and slots
    ("d4", (7, 5, 6, 4), 250, 3),
    ("d3", (6, 8, 5), 120, 4),
]


def _setup(oracle_mod, dims, nnz, seed):
    from oracle import slice as osl

    idx, val, dims = synth.random_sparse(dims, nnz, seed)
    res = oracle_mod.decompose(idx, val, dims, 0.0, do_round=False)
    A = _brute.dense_tensor(idx, val, dims)
    return osl, res, A, dims


@pytest.mark.parametrize("name,dims,nnz,seed", CASES)
def test_bond1_qr_gauge(oracle_mod, name, dims, nnz, seed):
    osl, res, A, dims = _setup(oracle_mod, dims, nnz, seed)
    G = res.exact_cores()
    b1 = osl.bond1_qr(res)
    X1 = G[0].reshape(dims[0], -1)
    assert np.array_equal(b1.X1, X1)
    m = b1.R1.shape[0]
    assert m == min(int(np.count_nonzero(np.any(X1 != 0, axis=1))), X1.shape[1])
    assert np.max(np.abs(b1.Q1.T @ b1.Q1 - np.eye(m))) <= 1e-13
    assert np.max(np.abs(b1.Q1 @ b1.R1 - X1)) <= 1e-13 * np.linalg.norm(X1)
    # SVD gauge: R_1 R_1^T = diag(sigma^2), sigma non-ascending; sign rule on Q_1
    RR = b1.R1 @ b1.R1.T
    assert np.max(np.abs(RR - np.diag(b1.sigma ** 2))) <= 1e-12 * b1.sigma[0] ** 2
    assert np.all(np.diff(b1.sigma) <= 0)
    for j in range(m):
        p = int(np.argmax(np.abs(b1.Q1[:, j])))
        assert b1.Q1[p, j] > 0


@pytest.mark.parametrize("name,dims,nnz,seed", CASES)
def test_x2_weights_and_gram_against_dense(oracle_mod, name, dims, nnz, seed):
    osl, res, A, dims = _setup(oracle_mod, dims, nnz, seed)
    G = res.exact_cores()
    sl = osl.Slice(res)
    m, n2, b2 = sl.m, dims[1], res.betas[2]
    # X_2 = unfold_2(R_1 x_1 G^(2)), rows a * n_2 + i
    X2 = np.einsum("ag,gib->aib", sl.b1.R1, G[1]).reshape(m * n2, b2)
    got = np.array([[sl.x2(a, i, j) for j in range(b2)] for a in range(m) for i in range(n2)])
    assert np.max(np.abs(got - X2)) <= 1e-13 * max(1.0, np.max(np.abs(X2)))
    # right part of bond 2: rows mutually orthogonal, squared norms w_2
    P = G[2].reshape(G[2].shape[0], -1)
    for Gk in G[3:]:
        P = (P.reshape(-1, Gk.shape[0]) @ Gk.reshape(Gk.shape[0], -1)).reshape(P.shape[0], -1)
    PP = P @ P.T
    assert np.max(np.abs(PP - np.diag(np.diag(PP)))) <= 1e-13 * np.max(np.diag(PP))
    assert np.max(np.abs(sl.w2 - np.diag(PP))) <= 1e-13 * np.max(np.diag(PP))
    # weighted Gram, slot-major rows q = i * m + a
    X2p = X2.reshape(m, n2, b2).transpose(1, 0, 2).reshape(n2 * m, b2)
    Gam = (X2p * sl.w2[None, :]) @ X2p.T
    N = n2 * m
    gg = np.array([[sl.gram(q, q2) for q2 in range(N)] for q in range(N)])
    assert np.max(np.abs(gg - Gam)) <= 1e-12 * np.max(np.abs(Gam))
    assert np.max(np.abs(sl.dense_x2() - X2p)) <= 1e-13 * max(1.0, np.max(np.abs(X2p)))
    assert np.max(np.abs(sl.dense_gram() - Gam)) <= 1e-12 * np.max(np.abs(Gam))
    # its eigenvalues are the squared singular values of the dense bond-2 unfolding of A
    s = np.linalg.svd(A.reshape(dims[0] * dims[1], -1), compute_uv=False)
    ev = np.sort(np.linalg.eigvalsh(Gam))[::-1]
    k = min(len(s), len(ev))
    nrm2 = float(np.sum(A * A))
    assert np.max(np.abs(ev[:k] - s[:k] ** 2)) <= 1e-12 * nrm2
    assert np.all(np.abs(ev[k:]) <= 1e-12 * nrm2)
    # trace = ||A||_F^2, three ways
    assert abs(np.trace(Gam) - nrm2) <= 1e-13 * nrm2
    assert abs(sl.weighted_norm2(chunk=7) - nrm2) <= 1e-13 * nrm2
    assert abs(sum(sl.block_trace(i) for i in range(n2)) - nrm2) <= 1e-13 * nrm2
    bt = sl.block_traces(chunk=5)
    for i in range(n2):
        assert abs(bt[i] - np.trace(Gam[i * m:(i + 1) * m, i * m:(i + 1) * m])) <= 1e-13 * nrm2


def test_x2_zero_off_support(oracle_mod):
    # a slot with no entries in a column gives exactly zero, and one-entry blocks are
    # exactly c * R_1[a, g]
    osl, res, A, dims = _setup(oracle_mod, (5, 6, 7, 4, 5), 300, 1)
    sl = osl.Slice(res)
    L2 = res.levels[1]
    j = 0
    rows = L2.n_row[L2.n_colptr[j]:L2.n_colptr[j + 1]]
    vals = L2.n_val[L2.n_colptr[j]:L2.n_colptr[j + 1]]
    slots = set(int(r) % dims[1] for r in rows)
    for i in range(dims[1]):
        for a in range(sl.m):
            want = sum(c * sl.b1.R1[a, int(r) // dims[1]] for r, c in zip(rows, vals) if int(r) % dims[1] == i)
            got = sl.x2(a, i, j)
            if i not in slots:
                assert got == 0.0
            assert abs(got - want) <= 1e-14 * max(1.0, abs(want))
