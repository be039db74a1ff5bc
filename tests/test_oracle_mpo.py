"""Pins of the oracle's matrix -> tensor front-end (matrix in TT format, Sec. 3.4).

The references do not use the oracle's digit arithmetic: a dense NumPy
reshape/transpose of tiny matrices into the order-2d tensor (i_1, j_1, ..., i_d, j_d),
the quantized Laplacian and FDM layouts built from grid coordinates, and MPO
matrix-vector products checked against the sparse product.
"""
import numpy as np
import pytest

from paper_1908_02721_amd import synth
from tests import _brute


def _dense_mpo_tensor(Md, m, n):
    """Dense M x N matrix -> d-way tensor with modes m_k n_k by reshape/transpose."""
    d = len(m)
    T = Md.reshape(tuple(m) + tuple(n))                      # (i_1..i_d, j_1..j_d)
    perm = [x for k in range(d) for x in (k, d + k)]         # (i_1, j_1, ..., i_d, j_d)
    return T.transpose(perm).reshape(tuple(a * b for a, b in zip(m, n)))


@pytest.mark.parametrize("m,n,nnz,seed", [((3, 4), (5, 2), 40, 1), ((2, 3, 2), (3, 1, 4), 60, 2),
                                          ((7,), (5,), 20, 3), ((2, 2, 2, 2), (3, 3, 1, 2), 200, 4)])
def test_coords_match_dense_reshape(oracle_mod, m, n, nnz, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    M, N = int(np.prod(m)), int(np.prod(n))
    lin = rng.choice(M * N, size=min(nnz, M * N), replace=False)
    rows, cols = lin // N, lin % N
    vals = rng.standard_normal(lin.size)
    Md = np.zeros((M, N))
    Md[rows, cols] = vals
    want = _dense_mpo_tensor(Md, m, n)
    idx = oracle_mod.matrix_coords(rows, cols, m, n)
    got = _brute.dense_tensor(idx, vals, [a * b for a, b in zip(m, n)])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_laplacian_quantized_layout(oracle_mod, L):
    r, c, v, m, n = synth.laplacian_matrix(L)
    idx = oracle_mod.matrix_coords(r, c, m, n)
    ref, rv, _ = synth.laplacian_qtt(L)
    assert np.array_equal(idx, ref) and np.array_equal(v, rv)


@pytest.mark.parametrize("n,coeff", [(3, "pattern"), (5, "random")])
def test_fdm_layout(oracle_mod, n, coeff):
    r, c, v, m, nn = synth.fdm3d_matrix(n, coeff, seed=1)
    idx = oracle_mod.matrix_coords(r, c, m, nn)
    ref, rv, _ = synth.fdm3d_mpo(n, coeff, seed=1)
    assert np.array_equal(idx, ref) and np.array_equal(v, rv)


def test_mpo_matvec(oracle_mod):
    """The MPO of the FDM matrix (n = 4, random coefficients) applied to a vector in
    TT-compatible layout equals the sparse matrix-vector product."""
    r, c, v, m, n = synth.fdm3d_matrix(4, "random", seed=3)
    idx = oracle_mod.matrix_coords(r, c, m, n)
    res = oracle_mod.decompose(idx, v, [a * b for a, b in zip(m, n)], 1e-14)
    cores = [G.reshape(G.shape[0], a, b, G.shape[2]) for G, a, b in zip(res.cores, m, n)]
    rng = np.random.Generator(np.random.PCG64(9))
    x = rng.standard_normal(int(np.prod(n)))
    y_ref = np.zeros(int(np.prod(m)))
    np.add.at(y_ref, r, v * x[c])
    # contract: y(i_1..i_d) = sum_j M1(:, i1, j1, :) ... Md(:, id, jd, :) x(j_1..j_d)
    X = x.reshape(tuple(n))
    T = np.tensordot(cores[0][0], X, axes=([1], [0]))           # (i1, r1, j2, j3)
    U = np.einsum("irjk,rpjs->ipsk", T, cores[1])              # (i1, i2, r2, j3)
    V = np.einsum("ipsk,sqkt->ipqt", U, cores[2])[..., 0]      # (i1, i2, i3)
    assert np.max(np.abs(V.reshape(-1) - y_ref)) <= 1e-12 * np.abs(v).sum()


def test_index_errors(oracle_mod):
    with pytest.raises(IndexError):
        oracle_mod.matrix_coords([4], [0], (2, 2), (2, 2))
    with pytest.raises(IndexError):
        oracle_mod.matrix_coords([0], [-1], (2, 2), (2, 2))
    assert oracle_mod.matrix_coords([], [], (2, 2), (3, 3)).shape == (0, 2)
