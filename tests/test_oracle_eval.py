"""Pins of the oracle's sampled-entry evaluation and its gradient.

References: the dense TT (NumPy tensordot chain), the rank-1 closed form of the
gradient, and central finite differences.
"""
import numpy as np
import pytest

from tests import _brute


def _rand_tt(rng, dims, ranks):
    r = [1] + list(ranks) + [1]
    return [rng.standard_normal((r[k], n, r[k + 1])) for k, n in enumerate(dims)]


def test_eval_matches_dense(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(1))
    dims = (4, 5, 3, 6)
    cores = _rand_tt(rng, dims, (3, 4, 2))
    X = _brute.tt_full(cores)
    idx = np.stack([rng.integers(0, n, 300) for n in dims], 1).astype(np.int32)
    y = oracle_mod.eval_entries(cores, idx)
    assert np.allclose(y, X[tuple(idx.T)], rtol=1e-13, atol=1e-13)


def test_grad_rank1_closed_form(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(2))
    dims = (5, 4, 6)
    g = [rng.standard_normal(n) for n in dims]
    cores = [x.reshape(1, -1, 1) for x in g]
    idx = np.array([[1, 2, 3]], dtype=np.int32)
    grads = oracle_mod.eval_grad(cores, idx, np.array([1.0]))
    for k in range(3):
        expect = np.zeros(dims[k])
        expect[idx[0, k]] = np.prod([g[j][idx[0, j]] for j in range(3) if j != k])
        assert np.allclose(grads[k].reshape(-1), expect, rtol=1e-14, atol=0)


def test_grad_finite_differences(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(3))
    dims = (4, 3, 5, 4)
    cores = _rand_tt(rng, dims, (3, 2, 3))
    idx = np.stack([rng.integers(0, n, 50) for n in dims], 1).astype(np.int32)
    a = rng.standard_normal(50)

    def loss(cs):
        y = oracle_mod.eval_entries(cs, idx)
        return np.sum((y - a) ** 2)

    y = oracle_mod.eval_entries(cores, idx)
    grads = oracle_mod.eval_grad(cores, idx, 2.0 * (y - a))
    checked = 0
    for k in range(len(dims)):
        flat = cores[k].reshape(-1)
        for e in rng.choice(flat.size, min(flat.size, 24), replace=False):
            h = 1e-6 * max(1.0, abs(flat[e]))
            cp = [c.copy() for c in cores]
            cm = [c.copy() for c in cores]
            cp[k].reshape(-1)[e] += h
            cm[k].reshape(-1)[e] -= h
            fd = (loss(cp) - loss(cm)) / (2 * h)
            an = grads[k].reshape(-1)[e]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
            checked += 1
    assert checked >= 64


def test_grad_zero_at_exact_tt(oracle_mod):
    # the exact TT from the sparse stage reproduces the data, so the gradient of
    # sum (TT(i) - a_i)^2 over the nonzeros vanishes
    from paper_1908_02721_amd import synth

    idx, val, dims = synth.random_sparse((6, 5, 6, 5), 120, 4)
    res = oracle_mod.decompose(idx, val, dims, 0.0, do_round=False)
    cores = res.exact_cores()
    y = oracle_mod.eval_entries(cores, idx)
    grads = oracle_mod.eval_grad(cores, idx, 2.0 * (y - val))
    assert max(np.max(np.abs(g)) for g in grads) <= 1e-13 * np.max(np.abs(val))


def test_eval_rejects_bad_index(oracle_mod):
    cores = [np.ones((1, 2, 1)), np.ones((1, 2, 1))]
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.eval_entries(cores, np.array([[0, 2]], dtype=np.int32))
