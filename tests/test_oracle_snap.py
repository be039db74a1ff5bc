"""Pins of the oracle's tolerant parallel test (canonical values rounded to key_bits
fraction bits, round half to even).

The references are independent of the oracle's bit arithmetic: NumPy's IEEE
conversions to binary32 (23 fraction bits) and binary16 (10), which round half to
even; hand-picked ties and carries; and the exact grouping of a noise-free tensor.
"""
import numpy as np
import pytest

from paper_1908_02721_amd import synth


def test_snap_23_bits_is_binary32_rounding(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(1))
    # binary32 normal range: |x| in [2^-126, 2^127]
    x = rng.uniform(0.5, 1, 20000) * np.exp2(rng.integers(-125, 128, 20000)) * rng.choice([-1, 1], 20000)
    # exact ties: 1 + 2^-24 rounds to 1 (even), 1 + 3 2^-24 to 1 + 2^-22
    ties = np.array([1 + 2.0 ** -24, 1 + 3 * 2.0 ** -24, -(1 + 2.0 ** -24), 1.5 + 2.0 ** -24])
    x = np.concatenate([x, ties, [1.0, 0.0, -0.0, 2.0 ** 100]])
    want = x.astype(np.float32).astype(np.float64)
    assert np.array_equal(oracle_mod.snap(x, 23), want)


def test_snap_10_bits_is_binary16_rounding(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(2))
    x = rng.uniform(0.5, 1, 20000) * np.exp2(rng.integers(-13, 15, 20000)) * rng.choice([-1, 1], 20000)
    want = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(oracle_mod.snap(x, 10), want)


def test_snap_carry_and_limits(oracle_mod):
    big = np.finfo(np.float64).max
    x = np.array([2 - 2.0 ** -40, big, -big, 1.0, 3.0])
    y = oracle_mod.snap(x, 10)
    assert y[0] == 2.0                                   # carry into the exponent
    assert np.isfinite(y[1]) and y[1] <= big and y[1] > 0.999 * big   # truncated, not inf
    assert y[2] == -y[1]
    assert y[3] == 1.0 and y[4] == 3.0
    assert np.array_equal(oracle_mod.snap(x, 52), x) and np.array_equal(oracle_mod.snap(x, 0), x)


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_snapped_grouping_of_noisy_columns_is_exact_grouping(oracle_mod, seed):
    # small-integer data: every canonical value is a ratio of integers below 2^10, so
    # its distance to a rounding boundary at 20 bits is far above the 1e-14 noise
    idx, clean, noisy, dims = synth.noisy_kronecker(seed, 1e-14)
    ex = oracle_mod.decompose(idx, clean, dims, 0.0, do_round=False)
    raw = oracle_mod.decompose(idx, noisy, dims, 0.0, do_round=False)
    sn = oracle_mod.decompose(idx, noisy, dims, 0.0, do_round=False, key_bits=20)
    assert any(a > b for a, b in zip(raw.betas, ex.betas)), "noise should break the exact test"
    assert sn.betas == ex.betas
    for Ls, Le in zip(sn.levels, ex.levels):
        assert np.array_equal(Ls.col, Le.col) and np.array_equal(Ls.g, Le.g)
        assert np.array_equal(Ls.n_colptr, Le.n_colptr) and np.array_equal(Ls.n_row, Le.n_row)
        assert np.array_equal(Ls.n_val, oracle_mod.snap(Le.n_val, 20))


@pytest.mark.parametrize("key_bits", [12, 30, 45])
def test_snapped_reconstruction_error_bound(oracle_mod, key_bits):
    """Each stored canonical value moves by at most 2^-(b+1) relative (plus the
    division's rounding); an entry is a product of d - 1 of them and one exact scale."""
    idx, val, dims = synth.kronecker_sum(5, 8, 6, 3, seed=7, continuous=True)
    res = oracle_mod.decompose(idx, val, dims, 0.0, do_round=False, key_bits=key_bits)
    y = oracle_mod.eval_entries(res.exact_cores(), idx)
    d = len(dims)
    u = 2.0 ** -(key_bits + 1) + 2.0 ** -53
    bound = (1 + u) ** (d - 1) * (1 + 2.0 ** -52) ** (2 * d) - 1
    assert np.max(np.abs(y - val) / np.abs(val)) <= bound


def test_key_bits_zero_and_52_are_exact(oracle_mod):
    idx, val, dims = synth.kronecker_sum(4, 7, 4, 3, seed=8, continuous=True)
    ex = oracle_mod.decompose(idx, val, dims, 1e-10)
    for b in (0, 52):
        r = oracle_mod.decompose(idx, val, dims, 1e-10, key_bits=b)
        assert r.betas == ex.betas and r.ranks == ex.ranks
        for a, c in zip(r.cores, ex.cores):
            assert np.array_equal(a, c)
