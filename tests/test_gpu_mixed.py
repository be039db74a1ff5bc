"""Mixed-precision rounding against the FP64 oracle.

In the two reduced-precision modes the dense contractions run on the matrix cores
with binary32 accumulation:
- FP32: binary32 operands;
- BF16: bfloat16 operands.

These contractions are W' = Q^T X, the last core, U = Q U_R and the merges. The
Gram matrices, R factors, triangular solves and the Jacobi SVD stay in binary64.

For every case the test prints ||B_mixed - B_oracle||_F / ||A||_F, the error against
the FP64 oracle's rounded TT. The gates are the accuracy each precision can support
(FP32 unit roundoff 6e-8, BF16 4e-3, times the growth of a few chained
contractions). They are not the FP64 1e-12 bar. Ranks are reported, not gated: a
contraction rounded to u cannot resolve singular values below about u ||A||.
"""
import numpy as np
import pytest
import torch

from paper_1908_02721_amd import synth

pytestmark = pytest.mark.gpu

GATE = {"fp32": 1e-4, "bf16": 5e-2}


def _gpu(idx, val):
    return torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda(), \
        torch.from_numpy(np.ascontiguousarray(val, dtype=np.float64)).cuda()


def check_mixed(oracle_mod, idx, val, dims, eps, label, precision):
    import paper_1908_02721_amd as tts

    print(f"[mixed] {label} dims={tuple(dims)} nnz={len(val)} eps={eps} precision={precision}", flush=True)
    res = oracle_mod.decompose(idx, val, dims, eps)
    gi, gv = _gpu(idx, val)
    tt = tts.decompose(gi, gv, dims, eps, precision=precision)
    cores = tt.cores
    assert all(c.dtype == torch.float32 for c in cores)
    c64 = [c.double().cpu().numpy() for c in cores]
    nrm = res.norm
    err = oracle_mod.tt_diff_norm(c64, res.cores) / nrm
    print(f"[mixed] {label} {precision}: ranks {tt.ranks} (fp64 oracle {res.ranks}); "
          f"||B - B_oracle|| / ||A|| = {err:.3e}", flush=True)
    assert np.isfinite(err)
    assert err <= GATE[precision] + eps, f"{precision} error {err:.3e}"
    if max(tt.ranks) > 256:  # beyond the evaluator's rank limit
        return tt, res, err
    # entries of the FP32 cores through the FP32 evaluation kernels
    rng = np.random.Generator(np.random.PCG64(3))
    pick = rng.choice(len(val), min(2048, len(val)), replace=False)
    y = tts.eval_entries(cores, gi[torch.from_numpy(pick).cuda()]).double().cpu().numpy()
    yo = oracle_mod.eval_entries(res.cores, idx[pick])
    assert np.max(np.abs(y - yo)) <= (GATE[precision] + eps) * nrm
    return tt, res, err


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mixed_kron_small(oracle_mod, precision):
    idx, val, dims = synth.kronecker_sum(6, 10, 6, 3, seed=4)
    check_mixed(oracle_mod, idx, val, dims, 1e-6, "kron d6 t6", precision)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mixed_laplacian(oracle_mod, precision):
    idx, val, dims = synth.laplacian_qtt(5)
    check_mixed(oracle_mod, idx, val, dims, 1e-10, "laplace L=5", precision)


def test_mixed_laplacian_full_size_fp32(oracle_mod):
    # the 1024 x 1024 grid (20 modes of size 4, 5,238,784 nonzeros): FP32 GPU against
    # the FP64 oracle at eps = 1e-10; the gate is FP32's error plus eps
    idx, val, dims, eps = synth.workload("laplace2d_qtt_L10")
    tt, res, err = check_mixed(oracle_mod, idx, val, dims, eps, "laplace2d_qtt_L10", "fp32")
    print(f"[mixed] laplace2d_qtt_L10 fp32 ranks {tt.ranks}, oracle {res.ranks}, error {err:.3e}", flush=True)
    assert res.ranks == [1] + [3] * 9 + [2] + [4] * 8 + [3] + [1]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mixed_random4d(oracle_mod, precision):
    idx, val, dims, eps = synth.workload("random4d_n20_nnz1k")
    check_mixed(oracle_mod, idx, val, dims, eps, "random4d_n20_nnz1k", precision)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mixed_kron8d_full_size(oracle_mod, precision):
    idx, val, dims, eps = synth.workload("kron8d_n32_t64")
    check_mixed(oracle_mod, idx, val, dims, eps, "kron8d_n32_t64", precision)


def test_fp64_unchanged_by_mode_switches(oracle_mod):
    """An FP64 call after mixed-precision calls still meets the FP64 bar."""
    import paper_1908_02721_amd as tts

    idx, val, dims = synth.kronecker_sum(6, 10, 6, 3, seed=4)
    gi, gv = _gpu(idx, val)
    for p in ("bf16", "fp32"):
        tts.decompose(gi, gv, dims, 1e-10, precision=p)
    tt = tts.decompose(gi, gv, dims, 1e-10)
    res = oracle_mod.decompose(idx, val, dims, 1e-10)
    assert tt.ranks == res.ranks
    assert tt.cores[0].dtype == torch.float64
    diff = oracle_mod.tt_diff_norm([c.cpu().numpy() for c in tt.cores], res.cores)
    assert diff <= 1e-12 * res.norm


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_fasttt_mixed_precision(oracle_mod, precision):
    """The fiber-trie variant's rounding in the precision form: FDM n = 20 with random
    coefficients (p = 2) and a tiny random tensor at every p, against the FP64 oracle."""
    import paper_1908_02721_amd as tts
    from oracle import ftt as oftt

    cases = [(synth.fdm3d_mpo(20, "random", seed=1), 1e-14, [2])]
    cases.append((synth.random_sparse((4, 3, 5, 2), 40, 1), 0.1, [1, 2, 3, 4]))
    for (idx, val, dims), eps, ps in cases:
        gi, gv = _gpu(idx, val)
        for p in ps:
            res = oftt.decompose(idx, val, dims, eps, p=p)
            tt = tts.fasttt_decompose(gi, gv, dims, eps, p=p, precision=precision)
            assert all(c.dtype == torch.float32 for c in tt.cores)
            c64 = [np.ascontiguousarray(c.double().cpu().numpy()) for c in tt.cores]
            err = oracle_mod.tt_diff_norm(c64, [np.ascontiguousarray(c) for c in res.cores]) / res.norm
            print(f"[mixed] fasttt {tuple(dims)} p={p} {precision}: ranks {tt.ranks} (fp64 oracle {res.ranks}); "
                  f"||B - B_oracle|| / ||A|| = {err:.3e}", flush=True)
            assert np.isfinite(err) and err <= GATE[precision] + eps


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_reduced_precision_deflation_is_certified(oracle_mod, precision):
    """A term at 2^-24 of the rest: the pivoted Cholesky drops its directions, and the
    residual test (the left-to-right sweep is FP64 in every mode) must reject every
    such deflation (threshold min(1e-2 delta, 1e-13 ||A||) in every mode), so each
    bond is redone with an exact QR: the QR ranks are the oracle's."""
    import paper_1908_02721_amd as tts

    idx1, val1, dims = synth.kronecker_sum(6, 10, 5, 3, seed=11)
    idx2, val2, _ = synth.kronecker_sum(6, 10, 1, 3, seed=12)
    keys = {}
    for ix, v in zip(idx1, val1):
        keys[tuple(ix)] = keys.get(tuple(ix), 0.0) + v
    for ix, v in zip(idx2, val2 * 2.0 ** -24):
        keys[tuple(ix)] = keys.get(tuple(ix), 0.0) + v
    idx = np.array(list(keys.keys()), dtype=np.int32)
    val = np.array(list(keys.values()), dtype=np.float64)
    res = oracle_mod.decompose(idx, val, dims, 1e-11)
    gi, gv = _gpu(idx, val)
    tt = tts.decompose(gi, gv, dims, 1e-11, precision=precision)
    print(f"[mixed] deflation certificate {precision}: qr ranks {tt.qr_ranks}, oracle {res.qr_ranks}", flush=True)
    assert tt.qr_ranks == res.qr_ranks
