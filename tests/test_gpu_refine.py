"""Refinement of truncated TT cores on the observed entries: the differentiation form.

Recipe (8-way Kronecker workload, 4,194,297 nonzeros):
1. FP64 decomposition with fixed-rank truncation at rank 32 (Sec. 3.4).
2. Every core entry is perturbed by N(0, 0.01^2), seeded.
3. The cores are refined in FP32 by Adam (lr 1e-3, 100 steps) on
   loss = sum_n (TT(i_n) - a_n)^2, through EvalEntries.

Forward and backward are the library's FP32 evaluation kernels. The loss curve is
printed. The FP32 gradient at the perturbed cores is checked against the FP64
oracle's gradient, with relative L2 <= 1e-5 per core, on a seeded sample of
entries.
"""
import numpy as np
import pytest
import torch

from paper_1908_02721_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_refine_truncated_cores(oracle_mod):
    import paper_1908_02721_amd as tts

    idx, val, dims, _ = synth.workload("kron8d_n32_t64")
    print(f"[refine] kron8d_n32_t64 nnz={len(val)} max_rank=32", flush=True)
    gi = torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda()
    gv = torch.from_numpy(np.ascontiguousarray(val, dtype=np.float64)).cuda()
    tt = tts.decompose(gi, gv, dims, 1e-8, max_rank=32)
    assert max(tt.ranks) == 32
    gen = torch.Generator().manual_seed(5)
    cores = [(c.cpu() + 1e-2 * torch.randn(c.shape, generator=gen, dtype=torch.float64)).float().cuda()
             for c in tt.cores]

    # gradient parity at the perturbed cores on a sample of the entries
    rng = np.random.Generator(np.random.PCG64(6))
    pick = rng.choice(len(val), 20000, replace=False)
    sub = gi[torch.from_numpy(pick).cuda()]
    c64 = [c.double().cpu().numpy() for c in cores]
    y32 = tts.eval_entries(cores, sub)
    gy32 = 2.0 * (y32 - gv[torch.from_numpy(pick).cuda()].float())
    g32 = tts.eval_entries_backward(cores, sub, gy32)
    y64 = oracle_mod.eval_entries(c64, idx[pick])
    g64 = oracle_mod.eval_grad(c64, idx[pick], 2.0 * (y64 - val[pick]))
    for k, (a, b) in enumerate(zip(g32, g64)):
        rel = np.linalg.norm(a.double().cpu().numpy() - b) / max(np.linalg.norm(b), 1e-30)
        assert rel <= 1e-5, f"core {k + 1}: relative L2 gradient error {rel:.2e}"

    # refinement on all nonzeros
    params = [c.clone().requires_grad_(True) for c in cores]
    opt = torch.optim.Adam(params, lr=1e-3)
    target = gv.float()
    losses = []
    for step in range(100):
        opt.zero_grad()
        y = tts.EvalEntries.apply(gi, *params)
        loss = ((y - target) ** 2).sum()
        loss.backward()
        opt.step()
        losses.append(float(loss.item()))
    curve = ", ".join(f"{i}:{losses[i]:.4e}" for i in list(range(0, 100, 10)) + [99])
    print(f"[refine] loss curve {curve}", flush=True)
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], (losses[0], losses[-1])
    # the loss the refinement reaches is far below that of the perturbed start and
    # moves monotonically over the last steps
    assert losses[-1] <= min(losses[-10:]) * (1 + 1e-3)
