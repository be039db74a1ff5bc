"""GPU parity of sampled-entry evaluation (forward) and its hand-written backward.

FP64 kernels against the FP64 oracle: relative 1e-12 (different summation order
only).  FP32 kernels against the FP64 oracle: relative L2 error <= 1e-5 (chains of
d vector-matrix products with rank <= 64 in binary32, unit roundoff 6e-8).
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _tts():
    import paper_1908_02721_amd as tts

    return tts


def _rand_tt(rng, dims, ranks, scale=None):
    r = [1] + list(ranks) + [1]
    cores = []
    for k, n in enumerate(dims):
        s = scale if scale is not None else 1.0 / np.sqrt(r[k])
        cores.append(rng.standard_normal((r[k], n, r[k + 1])) * s)
    return cores


def _idx(rng, dims, m):
    return np.stack([rng.integers(0, n, m) for n in dims], 1).astype(np.int32)


def _cuda(cores, dtype):
    return [torch.from_numpy(np.ascontiguousarray(c)).to(dtype).cuda() for c in cores]


CFGS = [
    ("d4r5", (6, 7, 5, 4), (5, 3, 6), 3000),
    ("d8r32", (32,) * 8, (32,) * 7, 20000),
    ("d5r64", (9, 8, 7, 6, 5), (40, 64, 50, 20), 5000),
    ("d3r200", (5, 6, 7), (150, 200), 2000),
    ("d2", (11, 13), (9,), 1000),
]


@pytest.mark.parametrize("name,dims,ranks,m", CFGS)
def test_forward_fp64_and_fp32(oracle_mod, name, dims, ranks, m):
    tts = _tts()
    print(f"[eval fwd] {name}", flush=True)
    rng = np.random.Generator(np.random.PCG64(len(name)))
    cores = _rand_tt(rng, dims, ranks)
    idx = _idx(rng, dims, m)
    ref = oracle_mod.eval_entries(cores, idx)
    gi = torch.from_numpy(idx).cuda()
    y64 = tts.eval_entries(_cuda(cores, torch.float64), gi).cpu().numpy()
    scale = np.linalg.norm(ref) / np.sqrt(m)
    assert np.max(np.abs(y64 - ref)) <= 1e-12 * max(scale, 1.0)
    y32 = tts.eval_entries(_cuda(cores, torch.float32), gi).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(y32 - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("name,dims,ranks,m", CFGS)
def test_backward_fp64_and_fp32(oracle_mod, name, dims, ranks, m):
    tts = _tts()
    print(f"[eval bwd] {name}", flush=True)
    rng = np.random.Generator(np.random.PCG64(100 + len(name)))
    cores = _rand_tt(rng, dims, ranks)
    m = min(m, 4000)
    idx = _idx(rng, dims, m)
    gy = rng.standard_normal(m)
    ref = oracle_mod.eval_grad(cores, idx, gy)
    gi = torch.from_numpy(idx).cuda()
    g64 = tts.eval_entries_backward(_cuda(cores, torch.float64), gi, torch.from_numpy(gy).cuda())
    for k, (a, b) in enumerate(zip(g64, ref)):
        a = a.cpu().numpy()
        assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b))), f"core {k}"
    g32 = tts.eval_entries_backward(_cuda(cores, torch.float32), gi, torch.from_numpy(gy).float().cuda())
    for k, (a, b) in enumerate(zip(g32, ref)):
        a = a.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(a - b) <= 1e-5 * max(np.linalg.norm(b), 1e-30), f"core {k} fp32"


def test_backward_finite_differences():
    tts = _tts()
    rng = np.random.Generator(np.random.PCG64(3))
    dims, ranks = (5, 4, 6, 3), (3, 4, 2)
    cores = _cuda(_rand_tt(rng, dims, ranks), torch.float64)
    idx = torch.from_numpy(_idx(rng, dims, 300)).cuda()
    a = torch.from_numpy(rng.standard_normal(300)).cuda()

    def loss(cs):
        return torch.sum((tts.eval_entries(cs, idx) - a) ** 2).item()

    y = tts.eval_entries(cores, idx)
    grads = tts.eval_entries_backward(cores, idx, 2.0 * (y - a))
    checked = 0
    for k in range(len(cores)):
        flat = cores[k].view(-1)
        for e in rng.choice(flat.numel(), min(flat.numel(), 24), replace=False):
            h = 1e-6 * max(1.0, abs(flat[e].item()))
            old = flat[e].item()
            flat[e] = old + h
            lp = loss(cores)
            flat[e] = old - h
            lm = loss(cores)
            flat[e] = old
            fd = (lp - lm) / (2 * h)
            an = grads[k].view(-1)[e].item()
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
            checked += 1
    assert checked >= 64


def test_autograd_function_gradcheck():
    tts = _tts()
    rng = np.random.Generator(np.random.PCG64(4))
    dims, ranks = (3, 4, 3), (2, 3)
    cores = [c.requires_grad_() for c in _cuda(_rand_tt(rng, dims, ranks), torch.float64)]
    idx = torch.from_numpy(_idx(rng, dims, 40)).cuda()
    assert torch.autograd.gradcheck(lambda *cs: tts.EvalEntries.apply(idx, *cs), cores, eps=1e-6, atol=1e-8)


def test_deterministic_backward_and_errors():
    tts = _tts()
    rng = np.random.Generator(np.random.PCG64(5))
    dims, ranks = (32,) * 6, (16,) * 5
    cores = _cuda(_rand_tt(rng, dims, ranks), torch.float32)
    idx = torch.from_numpy(_idx(rng, dims, 50000)).cuda()
    gy = torch.randn(50000, device="cuda")
    g1 = tts.eval_entries_backward(cores, idx, gy)
    g2 = tts.eval_entries_backward(cores, idx, gy)
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
    bad = idx.clone()
    bad[7, 3] = 32
    with pytest.raises(tts.TTError) as e:
        tts.eval_entries(cores, bad)
    assert e.value.status == "TT_ERR_INDEX"
    with pytest.raises(tts.TTError) as e:
        tts.eval_entries_backward(cores, bad, gy)
    assert e.value.status == "TT_ERR_INDEX"
    empty = idx[:0]
    assert tts.eval_entries(cores, empty).numel() == 0
    gz = tts.eval_entries_backward(cores, empty, gy[:0])
    assert all(float(g.abs().max()) == 0.0 for g in gz)


def test_repeated_and_shared_prefix_coordinates(oracle_mod):
    # repeated coordinates and heavy prefix sharing (every entry below a few prefixes)
    tts = _tts()
    rng = np.random.Generator(np.random.PCG64(9))
    dims, ranks = (4, 3, 50, 60), (3, 7, 9)
    cores = _rand_tt(rng, dims, ranks)
    idx = _idx(rng, dims, 4000)
    idx[:, 0] = 1
    idx[:, 1] = rng.integers(0, 2, 4000)
    idx = np.concatenate([idx, idx[:500]])
    gy = rng.standard_normal(len(idx))
    gi = torch.from_numpy(idx).cuda()
    y = tts.eval_entries(_cuda(cores, torch.float64), gi).cpu().numpy()
    assert np.max(np.abs(y - oracle_mod.eval_entries(cores, idx))) <= 1e-12
    g = tts.eval_entries_backward(_cuda(cores, torch.float64), gi, torch.from_numpy(gy).cuda())
    for a, b in zip(g, oracle_mod.eval_grad(cores, idx, gy)):
        assert np.max(np.abs(a.cpu().numpy() - b)) <= 1e-11 * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("name,dims,ranks,m", CFGS)
def test_plan_matches_one_shot_calls(oracle_mod, name, dims, ranks, m):
    """An EvalPlan gives bit-for-bit the results of the one-shot calls (same kernels,
    same order), whether the backward reuses the kept left products or recomputes
    them, over repeated calls and in both precisions."""
    tts = _tts()
    print(f"[eval plan] {name}", flush=True)
    rng = np.random.Generator(np.random.PCG64(100 + len(name)))
    cores = _rand_tt(rng, dims, ranks)
    idx = _idx(rng, dims, m)
    gy = rng.standard_normal(m)
    gi = torch.from_numpy(idx).cuda()
    plan = tts.EvalPlan(gi, dims)
    for dtype in (torch.float64, torch.float32):
        cs = _cuda(cores, dtype)
        g = torch.from_numpy(gy).to(dtype).cuda()
        y1 = tts.eval_entries(cs, gi)
        gr1 = tts.eval_entries_backward(cs, gi, g)
        for _ in range(2):
            y = plan.forward(cs, save=True)
            assert torch.equal(y, y1)
            for use_saved in (True, False, True):
                gr = plan.backward(cs, g, use_saved=use_saved)
                for a, b in zip(gr, gr1):
                    assert torch.equal(a, b)
        if dtype == torch.float64:
            ref = oracle_mod.eval_entries(cores, idx)
            assert np.max(np.abs(y.cpu().numpy() - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
            for a, b in zip(gr, oracle_mod.eval_grad(cores, idx, gy)):
                assert np.max(np.abs(a.cpu().numpy() - b)) <= 1e-11 * max(1.0, np.max(np.abs(b)))


def test_plan_wide_coordinates_and_errors(oracle_mod):
    """Coordinates too wide to pack into one 64-bit key (8 modes of 300) take the
    entry-by-entry path inside the plan; errors of the plan calls."""
    tts = _tts()
    rng = np.random.Generator(np.random.PCG64(11))
    dims, ranks = (300,) * 8, (4, 6, 5, 7, 3, 5, 4)
    cores = _rand_tt(rng, dims, ranks)
    idx = _idx(rng, dims, 3000)
    gy = rng.standard_normal(3000)
    gi = torch.from_numpy(idx).cuda()
    plan = tts.EvalPlan(gi, dims)
    del gi  # the plan keeps its own copy
    cs = _cuda(cores, torch.float64)
    y = plan.forward(cs, save=True).cpu().numpy()
    assert np.max(np.abs(y - oracle_mod.eval_entries(cores, idx))) <= 1e-12 * max(1.0, np.max(np.abs(y)))
    g = plan.backward(cs, torch.from_numpy(gy).cuda(), use_saved=True)
    for a, b in zip(g, oracle_mod.eval_grad(cores, idx, gy)):
        assert np.max(np.abs(a.cpu().numpy() - b)) <= 1e-11 * max(1.0, np.max(np.abs(b)))
    # use_saved after a saving forward of another dtype is refused
    plan.forward(_cuda(cores, torch.float32), save=True)
    with pytest.raises(tts.TTError) as e:
        plan.backward(cs, torch.from_numpy(gy).cuda(), use_saved=True)
    assert e.value.status == "TT_ERR_ARG"

    # packed-key path: errors
    dims2, ranks2 = (9, 8, 7), (3, 4)
    cores2 = _cuda(_rand_tt(rng, dims2, ranks2), torch.float64)
    idx2 = torch.from_numpy(_idx(rng, dims2, 500)).cuda()
    p2 = tts.EvalPlan(idx2, dims2)
    gy2 = torch.randn(500, dtype=torch.float64, device="cuda")
    with pytest.raises(tts.TTError) as e:
        p2.backward(cores2, gy2, use_saved=True)  # nothing kept yet
    assert e.value.status == "TT_ERR_ARG"
    p2.forward(cores2, save=False)
    with pytest.raises(tts.TTError):
        p2.backward(cores2, gy2, use_saved=True)  # that forward kept nothing
    p2.forward(cores2, save=True)
    other = _cuda(_rand_tt(rng, dims2, (2, 4)), torch.float64)
    with pytest.raises(tts.TTError):
        p2.backward(other, gy2, use_saved=True)  # other ranks
    with pytest.raises(ValueError):
        p2.forward(_cuda(_rand_tt(rng, (9, 8, 6), ranks2), torch.float64))
    bad = idx2.clone()
    bad[3, 2] = 7
    with pytest.raises(tts.TTError) as e:
        tts.EvalPlan(bad, dims2)
    assert e.value.status == "TT_ERR_INDEX"
    empty = tts.EvalPlan(idx2[:0], dims2)
    assert empty.forward(cores2, save=True).numel() == 0
    gz = empty.backward(cores2, gy2[:0], use_saved=True)
    assert all(float(g.abs().max()) == 0.0 for g in gz)


def test_plan_built_beside_a_decomposition():
    """A plan built on a second stream by a worker thread while a decomposition runs
    (both library calls release the GIL) gives bit-identical results to the same
    calls made one after the other."""
    import threading

    import paper_1908_02721_amd as tts
    from paper_1908_02721_amd import synth

    idx, val, dims = synth.kronecker_sum(6, 12, 8, 3, seed=21)
    gi = torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda()
    gv = torch.from_numpy(np.ascontiguousarray(val)).cuda()
    print(f"[plan concurrency] kron d6 nnz={len(val)}", flush=True)
    ref_tt = tts.decompose(gi, gv, dims, 1e-10)
    ref_plan = tts.EvalPlan(gi, dims)
    ref_y = ref_plan.forward(ref_tt.cores, save=True)
    ref_g = ref_plan.backward(ref_tt.cores, gv, use_saved=True)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    for _ in range(3):
        box = {}

        def build():
            side.wait_stream(main)
            box["plan"] = tts.EvalPlan(gi, dims, stream=side)

        th = threading.Thread(target=build)
        th.start()
        tt = tts.decompose(gi, gv, dims, 1e-10)
        th.join()
        cores = tt.cores
        side.wait_stream(main)
        with torch.cuda.stream(side):
            y = box["plan"].forward(cores, save=True, stream=side)
            g = box["plan"].backward(cores, gv, use_saved=True, stream=side)
        main.wait_stream(side)
        torch.cuda.synchronize()
        assert tt.ranks == ref_tt.ranks
        for a, b in zip(cores, ref_tt.cores):
            assert torch.equal(a, b)
        assert torch.equal(y, ref_y)
        for a, b in zip(g, ref_g):
            assert torch.equal(a, b)
