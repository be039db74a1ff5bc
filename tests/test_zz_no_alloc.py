"""The allocation-free evaluation entry point against tt_eval_entries.

tt_eval_entries_noalloc takes its scratch from a static device array instead of
allocating.  It must agree with tt_eval_entries on the same cores and coordinates
(entry formula of Sec. 2.3; FP64 within 1e-12 relative, FP32 within 1e-5 relative
L2, the bars of the evaluation tests), on two calls in a row, the second with a
smaller input, and it must leave no stale flag behind after a call that found an
out-of-range coordinate.
"""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1908_02721_amd import _lib as L

    return L


def _cores(dims, ranks, seed, dtype):
    g = torch.Generator().manual_seed(seed)
    return [torch.randn(ranks[k], dims[k], ranks[k + 1], generator=g, dtype=torch.float64).to(dtype).cuda()
            for k in range(len(dims))]


def _coords(dims, m, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return torch.from_numpy(np.stack([rng.integers(0, n, m) for n in dims], 1).astype(np.int32)).cuda()


def _call(fn, cores, idx):
    L = _lib()
    d = len(cores)
    dims = (ctypes.c_int64 * d)(*[c.shape[1] for c in cores])
    ranks = (ctypes.c_int64 * (d + 1))(*([c.shape[0] for c in cores] + [1]))
    ptrs = (ctypes.c_void_p * d)(*[c.data_ptr() for c in cores])
    dt = L.DTYPE_F64 if cores[0].dtype == torch.float64 else L.DTYPE_F32
    m = idx.shape[0]
    y = torch.full((m,), float("nan"), dtype=cores[0].dtype, device=cores[0].device)
    st = fn(d, dims, ranks, ptrs, dt, m, ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(y.data_ptr()), None)
    torch.cuda.synchronize()
    return st, y


@pytest.mark.parametrize("dtype,ranks", [(torch.float64, [1, 8, 16, 32, 16, 4, 1]),
                                         (torch.float32, [1, 24, 48, 64, 48, 12, 1])])
def test_noalloc_matches_eval_entries_twice(dtype, ranks):
    L = _lib().load()
    dims = [10, 7, 12, 9, 11, 6]
    cores = _cores(dims, ranks, 3, dtype)
    for call, m in enumerate((50_000, 777)):  # the second call is smaller
        idx = _coords(dims, m, 10 + call)
        print(f"[noalloc] dtype={dtype} ranks={ranks} call={call} m={m}", flush=True)
        st_a, y_a = _call(L.tt_eval_entries_noalloc, cores, idx)
        st_b, y_b = _call(L.tt_eval_entries, cores, idx)
        assert st_a == 0 and st_b == 0, (st_a, st_b)
        a, b = y_a.double().cpu().numpy(), y_b.double().cpu().numpy()
        assert np.all(np.isfinite(a))
        if dtype == torch.float64:
            assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b)))
        else:
            assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)


def test_noalloc_index_error_then_clean_call():
    L = _lib().load()
    dims = [5, 6, 7]
    cores = _cores(dims, [1, 3, 4, 1], 5, torch.float64)
    idx = _coords(dims, 1000, 21)
    bad = idx.clone()
    bad[417, 1] = 6  # one past the end of mode 2: caught by the kernel's range check
    print("[noalloc] out-of-range coordinate", flush=True)
    st, _ = _call(L.tt_eval_entries_noalloc, cores, bad)
    assert st == 2  # TT_ERR_INDEX
    st_a, y_a = _call(L.tt_eval_entries_noalloc, cores, idx[:300])
    st_b, y_b = _call(L.tt_eval_entries, cores, idx[:300])
    assert st_a == 0 and st_b == 0
    assert torch.max(torch.abs(y_a - y_b)).item() <= 1e-12 * max(1.0, torch.max(torch.abs(y_b)).item())
    st, _ = _call(L.tt_eval_entries_noalloc, cores, idx[:0])  # m = 0: nothing to evaluate
    assert st == 0
